"""Find the kernel scale s of each workload (writes nothing; prints the table).

The squared form of Sec. 4.3 needs A - B and A + B positive definite (the TDA
needs A positive definite for its eigenvalues to be excitation energies).  The
synthetic kernel has no such guarantee, so s is the largest power of two,
starting from 1, for which every eigenvalue of A - B and A + B (or A) stays
above a tenth of the smallest transition energy.  Uses only the oracle.

    python -m oracle.calibrate_scale [workload ...]
"""
from __future__ import annotations

import sys
from dataclasses import replace

import numpy as np

from bse_synth import WORKLOADS, make_inputs

from . import bse_oracle as O


def _min_eig(M: np.ndarray) -> float:
    if M.shape[0] <= 3000:
        return float(np.linalg.eigvalsh(M)[0])
    return float(np.linalg.eigvalsh(M, UPLO="U")[0])


def calibrate(name: str) -> float:
    w = WORKLOADS[name]
    d = make_inputs(replace(w, kernel_scale=1.0))
    A1, B1 = O.assemble(d)
    E = O.transition_energies(d)
    D = np.diag(E)
    margin = 0.1 * E.min()
    s = 1.0
    while s > 2.0 ** -20:
        A = D + s * (A1 - D)
        ok = _min_eig(A) > margin if B1 is None else (
            _min_eig(A - s * B1) > margin and _min_eig(A + s * B1) > margin)
        if ok:
            return s
        s *= 0.5
    raise RuntimeError(f"no scale found for {name}")


if __name__ == "__main__":
    names = sys.argv[1:] or [n for n, w in WORKLOADS.items() if w.n <= 3000]
    for n in names:
        print(f"{n}: kernel_scale = {calibrate(n)!r}", flush=True)
