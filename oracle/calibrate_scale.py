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


def _above(M: np.ndarray, margin: float) -> bool:
    """Every eigenvalue of the Hermitian M exceeds margin (Cholesky test)."""
    try:
        np.linalg.cholesky(M - margin * np.eye(M.shape[0]))
        return True
    except np.linalg.LinAlgError:
        return False


def calibrate_inputs(d: dict) -> float:
    A1, B1 = O.assemble(d)
    E = O.transition_energies(d)
    D = np.diag(E)
    margin = 0.1 * E.min()
    s = 1.0
    while s > 2.0 ** -20:
        A = D + s * (A1 - D)
        ok = _above(A, margin) if B1 is None else (
            _above(A - s * B1, margin) and _above(A + s * B1, margin))
        if ok:
            return s
        s *= 0.5
    raise RuntimeError("no kernel scale found")


def calibrate(name: str) -> float:
    return calibrate_inputs(make_inputs(replace(WORKLOADS[name], kernel_scale=1.0)))


def calibrate_batch(name: str) -> float:
    """Largest scale that keeps every member of the batch positive definite."""
    from bse_synth import BATCHES, make_batch_inputs
    bw = BATCHES[name]
    bw1 = replace(bw, master=replace(bw.master, kernel_scale=1.0),
                  members=tuple(replace(m, kernel_scale=1.0) for m in bw.members))
    s = 1.0
    for d in make_batch_inputs(bw1):
        s = min(s, calibrate_inputs(d))
        print(f"  {d['workload'].name}: n={d['workload'].n} -> {s!r}", flush=True)
    return s


if __name__ == "__main__":
    from bse_synth import BATCHES
    names = sys.argv[1:] or [n for n, w in WORKLOADS.items() if w.n <= 3000]
    for n in names:
        if n in BATCHES:
            print(f"{n}: kernel_scale = {calibrate_batch(n)!r}", flush=True)
        else:
            print(f"{n}: kernel_scale = {calibrate(n)!r}", flush=True)
