"""Write the oracle's reference results for the full-size workloads.

    python tests/golden/make_golden.py [name ...]

For each workload this runs the FP64 CPU oracle (oracle/bse_oracle.py) on the
seeded synthetic inputs of bse_synth and stores, in tests/golden/<name>.npz,
  E    the exciton energies, ascending (Sec. 4.3, the squared form with the
       literal (A-B)^1/2),
  t2   the oscillator strengths |t_l|^2 (Sec. 4.4, eq. osci),
  eps  eps_M on the workload's frequency grid (eq. chir in eps_M = 1 - v Pbar),
  fp   a fingerprint of the inputs (sums of a few arrays), so that a test can
       tell when the generator no longer produces the inputs these values
       belong to.
Nothing here calls the GPU library: every stored value comes from oracle/.
Batch members are named <batch>:<index> (e.g. batch16_k6_g89:0).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT = ("full_q0_k8_v3c4_g113", "batch16_k6_g89:0", "batch16_k6_g89:1",
           "batch16_k6_g89:11")


def fingerprint(d: dict) -> np.ndarray:
    """Sums that change whenever the generator's output changes."""
    f = [np.sum(np.abs(d["Mcv"]) ** 2), np.sum(d["eps_v"]), np.sum(d["eps_c"]),
         np.sum(np.abs(d["W"][0])), np.sum(np.abs(d["Mvv"][:64]) ** 2)]
    if d.get("Ncv") is not None:
        f.append(np.sum(np.abs(d["Ncv"][:64]) ** 2))
    return np.array(f, dtype=np.float64)


def load_inputs(name: str) -> dict:
    from bse_synth import BATCHES, get, make_batch_inputs, make_inputs
    if ":" in name:
        bname, i = name.split(":")
        return make_batch_inputs(BATCHES[bname])[int(i)]
    return make_inputs(get(name))


def path_of(name: str) -> str:
    return os.path.join(HERE, name.replace(":", "_m") + ".npz")


def write(name: str) -> str:
    from oracle import bse_oracle as O
    t0 = time.perf_counter()
    d = load_inputs(name)
    A, B = O.assemble(d)
    t1 = time.perf_counter()
    E, XpY, _ = O.solve(A, B)
    del A, B
    t2 = O.oscillator(XpY, O.probe(d))
    del XpY
    t3 = time.perf_counter()
    w = d["workload"]
    eps = O.spectrum(E, t2, d["omega"], w.eta, O.spectrum_prefactor(d))
    out = path_of(name)
    np.savez_compressed(out, E=E, t2=t2, eps=eps, fp=fingerprint(d),
                        n=np.int64(w.n), nw=np.int64(w.nw))
    print(f"{name}: N = {w.n}, assembly {t1 - t0:.1f} s, solve {t3 - t1:.1f} s -> "
          f"{os.path.relpath(out, ROOT)}", flush=True)
    return out


if __name__ == "__main__":
    for nm in (sys.argv[1:] or DEFAULT):
        write(nm)
