"""Pair elements formed on the GPU from orbitals (bse_pair_elements) against
the oracle's restricted plane-wave sums (oracle/orbitals.py, Sec. 4.1), and
the whole chain orbitals -> pair elements -> build -> solve -> spectrum
against the oracle's chain on its own pair elements.

Tolerances: every element is a sum of at most N_K products of coefficients
of norm <= 1 accumulated in FP64, so 1e-13 of the largest element; the chain
keeps the FP64 gates (eigenvalues and spectrum 1e-10).
"""
import numpy as np
import pytest

from oracle import bse_oracle as O
from oracle import orbitals as OR

pytestmark = pytest.mark.gpu

SMALL = ["tiny_orb_k2_v2c3_g15_o27", "small_orb_k3_v3c4_g27_o51", "mid_orb_tda_k4_v2c3_g59_o89"]


def _problem(d):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_05575_amd.bse import Problem
    return Problem(d)


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("name", SMALL)
def test_pair_elements_match_oracle(name):
    from bse_synth import get, make_inputs
    d = make_inputs(get(name))
    print(f"[gpu] pair elements {name}", flush=True)
    P = _problem(d)
    P.check_info()
    w = d["workload"]
    ref = OR.bse_pair_arrays(d["C"], w.nv, d["kvec"], d["gvec"], coupling=w.coupling == "full")
    keys = ["Mcv", "Mvv", "Mcc"] + (["Ncv", "Nvc"] if w.coupling == "full" else [])
    for k in keys:
        got = P.t[k].cpu().numpy().reshape(ref[k].shape)
        assert _rel(got, ref[k]) < 1e-13, k


@pytest.mark.parametrize("name", SMALL)
def test_chain_from_orbitals_matches_oracle(name):
    from bse_synth import get, make_inputs
    d = make_inputs(get(name))
    print(f"[gpu] chain from orbitals {name}", flush=True)
    P = _problem(d)
    out = P.run()
    r = O.run(OR.complete_inputs(d))
    eig = np.abs(out["E"] - r["E"]).max() / np.abs(r["E"]).min()
    spec = np.abs(out["eps"] - r["eps"]).max() / np.abs(r["eps"] - 1).max()
    assert eig < 1e-10 and spec < 1e-10, (eig, spec)


def test_pair_elements_at_full_size():
    """N = 6144 (8^3 mesh, 3 + 4 bands, 113 G, 113 K per orbital): sampled
    pairs of every array and M_cv rows against the oracle."""
    from bse_synth import get, make_inputs
    name = "full_orb_k8_v3c4_g113_o113"
    d = make_inputs(get(name))
    print(f"[gpu] pair elements {name}", flush=True)
    P = _problem(d)
    P.check_info()
    w = d["workload"]
    ik, jk = np.triu_indices(w.nk)
    rng = np.random.default_rng(3)
    sel = np.unique(np.concatenate([rng.choice(len(ik), 120, replace=False),
                                    [0, len(ik) - 1]]))
    pairs = np.stack([ik[sel], jk[sel]], axis=1)
    ref = OR.bse_pair_arrays(d["C"], w.nv, d["kvec"], d["gvec"], pairs=pairs)
    for k in ("Mvv", "Mcc", "Ncv", "Nvc"):
        got = P.t[k][sel].cpu().numpy()
        assert _rel(got, ref[k]) < 1e-13, k
    assert _rel(P.t["Mcv"].cpu().numpy(), ref["Mcv"]) < 1e-13
