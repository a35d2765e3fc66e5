"""The stored oracle results (tests/golden/*.npz) belong to today's inputs and
satisfy the sum rules they must (CPU only).

  * the fingerprint of the generated inputs equals the stored one;
  * E ascending and positive, |t|^2 >= 0, eps_M recomputed from the stored E
    and |t|^2 (eq. chir) equals the stored spectrum;
  * for the N = 1296 batch member, rebuilt here by the oracle: the f-sum rule
    sum_l E_l |t_l|^2 = p^H (A - B) p and the static limit
    sum_l |t_l|^2 / E_l = p^H (A + B)^-1 p (Sec. 4.3-4.4), which fail if the
    stored E or |t|^2 belong to another problem.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import bse_oracle as O
from tests.golden.make_golden import fingerprint, load_inputs, path_of

NAMES = ("batch16_k6_g89:0", "batch16_k6_g89:1", "batch16_k6_g89:11", "full_q0_k8_v3c4_g113")


def _load(name):
    with np.load(path_of(name)) as z:
        return {k: z[k] for k in z.files}


@pytest.mark.parametrize("name", NAMES)
def test_golden_belongs_to_inputs(name):
    g = _load(name)
    d = load_inputs(name)
    w = d["workload"]
    assert np.allclose(fingerprint(d), g["fp"], rtol=1e-12, atol=0)
    assert len(g["E"]) == w.n and len(g["eps"]) == w.nw
    assert np.all(np.diff(g["E"]) >= 0) and g["E"][0] > 0
    assert np.all(g["t2"] >= 0)
    eps = O.spectrum(g["E"], g["t2"], d["omega"], w.eta, O.spectrum_prefactor(d))
    assert np.abs(eps - g["eps"]).max() < 1e-13 * np.abs(g["eps"] - 1).max()


def test_golden_sum_rules():
    name = "batch16_k6_g89:0"
    g = _load(name)
    d = load_inputs(name)
    A, B = O.assemble(d)
    p = O.probe(d)
    fsum = np.vdot(p, (A - B) @ p).real
    assert abs(np.sum(g["E"] * g["t2"]) - fsum) < 1e-11 * fsum
    static = np.vdot(p, sl.cho_solve(sl.cho_factor(A + B), p)).real
    assert abs(np.sum(g["t2"] / g["E"]) - static) < 1e-11 * static


def test_golden_files_present():
    for nm in NAMES:
        assert os.path.exists(path_of(nm)), nm
