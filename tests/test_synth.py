"""Input generator: shapes, shells, determinism, screened interaction."""
import numpy as np
import pytest

from bse_synth import get, lattice, make_inputs
from bse_synth import generate as gen


@pytest.mark.parametrize("ng,bound", [(59, 12), (89, 19), (113, 20), (137, 24)])
def test_closed_shells(ng, bound):
    g = lattice.gvectors(ng)
    n2 = np.sum(g * g, axis=1)
    assert n2.max() == bound
    # all-even or all-odd triples (bcc reciprocal lattice of fcc)
    assert np.all((g[:, 0] % 2 == g[:, 1] % 2) & (g[:, 1] % 2 == g[:, 2] % 2))
    # closed: every lattice vector with |G|^2 <= bound is present, inversion symmetric
    s = {tuple(x) for x in g}
    assert all(tuple(-x) in s for x in g)
    assert np.all(np.diff(n2) >= 0) and n2[0] == 0


def test_fcc_volume_and_basis():
    b = lattice.recip_basis()
    a = lattice.A_LATT
    # reciprocal cell volume (2 pi)^3 / Omega
    assert np.isclose(abs(np.linalg.det(b)), (2 * np.pi) ** 3 / lattice.cell_volume())
    assert np.isclose(lattice.cell_volume(), a ** 3 / 4)


def test_qmaps_match_cartesian_differences():
    n = 3
    km = lattice.kmesh(n)
    b = lattice.recip_basis()
    kc = (km / n) @ b
    qmap, qramap = lattice.q_maps(n)
    binv = np.linalg.inv(b)
    for i in range(len(km)):
        for j in range(len(km)):
            for sign, m in ((1, qmap), (-1, qramap)):
                d = sign * kc[i] - kc[j] - kc[m[i, j]]
                coef = d @ binv  # must be an integer vector (a reciprocal lattice vector)
                assert np.allclose(coef, np.round(coef), atol=1e-12)


def test_determinism_and_thread_independence(monkeypatch):
    w = get("small_full_k3_v3c4_g27")
    a = make_inputs(w)
    monkeypatch.setattr(gen, "_threads", lambda: 1)
    monkeypatch.setattr(gen, "_CHUNK_ROWS", gen._CHUNK_ROWS)
    b = make_inputs(w)
    for k in ("eps_v", "eps_c", "Mcv", "Mvv", "Mcc", "Ncv", "Nvc", "W"):
        assert np.array_equal(a[k], b[k]), k


def test_shapes_and_ranges():
    w = get("tiny_full_k2_v2c3_g15")
    d = make_inputs(w)
    P = w.nk * (w.nk + 1) // 2
    assert d["Mcv"].shape == (w.n, 15)
    assert d["Mvv"].shape == (P, 2, 2, 15) and d["Mcc"].shape == (P, 3, 3, 15)
    assert d["Ncv"].shape == (P, 3, 2, 15) and d["Nvc"].shape == (P, 2, 3, 15)
    assert np.all((d["eps_v"] >= -3) & (d["eps_v"] <= 0))
    assert np.all((d["eps_c"] >= 1) & (d["eps_c"] <= 5))


def test_screened_interaction_hermitian_pd():
    d = make_inputs(get("tda_q0_k4_v2c3_g59"))
    W = d["W"]
    for q in range(W.shape[0]):
        assert np.allclose(W[q], W[q].conj().T, atol=1e-12 * abs(W[q]).max())
        assert np.linalg.eigvalsh(W[q])[0] > 0
    # q = 0 head: v(0) regularised to 4 pi / 0.01, screened by (I + L L^H)^-1 < 1
    assert 0 < W[0][0, 0].real < 4 * np.pi / 0.01


def test_complex_normal_statistics():
    d = make_inputs(get("tda_q0_k4_v2c3_g59"))
    G = lattice.gcart(59)
    x = d["Mvv"] * (1.0 + np.sum(G ** 2, axis=1))
    assert abs(np.mean(np.abs(x) ** 2) - 1.0) < 0.02
    assert abs(np.mean(x.real * x.imag)) < 0.01
