"""Pins of the screening oracle (RPA dielectric matrix and W = v eps^-1)
against routes that do not share its formulas."""
import numpy as np
import pytest

from bse_synth import get, lattice, make_screening_inputs
from oracle import screening as S


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def tiny():
    return make_screening_inputs(get("tiny_full_k2_v2c3_g15"))


def test_chi_sum_against_a_literal_loop_over_band_pairs(tiny):
    """Every band pair (i at k, j at k+q) with its occupation factors as
    printed: (f_j - f_i) / (e_j - e_i); pairs of equal occupation get random
    elements and must drop out; ordering of the two band sets must not matter."""
    d = tiny
    w = d["workload"]
    nv, nc, ng = w.nv, w.nc, w.ng
    rng = np.random.default_rng(5)
    inv_vc = 1.0 / (w.nk * d["cell_volume"])
    for iq in (0, 3, w.nk - 1):
        X = np.zeros((ng, ng), dtype=np.complex128)
        for k in range(w.nk):
            kq = d["kqmap"][iq, k]
            e_k = np.concatenate([d["eps_v"][k], d["eps_c"][k]])
            e_kq = np.concatenate([d["eps_v"][kq], d["eps_c"][kq]])
            f = np.concatenate([np.ones(nv), np.zeros(nc)])
            for i in range(nv + nc):
                for j in range(nv + nc):
                    if i < nv and j >= nv:
                        m = d["Svc"][iq, k, i, j - nv]
                    elif i >= nv and j < nv:
                        m = d["Scv"][iq, k, i - nv, j]
                    else:
                        m = rng.standard_normal(ng) + 1j * rng.standard_normal(ng)
                    df = f[j] - f[i]  # 0/0 for i = j at q = 0: the term vanishes with df
                    F = df / ((e_kq[j] - e_k[i]) / S.HARTREE_EV) if df != 0 else 0.0
                    for g in range(ng):
                        for g2 in range(ng):
                            X[g, g2] += F * np.conj(m[g]) * m[g2]
        X *= inv_vc
        ref = S.chi_sum(d["Svc"], d["Scv"], d["eps_v"], d["eps_c"], d["kqmap"], iq, inv_vc)
        assert _rel(ref, X) < 1e-13


def test_single_transition_sherman_morrison():
    """One k, one (v, c) pair: X = F conj(m) m^T / V_c is rank one, so
    eps^-1 = I + c conj(m) (v m)^T / (1 - c (v m)^T conj(m)), c = F / V_c."""
    rng = np.random.default_rng(2)
    ng = 7
    m = rng.standard_normal(ng) + 1j * rng.standard_normal(ng)
    Svc = m.reshape(1, 1, 1, 1, ng)
    Scv = np.zeros((1, 1, 1, 1, ng), dtype=np.complex128)
    ev, ec = np.array([[-1.0]]), np.array([[2.5]])
    kq = np.zeros((1, 1), dtype=np.int32)
    inv_vc = 0.013
    X = S.chi_sum(Svc, Scv, ev, ec, kq, 0, inv_vc)
    v = rng.uniform(0.5, 3.0, ng)
    c = inv_vc * (-S.HARTREE_EV / 3.5)
    vm = v * m
    einv = np.eye(ng) + c * np.outer(m.conj(), vm) / (1.0 - c * vm @ m.conj())
    assert _rel(S.screened_w(S.dielectric_matrix(X, v), v), v[:, None] * einv) < 1e-13


def test_bare_limit_and_screening_order(tiny):
    """No pair elements: W = v.  Otherwise W is Hermitian with
    0 < v^-1/2 W v^-1/2 <= 1 (the screening only weakens v), for every q."""
    d = dict(tiny)
    w = d["workload"]
    v = S.coulomb(d["qcart"], lattice.gcart(w.ng))
    W = S.screening(d)
    for iq in range(w.nk):
        sv = 1.0 / np.sqrt(v[iq])
        R = sv[:, None] * W[iq] * sv[None, :]
        assert _rel(R, R.conj().T) < 1e-13
        lam = np.linalg.eigvalsh(0.5 * (R + R.conj().T))
        assert lam.min() > 0.0 and lam.max() <= 1.0 + 1e-13
    d0 = dict(d)
    d0["Svc"], d0["Scv"] = np.zeros_like(d["Svc"]), np.zeros_like(d["Scv"])
    W0 = S.screening(d0)
    for iq in range(w.nk):
        assert np.array_equal(W0[iq], np.diag(v[iq]).astype(np.complex128))


def test_coulomb_regularised_only_at_zero():
    qc = np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0]])
    G = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 0.0]])
    v = S.coulomb(qc, G)
    assert v[0, 0] == 4.0 * np.pi / 0.01
    assert np.isclose(v[1, 0], 4.0 * np.pi / 0.01)   # |q| = 0.1 exactly: not regularised
    assert np.isclose(v[1, 1], 4.0 * np.pi / (1.1 ** 2 + 1.0))
