"""Pins of the observables oracle (dielectric tensor, loss function, S(Q, w))
against routes that do not use its formulas: the resolvent definition of
eps_M, the closed form of a single pole, the f-sum rule and X+Y = 1."""
import numpy as np
import pytest
from scipy import integrate

from oracle import bse_oracle as O
from oracle import observables as X
from tests._cache import inputs, oracle_run


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("name", ["tiny_tda_k2_v2c2_g9", "tiny_full_k2_v2c3_g15",
                                  "small_full_k3_v3c4_g27"])
def test_tensor_contractions_match_the_resolvent(name):
    """sum_ij conj(u_i) eps^ij u_j is eps_M for the probe sum_j u_j conj(D_j):
    checked against the resolvent w^H (H - z Delta)^-1 w (eqs. chiofh, Hetr),
    for axis, real oblique and complex u.  A tensor with its indices swapped,
    a conjugate on the wrong factor or a lost cross term fails the complex u."""
    d, r = inputs(name), oracle_run(name)
    D = d["Dcv"]
    t = X.transition_coefficients(r["XpY"], D)
    pref = X.tensor_prefactor(d)
    om = d["omega"][::97]
    eta = d["workload"].eta
    eps = X.dielectric_tensor(r["E"], t, om, eta, pref)
    rng = np.random.default_rng(7)
    us = [np.eye(3)[0], np.eye(3)[2], np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0)]
    for _ in range(3):
        u = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        us.append(u / np.linalg.norm(u))
    for u in us:
        p_u = D.conj() @ u
        ref = O.resolvent_spectrum(r["A"], r["B"], p_u, om, eta, pref)
        assert _rel(X.contract(eps, u), ref) < 1e-10, u


def test_transition_coefficients_special_cases():
    """X+Y = 1 gives t = -i conj(D); |t_j|^2 is the scalar oscillator strength
    of the probe conj(D_j) (eq. osci)."""
    d, r = inputs("tiny_full_k2_v2c3_g15"), oracle_run("tiny_full_k2_v2c3_g15")
    D = d["Dcv"]
    n = D.shape[0]
    assert np.array_equal(X.transition_coefficients(np.eye(n), D), -1j * D.conj())
    t = X.transition_coefficients(r["XpY"], D)
    for j in range(3):
        assert _rel(np.abs(t[:, j]) ** 2, O.oscillator(r["XpY"], D[:, j].conj())) < 1e-12


def test_single_direction_tensor_is_the_scalar_spectrum():
    rng = np.random.default_rng(3)
    E = np.sort(rng.uniform(1.0, 5.0, 40))
    t = rng.standard_normal((40, 1)) + 1j * rng.standard_normal((40, 1))
    om = np.linspace(0.0, 6.0, 50)
    eps = X.dielectric_tensor(E, t, om, 0.05, 3.0)[:, 0, 0]
    assert _rel(eps, O.spectrum(E, np.abs(t[:, 0]) ** 2, om, 0.05, 3.0)) < 1e-14


def _single_pole(E0, f, pref):
    """a = 2 E0 pref f: eps = 1 + a / (E0^2 - z^2), 1/eps = 1 - a / (E_L^2 - z^2)
    with E_L^2 = E0^2 + a (the loss peak sits at the shifted pole E_L)."""
    a = 2.0 * E0 * pref * f
    return a, np.sqrt(E0 ** 2 + a)


def test_single_pole_loss_function_closed_form():
    E0, f, pref, eta = 2.0, 0.3, 1.7, 0.02
    a, EL = _single_pole(E0, f, pref)
    om = np.linspace(0.0, 8.0, 801)
    eps = X.dielectric_tensor(np.array([E0]), np.array([[np.sqrt(f)]]), om, eta, pref)[:, 0, 0]
    z = om + 1j * eta
    closed = np.imag(a / (EL ** 2 - z ** 2))
    loss = X.loss_function(eps)
    assert _rel(loss, closed) < 1e-12
    assert np.all(loss[1:] > 0.0)
    assert abs(om[np.argmax(loss)] - EL) < 0.011  # grid step 0.01


def test_dynamic_structure_factor_f_sum_rule():
    """int_0^inf w S(Q, w) dw -> (pi/2) a / (pi v) = a / (2 v) as eta -> 0 (the
    f-sum rule of the loss function of a single pole)."""
    E0, f, pref, v = 1.5, 0.2, 2.5, 4.0
    a, EL = _single_pole(E0, f, pref)
    eta = 1e-4

    def wS(w):
        e = X.dielectric_tensor(np.array([E0]), np.array([[np.sqrt(f)]]), np.array([w]), eta,
                                pref)[0, 0, 0]
        return w * X.dynamic_structure_factor(np.array([e]), v)[0]

    lo = integrate.quad(wS, 0.0, EL - 0.5, limit=200)[0]
    mid = integrate.quad(wS, EL - 0.5, EL + 0.5, points=[EL], limit=400)[0]
    hi = integrate.quad(wS, EL + 0.5, np.inf, limit=200)[0]
    assert abs((lo + mid + hi) - a / (2.0 * v)) < 2e-3 * a / (2.0 * v)


def test_tensor_prefactor_is_the_small_q_limit_of_the_scalar_path():
    """With M_a(G=0, q) = i q sum_j qhat_j D_aj (eq. mofd) the scalar path at
    momentum q (probe conj M, prefactor 2 kappa v(q), v(q) = 4 pi / q^2) gives
    qhat^T eps qhat of the tensor path for every |q|: the 1/q^2 cancels."""
    from dataclasses import replace
    d, r = inputs("tiny_full_k2_v2c3_g15"), oracle_run("tiny_full_k2_v2c3_g15")
    D = d["Dcv"]
    om, eta = d["omega"][::50], d["workload"].eta
    t = X.transition_coefficients(r["XpY"], D)
    eps = X.dielectric_tensor(r["E"], t, om, eta, X.tensor_prefactor(d))
    qhat = np.array([0.6, 0.0, 0.8])
    for qlen in (1e-3, 0.2):
        dq = dict(d)
        dq["workload"] = replace(d["workload"], q=tuple(qlen * qhat))
        M0 = 1j * qlen * (D @ qhat)
        scalar = O.spectrum(r["E"], O.oscillator(r["XpY"], M0.conj()), om, eta,
                            O.spectrum_prefactor(dq))
        assert _rel(scalar, X.contract(eps, qhat)) < 1e-12, qlen
