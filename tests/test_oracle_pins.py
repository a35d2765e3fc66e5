"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each compares it with a
different route to the same quantity (literal double sums, closed forms of
special cases, the 2N non-Hermitian eigenproblem, the resolvent itself, a
LAPACK generalized eigensolver, sum rules and trace identities).
"""
from dataclasses import replace

import numpy as np
import pytest
import scipy.linalg as sl

from bse_synth import get, lattice, make_inputs
from oracle import bse_oracle as O
from tests._cache import inputs, oracle_run

TINY = ["tiny_tda_k2_v2c2_g9", "tiny_full_k2_v2c3_g15"]
SMALL = TINY + ["small_full_k3_v3c4_g27"]


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ----------------------------------------------------------------- assembly
SHIFTED = ["tiny_full_k2s_v2c3_g15", "small_full_k3s_v3c4_g27", "tiny_full_k2h_v2c3_g15"]


@pytest.mark.parametrize("name", TINY + SHIFTED[:1] + SHIFTED[2:])
def test_assembly_literal_double_sums(name):
    """Factorised per-q-class contraction == literal sums of eqs. vrrofM,
    wrrm, wrabar entry by entry."""
    d = inputs(name)
    A, B = O.assemble(d)
    A2, B2 = O.assemble(d, literal=True)
    assert _rel(A, A2) < 1e-13
    if B is not None:
        assert _rel(B, B2) < 1e-13


@pytest.mark.parametrize("name", ["small_full_k3_v3c4_g27", "small_full_k3s_v3c4_g27",
                                  "tiny_full_k2h_v2c3_g15"])
def test_q_index_against_cartesian_vectors(name):
    """The oracle's k-k' and -k-k' classes name a q-vector (of the q-mesh or,
    on a generically shifted k-mesh, of the second set) that differs from the
    Cartesian difference by a reciprocal lattice vector; the maps handed to
    the GPU agree with the oracle's."""
    d = inputs(name)
    w = d["workload"]
    n = w.mesh
    b = lattice.recip_basis()
    kc = ((d["kcoords"] + np.asarray(w.kshift)) / n) @ b
    qv = lattice.qset_cart(n, w.kshift)
    second = not np.allclose(2 * np.asarray(w.kshift), np.round(2 * np.asarray(w.kshift)))
    assert len(qv) == d["W"].shape[0] == (2 if second else 1) * w.nk
    binv = np.linalg.inv(b)
    for sign, gpu_map in ((1, d["qmap"]), (-1, d["qramap"])):
        qi = O.q_index_of(d, sign)
        assert np.array_equal(qi, gpu_map)
        for i in range(len(kc)):
            for j in range(len(kc)):
                diff = (sign * kc[i] - kc[j] - qv[qi[i, j]]) @ binv
                assert np.allclose(diff, np.round(diff), atol=1e-12)
        if sign == 1 or not second:
            assert qi.max() < w.nk
        else:
            assert qi.min() >= w.nk


def test_direct_uses_w_of_k_minus_kprime():
    """With W(q) = (q+1) * I and all pair elements equal to one, every entry of
    the (k, k') block of W^rr is (q(k-k') + 1) * NG and of W^ra (q(-k-k') + 1) * NG."""
    d = dict(inputs("tiny_full_k2_v2c3_g15"))
    w = d["workload"]
    nq, ng = d["W"].shape[0], w.ng
    d["W"] = np.stack([(q + 1.0) * np.eye(ng) for q in range(nq)]).astype(np.complex128)
    for k in ("Mvv", "Mcc", "Ncv", "Nvc"):
        d[k] = np.ones_like(d[k])
    qmap, qramap = lattice.q_maps(w.mesh)
    nvnc = w.nv * w.nc
    for which, qm in (("rr", qmap), ("ra", qramap)):
        K = O.direct(d, which).reshape(w.nk, nvnc, w.nk, nvnc)
        for i in range(w.nk):
            for j in range(i + 1, w.nk):
                assert np.allclose(K[i, :, j, :], (qm[i, j] + 1.0) * ng)


def test_direct_single_plane_wave_closed_form():
    """N_G = 1: W^rr_{(v,c),(v',c')} = W_00(k-k') M*_vv'(0) M_cc'(0)."""
    w = replace(get("tiny_full_k2_v2c3_g15"), ng=1, name="ng1")
    d = make_inputs(w)
    K = O.direct(d, "rr")
    nvnc = w.nv * w.nc
    ik, jk = np.triu_indices(w.nk)
    qm, _ = lattice.q_maps(w.mesh)
    for p, (i, j) in enumerate(zip(ik, jk)):
        for v in range(w.nv):
            for c in range(w.nc):
                for v2 in range(w.nv):
                    for c2 in range(w.nc):
                        a, b = i * nvnc + v * w.nc + c, j * nvnc + v2 * w.nc + c2
                        if a >= b:
                            continue
                        ref = d["W"][qm[i, j]][0, 0] * np.conj(d["Mvv"][p, v, v2, 0]) * \
                            d["Mcc"][p, c, c2, 0]
                        assert abs(K[a, b] - ref) < 1e-12 * abs(ref) + 1e-300


def test_exchange_rank_one_and_trace():
    """One nonzero vbar_g gives V = v_g M*(g) M(g)^T; the trace of V is
    sum_G vbar_G ||M(:, G)||^2."""
    d = inputs("tiny_full_k2_v2c3_g15")
    M = d["Mcv"]
    vb = np.zeros(M.shape[1])
    vb[3] = 2.5
    V = O.exchange(d, vb)
    ref = 2.5 * np.outer(np.conj(M[:, 3]), M[:, 3])
    assert _rel(V, ref) < 1e-14
    v = O.coulomb_vbar(d)
    V = O.exchange(d)
    assert abs(np.trace(V).real - np.sum(v * np.sum(np.abs(M) ** 2, axis=0))) < 1e-10
    assert np.linalg.eigvalsh(V)[0] > -1e-10 * np.abs(V).max()     # PSD
    assert np.linalg.matrix_rank(V, tol=1e-9 * np.abs(V).max()) <= M.shape[1] - 1


def test_vbar_and_coulomb():
    """vbar drops exactly the G_Q = 0 term at Q = 0 and is 4 pi / |G|^2 elsewhere
    (eq. vft with the Coulomb square, eq. vbar_def)."""
    d = inputs("tiny_full_k2_v2c3_g15")
    v = O.coulomb_vbar(d)
    G = lattice.gcart(15)
    assert v[0] == 0.0 and O.g_of_q(d) == 0
    assert np.allclose(v[1:], 4 * np.pi / np.sum(G[1:] ** 2, axis=1))
    assert np.isclose(O.coulomb_v0(d), 4 * np.pi / 0.01)


@pytest.mark.parametrize("name", SMALL + SHIFTED + ["tda_q0_k4_v2c3_g59"])
def test_hermitian_and_positive(name):
    """A (and B) Hermitian with real diagonal; the calibrated kernel scale keeps
    A - B and A + B (or A) positive definite with the 0.1 min(E) margin."""
    r = oracle_run(name)
    A, B = r["A"], r["B"]
    E = O.transition_energies(inputs(name))
    for M in (A,) if B is None else (A + B, A - B):
        assert np.array_equal(M, M.conj().T)
        assert np.linalg.eigvalsh(M)[0] > 0.1 * E.min()


def test_transition_energies_layout():
    d = inputs("tiny_full_k2_v2c3_g15")
    w = d["workload"]
    E = O.transition_energies(d)
    for ik in range(w.nk):
        for v in range(w.nv):
            for c in range(w.nc):
                assert E[(ik * w.nv + v) * w.nc + c] == d["eps_c"][ik, c] - d["eps_v"][ik, v]


# ----------------------------------------------------------------- solve
@pytest.mark.parametrize("name", ["tiny_full_k2_v2c3_g15", "tda_q0_k4_v2c3_g59"])
def test_two_n_brute_force(name):
    """Eigenvalues of Delta H (2N non-Hermitian, eq. gevpbse) are +-E."""
    r = oracle_run(name)
    ev, raw = O.brute_force_2n(r["A"], r["B"])
    n = len(r["E"])
    assert np.abs(raw.imag).max() < 1e-9
    assert _rel(ev[n:], r["E"]) < 1e-12
    assert _rel(-ev[:n][::-1], r["E"]) < 1e-12


def test_n1_closed_form():
    a, b = 3.0, 1.2
    E, XpY, XmY = O.solve_full(np.array([[a + 0j]]), np.array([[b + 0j]]))
    assert np.isclose(E[0], np.sqrt(a * a - b * b), rtol=1e-15)
    assert np.isclose(abs(XpY[0, 0]) ** 2, np.sqrt((a - b) / (a + b)), rtol=1e-14)


def test_coupling_zero_equals_tda():
    r = oracle_run("tiny_full_k2_v2c3_g15")
    A = r["A"]
    E, XpY, XmY = O.solve_full(A, np.zeros_like(A))
    Et, X = O.solve_tda(A)
    assert _rel(E, Et) < 1e-13
    # same projectors (gauge free)
    assert _rel(np.abs(XpY.conj().T @ X), np.eye(len(E))) < 1e-8


@pytest.mark.parametrize("name", ["tiny_full_k2_v2c3_g15", "small_full_k3_v3c4_g27"])
def test_lapack_generalized_type2(name):
    """scipy.linalg.eigh(A+B, A-B, type=2) solves (A+B)(A-B) x = E^2 x."""
    r = oracle_run(name)
    A, B = r["A"], r["B"]
    mu = sl.eigh(A + B, A - B, type=2, eigvals_only=True)
    assert _rel(np.sqrt(mu), r["E"]) < 1e-12


@pytest.mark.parametrize("name", ["tiny_full_k2_v2c3_g15", "small_full_k3_v3c4_g27"])
def test_cholesky_route_same_result(name):
    """U^H U = A - B gives the same E and X+Y as the literal (A-B)^1/2 (polar
    decomposition), with X+Y = U^H Z E^-1/2."""
    r = oracle_run(name)
    A, B = r["A"], r["B"]
    U = sl.cholesky(A - B, lower=False)
    S = U @ (A + B) @ U.conj().T
    mu, Z = np.linalg.eigh(0.5 * (S + S.conj().T))
    E = np.sqrt(mu)
    assert _rel(E, r["E"]) < 1e-12
    XpY = (U.conj().T @ Z) / np.sqrt(E)
    p = r["p"]
    assert _rel(np.abs(XpY.conj().T @ p) ** 2, r["t2"]) < 1e-9


@pytest.mark.parametrize("name", ["tiny_full_k2_v2c3_g15", "small_full_k3_v3c4_g27"])
def test_traces_residual_normalisation(name):
    r = oracle_run(name)
    A, B, E, XpY, XmY = r["A"], r["B"], r["E"], r["XpY"], r["XmY"]
    assert abs(np.sum(E ** 2) - np.trace((A - B) @ (A + B)).real) < 1e-11 * np.sum(E ** 2)
    X, Y = 0.5 * (XpY + XmY), 0.5 * (XpY - XmY)
    n = len(E)
    assert _rel(X.conj().T @ X - Y.conj().T @ Y, np.eye(n)) < 1e-11
    # H (X;Y) = E Delta (X;Y)
    assert np.abs(A @ X + B @ Y - X * E).max() < 1e-11 * E.max()
    assert np.abs(B @ X + A @ Y + Y * E).max() < 1e-11 * E.max()


def test_tda_trace():
    r = oracle_run("tda_q0_k4_v2c3_g59")
    assert abs(np.sum(r["E"]) - np.trace(r["A"]).real) < 1e-11 * np.sum(r["E"])


def test_rpa_rank_one_secular_equation():
    """gc = 0 and only the G_Q exchange (full v): A-B = diag(E),
    S = E^2 + 4 kappa v0 (E^1/2 p)(E^1/2 p)^H, whose eigenvalues solve
    1 = 4 kappa v0 sum_a E_a |p_a|^2 / (mu - E_a^2); roots found by bisection."""
    d = inputs("small_full_k3_v3c4_g27")
    gq = O.g_of_q(d)
    vb = np.zeros(d["workload"].ng)
    vb[gq] = O.coulomb_v0(d)
    A, B = O.assemble(d, "rpa", vbar=vb)
    E, XpY, _ = O.solve_full(A, B)
    Eip = O.transition_energies(d)
    p = O.probe(d)
    c = 4.0 * O.kappa(d) * O.coulomb_v0(d)
    wgt = c * Eip * np.abs(p) ** 2
    e2 = Eip ** 2
    order = np.argsort(e2)
    e2, wgt = e2[order], wgt[order]

    def f(mu):
        return 1.0 - np.sum(wgt / (mu - e2))

    roots = []
    for i in range(len(e2)):
        lo = e2[i]
        hi = e2[i + 1] if i + 1 < len(e2) else e2[-1] + np.sum(wgt) + 1.0
        if hi - lo < 1e-13 * hi:
            roots.append(hi)
            continue
        a, b = lo * (1 + 1e-15) + 1e-300, hi * (1 - 1e-15)
        for _ in range(200):
            m = 0.5 * (a + b)
            if f(m) > 0:
                b = m
            else:
                a = m
        roots.append(0.5 * (a + b))
    assert _rel(np.sqrt(np.array(roots)), E) < 1e-10


def test_ip_limit():
    """gx = gc = 0: E = sorted transition energies, |t|^2 = |p_a|^2, and the
    spectrum is the independent-particle sum."""
    d = inputs("tiny_full_k2_v2c3_g15")
    A, B = O.assemble(d, "ip")
    E, XpY, _ = O.solve_full(A, B)
    Eip = O.transition_energies(d)
    order = np.argsort(Eip)
    assert _rel(E, Eip[order]) < 1e-14
    p = O.probe(d)
    t2 = O.oscillator(XpY, p)
    assert _rel(t2, np.abs(p[order]) ** 2) < 1e-12
    om = d["omega"]
    pref, eta = O.spectrum_prefactor(d), d["workload"].eta
    ref = np.array([1 - pref * sum(abs(p[a]) ** 2 * (1 / (w - Eip[a] + 1j * eta) -
                                                     1 / (w + Eip[a] + 1j * eta))
                                   for a in range(len(p))) for w in om[:20]])
    assert _rel(O.spectrum(E, t2, om[:20], eta, pref), ref) < 1e-12


# ----------------------------------------------------------------- spectrum
@pytest.mark.parametrize("name", ["tiny_tda_k2_v2c2_g9", "tiny_full_k2_v2c3_g15",
                                  "small_full_k3_v3c4_g27", "tda_q0_k4_v2c3_g59"])
def test_eigen_sum_equals_resolvent(name):
    """The eigen-sum of eq. chir equals the plain definition
    1 + pref w^H (H - z Delta)^-1 w at z = w + i eta."""
    d = inputs(name)
    r = oracle_run(name)
    om = np.array([0.3, 1.5, 2.2, 3.7, 5.1, 8.9])
    eta = d["workload"].eta
    e1 = O.spectrum(r["E"], r["t2"], om, eta, r["pref"])
    e2 = O.resolvent_spectrum(r["A"], r["B"], r["p"], om, eta, r["pref"])
    assert _rel(e1, e2) < 1e-10


@pytest.mark.parametrize("name", ["tiny_full_k2_v2c3_g15", "small_full_k3_v3c4_g27",
                                  "tda_q0_k4_v2c3_g59"])
def test_f_sum_and_static_limit(name):
    """sum_l E_l |t_l|^2 = p^H (A-B) p and sum_l |t_l|^2 / E_l = p^H (A+B)^-1 p
    (A for both in the TDA's f-sum; (A)^-1 for the TDA's static limit)."""
    r = oracle_run(name)
    A, B, E, t2, p = r["A"], r["B"], r["E"], r["t2"], r["p"]
    AmB = A if B is None else A - B
    ApB = A if B is None else A + B
    assert abs(np.sum(E * t2) - np.vdot(p, AmB @ p).real) < 1e-11 * np.sum(E * t2)
    assert abs(np.sum(t2 / E) - np.vdot(p, np.linalg.solve(ApB, p)).real) < 1e-11 * np.sum(t2 / E)


def test_two_dielectric_routes():
    """1 / (1 + pref F_full(z)) == 1 - pref F_bar(z) (Sherman-Morrison): the
    full-v route of eq. for eps_M via P and the vbar route of eq. vbar_def."""
    d = inputs("small_full_k3_v3c4_g27")
    gq = O.g_of_q(d)
    vfull = O.coulomb_vbar(d).copy()
    vfull[gq] = O.coulomb_v0(d)
    om = np.linspace(0.5, 9.5, 37)
    eta, pref = d["workload"].eta, O.spectrum_prefactor(d)
    p = O.probe(d)
    Ab, Bb = O.assemble(d)
    Eb, Xb, _ = O.solve_full(Ab, Bb)
    eps_bar = O.spectrum(Eb, O.oscillator(Xb, p), om, eta, pref)
    Af, Bf = O.assemble(d, vbar=vfull)
    Ef, Xf, _ = O.solve_full(Af, Bf)
    Ff = (1.0 - O.spectrum(Ef, O.oscillator(Xf, p), om, eta, pref))  # = pref * F_full
    eps_full = 1.0 / (1.0 + Ff)
    assert _rel(eps_full, eps_bar) < 1e-10


def test_spectrum_retarded_sign():
    """Im eps_M >= 0 for w > 0 (absorption is positive with the retarded i delta)."""
    r = oracle_run("tda_q0_k4_v2c3_g59")
    assert np.all(r["eps"].imag[1:] > 0)


@pytest.mark.parametrize("bse_type", ["singlet", "triplet"])
def test_single_transition_closed_form(bse_type):
    """Nk = 1, one valence and one conduction band, N_G = 1 (so vbar = 0): A and
    B are numbers, A = E - gc kappa W_00 M*_vv M_cc, B = -gc kappa W_00 N*_cv N_vc,
    and the one excitation energy is sqrt(A^2 - B^2) (signs of eqs.
    diagonalblock / couplingblock)."""
    w = replace(get("tiny_full_k2_v2c3_g15"), mesh=1, nv=1, nc=1, ng=1,
                kernel_scale=1.0, name="n1")
    d = make_inputs(w)
    gc = O.BSE_TYPES[bse_type][1]
    kap = O.kappa(d)
    W00 = d["W"][0][0, 0].real
    Eip = d["eps_c"][0, 0] - d["eps_v"][0, 0]
    a = Eip - gc * kap * W00 * (np.conj(d["Mvv"][0, 0, 0, 0]) * d["Mcc"][0, 0, 0, 0]).real
    b = -gc * kap * W00 * (np.conj(d["Ncv"][0, 0, 0, 0]) * d["Nvc"][0, 0, 0, 0]).real
    A, B = O.assemble(d, bse_type)
    assert np.isclose(A[0, 0].real, a, rtol=1e-14) and np.isclose(B[0, 0].real, b, rtol=1e-14)
    if abs(b) < a:
        E, _, _ = O.solve_full(A, B)
        assert np.isclose(E[0], np.sqrt(a * a - b * b), rtol=1e-14)


def test_sampled_blocks_match_full_assembly():
    """kernel_blocks (used for sampled checks at full size) agrees with the
    assembled A+B and A-B on every pair of a small problem."""
    name = "small_full_k3_v3c4_g27"
    d = inputs(name)
    r = oracle_run(name)
    w = d["workload"]
    nvnc = w.nv * w.nc
    sel = np.arange(w.npairs)
    ApB, AmB = O.kernel_blocks(d, sel)
    ik, jk = np.triu_indices(w.nk)
    FA = (r["A"] + r["B"]).reshape(w.nk, nvnc, w.nk, nvnc)
    FM = (r["A"] - r["B"]).reshape(w.nk, nvnc, w.nk, nvnc)
    for p in sel:
        i, j = ik[p], jk[p]
        if i < j:
            assert np.abs(ApB[p] - FA[i, :, j, :]).max() < 1e-12
            assert np.abs(AmB[p] - FM[i, :, j, :]).max() < 1e-12
        else:
            iu = np.triu_indices(nvnc, 1)
            assert np.abs(ApB[p][iu] - FA[i, :, j, :][iu]).max() < 1e-12
            assert np.abs(ApB[p].diagonal().real - FA[i, :, j, :].diagonal().real).max() < 1e-12


# ----------------------------------------------------------------- finite momentum transfer
def _batch_members(name):
    from bse_synth import BATCHES, make_batch_inputs
    return make_batch_inputs(BATCHES[name])


def test_finite_q_vbar_drops_g_of_q():
    """At Q != 0, vbar removes exactly the G nearest to Q and is 4 pi/|G+q|^2
    with q = Q - G_Q elsewhere (eq. vbar_def)."""
    d = _batch_members("batch4_k2_g15")[-1]  # Q = (1.5, 0, 0)
    Q = np.asarray(d["workload"].q)
    G = lattice.gcart(15)
    gq = O.g_of_q(d)
    assert np.argmin(np.sum((G - Q) ** 2, axis=1)) == gq and gq != 0
    v = O.coulomb_vbar(d)
    q = Q - G[gq]
    keep = np.arange(15) != gq
    assert v[gq] == 0.0
    assert np.allclose(v[keep], 4 * np.pi / np.sum((G[keep] + q) ** 2, axis=1))
    assert np.isclose(O.coulomb_v0(d), 4 * np.pi / (Q @ Q))


@pytest.mark.parametrize("idx", [1, 2, 3])
def test_finite_q_members_resolvent_and_2n(idx):
    """Every member of a finite-Q batch: eigen-sum = resolvent, +-E pairs of
    the 2N problem, f-sum rule."""
    d = _batch_members("batch4_k2_g15")[idx]
    r = O.run(d)
    om = np.array([0.7, 2.1, 4.4, 8.0])
    eta = d["workload"].eta
    e1 = O.spectrum(r["E"], r["t2"], om, eta, r["pref"])
    e2 = O.resolvent_spectrum(r["A"], r["B"], r["p"], om, eta, r["pref"])
    assert _rel(e1, e2) < 1e-10
    ev, _ = O.brute_force_2n(r["A"], r["B"])
    n = len(r["E"])
    assert _rel(ev[n:], r["E"]) < 1e-12
    fs = np.vdot(r["p"], (r["A"] - r["B"]) @ r["p"]).real
    assert abs(np.sum(r["E"] * r["t2"]) - fs) < 1e-11 * fs


def test_batch_members_share_w_and_slice_pairs():
    ms = _batch_members("batch4_k2_g15")
    master = ms[0]["master"]
    for d in ms:
        w = d["workload"]
        assert d["W"] is master["W"]
        assert np.array_equal(d["Mvv"], master["Mvv"][:, :w.nv, :w.nv])
        assert np.array_equal(d["Nvc"], master["Nvc"][:, :w.nv, :w.nc])
    assert len({d["workload"].n for d in ms}) > 1  # uneven sizes
