"""GPU: the solve path on prescribed Hermitian matrices (TDA form), against LAPACK.

bse_solve is handed a matrix built here instead of an assembled one, so the
Householder reduction and the tridiagonal eigensolver meet spectra with the
structure that stresses them: near-degenerate pairs (Wilkinson's W21+),
eigenvalues of multiplicity three, split (block-diagonal) matrices and the
smallest orders.  Eigenvalues are compared with numpy.linalg.eigh; the
oscillator strengths |v^H p|^2 through sums over groups of eigenvalues closer
than 1e-4 ||A|| (rotations inside a group leave the sum unchanged, and mixing
with eigenvectors outside it is at most eps n ||A|| / gap); with vectors, the
residual and the orthonormality.  Eigenvectors of eigenvalues that are close
but not treated as one cluster (relative gap above 1e-5) are orthogonal to
about eps ||A|| / gap, hence the 1e-8 bound there.
"""
from dataclasses import replace

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _problem(nv, nc):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from bse_synth import get, make_inputs
    from paper_1904_05575_amd.bse import Problem
    w = replace(get("tiny_tda_k2_v2c2_g9"), mesh=1, nv=nv, nc=nc, name=f"prescribed_{nv}x{nc}")
    return Problem(make_inputs(w))


def _wilkinson(m):
    h = (m - 1) // 2
    return np.diag(np.abs(np.arange(-h, h + 1)).astype(float)) + np.diag(np.ones(m - 1), 1) \
        + np.diag(np.ones(m - 1), -1)


def _matrices():
    rng = np.random.default_rng(5)
    out = {}
    out["n1"] = (1, 1, np.array([[2.5]], dtype=complex))
    out["n2"] = (1, 2, np.array([[1.0, 0.3 - 0.2j], [0.3 + 0.2j, 1.5]]))
    out["wilkinson21"] = (3, 7, _wilkinson(21).astype(complex))
    q, _ = np.linalg.qr(rng.normal(size=(24, 24)) + 1j * rng.normal(size=(24, 24)))
    lam = np.r_[[1.0] * 3, [2.0] * 3, np.linspace(3.0, 9.0, 18)]
    out["triple24"] = (4, 6, (q * lam) @ q.conj().T)
    # five shifted copies of W21+ glued by 1e-9 (nearly split, many close pairs),
    # and the same blocks made dense by adding 0.37 b to every entry of block b
    for name, dense in (("glued105", False), ("blocks105", True)):
        a = np.zeros((105, 105))
        for b in range(5):
            shift = 0.37 * b * (np.ones((21, 21)) if dense else np.eye(21))
            a[21 * b:21 * (b + 1), 21 * b:21 * (b + 1)] = _wilkinson(21) + shift
        for b in range(4):
            a[21 * b + 20, 21 * b + 21] = a[21 * b + 21, 21 * b + 20] = 1e-9
        out[name] = (5, 21, a.astype(complex))
    d = np.r_[np.arange(1.0, 7.0), np.arange(1.0, 7.0)]
    out["diag12"] = (2, 6, np.diag(d).astype(complex))
    return out


MATS = _matrices()


def _solve(name, vectors):
    import torch
    nv, nc, a = MATS[name]
    a = 0.5 * (a + a.conj().T)
    P = _problem(nv, nc)
    n = P.n
    assert a.shape == (n, n)
    H0 = torch.tensor(a.T.copy(), dtype=torch.complex128, device="cuda")  # column-major
    print(f"[gpu] prescribed {name} n={n} vectors={vectors}", flush=True)
    E, XpY, osc = P.solve(H0, None, vectors=vectors)
    P.check_info()
    p = P.t["probe"].cpu().numpy()
    out = {"E": E.cpu().numpy(), "osc": osc.cpu().numpy(), "a": a, "p": p}
    if vectors:
        out["X"] = XpY.T.cpu().numpy()
    return out


def _clusters(e, tol):
    groups, cur = [], [0]
    for k in range(1, len(e)):
        if e[k] - e[k - 1] <= tol:
            cur.append(k)
        else:
            groups.append(cur)
            cur = [k]
    groups.append(cur)
    return groups


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("vectors", [False, True])
def test_prescribed_spectra(name, vectors):
    r = _solve(name, vectors)
    a, e, osc, p = r["a"], r["E"], r["osc"], r["p"]
    scale = np.abs(a).max()
    w, v = np.linalg.eigh(a)
    assert np.all(np.diff(e) >= 0)
    assert np.abs(e - w).max() <= 1e-12 * scale * len(e)
    # oscillator strengths summed over clusters of (numerically) equal eigenvalues
    ref = np.abs(v.conj().T @ p) ** 2
    pn2 = float(np.vdot(p, p).real)
    for g in _clusters(w, 1e-4 * scale):
        s, s_ref = osc[g].sum(), ref[g].sum()
        assert abs(s - s_ref) <= 1e-9 * pn2, (name, g, s, s_ref)
    if vectors:
        x = r["X"]
        assert np.abs(a @ x - x * e).max() <= 1e-11 * scale * len(e)
        assert np.abs(x.conj().T @ x - np.eye(len(e))).max() <= 1e-8


def _reflect(a, v):
    """H a H with H = I - 2 v v^H (|v| = 1), in O(n^2)."""
    av = a @ v
    vha = v.conj() @ a
    c = v.conj() @ av
    return (a - 2.0 * np.outer(v, vha) - 2.0 * np.outer(av, v.conj())
            + 4.0 * c * np.outer(v, v.conj()))


@pytest.mark.parametrize("nc", [3328, 4160])
def test_order_beyond_lds_staging_known_spectrum(nc):
    """n = 6656, above the order whose shared rows the eigenvector kernel keeps
    in LDS, and n = 8320, whose first trailing blocks have more than 128
    tile-rows, so that the Householder column kernel gathers each row's hemv
    slots in more than one round: A = Q diag(lam) Q^H with Q a product of three
    Householder reflectors, so the eigenvalues are lam and the oscillator
    strengths |(Q^H p)_l|^2 by construction.  lam holds two triples of equal
    values (the cluster path) among values spaced 3e-4 apart (2.4e-4 at
    n = 8320)."""
    torch = pytest.importorskip("torch")
    nv = 2
    P = _problem(nv, nc)
    n = P.n
    rng = np.random.default_rng(9)
    lam = np.linspace(1.0, 3.0, n)
    lam[100:103] = lam[100]
    lam[5000:5003] = lam[5000]
    perm = rng.permutation(n)
    a = np.diag(lam[perm]).astype(complex)
    p = P.t["probe"].cpu().numpy()
    vs = []
    for _ in range(3):
        v = rng.normal(size=n) + 1j * rng.normal(size=n)
        v /= np.linalg.norm(v)
        a = _reflect(a, v)
        vs.append(v)
    y = p.copy()  # A = Q D Q^H with Q = H3 H2 H1, so Q^H p = H1 H2 H3 p
    for v in vs[::-1]:
        y = y - 2.0 * v * np.vdot(v, y)
    a = 0.5 * (a + a.conj().T)
    ref_osc = np.abs(y) ** 2  # in the order of diag(lam[perm])
    H0 = torch.tensor(a.T.copy(), dtype=torch.complex128, device="cuda")
    del a
    print(f"[gpu] prescribed known-spectrum n={n}", flush=True)
    E, _, osc = P.solve(H0, None, vectors=False)
    P.check_info()
    e, o = E.cpu().numpy(), osc.cpu().numpy()
    assert np.all(np.diff(e) >= 0)
    assert np.abs(e - np.sort(lam)).max() <= 1e-12 * 3.0 * n
    order = np.argsort(lam[perm], kind="stable")
    ref = ref_osc[order]
    pn2 = float(np.vdot(p, p).real)
    for g in _clusters(np.sort(lam), 1e-6):
        assert abs(o[g].sum() - ref[g].sum()) <= 1e-9 * pn2, g
