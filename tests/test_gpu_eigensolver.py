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
