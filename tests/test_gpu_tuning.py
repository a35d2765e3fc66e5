"""Tile choices from a tuning table change rounding order only: parity with the
oracle holds for every choice of every tunable site (FP64 path)."""
import numpy as np
import pytest

from tests._cache import inputs, oracle_run

pytestmark = pytest.mark.gpu

SITES = ("gemm_squared", "gemm_squared_s", "gemm_potrf", "gemm_her2k", "gemm_exchange")


@pytest.mark.parametrize("unit,tile", [(1, 32), (8, 64), (2, 16)])
@pytest.mark.parametrize("name", ["mid_full_k4_v3c4_g59", "tda_q0_k4_v2c3_g59"])
def test_parity_under_forced_tile_choices(name, unit, tile):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_05575_amd import _lib as L
    from paper_1904_05575_amd.bse import Problem
    print(f"[gpu] {name} unit {unit} tile {tile}", flush=True)
    P = Problem(inputs(name))
    old = L.bse_tune_get()
    try:
        n = 1 << 20
        table = [(L.TUNE_SITES["hemv_unit"], n, unit), (L.TUNE_SITES["gemm_stage2"], n, 16)]
        table += [(L.TUNE_SITES[s], n, tile) for s in SITES]
        L.bse_tune_set(table)
        out = P.run()
    finally:
        L.bse_tune_set(old)
    r = oracle_run(name)
    eig = np.abs(out["E"] - r["E"]).max() / np.abs(r["E"]).min()
    spec = np.abs(out["eps"] - r["eps"]).max() / np.abs(r["eps"] - 1).max()
    assert eig < 1e-10 and spec < 1e-10, (eig, spec)


@pytest.mark.parametrize("choice", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9])
@pytest.mark.parametrize("name", ["mid_full_k4_v3c4_g59", "tda_q0_k4_v2c3_g59",
                                  "tiny_full_k2_v2c3_g15", "small_full_k3s_v3c4_g27",
                                  "small_full_k3_v3c4_g113", "tiny_full_k2_v3c4_g51"])
def test_direct_term_paths(name, choice):
    """The FP64 direct terms through the two-pass path (choice 0), the three
    fused variants (1-3), the three Gauss first products writing T (4-6), the
    two unpadded ones (7, 8) and the one pass with both products on the matrix
    cores (9): the assembled matrices against the oracle (1e-12 of max|H|, sums
    of <= 2 N_G products) and the same spectrum.  N_G = 113 and 51 take the
    vector-ALU columns and k (one and three of each), 59 and 27 the padded last
    tile and the k tail, 15 falls back to choice 4; the N_v = 2 workloads take
    7 in place of 9 (pair blocks of 4 and 6 rows)."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_05575_amd import _lib as L
    from paper_1904_05575_amd.bse import Problem
    print(f"[gpu] {name} direct choice {choice}", flush=True)
    P = Problem(inputs(name))
    old = L.bse_tune_get()
    try:
        L.bse_tune_set([(L.TUNE_SITES["direct"], 1 << 20, choice)])
        H0, H1 = P.build()
        P.check_info()
        r = oracle_run(name)
        ref0 = r["A"] if r["B"] is None else r["A"] + r["B"]
        assert np.abs(H0.T.cpu().numpy() - ref0).max() < 1e-12 * np.abs(ref0).max()
        if r["B"] is not None:
            ref1 = r["A"] - r["B"]
            assert np.abs(H1.T.cpu().numpy() - ref1).max() < 1e-12 * np.abs(ref1).max()
        out = P.run()
    finally:
        L.bse_tune_set(old)
    eig = np.abs(out["E"] - r["E"]).max() / np.abs(r["E"]).min()
    spec = np.abs(out["eps"] - r["eps"]).max() / np.abs(r["eps"] - 1).max()
    assert eig < 1e-10 and spec < 1e-10, (eig, spec)


@pytest.mark.parametrize("products", [3, 4])
@pytest.mark.parametrize("name", ["mid_full_k4_v3c4_g59", "tda_q0_k4_v2c3_g59"])
def test_gemm_products(name, products):
    """Every complex GEMM (exchange, Cholesky, squared form, Householder
    updates, back-transform) with three (Gauss) or four real products per
    complex one: eigenvalues and spectrum against the oracle (1e-10), and the
    eigenvectors through their residual."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_05575_amd import _lib as L
    from paper_1904_05575_amd.bse import Problem
    print(f"[gpu] {name} gemm products {products}", flush=True)
    P = Problem(inputs(name))
    old = L.bse_tune_get()
    try:
        L.bse_tune_set([(L.TUNE_SITES["gemm_products"], 1 << 20, products)])
        out = P.run(vectors=True)
    finally:
        L.bse_tune_set(old)
    r = oracle_run(name)
    eig = np.abs(out["E"] - r["E"]).max() / np.abs(r["E"]).min()
    spec = np.abs(out["eps"] - r["eps"]).max() / np.abs(r["eps"] - 1).max()
    assert eig < 1e-10 and spec < 1e-10, (eig, spec)
    A, B, E, X = r["A"], r["B"], out["E"], out["XpY"]
    if B is None:
        assert np.abs(A @ X - X * E).max() < 1e-11 * E.max()
    else:
        assert np.abs((A - B) @ ((A + B) @ X) - X * E ** 2).max() < 1e-10 * E.max() ** 2


@pytest.mark.parametrize("tile", [16, 32, 64])
def test_vectors_under_forced_tile_choices(tile):
    """The eigenvector path's products (back-transform, X+Y = U^H Z, the
    triangular solve for X-Y) under every tile edge of their site: the coupled
    equations (A+B)(X+Y) = (X-Y)E and (A-B)(X-Y) = (X+Y)E with the oracle's
    A and B, the normalisation (X+Y)^H (X-Y) = I and the oracle's eigenvalues.
    N = 768 spans three 256-row blocks of the solve and three reflector groups."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_05575_amd import _lib as L
    from paper_1904_05575_amd.bse import Problem
    name = "mid_full_k4_v3c4_g59"
    print(f"[gpu] {name} vectors tile {tile}", flush=True)
    P = Problem(inputs(name))
    old = L.bse_tune_get()
    try:
        L.bse_tune_set([(L.TUNE_SITES["gemm_vectors"], 1 << 20, tile)])
        H0, H1 = P.build()
        E, XpY, XmY, _ = P.solve(H0, H1, xmy=True)
        P.check_info()
    finally:
        L.bse_tune_set(old)
    E, XpY, XmY = E.cpu().numpy(), XpY.T.cpu().numpy(), XmY.T.cpu().numpy()
    r = oracle_run(name)
    A, B = r["A"], r["B"]
    n, scale = len(E), E.max()
    assert np.abs(E - r["E"]).max() / np.abs(r["E"]).min() < 1e-10
    assert np.abs((A + B) @ XpY - XmY * E).max() < 1e-10 * scale
    assert np.abs((A - B) @ XmY - XpY * E).max() < 1e-10 * scale
    assert np.abs(XpY.conj().T @ XmY - np.eye(n)).max() < 1e-10
