"""Tile choices from a tuning table change rounding order only: parity with the
oracle holds for every choice of every tunable site (FP64 path)."""
import numpy as np
import pytest

from tests._cache import inputs, oracle_run

pytestmark = pytest.mark.gpu

SITES = ("gemm_squared", "gemm_potrf", "gemm_her2k", "gemm_exchange")


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
