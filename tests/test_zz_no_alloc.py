"""bse_solve_noalloc (the solve with its scratch space in the library's fixed
device array) against bse_solve with a caller's workspace, through the C ABI.

Two calls in a row on the same GPU, the second with a smaller problem, so
that the second runs on an array still holding the first call's contents.
Both entry points run the same kernels in the same order on the same inputs,
so their outputs must agree bit for bit (every reduction of the solve has a
fixed order).  A problem whose workspace exceeds the array is refused.
"""
import pytest

pytestmark = pytest.mark.gpu

CASES = ("mid_full_k4_v3c4_g59", "small_full_k3_v3c4_g27", "tda_q0_k4_v2c3_g59")


def _noalloc(L, P, H0, H1, vectors):
    import torch
    n = P.n
    E = torch.empty(n, dtype=torch.float64, device=P.device)
    XpY = torch.empty((n, n), dtype=torch.complex128, device=P.device) if vectors else None
    osc = torch.empty(n, dtype=torch.float64, device=P.device)
    L.bse_solve_noalloc(P.desc, H0.data_ptr(), H1.data_ptr() if H1 is not None else 0,
                        E.data_ptr(), XpY.data_ptr() if XpY is not None else 0, 0, n,
                        P.t["probe"].data_ptr(), osc.data_ptr(), P.info.data_ptr(), P.stream())
    return E, XpY, osc


@pytest.mark.parametrize("vectors", [False, True])
def test_noalloc_matches_workspace_path(vectors):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_05575_amd import _lib as L
    from paper_1904_05575_amd.bse import Problem
    from tests._cache import inputs
    for name in CASES:  # largest first: the later calls reuse a dirty array
        print(f"[gpu] no-alloc solve {name} vectors={vectors}", flush=True)
        P = Problem(inputs(name))
        H0, H1 = P.build()
        G0, G1 = H0.clone(), (H1.clone() if H1 is not None else None)
        E, XpY, osc = P.solve(H0, H1, vectors=vectors)
        P.check_info()
        E2, XpY2, osc2 = _noalloc(L, P, G0, G1, vectors)
        P.check_info()
        assert torch.equal(E, E2) and torch.equal(osc, osc2), name
        if vectors:
            assert torch.equal(XpY, XpY2), name
        del P, H0, H1, G0, G1


def test_noalloc_refuses_large_problem():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_05575_amd import _lib as L
    n = 1536
    d = L.BseDesc(nk=128, nv=3, nc=4, ng=27, coupling=L.BSE_FULL, type=0, prec=0,
                  split_terms=0, kappa=1.0, scissor=0.0, ld=n)
    assert L.bse_workspace_size(d, L.BSE_STAGE_SOLVE) > L.NOALLOC_SCRATCH_BYTES
    with pytest.raises(L.BseError, match="BSE_ERR_WORKSPACE"):
        L.bse_solve_noalloc(d, 1, 1, 1, 0, 0, n, 1, 1, 1, 0)
