"""The library's Coulomb potential without the macroscopic term (bse_coulomb,
paper Sec. 4.2, eq. vbar_def) and probe vector (bse_probe, Sec. 4.4, eq. osci)
against the oracle's, element by element: the same G_Q, vbar to the last
rounding of 4 pi / |G + q|^2, the probe exactly (a gather).  Workloads at
Q = 0 and at finite Q (batch members up to |Q| = 1.5 bohr^-1, where G_Q is
still G = 0 or a neighbour)."""
import numpy as np
import pytest

from _cache import inputs
from oracle import bse_oracle as O

pytestmark = pytest.mark.gpu


def _members(name):
    from bse_synth import BATCHES, make_batch_inputs
    return make_batch_inputs(BATCHES[name])


def _cases():
    yield inputs("tiny_full_k2_v2c3_g15")
    yield inputs("mid_full_k4_v3c4_g59")
    for d in _members("batch4_k2_g15"):
        yield d
    for d in _members("batch16_k6_g89")[::5]:
        yield d


def test_coulomb_and_probe_match_the_oracle():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_05575_amd import _lib as L
    for d in _cases():
        w = d["workload"]
        print(f"[gpu] bse_coulomb / bse_probe: {w.name} Q = {w.q}", flush=True)
        g = torch.from_numpy(np.ascontiguousarray(d["gvec"], dtype=np.int32)).cuda()
        vbar = torch.empty(w.ng, dtype=torch.float64, device="cuda")
        gq = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        mcv = torch.from_numpy(np.ascontiguousarray(d["Mcv"])).cuda()
        probe = torch.empty(w.n, dtype=torch.complex128, device="cuda")
        s = torch.cuda.current_stream().cuda_stream
        L.bse_coulomb(w.ng, g.data_ptr(), d["alat"], w.q, vbar.data_ptr(), gq.data_ptr(), s)
        L.bse_probe(w.n, w.ng, mcv.data_ptr(), gq.data_ptr(), probe.data_ptr(), s)
        torch.cuda.synchronize()
        ref = O.coulomb_vbar(d)
        assert int(gq.item()) == O.g_of_q(d), w.name
        v = vbar.cpu().numpy()
        assert v[O.g_of_q(d)] == 0.0
        assert np.abs(v - ref).max() <= 4e-16 * np.abs(ref).max(), w.name
        assert np.array_equal(probe.cpu().numpy(), O.probe(d)), w.name
