"""Batched finite-Q problems replayed as one HIP graph, against the oracle."""
import contextlib

import numpy as np
import pytest

from oracle import bse_oracle as O

pytestmark = pytest.mark.gpu


def _members(name):
    from bse_synth import BATCHES, make_batch_inputs
    return make_batch_inputs(BATCHES[name])


def _batch(members, precision="fp64", nbranch=3):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_05575_amd.batch import Batch
    return Batch(members, precision=precision, nbranch=nbranch)


@contextlib.contextmanager
def _sweep_choice(choice, align=None):
    """The stored tuning table with its batched-sweep entries replaced by
    `choice` for every size (0: each problem's own hemv grid, whose values are
    those of the problem's own sweep bit for bit), and, if given, its
    start-alignment entries by `align`."""
    from paper_1904_05575_amd import _lib as L
    from paper_1904_05575_amd import tune
    tune.load()
    old = L.bse_tune_get()
    sites = {L.TUNE_SITES["batch_sweep"]: choice}
    if align is not None:
        sites[L.TUNE_SITES["batch_align"]] = align
    try:
        L.bse_tune_set([e for e in old if e[0] not in sites] +
                       [(site, 1 << 20, c) for site, c in sites.items()])
        yield
    finally:
        L.bse_tune_set(old)


@pytest.mark.parametrize("name", ["batch4_k2_g15", "batch18_k2_g15", "batch3_k1_g9"])
def test_batched_sweeps_ending_together(name):
    """Each problem's sweep started late so that all end together (tuning site
    batch_align): with each problem's own hemv grid every member's E, osc and
    eps equal the plain entry points bit for bit; with the hemv blocks shared
    among the problems a replay repeats its bits and the members agree with the
    plain entry points to rounding.  Uneven orders, two groups of launches
    (18 problems) and the smallest orders (N = 1, 2, 6)."""
    ms = _members(name)
    print(f"[gpu] sweeps ending together {name}: sizes {[m['workload'].n for m in ms]}",
          flush=True)
    with _sweep_choice(0, align=1):
        B = _batch(ms, nbranch=len(ms))
        B.run()
        own = B.results()
        B.run_sequential()
        seq = B.results()
        B.close()
    for i, (a, b) in enumerate(zip(own, seq)):
        for key in ("E", "osc", "eps"):
            assert np.array_equal(a[key], b[key]), (i, key)
    with _sweep_choice(4, align=1):
        B = _batch(ms, nbranch=len(ms))
        B.run()
        sh = B.results()
        B.run()
        again = B.results()
        B.close()
    for i in range(len(ms)):
        for key in ("E", "osc", "eps"):
            assert np.array_equal(sh[i][key], again[i][key]), (i, key)
        assert np.abs(sh[i]["E"] - seq[i]["E"]).max() <= 1e-12 * seq[i]["E"].max(), i
        assert np.abs(sh[i]["eps"] - seq[i]["eps"]).max() <= 1e-10 * np.abs(
            seq[i]["eps"] - 1).max(), i


@pytest.mark.parametrize("nbranch", [3, 16])
@pytest.mark.parametrize("name", ["batch4_k2_g15", "batch3_k3_g27"])
def test_graph_batch_matches_oracle(name, nbranch):
    """Each member's E and eps against the oracle (1e-10); with one branch per
    problem (nbranch >= members) the Householder sweeps run batched."""
    ms = _members(name)
    print(f"[gpu] batch {name} nbranch {nbranch}: sizes {[m['workload'].n for m in ms]}",
          flush=True)
    B = _batch(ms, nbranch=nbranch)
    B.run()
    res = B.results()
    for d, out in zip(ms, res):
        r = O.run(d)
        eig = np.abs(out["E"] - r["E"]).max() / np.abs(r["E"]).min()
        spec = np.abs(out["eps"] - r["eps"]).max() / np.abs(r["eps"] - 1).max()
        assert eig < 1e-10 and spec < 1e-10, (d["workload"].name, eig, spec)


def test_graph_replays_and_sequential_path_agree():
    """Several replays with eager work and synchronisation between them, and
    the plain entry points one problem after another, give identical results."""
    torch = pytest.importorskip("torch")
    ms = _members("batch3_k3_g27")
    B = _batch(ms, nbranch=2)
    B.run()
    first = B.results()
    for _ in range(3):
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        B.run()
        again = B.results()
        for a, b in zip(first, again):
            assert np.array_equal(a["E"], b["E"]) and np.array_equal(a["eps"], b["eps"])
    B.run_sequential()
    seq = B.results()
    for a, b in zip(first, seq):
        assert np.array_equal(a["E"], b["E"]) and np.array_equal(a["eps"], b["eps"])


def test_batched_sweep_reproduces_per_problem_sweeps():
    """Uneven sizes (short last panels at different steps, problems finishing
    early).  With each problem's own hemv grids (tuning choice 0, the default)
    the graph with the batched sweep (one branch per problem), the graph with
    per-branch sweeps and the plain entry points give identical E, osc and eps;
    with the blocks shared among the problems (choices 1, 2, 4) the batched
    graph repeats its own bits on replay and matches the others to rounding."""
    ms = _members("batch4_k2_g15")
    print(f"[gpu] batched sweep: sizes {[m['workload'].n for m in ms]}", flush=True)
    with _sweep_choice(0):
        Bb = _batch(ms, nbranch=len(ms))
        Bb.run()
        bat = Bb.results()
        Bp = _batch(ms, nbranch=2)
        Bp.run()
        per = Bp.results()
        Bb.run_sequential()
        seq = Bb.results()
        for i in range(len(ms)):
            for other in (per[i], seq[i]):
                for key in ("E", "osc", "eps"):
                    assert np.array_equal(bat[i][key], other[key]), (i, key)
        Bb.close()
        Bp.close()
    for per_cu in (1, 2, 4):
        with _sweep_choice(per_cu):
            Bs = _batch(ms, nbranch=len(ms))
            Bs.run()
            sh = Bs.results()
            Bs.run()
            for i in range(len(ms)):
                a = Bs.results()[i]
                assert np.array_equal(a["E"], sh[i]["E"]) and np.array_equal(a["eps"], sh[i]["eps"])
                assert np.abs(sh[i]["E"] - seq[i]["E"]).max() < 1e-12 * seq[i]["E"].max(), (per_cu, i)
                assert np.abs(sh[i]["eps"] - seq[i]["eps"]).max() < 1e-10 * np.abs(
                    seq[i]["eps"] - 1).max(), (per_cu, i)
            Bs.close()


@pytest.mark.parametrize("name", ["batch18_k2_g15", "batch5_tda_k2_g15", "batch3_k1_g9"])
def test_batched_stages_in_groups_and_tda(name):
    """One branch per problem, so the factorisations and sweeps run batched: 18
    problems (two groups of batched launches), Tamm-Dancoff problems (no
    factorisation) and the smallest orders (N = 1, 2, 6).  Each member against
    the oracle (1e-10) with the stored tuning table (a replay repeating its
    bits), and, with each problem's own hemv grids, bit for bit equal to the
    plain entry points one problem after another."""
    ms = _members(name)
    print(f"[gpu] batched stages {name}: sizes {[m['workload'].n for m in ms]}", flush=True)
    B = _batch(ms, nbranch=len(ms))
    B.run()
    res = B.results()
    for d, out in zip(ms, res):
        r = O.run(d)
        eig = np.abs(out["E"] - r["E"]).max() / np.abs(r["E"]).min()
        spec = np.abs(out["eps"] - r["eps"]).max() / np.abs(r["eps"] - 1).max()
        assert eig < 1e-10 and spec < 1e-10, (d["workload"].name, eig, spec)
    B.run()
    for i, (a, b) in enumerate(zip(res, B.results())):
        for key in ("E", "osc", "eps"):
            assert np.array_equal(a[key], b[key]), (i, key)
    B.close()
    with _sweep_choice(0):
        B = _batch(ms, nbranch=len(ms))
        B.run()
        own = B.results()
        B.run_sequential()
        for i, (a, b) in enumerate(zip(own, B.results())):
            for key in ("E", "osc", "eps"):
                assert np.array_equal(a[key], b[key]), (i, key)
        B.close()


def test_graph_batch_mixed_precision():
    ms = _members("batch3_k3_g27")
    B = _batch(ms, precision="bf16x6")
    B.run()
    for d, out in zip(ms, B.results()):
        r = O.run(d)
        assert np.abs(out["E"] - r["E"]).max() / np.abs(r["E"]).min() < 1e-6
        assert np.abs(out["eps"] - r["eps"]).max() / np.abs(r["eps"] - 1).max() < 1e-4


def test_full_size_batch_sum_rules():
    """16 momentum transfers, N = 1296..5184, one graph: every member's E is
    positive and ascending, Im eps >= 0, and for three members the f-sum rule
    sum E |t|^2 = p^H (A-B) p holds with A-B from the oracle's blocks; a
    replay gives identical results and the sequential path the same to
    rounding (the stored table shares the batched hemv blocks among the
    problems); with each problem's own hemv grids the graph and the sequential
    path agree bit for bit."""
    ms = _members("batch16_k6_g89")
    print(f"[gpu] batch16: sizes {[m['workload'].n for m in ms]}", flush=True)
    B = _batch(ms, nbranch=16)  # the benchmark's launch configuration
    B.run()
    res = B.results()
    for d, out in zip(ms, res):
        assert out["E"][0] > 0 and np.all(np.diff(out["E"]) >= 0)
        assert np.all(out["eps"].imag[1:] > -1e-12 * np.abs(out["eps"]).max())
    for idx in (0, 5, 11):
        d, out = ms[idx], res[idx]
        w = d["workload"]
        nvnc = w.nv * w.nc
        sel = np.arange(w.npairs)
        _, AmBb = O.kernel_blocks(d, sel)
        p = O.probe(d).reshape(w.nk, nvnc)
        ik, jk = np.triu_indices(w.nk)
        fs = 0.0
        for t in range(len(sel)):
            i, j = ik[t], jk[t]
            blk = AmBb[t]
            if i == j:
                U = np.triu(blk, 1)
                blk = U + U.conj().T + np.diag(blk.diagonal().real)
                fs += np.vdot(p[i], blk @ p[j]).real
            else:
                fs += 2.0 * np.vdot(p[i], blk @ p[j]).real
        assert abs(np.sum(out["E"] * out["osc"]) - fs) < 1e-9 * fs, (idx, fs)
    B.run()
    for i, (a, b) in enumerate(zip(res, B.results())):
        assert np.array_equal(a["E"], b["E"]) and np.array_equal(a["osc"], b["osc"]), i
    B.run_sequential()
    for i, (a, b) in enumerate(zip(res, B.results())):
        assert np.abs(a["E"] - b["E"]).max() < 1e-12 * b["E"].max(), i
        assert np.abs(a["osc"] - b["osc"]).max() < 1e-9 * b["osc"].max(), i
        assert np.abs(a["eps"] - b["eps"]).max() < 1e-10 * np.abs(b["eps"] - 1).max(), i
    B.close()
    # with each problem's own hemv grids, sixteen problems in one batched sweep
    # change the timing only: the plain entry points one problem after another
    # reproduce every bit (a kernel whose blocks read what another block of it
    # writes would not)
    with _sweep_choice(0):
        B = _batch(ms, nbranch=16)
        B.run()
        own = B.results()
        B.run_sequential()
        for i, (a, b) in enumerate(zip(own, B.results())):
            assert np.array_equal(a["E"], b["E"]) and np.array_equal(a["osc"], b["osc"]), i
        B.close()


def test_concurrent_streams_reproduce_the_sequential_path():
    """The plain entry points on four streams at once (each with its own
    workspace slice), largest problems of batch16 first: every bit equals the
    sequential path (no kernel reads what another of its blocks writes)."""
    torch = pytest.importorskip("torch")
    from paper_1904_05575_amd import _lib as L
    ms = _members("batch16_k6_g89")
    B = _batch(ms, nbranch=4)
    B.run_sequential()
    seq = B.results()
    slice_b = L.bse_batch_workspace_size(B.descs, 1)
    streams = [torch.cuda.Stream() for _ in range(4)]
    wss = [torch.empty(slice_b, dtype=torch.uint8, device="cuda") for _ in range(4)]
    order = sorted(range(len(ms)), key=lambda i: -ms[i]["workload"].n)[:8]
    print(f"[gpu] concurrent streams: members {order}", flush=True)
    torch.cuda.synchronize()
    for k, i in enumerate(order):
        s = streams[k % 4]
        t, d = B.t[i], B.descs[i]
        n = int(d.nk * d.nv * d.nc)
        info = B.info.data_ptr() + 4 * i
        L.bse_build(d, B.inputs[i], t["H0"].data_ptr(), t["H1"].data_ptr(), wss[k % 4].data_ptr(),
                    slice_b, info, s.cuda_stream)
        L.bse_solve(d, t["H0"].data_ptr(), t["H1"].data_ptr(), t["E"].data_ptr(), 0, 0, n,
                    t["probe"].data_ptr(), t["osc"].data_ptr(), wss[k % 4].data_ptr(), slice_b,
                    info, s.cuda_stream)
    torch.cuda.synchronize()
    conc = B.results()
    for i in order:
        assert np.array_equal(conc[i]["E"], seq[i]["E"]), i
        assert np.array_equal(conc[i]["osc"], seq[i]["osc"]), i
