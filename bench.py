#!/usr/bin/env python3
"""Benchmark of the BSE hot path on one MI355X.

Workload: full (non-TDA) BSE at Q = 0, k-mesh 8x8x8, 3 valence and 4
conduction bands (N = 6144, 2N = 12288), 113 plane waves, 4000 frequencies;
seeded synthetic inputs resident in HBM before the timed region.

One step = bse_build (kernel assembly) + bse_solve (squared-form Cholesky,
Householder tridiagonalisation, tridiagonal eigensolve, projection of the
probe) + bse_spectrum.  Printed metric: kernel-build TFLOP/s (algorithmic
flops of the exchange and both direct terms, 8 flops per complex
multiply-add, pairs ik <= ik') with the time to eps_M of the same steps.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def build_flops(w) -> dict:
    """Algorithmic flops of the assembly (8 per complex MAC, k-pairs ik <= ik')."""
    n, P, ng, nv, nc = w.n, w.npairs, w.ng, w.nv, w.nc
    exch = n * (n + 1) // 2 * ng * 8
    rr1 = P * nv * nv * ng * ng * 8
    rr2 = P * nv * nv * ng * nc * nc * 8
    full = w.coupling == "full"
    ra1 = P * nc * nv * ng * ng * 8 if full else 0
    ra2 = P * nc * nv * ng * nv * nc * 8 if full else 0
    return {"exchange": exch, "stage1": rr1 + ra1, "stage2": rr2 + ra2,
            "total": exch + rr1 + rr2 + ra1 + ra2}


def kernel_roofline_table(w) -> dict:
    """Per-step algorithmic work of the kernels that can dominate a step:
    (bound, amount, unit).  Bytes for HBM-bound kernels, flops for MFMA."""
    n = w.n
    f = build_flops(w)
    m = np.arange(1, n, dtype=np.float64)
    return {
        # lower triangle of the trailing Hermitian matrix (order m), one launch per reflector
        "k_trd_hemv": ("hbm", float(np.sum(m * (m + 1) / 2) * 16.0), "B"),
        "k_stage1_real": ("mfma", float(f["stage1"]), "flop"),
        "zgemm_direct_stage2": ("mfma", float(f["stage2"]), "flop"),
        "zgemm_exchange": ("mfma", float(f["exchange"]), "flop"),
        # triangular products of the squared form: n^3 / 2 complex MACs each
        "zgemm_sq_t1": ("mfma", n ** 3 / 2 * 8.0, "flop"),
        "zgemm_sq_s": ("mfma", n ** 3 / 4 * 8.0, "flop"),
        # trailing updates of the tridiagonalisation (lower triangle): m(m+1)/2 x 64 per panel
        "zgemm_her2k": ("mfma", float(np.sum(m[::32] * (m[::32] + 1) / 2)) * 64 * 8.0, "flop"),
    }


def measured_traffic(kernel: str, n: int):
    """Bytes per launch fetched by `kernel` at order n, from a committed
    rocprofv3 FETCH_SIZE summary (scaled by its copy-kernel calibration), or
    None when there is none or the kernel's source changed since it was taken."""
    import glob
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    for path in sorted(glob.glob(os.path.join(here, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("machine-readable:"):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
            if kv.get("kernel") != kernel or int(kv.get("order", -1)) != n:
                continue
            src = os.path.join(here, kv["source"])
            if hashlib.sha256(open(src, "rb").read()).hexdigest() != kv["sha256"]:
                return None
            return {"bytes": float(kv["fetch_bytes_per_launch"]),
                    "source": os.path.relpath(path, here),
                    "note": "FETCH_SIZE only (bytes read, calibrated against a 1 GiB copy); "
                            "no WRITE_SIZE count exists"}
    return None


def golden_errors(name: str, inputs, E, osc, eps):
    """Errors of a GPU result against the FP64 oracle's stored values
    (tests/golden/<name>.npz, written by tests/golden/make_golden.py from
    oracle/ only), or None when no stored values belong to these inputs."""
    path = os.path.join(ROOT, "tests", "golden", name.replace(":", "_m") + ".npz")
    if not os.path.exists(path):
        return None
    from tests.golden.make_golden import fingerprint
    with np.load(path) as z:
        g = {k: z[k] for k in z.files}
    if not np.allclose(fingerprint(inputs), g["fp"], rtol=1e-12, atol=0):
        return None
    return {"eig_rel": float(np.abs(E - g["E"]).max() / np.abs(g["E"]).min()),
            "spec_err": float(np.abs(eps - g["eps"]).max() / np.abs(g["eps"] - 1).max()),
            "reference": os.path.relpath(path, ROOT)}


def cpu_baseline(inputs, w) -> dict:
    """The FP64 oracle as it stands, timed stage by stage on bounded samples of
    the workload (about 20 s of CPU work in all):
      build    oracle kernel_blocks (exchange + W^rr + W^ra) on a strided sample
               of k-pairs, scaled to all pairs (value, in the metric's unit);
      solve    the oracle's squared-form solve (literal (A-B)^1/2, two eigh)
               of the principal sub-problem of the first k-points (its A+-B
               are principal submatrices of the workload's), scaled by N^3;
      spectrum the oracle's eigen-sum over all frequencies on that
               sub-problem's E and |t|^2, scaled by N."""
    from oracle import bse_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max(int(i.get("num_threads", 1)) for i in threadpool_info()) if threadpool_info() else 1
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    P = w.npairs
    stride = 64
    while True:
        sel = np.arange(0, P, stride)
        t0 = time.perf_counter()
        O.kernel_blocks(inputs, sel)
        dt = time.perf_counter() - t0
        if dt > 6.0 or stride == 1:
            break
        stride = max(1, stride // 4)
    f = build_flops(w)
    frac = len(sel) / P
    # exchange blocks of the sampled pairs: nvnc^2 * ng complex MACs per pair
    nvnc = w.nv * w.nc
    flops = (f["stage1"] + f["stage2"]) * frac + len(sel) * nvnc * nvnc * w.ng * 8
    build_s = f["total"] * dt / flops
    # principal sub-problem: k-points 0 .. ks-1 (N_sub = ks * nv * nc near 1536)
    ks = max(1, min(w.nk, 1536 // nvnc))
    ik, jk = np.triu_indices(w.nk)
    psel = np.nonzero(jk < ks)[0]
    ApB_b, AmB_b = O.kernel_blocks(inputs, psel)
    ns = ks * nvnc
    blocks = {}
    for M, blk in (("p", ApB_b), ("m", AmB_b)):
        K = np.zeros((ks, nvnc, ks, nvnc), dtype=np.complex128)
        K[ik[psel], :, jk[psel], :] = blk
        blocks[M] = O.hermitian_rule(K.reshape(ns, ns))
    A, B = (blocks["p"] + blocks["m"]) / 2, (blocks["p"] - blocks["m"]) / 2
    p = O.probe(inputs)[:ns]
    t0 = time.perf_counter()
    E, XpY, _ = O.solve(A, B)
    t2 = O.oscillator(XpY, p)
    solve_sub = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.spectrum(E, t2, inputs["omega"], w.eta, O.spectrum_prefactor(inputs))
    spec_sub = time.perf_counter() - t0
    solve_s = solve_sub * (w.n / ns) ** 3
    spec_s = spec_sub * (w.n / ns)
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"build: oracle kernel_blocks (exchange + W^rr + W^ra, FP64 NumPy) on every "
                      f"{stride}-th k-pair ({len(sel)} of {P} pairs), {dt:.1f} s; solve and "
                      f"spectrum: the oracle's squared-form solve (two eigh) and eigen-sum of "
                      f"the principal sub-problem of the first {ks} k-points (N = {ns}), "
                      f"{solve_sub:.1f} s and {spec_sub:.2f} s, scaled by N^3 and N",
            "stage_s": {"build": build_s, "solve": solve_s, "spectrum": spec_s},
            "time_to_eps_M_s": build_s + solve_s + spec_s}


def batched_section(name: str, steps: int) -> dict:
    """Many momentum transfers in one HIP graph (concurrent branches, the
    autotuner's tile choices, FP64 and mixed-precision assembly) against the
    per-Q sequential FP64 path with the built-in tile rules."""
    import torch
    from bse_synth import BATCHES, make_batch_inputs
    from paper_1904_05575_amd import _lib as L
    from paper_1904_05575_amd import tune
    from paper_1904_05575_amd.batch import Batch
    bw = BATCHES[name]
    members = make_batch_inputs(bw)
    B = Batch(members, precision="fp64", nbranch=16)  # one branch per problem (up to 16)
    tuned = L.bse_tune_get()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    L.bse_tune_set([])                       # built-in tile rules
    seq_ms = timed(B.run_sequential)
    graph_builtin_ms = timed(B.run)
    L.bse_tune_set(tuned)                    # the autotuner's table (captured anew)
    B.set_precision("fp64")
    seq_tuned_ms = timed(B.run_sequential)
    graph64_ms = timed(B.run)
    fp64 = B.results()
    B.set_precision("bf16x6")
    graph_mixed_ms = timed(B.run)
    mixed = B.results()
    # errors against the FP64 oracle's stored values of the members that have them
    vs_oracle = {}
    for i, d in enumerate(members):
        for prec, res in (("fp64", fp64[i]), ("bf16x6", mixed[i])):
            e = golden_errors(f"{name}:{i}", d, res["E"], res["osc"], res["eps"])
            if e:
                vs_oracle.setdefault(prec, {})[f"member{i}_n{d['workload'].n}"] = {
                    "eig_rel": e["eig_rel"], "spec_err": e["spec_err"]}
    B.close()
    print(f"[bench] batch {name}: sequential fp64 {seq_ms:.1f} ms (tuned {seq_tuned_ms:.1f}), "
          f"graph fp64 {graph_builtin_ms:.1f} ms (tuned {graph64_ms:.1f}), graph bf16x6 tuned "
          f"{graph_mixed_ms:.1f} ms", file=sys.stderr, flush=True)
    return {"workload": name, "problems": len(members), "sizes": [m["workload"].n for m in members],
            "tuning_entries": len(tuned), "tuning_table": os.path.basename(tune.TABLE),
            "sequential_fp64_builtin_tiles_ms": seq_ms, "sequential_fp64_tuned_ms": seq_tuned_ms,
            "graph_fp64_builtin_tiles_ms": graph_builtin_ms, "graph_fp64_tuned_ms": graph64_ms,
            "graph_bf16x6_tuned_ms": graph_mixed_ms,
            # same graph, same branches and tiles: what the split-BF16 assembly buys
            "mixed_speedup_graph_fp64_over_bf16x6": graph64_ms / graph_mixed_ms,
            # everything together (branches, tiles, precision) against one problem at a time
            "speedup_graph_bf16x6_vs_sequential_fp64_builtin": seq_ms / graph_mixed_ms,
            "error_vs_oracle": vs_oracle,
            "branches": min(16, len(members))}


def observables_section(P, H0, H1, reps: int) -> dict:
    """Optical-limit observables on the same problem: one solve with
    eigenvectors, then the transition coefficients along x, y, z (eq.
    tlambdai), the 3 x 3 dielectric tensor (eq. epsmij) on the frequency grid
    and the loss function with S(Q, w) of each diagonal element (eq. Lofeps),
    each timed with HIP events over `reps` repetitions."""
    import torch
    from paper_1904_05575_amd import _lib as L

    n = P.n
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    P.build(H0, H1)
    ev[1].record()
    E, XpY, _ = P.solve(H0, H1, vectors=True, probe=False)
    ev[2].record()
    torch.cuda.synchronize()
    P.check_info()
    solve_vec_ms = ev[1].elapsed_time(ev[2])
    t = P.transitions(XpY)
    eps = P.dielectric_tensor(E, t)
    torch.cuda.synchronize()
    L.bse_timing_enable(True)
    for _ in range(reps):
        t = P.transitions(XpY)
        eps = P.dielectric_tensor(E, t)
        for a in range(3):
            P.loss(eps, diag=a)
    torch.cuda.synchronize()
    L.bse_timing_enable(False)
    k = L.bse_timing_report()
    P.check_info()
    tr_ms = k["k_transitions"][1] / k["k_transitions"][0]
    te_ms = k["k_dielectric_tensor"][1] / k["k_dielectric_tensor"][0]
    lo_ms = k["k_loss"][1] / k["k_loss"][0]
    nw = P.t["omega"].numel()
    tr_bytes = n * n * 16 + 2 * 3 * n * 16      # X+Y once, the probes and t
    te_flop = nw * n * (9 * 14 + 12)            # 9 conj(t_a) t_b g products + g per term
    del XpY
    torch.cuda.empty_cache()
    return {"solve_with_vectors_ms": solve_vec_ms,
            "transitions": {"ms": tr_ms, "bytes": tr_bytes,
                            "achieved_GBps": tr_bytes / (tr_ms * 1e-3) / 1e9,
                            "frac_hbm_peak": tr_bytes / (tr_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "dielectric_tensor": {"ms": te_ms, "nw": nw, "flop": te_flop,
                                  "achieved_TFLOPs": te_flop / (te_ms * 1e-3) / 1e12,
                                  "frac_fp64_vector_peak":
                                      te_flop / (te_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS},
            "loss_ms": lo_ms}


def eigenpairs_section(P, H0, H1, steps: int) -> dict:
    """All eigenpairs and eps_M of the same workload: `steps` timed repetitions
    of bse_build + bse_solve with X+Y and X-Y (both halves of every exciton
    vector, Sec. 4.3) and oscillator strengths + bse_spectrum, HIP events
    around each stage."""
    import torch
    E, XpY, XmY, osc = P.solve(*P.build(H0, H1), xmy=True)  # warm-up
    del XpY, XmY
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for i in range(steps):
        evs[i][0].record()
        P.build(H0, H1)
        evs[i][1].record()
        E, XpY, XmY, osc = P.solve(H0, H1, xmy=True)
        evs[i][2].record()
        P.spectrum(E, osc)
        evs[i][3].record()
        del XpY, XmY
    torch.cuda.synchronize()
    P.check_info()
    torch.cuda.empty_cache()
    mean = lambda a, b: float(np.mean([e[a].elapsed_time(e[b]) for e in evs]))  # noqa: E731
    return {"steps": steps, "ms_per_step": mean(0, 3), "build_ms": mean(0, 1),
            "solve_with_vectors_ms": mean(1, 2), "spectrum_ms": mean(2, 3),
            "outputs": "E, X+Y, X-Y (n x n each), |t|^2, eps_M"}


def core_section(name: str) -> dict:
    """Core-level TDA workload (N = 32768, M^cc drawn in place, split-BF16
    assembly, FP64 eigensolve): one step of bse_build + bse_solve (spectrum
    path) + bse_spectrum, HIP events around each stage.  Its kernels are the
    ones the main workload already ran, so no warm-up step is taken."""
    import torch
    from bse_synth import get, make_inputs
    from paper_1904_05575_amd.bse import Problem
    w = get(name)
    t0 = time.perf_counter()
    d = make_inputs(w)
    gen_s = time.perf_counter() - t0
    P = Problem(d, precision="bf16x6")
    H0, _ = P.alloc_matrices()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record()
    P.build(H0)
    ev[1].record()
    E, _, osc = P.solve(H0, None)
    ev[2].record()
    P.spectrum(E, osc)
    ev[3].record()
    torch.cuda.synchronize()
    P.check_info()
    f = build_flops(w)
    out = {"workload": name, "n": w.n, "ng": w.ng, "assembly_precision": "bf16x6",
           "ms_per_step": ev[0].elapsed_time(ev[3]), "build_ms": ev[0].elapsed_time(ev[1]),
           "solve_ms": ev[1].elapsed_time(ev[2]), "spectrum_ms": ev[2].elapsed_time(ev[3]),
           "build_gflop": f["total"] / 1e9,
           "build_tflops": f["total"] / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e12,
           "input_generation_s": gen_s}
    del P, H0, E, osc
    torch.cuda.empty_cache()
    return out


def orbitals_section(name: str, reps: int) -> dict:
    """Pair elements formed on the device from synthetic orbitals
    (bse_pair_elements) for a workload of the benchmark's shape, then the FP64
    build on them; HIP events over `reps` repetitions.  Flops: 8 per complex
    multiply-add, one per K whose partner K + G (or -K - G) is in the sphere."""
    import torch
    from bse_synth import get, make_inputs
    from paper_1904_05575_amd.bse import Problem, sphere_partners
    w = get(name)
    d = make_inputs(w)
    P = Problem(d)
    H0, H1 = P.alloc_matrices()
    P.build(H0, H1)
    torch.cuda.synchronize()
    plus, minus = sphere_partners(d["kvec"], d["gvec"])
    cp, cm = float((plus >= 0).sum()), float((minus >= 0).sum())
    npairs = w.npairs
    flop = 8.0 * (npairs * ((w.nv ** 2 + w.nc ** 2) * cp + 2 * w.nv * w.nc * cm)
                  + w.nk * w.nv * w.nc * cp)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(reps):
        P.pair_elements()
    ev[1].record()
    for _ in range(reps):
        P.build(H0, H1)
    ev[2].record()
    torch.cuda.synchronize()
    P.check_info()
    gen_ms = ev[0].elapsed_time(ev[1]) / reps
    build_ms = ev[1].elapsed_time(ev[2]) / reps
    out = {"workload": name, "n": w.n, "ng": w.ng, "orbital_plane_waves": w.orbitals,
           "pair_elements_ms": gen_ms, "pair_elements_gflop": flop / 1e9,
           "pair_elements_TFLOPs": flop / (gen_ms * 1e-3) / 1e12,
           "pair_elements_frac_fp64_vector_peak": flop / (gen_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
           "pair_bytes_written": float(sum(P.t[k].numel() * 16 for k in
                                           ("Mcv", "Mvv", "Mcc", "Ncv", "Nvc"))),
           "build_on_formed_elements_ms": build_ms}
    del P, H0, H1
    torch.cuda.empty_cache()
    return out


def screening_section(w, reps: int) -> dict:
    """Static RPA screening on the workload's mesh and bands: W(q) for every q
    (bse_screening), timed with HIP events over `reps` calls; the two pair
    contractions on MFMA against the FP64 peak."""
    import torch
    from bse_synth import make_screening_inputs
    from paper_1904_05575_amd import _lib as L
    from paper_1904_05575_amd.bse import Screening

    t0 = time.perf_counter()
    sd = make_screening_inputs(w)
    gen_s = time.perf_counter() - t0
    Sc = Screening(sd)
    del sd
    W = Sc.run()
    Sc.check_info()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        Sc.run(W)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    L.bse_timing_enable(True)
    Sc.run(W)
    torch.cuda.synchronize()
    L.bse_timing_enable(False)
    k = L.bse_timing_report()
    Sc.check_info()
    k1 = w.nk * w.nv * w.nc
    # two pair sets, upper triangle of the Hermitian Xt, 8 flop per cMAC
    flop = 2 * 8 * w.nk * (w.ng * (w.ng + 1) // 2) * k1
    chi_ms = k.get("k_screen_chi", k.get("zgemm_screen_chi", (1, float("nan"))))[1]
    out = {"workload": f"{w.name} mesh", "nq": w.nk, "ng": w.ng, "pair_rows_per_q": 2 * k1,
           "ms": ms, "chi_gflop": flop / 1e9, "chi_ms": chi_ms,
           "chi_TFLOPs": flop / (chi_ms * 1e-3) / 1e12,
           "chi_frac_fp64_peak": flop / (chi_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
           "invert_ms": k.get("k_screen_invert_reg", k.get("k_screen_invert", (1, float("nan"))))[1],
           "weights_ms": k.get("k_screen_weights", (1, float("nan")))[1],
           "input_generation_s": gen_s}
    del Sc, W
    torch.cuda.empty_cache()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="full_q0_k8_v3c4_g113")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", default="batch16_k6_g89",
                    help="batched finite-Q workload timed after the main steps ('' to skip)")
    ap.add_argument("--precisions", default="fp32,bf16x6",
                    help="assembly precisions timed after the FP64 steps")
    ap.add_argument("--no-observables", action="store_true",
                    help="skip the optical-limit observables (eigenvector path) section")
    ap.add_argument("--no-screening", action="store_true",
                    help="skip the RPA screening section")
    ap.add_argument("--no-eigenpairs", action="store_true",
                    help="skip the all-eigenpairs (X+Y, X-Y) steps")
    ap.add_argument("--core", default="core_tda_k8_c2c32_g137",
                    help="core-level workload timed for one step ('' to skip)")
    ap.add_argument("--orbitals", default="full_orb_k8_v3c4_g113_o113",
                    help="workload whose pair elements are formed from orbitals ('' to skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import torch
    from bse_synth import get, make_inputs
    from paper_1904_05575_amd import _lib as L
    from paper_1904_05575_amd.bse import Problem

    w = get(args.workload)
    t0 = time.perf_counter()
    inputs = make_inputs(w)
    print(f"[bench] inputs generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    P = Problem(inputs)
    torch.cuda.synchronize()
    print("[bench] inputs resident on the GPU", file=sys.stderr, flush=True)
    H0, H1 = P.alloc_matrices()

    def step(ev=None):
        if ev:
            ev[0].record()
        P.build(H0, H1)
        if ev:
            ev[1].record()
        E, _, osc = P.solve(H0, H1, vectors=False)
        if ev:
            ev[2].record()
        eps = P.spectrum(E, osc)
        if ev:
            ev[3].record()
        return E, osc, eps

    for i in range(args.warmup):
        step()
        P.check_info()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    # one profiling step with every kernel timed: the per-kernel breakdown and
    # the dominant kernel (largest total time among the roofline candidates)
    table = kernel_roofline_table(w)
    L.bse_timing_enable(True)
    step()
    torch.cuda.synchronize()
    L.bse_timing_enable(False)
    breakdown = L.bse_timing_report()
    cands = {k: v for k, v in breakdown.items() if k in table}
    dom = max(cands, key=lambda k: cands[k][1]) if cands else None
    print(f"[bench] profiling step done; dominant kernel {dom}", file=sys.stderr, flush=True)

    # timed region: HIP events around each stage of every step
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        E, osc, eps = step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    P.check_info()
    build_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    solve_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    spec_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    step_ms = float(np.mean([e[0].elapsed_time(e[3]) for e in evs]))
    flops = build_flops(w)
    value = flops["total"] / (build_ms * 1e-3) / 1e12

    # the same steps again with HIP events around every launch of the dominant
    # kernel, recorded on the stream it runs on (the events add host overhead,
    # so these steps do not enter ms_per_step)
    if dom:
        L.bse_timing_enable(True, dom)
    evr = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    for i in range(args.steps):
        step(evr[i])
    torch.cuda.synchronize()
    L.bse_timing_enable(False)
    kern = L.bse_timing_report()
    roof_step_ms = float(np.mean([e[0].elapsed_time(e[3]) for e in evr]))

    roof = None
    if dom and dom in kern:
        bound, amount, unit = table[dom]
        launches, total_ms = kern[dom]
        per_launch = amount * args.steps / launches
        avg_s = total_ms / launches * 1e-3
        if bound == "hbm":
            ach, peak, u = per_launch / avg_s / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            ach, peak, u = per_launch / avg_s / 1e12, FP64_PEAK_TFLOPS, "TFLOP/s"
        tr = measured_traffic(dom, w.n) if bound == "hbm" else None
        roof = {"bound": bound, "kernel": dom, "achieved": ach, "peak": peak, "unit": u,
                "frac": ach / peak, "traffic": tr["bytes"] if tr else None,
                "traffic_unit": "B per launch", "traffic_source": tr["source"] if tr else None,
                "traffic_note": tr["note"] if tr else (
                    "no counter summary of this kernel's current source: counter runs of "
                    "processes that run the Householder sweep ended in a crash or a hang and "
                    "are not taken" if bound == "hbm"
                    else None),
                "launches_per_step": launches / args.steps,
                "avg_launch_us": total_ms / launches * 1e3,
                "ms_per_step_with_events": roof_step_ms,
                "per_launch_" + ("bytes" if bound == "hbm" else "flop"): per_launch}
    kernels_ms = {k: round(v[1], 3) for k, v in
                  sorted(breakdown.items(), key=lambda kv: -kv[1][1])}

    # precision form of the assembly: same inputs, FP32 and split-BF16 (6 products);
    # errors are against the FP64 oracle's stored values for this workload
    vs_oracle = {}
    e = golden_errors(w.name, inputs, E.cpu().numpy(), osc.cpu().numpy(), eps.cpu().numpy())
    if e:
        vs_oracle["fp64"] = e
    t2e = {"fp64": step_ms}
    b_ms = {"fp64": build_ms}
    for prec in args.precisions.split(","):
        if not prec:
            continue
        P.set_precision(prec)
        step()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        for i in range(args.steps):
            Ep, _, epsp = step(ev[i])
        torch.cuda.synchronize()
        P.check_info()
        t2e[prec] = float(np.mean([e[0].elapsed_time(e[3]) for e in ev]))
        b_ms[prec] = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
        e = golden_errors(w.name, inputs, Ep.cpu().numpy(), None, epsp.cpu().numpy())
        if e:
            vs_oracle[prec] = e
        print(f"[bench] precision {prec}: {t2e[prec]:.1f} ms/step", file=sys.stderr, flush=True)
    P.set_precision("fp64")

    out = {
        "metric": "kernel-build TFLOP/s + time-to-eps_M at N=6144 full BSE, FP64 vs split-BF16",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "nk": w.nk, "nv": w.nv, "nc": w.nc,
                   "ng": w.ng, "coupling": w.coupling, "nw": w.nw,
                   "assembly_precision": "fp64"},
        "time_to_eps_M_ms": t2e,
        "build_ms": b_ms,
        "build_tflops": {k: flops["total"] / (v * 1e-3) / 1e12 for k, v in b_ms.items()},
        "error_vs_oracle": vs_oracle,
        "stage_ms": {"build": build_ms, "solve": solve_ms, "spectrum": spec_ms},
        "wall_ms_per_step": wall / args.steps * 1e3,
        "build_gflop": flops["total"] / 1e9,
        "build_frac_fp64_peak": value / FP64_PEAK_TFLOPS,
        "roofline": roof,
        "kernels_ms_per_step": kernels_ms,
        "tile_choices": f"{len(L.bse_tune_get())} autotuner entries (paper_1904_05575_amd/tuning_gfx950.json)",
    }
    if not args.no_observables:
        out["observables"] = observables_section(P, H0, H1, args.steps)
        print("[bench] observables done", file=sys.stderr, flush=True)
    if not args.no_eigenpairs:
        out["all_eigenpairs"] = eigenpairs_section(P, H0, H1, min(args.steps, 5))
        print(f"[bench] all eigenpairs: {out['all_eigenpairs']['ms_per_step']:.1f} ms/step",
              file=sys.stderr, flush=True)
    if not args.no_screening:
        del P, H0, H1
        torch.cuda.empty_cache()
        out["screening"] = screening_section(w, args.steps)
        print("[bench] screening done", file=sys.stderr, flush=True)
    if args.orbitals:
        if "P" in locals():
            del P, H0, H1
            torch.cuda.empty_cache()
        out["pair_elements_from_orbitals"] = orbitals_section(args.orbitals, args.steps)
        print(f"[bench] pair elements from orbitals: "
              f"{out['pair_elements_from_orbitals']['pair_elements_ms']:.1f} ms",
              file=sys.stderr, flush=True)
    if args.core:
        if "P" in locals():
            del P, H0, H1
            torch.cuda.empty_cache()
        out["core_level"] = core_section(args.core)
        print(f"[bench] core level: {out['core_level']['ms_per_step']:.0f} ms/step",
              file=sys.stderr, flush=True)
    if args.batch:
        out["batched"] = batched_section(args.batch, min(args.steps, 3))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inputs, w)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
