"""Autotuner of the library's tile choices (run on the GPU; writes a JSON table).

    python -m paper_1904_05575_amd.tune [--out PATH] [--reps 2]
                                        [--hemv-only | --gemm-site SITE | --batch-sweep-only]

For every tunable call site of the FP64 path (see bse_tune_entry in
include/bse.h) the tuner builds and solves seeded synthetic problems of the
batched and single-problem workloads, times the site's kernels with the
library's per-kernel events under each candidate choice, and keeps the
fastest:
  * GEMM tile edge (32 or 64; 16 or 32 for the per-pair second contraction)
    for the squared form's two products, the Cholesky and Householder trailing updates, the
    per-pair contraction, the exchange term and the eigenvector path's
    products (timed in a solve with X+Y and X-Y), per problem order n;
  * the least number of tiles per block of the Householder hemv kernel
    (1, 2, 4, 8), per bucket of the trailing order m, on the largest problem;
  * the blocks of the batched sweep's hemv launches (each problem's own grid,
    or 1, 2, 4 per compute unit shared among the problems) together with when
    the problems' sweeps start (all at once, or late so that they end
    together), timed on the batch16 graph, for batches up to its largest
    order.
`load()` installs the table in the library (Problem and Batch call it once).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from . import _lib as L

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")

GEMM_SITES = {  # site -> (candidates, kernel tags timed)
    "gemm_squared": ((32, 64), ("zgemm_sq_t1",)),
    "gemm_squared_s": ((32, 64), ("zgemm_sq_s",)),
    "gemm_potrf": ((32, 64), ("zgemm_potrf_herk",)),
    "gemm_her2k": ((32, 64), ("zgemm_her2k",)),
    "gemm_stage2": ((16, 32), ("zgemm_direct_stage2",)),
    "gemm_exchange": ((32, 64), ("zgemm_exchange",)),
    "gemm_vectors": ((32, 64), ("zgemm_bt_vhz", "zgemm_bt_update", "zgemm_recon",
                                "zgemm_trsm", "zgemm_trsm_in")),
}
VECTOR_SITES = ("gemm_vectors",)  # timed in a solve that forms X+Y and X-Y
HEMV_BUCKETS = (1024, 2048, 3072, 4096, 8192)  # upper bounds of the trailing order m
HEMV_UNITS = (1, 2, 4, 8)
HEMV_TAGS = ("k_trd_hemv", "k_trd_col")
BATCH_SWEEP_CHOICES = (0, 1, 2, 4)
BATCH_ALIGN_CHOICES = (0, 1)
BATCH_SITES = ("batch_sweep", "batch_align")
BATCH_WORKLOAD = "batch16_k6_g89"

_loaded = False


def load(path: str | None = None, force: bool = False) -> int:
    """Install the tuning table (if the file exists); returns the number of entries."""
    global _loaded
    if _loaded and not force:
        return len(L.bse_tune_get())
    path = path or TABLE
    _loaded = True
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        tab = json.load(f)
    entries = [(L.TUNE_SITES[e["site"]], int(e["size_max"]), int(e["choice"]))
               for e in tab["entries"]]
    L.bse_tune_set(entries)
    return len(entries)


def _time_sites(P, tags, reps, vectors=False):
    """Best-of-reps total event time (ms) of the kernels named in tags for build +
    solve (with X+Y and X-Y when `vectors`)."""
    import torch
    best = None
    for _ in range(reps):
        H0, H1 = P.alloc_matrices()
        torch.cuda.synchronize()
        L.bse_timing_enable(True)
        P.build(H0, H1)
        out = P.solve(H0, H1, xmy=vectors)
        torch.cuda.synchronize()
        L.bse_timing_enable(False)
        P.check_info()
        k = L.bse_timing_report()
        t = sum(k[name][1] for name in tags if name in k)
        del out
        best = t if best is None else min(best, t)
        del H0, H1
    return best


def _tune_batch_sweep(base, reps, measured):
    """Time the batch16 graph (one branch per problem, FP64) under each pair of
    batched-sweep choices (hemv blocks; sweeps starting together or ending
    together) with the entries `base` installed; returns the two table entries."""
    import torch
    from bse_synth import BATCHES, make_batch_inputs
    from .batch import Batch

    load()  # Batch() installs the stored table once; do it before the candidates
    ms = make_batch_inputs(BATCHES[BATCH_WORKLOAD])
    nmax = max(d["workload"].n for d in ms)
    times = {}
    for al in BATCH_ALIGN_CHOICES:
        for c in BATCH_SWEEP_CHOICES:
            L.bse_tune_set(base + [(L.TUNE_SITES["batch_sweep"], nmax, c),
                                   (L.TUNE_SITES["batch_align"], nmax, al)])
            B = Batch(ms, precision="fp64", nbranch=len(ms))
            B.run()
            torch.cuda.synchronize()
            best = None
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                B.run()
                b.record()
                torch.cuda.synchronize()
                t = a.elapsed_time(b)
                best = t if best is None else min(best, t)
            B.results()  # raises on a device error
            B.close()
            del B
            torch.cuda.empty_cache()
            times[(c, al)] = best
    c, al = min(times, key=times.get)
    measured[f"batch_sweep@{BATCH_WORKLOAD}"] = {f"{k[0]}/align{k[1]}": round(v, 2)
                                                 for k, v in times.items()}
    print(f"[tune] {BATCH_WORKLOAD} batch_sweep/align: {times} -> {(c, al)}", file=sys.stderr,
          flush=True)
    return [{"site": "batch_sweep", "size_max": nmax, "choice": c},
            {"site": "batch_align", "size_max": nmax, "choice": al}]


def run_batch_sweep_only(out: str, reps: int = 2) -> dict:
    """Re-tune only the batched sweep's choices, keeping the table's other entries."""
    with open(TABLE) as f:
        tab = json.load(f)
    keep = [e for e in tab["entries"] if e["site"] not in BATCH_SITES]
    base = [(L.TUNE_SITES[e["site"]], int(e["size_max"]), int(e["choice"])) for e in keep]
    measured = {k: v for k, v in tab.get("measured_ms", {}).items()
                if not k.startswith("batch_sweep@")}
    t0 = time.time()
    new = _tune_batch_sweep(base, reps, measured)
    L.bse_tune_set([])
    tab["entries"], tab["measured_ms"] = keep + new, measured
    tab["seconds_batch_sweep"] = round(time.time() - t0, 1)
    with open(out, "w") as f:
        json.dump(tab, f, indent=1)
    return tab


def run_hemv_only(out: str, reps: int = 2) -> dict:
    """Re-tune only the hemv buckets, keeping the table's other entries (which
    stay installed while the hemv choices are timed)."""
    import torch
    from bse_synth import get, make_inputs
    from .bse import Problem

    with open(TABLE) as f:
        tab = json.load(f)
    keep = [e for e in tab["entries"] if e["site"] != "hemv_unit"]
    base = [(L.TUNE_SITES[e["site"]], int(e["size_max"]), int(e["choice"])) for e in keep]
    measured = {k: v for k, v in tab.get("measured_ms", {}).items()
                if not k.startswith("hemv_unit")}
    t0 = time.time()
    big = make_inputs(get("full_q0_k8_v3c4_g113"))
    P = Problem(big)
    entries = list(keep)
    lo = 0
    for hi in HEMV_BUCKETS:
        if lo >= big["workload"].n:
            break
        times = {}
        for K in HEMV_UNITS:
            L.bse_tune_set(base + [(L.TUNE_SITES["hemv_unit"], hi, K)])
            times[K] = _time_sites(P, HEMV_TAGS, reps)
        best = min(times, key=times.get)
        entries.append({"site": "hemv_unit", "size_max": hi, "choice": best})
        measured[f"hemv_unit@m<={hi}"] = {str(k): round(v, 4) for k, v in times.items()}
        print(f"[tune] m<={hi} hemv_unit: {times} -> {best}", file=sys.stderr, flush=True)
        lo = hi
    L.bse_tune_set([])
    del P
    torch.cuda.empty_cache()
    tab["entries"], tab["measured_ms"] = entries, measured
    tab["seconds_hemv"] = round(time.time() - t0, 1)
    with open(out, "w") as f:
        json.dump(tab, f, indent=1)
    return tab


def run_gemm_site_only(out: str, site: str, reps: int = 2) -> dict:
    """Re-tune one GEMM site on every problem order, keeping the table's other
    entries (installed while the site's choices are timed)."""
    import torch
    from bse_synth import BATCHES, get, make_batch_inputs, make_inputs
    from .bse import Problem

    cands, tags = GEMM_SITES[site]
    with open(TABLE) as f:
        tab = json.load(f)
    keep = [e for e in tab["entries"] if e["site"] != site]
    base = [(L.TUNE_SITES[e["site"]], int(e["size_max"]), int(e["choice"])) for e in keep]
    measured = {k: v for k, v in tab.get("measured_ms", {}).items()
                if not k.startswith(site + "@")}
    problems = {}
    for d in make_batch_inputs(BATCHES["batch16_k6_g89"]):
        problems.setdefault(d["workload"].n, d)
    big = make_inputs(get("full_q0_k8_v3c4_g113"))
    problems[big["workload"].n] = big
    t0 = time.time()
    entries = list(keep)
    for n in sorted(problems):
        P = Problem(problems[n])
        times = {}
        for c in cands:
            L.bse_tune_set(base + [(L.TUNE_SITES[site], n, c)])
            times[c] = _time_sites(P, tags, reps, site in VECTOR_SITES)
        best = min(times, key=times.get)
        entries.append({"site": site, "size_max": n, "choice": best})
        measured[f"{site}@{n}"] = {str(c): round(v, 4) for c, v in times.items()}
        print(f"[tune] n={n} {site}: {times} -> {best}", file=sys.stderr, flush=True)
        del P
        torch.cuda.empty_cache()
    L.bse_tune_set([])
    tab["entries"], tab["measured_ms"] = entries, measured
    tab[f"seconds_{site}"] = round(time.time() - t0, 1)
    with open(out, "w") as f:
        json.dump(tab, f, indent=1)
    return tab


def run(out: str, reps: int = 2) -> dict:
    import torch
    from bse_synth import BATCHES, get, make_batch_inputs, make_inputs
    from .bse import Problem

    problems = {}
    for d in make_batch_inputs(BATCHES["batch16_k6_g89"]):
        problems.setdefault(d["workload"].n, d)
    big = make_inputs(get("full_q0_k8_v3c4_g113"))
    problems[big["workload"].n] = big
    sizes = sorted(problems)
    entries, measured = [], {}
    t0 = time.time()
    L.bse_tune_set([])
    for n in sizes:
        P = Problem(problems[n])
        for site, (cands, tags) in GEMM_SITES.items():
            times = {}
            for c in cands:
                L.bse_tune_set([(L.TUNE_SITES[site], n, c)])
                times[c] = _time_sites(P, tags, reps, site in VECTOR_SITES)
            best = min(times, key=times.get)
            entries.append({"site": site, "size_max": n, "choice": best})
            measured[f"{site}@{n}"] = {str(c): round(v, 4) for c, v in times.items()}
            print(f"[tune] n={n} {site}: {times} -> {best}", file=sys.stderr, flush=True)
        del P
        torch.cuda.empty_cache()
    L.bse_tune_set([])
    P = Problem(big)
    lo = 0
    for hi in HEMV_BUCKETS:
        if lo >= big["workload"].n:
            break
        times = {}
        for K in HEMV_UNITS:
            L.bse_tune_set([(L.TUNE_SITES["hemv_unit"], hi, K)])
            times[K] = _time_sites(P, HEMV_TAGS, reps)
        best = min(times, key=times.get)
        entries.append({"site": "hemv_unit", "size_max": hi, "choice": best})
        measured[f"hemv_unit@m<={hi}"] = {str(k): round(v, 4) for k, v in times.items()}
        print(f"[tune] m<={hi} hemv_unit: {times} -> {best}", file=sys.stderr, flush=True)
        lo = hi
    del P
    torch.cuda.empty_cache()
    base = [(L.TUNE_SITES[e["site"]], int(e["size_max"]), int(e["choice"])) for e in entries]
    entries += _tune_batch_sweep(base, reps, measured)
    L.bse_tune_set([])
    tab = {"device": torch.cuda.get_device_name(0), "entries": entries,
           "measured_ms": measured, "seconds": round(time.time() - t0, 1),
           "workloads": {"sizes": sizes, "hemv": big["workload"].name}}
    with open(out, "w") as f:
        json.dump(tab, f, indent=1)
    return tab


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--hemv-only", action="store_true",
                    help="re-tune the hemv buckets only, keeping the other entries")
    ap.add_argument("--gemm-site", choices=sorted(GEMM_SITES),
                    help="re-tune one GEMM site only, keeping the other entries")
    ap.add_argument("--batch-sweep-only", action="store_true",
                    help="re-tune the batched sweep's choice only, keeping the other entries")
    args = ap.parse_args()
    if args.hemv_only:
        tab = run_hemv_only(args.out, args.reps)
    elif args.batch_sweep_only:
        tab = run_batch_sweep_only(args.out, args.reps)
    elif args.gemm_site:
        tab = run_gemm_site_only(args.out, args.gemm_site, args.reps)
    else:
        tab = run(args.out, args.reps)
    print(json.dumps({"entries": len(tab["entries"]), "seconds": tab.get("seconds"),
                      "out": args.out}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
