// Batches of independent BSE problems (one per momentum transfer Q: the BSE
// decouples per q, paper Sec. 2.3 eq. chimatrixq) recorded once into a HIP
// graph and replayed with one launch.  Problems are spread over `nbranch`
// concurrent branches (longest first, by N^3), each with its own slice of the
// caller's workspace.  With one branch per problem the Cholesky factorisations
// and the Householder sweeps of all problems run batched on the capture stream
// (one launch per step serving every problem), between rounds of per-problem
// work on the branches: assembly; squared form; eigenvalue stages and spectrum.
#include <algorithm>
#include <vector>

#include "bse_internal.h"
#include "solve_internal.h"
#include "timing.h"

struct bse_batch {
  int nprob = 0, nbranch = 0;
  std::vector<bse_desc> descs;
  std::vector<int> branch_of;
  std::vector<hipStream_t> streams;
  // per round r of branch work (one round without the batched stages, three
  // with them): [r (1 + nbranch)] fork, [r (1 + nbranch) + 1 + b] join of branch b
  std::vector<hipEvent_t> events;
  size_t slice = 0;
  // batched stages (one branch per problem): the sweep's device table sits in
  // the caller's workspace after the branch slices
  bool batched = false;
  size_t trd_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

bool batch_desc_ok(const bse_desc* d) { return bse_workspace_size(d, BSE_STAGE_BUILD) > 0; }

size_t slice_bytes(int nprob, const bse_desc* descs) {
  size_t s = 0;
  for (int i = 0; i < nprob; ++i) {
    s = std::max(s, bse_workspace_size(&descs[i], BSE_STAGE_BUILD));
    s = std::max(s, bse_workspace_size(&descs[i], BSE_STAGE_SOLVE));
  }
  return (s + 255) & ~(size_t)255;
}

// Bytes of the batched sweep's device table, rounded to 256.
size_t table_bytes(int nprob, const bse_desc* descs) {
  std::vector<int64_t> ns(nprob);
  for (int i = 0; i < nprob; ++i) ns[i] = (int64_t)descs[i].nk * descs[i].nv * descs[i].nc;
  return (trd_batch_table_bytes(ns.data(), nprob) + 255) & ~(size_t)255;
}

void release(bse_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

}  // namespace

extern "C" {

size_t bse_batch_workspace_size(int32_t nprob, const bse_desc* descs, int32_t nbranch) {
  if (nprob <= 0 || !descs || nbranch <= 0) return 0;
  for (int i = 0; i < nprob; ++i)
    if (!batch_desc_ok(&descs[i])) return 0;
  return slice_bytes(nprob, descs) * (size_t)std::min(nbranch, nprob) +
         (nbranch >= nprob ? table_bytes(nprob, descs) : 0);
}

bse_status bse_batch_create(int32_t nprob, const bse_desc* descs, int32_t nbranch,
                            bse_batch_t* out) {
  if (!out || nprob <= 0 || !descs || nbranch <= 0) return BSE_ERR_ARG;
  for (int i = 0; i < nprob; ++i)
    if (!batch_desc_ok(&descs[i])) return BSE_ERR_ARG;
  bse_batch* b = new bse_batch;
  b->nprob = nprob;
  b->nbranch = std::min(nbranch, nprob);
  b->descs.assign(descs, descs + nprob);
  b->slice = slice_bytes(nprob, descs);
  // longest processing time first: largest N^3 to the least loaded branch
  std::vector<int> order(nprob);
  for (int i = 0; i < nprob; ++i) order[i] = i;
  auto cost = [&](int i) {
    const double n = (double)descs[i].nk * descs[i].nv * descs[i].nc;
    return n * n * n;
  };
  std::sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
  std::vector<double> load(b->nbranch, 0.0);
  b->branch_of.assign(nprob, 0);
  for (int i : order) {
    const int br = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->branch_of[i] = br;
    load[br] += cost(i);
  }
  b->streams.assign(b->nbranch, nullptr);
  for (auto& s : b->streams)
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      bse_batch_destroy(b);
      return BSE_ERR_HIP;
    }
  b->events.assign(3 * (1 + b->nbranch), nullptr);
  for (auto& e : b->events)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      bse_batch_destroy(b);
      return BSE_ERR_HIP;
    }
  if (b->nbranch == nprob) {
    b->batched = true;
    b->trd_bytes = table_bytes(nprob, descs);
  }
  *out = b;
  return BSE_OK;
}

bse_status bse_batch_capture(bse_batch_t b, const bse_inputs* inputs, void* const* H0,
                             void* const* H1, double* const* E, const void* const* probe,
                             double* const* osc, const double* pref, const double* eta,
                             const int64_t* nw, const double* const* omega, void* const* eps,
                             void* ws, size_t ws_bytes, int32_t* info, hipStream_t stream) {
  launch_failure_reset();
  if (!b || !inputs || !H0 || !E || !probe || !osc || !pref || !eta || !nw || !omega || !eps ||
      !ws || !info)
    return BSE_ERR_ARG;
  if (stream == nullptr) return BSE_ERR_ARG;  // the legacy NULL stream cannot be captured
  if (ws_bytes < b->slice * (size_t)b->nbranch + b->trd_bytes) return BSE_ERR_WORKSPACE;
  for (int i = 0; i < b->nprob; ++i) {
    const bse_desc* d = &b->descs[i];
    const bse_inputs* in = &inputs[i];
    if (!H0[i] || !E[i] || !probe[i] || !osc[i] || !omega[i] || !eps[i] || nw[i] <= 0) return BSE_ERR_ARG;
    if (d->coupling == BSE_FULL && (!H1 || !H1[i] || !in->Ncv || !in->Nvc || !in->qramap))
      return BSE_ERR_ARG;
    if (!in->eps_v || !in->eps_c || !in->Mcv || !in->Mvv || (!in->Mcc && !in->mcc_env) ||
        !in->W || !in->vbar || !in->qmap || in->nq <= 0 || in->nq > kMaxQ)
      return BSE_ERR_ARG;
    if (!(eta[i] > 0.0)) return BSE_ERR_ARG;
    if (d->prec != BSE_PREC_FP64 && in->nq > d->nk) return BSE_ERR_ARG;
  }
  release(b);
  // batched sweep: every problem's sweep arguments, written to the device
  // table before capture (a blocking copy; no replay of this batch may run)
  const bool batched = b->batched;
  void* trd_table = (char*)ws + b->slice * (size_t)b->nbranch;
  std::vector<TrdItem> items;
  if (batched) {
    for (int i = 0; i < b->nprob; ++i) {
      void* wsb = (char*)ws + b->slice * (size_t)b->branch_of[i];
      items.push_back(solve_sweep_item(&b->descs[i], H0[i], wsb, true, info + i));
    }
    if (!trd_batch_table(items.data(), b->nprob, trd_table, b->trd_bytes)) return BSE_ERR_HIP;
  }
  const TimingState timing = timing_suspend();  // no events inside the graph
  bse_status st = BSE_OK;
  if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    timing_resume(timing);
    return BSE_ERR_HIP;
  }
  const int nb = b->nbranch;
  auto fork = [&](int r) {  // round r: events[r (1 + nb)] forks, the next nb join
    hipEvent_t e = b->events[r * (1 + nb)];
    hipEventRecord(e, stream);
    for (int br = 0; br < nb; ++br) hipStreamWaitEvent(b->streams[br], e, 0);
  };
  auto join = [&](int r) {
    for (int br = 0; br < nb; ++br) {
      hipEvent_t e = b->events[r * (1 + nb) + 1 + br];
      hipEventRecord(e, b->streams[br]);
      hipStreamWaitEvent(stream, e, 0);
    }
  };
  auto branch = [&](int i) { return b->streams[b->branch_of[i]]; };
  auto slice = [&](int i) { return (void*)((char*)ws + b->slice * (size_t)b->branch_of[i]); };
  auto h1_of = [&](int i) { return b->descs[i].coupling == BSE_FULL ? H1[i] : nullptr; };
  auto order_of = [&](int i) {
    return (int64_t)b->descs[i].nk * b->descs[i].nv * b->descs[i].nc;
  };
  // the solve's stages of problem i on its branch
  auto solve = [&](int i, int phase) {
    return solve_run(&b->descs[i], H0[i], h1_of(i), E[i], nullptr, nullptr, order_of(i),
                     probe[i], osc[i], slice(i), info + i, branch(i), phase);
  };
  auto spectrum = [&](int i) {
    return launch_spectrum(order_of(i), E[i], osc[i], pref[i], eta[i], nw[i], omega[i],
                           (double2*)eps[i], branch(i)) == hipSuccess
               ? BSE_OK
               : BSE_ERR_HIP;
  };
  launch_zero_ints(info, b->nprob, stream);
  // round 0 on the branches: assembly, and everything (one branch per problem:
  // the stages before the Cholesky factorisation)
  fork(0);
  for (int i = 0; i < b->nprob && st == BSE_OK; ++i) {
    st = build_fp64(&b->descs[i], &inputs[i], H0[i], h1_of(i), slice(i), info + i, branch(i));
    if (st == BSE_OK) st = solve(i, batched ? SOLVE_PRE1 : SOLVE_ALL);
    if (st == BSE_OK && !batched) st = spectrum(i);
  }
  join(0);
  if (batched && st == BSE_OK) {
    // the Cholesky factorisations in step (problems of one tuned GEMM tile
    // together), on the capture stream
    std::vector<CholItem> chol;
    std::vector<int> tiles;
    for (int i = 0; i < b->nprob; ++i)
      if (b->descs[i].coupling == BSE_FULL) {
        chol.push_back(solve_chol_item(&b->descs[i], H1[i], slice(i), info + i));
        tiles.push_back(tune_choice(BSE_TUNE_GEMM_POTRF, order_of(i), 0));
      }
    std::vector<char> done(chol.size(), 0);
    for (size_t i = 0; i < chol.size() && st == BSE_OK; ++i) {
      if (done[i]) continue;
      std::vector<CholItem> grp;
      for (size_t j = i; j < chol.size() && (int)grp.size() < CHOL_GROUP_MAX; ++j)
        if (!done[j] && tiles[j] == tiles[i]) {
          grp.push_back(chol[j]);
          done[j] = 1;
        }
      if (!cholesky_batch(grp.data(), (int)grp.size(), stream)) st = BSE_ERR_HIP;
    }
    // round 1 on the branches: squared form and the probe's projection
    fork(1);
    for (int i = 0; i < b->nprob && st == BSE_OK; ++i) st = solve(i, SOLVE_PRE2);
    join(1);
    // the Householder sweeps of all problems as one, on the capture stream
    if (st == BSE_OK && !tridiagonalise_batch(items.data(), b->nprob, trd_table, stream))
      st = BSE_ERR_HIP;
    // round 2 on the branches: eigenvalues, oscillator strengths, spectrum
    fork(2);
    for (int i = 0; i < b->nprob && st == BSE_OK; ++i) {
      st = solve(i, SOLVE_POST);
      if (st == BSE_OK) st = spectrum(i);
    }
    join(2);
  }
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(stream, &g);
  timing_resume(timing);  // the caller's switch and name filter
  if (st != BSE_OK || ec != hipSuccess || !g) {
    if (g) hipGraphDestroy(g);
    return st != BSE_OK ? st : BSE_ERR_HIP;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    release(b);
    return BSE_ERR_HIP;
  }
  return BSE_OK;
}

bse_status bse_batch_run(bse_batch_t b, hipStream_t stream) {
  launch_failure_reset();
  if (!b || !b->exec) return BSE_ERR_ARG;
  return hipGraphLaunch(b->exec, stream) == hipSuccess ? BSE_OK : BSE_ERR_HIP;
}

void bse_batch_destroy(bse_batch_t b) {
  if (!b) return;
  release(b);
  for (auto s : b->streams)
    if (s) hipStreamDestroy(s);
  for (auto e : b->events)
    if (e) hipEventDestroy(e);
  delete b;
}

}  // extern "C"
