// Batches of independent BSE problems (one per momentum transfer Q: the BSE
// decouples per q, paper Sec. 2.3 eq. chimatrixq) recorded once into a HIP
// graph and replayed with one launch.  Problems are spread over `nbranch`
// concurrent branches (longest first, by N^3), each with its own slice of the
// caller's workspace.  With one branch per problem the Householder sweeps of
// all problems run as one batched sweep (one launch per sweep step for every
// problem), between the branches' assembly and factorisation and their
// eigenvalue stages.
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
  // [0] fork, [1 + b] join of branch b, [1 + nbranch] second fork (after the
  // batched sweep), [2 + nbranch + b] second join
  std::vector<hipEvent_t> events;
  size_t slice = 0;
  void* trd_table = nullptr;  // device table of the batched sweep (one branch per problem)
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
  return slice_bytes(nprob, descs) * (size_t)std::min(nbranch, nprob);
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
  b->events.assign(2 + 2 * b->nbranch, nullptr);
  for (auto& e : b->events)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      bse_batch_destroy(b);
      return BSE_ERR_HIP;
    }
  if (b->nbranch == nprob) {
    std::vector<int64_t> ns(nprob);
    for (int i = 0; i < nprob; ++i) ns[i] = (int64_t)descs[i].nk * descs[i].nv * descs[i].nc;
    b->trd_bytes = trd_batch_table_bytes(ns.data(), nprob);
    if (hipMalloc(&b->trd_table, b->trd_bytes) != hipSuccess) {
      b->trd_table = nullptr;
      bse_batch_destroy(b);
      return BSE_ERR_HIP;
    }
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
  if (ws_bytes < b->slice * (size_t)b->nbranch) return BSE_ERR_WORKSPACE;
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
  const bool batched = b->trd_table != nullptr;
  std::vector<TrdItem> items;
  if (batched) {
    for (int i = 0; i < b->nprob; ++i) {
      void* wsb = (char*)ws + b->slice * (size_t)b->branch_of[i];
      items.push_back(solve_sweep_item(&b->descs[i], H0[i], wsb, true, info + i));
    }
    if (!trd_batch_table(items.data(), b->nprob, b->trd_table, b->trd_bytes)) return BSE_ERR_HIP;
  }
  const TimingState timing = timing_suspend();  // no events inside the graph
  bse_status st = BSE_OK;
  if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    timing_resume(timing);
    return BSE_ERR_HIP;
  }
  auto fork = [&](int ev) {
    hipEventRecord(b->events[ev], stream);
    for (int br = 0; br < b->nbranch; ++br) hipStreamWaitEvent(b->streams[br], b->events[ev], 0);
  };
  auto join = [&](int ev0) {
    for (int br = 0; br < b->nbranch; ++br) {
      hipEventRecord(b->events[ev0 + br], b->streams[br]);
      hipStreamWaitEvent(stream, b->events[ev0 + br], 0);
    }
  };
  launch_zero_ints(info, b->nprob, stream);
  fork(0);
  const int first = batched ? SOLVE_PRE : SOLVE_ALL;
  for (int i = 0; i < b->nprob && st == BSE_OK; ++i) {
    const bse_desc* d = &b->descs[i];
    hipStream_t s = b->streams[b->branch_of[i]];
    void* wsb = (char*)ws + b->slice * (size_t)b->branch_of[i];
    void* h1 = (d->coupling == BSE_FULL) ? H1[i] : nullptr;
    const int64_t n = (int64_t)d->nk * d->nv * d->nc;
    st = build_fp64(d, &inputs[i], H0[i], h1, wsb, info + i, s);
    if (st == BSE_OK)
      st = solve_run(d, H0[i], h1, E[i], nullptr, nullptr, n, probe[i], osc[i], wsb, info + i, s,
                     first);
    if (st == BSE_OK && !batched &&
        launch_spectrum(n, E[i], osc[i], pref[i], eta[i], nw[i], omega[i], (double2*)eps[i], s) !=
            hipSuccess)
      st = BSE_ERR_HIP;
  }
  join(1);
  if (batched && st == BSE_OK) {
    if (!tridiagonalise_batch(items.data(), b->nprob, b->trd_table, stream)) st = BSE_ERR_HIP;
    fork(1 + b->nbranch);
    for (int i = 0; i < b->nprob && st == BSE_OK; ++i) {
      const bse_desc* d = &b->descs[i];
      hipStream_t s = b->streams[b->branch_of[i]];
      void* wsb = (char*)ws + b->slice * (size_t)b->branch_of[i];
      void* h1 = (d->coupling == BSE_FULL) ? H1[i] : nullptr;
      const int64_t n = (int64_t)d->nk * d->nv * d->nc;
      st = solve_run(d, H0[i], h1, E[i], nullptr, nullptr, n, probe[i], osc[i], wsb, info + i, s,
                     SOLVE_POST);
      if (st == BSE_OK && launch_spectrum(n, E[i], osc[i], pref[i], eta[i], nw[i], omega[i],
                                          (double2*)eps[i], s) != hipSuccess)
        st = BSE_ERR_HIP;
    }
    join(2 + b->nbranch);
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
  if (b->trd_table) hipFree(b->trd_table);
  delete b;
}

}  // extern "C"
