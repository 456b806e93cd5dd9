// Many independent chains. The setups are spread over a few library
// streams, one host thread per stream, chains taken largest first from a
// shared counter; each chain's hierarchy is an ordinary handle. The solves
// run in one persistent launch (k_batch.hip, a workgroup per chain) and on
// the library streams (bamg_gmres_solve per chain) at the same time: by
// default the launch takes the chains of at most kBatchAutoMaxStates
// states, where one workgroup per chain beats a chain's launch-bound
// per-step solve, and the streams the larger ones and every chain the
// launch cannot take (other cycle shapes, a learned iteration fallback,
// restart lengths above its limit).
#include <algorithm>
#include <atomic>
#include <numeric>
#include <thread>
#include <vector>

#include "bamg_internal.h"

// Largest chain the default (automatic) split sends to the persistent
// launch. Measured per GMRES iteration on the 512-chain batched workload
// (mixed precision, MI355X, 1024-thread workgroups): one workgroup per
// chain 0.23 ms below 2k states, 0.47 ms at 2k-5k and 0.95 ms at 5k-10k;
// the per-step solve 0.43, 0.55 and 0.59 ms.
constexpr int kBatchAutoMaxStates = 5000;

struct bamg_batch {
  int n = 0;
  int dev = 0;
  std::vector<bamg_handle *> h;
  std::vector<bamg_status> st;
  std::vector<hipStream_t> streams;
  std::vector<int> order;  // chains by decreasing nonzeros
  int solver = BAMG_BATCH_AUTO;
};

namespace {

void join_into(hipStream_t from, hipStream_t to) {
  hipEvent_t e;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
    bamg::fail(BAMG_E_DEVICE, "event create failed");
  (void)hipEventRecord(e, from);
  (void)hipStreamWaitEvent(to, e, 0);
  (void)hipEventDestroy(e);
}

// run f(chain, stream) over the batch with one thread per stream
template <class F>
void for_each_chain(bamg_batch *b, F f) {
  std::atomic<int> next{0};
  auto work = [&](int w) {
    (void)hipSetDevice(b->dev);
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= b->n) break;
      f(b->order[k], b->streams[w]);
    }
  };
  std::vector<std::thread> th;
  for (int w = 1; w < (int)b->streams.size(); ++w) th.emplace_back(work, w);
  work(0);
  for (auto &t : th) t.join();
}

}  // namespace

extern "C" {

bamg_status bamg_setup_batched(int32_t nchains, const bamg_csr *A, const bamg_geometry *geom,
                               const bamg_options *opt, const bamg_allocator *alloc,
                               int32_t nstreams, void *hip_stream, bamg_batch **out) {
  if (nchains < 1 || !A || !opt || !out || nstreams < 0 || nstreams > 32) return BAMG_E_ARG;
  bamg_batch *b = new (std::nothrow) bamg_batch();
  if (!b) return BAMG_E_NOMEM;
  b->n = nchains;
  b->h.assign(nchains, nullptr);
  b->st.assign(nchains, BAMG_E_ARG);
  b->order.resize(nchains);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int x, int y) { return A[x].nnz > A[y].nnz; });
  hipStream_t caller = (hipStream_t)hip_stream;
  const int ns = std::min<int>(nstreams ? nstreams : 4, nchains);
  if (hipGetDevice(&b->dev) != hipSuccess) {
    delete b;
    return BAMG_E_DEVICE;
  }
  for (int w = 0; w < ns; ++w) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      bamg_batch_destroy(b);
      return BAMG_E_DEVICE;
    }
    b->streams.push_back(s);
  }
  try {
    for (hipStream_t s : b->streams) join_into(caller, s);  // inputs are ready
    for_each_chain(b, [&](int i, hipStream_t s) {
      b->st[i] = bamg_setup(&A[i], geom ? &geom[i] : nullptr, &opt[i], alloc, s, &b->h[i]);
    });
    for (hipStream_t s : b->streams) join_into(s, caller);
  } catch (const bamg::Error &e) {
    bamg_batch_destroy(b);
    return e.code;
  }
  *out = b;
  return BAMG_OK;
}

bamg_status bamg_batch_status(const bamg_batch *b, int32_t i, bamg_status *setup_status,
                              bamg_handle **handle) {
  if (!b || i < 0 || i >= b->n) return BAMG_E_ARG;
  if (setup_status) *setup_status = b->st[i];
  if (handle) *handle = b->h[i];
  return BAMG_OK;
}

bamg_status bamg_gmres_solve_batched(bamg_batch *b, double *const *x, int32_t restart,
                                     double tol, int32_t max_iters, bamg_solve_info *infos,
                                     bamg_status *statuses, void *hip_stream) {
  if (!b || !x || !infos) return BAMG_E_ARG;
  for (int i = 0; i < b->n; ++i)
    if (b->h[i] && !x[i]) return BAMG_E_ARG;
  if (restart < 1 || restart > 255 || max_iters < 0 || !(tol > 0.0)) return BAMG_E_ARG;
  std::vector<bamg_status> st(b->n, BAMG_E_ARG);
  hipStream_t caller = (hipStream_t)hip_stream;
  // the persistent launch's chains, largest first
  std::vector<char> done(b->n, 0);
  std::vector<bamg_handle *> ph;
  std::vector<int> pidx;
  std::vector<double *> px;
  if (b->solver != BAMG_BATCH_STREAMS)
    for (int k = 0; k < b->n; ++k) {
      const int i = b->order[k];
      if (b->h[i] && bamg::batch_persistent_eligible(b->h[i], restart) &&
          (b->solver == BAMG_BATCH_PERSISTENT || b->h[i]->lv[0].n <= kBatchAutoMaxStates)) {
        pidx.push_back(i);
        ph.push_back(b->h[i]);
        px.push_back(x[i]);
        done[i] = 1;
      }
    }
  try {
    // the streams start after what the caller queued, not after the launch
    for (hipStream_t s : b->streams) join_into(caller, s);
    auto per_chain = [&]() {
      if ((int)ph.size() == b->n) return;
      for_each_chain(b, [&](int i, hipStream_t s) {
        if (done[i]) return;
        infos[i] = bamg_solve_info{};
        if (!b->h[i]) {
          st[i] = b->st[i];
          return;
        }
        st[i] = bamg_gmres_solve(b->h[i], x[i], restart, tol, max_iters, 0, &infos[i], s);
      });
    };
    std::vector<int> ord(ph.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::vector<bamg_solve_info> pinf(ph.size());
    std::vector<bamg_status> pst(ph.size());
    bamg::batch_persistent_solve(ph, ord, px.data(), restart, tol, max_iters, pinf.data(),
                                 pst.data(), caller, per_chain);
    for (size_t k = 0; k < ph.size(); ++k) {
      infos[pidx[k]] = pinf[k];
      st[pidx[k]] = pst[k];
    }
    for (hipStream_t s : b->streams) join_into(s, caller);
  } catch (const bamg::Error &e) {
    return e.code;
  }
  bool all = true;
  for (int i = 0; i < b->n; ++i) {
    if (statuses) statuses[i] = st[i];
    all = all && st[i] == BAMG_OK;
  }
  return all ? BAMG_OK : BAMG_NOT_CONVERGED;
}

bamg_status bamg_batch_set_solver(bamg_batch *b, int32_t solver) {
  if (!b || solver < BAMG_BATCH_AUTO || solver > BAMG_BATCH_STREAMS) return BAMG_E_ARG;
  b->solver = solver;
  return BAMG_OK;
}

void bamg_batch_destroy(bamg_batch *b) {
  if (!b) return;
  for (bamg_handle *h : b->h) bamg_destroy(h);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  delete b;
}

}  // extern "C"
