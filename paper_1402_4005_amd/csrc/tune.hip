// Autotuner for the row-parallel sweeps of the V-cycle. Two choices per
// level, found by timing a few weighted-Jacobi sweeps of the level's own
// matrix with HIP events, once per (device, rows, nonzeros, value type) and
// cached for the life of the process:
//  * lanes per CSR row (1, 2 or 4): the sweeps sum each row in one fixed
//    order whatever the lane count (sparse_row.h, row_dot);
//  * workgroup size (128, 256, 512 or 1024 threads): a row's work does not
//    depend on the workgroup it falls in;
// so the choices change the speed only, never a bit of the result. The
// candidates are tried in a fixed order (the defaults first), and a later
// one replaces the choice only when at least 3% faster, so near-ties
// (within timing noise) usually resolve the same way in every process.
// Levels too small to fill the chip are not timed (see below).
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>

#include "bamg_internal.h"

namespace bamg {

namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, std::pair<int, int>> g_tune;
}  // namespace

template <class T>
void tune_sweeps(Pool &pool, Level &L, hipStream_t s) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  const auto key = std::make_tuple(dev, L.n, L.B.nnz, (int)sizeof(T));
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      L.lanes = it->second.first;
      L.threads = it->second.second;
      return;
    }
  }
  const int avg = L.n ? (L.B.nnz + L.n - 1) / L.n : 1;
  int base = 1;
  while (base < avg && base < 64) base <<= 1;
  const int dlanes = std::min(base, kMaxTunedLanes);
  if ((long)L.n * dlanes < 256L * 256) {
    // A level too small to fill the chip (under 256 workgroups of 256
    // threads at the default lanes): its sweep is bound by the launch and
    // one pass of dependent loads, so it takes the default lanes and the
    // most workgroups (128 threads) untimed. Back-to-back timing of such
    // short launches measures noise, and a choice of a few large
    // workgroups made a sweep inside the cycle twice as long (Delaunay
    // 262,144, level 3 of 1,814 rows: 7.0 against 3.5 us).
    L.lanes = dlanes;
    L.threads = 128;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune.emplace(key, std::make_pair(L.lanes, L.threads));
    return;
  }
  T *b = pool.get<T>(L.n), *x = pool.get<T>(L.n), *y = pool.get<T>(L.n);
  fill<T>(b, (T)1, L.n, s);
  fill<T>(x, (T)0, L.n, s);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int best = std::min(base, kMaxTunedLanes), best_threads = 256;
  float best_ms = 1e30f;
  const T om = (T)0.7;
  auto time_of = [&](int lanes, int threads) {
    jacobi<T>(L.B, (const T *)L.Bv, (const T *)L.dinv, om, b, x, y, lanes, s, threads);  // warm
    HIPCHK(hipEventRecord(e0, s));
    for (int it = 0; it < 4; ++it) {
      jacobi<T>(L.B, (const T *)L.Bv, (const T *)L.dinv, om, b, x, y, lanes, s, threads);
      jacobi<T>(L.B, (const T *)L.Bv, (const T *)L.dinv, om, b, y, x, lanes, s, threads);
    }
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    return ms;
  };
  // lanes at the default workgroup size, then the workgroup size at those lanes
  for (int lanes = std::max(1, base / 8); lanes <= std::min(kMaxTunedLanes, base * 2);
       lanes <<= 1) {
    const float ms = time_of(lanes, 256);
    if (ms < 0.97f * best_ms) {
      best_ms = ms;
      best = lanes;
    }
  }
  for (int threads : {128, 512, 1024}) {
    const float ms = time_of(best, threads);
    if (ms < 0.97f * best_ms) {
      best_ms = ms;
      best_threads = threads;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  pool.release(b);
  pool.release(x);
  pool.release(y);
  L.lanes = best;
  L.threads = best_threads;
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune.emplace(key, std::make_pair(best, best_threads));
}

template void tune_sweeps<double>(Pool &, Level &, hipStream_t);
template void tune_sweeps<float>(Pool &, Level &, hipStream_t);

}  // namespace bamg
