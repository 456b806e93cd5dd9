// Autotuner for the row-parallel sweeps of the V-cycle: the number of lanes
// that share one CSR row (1, 2 or 4) is chosen per level by timing a few
// weighted-Jacobi sweeps of the level's own matrix with HIP events, once per
// (device, rows, nonzeros, value type); the choice is cached for the life of
// the process. The sweeps sum each row in one fixed order whatever the lane
// count (k_sparse.hip, row_dot), so the choice changes the speed only, never
// a bit of the result. Candidates are tried from the fewest lanes up, and a
// wider one replaces the choice only when at least 3% faster, so near-ties
// (within timing noise) usually resolve the same way in every process.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "bamg_internal.h"

namespace bamg {

namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tune;
}  // namespace

template <class T>
int tune_lanes(Pool &pool, const Level &L, hipStream_t s) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  const auto key = std::make_tuple(dev, L.n, L.B.nnz, (int)sizeof(T));
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  const int avg = L.n ? (L.B.nnz + L.n - 1) / L.n : 1;
  int base = 1;
  while (base < avg && base < 64) base <<= 1;
  T *b = pool.get<T>(L.n), *x = pool.get<T>(L.n), *y = pool.get<T>(L.n);
  fill<T>(b, (T)1, L.n, s);
  fill<T>(x, (T)0, L.n, s);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int best = std::min(base, kMaxTunedLanes);
  float best_ms = 1e30f;
  const T om = (T)0.7;
  for (int lanes = std::max(1, base / 8); lanes <= std::min(kMaxTunedLanes, base * 2);
       lanes <<= 1) {
    jacobi<T>(L.B, (const T *)L.Bv, (const T *)L.dinv, om, b, x, y, lanes, s);  // warm
    HIPCHK(hipEventRecord(e0, s));
    for (int it = 0; it < 4; ++it) {
      jacobi<T>(L.B, (const T *)L.Bv, (const T *)L.dinv, om, b, x, y, lanes, s);
      jacobi<T>(L.B, (const T *)L.Bv, (const T *)L.dinv, om, b, y, x, lanes, s);
    }
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < 0.97f * best_ms) {
      best_ms = ms;
      best = lanes;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  pool.release(b);
  pool.release(x);
  pool.release(y);
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune.emplace(key, best);
  return best;
}

template int tune_lanes<double>(Pool &, const Level &, hipStream_t);
template int tune_lanes<float>(Pool &, const Level &, hipStream_t);

}  // namespace bamg
