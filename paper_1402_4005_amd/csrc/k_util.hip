// Integer utilities (prefix sums, CSR transposition), value permutations and
// the counter-based generator of the random test vectors.
#include <climits>

#include "bamg_internal.h"
#include "device_common.h"

namespace bamg {

// ------------------------------------------------------------ prefix sums
// Three passes: each block scans a tile of 2048 counts (8 per thread),
// one block scans the tile totals, then tile offsets are added.
constexpr int kScanThreads = 256, kScanItems = 8, kScanTile = kScanThreads * kScanItems;

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const int *__restrict__ in,
                                                             int *__restrict__ out, int n,
                                                             int *__restrict__ tile_sum) {
  __shared__ int sh[kScanThreads];
  const int t = threadIdx.x;
  const long base = (long)blockIdx.x * kScanTile + (long)t * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    long idx = base + i;
    v[i] = idx < n ? in[idx] : 0;
    s += v[i];
  }
  sh[t] = s;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int x = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  int run = sh[t] - s;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    long idx = base + i;
    run += v[i];
    if (idx < n) out[idx + 1] = run;
  }
  if (t == kScanThreads - 1) tile_sum[blockIdx.x] = sh[t];
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(int *__restrict__ tile_sum, int ntiles) {
  __shared__ int sh[kScanThreads];
  __shared__ int carry;
  const int t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int c0 = 0; c0 < ntiles; c0 += kScanThreads) {
    int idx = c0 + t;
    int v = idx < ntiles ? tile_sum[idx] : 0;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
      int x = t >= off ? sh[t - off] : 0;
      __syncthreads();
      sh[t] += x;
      __syncthreads();
    }
    if (idx < ntiles) tile_sum[idx] = carry + sh[t] - v;  // exclusive
    __syncthreads();
    if (t == kScanThreads - 1) carry += sh[t];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_add(int *__restrict__ out, int n,
                                                           const int *__restrict__ tile_off) {
  const long base = (long)blockIdx.x * kScanTile;
  const int off = tile_off[blockIdx.x];
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
    long idx = base + i;
    if (idx < n) out[idx + 1] += off;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
}

void scan_counts(Pool &pool, const int *counts, int *rp, int n, hipStream_t s) {
  if (n <= 0) {
    fill_i32(rp, 0, 1, s);
    return;
  }
  int ntiles = ceil_div(n, kScanTile);
  int *ts = pool.get<int>(ntiles);
  k_scan_tiles<<<ntiles, kScanThreads, 0, s>>>(counts, rp, n, ts);
  LAUNCHCHK();
  k_scan_sums<<<1, kScanThreads, 0, s>>>(ts, ntiles);
  LAUNCHCHK();
  k_scan_add<<<ntiles, kScanThreads, 0, s>>>(rp, n, ts);
  LAUNCHCHK();
  pool.release(ts);
}

int read_int(const int *dptr, hipStream_t s) {
  int v = 0;
  HIPCHK(hipMemcpyAsync(&v, dptr, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return v;
}

// ------------------------------------------------------------------ fills
template <class T>
__global__ void k_fill(T *p, T v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_iota(int *p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int)i;
}

void fill_i32(int *p, int v, size_t n, hipStream_t s) {
  if (!n) return;
  k_fill<int><<<ceil_div(n, 256), 256, 0, s>>>(p, v, n);
  LAUNCHCHK();
}
void iota_i32(int *p, size_t n, hipStream_t s) {
  if (!n) return;
  k_iota<<<ceil_div(n, 256), 256, 0, s>>>(p, n);
  LAUNCHCHK();
}
template <class T>
void fill(T *p, T v, size_t n, hipStream_t s) {
  if (!n) return;
  k_fill<T><<<ceil_div(n, 256), 256, 0, s>>>(p, v, n);
  LAUNCHCHK();
}
template void fill<double>(double *, double, size_t, hipStream_t);
template void fill<float>(float *, float, size_t, hipStream_t);

template <class T>
__global__ void k_copy_perm(T *__restrict__ out, const T *__restrict__ in,
                            const int *__restrict__ perm, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[perm[i]];
}
template <class T>
void copy_permuted(T *out, const T *in, const int *perm, int n, hipStream_t s) {
  if (n <= 0) return;
  k_copy_perm<T><<<ceil_div(n, 256), 256, 0, s>>>(out, in, perm, n);
  LAUNCHCHK();
}
template void copy_permuted<double>(double *, const double *, const int *, int, hipStream_t);
template void copy_permuted<float>(float *, const float *, const int *, int, hipStream_t);

template <class A, class B>
__global__ void k_convert(B *__restrict__ out, const A *__restrict__ in, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (B)in[i];
}
template <class A, class B>
void convert(B *out, const A *in, size_t n, hipStream_t s) {
  if (!n) return;
  k_convert<A, B><<<ceil_div(n, 256), 256, 0, s>>>(out, in, n);
  LAUNCHCHK();
}
template void convert<double, float>(float *, const double *, size_t, hipStream_t);
template void convert<float, double>(double *, const float *, size_t, hipStream_t);
template void convert<double, double>(double *, const double *, size_t, hipStream_t);

// ---------------------------------------------------------- CSR transpose
// Counting sort by column; entries of a column are then put in increasing
// row order so the result does not depend on the order of the atomics.
__global__ void k_count_cols(const int *__restrict__ ci, int nnz, int *__restrict__ cnt) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) atomicAdd(&cnt[ci[k]], 1);
}

__global__ void k_scatter_rows(const int *__restrict__ rp, const int *__restrict__ ci, int nr,
                               int *__restrict__ cursor, int *__restrict__ tci,
                               int *__restrict__ perm) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    int pos = atomicAdd(&cursor[ci[k]], 1);
    tci[pos] = i;
    perm[pos] = k;
  }
}

// Bitonic sorting network over N registers (static indices only, so the
// arrays stay in registers); entries past the segment hold INT_MAX.
template <int N>
__device__ __forceinline__ void bitonic_regs(int (&k)[N], int (&v)[N]) {
#pragma unroll
  for (int size = 2; size <= N; size <<= 1)
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ stride;
        if (l > i) {
          const bool up = (i & size) == 0;
          if ((k[i] > k[l]) == up) {
            const int t0 = k[i], t1 = v[i];
            k[i] = k[l];
            v[i] = v[l];
            k[l] = t0;
            v[l] = t1;
          }
        }
      }
}

template <int N>
__device__ __forceinline__ void sort_short(int *__restrict__ key, int *__restrict__ val, int a,
                                           int m) {
  int kk[N], vv[N];
#pragma unroll
  for (int p = 0; p < N; ++p) {
    kk[p] = p < m ? key[a + p] : INT_MAX;
    vv[p] = p < m ? val[a + p] : 0;
  }
  bitonic_regs<N>(kk, vv);
#pragma unroll
  for (int p = 0; p < N; ++p)
    if (p < m) {
      key[a + p] = kk[p];
      val[a + p] = vv[p];
    }
}

// Sort each CSR segment by key (keys within a segment are distinct), with
// the values permuted alongside. Segments of up to 32 entries are sorted by
// their own thread in registers; longer ones are appended to a list for
// k_sort_long (one counter update per wave).
__global__ void k_sort_segments(const int *__restrict__ rp, int nr, int *__restrict__ key,
                                int *__restrict__ val, int *__restrict__ longseg,
                                int *__restrict__ nlong) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  bool is_long = false;
  if (j < nr) {
    const int a = rp[j], m = rp[j + 1] - a;
    if (m > 32)
      is_long = true;
    else if (m > 16)
      sort_short<32>(key, val, a, m);
    else if (m > 8)
      sort_short<16>(key, val, a, m);
    else if (m > 1)
      sort_short<8>(key, val, a, m);
  }
  const unsigned long long bl = __ballot(is_long);
  if (bl) {
    const int lane = threadIdx.x % kWave;
    int base = 0;
    if (lane == 0) base = atomicAdd(nlong, (int)__popcll(bl));
    base = __shfl(base, 0, kWave);
    if (is_long) longseg[base + __popcll(bl & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))))] = j;
  }
}

// Long segments: one 64-thread workgroup per listed segment (grid-stride over
// the device-side count), bitonic sort in LDS of up to kLongCap entries;
// beyond that, an insertion sort by one thread.
constexpr int kLongCap = 2048;

__global__ void __launch_bounds__(64)
    k_sort_long(const int *__restrict__ rp, const int *__restrict__ longseg,
                const int *__restrict__ nlong, int *__restrict__ key, int *__restrict__ val) {
  __shared__ int ks[kLongCap], vs[kLongCap];
  const int nl = *nlong, t = threadIdx.x;
  for (int w = blockIdx.x; w < nl; w += gridDim.x) {
    const int j = longseg[w];
    const int a = rp[j], m = rp[j + 1] - a;
    if (m > kLongCap) {
      if (t == 0)
        for (int p = a + 1; p < a + m; ++p) {
          const int kk = key[p], vv = val[p];
          int q = p - 1;
          while (q >= a && key[q] > kk) {
            key[q + 1] = key[q];
            val[q + 1] = val[q];
            --q;
          }
          key[q + 1] = kk;
          val[q + 1] = vv;
        }
      __syncthreads();
      continue;
    }
    int P2 = 1;
    while (P2 < m) P2 <<= 1;
    for (int p = t; p < P2; p += 64) {
      ks[p] = p < m ? key[a + p] : INT_MAX;
      vs[p] = p < m ? val[a + p] : 0;
    }
    __syncthreads();
    for (int size = 2; size <= P2; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = t; i < (P2 >> 1); i += 64) {
          const int lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
          const bool up = (lo & size) == 0;
          if ((ks[lo] > ks[hi]) == up) {
            const int k0 = ks[lo], v0 = vs[lo];
            ks[lo] = ks[hi];
            vs[lo] = vs[hi];
            ks[hi] = k0;
            vs[hi] = v0;
          }
        }
        __syncthreads();
      }
    for (int p = t; p < m; p += 64) {
      key[a + p] = ks[p];
      val[a + p] = vs[p];
    }
    __syncthreads();
  }
}

void transpose_pattern(Pool &pool, const Csr &A, Csr &At, int *&perm, hipStream_t s) {
  At.nr = A.nc;
  At.nc = A.nr;
  At.nnz = A.nnz;
  At.rp = pool.get<int>(At.nr + 1);
  At.ci = pool.get<int>(At.nnz);
  perm = pool.get<int>(At.nnz);
  int *cnt = pool.get<int>(At.nr + 1);
  fill_i32(cnt, 0, At.nr, s);
  if (A.nnz) {
    k_count_cols<<<ceil_div(A.nnz, 256), 256, 0, s>>>(A.ci, A.nnz, cnt);
    LAUNCHCHK();
  }
  scan_counts(pool, cnt, At.rp, At.nr, s);
  HIPCHK(hipMemcpyAsync(cnt, At.rp, sizeof(int) * At.nr, hipMemcpyDeviceToDevice, s));
  if (A.nr) {
    k_scatter_rows<<<ceil_div(A.nr, 256), 256, 0, s>>>(A.rp, A.ci, A.nr, cnt, At.ci, perm);
    LAUNCHCHK();
  }
  if (At.nr) {
    int *longseg = pool.get<int>(At.nr + 1);  // [count, segments...]
    fill_i32(longseg, 0, 1, s);
    k_sort_segments<<<ceil_div(At.nr, 256), 256, 0, s>>>(At.rp, At.nr, At.ci, perm, longseg + 1,
                                                         longseg);
    LAUNCHCHK();
    k_sort_long<<<std::min(1024, At.nr), 64, 0, s>>>(At.rp, longseg + 1, longseg, At.ci, perm);
    LAUNCHCHK();
    pool.release(longseg);
  }
  pool.release(cnt);
}

__global__ void k_diag_pos(const int *__restrict__ rp, const int *__restrict__ ci, int n,
                           int *__restrict__ dpos) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int lo = rp[i], hi = rp[i + 1] - 1, pos = -1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    int c = ci[mid];
    if (c == i) {
      pos = mid;
      break;
    }
    if (c < i)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  dpos[i] = pos;
}

void diag_positions(const Csr &A, int *dpos, hipStream_t s) {
  if (!A.nr) return;
  k_diag_pos<<<ceil_div(A.nr, 256), 256, 0, s>>>(A.rp, A.ci, A.nr, dpos);
  LAUNCHCHK();
}

// ------------------------------------------------------ random test vectors
// Element (i, k) of side s (0 = right vectors V, 1 = left vectors U) is the
// top 53 bits of the first Philox-4x64-10 word for counter (i, k, s, 0) and
// key (seed, 0), mapped to [-1, 1). Column 0 of U is the constant vector.
template <class T>
__global__ void k_testvecs(T *__restrict__ U, T *__restrict__ V, int n, int r, uint64_t seed) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n * r) return;
  int i = (int)(idx / r), k = (int)(idx % r);
  V[idx] = (T)uniform_pm1(seed, 0, (uint64_t)k, (uint64_t)i);
  U[idx] = k == 0 ? (T)1 : (T)uniform_pm1(seed, 1, (uint64_t)k, (uint64_t)i);
}

void philox_testvecs(void *U, void *V, int prec, int n, int r, uint64_t seed, hipStream_t s) {
  long tot = (long)n * r;
  if (prec == 0)
    k_testvecs<double><<<ceil_div(tot, 256), 256, 0, s>>>((double *)U, (double *)V, n, r, seed);
  else
    k_testvecs<float><<<ceil_div(tot, 256), 256, 0, s>>>((float *)U, (float *)V, n, r, seed);
  LAUNCHCHK();
}

}  // namespace bamg
