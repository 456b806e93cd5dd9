// Sparse kernels on single vectors: SpMV variants, the fused weighted-Jacobi
// sweep of the smoother (Section 3), a colour-segment Kaczmarz sweep and the
// dense coarsest-level solve. All are HBM-bound: a CSR row is handled by a
// group of LPR lanes of a 64-wide wave so the column/value loads of a row
// are contiguous, and the group reduces its partial sums with cross-lane
// shuffles.
#include "bamg_internal.h"
#include "device_common.h"

namespace bamg {

constexpr int kSpThreads = 256;

// A lane's share of a CSR row, sum over k = k0, k0 + LPR, ... < e of
// val[k] * g(ci[k]), added in that order. U = 4 entries per round: their
// indices and values are loaded first, then the four gathers, so a short
// row costs one dependent round trip instead of a chain of them (8 per
// round raises the register count past what full occupancy allows, and is
// slower). Positions past the row end load the row's last entry again (no
// branches around the loads, so all of them are in flight together) and
// are not added.
template <class T, int LPR, class G>
__device__ __forceinline__ T lane_dot(int k0, int e, const int *__restrict__ ci,
                                      const T *__restrict__ val, G g) {
  constexpr int U = 4;
  T sum = 0;
  for (int k = k0; k < e; k += U * LPR) {
    int c[U];
    T v[U], xv[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int kk = min(k + j * LPR, e - 1);
      c[j] = ci[kk];
      v[j] = val[kk];
    }
#pragma unroll
    for (int j = 0; j < U; ++j) xv[j] = g(c[j]);
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (k + j * LPR < e) sum += v[j] * xv[j];
  }
  return sum;
}

// The sum of a CSR row, sum over k in [rs, e) of val[k] * g(ci[k]), in one
// fixed order whatever the number LPR <= 4 of lanes sharing the row, so
// results do not depend on the lanes a tuner picks: entry k goes to partial
// (k - rs) mod 4, each partial adds its entries in ascending order, and the
// four partials are combined as (p0+p1)+(p2+p3). Lane `lane` of the group
// holds the partials lane, lane + LPR, ...; a level of the combining tree is
// a cross-lane shuffle when the two partials sit in different lanes and a
// register add otherwise (both lanes of a shuffle form the same sum:
// addition is commutative). Every lane of the group returns the row sum.
// Loads as in lane_dot: U = 4 entries per round, indices and values first,
// then the gathers. Four partials keep every sweep kernel at full occupancy
// (eight took the one-lane sweep from 42 to 65 VGPRs).
constexpr int kCanon = 4;

template <class T, int LPR, class G>
__device__ __forceinline__ T row_dot(int rs, int e, int lane, const int *__restrict__ ci,
                                     const T *__restrict__ val, G g) {
  static_assert(LPR >= 1 && LPR <= kCanon, "canonical row sums take at most 4 lanes");
  constexpr int R = kCanon / LPR, U = 4, PH = R > U ? R / U : 1;
  T acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0;
  for (int k = rs + lane; k < e; k += PH * U * LPR) {
#pragma unroll
    for (int ph = 0; ph < PH; ++ph) {
      const int kp = k + ph * U * LPR;
      if (ph == 0 || kp < e) {
        int c[U];
        T v[U], xv[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
          const int kk = min(kp + j * LPR, e - 1);
          c[j] = ci[kk];
          v[j] = val[kk];
        }
#pragma unroll
        for (int j = 0; j < U; ++j) xv[j] = g(c[j]);
#pragma unroll
        for (int j = 0; j < U; ++j)
          if (kp + j * LPR < e) acc[(ph * U + j) % R] += v[j] * xv[j];
      }
    }
  }
#pragma unroll
  for (int st = 1; st < kCanon; st <<= 1) {
    if (st < LPR) {
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = acc[r] + __shfl_xor(acc[r], st, LPR);
    } else {
      const int step = st / LPR;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if ((r & step) == 0 && r + step < R) acc[r] = acc[r] + acc[r + step];
    }
  }
  return acc[0];
}

// Row sum for any LPR: the canonical order up to 4 lanes; wider groups
// (taken only by the transfers, whose lanes follow from the matrix shape)
// add their lanes' shares by a butterfly.
template <class T, int LPR, class G>
__device__ __forceinline__ T row_sum(int rs, int e, int lane, const int *__restrict__ ci,
                                     const T *__restrict__ val, G g) {
  if constexpr (LPR <= kCanon) {
    return row_dot<T, LPR>(rs, e, lane, ci, val, g);
  } else {
    return group_sum(lane_dot<T, LPR>(rs + lane, e, ci, val, g), LPR);
  }
}

// y = A x (mode 0), y = b - A x (mode 1), y = y + A x (mode 2)
template <class T, int LPR>
__global__ void __launch_bounds__(kSpThreads)
    k_spmv(int nr, const int *__restrict__ rp, const int *__restrict__ ci,
           const T *__restrict__ val, const T *__restrict__ x, T *__restrict__ y,
           const T *__restrict__ b, int mode) {
  const long gid = (long)xcd_block(blockIdx.x, gridDim.x) * kSpThreads + threadIdx.x;
  const int row = (int)(gid / LPR), lane = (int)(gid % LPR);
  if (row >= nr) return;  // whole groups leave together
  // row-wise operands are loaded first, beside the row pointers, so their
  // latency overlaps the row's gathers instead of following the reduction
  const T br = mode == 1 ? b[row] : mode == 2 ? y[row] : (T)0;
  const T sum = row_sum<T, LPR>(rp[row], rp[row + 1], lane, ci, val, [&](int c) { return x[c]; });
  if (lane == 0) {
    if (mode == 0)
      y[row] = sum;
    else if (mode == 1)
      y[row] = br - sum;
    else
      y[row] = br + sum;
  }
}

// x_out = x_in + omega dinv (b - A x_in); x_in == nullptr: x_in = 0.
template <class T, int LPR>
__global__ void __launch_bounds__(kSpThreads)
    k_jacobi(int nr, const int *__restrict__ rp, const int *__restrict__ ci,
             const T *__restrict__ val, const T *__restrict__ dinv, T omega,
             const T *__restrict__ b, const T *__restrict__ xin, T *__restrict__ xout) {
  const long gid = (long)xcd_block(blockIdx.x, gridDim.x) * kSpThreads + threadIdx.x;
  const int row = (int)(gid / LPR), lane = (int)(gid % LPR);
  if (row >= nr) return;
  if (xin == nullptr) {
    if (lane == 0) xout[row] = omega * dinv[row] * b[row];
    return;
  }
  const T xr = xin[row], dr = dinv[row], br = b[row];  // issued beside the row pointers
  const T sum =
      row_sum<T, LPR>(rp[row], rp[row + 1], lane, ci, val, [&](int c) { return xin[c]; });
  if (lane == 0) xout[row] = xr + omega * dr * (br - sum);
}

// Two sweeps from x = 0 in one pass: x1 = omega dinv b is formed on the fly
// wherever it is needed (same expression as the zero-start sweep, so the
// result equals two separate sweeps bit for bit), then
// x2 = x1 + omega dinv (b - A x1).
template <class T, int LPR>
__global__ void __launch_bounds__(kSpThreads)
    k_jacobi2(int nr, const int *__restrict__ rp, const int *__restrict__ ci,
              const T *__restrict__ val, const T *__restrict__ dinv, T omega,
              const T *__restrict__ b, T *__restrict__ xout) {
  const long gid = (long)xcd_block(blockIdx.x, gridDim.x) * kSpThreads + threadIdx.x;
  const int row = (int)(gid / LPR), lane = (int)(gid % LPR);
  if (row >= nr) return;
  const T dr = dinv[row], br = b[row];  // issued beside the row pointers
  const T sum = row_sum<T, LPR>(rp[row], rp[row + 1], lane, ci, val,
                                [&](int c) { return omega * dinv[c] * b[c]; });
  if (lane == 0) {
    const T x1 = omega * dr * br;
    xout[row] = x1 + omega * dr * (br - sum);
  }
}

int lanes_for(int nr, int nnz) {
  int avg = nr ? (nnz + nr - 1) / nr : 1;
  int l = 1;
  while (l < avg && l < 64) l <<= 1;
  return l;
}
static int pick_lanes(int nr, int nnz) { return lanes_for(nr, nnz); }

#define BAMG_LPR_SWITCH(LANES, KERNEL, GRIDROWS, ...)                                        \
  do {                                                                                       \
    const int lpr_ = (LANES);                                                                \
    const long thr_ = (long)(GRIDROWS) * lpr_;                                               \
    const int nb_ = ceil_div(thr_, kSpThreads);                                              \
    switch (lpr_) {                                                                          \
      case 1: KERNEL<T, 1><<<nb_, kSpThreads, 0, s>>>(__VA_ARGS__); break;                   \
      case 2: KERNEL<T, 2><<<nb_, kSpThreads, 0, s>>>(__VA_ARGS__); break;                   \
      case 4: KERNEL<T, 4><<<nb_, kSpThreads, 0, s>>>(__VA_ARGS__); break;                   \
      case 8: KERNEL<T, 8><<<nb_, kSpThreads, 0, s>>>(__VA_ARGS__); break;                   \
      case 16: KERNEL<T, 16><<<nb_, kSpThreads, 0, s>>>(__VA_ARGS__); break;                 \
      case 32: KERNEL<T, 32><<<nb_, kSpThreads, 0, s>>>(__VA_ARGS__); break;                 \
      default: KERNEL<T, 64><<<nb_, kSpThreads, 0, s>>>(__VA_ARGS__); break;                 \
    }                                                                                        \
    LAUNCHCHK();                                                                             \
  } while (0)

template <class T>
void spmv(const Csr &A, const T *val, const T *x, T *y, const T *b, int mode, int lanes,
          hipStream_t s) {
  if (A.nr <= 0) return;
  if (lanes <= 0) lanes = pick_lanes(A.nr, A.nnz);
  BAMG_LPR_SWITCH(lanes, k_spmv, A.nr, A.nr, A.rp, A.ci, val, x, y, b, mode);
}

template <class T>
void jacobi(const Csr &A, const T *val, const T *dinv, T omega, const T *b, const T *xin, T *xout,
            int lanes, hipStream_t s) {
  if (A.nr <= 0) return;
  if (lanes <= 0) lanes = pick_lanes(A.nr, A.nnz);
  if (xin == nullptr) lanes = 1;
  BAMG_LPR_SWITCH(lanes, k_jacobi, A.nr, A.nr, A.rp, A.ci, val, dinv, omega, b, xin, xout);
}

template <class T>
void jacobi2_from_zero(const Csr &A, const T *val, const T *dinv, T omega, const T *b, T *xout,
                       int lanes, hipStream_t s) {
  if (A.nr <= 0) return;
  if (lanes <= 0) lanes = pick_lanes(A.nr, A.nnz);
  BAMG_LPR_SWITCH(lanes, k_jacobi2, A.nr, A.nr, A.rp, A.ci, val, dinv, omega, b, xout);
}

// GMRES products on the finest level (FP64), with the level's lanes per row:
// y1 = y2 = A x (the second copy is the V-cycle's fixed input), and the
// same with x = w * scal[0] formed where it is gathered and stored as v
// (the next Arnoldi basis vector).
template <class T, int LPR>
__global__ void __launch_bounds__(kSpThreads)
    k_spmv_dual(int nr, const int *__restrict__ rp, const int *__restrict__ ci,
                const T *__restrict__ val, const T *__restrict__ x, T *__restrict__ y1,
                T *__restrict__ y2) {
  const long gid = (long)xcd_block(blockIdx.x, gridDim.x) * kSpThreads + threadIdx.x;
  const int row = (int)(gid / LPR), lane = (int)(gid % LPR);
  if (row >= nr) return;
  const T sum = row_sum<T, LPR>(rp[row], rp[row + 1], lane, ci, val, [&](int c) { return x[c]; });
  if (lane == 0) {
    y1[row] = sum;
    y2[row] = sum;
  }
}

template <class T, int LPR>
__global__ void __launch_bounds__(kSpThreads)
    k_spmv_dual_scaled(int nr, const int *__restrict__ rp, const int *__restrict__ ci,
                       const T *__restrict__ val, const T *__restrict__ w,
                       const T *__restrict__ scal, T *__restrict__ v, T *__restrict__ y1,
                       T *__restrict__ y2) {
  const long gid = (long)xcd_block(blockIdx.x, gridDim.x) * kSpThreads + threadIdx.x;
  const int row = (int)(gid / LPR), lane = (int)(gid % LPR);
  if (row >= nr) return;
  const T sc = scal[0], wr = w[row];
  const T sum = row_sum<T, LPR>(rp[row], rp[row + 1], lane, ci, val,
                                [&](int c) { return w[c] * sc; });
  if (lane == 0) {
    v[row] = wr * sc;
    y1[row] = sum;
    y2[row] = sum;
  }
}

void spmv_dual(const Csr &A, const double *val, const double *x, double *y1, double *y2,
               int lanes, hipStream_t s) {
  using T = double;
  if (A.nr <= 0) return;
  if (lanes <= 0) lanes = pick_lanes(A.nr, A.nnz);
  BAMG_LPR_SWITCH(lanes, k_spmv_dual, A.nr, A.nr, A.rp, A.ci, val, x, y1, y2);
}

void spmv_dual_scaled(const Csr &A, const double *val, const double *w, const double *scal,
                      double *v, double *y1, double *y2, int lanes, hipStream_t s) {
  using T = double;
  if (A.nr <= 0) return;
  if (lanes <= 0) lanes = pick_lanes(A.nr, A.nnz);
  BAMG_LPR_SWITCH(lanes, k_spmv_dual_scaled, A.nr, A.nr, A.rp, A.ci, val, w, scal, v, y1, y2);
}

// Kaczmarz row projections x <- x + (b_i - A_i x) / ||A_i||^2 A_i^T for the
// rows of one colour; rows of one colour share no column, so their updates
// touch disjoint entries of x and may run in any order.
template <class T>
__global__ void k_kaczmarz(const int *__restrict__ rp, const int *__restrict__ ci,
                           const T *__restrict__ val, const T *__restrict__ rowinv,
                           const int *__restrict__ rows, int nrows, const T *__restrict__ b,
                           T *__restrict__ x) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows) return;
  const int i = rows[t];
  T ax = 0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) ax += val[k] * x[ci[k]];
  const T c = (b[i] - ax) * rowinv[i];
  for (int k = rp[i]; k < rp[i + 1]; ++k) x[ci[k]] += c * val[k];
}

template <class T>
void kaczmarz_colour(const Csr &A, const T *val, const T *rowinv, const int *rows, int nrows,
                     const T *b, T *x, hipStream_t s) {
  if (nrows <= 0) return;
  if (!rowinv || !rows || !val) fail(BAMG_E_DEVICE, "kaczmarz_colour: missing buffer");
  k_kaczmarz<T><<<ceil_div(nrows, 128), 128, 0, s>>>(A.rp, A.ci, val, rowinv, rows, nrows, b, x);
  LAUNCHCHK();
}

// x = Bdag b (add: x += Bdag b) with Bdag dense FP64 row-major; one wave per row.
template <class T>
__global__ void __launch_bounds__(256) k_coarse_gemv(const double *__restrict__ Bd, int n,
                                                     const T *__restrict__ b, T *__restrict__ x,
                                                     int add) {
  const int row = blockIdx.x * 4 + threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (row >= n) return;
  double s = 0.0;
  const double *r = Bd + (size_t)row * n;
  for (int j = lane; j < n; j += kWave) s += r[j] * (double)b[j];
  s = group_sum(s, kWave);
  if (lane == 0) x[row] = add ? (T)((double)x[row] + s) : (T)s;
}

template <class T>
void coarse_gemv(const double *bdag, int n, const T *b, T *x, hipStream_t s, int add) {
  k_coarse_gemv<T><<<ceil_div(n, 4), 256, 0, s>>>(bdag, n, b, x, add);
  LAUNCHCHK();
}

__global__ void __launch_bounds__(256) k_dot_part(const double *__restrict__ x,
                                                  const double *__restrict__ y, int n,
                                                  double *__restrict__ part) {
  __shared__ double sh[4];
  double v = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256)
    v += x[i] * y[i];
  v = block_sum<256>(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

void dot_partials(const double *x, const double *y, int n, double *part, int nblk, hipStream_t s) {
  k_dot_part<<<nblk, 256, 0, s>>>(x, y, n, part);
  LAUNCHCHK();
}

#define INST(T)                                                                              \
  template void spmv<T>(const Csr &, const T *, const T *, T *, const T *, int, int,         \
                        hipStream_t);                                                        \
  template void jacobi<T>(const Csr &, const T *, const T *, T, const T *, const T *, T *,   \
                          int, hipStream_t);                                                 \
  template void jacobi2_from_zero<T>(const Csr &, const T *, const T *, T, const T *, T *,   \
                                     int, hipStream_t);                                      \
  template void kaczmarz_colour<T>(const Csr &, const T *, const T *, const int *, int,      \
                                   const T *, T *, hipStream_t);                             \
  template void coarse_gemv<T>(const double *, int, const T *, T *, hipStream_t, int);
INST(double)
INST(float)
#undef INST

}  // namespace bamg
