// Sparse kernels on single vectors: SpMV variants, the fused weighted-Jacobi
// sweep of the smoother (Section 3), a colour-segment Kaczmarz sweep and the
// dense coarsest-level solve. All are HBM-bound: a CSR row is handled by a
// group of LPR lanes of a 64-wide wave so the column/value loads of a row
// are contiguous, and the group reduces its partial sums with cross-lane
// shuffles.
#include "bamg_internal.h"
#include "device_common.h"
#include "sparse_row.h"

namespace bamg {

constexpr int kSpThreads = 256;      // default workgroup size of the row kernels
constexpr int kSpMaxThreads = 1024;  // largest the tuner may pick

// y = A x (mode 0), y = b - A x (mode 1), y = y + A x (mode 2)
template <class T, int LPR>
__global__ void __launch_bounds__(kSpMaxThreads)
    k_spmv(int nr, const int *__restrict__ rp, const int *__restrict__ ci,
           const T *__restrict__ val, const T *__restrict__ x, T *__restrict__ y,
           const T *__restrict__ b, int mode) {
  const long gid = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
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
__global__ void __launch_bounds__(kSpMaxThreads)
    k_jacobi(int nr, const int *__restrict__ rp, const int *__restrict__ ci,
             const T *__restrict__ val, const T *__restrict__ dinv, T omega,
             const T *__restrict__ b, const T *__restrict__ xin, T *__restrict__ xout) {
  const long gid = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int row = (int)(gid / LPR), lane = (int)(gid % LPR);
  if (row >= nr) return;
  if (xin == nullptr) {
    if (lane == 0) xout[row] = jacobi_first(omega, dinv[row], b[row]);
    return;
  }
  const T xr = xin[row], dr = dinv[row], br = b[row];  // issued beside the row pointers
  const T sum =
      row_sum<T, LPR>(rp[row], rp[row + 1], lane, ci, val, [&](int c) { return xin[c]; });
  if (lane == 0) xout[row] = jacobi_next(xr, omega, dr, br, sum);
}

// Two sweeps from x = 0 in one pass: x1 = omega dinv b is formed on the fly
// wherever it is needed (same expression as the zero-start sweep, so the
// result equals two separate sweeps bit for bit), then
// x2 = x1 + omega dinv (b - A x1).
template <class T, int LPR>
__global__ void __launch_bounds__(kSpMaxThreads)
    k_jacobi2(int nr, const int *__restrict__ rp, const int *__restrict__ ci,
              const T *__restrict__ val, const T *__restrict__ dinv, T omega,
              const T *__restrict__ b, T *__restrict__ xout) {
  const long gid = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int row = (int)(gid / LPR), lane = (int)(gid % LPR);
  if (row >= nr) return;
  const T dr = dinv[row], br = b[row];  // issued beside the row pointers
  const T sum = row_sum<T, LPR>(rp[row], rp[row + 1], lane, ci, val,
                                [&](int c) { return jacobi_first(omega, dinv[c], b[c]); });
  if (lane == 0) xout[row] = jacobi_next(jacobi_first(omega, dr, br), omega, dr, br, sum);
}

int lanes_for(int nr, int nnz) {
  int avg = nr ? (nnz + nr - 1) / nr : 1;
  int l = 1;
  while (l < avg && l < 64) l <<= 1;
  return l;
}
static int pick_lanes(int nr, int nnz) { return lanes_for(nr, nnz); }

#define BAMG_LPR_SWITCH(LANES, THREADS, KERNEL, GRIDROWS, ...)                               \
  do {                                                                                       \
    const int lpr_ = (LANES), nt_ = (THREADS) > 0 ? (THREADS) : kSpThreads;                  \
    const long thr_ = (long)(GRIDROWS) * lpr_;                                               \
    const int nb_ = ceil_div(thr_, nt_);                                                     \
    switch (lpr_) {                                                                          \
      case 1: KERNEL<T, 1><<<nb_, nt_, 0, s>>>(__VA_ARGS__); break;                          \
      case 2: KERNEL<T, 2><<<nb_, nt_, 0, s>>>(__VA_ARGS__); break;                          \
      case 4: KERNEL<T, 4><<<nb_, nt_, 0, s>>>(__VA_ARGS__); break;                          \
      case 8: KERNEL<T, 8><<<nb_, nt_, 0, s>>>(__VA_ARGS__); break;                          \
      case 16: KERNEL<T, 16><<<nb_, nt_, 0, s>>>(__VA_ARGS__); break;                        \
      case 32: KERNEL<T, 32><<<nb_, nt_, 0, s>>>(__VA_ARGS__); break;                        \
      default: KERNEL<T, 64><<<nb_, nt_, 0, s>>>(__VA_ARGS__); break;                        \
    }                                                                                        \
    LAUNCHCHK();                                                                             \
  } while (0)

template <class T>
void spmv(const Csr &A, const T *val, const T *x, T *y, const T *b, int mode, int lanes,
          hipStream_t s, int threads) {
  if (A.nr <= 0) return;
  if (lanes <= 0) lanes = pick_lanes(A.nr, A.nnz);
  BAMG_LPR_SWITCH(lanes, threads, k_spmv, A.nr, A.nr, A.rp, A.ci, val, x, y, b, mode);
}

template <class T>
void jacobi(const Csr &A, const T *val, const T *dinv, T omega, const T *b, const T *xin, T *xout,
            int lanes, hipStream_t s, int threads) {
  if (A.nr <= 0) return;
  if (lanes <= 0) lanes = pick_lanes(A.nr, A.nnz);
  if (xin == nullptr) lanes = 1;
  BAMG_LPR_SWITCH(lanes, threads, k_jacobi, A.nr, A.nr, A.rp, A.ci, val, dinv, omega, b, xin, xout);
}

template <class T>
void jacobi2_from_zero(const Csr &A, const T *val, const T *dinv, T omega, const T *b, T *xout,
                       int lanes, hipStream_t s, int threads) {
  if (A.nr <= 0) return;
  if (lanes <= 0) lanes = pick_lanes(A.nr, A.nnz);
  BAMG_LPR_SWITCH(lanes, threads, k_jacobi2, A.nr, A.nr, A.rp, A.ci, val, dinv, omega, b, xout);
}

// GMRES products on the finest level (FP64), with the level's lanes per row:
// y1 = y2 = A x (the second copy is the V-cycle's fixed input), and the
// same with x = w * scal[0] formed where it is gathered and stored as v
// (the next Arnoldi basis vector).
template <class T, int LPR>
__global__ void __launch_bounds__(kSpMaxThreads)
    k_spmv_dual(int nr, const int *__restrict__ rp, const int *__restrict__ ci,
                const T *__restrict__ val, const T *__restrict__ x, T *__restrict__ y1,
                T *__restrict__ y2) {
  const long gid = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int row = (int)(gid / LPR), lane = (int)(gid % LPR);
  if (row >= nr) return;
  const T sum = row_sum<T, LPR>(rp[row], rp[row + 1], lane, ci, val, [&](int c) { return x[c]; });
  if (lane == 0) {
    y1[row] = sum;
    y2[row] = sum;
  }
}

template <class T, int LPR>
__global__ void __launch_bounds__(kSpMaxThreads)
    k_spmv_dual_scaled(int nr, const int *__restrict__ rp, const int *__restrict__ ci,
                       const T *__restrict__ val, const T *__restrict__ w,
                       const T *__restrict__ scal, T *__restrict__ v, T *__restrict__ y1,
                       T *__restrict__ y2) {
  const long gid = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
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
               int lanes, hipStream_t s, int threads) {
  using T = double;
  if (A.nr <= 0) return;
  if (lanes <= 0) lanes = pick_lanes(A.nr, A.nnz);
  BAMG_LPR_SWITCH(lanes, threads, k_spmv_dual, A.nr, A.nr, A.rp, A.ci, val, x, y1, y2);
}

void spmv_dual_scaled(const Csr &A, const double *val, const double *w, const double *scal,
                      double *v, double *y1, double *y2, int lanes, hipStream_t s, int threads) {
  using T = double;
  if (A.nr <= 0) return;
  if (lanes <= 0) lanes = pick_lanes(A.nr, A.nnz);
  BAMG_LPR_SWITCH(lanes, threads, k_spmv_dual_scaled, A.nr, A.nr, A.rp, A.ci, val, w, scal, v, y1, y2);
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
                        hipStream_t, int);                                                   \
  template void jacobi<T>(const Csr &, const T *, const T *, T, const T *, const T *, T *,   \
                          int, hipStream_t, int);                                            \
  template void jacobi2_from_zero<T>(const Csr &, const T *, const T *, T, const T *, T *,   \
                                     int, hipStream_t, int);                                 \
  template void kaczmarz_colour<T>(const Csr &, const T *, const T *, const int *, int,      \
                                   const T *, T *, hipStream_t);                             \
  template void coarse_gemv<T>(const double *, int, const T *, T *, hipStream_t, int);
INST(double)
INST(float)
#undef INST

}  // namespace bamg
