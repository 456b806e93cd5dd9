// Coarsest-level dense algebra (FP64 always):
//  * the r smallest generalized singular triplets of eq.
//    generalized_eigenvalue: B_L v = sigma M_L u, B_L^T u = sigma N_L v. With
//    Cholesky factors M = L_M L_M^T, N = L_N L_N^T this is the ordinary SVD of
//    Bt = L_M^-1 B_L L_N^-T; u = L_M^-T ut, v = L_N^-T vt.
//  * the Moore-Penrose pseudo-inverse of B_L used by the coarse-grid
//    correction (eq. coarse_grid_correction), from the SVD of B_L with the
//    one zero singular value (1^T B_L = 0, Section 5) dropped.
// The SVD is one-sided Jacobi (Hestenes): column pairs of W are rotated until
// orthogonal. Blocks of columns are paired by the round-robin (circle)
// schedule, so one round treats disjoint block pairs in parallel, one
// workgroup per block pair, one launch per round.
#include <algorithm>

#include "bamg_internal.h"
#include "device_common.h"

namespace bamg {

template <class T>
__global__ void k_csr_to_dense(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                               const T *__restrict__ v, double *__restrict__ D) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int a = rp[i]; a < rp[i + 1]; ++a) D[(size_t)i * n + ci[a]] += (double)v[a];
}

void csr_to_dense(const Csr &A, const void *val, int prec, double *D, hipStream_t s) {
  const int n = A.nr;
  HIPCHK(hipMemsetAsync(D, 0, sizeof(double) * (size_t)n * n, s));
  if (prec == 0)
    k_csr_to_dense<double><<<ceil_div(n, 128), 128, 0, s>>>(n, A.rp, A.ci, (const double *)val, D);
  else
    k_csr_to_dense<float><<<ceil_div(n, 128), 128, 0, s>>>(n, A.rp, A.ci, (const float *)val, D);
  LAUNCHCHK();
}

// Cholesky factorisations A = L L^T in place (lower triangle, row-major;
// the strict upper triangle is zeroed), one workgroup per matrix (blockIdx
// 0: A0, 1: A1). Right-looking by panels of nb columns: the panel (rows
// j0.., nb columns) is factored in LDS, written back, and the trailing lower
// triangle is updated with the panel's columns. Every entry receives the
// same updates in the same order as the column-by-column algorithm
// (a -= l_ij l_kj for j ascending), so the factor equals it bit for bit.
// flag[0] = 1 if a pivot is not positive (not SPD).
__global__ void __launch_bounds__(1024) k_cholesky(double *__restrict__ A0, double *__restrict__ A1,
                                                   int n, int nbmax, int *__restrict__ flag) {
  extern __shared__ double pan[];  // (n - j0) x nb, row-major, stride nbmax + 1 (odd: no
                                   // bank conflicts down a column)
  double *__restrict__ A = blockIdx.x == 0 ? A0 : A1;
  const int t = threadIdx.x, nt = blockDim.x, ld = nbmax + 1;
  for (int j0 = 0; j0 < n; j0 += nbmax) {
    const int nb = min(nbmax, n - j0), m = n - j0;
    for (int e = t; e < m * nb; e += nt) {
      const int i = e / nb, c = e % nb;
      pan[i * ld + c] = A[(size_t)(j0 + i) * n + j0 + c];
    }
    __syncthreads();
    for (int c = 0; c < nb; ++c) {
      if (t == 0) {
        const double d = pan[c * ld + c];
        if (!(d > 0.0)) {
          flag[0] = 1;
          pan[c * ld + c] = 1.0;
        } else {
          pan[c * ld + c] = sqrt(d);
        }
      }
      __syncthreads();
      const double inv = 1.0 / pan[c * ld + c];
      for (int i = c + 1 + t; i < m; i += nt) pan[i * ld + c] *= inv;
      __syncthreads();
      // remaining panel columns cc > c, rows i >= cc
      const int w = nb - c - 1;
      for (int e = t; e < (m - c - 1) * w; e += nt) {
        const int i = c + 1 + e / w, cc = c + 1 + e % w;
        if (cc <= i) pan[i * ld + cc] -= pan[i * ld + c] * pan[cc * ld + c];
      }
      __syncthreads();
    }
    for (int e = t; e < m * nb; e += nt) {
      const int i = e / nb, c = e % nb;
      A[(size_t)(j0 + i) * n + j0 + c] = pan[i * ld + c];
    }
    // trailing lower triangle: rows i, columns k with j0 + nb <= k <= i
    const int mt = m - nb;
    for (long e = t; e < (long)mt * mt; e += nt) {
      const int ii = (int)(e / mt), kk = (int)(e % mt);
      if (kk > ii) continue;
      const double *li = pan + (size_t)(nb + ii) * ld, *lk = pan + (size_t)(nb + kk) * ld;
      double a = A[(size_t)(j0 + nb + ii) * n + j0 + nb + kk];
      for (int c = 0; c < nb; ++c) a -= li[c] * lk[c];
      A[(size_t)(j0 + nb + ii) * n + j0 + nb + kk] = a;
    }
    __syncthreads();
  }
  for (long e = t; e < (long)n * n; e += nt) {
    const int i = (int)(e / n), k = (int)(e % n);
    if (k > i) A[e] = 0.0;
  }
}

// Factor A0 and (when not null) A1, both n x n; flag is a device int the
// caller owns. Returns BAMG_E_COARSE if either is not positive definite.
static void cholesky_blocked(double *A0, double *A1, int n, int *flag, hipStream_t s);

// Above this order the factorisation runs blocked over many workgroups
// (cholesky_blocked); one workgroup per matrix at or below it.
constexpr int kCholOneWorkgroupMax = 384;

int cholesky2(double *A0, double *A1, int n, int *flag, hipStream_t s) {
  if (n > kCholOneWorkgroupMax) {
    fill_i32(flag, 0, 1, s);
    cholesky_blocked(A0, A1, n, flag, s);
    return read_int(flag, s) ? BAMG_E_COARSE : BAMG_OK;
  }
  int dev = 0, maxlds = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  int nb = 32;
  while (nb > 1 && sizeof(double) * (size_t)n * (nb + 1) > (size_t)maxlds) nb >>= 1;
  const size_t shm = sizeof(double) * (size_t)n * (nb + 1);
  if (shm > (size_t)maxlds) fail(BAMG_E_ARG, "cholesky: matrix too large for an LDS panel");
  HIPCHK(hipFuncSetAttribute((const void *)k_cholesky, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)shm));
  fill_i32(flag, 0, 1, s);
  k_cholesky<<<A1 ? 2 : 1, 1024, shm, s>>>(A0, A1, n, nb, flag);
  LAUNCHCHK();
  return read_int(flag, s) ? BAMG_E_COARSE : BAMG_OK;
}

// Forward substitution L Y = X for the columns of X (n x ncols, row-major,
// leading dimension ldx), in place. Each workgroup holds a slab of sw
// columns in LDS and eliminates row by row (right-looking): once row k is
// final, every later row subtracts L[i][k] times it. The columns of L are
// staged in LDS pw at a time (rows k0..n-1 of columns k0..k0+pw-1, row
// stride pw + 1), so a step waits on LDS and a workgroup barrier only.
constexpr int kTrsmStep = 8;

__global__ void __launch_bounds__(1024) k_trsm_slab(const double *__restrict__ L,
                                                    double *__restrict__ X, int n, int ncols,
                                                    int ldx, int sw, int pw) {
  extern __shared__ double xs[];  // n x sw, then the panel of L
  double *lp = xs + (size_t)n * sw;
  const int t = threadIdx.x, nt = blockDim.x;
  const int c = t % sw, ro = t / sw, nro = nt / sw;
  const int col = blockIdx.x * sw + c;
  for (int e = t; e < n * sw; e += nt) {
    const int i = e / sw, cc = e % sw, g = blockIdx.x * sw + cc;
    xs[e] = g < ncols ? X[(size_t)i * ldx + g] : 0.0;
  }
  for (int k0 = 0; k0 < n; k0 += pw) {
    const int w = min(pw, n - k0);
    __syncthreads();  // the previous panel is no longer read
    for (int e = t; e < (n - k0) * w; e += nt) {
      const int i = e / w, j = e % w;
      lp[(size_t)i * (pw + 1) + j] = L[(size_t)(k0 + i) * n + k0 + j];
    }
    __syncthreads();
    // kTrsmStep rows per step: every thread of column c solves the step's
    // diagonal block itself (the same operations in the same order as one
    // row at a time), then the rows below subtract the step's columns in
    // order, so a workgroup barrier comes once per step
    for (int k = k0; k < k0 + w; k += kTrsmStep) {
      const int b = min(kTrsmStep, k0 + w - k);
      double xb[kTrsmStep];
#pragma unroll
      for (int q = 0; q < kTrsmStep; ++q) {
        if (q < b) {
          const double *lr = lp + (size_t)(k + q - k0) * (pw + 1) + (k - k0);  // row k + q
          double v = xs[(k + q) * sw + c];
#pragma unroll
          for (int p = 0; p < q; ++p) v -= lr[p] * xb[p];
          xb[q] = v / lr[q];
        }
      }
      if (ro == 0 && col < ncols)
        for (int q = 0; q < b; ++q) X[(size_t)(k + q) * ldx + col] = xb[q];
      for (int i = k + b + ro; i < n; i += nro) {
        const double *lr = lp + (size_t)(i - k0) * (pw + 1) + (k - k0);
        double v = xs[i * sw + c];
#pragma unroll
        for (int q = 0; q < kTrsmStep; ++q)
          if (q < b) v -= lr[q] * xb[q];
        xs[i * sw + c] = v;
      }
      __syncthreads();
    }
  }
}

void trsm_lower_cols(const double *L, double *X, int n, int ncols, int ldx, hipStream_t s) {
  int dev = 0, maxlds = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  // slab of sw columns of X and a panel of pw columns of L (rows padded to
  // pw + 1): the widest that fit, the panel shrinking to 8 first, then the
  // slab to 8, then either further
  auto bytes = [&](int sw, int pw) {
    return sizeof(double) * ((size_t)n * sw + (size_t)n * (pw + 1));
  };
  int sw = 32, pw = 32;
  while (bytes(sw, pw) > (size_t)maxlds && (sw > 1 || pw > 1)) {
    if (pw > 8 || (sw <= 8 && pw > 1))
      pw >>= 1;
    else
      sw >>= 1;
  }
  const size_t shm = bytes(sw, pw);
  if (shm > (size_t)maxlds) fail(BAMG_E_ARG, "trsm: matrix too large for an LDS slab");
  HIPCHK(hipFuncSetAttribute((const void *)k_trsm_slab,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  k_trsm_slab<<<ceil_div(ncols, sw), 1024, shm, s>>>(L, X, n, ncols, ldx, sw, pw);
  LAUNCHCHK();
}

__global__ void k_transpose_dense(const double *__restrict__ A, double *__restrict__ At, int n) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int y = threadIdx.y; y < 32; y += blockDim.y) {
    const int r = by + y, c = bx + threadIdx.x;
    if (r < n && c < n) tile[y][threadIdx.x] = A[(size_t)r * n + c];
  }
  __syncthreads();
  for (int y = threadIdx.y; y < 32; y += blockDim.y) {
    const int r = bx + y, c = by + threadIdx.x;
    if (r < n && c < n) At[(size_t)r * n + c] = tile[threadIdx.x][y];
  }
}

void transpose_dense(const double *A, double *At, int n, hipStream_t s) {
  dim3 g(ceil_div(n, 32), ceil_div(n, 32)), b(32, 8);
  k_transpose_dense<<<g, b, 0, s>>>(A, At, n);
  LAUNCHCHK();
}

// ------------------------------------------------------------ Jacobi SVD
// Block one-sided Jacobi. The columns of W are split into blocks of bs
// columns (bs = 8 or 16); the blocks are paired by the round-robin schedule,
// one workgroup per block pair. A workgroup loads its 2 bs columns Wc into
// LDS and forms their Gram matrix G = Wcᵀ Wc once (FP64 MFMA). The pair's
// rotations are then found and applied on G (G <- Jᵀ G J, bs disjoint pairs
// at a time): in the first round of a sweep all pairs of the 2 bs columns,
// afterwards only the pairs across the two blocks, so each column pair of W
// is visited once per sweep. They accumulate in a 2bs x 2bs matrix R, and
// the columns of W and J are multiplied by R once (FP64 MFMA), from the LDS
// copy straight to memory. The rotation test and angle are those of
// one-sided Jacobi: the inner products of the rotated columns are the
// entries of the rotated G. A sweep ends the iteration when it finds nothing
// to rotate; its tests are made on Gram matrices formed afresh from W. Only
// the block rounds need a grid-wide barrier.
constexpr int kSvdMaxSweeps = 80;

typedef double svd_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int rr_index(int j, int round, int m) {
  return j == 0 ? 0 : 1 + (j - 1 + round) % (m - 1);
}

// Columns (p, q), p < q, rotated as pair k (0 <= k < bs) in inner round ir
// (0 <= ir < 2 bs - 1) of a block pair of 2 bs columns, bs a power of two:
// all pairs by the round-robin schedule (all = true), else column k of the
// first block with column bs + (k + ir) mod bs. The schedule's remainders
// are taken by one conditional subtraction, not an integer division.
__device__ __forceinline__ void svd_pair(int k, int ir, int bs, bool all, int &p, int &q) {
  if (!all) {
    p = k;
    q = bs + ((k + ir) & (bs - 1));
    return;
  }
  const int m1 = 2 * bs - 1;
  int a = 0;
  if (k != 0) {
    a = k - 1 + ir;
    if (a >= m1) a -= m1;
    ++a;
  }
  int b = m1 - 1 - k + ir;  // position 2 bs - 1 - k >= 1
  if (b >= m1) b -= m1;
  ++b;
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// One-sided Jacobi rotation of columns p < q with inner products
// al = |w_p|^2, be = |w_q|^2, ga = w_p . w_q: (c, s) with w_p <- c w_p - s w_q,
// w_q <- s w_p + c w_q, zeroing the new inner product; none when the pair is
// orthogonal to the tolerance (|ga| <= tol sqrt(al be)).
constexpr double kSvdTol = 1e-15;
// whether svd_rotation rotates the pair (the same test, without the angle)
__device__ __forceinline__ bool svd_needs_rotation(double al, double be, double ga) {
  return !(ga == 0.0 || ga * ga <= kSvdTol * kSvdTol * (al * be));
}
__device__ __forceinline__ bool svd_rotation(double al, double be, double ga, double &c,
                                             double &sn) {
  c = 1.0;
  sn = 0.0;
  if (!svd_needs_rotation(al, be, ga)) return false;
  const double zeta = (be - al) / (2.0 * ga);
  const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  c = rsqrt(1.0 + t * t);
  sn = c * t;
  return true;
}

// D (16 x 16 tile) += A B over k = 4 k0 .. 4 k1 - 1 with A[i][k] = a(i, k),
// B[k][j] = b(k, j); lane l supplies A[l % 16][k] and B[k][l % 16] for
// k = 4 kk + l / 16 and receives D[l / 16 + 4 r][l % 16] in acc[r].
template <class FA, class FB>
__device__ __forceinline__ svd_d4 mfma_tile(int k0, int k1, FA a, FB b, svd_d4 acc) {
  const int l = threadIdx.x % kWave;
  for (int kk = k0; kk < k1; ++kk) {
    const int k = 4 * kk + l / 16;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a(l % 16, k), b(k, l % 16), acc, 0, 0, 0);
  }
  return acc;
}

// Make this wave's LDS writes visible to its other lanes before they read
// (one wave only: no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- blocked Cholesky
// A = L L^T by kCb-column block steps, each three launches over both
// matrices (A0 and A1 by grid index): the diagonal block factored in LDS by
// the column algorithm; the block column below it solved against that
// factor (a row per lane); the trailing lower triangle updated tile by tile,
// C_IJ -= A_Ik A_Jk^T, on FP64 MFMA. Lower triangle row-major in place; the
// strict upper triangle is zeroed; flag[0] |= 1 if a pivot is not positive.
constexpr int kCb = 32;

__global__ void __launch_bounds__(256) k_chol_diag(double *__restrict__ A0,
                                                   double *__restrict__ A1, int n, int k0,
                                                   int *__restrict__ flag) {
  __shared__ double D[kCb][kCb + 1];
  double *__restrict__ A = blockIdx.x == 0 ? A0 : A1;
  const int b = min(kCb, n - k0), t = threadIdx.x;
  for (int e = t; e < b * b; e += 256) D[e / b][e % b] = A[(size_t)(k0 + e / b) * n + k0 + e % b];
  __syncthreads();
  for (int c = 0; c < b; ++c) {
    if (t == 0) {
      double d = D[c][c];
      if (!(d > 0.0)) {
        atomicOr(flag, 1);
        d = 1.0;
      }
      D[c][c] = sqrt(d);
    }
    __syncthreads();
    const double inv = 1.0 / D[c][c];
    for (int i = c + 1 + t; i < b; i += 256) D[i][c] *= inv;
    __syncthreads();
    const int w = b - c - 1;
    for (int e = t; e < w * w; e += 256) {
      const int i = c + 1 + e / w, j = c + 1 + e % w;
      if (j <= i) D[i][j] -= D[i][c] * D[j][c];
    }
    __syncthreads();
  }
  for (int e = t; e < b * b; e += 256) {
    const int i = e / b, j = e % b;
    A[(size_t)(k0 + i) * n + k0 + j] = j <= i ? D[i][j] : 0.0;
  }
}

// rows below the diagonal block: x L_kk^T = a by forward substitution, one
// row per lane; the mirrored strict-upper entries are zeroed
__global__ void __launch_bounds__(64) k_chol_panel(double *__restrict__ A0,
                                                   double *__restrict__ A1, int n, int k0) {
  __shared__ double L[kCb][kCb + 1];
  double *__restrict__ A = blockIdx.y == 0 ? A0 : A1;
  const int b = min(kCb, n - k0), t = threadIdx.x;
  for (int e = t; e < b * b; e += 64) L[e / b][e % b] = A[(size_t)(k0 + e / b) * n + k0 + e % b];
  __syncthreads();
  const int row = k0 + b + blockIdx.x * 64 + t;
  if (row >= n) return;
  double *__restrict__ ar = A + (size_t)row * n + k0;
  double x[kCb];
#pragma unroll
  for (int j = 0; j < kCb; ++j) x[j] = j < b ? ar[j] : 0.0;
#pragma unroll
  for (int j = 0; j < kCb; ++j) {
    if (j < b) {
      double sum = x[j];
#pragma unroll
      for (int q = 0; q < j; ++q) sum -= x[q] * L[j][q];
      x[j] = sum / L[j][j];
    }
  }
#pragma unroll
  for (int j = 0; j < kCb; ++j)
    if (j < b) {
      ar[j] = x[j];
      A[(size_t)(k0 + j) * n + row] = 0.0;
    }
}

// trailing tile (I, J), I >= J >= kb1 (tile index blockIdx.x in row order):
// C_IJ -= A_Ik A_Jk^T over the kCb columns of block step k0; four waves, one
// 16 x 16 quarter each; on a diagonal tile only the lower triangle
__global__ void __launch_bounds__(256) k_chol_update(double *__restrict__ A0,
                                                     double *__restrict__ A1, int n, int k0,
                                                     int kb1) {
  __shared__ double LA[kCb][kCb + 1], LB[kCb][kCb + 1];
  double *__restrict__ A = blockIdx.y == 0 ? A0 : A1;
  int I = 0;
  const int tix = blockIdx.x;
  while ((I + 1) * (I + 2) / 2 <= tix) ++I;
  const int J = tix - I * (I + 1) / 2 + kb1;
  I += kb1;
  const int b = min(kCb, n - k0), r0 = I * kCb, c0 = J * kCb;
  for (int e = threadIdx.x; e < kCb * kCb; e += 256) {
    const int i = e / kCb, k = e % kCb;
    LA[i][k] = r0 + i < n && k < b ? A[(size_t)(r0 + i) * n + k0 + k] : 0.0;
    LB[i][k] = c0 + i < n && k < b ? A[(size_t)(c0 + i) * n + k0 + k] : 0.0;
  }
  __syncthreads();
  const int wv = threadIdx.x / kWave, ln = threadIdx.x % kWave, si = wv >> 1, sj = wv & 1;
  svd_d4 acc = {0.0, 0.0, 0.0, 0.0};
  acc = mfma_tile(
      0, kCb / 4, [&](int i, int k) { return LA[16 * si + i][k]; },
      [&](int k, int j) { return LB[16 * sj + j][k]; }, acc);
  for (int r = 0; r < 4; ++r) {
    const int i = r0 + 16 * si + ln / 16 + 4 * r, j = c0 + 16 * sj + ln % 16;
    if (i < n && j <= i) A[(size_t)i * n + j] -= acc[r];
  }
}

static void cholesky_blocked(double *A0, double *A1, int n, int *flag, hipStream_t s) {
  const int nmat = A1 ? 2 : 1, nbk = ceil_div(n, kCb);
  for (int kb = 0; kb < nbk; ++kb) {
    const int k0 = kb * kCb, below = n - std::min(n, k0 + kCb);
    k_chol_diag<<<nmat, 256, 0, s>>>(A0, A1, n, k0, flag);
    LAUNCHCHK();
    if (below <= 0) continue;
    k_chol_panel<<<dim3(ceil_div(below, 64), nmat), 64, 0, s>>>(A0, A1, n, k0);
    LAUNCHCHK();
    const int m = nbk - kb - 1;
    k_chol_update<<<dim3(m * (m + 1) / 2, nmat), 256, 0, s>>>(A0, A1, n, k0, kb + 1);
    LAUNCHCHK();
  }
}

// One round of the block one-sided Jacobi sweep `sweep`: workgroup pm treats
// block pair pm % (nbp / 2) of the round-robin round `round` of W (pm <
// nbp / 2) or of W2. W and J column-major n x n; nbp = number of column
// blocks rounded up to even (columns >= n are zero and never written).
// ctrl[s] counts the rotations of sweep s; ctrl[kSvdMaxSweeps + 1] != 0 once
// a sweep has found nothing to rotate, which turns the remaining launches
// into no-ops. grid = nmat * nbp / 2; blockDim.x = 64 BS (BS = 8 or 16
// columns per block); dynamic LDS = block_jacobi_lds(). NP rows of J per
// thread are fetched into registers when the workgroup starts, so their
// latency overlaps the load, Gram matrix and rotations of W (NP * 32 >= n
// fetches J whole).
template <int BS, int NP>
__global__ void __launch_bounds__(64 * BS)
    k_block_jacobi_round(double *__restrict__ W, double *__restrict__ J, double *__restrict__ W2,
                         double *__restrict__ J2, int n, int nbp, int *__restrict__ ctrl,
                         int sweep, int round) {
  if (ctrl[kSvdMaxSweeps + 1]) return;
  constexpr int bs = BS, cols = 2 * BS, cc = cols * cols, nt = 64 * BS, nw = nt / kWave;
  constexpr int ct = cols / 16;        // 16-column tiles per block pair
  constexpr int nsl = nw / (ct * ct);  // K-slices of the Gram product
  extern __shared__ double lds[];
  const int wv = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  double *Ws = lds;                // column c at Ws + c * n
  double *Ga = Ws + (size_t)cols * n, *Ra = Ga + cc;  // G and R, row-major cols x cols
  double *part = Ra + cc;                              // nw 16 x 16 partial tiles of G
  double *rc = part + (size_t)nw * 256, *rs = rc + bs;  // rotation of each pair
  __shared__ int nrot, need;
  const int pm = blockIdx.x;
  // pair pr of matrix pm / (nbp / 2): (W, J) or (W2, J2)
  const int pr = pm % (nbp / 2);
  double *__restrict__ Wm = pm < nbp / 2 ? W : W2;
  double *__restrict__ Jm = pm < nbp / 2 ? J : J2;
  const int ba = rr_index(pr, round, nbp), bb = rr_index(nbp - 1 - pr, round, nbp);
  // local column c -> global column
  auto gcol = [&](int c) { return c < bs ? ba * bs + c : bb * bs + (c - bs); };
  // 32 threads per column (blockDim.x = 32 cols)
  const int lc = threadIdx.x / 32, li = threadIdx.x % 32, lg = gcol(lc);
  const double *jsrc = Jm + (size_t)lg * n;
  // J fetched at the start. With 8-column blocks straight into the MFMA
  // operand layout of the J product (tile p of this wave, row tile
  // it = wv + 8 p: lane ln holds J[16 it + ln % 16][column 4 kk + ln / 16]),
  // so that product reads registers, not LDS; with 16-column blocks NP rows
  // of one column per thread, staged through LDS for the product.
  double jr[NP];
  if constexpr (BS == 8) {
    static_assert(NP == 36, "9 row tiles of 4 k-steps per lane");
    const int wv0 = threadIdx.x / kWave, l0 = threadIdx.x % kWave;
#pragma unroll
    for (int pt = 0; pt < 9; ++pt)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int row = 16 * (wv0 + 8 * pt) + l0 % 16, g = gcol(4 * kk + l0 / 16);
        jr[4 * pt + kk] = row < n && g < n ? Jm[(size_t)g * n + row] : 0.0;
      }
  } else {
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int i = li + 32 * j;
      jr[j] = lg < n && i < n ? jsrc[i] : 0.0;
    }
  }
  {
    // W's columns in chunks of NP rows per thread, every load of a chunk in
    // flight before its LDS stores (one memory latency per chunk; n <= 32 NP
    // is a single chunk)
    double *dst = Ws + (size_t)lc * n;
    const double *src = Wm + (size_t)lg * n;
    for (int i0 = li; i0 < n; i0 += 32 * NP) {
      double w[NP];
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        const int i = i0 + 32 * j;
        w[j] = lg < n && i < n ? src[i] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < NP; ++j)
        if (i0 + 32 * j < n) dst[i0 + 32 * j] = w[j];
    }
  }
  if (threadIdx.x == 0) {
    nrot = 0;
    need = 0;
  }
  __syncthreads();
  // Gram matrix: wave wv forms tile (wv % (ct ct)) over K-slice
  // wv / (ct ct); the slices are added in order below. A diagonal tile
  // (one 16-column tile per pair when bs = 8) multiplies a matrix by its own
  // transpose, so one LDS load feeds both operands; four accumulators over
  // interleaved K steps keep four MFMA chains in flight.
  {
    const int tile = wv % (ct * ct), sl = wv / (ct * ct);
    const int ta = tile / ct, tb = tile % ct, ks = (n + 3) / 4;
    const int k0 = sl * ks / nsl, k1 = (sl + 1) * ks / nsl;
    svd_d4 acc = {0.0, 0.0, 0.0, 0.0};
    if (ta == tb) {
      const double *cw = Ws + (size_t)(16 * ta + ln % 16) * n + ln / 16;
      svd_d4 a1 = acc, a2 = acc, a3 = acc;
      int kk = k0;
      for (; kk + 3 < k1; kk += 4) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = 4 * (kk + u) + ln / 16;
          v[u] = k < n ? cw[4 * (kk + u)] : 0.0;
        }
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v[0], v[0], acc, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(v[1], v[1], a1, 0, 0, 0);
        a2 = __builtin_amdgcn_mfma_f64_16x16x4f64(v[2], v[2], a2, 0, 0, 0);
        a3 = __builtin_amdgcn_mfma_f64_16x16x4f64(v[3], v[3], a3, 0, 0, 0);
      }
      for (; kk < k1; ++kk) {
        const int k = 4 * kk + ln / 16;
        const double v = k < n ? cw[4 * kk] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc, 0, 0, 0);
      }
      acc = (acc + a1) + (a2 + a3);
    } else {
      acc = mfma_tile(
          k0, k1, [&](int i, int k) { return k < n ? Ws[(size_t)(16 * ta + i) * n + k] : 0.0; },
          [&](int k, int j) { return k < n ? Ws[(size_t)(16 * tb + j) * n + k] : 0.0; }, acc);
    }
    for (int r = 0; r < 4; ++r) part[(size_t)wv * 256 + (ln / 16 + 4 * r) * 16 + ln % 16] = acc[r];
  }
  __syncthreads();
  // G[a][b] from the upper-triangle tiles only, so G is exactly
  // symmetric; R = I; does any pair this visit rotates need it?
  for (int e = threadIdx.x; e < cc; e += nt) {
    int a = e / cols, b = e % cols;
    if (a > b) {
      const int x = a;
      a = b;
      b = x;
    }
    const int tile = (a / 16) * ct + b / 16, off = (a % 16) * 16 + b % 16;
    double g = 0.0;
    for (int sl = 0; sl < nsl; ++sl) g += part[(size_t)(sl * ct * ct + tile) * 256 + off];
    Ga[e] = g;
    Ra[e] = (e / cols) == (e % cols);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < cc; e += nt) {
    const int a = e / cols, b = e % cols;
    if (a < b && (round == 0 || (a < bs && b >= bs)) &&
        svd_needs_rotation(Ga[a * cols + a], Ga[b * cols + b], Ga[e]))
      need = 1;
  }
  __syncthreads();
  // Inner rounds: the rotation of each of the bs pairs (lane k: pair k) from
  // G; then the 2 x 2 block of G at rows of pair k1 and columns of pair k2
  // becomes that of J^T G J, and the two entries of row r of R at pair k2
  // those of R J. The blocks are disjoint, so both updates are in place.
  if (need) {
    const bool all0 = round == 0;
    const int ninner = all0 ? cols - 1 : bs;
    if constexpr (BS == 8) {
      // 8-column blocks: one wave runs every inner round (64 block updates of
      // G and 128 entries of R per round, the rotations passed by shuffles),
      // so a round costs no workgroup barrier
      if (wv == 0) {
        int count = 0;
        for (int ir = 0; ir < ninner; ++ir) {
          double c = 1.0, sn = 0.0;
          bool did = false;
          if (ln < bs) {
            int p, q;
            svd_pair(ln, ir, bs, all0, p, q);
            did = svd_rotation(Ga[p * cols + p], Ga[q * cols + q], Ga[p * cols + q], c, sn);
          }
          count += __popcll(__ballot(did));
          {
            const int k1 = ln >> 3, k2 = ln & 7;
            int p1, q1, p2, q2;
            svd_pair(k1, ir, bs, all0, p1, q1);
            svd_pair(k2, ir, bs, all0, p2, q2);
            const double c1 = __shfl(c, k1), s1 = __shfl(sn, k1);
            const double c2 = __shfl(c, k2), s2 = __shfl(sn, k2);
            double *g1 = Ga + p1 * cols, *g2 = Ga + q1 * cols;
            const double gpp = g1[p2], gpq = g1[q2], gqp = g2[p2], gqq = g2[q2];
            const double hpp = c1 * gpp - s1 * gqp, hpq = c1 * gpq - s1 * gqq;
            const double hqp = s1 * gpp + c1 * gqp, hqq = s1 * gpq + c1 * gqq;
            g1[p2] = c2 * hpp - s2 * hpq;
            g1[q2] = s2 * hpp + c2 * hpq;
            g2[p2] = c2 * hqp - s2 * hqq;
            g2[q2] = s2 * hqp + c2 * hqq;
          }
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const int e2 = ln + 64 * hh, r = e2 >> 3, k2 = e2 & 7;
            int p2, q2;
            svd_pair(k2, ir, bs, all0, p2, q2);
            const double c2 = __shfl(c, k2), s2 = __shfl(sn, k2);
            double *rr = Ra + r * cols;
            const double x = rr[p2], y = rr[q2];
            rr[p2] = c2 * x - s2 * y;
            rr[q2] = s2 * x + c2 * y;
          }
          wave_lds_sync();
        }
        if (ln == 0) nrot = count;
      }
      __syncthreads();
    } else {
      for (int ir = 0; ir < ninner; ++ir) {
        if (wv == 0) {
          bool did = false;
          if (ln < bs) {
            int p, q;
            svd_pair(ln, ir, bs, all0, p, q);
            double c, sn;
            did = svd_rotation(Ga[p * cols + p], Ga[q * cols + q], Ga[p * cols + q], c, sn);
            rc[ln] = c;
            rs[ln] = sn;
          }
          const unsigned long long m = __ballot(did);
          if (ln == 0) nrot += __popcll(m);
        }
        __syncthreads();
        const int e = threadIdx.x;
        if (e < bs * bs) {
          const int k1 = e / bs, k2 = e % bs;
          int p1, q1, p2, q2;
          svd_pair(k1, ir, bs, all0, p1, q1);
          svd_pair(k2, ir, bs, all0, p2, q2);
          const double c1 = rc[k1], s1 = rs[k1], c2 = rc[k2], s2 = rs[k2];
          double *g1 = Ga + p1 * cols, *g2 = Ga + q1 * cols;
          const double gpp = g1[p2], gpq = g1[q2], gqp = g2[p2], gqq = g2[q2];
          const double hpp = c1 * gpp - s1 * gqp, hpq = c1 * gpq - s1 * gqq;
          const double hqp = s1 * gpp + c1 * gqp, hqq = s1 * gpq + c1 * gqq;
          g1[p2] = c2 * hpp - s2 * hpq;
          g1[q2] = s2 * hpp + c2 * hpq;
          g2[p2] = c2 * hqp - s2 * hqq;
          g2[q2] = s2 * hqp + c2 * hqq;
        } else if (e < bs * bs + cols * bs) {
          const int r = (e - bs * bs) / bs, k2 = (e - bs * bs) % bs;
          int p2, q2;
          svd_pair(k2, ir, bs, all0, p2, q2);
          const double c2 = rc[k2], s2 = rs[k2];
          double *rr = Ra + r * cols;
          const double x = rr[p2], y = rr[q2];
          rr[p2] = c2 * x - s2 * y;
          rr[q2] = s2 * x + c2 * y;
        }
        __syncthreads();
      }
    }
  }
  const double *R = Ra;
  if (nrot > 0) {
    // X[:, pair] <- X[:, pair] R for X = W (from Ws), then X = J (from the
    // registers fetched at the start: as MFMA operands with 8-column blocks,
    // else staged through Ws, the rows past NP * 32 from memory).
    // Each tile is formed transposed, (R^T X^T) for 16 pair columns x 16
    // rows: the FP64 MFMA leaves entry (l / 16 + 4 r, l % 16) of its output
    // tile in lane l, register r, so lane l holds row 16 it + l % 16 and a
    // store instruction writes 16 consecutive rows of each of 4 columns (X
    // is column-major); two tiles per step, round-robin over the waves
    const int rt = (n + 15) / 16, ntl = rt * ct;
    for (int pass = 0; pass < 2; ++pass) {
      double *__restrict__ Xm = pass == 0 ? Wm : Jm;
      if (BS == 8 && pass == 1) {
        // J from the registers: tiles wv + 8 p, p = 0 .. 8 (n <= 1152)
#pragma unroll
        for (int pt = 0; pt < 9; ++pt) {
          const int it = wv + 8 * pt;
          if (it >= rt) break;
          svd_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int k = 4 * kk + ln / 16;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(R[k * cols + ln % 16], jr[4 * pt + kk], acc,
                                                       0, 0, 0);
          }
          const int i = 16 * it + ln % 16;
          for (int r = 0; r < 4; ++r) {
            const int g = gcol(ln / 16 + 4 * r);
            if (i < n && g < n) Jm[(size_t)g * n + i] = acc[r];
          }
        }
        continue;
      }
      if (pass == 1) {
        double *dst = Ws + (size_t)lc * n;
#pragma unroll
        for (int j = 0; j < NP; ++j)
          if (li + 32 * j < n) dst[li + 32 * j] = jr[j];
        for (int i = li + 32 * NP; i < n; i += 32) dst[i] = lg < n ? jsrc[i] : 0.0;
        __syncthreads();
      }
      auto tile_ops = [&](int tl, int kk, double &a, double &b) {
        const int it = tl / ct, cj = tl % ct, k = 4 * kk + ln / 16;
        a = R[k * cols + 16 * cj + ln % 16];                      // (R^T)[j][k]
        b = Ws[(size_t)k * n + min(16 * it + ln % 16, n - 1)];    // (X^T)[k][i]
      };
      auto tile_store = [&](int tl, const svd_d4 &acc) {
        const int it = tl / ct, cj = tl % ct, i = 16 * it + ln % 16;
        for (int r = 0; r < 4; ++r) {
          const int g = gcol(16 * cj + ln / 16 + 4 * r);
          if (i < n && g < n) Xm[(size_t)g * n + i] = acc[r];
        }
      };
      for (int tl = wv; tl < ntl; tl += 2 * nw) {
        const int t2 = tl + nw;
        svd_d4 a0 = {0.0, 0.0, 0.0, 0.0}, a1 = a0;
#pragma unroll
        for (int kk = 0; kk < cols / 4; ++kk) {
          double x0, y0, x1 = 0.0, y1 = 0.0;
          tile_ops(tl, kk, x0, y0);
          if (t2 < ntl) tile_ops(t2, kk, x1, y1);
          a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, a0, 0, 0, 0);
          a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, a1, 0, 0, 0);
        }
        tile_store(tl, a0);
        if (t2 < ntl) tile_store(t2, a1);
      }
      // the J pass of 16-column blocks overwrites Ws; that of 8-column
      // blocks reads only registers and R, so no wave waits for the others
      if (BS != 8) __syncthreads();
    }
    if (threadIdx.x == 0) {
      atomicAdd(&ctrl[sweep], nrot);
      atomicAdd(&ctrl[kSvdMaxSweeps + 2], 1);  // blocks that rotated (written back)
    }
  }
}

// After the last round of sweep `sweep`: a sweep without a rotation ends the
// iteration, and ctrl[kSvdMaxSweeps] records its index (it stays
// kSvdMaxSweeps if no sweep converges).
__global__ void k_block_jacobi_sweep_end(int *__restrict__ ctrl, int sweep) {
  if (threadIdx.x == 0 && ctrl[kSvdMaxSweeps + 1] == 0 && ctrl[sweep] == 0) {
    ctrl[kSvdMaxSweeps + 1] = 1;
    ctrl[kSvdMaxSweeps] = sweep;
  }
}

__global__ void k_block_jacobi_init(int *__restrict__ ctrl) {
  const int i = threadIdx.x;
  if (i < kSvdMaxSweeps + 3) ctrl[i] = i == kSvdMaxSweeps ? kSvdMaxSweeps : 0;
}

__global__ void k_identity_dense(double *__restrict__ J, int n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  J[e] = (e / n) == (e % n) ? 1.0 : 0.0;
}

// Ws (2 bs columns), G, R, one 16 x 16 partial tile per wave, and the
// rotation (c, s) of each of the bs pairs of an inner round
static size_t block_jacobi_lds(int n, int bs) {
  const size_t cols = 2 * (size_t)bs;
  return sizeof(double) * (cols * n + 2 * cols * cols + (size_t)bs * 256 + 2 * (size_t)bs);
}

int jacobi_svd(Pool &pool, double *W, double *J, int n, hipStream_t s) {
  return jacobi_svd2(pool, W, J, nullptr, nullptr, n, s);
}

// The SVDs of W (and of W2 when given) by rounds of the block Jacobi sweep,
// one launch per round: kernel boundaries order the rounds, so no grid
// barrier and no co-residency of the workgroups is needed, and several
// setups on concurrent streams do not wait on each other. The two matrices
// share the launches and stop after the first sweep in which neither
// rotates. Sweeps are enqueued in groups and the convergence flag is read
// back after each group; launches behind the converged sweep return at once.
int jacobi_svd2(Pool &pool, double *W, double *J, double *W2, double *J2, int n, hipStream_t s,
                bamg_handle *prof, void (*after_first)(void *), void *ctx) {
  int dev = 0, maxlds = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  // Column blocks of 16 where they fit in LDS (n <= 446 on 160 KB), else of
  // 8 (n <= 1117): with the rotations made on the Gram matrix a wider block
  // costs little more per round and halves the rounds (n = 289, tandem
  // 1025^2 setup: 10.4 ms for both SVDs with 16, 10.5 with 8, before the
  // later tuning).
  int bs = 16;
  if (block_jacobi_lds(n, bs) + 256 > (size_t)maxlds) bs = 8;
  if (block_jacobi_lds(n, bs) + 256 > (size_t)maxlds)
    fail(BAMG_E_ARG, "coarsest level too large for the LDS-staged Jacobi SVD");
  const size_t shm = block_jacobi_lds(n, bs);
  const int threads = kWave * bs;
  const int nb = ceil_div(n, bs);
  int nbp = nb + (nb & 1);
  if (nbp < 2) nbp = 2;
  int *ctrl = pool.get<int>(kSvdMaxSweeps + 3);
  k_block_jacobi_init<<<1, 128, 0, s>>>(ctrl);
  LAUNCHCHK();
  const int nmat = W2 ? 2 : 1;
  k_identity_dense<<<ceil_div((long)n * n, 256), 256, 0, s>>>(J, n);  // J = I
  LAUNCHCHK();
  if (W2) {
    k_identity_dense<<<ceil_div((long)n * n, 256), 256, 0, s>>>(J2, n);
    LAUNCHCHK();
  }
  // J fetched at the start: 12 rows per thread with 16-column blocks (n <=
  // 384 whole), 36 with 8-column blocks (n <= 1152 whole)
  const void *kern = bs == 16 ? (const void *)k_block_jacobi_round<16, 12>
                              : (const void *)k_block_jacobi_round<8, 36>;
  HIPCHK(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  const int grid = nmat * (nbp / 2);
  int *hp = pool.pinned();
  // about 12 sweeps converge a coarsest level of a few hundred states: the
  // first check comes after 8, later ones after every 2
  int sweep = 0, done = 0;
  while (!done && sweep < kSvdMaxSweeps) {
    const int upto = std::min(kSvdMaxSweeps, sweep == 0 ? 8 : sweep + 2);
    if (prof) profile_mark(prof, s, true);
    for (; sweep < upto; ++sweep) {
      for (int round = 0; round < nbp - 1; ++round) {
        if (bs == 16)
          k_block_jacobi_round<16, 12>
              <<<grid, threads, shm, s>>>(W, J, W2, J2, n, nbp, ctrl, sweep, round);
        else
          k_block_jacobi_round<8, 36>
              <<<grid, threads, shm, s>>>(W, J, W2, J2, n, nbp, ctrl, sweep, round);
        LAUNCHCHK();
      }
      k_block_jacobi_sweep_end<<<1, 64, 0, s>>>(ctrl, sweep);
      LAUNCHCHK();
    }
    if (prof) profile_mark(prof, s, false);
    if (after_first) {
      after_first(ctx);
      after_first = nullptr;
    }
    HIPCHK(hipMemcpyAsync(hp, ctrl + kSvdMaxSweeps, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    done = hp[1];
  }
  const int sweeps = hp[0];
  if (prof) {
    // launches that did work: the sweeps up to the one that found nothing
    // to rotate; each block reads its W and J columns, a rotating block
    // writes both back
    const double colbytes = 2.0 * bs * n * sizeof(double);
    const long active = (long)std::min(sweeps + 1, sweep) * (nbp - 1);
    prof->prof_launches += active;
    prof->prof_bytes += (double)active * grid * 2.0 * colbytes + (double)hp[2] * 2.0 * colbytes;
  }
  pool.release(ctrl);
  return done && sweeps < kSvdMaxSweeps ? BAMG_OK : BAMG_E_COARSE;
}

__global__ void k_column_norms(const double *__restrict__ W, int n, double *__restrict__ sv) {
  __shared__ double sh[4];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double x = W[(size_t)k * n + i];
    s += x * x;
  }
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) sv[k] = sqrt(s);
}

void column_norms(const double *W, int n, double *sv, hipStream_t s) {
  k_column_norms<<<n, 256, 0, s>>>(W, n, sv);
  LAUNCHCHK();
}

// The r smallest singular values in ascending order (ties: lower index).
// Thread per value: its rank among all n is the count of smaller values
// plus equal ones at lower index; ranks below r give the order.
__global__ void k_select_smallest(const double *__restrict__ sv, int n, int r,
                                  int *__restrict__ order) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double v = sv[k];
  int rank = 0;
  for (int j = 0; j < n; ++j) {
    const double u = sv[j];
    rank += (u < v || (u == v && j < k)) ? 1 : 0;
  }
  if (rank < r) order[rank] = k;
}

// One block per requested triplet t: x = L^-T (column of W / sigma or of J),
// solved column-wise in LDS, then the pair sign fixed by sum(v) >= 0.
template <class T>
__global__ void __launch_bounds__(256)
    k_triplets(const double *__restrict__ LM, const double *__restrict__ LN,
               const double *__restrict__ W, const double *__restrict__ J,
               const double *__restrict__ sv, const int *__restrict__ order, int n, int r,
               T *__restrict__ U, T *__restrict__ V, double *__restrict__ sigma) {
  extern __shared__ double xs[];  // 2n doubles: u then v
  __shared__ double sh[4];
  const int t = blockIdx.x;
  const int k = order[t];
  const double sk = sv[k];
  double *xu = xs, *xv = xs + n;
  for (int i = threadIdx.x; i < n; i += 256) {
    xu[i] = sk > 0.0 ? W[(size_t)k * n + i] / sk : 0.0;
    xv[i] = J[(size_t)k * n + i];
  }
  __syncthreads();
  for (int i = n - 1; i >= 0; --i) {
    if (threadIdx.x == 0) {
      xu[i] /= LM[(size_t)i * n + i];
      xv[i] /= LN[(size_t)i * n + i];
    }
    __syncthreads();
    const double ui = xu[i], vi = xv[i];
    for (int q = threadIdx.x; q < i; q += 256) {
      xu[q] -= LM[(size_t)i * n + q] * ui;
      xv[q] -= LN[(size_t)i * n + q] * vi;
    }
    __syncthreads();
  }
  double sv_sum = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) sv_sum += xv[i];
  sv_sum = block_sum<256>(sv_sum, sh);
  __shared__ double sg;
  if (threadIdx.x == 0) {
    sg = sv_sum < 0.0 ? -1.0 : 1.0;
    sigma[t] = sk;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 256) {
    V[(size_t)i * r + t] = (T)(sg * xv[i]);
    U[(size_t)i * r + t] = t == 0 ? (T)1 : (T)(sg * xu[i]);
  }
}

void coarse_triplets_out(const double *LM, const double *LN, const double *W, const double *J,
                         const double *sv, int n, int r, void *U, void *V, int prec,
                         double *sigma, double *work, hipStream_t s) {
  int *order = reinterpret_cast<int *>(work);
  k_select_smallest<<<ceil_div(n, 256), 256, 0, s>>>(sv, n, r, order);
  LAUNCHCHK();
  const size_t shm = sizeof(double) * 2 * (size_t)n;
  if (prec == 0)
    k_triplets<double><<<r, 256, shm, s>>>(LM, LN, W, J, sv, order, n, r, (double *)U,
                                           (double *)V, sigma);
  else
    k_triplets<float><<<r, 256, shm, s>>>(LM, LN, W, J, sv, order, n, r, (float *)U, (float *)V,
                                          sigma);
  LAUNCHCHK();
}

// is2[k] = 1 / sigma_k^2, 0 for the dropped (null) direction kmin
__global__ void k_inv_sq(const double *__restrict__ sv, int n, int kmin, double *__restrict__ is2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) is2[k] = k == kmin ? 0.0 : 1.0 / (sv[k] * sv[k]);
}

// Bdag = sum over kept k of J_k W_k^T / sigma_k^2 (W_k = sigma_k u_k), row-
// major: Bdag[i][j] = sum_k J[k n + i] (W[k n + j] is2[k]) on FP64 MFMA, a
// 64 x 64 output tile per workgroup, 32 x 32 (2 x 2 MFMA tiles) per wave,
// operands straight from memory (J's and W's columns are contiguous, so 16
// lanes read 128 consecutive bytes).
__global__ void __launch_bounds__(256) k_pinv(const double *__restrict__ W,
                                              const double *__restrict__ J,
                                              const double *__restrict__ is2, int n,
                                              double *__restrict__ bdag) {
  const int wv = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  const int i0 = blockIdx.y * 64 + (wv / 2) * 32, j0 = blockIdx.x * 64 + (wv % 2) * 32;
  svd_d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = svd_d4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < n; k0 += 4) {
    const int k = k0 + ln / 16;
    const bool kok = k < n;
    const double sc = kok ? is2[k] : 0.0;
    double a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int i = i0 + 16 * t + ln % 16, j = j0 + 16 * t + ln % 16;
      a[t] = kok && i < n ? J[(size_t)k * n + i] : 0.0;
      b[t] = kok && j < n ? W[(size_t)k * n + j] * sc : 0.0;
    }
#pragma unroll
    for (int ta = 0; ta < 2; ++ta)
#pragma unroll
      for (int tb = 0; tb < 2; ++tb)
        acc[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta], b[tb], acc[ta][tb], 0, 0, 0);
  }
  // lane ln, register r: row 16 ta + ln / 16 + 4 r, column 16 tb + ln % 16
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 16 * ta + ln / 16 + 4 * r, j = j0 + 16 * tb + ln % 16;
        if (i < n && j < n) bdag[(size_t)i * n + j] = acc[ta][tb][r];
      }
}

int build_pinv(Pool &pool, const double *W, const double *J, const double *sv, int n,
               double *bdag, hipStream_t s) {
  std::vector<double> h(n);
  HIPCHK(hipMemcpyAsync(h.data(), sv, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int kmin = 0;
  double smax = 0.0;
  for (int k = 0; k < n; ++k) {
    if (h[k] < h[kmin]) kmin = k;
    smax = h[k] > smax ? h[k] : smax;
  }
  double s2 = 1e300;
  for (int k = 0; k < n; ++k)
    if (k != kmin && h[k] < s2) s2 = h[k];
  if (!(h[kmin] <= 1e-10 * smax) || !(s2 > 1e-13 * smax)) return BAMG_E_COARSE;
  double *is2 = pool.get<double>(n);
  k_inv_sq<<<ceil_div(n, 256), 256, 0, s>>>(sv, n, kmin, is2);
  LAUNCHCHK();
  k_pinv<<<dim3(ceil_div(n, 64), ceil_div(n, 64)), 256, 0, s>>>(W, J, is2, n, bdag);
  LAUNCHCHK();
  pool.release(is2);
  return BAMG_OK;
}

}  // namespace bamg

namespace bamg {

// ------------------------------------------------ LDS-resident coarse solver
// One workgroup of 1024 threads solves the whole coarsest-level problem when
// n is small enough for two n x (n+1) FP64 arrays to live in LDS:
//   mode 0 (triplets): Cholesky of M and N (in place, global memory), then
//     C = Bt^T = L_N^-1 B^T L_M^-T in LDS (row k of C = column k of Bt),
//     one-sided Jacobi on the rows of C with the rotations accumulated in J^T
//     (LDS), the r smallest sigma, u = L_M^-T C_k / sigma_k and
//     v = L_N^-T J_k, sign fixed by sum(v) >= 0, u_0 = 1;
//   mode 1 (pseudo-inverse): the same SVD of B (M = N = I) and
//     Bdag = sum over k != argmin sigma of J_k (C_k)^T / sigma_k^2.
// Rows of C and J^T are contiguous, so a pair rotation is two contiguous row
// updates by one wave; the 16 waves take disjoint pairs of a round.
constexpr int kSmallThreads = 1024;

// order LDS accesses of one wave: compiler fence plus wave barrier
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double wave_sum_all(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// right-looking Cholesky in place (lower, row-major), by the whole workgroup
__device__ void chol_block(double *A, int n, int *flag) {
  __shared__ double piv;
  const int t = threadIdx.x;
  for (int j = 0; j < n; ++j) {
    if (t == 0) {
      const double d = A[j * n + j];
      if (!(d > 0.0)) atomicOr(flag, 1);
      piv = d > 0.0 ? sqrt(d) : 1.0;
      A[j * n + j] = piv;
    }
    __syncthreads();
    const double d = piv;
    for (int i = j + 1 + t; i < n; i += blockDim.x) A[i * n + j] /= d;
    __syncthreads();
    const int m = n - j - 1;
    for (int e = t; e < m * m; e += blockDim.x) {
      const int ii = e / m, kk = e % m;
      if (kk > ii) continue;
      const int i = j + 1 + ii, k = j + 1 + kk;
      A[i * n + k] -= A[i * n + j] * A[k * n + j];
    }
    __syncthreads();
  }
  for (int e = t; e < n * n; e += blockDim.x)
    if (e % n > e / n) A[e] = 0.0;
  __syncthreads();
}

template <class T>
__global__ void __launch_bounds__(kSmallThreads)
    k_coarse_small(int mode, int n, int r, const double *__restrict__ Bd, double *__restrict__ Md,
                   double *__restrict__ Nd, T *__restrict__ U, T *__restrict__ V,
                   double *__restrict__ sigma, double *__restrict__ bdag, int *__restrict__ flag,
                   int gram) {
  extern __shared__ double lds[];
  const int ld = n + 1;
  double *C = lds;                 // n x ld
  double *Jt = lds + n * ld;       // n x ld, row k = column k of J
  double *sv = Jt + n * ld;        // n
  __shared__ int order[16];
  __shared__ int rotated;
  __shared__ int kmin;
  const int t = threadIdx.x, w = t / kWave, lane = t % kWave, nw = kSmallThreads / kWave;
  // mode 2: both at once, workgroup 0 the triplets and workgroup 1 the
  // pseudo-inverse (they share only the read-only B)
  if (mode == 2) mode = (int)blockIdx.x;
  // Until J^T is set up its LDS rows hold one n x n factor at a time: each
  // Cholesky runs there (workgroup barriers, no global round trips), is
  // copied back for the final back-substitutions and used in place for its
  // triangular solve.
  double *S = Jt;
  auto factor = [&](double *A) {
    for (int e = t; e < n * n; e += blockDim.x) S[e] = A[e];
    __syncthreads();
    chol_block(S, n, flag);
    for (int e = t; e < n * n; e += blockDim.x) A[e] = S[e];
  };
  if (mode == 0) factor(Nd);
  // Y = L_N^-1 B^T (column j per thread), stored in C; B^T is copied into C
  // first by the whole workgroup
  for (int e = t; e < n * n; e += blockDim.x) C[(e % n) * ld + e / n] = Bd[e];
  __syncthreads();
  for (int j = t; j < n; j += blockDim.x) {
    for (int i = 0; i < n; ++i) {
      double s = C[i * ld + j];
      if (mode == 0) {
        for (int k = 0; k < i; ++k) s -= S[i * n + k] * C[k * ld + j];
        s /= S[i * n + i];
      }
      C[i * ld + j] = s;
    }
  }
  __syncthreads();
  // C = Y L_M^-T (row i per thread, in place)
  if (mode == 0) {
    factor(Md);
    for (int i = t; i < n; i += blockDim.x) {
      for (int k = 0; k < n; ++k) {
        double s = C[i * ld + k];
        for (int j = 0; j < k; ++j) s -= S[k * n + j] * C[i * ld + j];
        C[i * ld + k] = s / S[k * n + k];
      }
    }
    __syncthreads();
  }
  for (int e = t; e < n * ld; e += blockDim.x) Jt[e] = (e / ld == e % ld) ? 1.0 : 0.0;
  __syncthreads();
  // one-sided Jacobi on the rows of C, round-robin pairs; each pair is
  // handled by a group of kPairLanes lanes so a round's pairs run together
  constexpr int kPairLanes = 16;
  const int grp = t / kPairLanes, gl = t % kPairLanes, ngrp = kSmallThreads / kPairLanes;
  const int m = n + (n & 1);
  const double tol = 1e-15;
  if (gram) {
    // The same sweeps with the inner products taken from the Gram matrix
    // G = C Cᵀ, formed afresh at the start of each sweep (so a sweep that
    // rotates nothing has tested fresh inner products). Per round, lane k of
    // wave 0 finds pair k's rotation from G; then the rows of C and Jᵀ are
    // rotated and G's 2 x 2 blocks rewritten to Jᵀ G J, in place.
    const int gld = m + 1, np = m / 2;
    double *G = sv + n;                 // m x gld
    double *rc = G + (size_t)m * gld;   // per pair: c, s
    double *rs = rc + np;
    int *pp = reinterpret_cast<int *>(rs + np), *qq = pp + np;
    // this thread's tasks, the same every round (at most kTasks of each kind)
    constexpr int kTasks = 4;
    int rk[kTasks], ri[kTasks], g1k[kTasks], g2k[kTasks];
#pragma unroll
    for (int u = 0; u < kTasks; ++u) {
      const int e = t + u * (int)blockDim.x;
      rk[u] = e < np * n ? e / n : -1;
      ri[u] = e < np * n ? e % n : 0;
      g1k[u] = e < np * np ? e / np : -1;
      g2k[u] = e < np * np ? e % np : 0;
    }
    for (int sweep = 0; sweep < 80; ++sweep) {
      if (t == 0) rotated = 0;
      for (int e = t; e < m * m; e += blockDim.x) {
        const int a = e / m, b = e % m;
        if (a > b) continue;
        double g = 0.0;
        if (b < n)
          for (int i = 0; i < n; ++i) g += C[a * ld + i] * C[b * ld + i];
        G[a * gld + b] = g;
        G[b * gld + a] = g;
      }
      __syncthreads();
      for (int round = 0; round < m - 1; ++round) {
        if (w == 0 && lane < np) {
          // round-robin positions lane and m - 1 - lane, remainders mod m - 1
          // by one conditional subtraction
          int p = 0, q = m - 1 - lane + round - 1;
          if (lane != 0) {
            p = lane - 1 + round;
            if (p >= m - 1) p -= m - 1;
            ++p;
          }
          if (q >= m - 1) q -= m - 1;
          ++q;
          if (p > q) {
            const int x = p;
            p = q;
            q = x;
          }
          double c = 1.0, sn = 0.0;
          const double al = G[p * gld + p], be = G[q * gld + q], ga = G[p * gld + q];
          if (q < n && ga != 0.0 && ga * ga > tol * tol * (al * be)) {
            // tan of the smaller rotation angle, with one division
            const double d = be - al;
            const double tt = (d >= 0 ? 2.0 : -2.0) * ga / (fabs(d) + sqrt(d * d + 4.0 * ga * ga));
            c = rsqrt(1.0 + tt * tt);
            sn = c * tt;
            rotated = 1;
          }
          rc[lane] = c;
          rs[lane] = sn;
          pp[lane] = p;
          qq[lane] = q;
        }
        __syncthreads();
        // rows of C and Jᵀ: task (k, i), i < n
#pragma unroll
        for (int u = 0; u < kTasks; ++u) {
          const int k = rk[u], i = ri[u];
          if (k < 0) continue;
          const int p = pp[k], q = qq[k];
          const double c = rc[k], sn = rs[k];
          if (sn == 0.0) continue;
          const double a = C[p * ld + i], b = C[q * ld + i];
          C[p * ld + i] = c * a - sn * b;
          C[q * ld + i] = sn * a + c * b;
          const double x = Jt[p * ld + i], y = Jt[q * ld + i];
          Jt[p * ld + i] = c * x - sn * y;
          Jt[q * ld + i] = sn * x + c * y;
        }
        // G: the 2 x 2 block of pairs (k1, k2)
#pragma unroll
        for (int u = 0; u < kTasks; ++u) {
          const int k1 = g1k[u], k2 = g2k[u];
          if (k1 < 0) continue;
          const int p1 = pp[k1], q1 = qq[k1], p2 = pp[k2], q2 = qq[k2];
          const double c1 = rc[k1], s1 = rs[k1], c2 = rc[k2], s2 = rs[k2];
          double *g1 = G + p1 * gld, *g2 = G + q1 * gld;
          const double gpp = g1[p2], gpq = g1[q2], gqp = g2[p2], gqq = g2[q2];
          const double hpp = c1 * gpp - s1 * gqp, hpq = c1 * gpq - s1 * gqq;
          const double hqp = s1 * gpp + c1 * gqp, hqq = s1 * gpq + c1 * gqq;
          g1[p2] = c2 * hpp - s2 * hpq;
          g1[q2] = s2 * hpp + c2 * hpq;
          g2[p2] = c2 * hqp - s2 * hqq;
          g2[q2] = s2 * hqp + c2 * hqq;
        }
        __syncthreads();
      }
      const int any = rotated;
      __syncthreads();
      if (!any) break;
      if (sweep == 79 && t == 0) atomicOr(flag, 2);
    }
  }
  for (int sweep = 0; sweep < 80 && !gram; ++sweep) {
    if (t == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < m - 1; ++round) {
      for (int pair = grp; pair < m / 2; pair += ngrp) {
        int p = rr_index(pair, round, m), q = rr_index(m - 1 - pair, round, m);
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        if (q >= n) continue;  // dummy column, uniform in the group
        double *cp = C + p * ld, *cq = C + q * ld;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = gl; i < n; i += kPairLanes) {
          const double a = cp[i], b = cq[i];
          al += a * a;
          be += b * b;
          ga += a * b;
        }
        group_sum3(al, be, ga, kPairLanes);
        if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
          double *jp = Jt + p * ld, *jq = Jt + q * ld;
          for (int i = gl; i < n; i += kPairLanes) {
            const double a = cp[i], b = cq[i];
            cp[i] = c * a - sn * b;
            cq[i] = sn * a + c * b;
            const double x = jp[i], y = jq[i];
            jp[i] = c * x - sn * y;
            jq[i] = sn * x + c * y;
          }
          if (gl == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
    if (sweep == 79 && t == 0) atomicOr(flag, 2);
  }
  // singular values
  for (int k = w; k < n; k += nw) {
    double s = 0.0;
    for (int i = lane; i < n; i += kWave) s += C[k * ld + i] * C[k * ld + i];
    s = wave_sum_all(s);
    if (lane == 0) sv[k] = sqrt(s);
  }
  __syncthreads();
  if (mode == 1) {
    if (t == 0) {
      int km = 0;
      double smax = 0.0;
      for (int k = 0; k < n; ++k) {
        if (sv[k] < sv[km]) km = k;
        smax = fmax(smax, sv[k]);
      }
      double s2 = 1e300;
      for (int k = 0; k < n; ++k)
        if (k != km) s2 = fmin(s2, sv[k]);
      if (!(sv[km] <= 1e-10 * smax) || !(s2 > 1e-13 * smax)) atomicOr(flag, 4);
      kmin = km;
    }
    __syncthreads();
    for (int e = t; e < n * n; e += blockDim.x) {
      const int i = e / n, j = e % n;
      double s = 0.0;
      for (int k = 0; k < n; ++k)
        if (k != kmin) s += Jt[k * ld + i] * C[k * ld + j] / (sv[k] * sv[k]);
      bdag[e] = s;
    }
    return;
  }
  // the r smallest singular values in ascending order, ties by index: the
  // value of rank q (strictly smaller ones, or equal ones of lower index).
  // Every slot first holds a valid row, in case non-finite values leave a
  // rank unassigned.
  if (t < r) order[t] = t < n ? t : n - 1;
  __syncthreads();
  for (int k = t; k < n; k += blockDim.x) {
    int rank = 0;
    for (int j = 0; j < n; ++j) rank += sv[j] < sv[k] || (sv[j] == sv[k] && j < k);
    if (rank < r) order[rank] = k;
  }
  __syncthreads();
  // back-substitutions: wave 2q solves L_M^T u = C_k / sigma_k, wave 2q+1
  // solves L_N^T v = J_k, in place in the LDS rows (k = order[q]); an entry
  // is written only by its owning lane (i mod 64)
  for (int task = w; task < 2 * r; task += nw) {
    const int q = task / 2, side = task % 2, k = order[q];
    double *x = side == 0 ? C + k * ld : Jt + k * ld;
    const double *L = side == 0 ? Md : Nd;
    if (side == 0) {
      const double s = sv[k];
      for (int i = lane; i < n; i += kWave) x[i] = s > 0.0 ? x[i] / s : 0.0;
    }
    wave_sync();
    for (int i = n - 1; i >= 0; --i) {
      const double xi = mode == 0 ? x[i] / L[i * n + i] : x[i];
      wave_sync();
      if (lane == i % kWave) x[i] = xi;
      for (int z = lane; z < i; z += kWave) x[z] -= L[i * n + z] * xi;
      wave_sync();
    }
  }
  __syncthreads();
  // sign of each pair from sum(v); write U, V (n x r row-major) and sigma
  for (int q = w; q < r; q += nw) {
    const int k = order[q];
    double s = 0.0;
    for (int i = lane; i < n; i += kWave) s += Jt[k * ld + i];
    s = wave_sum_all(s);
    const double sg = s < 0.0 ? -1.0 : 1.0;
    for (int i = lane; i < n; i += kWave) {
      V[(size_t)i * r + q] = (T)(sg * Jt[k * ld + i]);
      U[(size_t)i * r + q] = q == 0 ? (T)1 : (T)(sg * C[k * ld + i]);
    }
    if (lane == 0) sigma[q] = sv[k];
  }
}

size_t coarse_small_lds(int n) { return sizeof(double) * ((size_t)2 * n * (n + 1) + n); }
// with the Gram matrix (m = n rounded up to even, row stride m + 1), the
// rotations (c, s) and the pairs (p, q) of a round
static size_t coarse_small_gram_lds(int n) {
  const size_t m = n + (n & 1);
  return coarse_small_lds(n) + sizeof(double) * (m * (m + 1) + m) + sizeof(int) * m;
}

int coarse_small_max(void) {
  static const int nmax = [] {  // thread-safe one-time initialisation
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      lds = 65536;
    int n = 2;
    while (coarse_small_lds(n + 1) + 1024 <= (size_t)lds && n < 128) ++n;
    return n;
  }();
  return nmax;
}

int coarse_small(int mode, int n, int r, const double *Bd, double *Md, double *Nd, void *U,
                 void *V, int prec, double *sigma, double *bdag, int *flag, hipStream_t s) {
  int dev = 0, maxlds = 65536;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  // the Gram form where it fits in LDS and each thread has at most 4 row
  // tasks and 4 block tasks per round (n <= 80 on 160 KB of LDS)
  const int np = (n + (n & 1)) / 2;
  const int gram = coarse_small_gram_lds(n) + 1024 <= (size_t)maxlds &&
                           np * n <= 4 * kSmallThreads && np * np <= 4 * kSmallThreads
                       ? 1
                       : 0;
  const size_t shm = gram ? coarse_small_gram_lds(n) : coarse_small_lds(n);
  fill_i32(flag, 0, 1, s);
  if (prec == 0) {
    HIPCHK(hipFuncSetAttribute((const void *)k_coarse_small<double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    k_coarse_small<double><<<mode == 2 ? 2 : 1, kSmallThreads, shm, s>>>(
        mode, n, r, Bd, Md, Nd, (double *)U, (double *)V, sigma, bdag, flag, gram);
  } else {
    HIPCHK(hipFuncSetAttribute((const void *)k_coarse_small<float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    k_coarse_small<float><<<mode == 2 ? 2 : 1, kSmallThreads, shm, s>>>(
        mode, n, r, Bd, Md, Nd, (float *)U, (float *)V, sigma, bdag, flag, gram);
  }
  LAUNCHCHK();
  const int f = read_int(flag, s);
  if (f & 1) return BAMG_E_COARSE;
  if (f & 2) return BAMG_E_COARSE;
  if (f & 4) return BAMG_E_COARSE;
  return BAMG_OK;
}

}  // namespace bamg

namespace bamg {

// Section 5 makes the column sums of every B_l zero (1^T B_l = 0). A
// coarsest operator built in FP32 keeps them only to FP32 accuracy; in FP64
// the residue of each column is moved into its diagonal so the dense
// operator has the exact left null vector again.
__global__ void k_zero_colsums(double *__restrict__ D, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += D[(size_t)i * n + j];
  D[(size_t)j * n + j] -= s;
}

void zero_colsums(double *D, int n, hipStream_t s) {
  k_zero_colsums<<<ceil_div(n, 64), 64, 0, s>>>(D, n);
  LAUNCHCHK();
}

}  // namespace bamg
