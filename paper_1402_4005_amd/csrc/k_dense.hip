// Coarsest-level dense algebra (FP64 always):
//  * the r smallest generalized singular triplets of eq.
//    generalized_eigenvalue: B_L v = sigma M_L u, B_L^T u = sigma N_L v. With
//    Cholesky factors M = L_M L_M^T, N = L_N L_N^T this is the ordinary SVD of
//    Bt = L_M^-1 B_L L_N^-T; u = L_M^-T ut, v = L_N^-T vt.
//  * the Moore-Penrose pseudo-inverse of B_L used by the coarse-grid
//    correction (eq. coarse_grid_correction), from the SVD of B_L with the
//    one zero singular value (1^T B_L = 0, Section 5) dropped.
// The SVD is one-sided Jacobi (Hestenes): column pairs of W are rotated until
// orthogonal. Pairs follow the round-robin (circle) schedule, so one round
// rotates n/2 disjoint pairs in parallel, one workgroup per pair, with a
// grid-wide barrier between rounds (cooperative launch).
#include <hip/hip_cooperative_groups.h>

#include <mutex>

#include "bamg_internal.h"
#include "device_common.h"

namespace cg = cooperative_groups;

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
int cholesky2(double *A0, double *A1, int n, int *flag, hipStream_t s) {
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
// final, every later row subtracts L[i][k] times it.
__global__ void __launch_bounds__(1024) k_trsm_slab(const double *__restrict__ L,
                                                    double *__restrict__ X, int n, int ncols,
                                                    int ldx, int sw) {
  extern __shared__ double xs[];  // n x sw
  const int t = threadIdx.x, nt = blockDim.x;
  const int c = t % sw, ro = t / sw, nro = nt / sw;
  const int col = blockIdx.x * sw + c;
  for (int e = t; e < n * sw; e += nt) {
    const int i = e / sw, cc = e % sw, g = blockIdx.x * sw + cc;
    xs[e] = g < ncols ? X[(size_t)i * ldx + g] : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double xk = xs[k * sw + c] / L[(size_t)k * n + k];
    if (ro == 0 && col < ncols) X[(size_t)k * ldx + col] = xk;
    for (int i = k + 1 + ro; i < n; i += nro) xs[i * sw + c] -= L[(size_t)i * n + k] * xk;
    __syncthreads();
  }
}

void trsm_lower_cols(const double *L, double *X, int n, int ncols, int ldx, hipStream_t s) {
  int dev = 0, maxlds = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  int sw = 32;
  while (sw > 1 && sizeof(double) * (size_t)n * sw > (size_t)maxlds) sw >>= 1;
  const size_t shm = sizeof(double) * (size_t)n * sw;
  if (shm > (size_t)maxlds) fail(BAMG_E_ARG, "trsm: matrix too large for an LDS slab");
  HIPCHK(hipFuncSetAttribute((const void *)k_trsm_slab,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  k_trsm_slab<<<ceil_div(ncols, sw), 1024, shm, s>>>(L, X, n, ncols, ldx, sw);
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
// columns; the blocks are paired by the round-robin schedule, one workgroup
// per block pair. A workgroup holds its 2 bs columns in LDS and rotates
// their pairs (bs disjoint pairs at a time, one wave per pair): in the first
// round of a sweep all pairs of the 2 bs columns, afterwards only the pairs
// across the two blocks, so each column pair of W is visited once per
// sweep. The rotations accumulate in a 2bs x 2bs matrix R, and the matching
// columns of J are multiplied by R once. Only the block rounds need a
// grid-wide barrier: a sweep costs about n workgroup barriers and n/bs grid
// barriers.
constexpr int kSvdMaxSweeps = 80;

__device__ __forceinline__ int rr_index(int j, int round, int m) {
  return j == 0 ? 0 : 1 + (j - 1 + round) % (m - 1);
}

// W and J column-major n x n; nbp = number of column blocks rounded up to
// even (columns >= n are zero and never written). ctrl[s] counts rotations
// of sweep s; ctrl[kSvdMaxSweeps] receives the number of sweeps run.
// blockDim.x = 64 * bs; dynamic LDS = (2 bs n + 4 bs^2) doubles.
__global__ void __launch_bounds__(1024)
    k_block_jacobi_svd(double *__restrict__ W, double *__restrict__ J, double *__restrict__ W2,
                       double *__restrict__ J2, int nmat, int n, int bs, int nbp,
                       int *__restrict__ ctrl) {
  cg::grid_group grid = cg::this_grid();
  extern __shared__ double lds[];
  const int cols = 2 * bs;
  double *Ws = lds;                         // column c at Ws + c * n
  double *R = lds + (size_t)cols * n;       // cols x cols, column-major
  __shared__ int nrot;
  const int nt = blockDim.x;
  const int wv = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  const double tol = 1e-15;
  int sweep = 0;
  for (; sweep < kSvdMaxSweeps; ++sweep) {
    for (int round = 0; round < nbp - 1; ++round) {
      for (int pm = blockIdx.x; pm < nmat * (nbp / 2); pm += gridDim.x) {
        // pair pr of matrix pm / (nbp / 2): (W, J) or (W2, J2)
        const int pr = pm % (nbp / 2);
        double *__restrict__ Wm = pm < nbp / 2 ? W : W2;
        double *__restrict__ Jm = pm < nbp / 2 ? J : J2;
        const int ba = rr_index(pr, round, nbp), bb = rr_index(nbp - 1 - pr, round, nbp);
        // local column c -> global column
        auto gcol = [&](int c) { return c < bs ? ba * bs + c : bb * bs + (c - bs); };
        for (int e = threadIdx.x; e < cols * n; e += nt) {
          const int c = e / n, i = e % n, g = gcol(c);
          Ws[e] = g < n ? Wm[(size_t)g * n + i] : 0.0;
        }
        for (int e = threadIdx.x; e < cols * cols; e += nt) R[e] = (e / cols) == (e % cols);
        if (threadIdx.x == 0) nrot = 0;
        __syncthreads();
        // Round 0 of a sweep: every pair of the 2 bs columns (round-robin,
        // bs disjoint pairs at a time), which covers each block's own pairs
        // once per sweep. Later rounds: only the bs x bs cross pairs of the
        // two blocks, column wv of block a with column (wv + ir) mod bs of
        // block b. Every column pair of W is rotated once per sweep.
        const int ninner = round == 0 ? cols - 1 : bs;
        for (int ir = 0; ir < ninner; ++ir) {
          int p, q;
          if (round == 0) {
            p = rr_index(wv, ir, cols);
            q = rr_index(cols - 1 - wv, ir, cols);
            if (p > q) {
              const int x = p;
              p = q;
              q = x;
            }
          } else {
            p = wv;
            q = bs + (wv + ir) % bs;
          }
          double *wp = Ws + (size_t)p * n, *wq = Ws + (size_t)q * n;
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int i = ln; i < n; i += kWave) {
            const double x = wp[i], y = wq[i];
            al += x * x;
            be += y * y;
            ga += x * y;
          }
          group_sum3(al, be, ga, kWave);
          if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
            const double zeta = (be - al) / (2.0 * ga);
            const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
            for (int i = ln; i < n; i += kWave) {
              const double x = wp[i], y = wq[i];
              wp[i] = c * x - sn * y;
              wq[i] = sn * x + c * y;
            }
            double *rp = R + (size_t)p * cols, *rq = R + (size_t)q * cols;
            for (int i = ln; i < cols; i += kWave) {
              const double x = rp[i], y = rq[i];
              rp[i] = c * x - sn * y;
              rq[i] = sn * x + c * y;
            }
            if (ln == 0) atomicAdd(&nrot, 1);
          }
          __syncthreads();
        }
        for (int e = threadIdx.x; e < cols * n; e += nt) {
          const int c = e / n, i = e % n, g = gcol(c);
          if (g < n) Wm[(size_t)g * n + i] = Ws[e];
        }
        __syncthreads();
        if (nrot > 0) {
          // J[:, pair] = J[:, pair] R, staged through the (now free) W slice
          for (int e = threadIdx.x; e < cols * n; e += nt) {
            const int c = e / n, i = e % n, g = gcol(c);
            Ws[e] = g < n ? Jm[(size_t)g * n + i] : 0.0;
          }
          __syncthreads();
          for (int e = threadIdx.x; e < cols * n; e += nt) {
            const int c = e / n, i = e % n, g = gcol(c);
            if (g >= n) continue;
            double acc = 0.0;
            for (int d = 0; d < cols; ++d) acc += Ws[(size_t)d * n + i] * R[(size_t)c * cols + d];
            Jm[(size_t)g * n + i] = acc;
          }
          if (threadIdx.x == 0) atomicAdd(&ctrl[sweep], nrot);
        }
        __syncthreads();
      }
      grid.sync();
    }
    const int rotated = atomicAdd(&ctrl[sweep], 0);
    grid.sync();
    if (rotated == 0) break;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl[kSvdMaxSweeps] = sweep;
}

__global__ void k_identity_dense(double *__restrict__ J, int n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  J[e] = (e / n) == (e % n) ? 1.0 : 0.0;
}

static size_t block_jacobi_lds(int n, int bs) {
  return sizeof(double) * ((size_t)2 * bs * n + (size_t)4 * bs * bs);
}

int jacobi_svd(Pool &pool, double *W, double *J, int n, hipStream_t s) {
  return jacobi_svd2(pool, W, J, nullptr, nullptr, n, s);
}

// One cooperative launch for the SVDs of W (and of W2 when given): the two
// matrices share the grid barriers and stop when neither rotates.
int jacobi_svd2(Pool &pool, double *W, double *J, double *W2, double *J2, int n, hipStream_t s) {
  int dev = 0, maxlds = 0, ncu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  // Column blocks of bs: 16 when that still gives 32 or more blocks, else 8.
  // Fewer, wider blocks leave most compute units idle in a round; narrower
  // ones than 8 add rounds faster than they shorten them (n = 289, tandem
  // 1025^2 setup: 47.9 ms with bs 16, 45.3 with 8, 57.7 with 4).
  int bs = ceil_div(n, 16) >= 32 ? 16 : 8;
  while (bs > 1 && block_jacobi_lds(n, bs) + 256 > (size_t)maxlds) bs >>= 1;
  if (block_jacobi_lds(n, bs) + 256 > (size_t)maxlds)
    fail(BAMG_E_ARG, "coarsest level too large for the LDS-staged Jacobi SVD");
  const size_t shm = block_jacobi_lds(n, bs);
  const int threads = kWave * bs;
  const int nb = ceil_div(n, bs);
  int nbp = nb + (nb & 1);
  if (nbp < 2) nbp = 2;
  int *ctrl = pool.get<int>(kSvdMaxSweeps + 1);
  fill_i32(ctrl, 0, kSvdMaxSweeps + 1, s);
  const int nmat = W2 ? 2 : 1;
  k_identity_dense<<<ceil_div((long)n * n, 256), 256, 0, s>>>(J, n);  // J = I
  LAUNCHCHK();
  if (W2) {
    k_identity_dense<<<ceil_div((long)n * n, 256), 256, 0, s>>>(J2, n);
    LAUNCHCHK();
  }
  HIPCHK(hipFuncSetAttribute((const void *)k_block_jacobi_svd,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  int per = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_block_jacobi_svd,
                                                      threads, shm));
  int grid = nmat * (nbp / 2);
  const int cap = ncu * (per > 0 ? per : 1);
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  void *args[] = {(void *)&W,  (void *)&J,  (void *)&W2,  (void *)&J2,  (void *)&nmat,
                  (void *)&n,  (void *)&bs, (void *)&nbp, (void *)&ctrl};
  int sweeps = 0;
  {
    // A cooperative grid is sized to be co-resident on an otherwise idle
    // device; two of them at once (chains set up on concurrent streams)
    // could not both be resident and their grid barriers could wait
    // forever. One in flight per process, held until it has finished.
    static std::mutex coop_mu;
    std::lock_guard<std::mutex> lock(coop_mu);
    HIPCHK(hipLaunchCooperativeKernel((const void *)k_block_jacobi_svd, dim3(grid),
                                      dim3(threads), args, shm, s));
    HIPCHK(hipMemcpyAsync(&sweeps, ctrl + kSvdMaxSweeps, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  pool.release(ctrl);
  return sweeps < kSvdMaxSweeps ? BAMG_OK : BAMG_E_COARSE;
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

// Bdag = sum over kept k of J_k W_k^T / sigma_k^2 (W_k = sigma_k u_k).
__global__ void k_pinv(const double *__restrict__ W, const double *__restrict__ J,
                       const double *__restrict__ sv, int n, int kmin,
                       double *__restrict__ bdag) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
  if (j >= n) return;
  double s = 0.0;
  for (int k = 0; k < n; ++k) {
    if (k == kmin) continue;
    s += J[(size_t)k * n + i] * W[(size_t)k * n + j] / (sv[k] * sv[k]);
  }
  bdag[(size_t)i * n + j] = s;
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
  dim3 g(ceil_div(n, 128), n);
  k_pinv<<<g, 128, 0, s>>>(W, J, sv, n, kmin, bdag);
  LAUNCHCHK();
  (void)pool;
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

// right-looking Cholesky in place (lower, row-major, global memory)
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
                   double *__restrict__ sigma, double *__restrict__ bdag, int *__restrict__ flag) {
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
  if (mode == 0) {
    chol_block(Md, n, flag);
    chol_block(Nd, n, flag);
  }
  // Y = L_N^-1 B^T (column j per thread), stored in C
  for (int j = t; j < n; j += blockDim.x) {
    for (int i = 0; i < n; ++i) {
      double s = Bd[j * n + i];
      if (mode == 0) {
        for (int k = 0; k < i; ++k) s -= Nd[i * n + k] * C[k * ld + j];
        s /= Nd[i * n + i];
      }
      C[i * ld + j] = s;
    }
  }
  __syncthreads();
  // C = Y L_M^-T (row i per thread, in place)
  if (mode == 0) {
    for (int i = t; i < n; i += blockDim.x) {
      for (int k = 0; k < n; ++k) {
        double s = C[i * ld + k];
        for (int j = 0; j < k; ++j) s -= Md[k * n + j] * C[i * ld + j];
        C[i * ld + k] = s / Md[k * n + k];
      }
    }
  }
  for (int e = t; e < n * ld; e += blockDim.x) Jt[e] = (e / ld == e % ld) ? 1.0 : 0.0;
  __syncthreads();
  // one-sided Jacobi on the rows of C, round-robin pairs; each pair is
  // handled by a group of kPairLanes lanes so a round's pairs run together
  constexpr int kPairLanes = 16;
  const int grp = t / kPairLanes, gl = t % kPairLanes, ngrp = kSmallThreads / kPairLanes;
  const int m = n + (n & 1);
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 80; ++sweep) {
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
  if (t == 0) {
    for (int q = 0; q < r; ++q) {
      int best = -1;
      for (int k = 0; k < n; ++k) {
        bool taken = false;
        for (int z = 0; z < q; ++z) taken |= (order[z] == k);
        if (!taken && (best < 0 || sv[k] < sv[best])) best = k;
      }
      order[q] = best;
    }
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
  const size_t shm = coarse_small_lds(n);
  fill_i32(flag, 0, 1, s);
  if (prec == 0) {
    HIPCHK(hipFuncSetAttribute((const void *)k_coarse_small<double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    k_coarse_small<double><<<mode == 2 ? 2 : 1, kSmallThreads, shm, s>>>(
        mode, n, r, Bd, Md, Nd, (double *)U, (double *)V, sigma, bdag, flag);
  } else {
    HIPCHK(hipFuncSetAttribute((const void *)k_coarse_small<float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    k_coarse_small<float><<<mode == 2 ? 2 : 1, kSmallThreads, shm, s>>>(
        mode, n, r, Bd, Md, Nd, (float *)U, (float *)V, sigma, bdag, flag);
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
