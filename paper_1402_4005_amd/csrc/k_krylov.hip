// FP64 kernels of GMRES(m) on the preconditioned residual equation
// C B e = -C B x0 (Section 6): Gram-Schmidt applied twice with fused
// multi-vector dots and updates, a one-workgroup Hessenberg/Givens update,
// and the true scaled residual ||B x|| / ||x|| of x = x0 + V y (Section 7),
// formed from the stored products B v_t so no extra SpMV is needed.
// All reductions are two-stage with a fixed order, so results do not depend
// on scheduling.
#include "bamg_internal.h"
#include "device_common.h"
#include "givens.h"

namespace bamg {

constexpr int kKT = 256;
constexpr int kArnoldiLds = 32;  // restart lengths below this stage H in LDS

// part[t * nblk + b] = sum over block b's rows of V_t . w  (t < k); t == k: w . w
__global__ void __launch_bounds__(kKT) k_multi_dot(const double *__restrict__ Vb, int n, int k,
                                                   const double *__restrict__ w,
                                                   double *__restrict__ part) {
  __shared__ double sh[kKT / kWave];
  const int t = blockIdx.y;
  const double *v = t < k ? Vb + (size_t)t * n : w;
  double s = 0.0;
  for (long i = (long)blockIdx.x * kKT + threadIdx.x; i < n; i += (long)gridDim.x * kKT)
    s += v[i] * w[i];
  s = block_sum<kKT>(s, sh);
  if (threadIdx.x == 0) part[(size_t)t * gridDim.x + blockIdx.x] = s;
}

void multi_dot(const double *Vb, int n, int k, const double *w, double *part, int nblk,
               hipStream_t s) {
  k_multi_dot<<<dim3(nblk, k + 1), kKT, 0, s>>>(Vb, n, k, w, part);
  LAUNCHCHK();
}

// out[t] = sum_b part[t * nblk + b], one block per t, fixed order
__global__ void __launch_bounds__(kKT) k_finalize_multi(const double *__restrict__ part, int nblk,
                                                        double *__restrict__ out) {
  __shared__ double sh[kKT / kWave];
  const int t = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kKT) s += part[(size_t)t * nblk + b];
  s = block_sum<kKT>(s, sh);
  if (threadIdx.x == 0) out[t] = s;
}

void finalize_multi(const double *part, int nblk, int k, double *out, hipStream_t s) {
  k_finalize_multi<<<k, kKT, 0, s>>>(part, nblk, out);
  LAUNCHCHK();
}

// w <- w - sum_t h[t] V_t ; part[b] = block partial of |w|^2
__global__ void __launch_bounds__(kKT)
    k_multi_axpy_norm(const double *__restrict__ Vb, int n, int k, const double *__restrict__ h,
                      double *__restrict__ w, double *__restrict__ part) {
  __shared__ double sh[kKT / kWave];
  __shared__ double hs[256];
  for (int t = threadIdx.x; t < k; t += kKT) hs[t] = h[t];
  __syncthreads();
  double s = 0.0;
  for (long i = (long)blockIdx.x * kKT + threadIdx.x; i < n; i += (long)gridDim.x * kKT) {
    double x = w[i];
    for (int t = 0; t < k; ++t) x -= hs[t] * Vb[(size_t)t * n + i];
    w[i] = x;
    s += x * x;
  }
  s = block_sum<kKT>(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void multi_axpy_norm(const double *Vb, int n, int k, const double *h, double *w, double *part,
                     int nblk, hipStream_t s) {
  if (k > 256) fail(BAMG_E_ARG, "restart length above 255");
  k_multi_axpy_norm<<<nblk, kKT, 0, s>>>(Vb, n, k, h, w, part);
  LAUNCHCHK();
}

// The first Gram-Schmidt update fused with the second pass's dots:
// w <- w - sum_t h[t] V_t, then part[t * nblk + b] = block b's partial of
// V_t . w (t < k). Each row's V entries are loaded once for both. Rows are
// distributed over the blocks and reduced exactly as in k_multi_dot and
// k_multi_axpy_norm, so w and the partials equal the two separate kernels'
// bit for bit. KF >= k is the compile-time bound of the register arrays
// (loads past column k - 1 re-read that column and are not used).
constexpr int kFusedK = 24;

template <int KF>
__global__ void __launch_bounds__(kKT)
    k_multi_axpy_dot(const double *__restrict__ Vb, int n, int k, const double *__restrict__ h,
                     double *__restrict__ w, double *__restrict__ part) {
  __shared__ double sh[kKT / kWave][KF];
  __shared__ double hs[KF];
  if (threadIdx.x < KF) hs[threadIdx.x] = threadIdx.x < k ? h[threadIdx.x] : 0.0;
  __syncthreads();
  double acc[KF];
#pragma unroll
  for (int t = 0; t < KF; ++t) acc[t] = 0.0;
  for (long i = (long)blockIdx.x * kKT + threadIdx.x; i < n; i += (long)gridDim.x * kKT) {
    double v[KF];
#pragma unroll
    for (int t = 0; t < KF; ++t) v[t] = Vb[(size_t)min(t, k - 1) * n + i];
    double x = w[i];
#pragma unroll
    for (int t = 0; t < KF; ++t)
      if (t < k) x -= hs[t] * v[t];
    w[i] = x;
#pragma unroll
    for (int t = 0; t < KF; ++t)
      if (t < k) acc[t] += v[t] * x;
  }
  const int wv = threadIdx.x / kWave, l = threadIdx.x % kWave;
#pragma unroll
  for (int t = 0; t < KF; ++t) {
    const double r = group_sum(acc[t], kWave);
    if (l == 0) sh[wv][t] = r;
  }
  __syncthreads();
  if (threadIdx.x < k) {
    double r = 0.0;
    for (int q = 0; q < kKT / kWave; ++q) r += sh[q][threadIdx.x];
    part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = r;
  }
}

bool multi_axpy_dot(const double *Vb, int n, int k, const double *h, double *w, double *part,
                    int nblk, hipStream_t s) {
  if (k < 1 || k > kFusedK) return false;
  switch ((k + 3) / 4) {
    case 1: k_multi_axpy_dot<4><<<nblk, kKT, 0, s>>>(Vb, n, k, h, w, part); break;
    case 2: k_multi_axpy_dot<8><<<nblk, kKT, 0, s>>>(Vb, n, k, h, w, part); break;
    case 3: k_multi_axpy_dot<12><<<nblk, kKT, 0, s>>>(Vb, n, k, h, w, part); break;
    case 4: k_multi_axpy_dot<16><<<nblk, kKT, 0, s>>>(Vb, n, k, h, w, part); break;
    case 5: k_multi_axpy_dot<20><<<nblk, kKT, 0, s>>>(Vb, n, k, h, w, part); break;
    default: k_multi_axpy_dot<24><<<nblk, kKT, 0, s>>>(Vb, n, k, h, w, part); break;
  }
  LAUNCHCHK();
  return true;
}

// Arnoldi step j of the Hessenberg matrix H ((m+1) x m, row-major), Givens
// rotations cs/sn, right-hand side g, solution y of the leading j+1 system.
// h1, h2: the two Gram-Schmidt coefficient passes (j+1 values each, plus the
// pre-orthogonalisation |w|^2 at h1[j+1]); wpart: nblk partials of the final
// |w|^2. flags[1] = breakdown, flags[3] = 1/h_{j+1,j}, flags[4] = |g_{j+1}|.
__global__ void __launch_bounds__(kKT)
    k_arnoldi_update(double *__restrict__ H, double *__restrict__ cs, double *__restrict__ sn,
                     double *__restrict__ g, double *__restrict__ y,
                     const double *__restrict__ h1, const double *__restrict__ h2,
                     const double *__restrict__ wpart, int nblk, int j, int m,
                     double *__restrict__ flags) {
  // The serial part (rotations, back substitution) runs in one thread; the
  // rows 0..j of columns 0..j of H, the rotations and g are first staged in
  // LDS by the whole block so that thread never waits on global memory.
  constexpr int kS = kArnoldiLds;  // j < kS uses the LDS copy
  __shared__ double sh[kKT / kWave];
  __shared__ double Hs[kS * kS], css[kS], sns[kS], gs[kS + 1], ys[kS], col[kS + 1];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kKT) s += wpart[b];
  s = block_sum<kKT>(s, sh);
  const bool lds = j < kS;
  if (lds) {
    for (int e = threadIdx.x; e < (j + 1) * (j + 1); e += kKT) {
      const int i = e / (j + 1), q = e % (j + 1);
      if (q >= i && q < j) Hs[i * kS + q] = H[(size_t)i * m + q];
    }
    for (int i = threadIdx.x; i <= j; i += kKT) {
      css[i] = i < j ? cs[i] : 0.0;
      sns[i] = i < j ? sn[i] : 0.0;
      gs[i] = g[i];
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  // Hr(i, q): the LDS copy when it exists, else H itself
  double *const Hb = lds ? Hs : H;
  const int ld = lds ? kS : m;
  double *const cb = lds ? css : cs, *const sb = lds ? sns : sn, *const gb = lds ? gs : g;
  double *const yb = lds ? ys : y;
  const double hn = sqrt(s);
  const double w0 = sqrt(h1[j + 1]);
  // col: column j of H, rows 0..j+1 (used when staged)
  auto cget = [&](int i) -> double { return lds ? col[i] : H[(size_t)i * m + j]; };
  auto cset = [&](int i, double v) {
    if (lds)
      col[i] = v;
    else
      H[(size_t)i * m + j] = v;
  };
  for (int i = 0; i <= j; ++i) cset(i, h1[i] + h2[i]);
  cset(j + 1, hn);
  const bool broke = !(hn > 1e-14 * w0);
  for (int i = 0; i < j; ++i) {
    double a = cget(i), b = cget(i + 1);
    givens_apply(cb[i], sb[i], a, b);
    cset(i, a);
    cset(i + 1, b);
  }
  const double a = cget(j), b = cget(j + 1);
  const double den = givens_norm(a, b);
  const double cj = den > 0 ? a / den : 1.0, sj = den > 0 ? b / den : 0.0;
  cs[j] = cj;
  sn[j] = sj;
  cset(j, den);
  cset(j + 1, 0.0);
  const double gj = gb[j];
  g[j + 1] = -sj * gj;
  g[j] = cj * gj;
  if (lds) gs[j] = cj * gj;
  if (lds)
    for (int i = 0; i <= j; ++i) Hs[i * kS + j] = col[i];
  for (int i = j; i >= 0; --i) {
    double t = gb[i];
    for (int q = i + 1; q <= j; ++q) t -= Hb[(size_t)i * ld + q] * yb[q];
    yb[i] = t / Hb[(size_t)i * ld + i];
  }
  if (lds) {
    for (int i = 0; i <= j + 1; ++i) H[(size_t)i * m + j] = col[i];
    for (int i = 0; i <= j; ++i) y[i] = ys[i];
  }
  flags[1] = broke ? 1.0 : 0.0;
  flags[3] = broke ? 0.0 : 1.0 / hn;
  flags[4] = fabs(-sj * gj);
}

void gmres_arnoldi_update(double *H, double *cs, double *sn, double *g, double *y, double *h1,
                          double *h2, const double *wnorm_part, int nblk, double *vnext_scale,
                          int j, int m, double *flags, hipStream_t s) {
  (void)vnext_scale;
  k_arnoldi_update<<<1, kKT, 0, s>>>(H, cs, sn, g, y, h1, h2, wnorm_part, nblk, j, m, flags);
  LAUNCHCHK();
}

__global__ void k_scale_vec(const double *__restrict__ in, const double *__restrict__ scal,
                            double *__restrict__ out, int n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i] * scal[0];
}

void scale_vec(const double *in, const double *scal, double *out, int n, hipStream_t s) {
  k_scale_vec<<<ceil_div(n, 256), 256, 0, s>>>(in, scal, out, n);
  LAUNCHCHK();
}

// partials of |B x0 + sum_t y_t B v_t|^2 and |x0 + sum_t y_t v_t|^2
__global__ void __launch_bounds__(kKT)
    k_resid_part(const double *__restrict__ x0, const double *__restrict__ bx0,
                 const double *__restrict__ Vb, const double *__restrict__ BVb,
                 const double *__restrict__ y, int n, int k, double *__restrict__ part) {
  __shared__ double sh[kKT / kWave];
  __shared__ double ys[256];
  for (int t = threadIdx.x; t < k; t += kKT) ys[t] = y[t];
  __syncthreads();
  double sb = 0.0, sx = 0.0;
  for (long i = (long)blockIdx.x * kKT + threadIdx.x; i < n; i += (long)gridDim.x * kKT) {
    double bx = bx0[i], xx = x0[i];
    for (int t = 0; t < k; ++t) {
      bx += ys[t] * BVb[(size_t)t * n + i];
      xx += ys[t] * Vb[(size_t)t * n + i];
    }
    sb += bx * bx;
    sx += xx * xx;
  }
  sb = block_sum<kKT>(sb, sh);
  sx = block_sum<kKT>(sx, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sb;
    part[gridDim.x + blockIdx.x] = sx;
  }
}

void residual_check_partials(const double *x0, const double *bx0, const double *Vb,
                             const double *BVb, const double *y, int n, int k, double *part,
                             int nblk, hipStream_t s) {
  k_resid_part<<<nblk, kKT, 0, s>>>(x0, bx0, Vb, BVb, y, n, k, part);
  LAUNCHCHK();
}

// flags[0] = converged, flags[2] = ||Bx||/||x||; then all 16 flags are
// copied to host_out (mapped pinned memory) when it is not null.
__global__ void __launch_bounds__(kKT) k_resid_final(const double *__restrict__ part, int nblk,
                                                     double tol, double *__restrict__ flags,
                                                     double *__restrict__ host_out) {
  __shared__ double sh[kKT / kWave];
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < nblk; q += kKT) {
    a += part[q];
    b += part[nblk + q];
  }
  a = block_sum<kKT>(a, sh);
  b = block_sum<kKT>(b, sh);
  if (threadIdx.x == 0) {
    const double rel = b > 0.0 ? sqrt(a) / sqrt(b) : INFINITY;
    flags[2] = rel;
    flags[0] = rel < tol ? 1.0 : 0.0;
    if (host_out)
      for (int q = 0; q < 16; ++q) host_out[q] = flags[q];
  }
}

void residual_check_finalize(const double *part, int nblk, double tol, double *flags,
                             double *host_out, hipStream_t s) {
  k_resid_final<<<1, kKT, 0, s>>>(part, nblk, tol, flags, host_out);
  LAUNCHCHK();
}

__global__ void k_update_iterate(double *__restrict__ x0, const double *__restrict__ Vb,
                                 const double *__restrict__ y, int n, int k) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = x0[i];
  for (int t = 0; t < k; ++t) x += y[t] * Vb[(size_t)t * n + i];
  x0[i] = x;
}

void update_iterate(double *x0, const double *Vb, const double *y, int n, int k, hipStream_t s) {
  k_update_iterate<<<ceil_div(n, 256), 256, 0, s>>>(x0, Vb, y, n, k);
  LAUNCHCHK();
}

__global__ void k_negate(const double *__restrict__ in, double *__restrict__ out, int n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = -in[i];
}

void negate_copy(const double *in, double *out, int n, hipStream_t s) {
  k_negate<<<ceil_div(n, 256), 256, 0, s>>>(in, out, n);
  LAUNCHCHK();
}

// x <- x / sum(x); flags[5] = min x afterwards, flags[6] = sum before
__global__ void __launch_bounds__(kKT) k_sum_min_part(const double *__restrict__ x, int n,
                                                      double *__restrict__ part) {
  __shared__ double sh[kKT / kWave];
  double s = 0.0;
  for (long i = (long)blockIdx.x * kKT + threadIdx.x; i < n; i += (long)gridDim.x * kKT) s += x[i];
  s = block_sum<kKT>(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kKT) k_sum_final(const double *__restrict__ part, int nblk,
                                                   double *__restrict__ flags) {
  __shared__ double sh[kKT / kWave];
  double s = 0.0;
  for (int q = threadIdx.x; q < nblk; q += kKT) s += part[q];
  s = block_sum<kKT>(s, sh);
  if (threadIdx.x == 0) {
    flags[6] = s;
    flags[7] = s != 0.0 ? 1.0 / s : 1.0;
  }
}

__global__ void __launch_bounds__(kKT) k_scale_min(double *__restrict__ x, int n,
                                                   const double *__restrict__ flags,
                                                   double *__restrict__ part) {
  __shared__ double sh[kKT / kWave];
  const double sc = flags[7];
  double mn = INFINITY;
  for (long i = (long)blockIdx.x * kKT + threadIdx.x; i < n; i += (long)gridDim.x * kKT) {
    const double v = x[i] * sc;
    x[i] = v;
    mn = fmin(mn, v);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) mn = fmin(mn, __shfl_xor(mn, off, kWave));
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  if (l == 0) sh[w] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int q = 1; q < kKT / kWave; ++q) r = fmin(r, sh[q]);
    part[blockIdx.x] = r;
  }
}

__global__ void __launch_bounds__(kKT) k_min_final(const double *__restrict__ part, int nblk,
                                                   double *__restrict__ flags) {
  __shared__ double sh[kKT / kWave];
  double r = INFINITY;
  for (int q = threadIdx.x; q < nblk; q += kKT) r = fmin(r, part[q]);
  for (int off = kWave / 2; off > 0; off >>= 1) r = fmin(r, __shfl_xor(r, off, kWave));
  if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = sh[0];
    for (int q = 1; q < kKT / kWave; ++q) m = fmin(m, sh[q]);
    flags[5] = m;
  }
}

void normalize_sum(double *x, int n, double *part, int nblk, double *flags, hipStream_t s) {
  k_sum_min_part<<<nblk, kKT, 0, s>>>(x, n, part);
  LAUNCHCHK();
  k_sum_final<<<1, kKT, 0, s>>>(part, nblk, flags);
  LAUNCHCHK();
  k_scale_min<<<nblk, kKT, 0, s>>>(x, n, flags, part);
  LAUNCHCHK();
  k_min_final<<<1, kKT, 0, s>>>(part, nblk, flags);
  LAUNCHCHK();
}

}  // namespace bamg
