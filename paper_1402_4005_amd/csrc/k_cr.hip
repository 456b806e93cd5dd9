// Compatible-relaxation C/F splitting: the algebraic coarsening Section 7
// names and cites. Per level, rounds of weighted-Jacobi F-relaxation on
// B_ff e_f = 0 measure how fast the current C set lets relaxation alone
// remove error; slow F points become candidates and a greedy independent
// set of them joins C, until a round's rate is below the target. A last
// step gives every F point a coarse neighbour (its interpolation set comes
// from the graph neighbours).
//
// The relaxation is integer-decision work done in floating point: each
// sweep forms a row's sum in row order with separate multiplies and adds
// (no fused multiply-add), as plain IEEE FP64 arithmetic does, so the error
// vectors, and with them the candidate sets, do not depend on the kernel's
// summation choices. The rate decision compares two norms whose sums are
// formed by block reductions.
#include <cmath>

#include "bamg_internal.h"
#include "device_common.h"

namespace bamg {

namespace {

constexpr int kCrThreads = 256;

// start error 0.5 + (priority >> 11) 2^-53 (exact in FP64), priorities as the
// MIS uses them, the diagonal, and every point F
__global__ void k_cr_start(int n, uint64_t seed, int level, const int *__restrict__ dpos,
                           const double *__restrict__ bv, uint64_t *__restrict__ pr,
                           double *__restrict__ e0, double *__restrict__ d, int *__restrict__ cf,
                           int *__restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = philox_word0((uint64_t)i, (uint64_t)level, 2, 0, seed, 0);
  pr[i] = k;
  e0[i] = 0.5 + (double)(k >> 11) * 0x1p-53;
  const double di = dpos[i] >= 0 ? bv[dpos[i]] : 0.0;
  d[i] = di;
  if (!(di != 0.0)) atomicOr(bad, 1);
  cf[i] = 0;
}

__global__ void k_cr_reset(int n, const int *__restrict__ cf, const double *__restrict__ e0,
                           double *__restrict__ e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) e[i] = cf[i] ? 0.0 : e0[i];
}

// f_i = e_i - omega (sum_j b_ij e_j) / b_ii on F points, 0 on C points
__global__ void k_cr_sweep(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                           const double *__restrict__ bv, const double *__restrict__ d,
                           double omega, const int *__restrict__ cf, const double *__restrict__ e,
                           double *__restrict__ f) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (cf[i]) {
    f[i] = 0.0;
    return;
  }
  double acc = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) acc += bv[k] * e[ci[k]];
  f[i] = e[i] - omega * (acc / d[i]);
}

// part[3 b + 0..2]: block b's sum of e_prev^2, of e^2 (F points), max |e|
__global__ void __launch_bounds__(kCrThreads)
    k_cr_norms(int n, const int *__restrict__ cf, const double *__restrict__ ep,
               const double *__restrict__ e, double *__restrict__ part) {
  __shared__ double sh[kCrThreads / kWave];
  double a = 0.0, b = 0.0, m = 0.0;
  for (long i = (long)blockIdx.x * kCrThreads + threadIdx.x; i < n;
       i += (long)gridDim.x * kCrThreads)
    if (!cf[i]) {
      a += ep[i] * ep[i];
      b += e[i] * e[i];
      m = fmax(m, fabs(e[i]));
    }
  a = block_sum<kCrThreads>(a, sh);
  b = block_sum<kCrThreads>(b, sh);
  for (int off = kWave / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, kWave));
  if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kCrThreads / kWave; ++q) m = fmax(m, sh[q]);
    part[3 * blockIdx.x] = a;
    part[3 * blockIdx.x + 1] = b;
    part[3 * blockIdx.x + 2] = m;
  }
}

__global__ void __launch_bounds__(kCrThreads)
    k_cr_norms_final(int nblk, const double *__restrict__ part, double *__restrict__ out) {
  __shared__ double sh[kCrThreads / kWave];
  double a = 0.0, b = 0.0, m = 0.0;
  for (int q = threadIdx.x; q < nblk; q += kCrThreads) {
    a += part[3 * q];
    b += part[3 * q + 1];
    m = fmax(m, part[3 * q + 2]);
  }
  a = block_sum<kCrThreads>(a, sh);
  b = block_sum<kCrThreads>(b, sh);
  for (int off = kWave / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, kWave));
  if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kCrThreads / kWave; ++q) m = fmax(m, sh[q]);
    out[0] = a;
    out[1] = b;
    out[2] = m;
  }
}

// candidates: F points with |e_i| >= beta max |e|
__global__ void k_cr_candidates(int n, const int *__restrict__ cf, const double *__restrict__ e,
                                double beta, const double *__restrict__ norms,
                                int *__restrict__ cand) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lim = beta * norms[2];
  cand[i] = !cf[i] && fabs(e[i]) >= lim;
}

// ordering key of a candidate: (candidate neighbours) 2^48 + (priority >> 16);
// state -1 for candidates (undecided), 2 for every other point
__global__ void k_cr_keys(int n, const int *__restrict__ grp, const int *__restrict__ gci,
                          const int *__restrict__ cand, const uint64_t *__restrict__ pr,
                          uint64_t *__restrict__ key, int *__restrict__ state) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!cand[i]) {
    state[i] = 2;
    return;
  }
  uint64_t w = 0;
  for (int k = grp[i]; k < grp[i + 1]; ++k) w += cand[gci[k]] != 0;
  key[i] = (w << 48) + (pr[i] >> 16);
  state[i] = -1;
}

// F points without a coarse neighbour start undecided, every other point 2
__global__ void k_cr_uncovered(int n, const int *__restrict__ grp, const int *__restrict__ gci,
                               const int *__restrict__ cf, int *__restrict__ state) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool has = cf[i] != 0;
  for (int k = grp[i]; k < grp[i + 1] && !has; ++k) has = cf[gci[k]] == 1;
  state[i] = has ? 2 : -1;
}

__global__ void k_cr_join(int n, const int *__restrict__ state, int *__restrict__ cf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && state[i] == 1) cf[i] = 1;
}

}  // namespace

void cr_cf(Pool &pool, const Csr &B, const double *bv, const int *dpos, const Csr &G,
           uint64_t seed, int level, const bamg_options &o, int *cf, hipStream_t s) {
  const int n = B.nr;
  const int nb = ceil_div(n, kCrThreads), nblk = std::min(nb, kRedBlocks);
  uint64_t *pr = pool.get<uint64_t>(n), *key = pool.get<uint64_t>(n);
  double *e0 = pool.get<double>(n), *d = pool.get<double>(n);
  double *e = pool.get<double>(n), *f = pool.get<double>(n);
  double *part = pool.get<double>(3 * (size_t)nblk + 3);
  double *norms = part + 3 * (size_t)nblk;
  int *state = pool.get<int>(n), *cand = pool.get<int>(n), *bad = pool.get<int>(1);
  fill_i32(bad, 0, 1, s);
  k_cr_start<<<nb, kCrThreads, 0, s>>>(n, seed, level, dpos, bv, pr, e0, d, cf, bad);
  LAUNCHCHK();
  if (read_int(bad, s)) fail(BAMG_E_BAD_DIAG, "compatible relaxation: zero diagonal");
  for (int round = 0; round < o.cr_rounds; ++round) {
    k_cr_reset<<<nb, kCrThreads, 0, s>>>(n, cf, e0, e);
    LAUNCHCHK();
    for (int sw = 0; sw < o.cr_sweeps; ++sw) {
      k_cr_sweep<<<nb, kCrThreads, 0, s>>>(n, B.rp, B.ci, bv, d, o.omega, cf, e, f);
      LAUNCHCHK();
      std::swap(e, f);  // e: the newest sweep, f: the one before
    }
    k_cr_norms<<<nblk, kCrThreads, 0, s>>>(n, cf, f, e, part);
    LAUNCHCHK();
    k_cr_norms_final<<<1, kCrThreads, 0, s>>>(nblk, part, norms);
    LAUNCHCHK();
    double h[3];
    HIPCHK(hipMemcpyAsync(h, norms, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double rate = h[0] > 0.0 ? std::sqrt(h[1]) / std::sqrt(h[0]) : 0.0;
    if (rate <= o.cr_theta) break;
    k_cr_candidates<<<nb, kCrThreads, 0, s>>>(n, cf, e, o.cr_beta, norms, cand);
    LAUNCHCHK();
    k_cr_keys<<<nb, kCrThreads, 0, s>>>(n, G.rp, G.ci, cand, pr, key, state);
    LAUNCHCHK();
    mis_rounds(pool, G, key, state, s);
    k_cr_join<<<nb, kCrThreads, 0, s>>>(n, state, cf);
    LAUNCHCHK();
  }
  k_cr_uncovered<<<nb, kCrThreads, 0, s>>>(n, G.rp, G.ci, cf, state);
  LAUNCHCHK();
  mis_rounds(pool, G, pr, state, s);
  k_cr_join<<<nb, kCrThreads, 0, s>>>(n, state, cf);
  LAUNCHCHK();
  for (void *p : {(void *)pr, (void *)key, (void *)e0, (void *)d, (void *)e, (void *)f,
                  (void *)part, (void *)state, (void *)cand, (void *)bad})
    pool.release(p);
}

}  // namespace bamg
