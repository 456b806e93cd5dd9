// Batched solve in one persistent launch: GMRES(m) on the residual equation
// (Section 6) with the V-cycle of Section 3 as preconditioner and the
// stopping test of Section 7, for many independent chains at once.
//
// Every workgroup takes the next chain from a device counter (largest chains
// first) and runs its whole solve with workgroup barriers only: no host
// round trip and no launch per step, which is what a chain of a few thousand
// to a few tens of thousands of states is otherwise bound by. Workgroups
// never wait for each other; each leaves when the counter passes the last
// chain.
//
// The arithmetic is that of the one-kernel-per-step solve of the same
// handle, step for step and in the same summation orders, so a chain's
// result does not depend on which of the two ran it:
//  * sweeps and residuals form their row sums canonically (sparse_row.h),
//    the transfers too (at most 4 lanes per row on both paths);
//  * the fused last level (one workgroup there too) keeps its W-lane sums;
//  * GMRES's dot products are formed as the two-stage reductions of the
//    per-step kernels: each wave here forms the partial of one of their
//    256-thread blocks, from the same per-thread sequential sums, the same
//    64-lane butterfly and the same in-order sum of the four waves, and the
//    final sums follow the same pattern over the partials.
#include <algorithm>
#include <cstring>
#include <functional>
#include <vector>

#include "bamg_internal.h"
#include "device_common.h"
#include "givens.h"
#include "sparse_row.h"

namespace bamg {

constexpr int kBatchThreads = 1024;
constexpr int kBatchWaves = kBatchThreads / kWave;
constexpr int kRedThreads = 256;  // block size of the per-step reductions
constexpr int kRedWaves = kRedThreads / kWave;

// one level of a chain's hierarchy; T-typed arrays as void*
struct BatchLevel {
  int n = 0, nc = 0, lanes = 1, fused_w = 0;
  const int *brp = nullptr, *bci = nullptr;
  const void *bv = nullptr, *dinv = nullptr;
  const int *prp = nullptr, *pci = nullptr;  // P: n x nc
  const void *pv = nullptr;
  int plpr = 1;
  const int *qrp = nullptr, *qci = nullptr;  // Q: nc x n
  const void *qv = nullptr;
  int qlpr = 1;
  void *xb = nullptr, *bb = nullptr, *rb = nullptr, *tb = nullptr;
  int ncol = 0;  // Kaczmarz: colours, rows by colour, colour offsets
  const int *kord = nullptr, *koff = nullptr;
  const void *rowinv = nullptr;
};

struct BatchChain {
  int L = 0, n = 0, prec = 0, smoother = 0, cycle = 0, nu1 = 0, nu2 = 0;
  int m = 0, maxit = 0, nblk = 1, lanes0 = 1, nL = 0;
  double tol = 0.0, omega = 0.0;
  const int *rp = nullptr, *ci = nullptr;
  const double *b64 = nullptr, *bdag = nullptr, *xstart = nullptr;
  double *xout = nullptr;
  double *V = nullptr, *BV = nullptr, *w = nullptr, *x0 = nullptr, *bx0 = nullptr;
  double *vcin = nullptr, *part = nullptr;
  float *vb = nullptr, *vx = nullptr;
  const BatchLevel *lv = nullptr;  // device, L entries
};

struct BatchResult {
  int status, iterations, restarts, converged, breakdowns, pad;
  double rel, xmin;
  long long ticks;
};

namespace {

__device__ __forceinline__ void wg_sync() { __syncthreads(); }

// ---------------------------------------------------------------- rows
// f(row, lane) for every row, by groups of LPR consecutive lanes
template <int LPR, class F>
__device__ __forceinline__ void rows_by(int nr, F f) {
  const int grp = threadIdx.x / LPR, lane = threadIdx.x % LPR, ng = kBatchThreads / LPR;
  for (int r0 = 0; r0 < nr; r0 += ng) {
    const int row = r0 + grp;
    if (row < nr) f(row, lane);  // whole groups take the same branch
  }
}

// out(row, sum of row's val * g(col)) with LPR lanes per row, as k_spmv
template <class T, int LPR, class G, class O>
__device__ __forceinline__ void csr_rows_lpr(int nr, const int *rp, const int *ci, const T *val,
                                             G g, O out) {
  rows_by<LPR>(nr, [&](int row, int lane) {
    const T s = row_sum<T, LPR>(rp[row], rp[row + 1], lane, ci, val, g);
    if (lane == 0) out(row, s);
  });
}

// B-operator and transfer rows: canonical sums, so 1, 2 or 4 lanes give the
// same bits
template <class T, class G, class O>
__device__ void csr_rows_canon(int lanes, int nr, const int *rp, const int *ci, const T *val, G g,
                               O out) {
  if (lanes >= 4)
    csr_rows_lpr<T, 4>(nr, rp, ci, val, g, out);
  else if (lanes == 2)
    csr_rows_lpr<T, 2>(nr, rp, ci, val, g, out);
  else
    csr_rows_lpr<T, 1>(nr, rp, ci, val, g, out);
}

// ---------------------------------------------------------------- V-cycle
template <class T>
__device__ void smooth(const BatchChain &c, const BatchLevel &L, const T *b, T *x, int steps,
                       bool from_zero) {
  const T *bv = (const T *)L.bv, *dinv = (const T *)L.dinv;
  const int n = L.n;
  if (steps <= 0) {
    if (from_zero) {
      for (int i = threadIdx.x; i < n; i += kBatchThreads) x[i] = (T)0;
      wg_sync();
    }
    return;
  }
  if (c.smoother == BAMG_SMOOTH_KACZMARZ) {
    if (from_zero) {
      for (int i = threadIdx.x; i < n; i += kBatchThreads) x[i] = (T)0;
      wg_sync();
    }
    const T *rowinv = (const T *)L.rowinv;
    for (int it = 0; it < steps; ++it)
      for (int col = 0; col < L.ncol; ++col) {
        const int a = L.koff[col], e = L.koff[col + 1];
        for (int t = a + threadIdx.x; t < e; t += kBatchThreads) {
          const int i = L.kord[t];
          T ax = 0;
          for (int k = L.brp[i]; k < L.brp[i + 1]; ++k) ax += bv[k] * x[L.bci[k]];
          const T cc = (b[i] - ax) * rowinv[i];
          for (int k = L.brp[i]; k < L.brp[i + 1]; ++k) x[L.bci[k]] += cc * bv[k];
        }
        wg_sync();
      }
    return;
  }
  const T om = (T)c.omega;
  T *spare = (T *)L.tb;
  T *cur = x, *oth = spare;
  if (from_zero) {
    const int done = steps >= 2 ? 2 : 1;
    T *first = ((steps - done) % 2 == 0) ? x : spare;
    if (done == 2)
      csr_rows_canon<T>(
          L.lanes, n, L.brp, L.bci, bv, [&](int col) { return jacobi_first(om, dinv[col], b[col]); },
          [&](int row, T s) {
            const T dr = dinv[row], br = b[row];
            first[row] = jacobi_next(jacobi_first(om, dr, br), om, dr, br, s);
          });
    else
      for (int i = threadIdx.x; i < n; i += kBatchThreads) first[i] = jacobi_first(om, dinv[i], b[i]);
    wg_sync();
    cur = first;
    oth = first == x ? spare : x;
    steps -= done;
  } else if (steps % 2 == 1) {
    cur = spare;
    oth = x;
  }
  for (int it = 0; it < steps; ++it) {
    const T *xi = cur;
    T *xo = oth;
    csr_rows_canon<T>(L.lanes, n, L.brp, L.bci, bv, [&](int col) { return xi[col]; },
                      [&](int row, T s) { xo[row] = jacobi_next(xi[row], om, dinv[row], b[row], s); });
    wg_sync();
    T *tmp = cur;
    cur = oth;
    oth = tmp;
  }
}

// the last smoothed level and the coarsest solve as the fused one-workgroup
// form computes them: W lanes per row striding over its entries, then a
// W-lane butterfly; the dense solve in FP64 with the same lanes
template <class T>
__device__ void fused_last(const BatchChain &c, const BatchLevel &L, const BatchLevel &C,
                           const T *b, T *xg) {
  const int W = L.fused_w, n = L.n, nc = C.n;
  const int grp = threadIdx.x / W, lane = threadIdx.x % W, ngrp = kBatchThreads / W;
  const T *val = (const T *)L.bv, *dinv = (const T *)L.dinv;
  const T *pv = (const T *)L.pv, *qv = (const T *)L.qv;
  // x (the output buffer) and y ping-pong, r the residual; bc and xc in the
  // coarsest level's vectors
  T *x = xg, *y = (T *)L.tb, *r = (T *)L.rb, *bc = (T *)C.bb, *xc = (T *)C.xb;
  auto rows_w = [&](int nrows, const int *rr, const int *cc, const T *vv, const T *v, auto &&f) {
    for (int i0 = 0; i0 < nrows; i0 += ngrp) {
      const int i = i0 + grp;
      T s = 0;
      if (i < nrows)
        for (int k = rr[i] + lane; k < rr[i + 1]; k += W) s += vv[k] * v[cc[k]];
      s = group_sum(s, W);
      if (i < nrows && lane == 0) f(i, s);
    }
  };
  const T om = (T)c.omega;
  for (int i = threadIdx.x; i < n; i += kBatchThreads)
    x[i] = c.nu1 > 0 ? jacobi_first(om, dinv[i], b[i]) : (T)0;
  wg_sync();
  T *cur = x, *oth = y;
  for (int it = 1; it < c.nu1; ++it) {
    const T *xi = cur;
    T *xo = oth;
    rows_w(n, L.brp, L.bci, val, xi,
           [&](int i, T s) { xo[i] = jacobi_next(xi[i], om, dinv[i], b[i], s); });
    wg_sync();
    T *tmp = cur;
    cur = oth;
    oth = tmp;
  }
  {
    const T *xi = cur;
    rows_w(n, L.brp, L.bci, val, xi, [&](int i, T s) { r[i] = b[i] - s; });
  }
  wg_sync();
  rows_w(nc, L.qrp, L.qci, qv, r, [&](int j, T s) { bc[j] = s; });
  wg_sync();
  for (int j0 = 0; j0 < nc; j0 += ngrp) {
    const int j = j0 + grp;
    double s = 0.0;
    if (j < nc)
      for (int q = lane; q < nc; q += W) s += c.bdag[(size_t)j * nc + q] * (double)bc[q];
    s = group_sum(s, W);
    if (j < nc && lane == 0) xc[j] = (T)s;
  }
  wg_sync();
  {
    T *xo = cur;
    rows_w(n, L.prp, L.pci, pv, xc, [&](int i, T s) { xo[i] += s; });
  }
  wg_sync();
  for (int it = 0; it < c.nu2; ++it) {
    const T *xi = cur;
    T *xo = oth;
    rows_w(n, L.brp, L.bci, val, xi,
           [&](int i, T s) { xo[i] = jacobi_next(xi[i], om, dinv[i], b[i], s); });
    wg_sync();
    T *tmp = cur;
    cur = oth;
    oth = tmp;
  }
  if (cur != xg) {
    for (int i = threadIdx.x; i < n; i += kBatchThreads) xg[i] = cur[i];
    wg_sync();
  }
}

// x = C b: one V-cycle from zero (or the identity for no preconditioner)
template <class T>
__device__ void vcycle(const BatchChain &c, const T *b0, T *x0) {
  const BatchLevel *lv = c.lv;
  if (c.cycle == BAMG_CYCLE_NONE) {
    for (int i = threadIdx.x; i < c.n; i += kBatchThreads) x0[i] = b0[i];
    wg_sync();
    return;
  }
  const bool jac = c.smoother != BAMG_SMOOTH_KACZMARZ;
  int lf = -1;  // the level the fused form handled
  for (int l = 0; l + 1 < c.L; ++l) {
    const BatchLevel &L = lv[l], &C = lv[l + 1];
    const T *b = l == 0 ? b0 : (const T *)L.bb;
    T *x = l == 0 ? x0 : (T *)L.xb;
    if (L.fused_w > 0) {
      fused_last<T>(c, L, C, b, x);
      lf = l;
      break;
    }
    smooth<T>(c, L, b, x, c.nu1, true);
    const T *bv = (const T *)L.bv;
    T *rb = (T *)L.rb;
    const T *xc = x;
    csr_rows_canon<T>(L.lanes, L.n, L.brp, L.bci, bv, [&](int col) { return xc[col]; },
                      [&](int row, T s) { rb[row] = b[row] - s; });
    wg_sync();
    T *bbc = (T *)C.bb;
    csr_rows_canon<T>(L.qlpr, L.nc, L.qrp, L.qci, (const T *)L.qv,
                    [&](int col) { return rb[col]; }, [&](int row, T s) { bbc[row] = s; });
    wg_sync();
  }
  if (lf < 0) {
    // coarsest: x = B_L^+ b, one wave per row
    const BatchLevel &C = lv[c.L - 1];
    const T *bb = c.L == 1 ? b0 : (const T *)C.bb;
    T *xb = c.L == 1 ? x0 : (T *)C.xb;
    const int nL = C.n, wv = threadIdx.x / kWave, ln = threadIdx.x % kWave;
    for (int row = wv; row < nL; row += kBatchWaves) {
      double s = 0.0;
      const double *rr = c.bdag + (size_t)row * nL;
      for (int j = ln; j < nL; j += kWave) s += rr[j] * (double)bb[j];
      s = group_sum(s, kWave);
      if (ln == 0) xb[row] = (T)s;
    }
    wg_sync();
  }
  for (int l = (lf < 0 ? c.L - 2 : lf - 1); l >= 0; --l) {
    const BatchLevel &L = lv[l], &C = lv[l + 1];
    const T *b = l == 0 ? b0 : (const T *)L.bb;
    T *x = l == 0 ? x0 : (T *)L.xb;
    const T *xcor = (const T *)C.xb, *pv = (const T *)L.pv;
    if (jac && c.nu2 % 2 == 1) {
      // spare = x + P x_c (sequential row sums), then an odd sweep count ends in x
      T *tb = (T *)L.tb;
      for (int i = threadIdx.x; i < L.n; i += kBatchThreads) {
        T s = 0;
        for (int a = L.prp[i]; a < L.prp[i + 1]; ++a) s += pv[a] * xcor[L.pci[a]];
        tb[i] = x[i] + s;
      }
    } else {
      csr_rows_canon<T>(L.plpr, L.n, L.prp, L.pci, pv, [&](int col) { return xcor[col]; },
                      [&](int row, T s) { x[row] = x[row] + s; });
    }
    wg_sync();
    smooth<T>(c, L, b, x, c.nu2, false);
  }
}

// ---------------------------------------------------------------- reductions
// Partial of one 256-thread block b of nblk of a per-step reduction kernel:
// thread tt of the block holds the sequential sum acc(s, i) over rows
// i = 256 b + tt + 256 nblk k (k = 0, 1, ...), the block adds its four
// waves' butterflies in order. Formed here by one wave; every lane returns it.
template <class Acc>
__device__ __forceinline__ double block_partial(int b, int nblk, int n, Acc acc) {
  const int ln = threadIdx.x % kWave;
  double r = 0.0;
  for (int q = 0; q < kRedWaves; ++q) {
    double s = 0.0;
    for (long i = (long)b * kRedThreads + q * kWave + ln; i < n; i += (long)nblk * kRedThreads)
      acc(s, i);
    r += group_sum(s, kWave);
  }
  return r;
}

// The same partial when every thread of the 256-thread block holds at most
// one row (nblk * 256 >= n, so the stride passes the end): the lane holds
// row 256 b + 64 q + ln of each sub-wave q, rows[q] < 0 past the end, and
// the four sub-waves' loads and butterflies are independent of each other.
__device__ __forceinline__ void block_rows(int b, int n, long rows[kRedWaves]) {
  const int ln = threadIdx.x % kWave;
#pragma unroll
  for (int q = 0; q < kRedWaves; ++q) {
    const long i = (long)b * kRedThreads + q * kWave + ln;
    rows[q] = i < n ? i : -1;
  }
}
__device__ __forceinline__ double block_combine(double s[kRedWaves]) {
#pragma unroll
  for (int q = 0; q < kRedWaves; ++q) s[q] = group_sum(s[q], kWave);
  double r = 0.0;
#pragma unroll
  for (int q = 0; q < kRedWaves; ++q) r += s[q];
  return r;
}

// the final stage: thread tt adds partials tt, tt + 256, ... in order, then
// the block sum as above; one wave
__device__ __forceinline__ double final_sum(const double *part, int nblk) {
  const int ln = threadIdx.x % kWave;
  double r = 0.0;
  for (int q = 0; q < kRedWaves; ++q) {
    double s = 0.0;
    for (int b = q * kWave + ln; b < nblk; b += kRedThreads) s += part[b];
    r += group_sum(s, kWave);
  }
  return r;
}

// part[t * nblk + b]: V_t . w for t < k, and w . w at t == k when with_ww
__device__ void multi_dot(const BatchChain &c, int k, bool with_ww) {
  const int nb = c.nblk, n = c.n, wv = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  const int nt = with_ww ? k + 1 : k;
  const double *w = c.w;
  if ((long)nb * kRedThreads >= n) {
    // a wave per block, every vector of it: w loaded once, two vectors'
    // loads in flight at a time
    for (int b = wv; b < nb; b += kBatchWaves) {
      long rows[kRedWaves];
      double wq[kRedWaves];
      block_rows(b, n, rows);
#pragma unroll
      for (int q = 0; q < kRedWaves; ++q) wq[q] = rows[q] >= 0 ? w[rows[q]] : 0.0;
      for (int t = 0; t < nt; t += 2) {
        const double *v0 = t < k ? c.V + (size_t)t * n : w;
        const double *v1 = t + 1 < k ? c.V + (size_t)(t + 1) * n : w;
        double s0[kRedWaves], s1[kRedWaves];
#pragma unroll
        for (int q = 0; q < kRedWaves; ++q) {
          s0[q] = 0.0;
          s1[q] = 0.0;
          if (rows[q] >= 0) {
            s0[q] += v0[rows[q]] * wq[q];
            if (t + 1 < nt) s1[q] += v1[rows[q]] * wq[q];
          }
        }
        const double r0 = block_combine(s0);
        if (ln == 0) c.part[(size_t)t * nb + b] = r0;
        if (t + 1 < nt) {
          const double r1 = block_combine(s1);
          if (ln == 0) c.part[(size_t)(t + 1) * nb + b] = r1;
        }
      }
    }
    wg_sync();
    return;
  }
  for (int idx = wv; idx < nt * nb; idx += kBatchWaves) {
    const int t = idx / nb, b = idx % nb;
    const double *v = t < k ? c.V + (size_t)t * n : w;
    const double r = block_partial(b, nb, n, [&](double &s, long i) { s += v[i] * w[i]; });
    if (ln == 0) c.part[(size_t)t * nb + b] = r;
  }
  wg_sync();
}

// out[t] = final sum of part[t * nblk ...] for t < cnt (out in LDS)
__device__ void finalize(const BatchChain &c, int cnt, double *out) {
  const int wv = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  for (int t = wv; t < cnt; t += kBatchWaves) {
    const double r = final_sum(c.part + (size_t)t * c.nblk, c.nblk);
    if (ln == 0) out[t] = r;
  }
  wg_sync();
}

// w <- w - sum_t h[t] V_t (t < k); with norm, part2[b] = partial of |w|^2
__device__ void multi_axpy(const BatchChain &c, int k, const double *h, double *part2) {
  const int nb = c.nblk, n = c.n, wv = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  double *w = c.w;
  const double *V = c.V;
  if ((long)nb * kRedThreads >= n) {
    for (int b = wv; b < nb; b += kBatchWaves) {
      long rows[kRedWaves];
      double x[kRedWaves], sq[kRedWaves];
      block_rows(b, n, rows);
#pragma unroll
      for (int q = 0; q < kRedWaves; ++q) x[q] = rows[q] >= 0 ? w[rows[q]] : 0.0;
      for (int t = 0; t < k; ++t) {
        const double ht = h[t];
        const double *vt = V + (size_t)t * n;
#pragma unroll
        for (int q = 0; q < kRedWaves; ++q)
          if (rows[q] >= 0) x[q] -= ht * vt[rows[q]];
      }
#pragma unroll
      for (int q = 0; q < kRedWaves; ++q) {
        sq[q] = 0.0;
        if (rows[q] >= 0) {
          w[rows[q]] = x[q];
          sq[q] += x[q] * x[q];
        }
      }
      const double r = block_combine(sq);
      if (part2 && ln == 0) part2[b] = r;
    }
    wg_sync();
    return;
  }
  for (int b = wv; b < nb; b += kBatchWaves) {
    const double r = block_partial(b, nb, n, [&](double &s, long i) {
      double x = w[i];
      for (int t = 0; t < k; ++t) x -= h[t] * V[(size_t)t * n + i];
      w[i] = x;
      s += x * x;
    });
    if (part2 && ln == 0) part2[b] = r;
  }
  wg_sync();
}

}  // namespace

// ---------------------------------------------------------------- one chain
// The solver state in LDS: Hessenberg matrix, rotations, g, y, the two
// Gram-Schmidt coefficient passes, a column and flags.
struct Krylov {
  static constexpr int kM = kBatchMaxRestart;
  double *H, *cs, *sn, *g, *y, *c1, *c2, *col, *fl;  // fl: 8 flags
  __device__ Krylov(double *Hs, double *sh)
      : H(Hs), cs(sh), sn(sh + kM + 2), g(sh + 2 * (kM + 2)), y(sh + 3 * (kM + 2)),
        c1(sh + 4 * (kM + 2)), c2(sh + 5 * (kM + 2)), col(sh + 6 * (kM + 2)),
        fl(sh + 7 * (kM + 2)) {}
};

// FP64 products with the finest B: mode 0 bx0 = B x0; mode 1 BV_j = B V_j
// (and into vcin); mode 2 V_j = w sc, BV_j = B V_j (and into vcin)
__device__ void b_product(const BatchChain &c, int mode, int j, double sc) {
  const int n = c.n;
  if (mode == 0) {
    const double *x0 = c.x0;
    double *bx0 = c.bx0;
    csr_rows_canon<double>(c.lanes0, n, c.rp, c.ci, c.b64, [&](int col) { return x0[col]; },
                           [&](int row, double s) { bx0[row] = s; });
  } else if (mode == 1) {
    const double *vj = c.V + (size_t)j * n;
    double *bvj = c.BV + (size_t)j * n, *vcin = c.vcin;
    csr_rows_canon<double>(c.lanes0, n, c.rp, c.ci, c.b64, [&](int cc) { return vj[cc]; },
                           [&](int row, double s) {
                             bvj[row] = s;
                             vcin[row] = s;
                           });
  } else {
    const double *w = c.w;
    double *vj = c.V + (size_t)j * n, *bvj = c.BV + (size_t)j * n, *vcin = c.vcin;
    csr_rows_canon<double>(c.lanes0, n, c.rp, c.ci, c.b64, [&](int cc) { return w[cc] * sc; },
                           [&](int row, double s) {
                             vj[row] = w[row] * sc;
                             bvj[row] = s;
                             vcin[row] = s;
                           });
  }
  wg_sync();
}

// ||B x|| / ||x|| for x = x0 + V y (k terms) from the stored products:
// fl[2] = the ratio, fl[0] = 1 when below tol
__device__ void residual_check(const BatchChain &c, int k, const double *y,
                                            double *fl) {
  const int n = c.n, nb = c.nblk, wv = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  double *part3 = c.part + (size_t)(c.m + 3) * nb;
  const double *x0 = c.x0, *bx0 = c.bx0, *V = c.V, *BV = c.BV;
  if ((long)nb * kRedThreads >= n) {
    for (int b = wv; b < nb; b += kBatchWaves) {
      long rows[kRedWaves];
      double bx[kRedWaves], xx[kRedWaves], sb[kRedWaves], sx[kRedWaves];
      block_rows(b, n, rows);
#pragma unroll
      for (int q = 0; q < kRedWaves; ++q) {
        bx[q] = rows[q] >= 0 ? bx0[rows[q]] : 0.0;
        xx[q] = rows[q] >= 0 ? x0[rows[q]] : 0.0;
      }
      for (int t = 0; t < k; ++t) {
        const double yt = y[t];
        const double *bvt = BV + (size_t)t * n, *vt = V + (size_t)t * n;
#pragma unroll
        for (int q = 0; q < kRedWaves; ++q)
          if (rows[q] >= 0) {
            bx[q] += yt * bvt[rows[q]];
            xx[q] += yt * vt[rows[q]];
          }
      }
#pragma unroll
      for (int q = 0; q < kRedWaves; ++q) {
        sb[q] = 0.0;
        sx[q] = 0.0;
        if (rows[q] >= 0) {
          sb[q] += bx[q] * bx[q];
          sx[q] += xx[q] * xx[q];
        }
      }
      const double ra = block_combine(sb), rb = block_combine(sx);
      if (ln == 0) {
        part3[b] = ra;
        part3[nb + b] = rb;
      }
    }
  } else
  for (int b = wv; b < nb; b += kBatchWaves) {
    double ra = 0.0, rb = 0.0;
    for (int q = 0; q < kRedWaves; ++q) {
      double sb = 0.0, sx = 0.0;
      for (long i = (long)b * kRedThreads + q * kWave + ln; i < n; i += (long)nb * kRedThreads) {
        double bx = bx0[i], xx = x0[i];
        for (int t = 0; t < k; ++t) {
          bx += y[t] * BV[(size_t)t * n + i];
          xx += y[t] * V[(size_t)t * n + i];
        }
        sb += bx * bx;
        sx += xx * xx;
      }
      ra += group_sum(sb, kWave);
      rb += group_sum(sx, kWave);
    }
    if (ln == 0) {
      part3[b] = ra;
      part3[nb + b] = rb;
    }
  }
  wg_sync();
  if (threadIdx.x < kWave) {
    const double a = final_sum(part3, nb), bb = final_sum(part3 + nb, nb);
    if (threadIdx.x == 0) {
      const double rel = bb > 0.0 ? sqrt(a) / sqrt(bb) : INFINITY;
      fl[2] = rel;
      fl[0] = rel < c.tol ? 1.0 : 0.0;
    }
  }
  wg_sync();
}

// w = C vcin (FP32 inside for a mixed-precision chain)
template <class T>
__device__ void precondition(const BatchChain &c) {
  if constexpr (sizeof(T) == sizeof(double)) {
    vcycle<double>(c, c.vcin, c.w);
  } else {
    const int n = c.n;
    for (int i = threadIdx.x; i < n; i += kBatchThreads) c.vb[i] = (float)c.vcin[i];
    wg_sync();
    vcycle<float>(c, c.vb, c.vx);
    for (int i = threadIdx.x; i < n; i += kBatchThreads) c.w[i] = (double)c.vx[i];
    wg_sync();
  }
}

// Hessenberg column j from the two coefficient passes and |w|^2 (partials
// in part2), the Givens rotations, g and y; fl[1] = breakdown, fl[3] =
// 1 / h_{j+1,j}. One thread, LDS only.
__device__ void arnoldi_step(const BatchChain &c, Krylov &k, int j) {
  constexpr int kM = Krylov::kM;
  if (threadIdx.x < kWave) {
    const double s = final_sum(c.part + (size_t)(c.m + 2) * c.nblk, c.nblk);
    if (threadIdx.x == 0) {
      double *col = k.col, *cs = k.cs, *sn = k.sn, *g = k.g, *y = k.y, *H = k.H;
      const double hn = sqrt(s);
      const double w0 = sqrt(k.c1[j + 1]);
      for (int i = 0; i <= j; ++i) col[i] = k.c1[i] + k.c2[i];
      col[j + 1] = hn;
      const bool bk = !(hn > 1e-14 * w0);
      for (int i = 0; i < j; ++i) {
        double a = col[i], bb = col[i + 1];
        givens_apply(cs[i], sn[i], a, bb);
        col[i] = a;
        col[i + 1] = bb;
      }
      const double a = col[j], bb = col[j + 1];
      const double den = givens_norm(a, bb);
      const double cj = den > 0 ? a / den : 1.0, sj = den > 0 ? bb / den : 0.0;
      cs[j] = cj;
      sn[j] = sj;
      col[j] = den;
      col[j + 1] = 0.0;
      const double gj = g[j];
      g[j + 1] = -sj * gj;
      g[j] = cj * gj;
      for (int i = 0; i <= j; ++i) H[i * kM + j] = col[i];
      for (int i = j; i >= 0; --i) {
        double t = g[i];
        for (int q = i + 1; q <= j; ++q) t -= H[i * kM + q] * y[q];
        y[i] = t / H[i * kM + i];
      }
      k.fl[1] = bk ? 1.0 : 0.0;
      k.fl[3] = bk ? 0.0 : 1.0 / hn;
    }
  }
  wg_sync();
}

// x_out = x0 / (1^T x0) (the sum formed as the per-step kernels form it);
// returns the smallest entry
__device__ double normalize_out(const BatchChain &c, double *tmp) {
  const int n = c.n, nb = c.nblk, wv = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  const double *x0 = c.x0;
  for (int b = wv; b < nb; b += kBatchWaves) {
    const double r = block_partial(b, nb, n, [&](double &s, long i) { s += x0[i]; });
    if (ln == 0) c.part[b] = r;
  }
  wg_sync();
  if (threadIdx.x < kWave) {
    const double s = final_sum(c.part, nb);
    if (threadIdx.x == 0) tmp[kBatchWaves] = s != 0.0 ? 1.0 / s : 1.0;
  }
  wg_sync();
  const double sc = tmp[kBatchWaves];
  double mn = INFINITY;
  for (int i = threadIdx.x; i < n; i += kBatchThreads) {
    const double v = x0[i] * sc;
    c.xout[i] = v;
    mn = fmin(mn, v);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) mn = fmin(mn, __shfl_xor(mn, off, kWave));
  if (ln == 0) tmp[wv] = mn;
  wg_sync();
  double r = tmp[0];
  for (int q = 1; q < kBatchWaves; ++q) r = fmin(r, tmp[q]);
  wg_sync();
  return r;
}

template <class T>
__device__ void solve_chain(const BatchChain &c, BatchResult &res, double *Hs,
                                         double *sh) {
  Krylov k(Hs, sh);
  double *fl = k.fl;
  const long long t0 = wall_clock64();
  const int n = c.n, m = c.m;
  double *part2 = c.part + (size_t)(m + 2) * c.nblk;
  for (int i = threadIdx.x; i < n; i += kBatchThreads) c.x0[i] = c.xstart[i];
  wg_sync();
  b_product(c, 0, 0, 0.0);
  residual_check(c, 0, k.y, fl);
  int it = 0, restarts = 0, breakdowns = 0, status = BAMG_OK;
  bool conv = fl[0] != 0.0;
  double rel = fl[2];
  while (!conv && it < c.maxit) {
    b_product(c, 0, 0, 0.0);  // B x0
    for (int i = threadIdx.x; i < n; i += kBatchThreads) c.vcin[i] = -c.bx0[i];
    wg_sync();
    precondition<T>(c);  // z = C r0
    multi_dot(c, 0, true);
    finalize(c, 1, k.c1);
    if (threadIdx.x == 0) {
      const double beta = sqrt(k.c1[0]);
      for (int i = 0; i <= m; ++i) k.g[i] = 0.0;
      k.g[0] = beta;
      fl[3] = beta > 0.0 ? 1.0 / beta : 0.0;
    }
    wg_sync();
    {
      const double sc = fl[3];
      for (int i = threadIdx.x; i < n; i += kBatchThreads) c.V[i] = c.w[i] * sc;
    }
    wg_sync();
    int used = 0;
    bool broke = false;
    for (int j = 0;; ++j) {
      b_product(c, j == 0 ? 1 : 2, j, fl[3]);
      precondition<T>(c);  // w = C B v_j
      // Gram-Schmidt, twice
      multi_dot(c, j + 1, true);
      finalize(c, j + 2, k.c1);
      multi_axpy(c, j + 1, k.c1, nullptr);
      multi_dot(c, j + 1, false);
      finalize(c, j + 1, k.c2);
      multi_axpy(c, j + 1, k.c2, part2);
      arnoldi_step(c, k, j);
      residual_check(c, j + 1, k.y, fl);
      ++it;
      used = j + 1;
      rel = fl[2];
      if (!isfinite(rel)) {
        status = BAMG_E_NONFINITE;
        break;
      }
      if (fl[0] != 0.0) {
        conv = true;
        break;
      }
      if (fl[1] != 0.0) {
        broke = true;
        break;
      }
      if (!(j + 1 < m && it < c.maxit)) break;
    }
    // x0 += V y
    for (int i = threadIdx.x; i < n; i += kBatchThreads) {
      double xv = c.x0[i];
      for (int t = 0; t < used; ++t) xv += k.y[t] * c.V[(size_t)t * n + i];
      c.x0[i] = xv;
    }
    wg_sync();
    if (status != BAMG_OK) break;
    if (broke && !conv && ++breakdowns >= 2) {
      status = BAMG_E_BREAKDOWN;
      break;
    }
    if (!conv) ++restarts;
  }
  const double xmin = normalize_out(c, k.col);
  if (threadIdx.x == 0) {
    if (status == BAMG_OK && !conv) status = BAMG_NOT_CONVERGED;
    res.status = status;
    res.iterations = it;
    res.restarts = restarts;
    res.converged = conv ? 1 : 0;
    res.breakdowns = breakdowns;
    res.rel = rel;
    res.xmin = xmin;
    res.ticks = wall_clock64() - t0;
  }
  wg_sync();
}

// Persistent: workgroups take chains order[counter++] until none is left.
__global__ void __launch_bounds__(kBatchThreads)
    k_batch_solve(const BatchChain *__restrict__ chains, const int *__restrict__ order,
                  int nchains, int *__restrict__ counter, BatchResult *__restrict__ res) {
  __shared__ double Hs[(kBatchMaxRestart + 1) * kBatchMaxRestart];
  __shared__ double sh[8 * (kBatchMaxRestart + 2) + 8];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    // uniform across the workgroup: descriptor fields load into scalar registers
    const int q = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();  // every thread has read it before thread 0 takes the next
    if (q >= nchains) break;
    const int ci = __builtin_amdgcn_readfirstlane(order[q]);
    const BatchChain &c = chains[ci];
    if (c.prec == 0)
      solve_chain<double>(c, res[ci], Hs, sh);
    else
      solve_chain<float>(c, res[ci], Hs, sh);
  }
}

// ---------------------------------------------------------------- host side
namespace {

template <class T>
void describe_levels(bamg_handle *h, std::vector<BatchLevel> &out,
                     std::vector<std::vector<int>> &koffs) {
  for (int l = 0; l < h->L; ++l) {
    const Level &L = h->lv[l];
    BatchLevel d;
    d.n = L.n;
    d.xb = L.xb;
    d.bb = L.bb;
    d.rb = L.rb;
    d.tb = L.tb;
    if (l + 1 < h->L) {
      d.nc = h->lv[l + 1].n;
      d.lanes = L.lanes > 0 ? L.lanes : sweep_lanes_default(L.n, L.B.nnz);
      d.fused_w = h->opt.cycle == BAMG_CYCLE_V ? last_level_lanes<T>(h, l) : 0;
      d.brp = L.B.rp;
      d.bci = L.B.ci;
      d.bv = L.Bv;
      d.dinv = L.dinv;
      d.prp = L.P.rp;
      d.pci = L.P.ci;
      d.pv = L.Pv;
      d.plpr = transfer_lanes(L.P.nr, L.P.nnz);
      d.qrp = L.Pc.rp;
      d.qci = L.Pc.ci;
      d.qv = L.Qv;
      d.qlpr = transfer_lanes(L.Pc.nr, L.Pc.nnz);
      if (h->opt.smoother == BAMG_SMOOTH_KACZMARZ) {
        d.ncol = (int)L.offB.size() - 1;
        d.kord = L.ordB;
        d.rowinv = L.rowinvB;
        koffs.push_back(L.offB);  // device copy made by the caller
      }
    }
    out.push_back(d);
  }
}

}  // namespace

// Chains this launch can take: a V-cycle (or no preconditioner), restart
// length at most kBatchMaxRestart, and no learned iteration fallback.
bool batch_persistent_eligible(const bamg_handle *h, int restart) {
  if (!h || restart < 1 || restart > kBatchMaxRestart) return false;
  if (h->opt.cycle != BAMG_CYCLE_V && h->opt.cycle != BAMG_CYCLE_NONE) return false;
  if (h->opt.learned == BAMG_LEARNED_USE && h->opt.learned_max_iters > 0) return false;
  if (h->opt.flexible) return false;  // the launch runs the left-preconditioned GMRES only
  return h->L >= 1 && h->prof_kernel < 0 && !h->aux;  // no validation still running
}

void batch_persistent_solve(const std::vector<bamg_handle *> &hs, const std::vector<int> &order,
                            double *const *x, int restart, double tol, int maxit,
                            bamg_solve_info *infos, bamg_status *st, hipStream_t s,
                            const std::function<void()> &meanwhile) {
  const int nc = (int)hs.size();
  if (nc == 0) {
    if (meanwhile) meanwhile();
    return;
  }
  std::vector<BatchChain> ch(nc);
  std::vector<BatchLevel> lv;
  std::vector<size_t> lv_at(nc);
  std::vector<std::vector<int>> koffs;
  std::vector<std::pair<size_t, size_t>> koff_at;  // (level index, koffs index)
  for (int i = 0; i < nc; ++i) {
    bamg_handle *h = hs[i];
    hipStream_t keep = h->pool.s;
    h->pool.s = s;  // a caller's allocator orders its allocations on s
    try {
      gmres_buffers(h, restart);
    } catch (...) {
      h->pool.s = keep;
      throw;
    }
    h->pool.s = keep;
    lv_at[i] = lv.size();
    const size_t k0 = koffs.size();
    if (h->prec == 0)
      describe_levels<double>(h, lv, koffs);
    else
      describe_levels<float>(h, lv, koffs);
    for (size_t k = k0, l = lv_at[i]; k < koffs.size(); ++k, ++l) koff_at.push_back({l, k});
    BatchChain &c = ch[i];
    const Level &L0 = h->lv[0];
    c.L = h->L;
    c.n = L0.n;
    c.prec = h->prec;
    c.smoother = h->opt.smoother;
    c.cycle = h->opt.cycle;
    c.nu1 = h->opt.nu_pre;
    c.nu2 = h->opt.nu_post;
    c.m = restart;
    c.maxit = maxit;
    c.nblk = gmres_blocks(L0.n);
    c.lanes0 = L0.lanes > 0 ? L0.lanes : sweep_lanes_default(L0.n, L0.B.nnz);
    c.nL = h->lv[h->L - 1].n;
    c.tol = tol;
    c.omega = h->opt.omega;
    c.rp = L0.B.rp;
    c.ci = L0.B.ci;
    c.b64 = h->B64;
    c.bdag = h->bdag;
    c.xstart = h->x0;
    c.xout = x[i];
    c.V = h->gV;
    c.BV = h->gBV;
    c.w = h->gw;
    c.x0 = h->gx0;
    c.bx0 = h->gbx0;
    c.vcin = h->vcin;
    c.part = h->gsc;
    c.vb = (float *)h->vb;
    c.vx = (float *)h->vx;
  }
  // one device block: chains, levels, colour offsets, order, counter, results
  size_t nko = 0;
  for (auto &k : koffs) nko += k.size();
  const size_t bytes_ch = sizeof(BatchChain) * nc, bytes_lv = sizeof(BatchLevel) * lv.size();
  const size_t off_lv = (bytes_ch + 255) & ~size_t(255);
  const size_t off_ko = (off_lv + bytes_lv + 255) & ~size_t(255);
  const size_t off_or = (off_ko + sizeof(int) * nko + 255) & ~size_t(255);
  const size_t off_ct = (off_or + sizeof(int) * nc + 255) & ~size_t(255);
  const size_t off_rs = off_ct + 256;
  const size_t total = off_rs + sizeof(BatchResult) * nc;
  unsigned char *dev = nullptr;
  HIPCHK(hipMalloc((void **)&dev, total));
  struct Free {
    unsigned char *p;
    ~Free() { (void)hipFree(p); }
  } guard{dev};
  // device addresses inside the descriptors
  std::vector<int> kflat;
  kflat.reserve(nko);
  std::vector<size_t> kpos(koffs.size());
  for (size_t k = 0; k < koffs.size(); ++k) {
    kpos[k] = kflat.size();
    kflat.insert(kflat.end(), koffs[k].begin(), koffs[k].end());
  }
  for (auto &[l, k] : koff_at) lv[l].koff = (const int *)(dev + off_ko) + kpos[k];
  for (int i = 0; i < nc; ++i) ch[i].lv = (const BatchLevel *)(dev + off_lv) + lv_at[i];
  std::vector<unsigned char> host(off_rs, 0);
  std::memcpy(host.data(), ch.data(), bytes_ch);
  std::memcpy(host.data() + off_lv, lv.data(), bytes_lv);
  if (nko) std::memcpy(host.data() + off_ko, kflat.data(), sizeof(int) * nko);
  std::memcpy(host.data() + off_or, order.data(), sizeof(int) * nc);
  // host buffer must outlive the copy: synchronous copy (pageable memory)
  HIPCHK(hipMemcpyAsync(dev, host.data(), off_rs, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  int dev_id = 0, cus = 0, per_cu = 0;
  HIPCHK(hipGetDevice(&dev_id));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id));
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_batch_solve,
                                                      kBatchThreads, 0));
  const int grid = std::max(1, std::min(nc, std::max(1, per_cu) * cus));
  k_batch_solve<<<grid, kBatchThreads, 0, s>>>((const BatchChain *)dev,
                                                (const int *)(dev + off_or), nc,
                                                (int *)(dev + off_ct),
                                                (BatchResult *)(dev + off_rs));
  LAUNCHCHK();
  if (meanwhile) meanwhile();  // host work while the launch runs
  std::vector<BatchResult> res(nc);
  HIPCHK(hipMemcpyAsync(res.data(), dev + off_rs, sizeof(BatchResult) * nc,
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int khz = 0;
  HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev_id));
  for (int i = 0; i < nc; ++i) {
    const BatchResult &r = res[i];
    bamg_solve_info &inf = infos[i];
    inf = bamg_solve_info{};
    inf.iterations = r.iterations;
    inf.restarts = r.restarts;
    inf.converged = r.converged;
    inf.breakdowns = r.breakdowns;
    inf.rel_residual = r.rel;
    inf.x_min = r.xmin;
    inf.t_solve_ms = khz > 0 ? (double)r.ticks / khz : 0.0;
    inf.setup_cycles = hs[i]->opt.setup_cycles;
    inf.t_setup_ms = hs[i]->t_setup_ms;
    st[i] = (bamg_status)r.status;
  }
}

}  // namespace bamg
