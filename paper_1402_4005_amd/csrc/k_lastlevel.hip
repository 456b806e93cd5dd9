// The V-cycle on the last smoothed level and the coarsest solve (Section 3;
// pseudo-inverse of Section 6) in one workgroup, when that level is small.
//
// On such a level every step of the cycle is a kernel whose time is set by
// its launch and a few dependent memory round trips. When the level's
// operator, transfers, pseudo-inverse and vectors fit in one workgroup's LDS
// and one pass of the workgroup covers its rows, a single launch loads
// them once and runs every step with workgroup barriers only: the
// pre-smoothing sweeps from zero, the residual, the restriction, the dense
// coarsest solve, the prolongation and the post-smoothing sweeps.
//
// Rows are handled by groups of W lanes (W a power of two, at most 16)
// that stride over the row's entries and reduce with cross-lane shuffles;
// the arithmetic is that of the one-kernel-per-step cycle up to the order
// of the partial sums.
#include <algorithm>

#include "bamg_internal.h"
#include "device_common.h"

namespace bamg {

namespace {

constexpr int kLastThreads = 1024;

template <class T>
struct LastLevel {
  int n, nnz, nnzp, nc, nnzq, w;
  const int *rp, *ci, *prp, *pci, *qrp, *qci;
  const T *val, *pv, *qv, *dinv;
  const double *bdag;  // nc x nc, row-major
  T omega;
  int nu1, nu2;
};

// bytes of LDS the level needs (T arrays first, 8-byte aligned, then ints)
template <class T>
size_t last_level_lds(int n, int nnz, int nnzp, int nc, int nnzq) {
  const size_t t = (size_t)nnz + nnzp + nnzq + 5 * (size_t)n + 2 * (size_t)nc;
  const size_t d = (size_t)nc * nc;
  const size_t i = (size_t)(n + 1) + nnz + (n + 1) + nnzp + (nc + 1) + nnzq;
  return sizeof(double) * d + sizeof(T) * t + sizeof(int) * i;
}

template <class T>
__global__ void __launch_bounds__(kLastThreads)
    k_vcycle_last(const LastLevel<T> a, const T *__restrict__ bg, T *__restrict__ xg) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  double *bd = reinterpret_cast<double *>(smem);
  T *val = reinterpret_cast<T *>(bd + (size_t)a.nc * a.nc);
  T *pv = val + a.nnz, *qv = pv + a.nnzp, *dinv = qv + a.nnzq;
  T *x = dinv + a.n, *y = x + a.n, *b = y + a.n, *r = b + a.n, *bc = r + a.n, *xc = bc + a.nc;
  int *rp = reinterpret_cast<int *>(xc + a.nc);
  int *ci = rp + a.n + 1, *prp = ci + a.nnz, *pci = prp + a.n + 1, *qrp = pci + a.nnzp;
  int *qci = qrp + a.nc + 1;
  const int t = threadIdx.x, nt = blockDim.x;
  const int n = a.n, nc = a.nc, W = a.w;
  for (int e = t; e < a.nnz; e += nt) {
    ci[e] = a.ci[e];
    val[e] = a.val[e];
  }
  for (int e = t; e <= n; e += nt) {
    rp[e] = a.rp[e];
    prp[e] = a.prp[e];
  }
  for (int e = t; e < a.nnzp; e += nt) {
    pci[e] = a.pci[e];
    pv[e] = a.pv[e];
  }
  for (int e = t; e <= nc; e += nt) qrp[e] = a.qrp[e];
  for (int e = t; e < a.nnzq; e += nt) {
    qci[e] = a.qci[e];
    qv[e] = a.qv[e];
  }
  for (int e = t; e < nc * nc; e += nt) bd[e] = a.bdag[e];
  for (int e = t; e < n; e += nt) {
    dinv[e] = a.dinv[e];
    b[e] = bg[e];
  }
  __syncthreads();
  const int grp = t / W, lane = t % W, ngrp = nt / W;
  // out[i] = f(i, sum over row i of the entries of (rows, cols, vals) times v)
  auto rows_dot = [&](int nrows, const int *rr, const int *cc, const T *vv, const T *v,
                      auto &&f) {
    // every lane of a group runs the same trip count, so the shuffles are uniform
    for (int i0 = 0; i0 < nrows; i0 += ngrp) {
      const int i = i0 + grp;
      T s = 0;
      if (i < nrows)
        for (int k = rr[i] + lane; k < rr[i + 1]; k += W) s += vv[k] * v[cc[k]];
      s = group_sum(s, W);
      if (i < nrows && lane == 0) f(i, s);
    }
  };
  const T om = a.omega;
  auto sweep = [&](const T *xi, T *xo) {
    rows_dot(n, rp, ci, val, xi, [&](int i, T s) { xo[i] = xi[i] + om * dinv[i] * (b[i] - s); });
  };
  // pre-smoothing from zero
  T *cur = x, *oth = y;
  for (int i = t; i < n; i += nt) x[i] = a.nu1 > 0 ? om * dinv[i] * b[i] : (T)0;
  __syncthreads();
  for (int it = 1; it < a.nu1; ++it) {
    sweep(cur, oth);
    __syncthreads();
    T *tmp = cur;
    cur = oth;
    oth = tmp;
  }
  // r = b - B x, bc = Q r
  rows_dot(n, rp, ci, val, cur, [&](int i, T s) { r[i] = b[i] - s; });
  __syncthreads();
  rows_dot(nc, qrp, qci, qv, r, [&](int j, T s) { bc[j] = s; });
  __syncthreads();
  // xc = Bdag bc, FP64
  for (int j0 = 0; j0 < nc; j0 += ngrp) {
    const int j = j0 + grp;
    double s = 0.0;
    if (j < nc)
      for (int q = lane; q < nc; q += W) s += bd[(size_t)j * nc + q] * (double)bc[q];
    s = group_sum(s, W);
    if (j < nc && lane == 0) xc[j] = (T)s;
  }
  __syncthreads();
  // x += P xc
  rows_dot(n, prp, pci, pv, xc, [&](int i, T s) { cur[i] += s; });
  __syncthreads();
  for (int it = 0; it < a.nu2; ++it) {
    sweep(cur, oth);
    __syncthreads();
    T *tmp = cur;
    cur = oth;
    oth = tmp;
  }
  for (int i = t; i < n; i += nt) xg[i] = cur[i];
}

}  // namespace

// Lanes per row of the fused last level for level l (the one above the
// coarsest), or 0 when level l's V-cycle does not take that form.
template <class T>
int last_level_lanes(const bamg_handle *h, int l) {
  if (!h->last_fused || l != h->L - 2 || l < 1 || h->opt.smoother != BAMG_SMOOTH_JACOBI)
    return 0;
  const Level &L = h->lv[l], &C = h->lv[l + 1];
  // lanes per row: the largest power of two up to 16 with one pass over the rows
  int w = 16;
  while (w > 1 && (long)L.n * w > kLastThreads) w >>= 1;
  if ((long)L.n * w > kLastThreads || C.n > kLastThreads) return 0;
  static const int maxlds = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 65536;
    return v;
  }();
  const size_t shm = last_level_lds<T>(L.n, L.B.nnz, L.P.nnz, C.n, L.Pc.nnz);
  return shm + 64 > (size_t)maxlds ? 0 : w;
}

// Launches the fused last level for level l (the one above the coarsest) if
// it fits; returns false (nothing launched) otherwise.
template <class T>
bool vcycle_last_level(bamg_handle *h, int l, const T *b, T *x, hipStream_t s) {
  const int w = last_level_lanes<T>(h, l);
  if (w == 0) return false;
  const Level &L = h->lv[l], &C = h->lv[l + 1];
  const size_t shm = last_level_lds<T>(L.n, L.B.nnz, L.P.nnz, C.n, L.Pc.nnz);
  LastLevel<T> a{};
  a.n = L.n;
  a.nnz = L.B.nnz;
  a.nnzp = L.P.nnz;
  a.nc = C.n;
  a.nnzq = L.Pc.nnz;
  a.w = w;
  a.rp = L.B.rp;
  a.ci = L.B.ci;
  a.val = (const T *)L.Bv;
  a.dinv = (const T *)L.dinv;
  a.prp = L.P.rp;
  a.pci = L.P.ci;
  a.pv = (const T *)L.Pv;
  a.qrp = L.Pc.rp;
  a.qci = L.Pc.ci;
  a.qv = (const T *)L.Qv;
  a.bdag = h->bdag;
  a.omega = (T)h->opt.omega;
  a.nu1 = h->opt.nu_pre;
  a.nu2 = h->opt.nu_post;
  HIPCHK(hipFuncSetAttribute((const void *)k_vcycle_last<T>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  k_vcycle_last<T><<<1, kLastThreads, shm, s>>>(a, b, x);
  LAUNCHCHK();
  return true;
}

template int last_level_lanes<double>(const bamg_handle *, int);
template int last_level_lanes<float>(const bamg_handle *, int);
template bool vcycle_last_level<double>(bamg_handle *, int, const double *, double *,
                                        hipStream_t);
template bool vcycle_last_level<float>(bamg_handle *, int, const float *, float *, hipStream_t);

}  // namespace bamg
