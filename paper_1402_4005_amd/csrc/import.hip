// bamg_setup_from_levels: a handle whose hierarchy is given operator by
// operator instead of built by the bootstrap setup. The V-cycle of Section
// 3 (eq. coarse_grid_correction) needs only B_l, the transfers P_l and Q_l,
// the smoother's diagonal and the coarsest pseudo-inverse, and GMRES on the
// residual equation (Section 6) needs B_0 and x0 besides; those are copied
// in as given. The kernels that run on such a handle are the ones that run
// after bamg_setup, with the same launch choices, so a hierarchy built
// elsewhere (a checkpoint, another implementation) is solved by the same
// code on exactly its operators.
#include <cmath>
#include <string>

#include "bamg_internal.h"

namespace bamg {

namespace {

// host checks of one CSR: sizes, row pointers, column range and order
void check_csr(const bamg_host_csr &A, int64_t nr, int64_t nc, const char *what, int l) {
  const std::string tag = std::string(what) + " of level " + std::to_string(l);
  if (A.nrows != nr || A.ncols != nc || A.nnz < 1 || A.nnz > 0x7fffffffLL || !A.row_ptr ||
      !A.col_idx || !A.val)
    fail(BAMG_E_ARG, tag + ": wrong shape or missing array");
  if (A.row_ptr[0] != 0 || A.row_ptr[nr] != A.nnz) fail(BAMG_E_ARG, tag + ": row_ptr ends");
  for (int64_t i = 0; i < nr; ++i) {
    const int a = A.row_ptr[i], b = A.row_ptr[i + 1];
    if (b < a) fail(BAMG_E_ARG, tag + ": row_ptr decreases");
    for (int k = a; k < b; ++k) {
      const int c = A.col_idx[k];
      if (c < 0 || c >= nc || (k > a && c <= A.col_idx[k - 1]))
        fail(BAMG_E_ARG, tag + ": column out of range or not ascending");
      if (!std::isfinite(A.val[k])) fail(BAMG_E_NONFINITE, tag + ": non-finite value");
    }
  }
}

// device copy of a host CSR; values converted to T (via an FP64 staging
// buffer that *v64 receives when asked for)
template <class T>
void upload(Pool &pool, const bamg_host_csr &A, Csr &C, void *&val, double **v64, hipStream_t s) {
  C.nr = (int)A.nrows;
  C.nc = (int)A.ncols;
  C.nnz = (int)A.nnz;
  C.rp = pool.get<int>((size_t)C.nr + 1);
  C.ci = pool.get<int>(C.nnz);
  HIPCHK(hipMemcpyAsync(C.rp, A.row_ptr, sizeof(int) * (C.nr + 1), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(C.ci, A.col_idx, sizeof(int) * C.nnz, hipMemcpyHostToDevice, s));
  double *d64 = pool.get<double>(C.nnz);
  HIPCHK(hipMemcpyAsync(d64, A.val, sizeof(double) * C.nnz, hipMemcpyHostToDevice, s));
  if (sizeof(T) == sizeof(double)) {
    val = d64;
  } else {
    val = pool.get<T>(C.nnz);
    convert<double, T>((T *)val, d64, C.nnz, s);
  }
  if (v64) *v64 = d64;
}

}  // namespace

template <class T>
void import_all(bamg_handle *h, int nlev, const bamg_level_ops *ops, const double *pinv,
                const double *x0) {
  Pool &pool = h->pool;
  hipStream_t s = pool.s;
  const bamg_options &o = h->opt;
  // ---- host checks of every operator before any device work
  for (int l = 0; l < nlev; ++l) {
    const int64_t n = ops[l].B.nrows;
    if (n < 1 || n > 0x7fffffffLL) fail(BAMG_E_ARG, "level size out of range");
    check_csr(ops[l].B, n, n, "B", l);
    if (l + 1 < nlev) {
      const int64_t nc = ops[l + 1].B.nrows;
      if (nc < 1 || nc >= n) fail(BAMG_E_ARG, "a coarse level must be smaller than its fine level");
      check_csr(ops[l].P, n, nc, "P", l);
      check_csr(ops[l].Q, nc, n, "Q", l);
    }
  }
  const int nL = (int)ops[nlev - 1].B.nrows;
  if (nL > 2048) fail(BAMG_E_ARG, "coarsest level above 2048 states");
  for (size_t i = 0; i < (size_t)nL * nL; ++i)
    if (!std::isfinite(pinv[i])) fail(BAMG_E_NONFINITE, "non-finite coarsest pseudo-inverse");
  // ---- device copies
  h->lv.assign(nlev, Level());
  int *flag = pool.get<int>(4);
  for (int l = 0; l < nlev; ++l) {
    Level &L = h->lv[l];
    L.n = (int)ops[l].B.nrows;
    double *b64 = nullptr;
    upload<T>(pool, ops[l].B, L.B, L.Bv, &b64, s);
    if (l == 0) h->B64 = b64;
    L.dpos = pool.get<int>(L.n);
    diag_positions(L.B, L.dpos, s);
    L.dinv = pool.get<T>(L.n);
    dinv_from_diag<T>(L, (const T *)L.Bv, (T *)L.dinv, flag, true, s);
    L.xb = pool.get<T>(L.n);
    L.bb = pool.get<T>(L.n);
    L.rb = pool.get<T>(L.n);
    L.tb = pool.get<T>(L.n);
    if (l + 1 < nlev) {
      L.nc = (int)ops[l + 1].B.nrows;
      upload<T>(pool, ops[l].P, L.P, L.Pv, nullptr, s);
      upload<T>(pool, ops[l].Q, L.Pc, L.Qv, nullptr, s);
      if (o.smoother == BAMG_SMOOTH_KACZMARZ) {
        transpose_pattern(pool, L.B, L.Bt, L.btperm, s);
        L.colB = pool.get<int>(L.n);
        row_colouring(pool, L.B, L.Bt, L.colB, L.ncolB, L.ordB, L.offB, s);
        L.rowinvB = pool.get<T>(L.n);
        row_inv_norms<T>(L.B, (const T *)L.Bv, (T *)L.rowinvB, s);
      }
    }
  }
  h->L = nlev;
  h->bdag = pool.get<double>((size_t)nL * nL);
  HIPCHK(hipMemcpyAsync(h->bdag, pinv, sizeof(double) * nL * nL, hipMemcpyHostToDevice, s));
  const int n = h->lv[0].n;
  h->x0 = pool.get<double>(n);
  HIPCHK(hipMemcpyAsync(h->x0, x0, sizeof(double) * n, hipMemcpyHostToDevice, s));
  h->sigma = pool.get<double>(64);
  fill<double>(h->sigma, 0.0, 64, s);
  if (h->prec != 0) {
    h->vb = pool.get<float>(n);
    h->vx = pool.get<float>(n);
  }
  for (int l = 0; l + 1 < h->L; ++l) {
    if (o.autotune)
      tune_sweeps<T>(pool, h->lv[l], s);
    else
      h->lv[l].lanes = sweep_lanes_default(h->lv[l].n, h->lv[l].B.nnz);
  }
  // the host arrays are the caller's: every copy ends before the return
  HIPCHK(hipStreamSynchronize(s));
  pool.flush();
}

template void import_all<double>(bamg_handle *, int, const bamg_level_ops *, const double *,
                                 const double *);
template void import_all<float>(bamg_handle *, int, const bamg_level_ops *, const double *,
                                const double *);

}  // namespace bamg
