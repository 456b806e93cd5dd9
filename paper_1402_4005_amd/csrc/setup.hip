// Host orchestration of bamg_setup: validation and B = I - A (Section 2),
// the integer structure of the hierarchy, the bootstrap cycles (Algorithm 1
// with the Markov-chain constraint of Section 5), the coarsest
// pseudo-inverse and x0 (Section 6). Every numeric step is a kernel launch on
// the handle's stream; the host only reads back sizes and status flags.
#include <algorithm>
#include <cmath>

#include "bamg_internal.h"
#include "device_common.h"

namespace bamg {

namespace {

template <class T>
struct Setup {
  bamg_handle *h;
  hipStream_t s;
  int r;
  // reduction scratch
  double *part = nullptr, *prod = nullptr, *wv = nullptr, *wu = nullptr, *scales = nullptr;
  int nblk = 0;
  int *flag = nullptr;
  // coarsest dense work
  int nL = 0;
  double *Bd = nullptr, *Md = nullptr, *Nd = nullptr, *X = nullptr, *W = nullptr, *J = nullptr;
  double *sv = nullptr, *work = nullptr;
  double *W2 = nullptr, *J2 = nullptr, *sv2 = nullptr;  // SVD of B_L for the pseudo-inverse
  bool pinv_done = false;

  Pool &pool() { return h->pool; }

  void swap_uv(Level &L) {
    std::swap(L.U, L.U2);
    std::swap(L.V, L.V2);
  }

  void products(Level &L, int which, int epi = 0, double *aux = nullptr) {
    const int nb = pair_products<T>(L, r, (const T *)L.U, (const T *)L.V, which, part, nblk, s);
    finalize_products(part, nb, r, which, epi, prod, aux, s);
  }

  // nu_setup smoothing steps of Algorithm 1 on the test-vector pairs
  void relax(Level &L, int with_rhs) {
    const T om = (T)h->opt.omega;
    for (int it = 0; it < h->opt.nu_setup; ++it) {
      if (h->opt.smoother == BAMG_SMOOTH_KACZMARZ) {
        relax_kaczmarz(L, with_rhs);
      } else {
        relax_pairs<T>(L, r, om, with_rhs, h->sigma, (const T *)L.U, (const T *)L.V, (T *)L.U2,
                       (T *)L.V2, s);
        swap_uv(L);
      }
      if (with_rhs) products(L, 1, 1, h->sigma);
    }
  }

  // Kaczmarz variant: right-hand sides sigma M u / sigma N v are formed from
  // the old vectors (kept in U2/V2 as copies), then each column is swept in
  // colour order in place.
  void relax_kaczmarz(Level &L, int with_rhs) {
    const size_t nr = (size_t)L.n * r;
    T *rhsV = (T *)L.U2, *rhsU = (T *)L.V2;  // scratch: n x r each
    if (with_rhs) {
      const void *mv = L.Mv, *nv = L.Nv;
      spmm<T>(L.M, (const T *)mv, r, (const T *)L.U, rhsV, 0, s);
      spmm<T>(L.M, (const T *)nv, r, (const T *)L.V, rhsU, 0, s);
      scale_columns<T>(rhsV, L.n, r, h->sigma, 0, s);
      scale_columns<T>(rhsU, L.n, r, h->sigma, 0, s);
    } else {
      fill<T>(rhsV, (T)0, nr, s);
      fill<T>(rhsU, (T)0, nr, s);
    }
    kaczmarz_block(L, rhsV, (T *)L.V, false, 0);
    kaczmarz_block(L, rhsU, (T *)L.U, true, 1);
  }

  // sweep every column of X (n x r, row-major) in place on B_l or B_l^T
  void kaczmarz_block(Level &L, const T *rhs, T *X, bool transpose, int k0) {
    T *x = (T *)L.tb, *b = (T *)L.rb;
    for (int k = k0; k < r; ++k) {
      column_get(X, L.n, r, k, x);
      column_get(rhs, L.n, r, k, b);
      const Csr &A = transpose ? L.Bt : L.B;
      const T *val = (const T *)(transpose ? L.Btv : L.Bv);
      const T *ri = (const T *)(transpose ? L.rowinvBt : L.rowinvB);
      const int *ord = transpose ? L.ordBt : L.ordB;
      const std::vector<int> &off = transpose ? L.offBt : L.offB;
      for (size_t c = 0; c + 1 < off.size(); ++c)
        kaczmarz_colour<T>(A, val, ri, ord + off[c], off[c + 1] - off[c], b, x, s);
      column_set(X, L.n, r, k, x);
    }
  }

  void column_get(const T *X, int n, int r_, int k, T *out);
  void column_set(T *X, int n, int r_, int k, const T *in);

  void normalize(Level &L) {
    products(L, 1, 2, scales);
    scale_columns<T>((T *)L.V, L.n, r, scales, 0, s);
    scale_columns<T>((T *)L.U, L.n, r, scales + 16, 1, s);
  }

  void weights(Level &L) {
    products(L, 2);
    ls_weights(prod, r, wv, wu, s);
  }

  void galerkin(int l) {
    Level &L = h->lv[l];
    Level &C = h->lv[l + 1];
    copy_permuted<T>((T *)L.Ptv, (const T *)L.Pv, L.pcperm, L.P.nnz, s);
    copy_permuted<T>((T *)L.Qv, (const T *)L.Qtv, L.pcperm, L.P.nnz, s);
    int *sc = pool().template get<int>((size_t)L.n + 1);  // long-row lists (n >= nc)
    spgemm_numeric<T>(L.B, (const T *)L.Bv, L.P, (const T *)L.Pv, L.T1, (T *)L.T1v, sc, s);
    spgemm_numeric<T>(L.Pc, (const T *)L.Qv, L.T1, (const T *)L.T1v, C.B, (T *)C.Bv, sc, s);
    spgemm_numeric<T>(L.M, (const T *)L.Mv, L.P, (const T *)L.Qtv, L.T2, (T *)L.T2v, sc, s);
    spgemm_numeric<T>(L.Pc, (const T *)L.Qv, L.T2, (const T *)L.T2v, C.M, (T *)C.Mv, sc, s);
    spgemm_numeric<T>(L.M, (const T *)L.Nv, L.P, (const T *)L.Pv, L.T2, (T *)L.T3v, sc, s);
    spgemm_numeric<T>(L.Pc, (const T *)L.Ptv, L.T2, (const T *)L.T3v, C.M, (T *)C.Nv, sc, s);
    pool().release(sc);
    copy_permuted<T>((T *)C.Btv, (const T *)C.Bv, C.btperm, C.B.nnz, s);
    dinv_from_diag<T>(C, (const T *)C.Bv, (T *)C.dinv, flag + 3, false, s);
    // Kaczmarz row norms exist only where the smoother runs (not on the
    // coarsest level, which is solved directly)
    if (h->opt.smoother == BAMG_SMOOTH_KACZMARZ && l + 1 < h->L - 1) {
      row_inv_norms<T>(C.B, (const T *)C.Bv, (T *)C.rowinvB, s);
      row_inv_norms<T>(C.Bt, (const T *)C.Btv, (T *)C.rowinvBt, s);
    }
  }

  // Learned interpolation (cycle 1): the exact LS row plus the MLP's
  // correction replaces the exact row where its LS objective is within twice
  // the optimum; in record mode the features are kept for bamg_harvest.
  void learned_rows(Level &L) {
    level_fpoints(h, L, s);
    if (L.nF <= 0) return;
    const size_t nf = (size_t)L.nF;
    if (h->opt.learned == BAMG_LEARNED_RECORD) {
      if (!L.feat) L.feat = pool().template get<float>(nf * BAMG_MLP_IN);
      mlp_features<T>(L, r, (const T *)L.V, wv, (const T *)L.Pv, L.feat, s);
      return;
    }
    // features, network and objective test of every F row in one launch
    mlp_apply<T>(L, r, (const T *)L.V, wv, h->opt.mlp, (T *)L.Pv, h->lcount, s);
  }

  // Algorithm 1 (bamg_mle) from level l: smoothing, then mu passes of the
  // inner loop (fits, Galerkin products, injection, recursion,
  // interpolation back, smoothing with the sigma right-hand sides)
  void mle(int l, int cycle) {
    if (l == h->L - 1) {
      coarsest(cycle == h->opt.setup_cycles);
      return;
    }
    relax(h->lv[l], cycle > 1);
    for (int pass = 0; pass < h->opt.mu; ++pass) {
      Level &L = h->lv[l];
      normalize(L);
      weights(L);
      ls_fit<T>(L, r, h->opt.max_interp, (const T *)L.U, (const T *)L.V, wv, wu,
                h->opt.interp_rule, h->opt.restriction, (T *)L.Pv, (T *)L.Qtv, s);
      if (h->opt.learned != BAMG_LEARNED_OFF && cycle == 1 && pass == 0) learned_rows(L);
      galerkin(l);
      Level &C = h->lv[l + 1];
      inject<T>(L.cpts, C.n, r, (const T *)L.U, (T *)C.U, s);
      inject<T>(L.cpts, C.n, r, (const T *)L.V, (T *)C.V, s);
      mle(l + 1, cycle);
      Level &L2 = h->lv[l];
      Level &C2 = h->lv[l + 1];
      spmm<T>(L2.P, (const T *)L2.Qtv, r, (const T *)C2.U, (T *)L2.U, 1, s);
      spmm<T>(L2.P, (const T *)L2.Pv, r, (const T *)C2.V, (T *)L2.V, 0, s);
      relax(L2, 1);
    }
  }

  void alloc_dense(int n) {
    nL = n;
    const size_t nn = (size_t)n * n;
    Bd = pool().template get<double>(nn);
    Md = pool().template get<double>(nn);
    Nd = pool().template get<double>(nn);
    X = pool().template get<double>(nn);
    W = pool().template get<double>(nn);
    J = pool().template get<double>(nn);
    sv = pool().template get<double>(n);
    work = pool().template get<double>(n + 64);
    if (n > coarse_small_max()) {
      W2 = pool().template get<double>(nn);
      J2 = pool().template get<double>(nn);
      sv2 = pool().template get<double>(n);
    }
  }

  // the deferred levels of the strong-connectivity search go beside the
  // SVD rounds, which leave most CUs and most of the memory bandwidth free
  static void search_hook(void *p) { static_cast<bamg_handle *>(p)->search_more(); }

  // r smallest generalized singular triplets on the coarsest level. In the
  // last setup cycle B_L is final, so its pseudo-inverse (the coarse solve
  // of the V-cycle) is computed in the same launches.
  void coarsest(bool last) {
    // every coarse diagonal of this cycle exists now: report a bad one
    // before anything the coarsest solve might say about it
    if (read_int(flag + 3, s)) fail(BAMG_E_BAD_DIAG, "zero or non-finite diagonal in some B_l");
    Level &C = h->lv[h->L - 1];
    const int n = C.n;
    csr_to_dense(C.B, C.Bv, h->prec, Bd, s);
    if (h->prec) zero_colsums(Bd, n, s);
    csr_to_dense(C.M, C.Mv, h->prec, Md, s);
    csr_to_dense(C.M, C.Nv, h->prec, Nd, s);
    if (last && !h->bdag) h->bdag = pool().template get<double>((size_t)n * n);
    if (n <= coarse_small_max()) {
      const int st = coarse_small(last ? 2 : 0, n, r, Bd, Md, Nd, C.U, C.V, h->prec, h->sigma,
                                  last ? h->bdag : nullptr, flag, s);
      if (st != BAMG_OK)
        fail(BAMG_E_COARSE,
             last ? "coarsest generalized SVD failed or coarsest operator not of rank n_L - 1"
                  : "coarsest generalized SVD failed (M_L, N_L not SPD or no convergence)");
      pinv_done = last;
      return;
    }
    if (last) transpose_dense(Bd, W2, n, s);  // B_L column-major, for its own SVD
    if (cholesky2(Md, Nd, n, flag, s) != BAMG_OK)
      fail(BAMG_E_COARSE, "coarsest M_L or N_L not positive definite");
    HIPCHK(hipMemcpyAsync(X, Bd, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToDevice, s));
    trsm_lower_cols(Md, X, n, n, n, s);  // X = L_M^-1 B
    transpose_dense(X, W, n, s);
    trsm_lower_cols(Nd, W, n, n, n, s);  // W = L_N^-1 X^T, i.e. Bt column-major
    bamg_handle *prof = h->prof_kernel == BAMG_PROFILE_COARSEST_SVD ? h : nullptr;
    if (jacobi_svd2(pool(), W, J, last ? W2 : nullptr, last ? J2 : nullptr, n, s, prof,
                    &search_hook, h) != BAMG_OK)
      fail(BAMG_E_COARSE, "Jacobi SVD did not converge");
    column_norms(W, n, sv, s);
    coarse_triplets_out(Md, Nd, W, J, sv, n, r, C.U, C.V, h->prec, h->sigma, work, s);
    if (last) {
      column_norms(W2, n, sv2, s);
      if (build_pinv(pool(), W2, J2, sv2, n, h->bdag, s) != BAMG_OK)
        fail(BAMG_E_COARSE, "coarsest operator is not of rank n_L - 1");
      pinv_done = true;
    }
  }

  void pinv() {
    if (pinv_done) return;
    Level &C = h->lv[h->L - 1];
    const int n = C.n;
    csr_to_dense(C.B, C.Bv, h->prec, Bd, s);
    if (h->prec) zero_colsums(Bd, n, s);
    if (!h->bdag) h->bdag = pool().template get<double>((size_t)n * n);
    if (n <= coarse_small_max()) {
      if (coarse_small(1, n, r, Bd, nullptr, nullptr, nullptr, nullptr, h->prec, nullptr, h->bdag,
                       flag, s) != BAMG_OK)
        fail(BAMG_E_COARSE, "coarsest operator is not of rank n_L - 1");
      return;
    }
    transpose_dense(Bd, W, n, s);  // W = B_L column-major
    if (jacobi_svd(pool(), W, J, n, s) != BAMG_OK) fail(BAMG_E_COARSE, "Jacobi SVD did not converge");
    column_norms(W, n, sv, s);
    if (build_pinv(pool(), W, J, sv, n, h->bdag, s) != BAMG_OK)
      fail(BAMG_E_COARSE, "coarsest operator is not of rank n_L - 1");
  }
};

template <class T>
__global__ void k_col_get(const T *__restrict__ X, int n, int r, int k, T *__restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = X[(size_t)i * r + k];
}
template <class T>
__global__ void k_col_set(T *__restrict__ X, int n, int r, int k, const T *__restrict__ in) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) X[(size_t)i * r + k] = in[i];
}
template <class T>
void Setup<T>::column_get(const T *Xm, int n, int r_, int k, T *out) {
  k_col_get<T><<<ceil_div(n, 256), 256, 0, s>>>(Xm, n, r_, k, out);
  LAUNCHCHK();
}
template <class T>
void Setup<T>::column_set(T *Xm, int n, int r_, int k, const T *in) {
  k_col_set<T><<<ceil_div(n, 256), 256, 0, s>>>(Xm, n, r_, k, in);
  LAUNCHCHK();
}

// x0 = column kx of V on level 0, in FP64
template <class T>
__global__ void k_extract_col(const T *__restrict__ V, int n, int r, int k,
                              double *__restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)V[(size_t)i * r + k];
}

__global__ void k_identity_csr(int n, int *__restrict__ rp, int *__restrict__ ci) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    ci[i] = i;
    rp[i + 1] = i + 1;
  }
  if (i == 0) rp[0] = 0;
}

}  // namespace

template <class T>
void setup_all(bamg_handle *h, const bamg_csr *A, const bamg_geometry *geom) {
  const bamg_options &o = h->opt;
  Pool &pool = h->pool;
  hipStream_t s = pool.s;
  const int n = (int)A->n, nnz = (int)A->nnz, r = o.r;
  // ---- input on the device
  const int *arp = A->row_ptr, *aci = A->col_idx;
  const double *aval = A->val;
  if (!A->on_device) {
    int *drp = pool.get<int>(n + 1), *dci = pool.get<int>(nnz);
    double *dv = pool.get<double>(nnz);
    HIPCHK(hipMemcpyAsync(drp, arp, sizeof(int) * (n + 1), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dci, aci, sizeof(int) * nnz, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dv, aval, sizeof(double) * nnz, hipMemcpyHostToDevice, s));
    arp = drp;
    aci = dci;
    aval = dv;
  }
  int st = check_input(pool, arp, aci, aval, n, nnz, s);
  if (st != BAMG_OK) fail(st, "input CSR rejected");

  const bool geometric = o.coarsening == BAMG_COARSEN_GEOMETRIC && geom && geom->kind != 0;
  h->lv.clear();
  h->lv.emplace_back();
  {
    Level &L0 = h->lv[0];
    L0.n = n;
    L0.gkind = geometric ? geom->kind : 0;
    L0.nx = geometric ? geom->nx : 0;
    L0.ny = geometric ? (geom->kind == 2 ? geom->ny : 1) : 0;
    double *b64 = nullptr;
    build_B(arp, aci, aval, n, pool, L0.B, b64, s);
    transpose_pattern(pool, L0.B, L0.Bt, L0.btperm, s);
    double *bt64 = pool.get<double>(L0.B.nnz);
    copy_permuted<double>(bt64, b64, L0.btperm, L0.B.nnz, s);
    if (o.validate) {
      // column sums on the main stream; reachability (a long chain of small
      // dependent steps on two CUs) beside the setup on an auxiliary stream,
      // joined before bamg_setup returns (validate = 3: by the first
      // computation on the hierarchy)
      h->vflag = pool.get<int>(4);
      fill_i32(h->vflag, 0, 4, s);
      colsum_launch(L0.Bt, bt64, h->vflag, s);
      HIPCHK(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&h->aux_ready, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&h->aux_done, hipEventDisableTiming));
      HIPCHK(hipEventRecord(h->aux_ready, s));
      HIPCHK(hipStreamWaitEvent(h->aux, h->aux_ready, 0));
      unsigned *visited = pool.get<unsigned>(2 * (size_t)((n + 31) / 32));
      int *queues = pool.get<int>(4 * (size_t)n + 64);
      h->vlevels = reach_launch(L0.B, L0.Bt, visited, queues, h->vflag, o.validate == 2, h->aux);
      h->vdeferred = h->vlevels > 0;  // global form: the rest by search_more
      HIPCHK(hipEventRecord(h->aux_done, h->aux));
      h->vvisited = visited;  // released after the join
      h->vqueues = queues;
    }
    L0.dpos = pool.get<int>(n);
    diag_positions(L0.B, L0.dpos, s);
    h->B64 = b64;
    if (h->prec == 0) {
      L0.Bv = b64;
      L0.Btv = bt64;
    } else {
      L0.Bv = pool.get<T>(L0.B.nnz);
      L0.Btv = pool.get<T>(L0.B.nnz);
      convert<double, T>((T *)L0.Bv, b64, L0.B.nnz, s);
      convert<double, T>((T *)L0.Btv, bt64, L0.B.nnz, s);
    }
    L0.M.nr = L0.M.nc = L0.M.nnz = n;
    L0.M.rp = pool.get<int>(n + 1);
    L0.M.ci = pool.get<int>(n);
    k_identity_csr<<<ceil_div(n, 256), 256, 0, s>>>(n, L0.M.rp, L0.M.ci);
    LAUNCHCHK();
    L0.Mv = pool.get<T>(n);
    L0.Nv = pool.get<T>(n);
    fill<T>((T *)L0.Mv, (T)1, n, s);
    fill<T>((T *)L0.Nv, (T)1, n, s);
    L0.identity_mn = true;
    L0.dinv = pool.get<T>(n);
  }
  int *flag = pool.get<int>(4);  // [3]: coarse-level diagonal failures, read per cycle
  fill_i32(flag, 0, 4, s);
  dinv_from_diag<T>(h->lv[0], (const T *)h->lv[0].Bv, (T *)h->lv[0].dinv, flag, true, s);

  // ---- integer structure of the hierarchy
  for (int l = 0;; ++l) {
    {
      Level &L = h->lv[l];
      if (L.n <= o.coarse_max || l == o.max_levels - 1 || l == 31) break;
      sym_graph(pool, L.B, L.Bt, L.G, s);
      L.cf = pool.get<int>(L.n);
      L.cidx = pool.get<int>(L.n);
      if (geometric) {
        geom_cf(L.n, L.nx, L.gkind, L.cf, s);
      } else if (o.coarsening == BAMG_COARSEN_CR) {
        // FP64 operator values: the input's on the first level, the
        // averaging Galerkin product below (formed when the level was made)
        const double *bv = l == 0 ? h->B64 : (const double *)L.Bv;
        double *tmp = nullptr;
        if (l > 0 && sizeof(T) != sizeof(double)) {
          tmp = pool.get<double>(L.B.nnz);
          convert<T, double>(tmp, (const T *)L.Bv, L.B.nnz, s);
          bv = tmp;
        }
        cr_cf(pool, L.B, bv, L.dpos, L.G, o.seed, l, o, L.cf, s);
        if (tmp) pool.release(tmp);
      } else {
        mis_cf(pool, L.G, o.seed, l, L.cf, s);
      }
      L.nc = coarse_numbering(pool, L.cf, L.n, L.cidx, L.cpts, s);
      if (L.nc == 0 || L.nc >= L.n) break;
      interp_pattern(pool, L, o.max_interp, geometric ? 1 : 0, L.P, s);
      transpose_pattern(pool, L.P, L.Pc, L.pcperm, s);
      spgemm_symbolic2(pool, L.B, L.P, L.M, L.P, 0, L.T1, L.T2, s);
    }
    Level C;
    {
      Level &L = h->lv[l];
      C.n = L.nc;
      C.gkind = L.gkind;
      C.nx = (L.nx + 1) / 2;
      C.ny = L.gkind == 2 ? (L.ny + 1) / 2 : 1;
      spgemm_symbolic2(pool, L.Pc, L.T1, L.Pc, L.T2, 1, C.B, C.M, s);
      L.Pv = pool.get<T>(L.P.nnz);
      L.Qtv = pool.get<T>(L.P.nnz);
      L.Ptv = pool.get<T>(L.P.nnz);
      L.Qv = pool.get<T>(L.P.nnz);
      L.T1v = pool.get<T>(L.T1.nnz);
      L.T2v = pool.get<T>(L.T2.nnz);
      L.T3v = pool.get<T>(L.T2.nnz);
    }
    transpose_pattern(pool, C.B, C.Bt, C.btperm, s);
    C.dpos = pool.get<int>(C.n);
    diag_positions(C.B, C.dpos, s);
    C.Bv = pool.get<T>(C.B.nnz);
    C.Btv = pool.get<T>(C.B.nnz);
    C.Mv = pool.get<T>(C.M.nnz);
    C.Nv = pool.get<T>(C.M.nnz);
    C.dinv = pool.get<T>(C.n);
    h->lv.push_back(C);
    if (o.coarsening == BAMG_COARSEN_CR && !geometric) {
      // the next level's compatible relaxation runs on Q B P with the
      // averaging transfers (1 / |J_i| on J_i); the bootstrap cycles refit P
      // and Q and form the operator again
      Level &L = h->lv[l], &N = h->lv[l + 1];
      fill_transfer_identity<T>(L, (T *)L.Pv, (T *)L.Qtv, s);
      copy_permuted<T>((T *)L.Qv, (const T *)L.Qtv, L.pcperm, L.P.nnz, s);
      int *sc = pool.get<int>((size_t)L.n + 1);
      spgemm_numeric<T>(L.B, (const T *)L.Bv, L.P, (const T *)L.Pv, L.T1, (T *)L.T1v, sc, s);
      spgemm_numeric<T>(L.Pc, (const T *)L.Qv, L.T1, (const T *)L.T1v, N.B, (T *)N.Bv, sc, s);
      pool.release(sc);
    }
  }
  h->L = (int)h->lv.size();
  if (h->L < 2) fail(BAMG_E_ARG, "no coarsening happened (check coarse_max and max_levels)");
  const int nL = h->lv[h->L - 1].n;
  if (nL > 2048) fail(BAMG_E_ARG, "coarsest level above 2048 states; lower coarse_max or raise max_levels");
  if (r > nL) fail(BAMG_E_ARG, "more test vectors than coarsest states");

  // ---- vectors and work space
  for (int l = 0; l < h->L; ++l) {
    Level &L = h->lv[l];
    const size_t nr = (size_t)L.n * r;
    L.U = pool.get<T>(nr);
    L.V = pool.get<T>(nr);
    L.U2 = pool.get<T>(nr);
    L.V2 = pool.get<T>(nr);
    L.xb = pool.get<T>(L.n);
    L.bb = pool.get<T>(L.n);
    L.rb = pool.get<T>(L.n);
    L.tb = pool.get<T>(L.n);
    if (o.smoother == BAMG_SMOOTH_KACZMARZ && l < h->L - 1) {
      L.colB = pool.get<int>(L.n);
      L.colBt = pool.get<int>(L.n);
      row_colouring(pool, L.B, L.Bt, L.colB, L.ncolB, L.ordB, L.offB, s);
      row_colouring(pool, L.Bt, L.B, L.colBt, L.ncolBt, L.ordBt, L.offBt, s);
      L.rowinvB = pool.get<T>(L.n);
      L.rowinvBt = pool.get<T>(L.n);
      if (l == 0) {
        row_inv_norms<T>(L.B, (const T *)L.Bv, (T *)L.rowinvB, s);
        row_inv_norms<T>(L.Bt, (const T *)L.Btv, (T *)L.rowinvBt, s);
      }
    }
  }
  h->sigma = pool.get<double>(64);
  fill<double>(h->sigma, 0.0, 64, s);

  Setup<T> S;
  S.h = h;
  S.s = s;
  S.r = r;
  S.nblk = kProdBlocks;
  S.part = pool.get<double>((size_t)S.nblk * 5 * 16);
  S.prod = pool.get<double>(5 * 16);
  S.wv = pool.get<double>(16);
  S.wu = pool.get<double>(16);
  S.scales = pool.get<double>(32);
  S.flag = flag;
  S.alloc_dense(nL);

  if (o.learned != BAMG_LEARNED_OFF) {
    h->lcount = pool.get<int>(2);
    fill_i32(h->lcount, 0, 2, s);
  }

  // ---- bootstrap cycles
  philox_testvecs(h->lv[0].U, h->lv[0].V, h->prec, n, r, o.seed, s);
  for (int cyc = 1; cyc <= o.setup_cycles; ++cyc) S.mle(0, cyc);


  // ---- coarse pseudo-inverse and x0
  S.pinv();
  std::vector<double> sig(r);
  HIPCHK(hipMemcpyAsync(sig.data(), h->sigma, sizeof(double) * r, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int kx = 0;
  for (int k = 1; k < r; ++k)
    if (sig[k] < sig[kx]) kx = k;
  h->x0 = pool.get<double>(n);
  k_extract_col<T><<<ceil_div(n, 256), 256, 0, s>>>((const T *)h->lv[0].V, n, r, kx, h->x0);
  LAUNCHCHK();
  const int nb = std::min(kRedBlocks, std::max(1, ceil_div(n, 256)));
  double *part = pool.get<double>(nb + 8);
  double *fl = pool.get<double>(16);
  normalize_sum(h->x0, n, part, nb, fl, s);
  pool.release(part);
  pool.release(fl);
  for (int l = 0; l + 1 < h->L; ++l) {
    if (o.autotune)
      tune_sweeps<T>(pool, h->lv[l], s);
    else
      h->lv[l].lanes = sweep_lanes_default(h->lv[l].n, h->lv[l].B.nnz);
  }
  h->search_more();  // when no SVD round loop took them
  if (o.validate != 3) {
    st = h->finish_validation();
    if (st != BAMG_OK) fail(st, "transition matrix rejected");
  }
  HIPCHK(hipStreamSynchronize(s));
  pool.flush();
}

template void setup_all<double>(bamg_handle *, const bamg_csr *, const bamg_geometry *);
template void setup_all<float>(bamg_handle *, const bamg_csr *, const bamg_geometry *);

}  // namespace bamg
