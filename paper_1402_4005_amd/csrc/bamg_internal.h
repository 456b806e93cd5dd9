// Internal declarations of the BAMG HIP library (gfx950).
//
// Layout in HBM, per level l of the hierarchy:
//   B_l      CSR, int32 row_ptr/col_idx, values of type T (diagonal always
//            stored, position in dpos); B_l^T as a separate CSR pattern whose
//            values are a gather of B_l's through a permutation.
//   M_l,N_l  one shared CSR pattern (M_0 = N_0 = I), two value arrays.
//   P_l      n_l x n_{l+1} CSR by fine row (|row| <= c); holds P and Q^T values.
//   Pc_l     its transpose, n_{l+1} x n_l by coarse row; holds P^T and Q values.
//   U_l,V_l  test vectors, n_l x r row-major so a neighbour gather reads r
//            contiguous values.
// Everything is FP64, or FP32 for the setup and the V-cycle of a
// mixed-precision handle; Krylov vectors and the coarsest solve stay FP64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/bamg.h"

namespace bamg {

// Raised inside the library, caught at the C boundary.
struct Error {
  bamg_status code;
  std::string msg;
};

[[noreturn]] void fail(bamg_status code, const std::string &msg);
void check_hip(hipError_t e, const char *what, const char *file, int line);
#define HIPCHK(x) ::bamg::check_hip((x), #x, __FILE__, __LINE__)
#define LAUNCHCHK() ::bamg::check_hip(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

// Device memory owned by a handle: every allocation is recorded and freed at
// destruction.
struct Pool {
  bamg_allocator a{};
  bool custom = false;
  hipStream_t s = nullptr;
  std::vector<void *> live;
  void *raw(size_t bytes);
  template <class X>
  X *get(size_t count) {
    return static_cast<X *>(raw(sizeof(X) * (count ? count : 1)));
  }
  std::vector<void *> chunks;    // sub-allocation chunks (in live as well)
  char *chunk_cur = nullptr;
  size_t chunk_left = 0;
  std::vector<void *> deferred;  // released temporaries, freed after a sync
  void release(void *p);          // defer the free of a temporary
  void flush();                   // synchronise s, then free the deferred
  void release_all();
  // kPinnedInts ints of pinned host memory for device-to-host copies of
  // sizes and flags: copies into it are queued without staging, so several
  // of them need one synchronisation only
  static constexpr int kPinnedInts = 64;
  int *hpin = nullptr;
  int *pinned();
};

struct Csr {
  int nr = 0, nc = 0, nnz = 0;
  int *rp = nullptr, *ci = nullptr;
};

struct Level {
  int n = 0, nc = 0, nx = 0, ny = 0, gkind = 0;
  Csr B, Bt, M, G, P, Pc, T1, T2;
  int *btperm = nullptr, *pcperm = nullptr, *dpos = nullptr;
  int *cf = nullptr, *cidx = nullptr, *cpts = nullptr;
  bool identity_mn = false;  // level 0: M = N = I
  // values (type T of the handle); void* so one struct serves both types
  void *Bv = nullptr, *Btv = nullptr, *Mv = nullptr, *Nv = nullptr, *dinv = nullptr;
  void *Pv = nullptr, *Qtv = nullptr, *Ptv = nullptr, *Qv = nullptr;
  void *T1v = nullptr, *T2v = nullptr, *T3v = nullptr;
  void *U = nullptr, *V = nullptr, *U2 = nullptr, *V2 = nullptr;
  // V-cycle work vectors
  void *xb = nullptr, *bb = nullptr, *rb = nullptr, *tb = nullptr;
  // Kaczmarz: rows of B (and of B^T) grouped by colour
  int ncolB = 0, ncolBt = 0;
  int *colB = nullptr, *colBt = nullptr;        // colour of each row
  int *ordB = nullptr, *ordBt = nullptr;        // rows sorted by colour
  std::vector<int> offB, offBt;                 // host: colour segment offsets
  void *rowinvB = nullptr, *rowinvBt = nullptr; // 1/||row||^2
  int lanes = 0;                                // lanes per CSR row (0 = from nnz/row)
  int threads = 0;                              // sweep workgroup size (0 = 256)
  // learned interpolation: F points (ascending) and recorded cycle-1 features
  int *fpts = nullptr;
  int nF = -1;
  float *feat = nullptr;  // nF x BAMG_MLP_IN (learned = record)
};

}  // namespace bamg

struct bamg_mlp {
  float *p = nullptr, *m = nullptr, *v = nullptr;  // FP32 parameters, Adam moments
  __bf16 *wb = nullptr;                            // BF16 weights for MFMA inference
  int step = 0;                                    // Adam steps taken
};

struct bamg_handle {
  bamg_options opt{};
  int prec = 0;  // 0 = FP64, 1 = FP32 setup/V-cycle
  bamg::Pool pool;
  std::vector<bamg::Level> lv;
  int L = 0;
  // level-0 B in FP64 for the Krylov solver (== lv[0].Bv when prec == 0)
  double *B64 = nullptr;
  double *sigma = nullptr;  // device, r (FP64)
  double *bdag = nullptr;   // device, n_L x n_L row-major (FP64)
  double *x0 = nullptr;     // device, n (FP64)
  double *red = nullptr;    // device reduction scratch
  size_t red_cap = 0;
  double *hred = nullptr;   // pinned host mirror: 2 x 16 flag slots
  double *hred_dev = nullptr;  // the same memory as the device addresses it
  hipEvent_t gm_ev[2] = {nullptr, nullptr};  // flag copies of alternate iterations
  // GMRES storage, allocated on first use
  int gm_m = 0;
  double *gV = nullptr, *gBV = nullptr, *gw = nullptr, *gx0 = nullptr, *gbx0 = nullptr;
  double *gZ = nullptr;  // flexible GMRES: z_j = C v_j (then gBV holds B z_j)
  double *gH = nullptr, *gsc = nullptr;
  void *vb = nullptr, *vx = nullptr;  // FP32 staging for a mixed V-cycle
  double *vcin = nullptr;             // fixed V-cycle input inside GMRES
  hipGraphExec_t vc_exec = nullptr;   // captured V-cycle: vcin -> gw
  hipStream_t cap_stream = nullptr;   // stream the V-cycle is captured on
  int use_graph = 1;
  int last_fused = 1;  // one-workgroup cycle on a small last level (option fuse_last_level)
  int imported = 0;    // hierarchy given by bamg_setup_from_levels (no setup data)
  double t_setup_ms = 0.0;  // host wall time of the setup(s) behind this hierarchy
  // event timing of one kernel (bamg_kernel_profile_*)
  int prof_kernel = -1;
  std::vector<hipEvent_t> prof_ev;  // pairs (start, stop)
  size_t prof_used = 0;
  double prof_bytes = 0.0;
  long prof_launches = 0;
  hipStream_t prof_stream = nullptr;
  // input validation running beside the setup on an auxiliary stream
  hipStream_t aux = nullptr;
  hipEvent_t aux_ready = nullptr, aux_done = nullptr;
  int *lcount = nullptr;  // device: [MLP rows, LS fallback rows]
  int *vflag = nullptr;  // device: [colsum bits, reached forward, reached backward, -]
  unsigned *vvisited = nullptr;  // the search's buffers, released after the join
  int *vqueues = nullptr;
  int vlevels = 0;               // levels the global-form search enqueued
  bool vdeferred = false;        // its later levels are still to be enqueued
  // enqueue the deferred levels of the global-form search (no-op otherwise)
  void search_more();
  int vstatus = BAMG_OK;         // outcome once joined
  void join_validation(bool wait_main);
  int validation_result();
  // join a validation still running (validate = 3: after the setup), keep
  // and return its outcome
  int finish_validation();
};

namespace bamg {

// ---- launchers: utilities (k_util.hip)
void scan_counts(Pool &pool, const int *counts, int *rp, int n, hipStream_t s);  // rp[0]=0..rp[n]
int read_int(const int *dptr, hipStream_t s);
void fill_i32(int *p, int v, size_t n, hipStream_t s);
void iota_i32(int *p, size_t n, hipStream_t s);
template <class T> void fill(T *p, T v, size_t n, hipStream_t s);
template <class T> void copy_permuted(T *out, const T *in, const int *perm, int n, hipStream_t s);
template <class A, class B> void convert(B *out, const A *in, size_t n, hipStream_t s);
// transposed pattern of A (nr x nc) and the permutation: At.val[k] = A.val[perm[k]]
void transpose_pattern(Pool &pool, const Csr &A, Csr &At, int *&perm, hipStream_t s);
void diag_positions(const Csr &A, int *dpos, hipStream_t s);  // -1 if absent
void philox_testvecs(void *U, void *V, int prec, int n, int r, uint64_t seed, hipStream_t s);

// ---- launchers: sparse kernels on vectors (k_sparse.hip); lanes per CSR row
// (0: from the average row length) and threads per workgroup (0: 256; the
// tuner's choice for a level's sweeps), neither of which changes a result
// y = A x (mode 0), y = b - A x (mode 1), y = y + A x (mode 2)
template <class T>
void spmv(const Csr &A, const T *val, const T *x, T *y, const T *b, int mode, int lanes,
          hipStream_t s, int threads = 0);
// x_out = x_in + omega dinv (b - A x_in); x_in == nullptr means x_in = 0
template <class T>
void jacobi(const Csr &A, const T *val, const T *dinv, T omega, const T *b, const T *xin, T *xout,
            int lanes, hipStream_t s, int threads = 0);
template <class T>
void jacobi2_from_zero(const Csr &A, const T *val, const T *dinv, T omega, const T *b, T *xout,
                       int lanes, hipStream_t s, int threads = 0);  // two sweeps from x = 0
// GMRES products (FP64): y1 = y2 = A x; and v = w scal[0], y1 = y2 = A v
void spmv_dual(const Csr &A, const double *val, const double *x, double *y1, double *y2,
               int lanes, hipStream_t s, int threads = 0);
void spmv_dual_scaled(const Csr &A, const double *val, const double *w, const double *scal,
                      double *v, double *y1, double *y2, int lanes, hipStream_t s,
                      int threads = 0);
// Kaczmarz sweep over one colour segment (in place)
template <class T>
void kaczmarz_colour(const Csr &A, const T *val, const T *rowinv, const int *rows, int nrows,
                     const T *b, T *x, hipStream_t s);
// dense coarse solve x = Bdag b (Bdag FP64); add != 0: x += Bdag b
template <class T>
void coarse_gemv(const double *bdag, int n, const T *b, T *x, hipStream_t s, int add = 0);
// partial sums for dot products: out[block] = sum x_i y_i (FP64)
void dot_partials(const double *x, const double *y, int n, double *part, int nblk, hipStream_t s);

// ---- launchers: setup (k_setup.hip)
void build_B(const int *arp, const int *aci, const double *aval, int n, Pool &pool, Csr &B,
             double *&bval, hipStream_t s);
int check_input(Pool &pool, const int *arp, const int *aci, const double *aval, int n, int nnz,
                hipStream_t s);
void colsum_launch(const Csr &Bt, const double *btv, int *flag, hipStream_t s);
// visited: 2 ceil(n / 32) words of device scratch (bitmaps, used when they
// do not fit in LDS or when force_global is set); queues: 4 n ints
int reach_launch(const Csr &B, const Csr &Bt, unsigned *visited, int *queues, int *flag,
                 bool force_global, hipStream_t s);
int reach_more(const Csr &B, const Csr &Bt, unsigned *visited, int *queues, int *flag, int k0,
               hipStream_t s);
void reach_finish(const Csr &B, const Csr &Bt, unsigned *visited, int *queues, int *flag,
                  int levels, hipStream_t s);
int validation_status(const int *h, int n);
void sym_graph(Pool &pool, const Csr &B, const Csr &Bt, Csr &G, hipStream_t s);
void geom_cf(int n, int nx, int gkind, int *cf, hipStream_t s);
void mis_cf(Pool &pool, const Csr &G, uint64_t seed, int level, int *cf, hipStream_t s);
void mis_rounds(Pool &pool, const Csr &G, const uint64_t *key, int *state, hipStream_t s);
// compatible-relaxation C/F splitting of the operator (B, bv FP64, diagonal
// positions dpos) on the graph G (k_cr.hip)
void cr_cf(Pool &pool, const Csr &B, const double *bv, const int *dpos, const Csr &G,
           uint64_t seed, int level, const bamg_options &o, int *cf, hipStream_t s);
int coarse_numbering(Pool &pool, const int *cf, int n, int *cidx, int *&cpts, hipStream_t s);
void interp_pattern(Pool &pool, const Level &L, int cap, int geometric, Csr &P, hipStream_t s);
// C1 = A1 B1 and C2 = A2 B2 (patterns) with one host round trip for both
void spgemm_symbolic2(Pool &pool, const Csr &A1, const Csr &B1, const Csr &A2, const Csr &B2,
                      int force_diag, Csr &C1, Csr &C2, hipStream_t s);
template <class T>
void spgemm_numeric(const Csr &A, const T *av, const Csr &B, const T *bv, const Csr &C, T *cv,
                    int *scratch, hipStream_t s);  // scratch: A.nr + 1 ints
template <class T>
void fill_transfer_identity(const Level &L, T *Pv, T *Qtv, hipStream_t s);
template <class T>
void ls_fit(const Level &L, int r, int mmax, const T *U, const T *V, const double *wv,
            const double *wu, int rule, int average, T *Pv, T *Qtv, hipStream_t s);
template <class T>
void dinv_from_diag(const Level &L, const T *bv, T *dinv, int *flag, bool check, hipStream_t s);
template <class T>
void inject(const int *cpts, int nc, int r, const T *X, T *Xc, hipStream_t s);
// Y = A X for r columns (row-major); if reset0, column 0 of Y is set to 1
template <class T>
void spmm(const Csr &A, const T *av, int r, const T *X, T *Y, int reset0, hipStream_t s);
// one simultaneous relaxation sweep of the test vectors (Algorithm 1)
template <class T>
void relax_pairs(const Level &L, int r, T omega, int with_rhs, const double *sigma, const T *U,
                 const T *V, T *Uo, T *Vo, hipStream_t s);
// per-block partial sums of u.Bv, u.Mu, v.Nv, |Bv|^2, |B^T u|^2 per column
// over at most nmax blocks; returns the number of blocks used
template <class T>
int pair_products(const Level &L, int r, const T *U, const T *V, int which, double *part,
                  int nmax, hipStream_t s);
template <class T>
void scale_columns(T *X, int n, int r, const double *scale, int skip0, hipStream_t s);
// sums of the product partials into out[16 t + k]; epi 1 also writes
// sigma_k to aux[k], epi 2 the normalisation scales (aux[k] for v_k,
// aux[16 + k] for u_k)
constexpr int kProdBlocks = 2048;
void finalize_products(const double *part, int nblk, int r, int which, int epi, double *out,
                       double *aux, hipStream_t s);
void ls_weights(const double *prod, int r, double *wv, double *wu, hipStream_t s);
// Kaczmarz colouring of the rows of A (columns listed by At)
void row_colouring(Pool &pool, const Csr &A, const Csr &At, int *colour, int &ncol,
                   int *&order, std::vector<int> &offsets, hipStream_t s);
template <class T>
void row_inv_norms(const Csr &A, const T *val, T *out, hipStream_t s);

// ---- launchers: coarsest level dense algebra (k_dense.hip)
void csr_to_dense(const Csr &A, const void *val, int prec, double *D, hipStream_t s);
// A0 = L L^T and A1 = L L^T (A1 may be null) in place, lower, row-major
int cholesky2(double *A0, double *A1, int n, int *flag, hipStream_t s);
void trsm_lower_cols(const double *L, double *X, int n, int ncols, int ldx,
                     hipStream_t s);  // X <- L^-1 X, column by column
void transpose_dense(const double *A, double *At, int n, hipStream_t s);
int jacobi_svd(Pool &pool, double *W, double *J, int n, hipStream_t s);
// both SVDs in the same launches (W2 nullable); W, J col-major. prof: a
// handle whose profiled kernel is the coarsest SVD (its round launches are
// bracketed by events and their algorithmic bytes summed), else nullptr
// after_first(ctx), when given, runs on the host once the first group of
// round launches is enqueued (the stream then holds tens of ms of work)
int jacobi_svd2(Pool &pool, double *W, double *J, double *W2, double *J2, int n, hipStream_t s,
                bamg_handle *prof = nullptr, void (*after_first)(void *) = nullptr,
                void *ctx = nullptr);
void column_norms(const double *W, int n, double *sv, hipStream_t s);
void coarse_triplets_out(const double *LM, const double *LN, const double *W, const double *J,
                         const double *sv, int n, int r, void *U, void *V, int prec,
                         double *sigma, double *work, hipStream_t s);
void zero_colsums(double *D, int n, hipStream_t s);  // D[j][j] -= sum_i D[i][j]
int coarse_small_max(void);  // largest n the LDS-resident solver takes
int coarse_small(int mode, int n, int r, const double *Bd, double *Md, double *Nd, void *U,
                 void *V, int prec, double *sigma, double *bdag, int *flag, hipStream_t s);
int build_pinv(Pool &pool, const double *W, const double *J, const double *sv, int n,
               double *bdag, hipStream_t s);

// ---- launchers: Krylov (k_krylov.hip)
void multi_dot(const double *Vb, int n, int k, const double *w, double *part, int nblk,
               hipStream_t s);
void finalize_multi(const double *part, int nblk, int k, double *out, hipStream_t s);
void multi_axpy_norm(const double *Vb, int n, int k, const double *h, double *w, double *part,
                     int nblk, hipStream_t s);
void gmres_arnoldi_update(double *H, double *cs, double *sn, double *g, double *y, double *h1,
                          double *h2, const double *wnorm_part, int nblk, double *vnext_scale,
                          int j, int m, double *flags, hipStream_t s);
void scale_vec(const double *in, const double *scal, double *out, int n, hipStream_t s);
void residual_check_partials(const double *x0, const double *bx0, const double *Vb,
                             const double *BVb, const double *y, int n, int k, double *part,
                             int nblk, hipStream_t s);
void residual_check_finalize(const double *part, int nblk, double tol, double *flags,
                             double *host_out, hipStream_t s);
// w <- w - sum_t h[t] V_t with the partials of V_t . w (t < k) in one pass;
// false (nothing launched) when k is above the fused kernel's bound
bool multi_axpy_dot(const double *Vb, int n, int k, const double *h, double *w, double *part,
                    int nblk, hipStream_t s);
void update_iterate(double *x0, const double *Vb, const double *y, int n, int k, hipStream_t s);
void negate_copy(const double *in, double *out, int n, hipStream_t s);
void normalize_sum(double *x, int n, double *part, int nblk, double *flags, hipStream_t s);

// one event of a bracketed run of launches of the profiled kernel
void profile_mark(bamg_handle *h, hipStream_t s, bool start);

// host-side orchestration
template <class T> void setup_all(bamg_handle *h, const bamg_csr *A, const bamg_geometry *g);
template <class T>
void import_all(bamg_handle *h, int nlev, const bamg_level_ops *ops, const double *pinv,
                const double *x0);
template <class T> void vcycle_run(bamg_handle *h, const T *b, T *x, hipStream_t s);
void gmres_run(bamg_handle *h, double *x, int m, double tol, int maxit, int use_x0,
               bamg_solve_info *info, hipStream_t s);
// partial-sum blocks of GMRES's reductions for n rows, and the Krylov
// storage of restart length m (allocated when m changes)
int gmres_blocks(int n);
void gmres_buffers(bamg_handle *h, int m);

// batched solve in one persistent launch (k_batch.hip): chains it can take,
// and the solve of hs[i] into x[i] (order: chains largest first); meanwhile
// runs on the host after the launch is queued and before its results are
// read back
constexpr int kBatchMaxRestart = 32;
bool batch_persistent_eligible(const bamg_handle *h, int restart);
void batch_persistent_solve(const std::vector<bamg_handle *> &hs, const std::vector<int> &order,
                            double *const *x, int restart, double tol, int maxit,
                            bamg_solve_info *infos, bamg_status *st, hipStream_t s,
                            const std::function<void()> &meanwhile);

constexpr int kRedBlocks = 1024;  // partial-sum blocks of the reductions

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// default lanes per CSR row: the average row length rounded up to a power of two
int lanes_for(int nr, int nnz);
// lanes per row of the V-cycle sweeps and residuals: 1, 2 or 4, where the
// row sums are formed in one order whatever the count (tuned, or else the
// average row length rounded up to a power of two, at most 4)
constexpr int kMaxTunedLanes = 4;
inline int sweep_lanes_default(int nr, int nnz) {
  const int l = lanes_for(nr, nnz);
  return l < kMaxTunedLanes ? l : kMaxTunedLanes;
}
// lanes per row of the V-cycle transfers (b_c = Q r, x += P x_c): the same
// rule, so their row sums take the canonical order too (a row of Q on a
// 2-D grid holds ~16 entries; 4 lanes of 4 entries each beat 16 lanes of
// one and a butterfly)
inline int transfer_lanes(int nr, int nnz) { return sweep_lanes_default(nr, nnz); }

// the V-cycle of the level above the coarsest and the coarsest solve in one
// workgroup (k_lastlevel.hip); false when the level does not fit (nothing
// launched)
template <class T>
bool vcycle_last_level(bamg_handle *h, int l, const T *b, T *x, hipStream_t s);
template <class T>
int last_level_lanes(const bamg_handle *h, int l);

// lanes per CSR row and workgroup size of a level's sweeps, by timing
// (tune.hip); sets L.lanes and L.threads
template <class T>
void tune_sweeps(Pool &pool, Level &L, hipStream_t s);

// learned interpolation weights (k_mlp.hip)
void mlp_refresh_bf16(bamg_mlp *m, hipStream_t s);
void mlp_forward(const bamg_mlp *m, const float *X, long npts, float *Y, int mode, hipStream_t s);
double mlp_loss_grad(const bamg_mlp *m, const float *X, const float *T, const float *M, long npts,
                     float *grad, hipStream_t s);
// the same with the scratch in the library's fixed per-GPU array (no allocation)
double mlp_loss_grad_noalloc(const bamg_mlp *m, const float *X, const float *T, const float *M,
                             long npts, float *grad, hipStream_t s);
void mlp_train(bamg_mlp *m, const float *X, const float *T, const float *M, long npts, int batch,
               int epochs, float lr, double *loss_per_epoch, hipStream_t s);
void level_fpoints(bamg_handle *h, Level &L, hipStream_t s);
template <class T>
void mlp_features(const Level &L, int r, const T *V, const double *wv, const T *Pv, float *F,
                  hipStream_t s);
template <class T>
void mlp_apply(const Level &L, int r, const T *V, const double *wv, const bamg_mlp *m, T *Pv,
               int *counts, hipStream_t s);
template <class T>
void mlp_targets(const Level &L, const T *Pv, float *Tg, float *Mk, hipStream_t s);

}  // namespace bamg
