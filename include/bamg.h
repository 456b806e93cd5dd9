/*
 * bamg.h -- C ABI of the MI355X (gfx950) implementation of bootstrap
 * algebraic multigrid (BAMG) preconditioned GMRES for the stationary vector
 * of an irreducible Markov chain.
 *
 * Method: Brannick, Kahl, Sokolovic, "An adaptively constructed algebraic
 * multigrid preconditioner for irreducible Markov chains". Given the
 * column-stochastic transition matrix A (a_ij = p_ji, Section 2), find
 * x > 0 with A x = x, i.e. B x = 0 with B = I - A (eq. Bx0). A bootstrap
 * setup (Algorithm 1, Sections 4 and 5) builds a multigrid hierarchy from
 * relaxed left/right test vectors by least-squares fits of interpolation P
 * and restriction Q and Petrov-Galerkin products Q B P; one V-cycle with a
 * zero initial guess is then the preconditioner C of GMRES on the residual
 * equation C B e = -C B x0 (Section 6), stopped when ||Bx||/||x|| < tol
 * (Section 7).
 *
 * Conventions for every call:
 *  - Return value: bamg_status. 0 = success; > 0 = warning, the outputs are
 *    valid; < 0 = error, the outputs are unspecified and no handle passed in
 *    is changed. No C++ exception crosses this boundary.
 *  - Indices are 0-based int32, values FP64 unless stated.
 *  - "device" pointers are HIP device memory on the current device; "host"
 *    pointers are ordinary host memory. Input arrays are only read during
 *    the call (they are copied); the library keeps no reference to them.
 *  - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *    All device work of a call is enqueued on it; calls that fill host
 *    outputs synchronise that stream before returning.
 *  - A handle is not thread-safe: calls on one handle must not overlap.
 *    Distinct handles are independent.
 */
#ifndef BAMG_H
#define BAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bamg_status;
enum {
  BAMG_OK = 0,
  BAMG_NOT_CONVERGED = 1,      /* iteration cap reached; best iterate returned */
  BAMG_E_ARG = -1,             /* bad argument, size or option */
  BAMG_E_NOT_STOCHASTIC = -2,  /* a_ij < 0 or a column sum differs from 1 by > 1e-12 */
  BAMG_E_REDUCIBLE = -3,       /* the chain's graph is not strongly connected */
  BAMG_E_BAD_DIAG = -4,        /* a zero or non-finite diagonal entry of some B_l */
  BAMG_E_COARSE = -5,          /* coarsest operator not of rank n_L - 1, or SVD failed */
  BAMG_E_BREAKDOWN = -6,       /* GMRES broke down twice without converging */
  BAMG_E_NONFINITE = -7,       /* NaN or Inf in an input entry or met in an iterate */
  BAMG_E_DEVICE = -8,          /* a HIP runtime call failed */
  BAMG_E_NOMEM = -9            /* device allocation failed */
};

enum { BAMG_COARSEN_GEOMETRIC = 0, BAMG_COARSEN_MIS = 1, BAMG_COARSEN_CR = 2 };
enum { BAMG_SMOOTH_JACOBI = 0, BAMG_SMOOTH_KACZMARZ = 1 };
enum { BAMG_PRECISION_FP64 = 0, BAMG_PRECISION_MIXED = 1 };
enum { BAMG_DTYPE_F64 = 0, BAMG_DTYPE_F32 = 1 };
enum { BAMG_GEOM_NONE = 0, BAMG_GEOM_LINE = 1, BAMG_GEOM_GRID2D = 2 };

/* Transition matrix A in CSR by destination state: row i lists the states j
 * with p_ji > 0 and holds a_ij = p_ji (Section 2). Columns strictly
 * ascending within each row. on_device != 0: the three arrays are device
 * pointers; otherwise host pointers. */
typedef struct {
  int64_t n, nnz;
  const int32_t *row_ptr; /* n + 1 */
  const int32_t *col_idx; /* nnz */
  const double *val;      /* nnz */
  int32_t on_device;
} bamg_csr;

/* Optional geometry: kind BAMG_GEOM_GRID2D with state index iy*nx + ix
 * (nx*ny == n), or BAMG_GEOM_LINE with nx == n. Used by geometric
 * coarsening, which takes every other point in each direction (Section 7). */
typedef struct {
  int32_t kind, nx, ny;
} bamg_geometry;

/* Options. bamg_default_options fills the paper's standard parameters
 * (Section 7): r = 8 test vectors, 3 + 3 weighted-Jacobi sweeps with
 * omega = 0.7, interpolation from at most c = 4 coarse points. */
typedef struct {
  int32_t r;            /* test vectors per side, 2..16 (Section 4.1) */
  int32_t setup_cycles; /* 1 = BAMG, 2 = BAMG^2 (Section 7) */
  int32_t nu_pre, nu_post; /* V-cycle smoothing steps (Section 3) */
  int32_t nu_setup;     /* smoothing steps per level visit in the setup (Algorithm 1) */
  double omega;         /* Jacobi damping: x <- x + omega D^-1 (b - B x) */
  int32_t max_interp;   /* c: at most c interpolation points per F point, 1..8 */
  int32_t max_levels;   /* cap on the number of levels, >= 2 */
  int32_t coarse_max;   /* stop coarsening once n_l <= coarse_max (<= 2048) */
  int32_t coarsening;   /* BAMG_COARSEN_GEOMETRIC (needs geometry), BAMG_COARSEN_MIS, or
                           BAMG_COARSEN_CR (compatible relaxation, the cr_* fields) */
  uint64_t seed;        /* test vectors and MIS priorities (Philox-4x64-10) */
  int32_t smoother;     /* BAMG_SMOOTH_JACOBI or BAMG_SMOOTH_KACZMARZ (Section 3) */
  int32_t precision;    /* BAMG_PRECISION_FP64 or BAMG_PRECISION_MIXED */
  int32_t interp_rule;  /* 0 = plain LS over J_i, 1 = LS with negative weights removed */
  int32_t validate;     /* 1 = check stochasticity and strong connectivity; 2 = the
                           same with the search's visited set in global memory
                           whatever the size (the form large chains take); 3 = the
                           check of 1, not waited for by bamg_setup: the
                           strong-connectivity search keeps running beside the
                           hierarchy and the first bamg_gmres_solve or bamg_vcycle
                           waits for it at its end and returns BAMG_E_REDUCIBLE or
                           BAMG_E_NOT_STOCHASTIC instead of its result when the
                           chain fails (bamg_setup still reports them when it fails
                           itself); 0 = no check */
  int32_t use_graph;    /* 1 = GMRES replays the V-cycle from a captured HIP graph;
                           0 (default) = its kernels are launched one by one (the
                           host enqueues an iteration ahead, and on MI355X a graph
                           replay costs more than the launches it saves) */
  int32_t learned;      /* BAMG_LEARNED_*: interpolation weights from an MLP (see below) */
  const struct bamg_mlp *mlp; /* network for BAMG_LEARNED_USE, else ignored */
  int32_t autotune;     /* 1 = time the lanes-per-row choices of each level's
                           sweeps once per matrix shape (cached per process) */
  int32_t fuse_last_level; /* 1 = when the level above the coarsest (not the
                           finest) fits in one workgroup's LDS, its part of the
                           V-cycle and the coarsest solve run as one launch
                           (the same steps, Jacobi smoother only); 0 = one
                           kernel per step */
  int32_t cycle;        /* preconditioner C of GMRES and bamg_vcycle: BAMG_CYCLE_V
                           (default), _W, _F (Section 3), or _NONE (C = I: GMRES
                           without preconditioner, the GMRES(m) rows of Section 7) */
  int32_t mu;           /* passes of the inner loop of Algorithm 1 per level visit, 1..8
                           (1 = default) */
  int32_t restriction;  /* 0 = Q fitted with 1^T Q = 1^T (Section 5), 1 = simple
                           averaging: column i of Q has 1 / |J_i| on J_i */
  int32_t profile_setup; /* 1 = time the round launches of the coarsest-level
                           Jacobi SVD during bamg_setup with HIP events (read them
                           with bamg_kernel_profile_end); 0 = off */
  int32_t learned_max_iters; /* BAMG_LEARNED_USE only: when GMRES has not converged
                           after this many iterations, the hierarchy is rebuilt with
                           the exact LS fits (same options, learned off) and GMRES
                           continues from its iterate; 0 = never */
  /* Compatible-relaxation coarsening (BAMG_COARSEN_CR; Section 7 names the
   * method, whose algorithm it cites): per level, rounds of cr_sweeps
   * weighted-Jacobi sweeps (weight omega) on B_ff e_f = 0 from a fixed
   * pseudo-random start with the C entries zero; a round whose last-sweep
   * rate ||e^k|| / ||e^(k-1)|| is at most cr_theta ends the search, else the
   * F points with |e_i| >= cr_beta max |e| are candidates and the greedy
   * independent set of their graph, by decreasing (number of candidate
   * neighbours, priority), joins C; at most cr_rounds rounds. Then F points
   * without a coarse neighbour take a greedy independent set of their own.
   * Levels below the first use the Galerkin product with averaging
   * transfers (the bootstrap refits P and Q afterwards). */
  double cr_theta;      /* 0.8 */
  double cr_beta;       /* 0.7, in [0, 1] */
  int32_t cr_sweeps;    /* 5, 1..64 */
  int32_t cr_rounds;    /* 10, 0..64 */
  /* 1 = flexible GMRES: right preconditioning with the preconditioned
   * vectors z_j = C v_j kept (x = x0 + Z y, and B z_j enters the Arnoldi
   * process), so a preconditioner that is not exactly one linear map (the
   * FP32 V-cycles of BAMG_PRECISION_MIXED round differently for each input)
   * still gives the least true residual over the space it spans; n x restart
   * more FP64 storage. 0 (default) = GMRES on the left-preconditioned residual
   * equation C B e = -C B x^(0) of Section 6. In a batch, flexible chains
   * solve on the library streams, not in the persistent launch. */
  int32_t flexible;
} bamg_options;

/* Cycle shapes. A W-cycle takes two cycles of its own shape on the next
 * level, the second from the first's result; an F-cycle one F-cycle and
 * then one V-cycle. On the coarsest level a cycle from a guess x is
 * x + B_L^+ (b - B_L x). */
enum { BAMG_CYCLE_V = 0, BAMG_CYCLE_W = 1, BAMG_CYCLE_F = 2, BAMG_CYCLE_NONE = 3 };

/* Learned interpolation weights. Not part of the paper: an addition whose
 * aim is to replace the second bootstrap cycle (BAMG^2, Section 7). In
 * BAMG_LEARNED_USE mode, setup cycle 1 takes each F row of P from the MLP
 * instead of from the least-squares fit of eq. ls_interpolation. The exact
 * LS fit is kept for a row whenever the MLP weights give an LS objective
 * above twice the exact fit's value. BAMG_LEARNED_RECORD keeps the MLP
 * input features of cycle 1 so that bamg_harvest can return them together
 * with the final P rows (training data). */
enum { BAMG_LEARNED_OFF = 0, BAMG_LEARNED_USE = 1, BAMG_LEARNED_RECORD = 2 };

/* Device allocator used for every library allocation (NULL = hipMalloc /
 * hipFree). alloc returns NULL on failure. */
typedef struct {
  void *ctx;
  void *(*alloc)(void *ctx, size_t bytes, void *hip_stream);
  void (*free)(void *ctx, void *ptr, void *hip_stream);
} bamg_allocator;

typedef struct {
  int32_t iterations;    /* preconditioned GMRES iterations after the setup (Section 7) */
  int32_t restarts;
  int32_t converged;
  int32_t breakdowns;
  double rel_residual;   /* final ||Bx||_2 / ||x||_2, FP64 */
  double x_min;          /* min_i x_i after scaling to 1^T x = 1 */
  double t_solve_ms;     /* host wall time of the call */
  int32_t setup_cycles;  /* bootstrap cycles of the hierarchy used at the end */
  int32_t mlp_fallback;  /* 1 if a learned hierarchy was replaced by the exact-LS one
                            during this solve (bamg_options.learned_max_iters) */
  double t_setup_ms;     /* host wall time of the setup(s) behind the final hierarchy */
  int64_t mlp_rows;      /* learned form: F rows of the final hierarchy that took the
                            network's correction (0 otherwise) */
  int64_t ls_fallbacks;  /* learned form: F rows that kept the exact LS fit because the
                            network's row failed the objective test (0 otherwise) */
} bamg_solve_info;

typedef struct bamg_handle bamg_handle;

/* ---------------------------------------------------------------------
 * Interpolation-weight MLP: 96 inputs -> 64 -> 64 (ReLU) -> 8 outputs.
 * Parameters, FP32, in this order (row-major, out x in):
 *   W1[64][96], b1[64], W2[64][64], b2[64], W3[8][64], b3[8]
 * (BAMG_MLP_NPARAMS values). Inference runs on MFMA in BF16 (weights and
 * activations rounded to nearest-even BF16, FP32 accumulation); training
 * runs in FP32.
 *
 * Features of an F point i with interpolation set J_i = (j_1..j_m), m <= 8,
 * and r = 8 normalised test vectors v^(k) with LS weights w_k (eq.
 * ls_weights, divided by their maximum):
 *   f[9k]         = sqrt(w_k) v^(k)_i / S          k = 0..7
 *   f[9k + 1 + t] = sqrt(w_k) v^(k)_{j_t} / S      t < m, else 0
 *   f[72 + t] = B_{i j_t} / B_ii                    (t < m, else 0)
 *   f[80 + t] = p^LS_{i j_t}, the exact cycle-1 fit of the row
 *   f[88 + t] = 1 if t < m else 0
 * with S the largest |sqrt(w_k) v^(k)| among the gathered values (1 if 0).
 * Outputs y_t are corrections: the network's row is p^LS_{i j_t} + y_t,
 * t < m (entries t >= m are ignored). */
#define BAMG_MLP_IN 96
#define BAMG_MLP_HIDDEN 64
#define BAMG_MLP_OUT 8
#define BAMG_MLP_NPARAMS 10888
typedef struct bamg_mlp bamg_mlp;

/* Fill *out with the defaults above. */
bamg_status bamg_default_options(bamg_options *out);

/* Validate A, build B = I - A (eq. Bx0), the integer structure of the
 * hierarchy (C/F splittings, interpolation sets J_i, Galerkin patterns),
 * then run setup_cycles bootstrap cycles (Algorithm 1 with the constraint
 * 1^T Q = 1^T of Section 5), the coarsest pseudo-inverse (eq.
 * coarse_grid_correction) and the initial iterate x0 (Section 6).
 * geom may be NULL. alloc may be NULL. On success *out owns all device
 * memory of the hierarchy; free it with bamg_destroy. Input errors:
 * BAMG_E_ARG for a malformed CSR (row pointers, column range or order),
 * BAMG_E_NONFINITE for a NaN or Inf entry, BAMG_E_NOT_STOCHASTIC for a
 * negative entry or a column sum off 1, BAMG_E_REDUCIBLE for a chain that
 * is not strongly connected (with validate = 3 these two may come from the
 * first solve instead, as stated for bamg_options.validate). */
bamg_status bamg_setup(const bamg_csr *A, const bamg_geometry *geom, const bamg_options *opt,
                       const bamg_allocator *alloc, void *hip_stream, bamg_handle **out);

/* One application of the preconditioner with zero initial guess, x = C b
 * (Section 6, eq. iterate_preconditioner): a V-cycle by default, or the
 * handle's cycle shape (bamg_options.cycle, bamg_set_cycle). b and x are
 * device arrays of n values of type dtype (BAMG_DTYPE_F64 or, for a
 * mixed-precision handle, BAMG_DTYPE_F32); they must not overlap.
 * Asynchronous on hip_stream. */
bamg_status bamg_vcycle(bamg_handle *h, const void *b, void *x, int32_t dtype, void *hip_stream);

/* GMRES(restart) on the preconditioned residual equation C B e = -C B x0
 * (Section 6, eq. prec_residual), Arnoldi in FP64 with classical
 * Gram-Schmidt applied twice, the true scaled residual ||Bx||/||x|| tested
 * after every iteration (Section 7). x: device, n FP64; on entry the
 * initial iterate if use_x0 != 0 (else the setup's x0 is used); on exit the
 * iterate scaled to 1^T x = 1. info (host, may be NULL) is filled after a
 * stream synchronisation. For a learned hierarchy with learned_max_iters >
 * 0 the iteration fallback may replace h's hierarchy by the exact-LS one
 * (the handle stays valid; info->mlp_fallback says so; iterations count
 * both parts). */
bamg_status bamg_gmres_solve(bamg_handle *h, void *x, int32_t restart, double tol,
                             int32_t max_iters, int32_t use_x0, bamg_solve_info *info,
                             void *hip_stream);

/* A CSR matrix in host memory with nrows x ncols, columns strictly
 * ascending within each row, FP64 values. */
typedef struct {
  int64_t nrows, ncols, nnz;
  const int32_t *row_ptr; /* nrows + 1 */
  const int32_t *col_idx; /* nnz */
  const double *val;      /* nnz */
} bamg_host_csr;

/* One level of an explicitly given hierarchy: B_l (n_l x n_l, diagonal
 * stored and non-zero), the interpolation P_l (n_l x n_{l+1}) and the
 * restriction Q_l (n_{l+1} x n_l); P and Q are ignored on the last level. */
typedef struct {
  bamg_host_csr B, P, Q;
} bamg_level_ops;

/* A handle whose hierarchy is given instead of built: nlevels (2..32)
 * levels of operators, coarse_pinv the n_L x n_L row-major pseudo-inverse
 * of B_L used as the coarsest solve (eq. coarse_grid_correction), x0 the
 * n_0 initial iterate of GMRES (Section 6); all host memory, copied before
 * the call returns. The V-cycle (Section 3) and GMRES then run on exactly
 * these operators with the kernels bamg_setup's handles use. From opt only
 * the solve-phase fields are read: nu_pre, nu_post, omega, smoother,
 * precision, use_graph, autotune, fuse_last_level (r, setup and coarsening
 * fields are ignored). Errors: BAMG_E_ARG for a shape, pointer, ordering or
 * size fault (each coarse level smaller than its fine level, n_L <= 2048),
 * BAMG_E_NONFINITE for a non-finite value, BAMG_E_BAD_DIAG for a zero or
 * missing diagonal of some B_l. The setup-only inspection calls
 * (bamg_level_cf, bamg_level_vectors, M/N/B^T in bamg_level_csr,
 * bamg_harvest) return BAMG_E_ARG on such a handle. */
bamg_status bamg_setup_from_levels(int32_t nlevels, const bamg_level_ops *levels,
                                   const double *coarse_pinv, const double *x0,
                                   const bamg_options *opt, const bamg_allocator *alloc,
                                   void *hip_stream, bamg_handle **out);

/* Change the preconditioner shape of h (BAMG_CYCLE_*) without a new
 * setup; BAMG_E_ARG for another value. */
bamg_status bamg_set_cycle(bamg_handle *h, int32_t cycle);

/* Hierarchy summary (host outputs, each may be NULL): number of levels,
 * n_l and nnz(B_l) for l < *levels (arrays sized >= 32), operator and grid
 * complexity (Section 4.1 eq. operator_complexity_def, Section 7). */
bamg_status bamg_hierarchy_info(const bamg_handle *h, int32_t *levels, int64_t *n_l,
                                int64_t *nnz_l, double *oc, double *og);

/* Copy one level out to host buffers (for checking and checkpoints).
 * what: 0 = B_l, 1 = B_l^T, 2 = M_l, 3 = N_l, 4 = P_l (n_l x n_{l+1}, fine
 * rows), 5 = Q_l (n_{l+1} x n_l, coarse rows), 6 = Q_l^T (fine rows, the
 * pattern of P_l). nnz is read from bamg_level_nnz. Values are FP64
 * (converted for a mixed-precision handle). Any output may be NULL. */
bamg_status bamg_level_nnz(const bamg_handle *h, int32_t l, int32_t what, int64_t *rows,
                           int64_t *nnz);
bamg_status bamg_level_csr(const bamg_handle *h, int32_t l, int32_t what, int32_t *row_ptr,
                           int32_t *col_idx, double *val);
/* C/F splitting of level l < levels-1: cf[i] = 1 for C points; cidx[i] the
 * coarse index or -1. Host outputs of n_l int32 each, may be NULL. */
bamg_status bamg_level_cf(const bamg_handle *h, int32_t l, int32_t *cf, int32_t *cidx);
/* Test vectors of level l after the last setup cycle: U, V host n_l x r
 * row-major FP64; sigma host r values. Any output may be NULL. */
bamg_status bamg_level_vectors(const bamg_handle *h, int32_t l, double *U, double *V);
bamg_status bamg_sigma(const bamg_handle *h, double *sigma);
/* x0 of Section 6 (device n FP64 output), the coarsest pseudo-inverse
 * (host n_L x n_L row-major FP64 output). */
bamg_status bamg_x0(const bamg_handle *h, void *x_device, void *hip_stream);
bamg_status bamg_coarse_pinv(const bamg_handle *h, double *bdag);

/* Algorithmic HBM bytes of one V-cycle on this hierarchy: every CSR value
 * and index read once, every vector read or written once per kernel that
 * touches it, the dense coarsest solve; FP64 or FP32 values as stored. */
bamg_status bamg_vcycle_bytes(const bamg_handle *h, double *bytes);
/* Lanes of a 64-wide wave that share one CSR row in the sweeps and
 * residual of level l (after autotuning, if it was requested; otherwise the
 * average row length rounded up to a power of two, at most 4). */
bamg_status bamg_level_lanes(const bamg_handle *h, int32_t l, int32_t *lanes);
/* Set the lanes per row (1, 2 or 4) of level l's sweeps and residual
 * (l < levels - 1), e.g. to pin a launch shape for profiling. Each row is
 * summed in one fixed order whatever the lane count, so results are bitwise
 * the same for every choice. BAMG_E_ARG for another value, or once GMRES
 * has captured the V-cycle into a graph (use_graph = 1). */
bamg_status bamg_level_set_lanes(bamg_handle *h, int32_t l, int32_t lanes);
/* Workgroup size (threads) of level l's sweeps and residual, and on level 0
 * of GMRES's products with B: 256 unless autotuning picked 128, 512 or 1024
 * (l < levels - 1). */
bamg_status bamg_level_threads(const bamg_handle *h, int32_t l, int32_t *threads);
/* Set it (64, 128, 256, 512 or 1024), e.g. to pin a launch shape. A row's
 * sum does not depend on the workgroup it falls in, so results are bitwise
 * the same for every choice. BAMG_E_ARG for another value, or once GMRES has
 * captured the V-cycle into a graph (use_graph = 1). */
bamg_status bamg_level_set_threads(bamg_handle *h, int32_t l, int32_t threads);

/* Kernel timing with HIP events on the launch stream. Kernel
 * BAMG_PROFILE_FINEST_SWEEP: the weighted-Jacobi sweep on the finest level
 * (the V-cycle smoother that starts from a nonzero iterate); after begin,
 * every run of back-to-back launches of that kernel on h is bracketed by two
 * events. Kernel BAMG_PROFILE_COARSEST_SVD: the round launches of the
 * coarsest-level Jacobi SVD, recorded during bamg_setup when
 * bamg_options.profile_setup = 1 (each group of sweeps bracketed; bytes:
 * every W and J column block read, written where the block rotated). end
 * synchronises h's last stream and returns the number of launches, their
 * summed duration (ms) and their summed algorithmic bytes. */
enum { BAMG_PROFILE_FINEST_SWEEP = 0, BAMG_PROFILE_COARSEST_SVD = 1 };
bamg_status bamg_kernel_profile_begin(bamg_handle *h, int32_t kernel);
bamg_status bamg_kernel_profile_end(bamg_handle *h, int64_t *launches, double *ms_total,
                                    double *bytes_total);

/* Free every resource of h (NULL is ignored). */
void bamg_destroy(bamg_handle *h);

/* ---------------------------------------------------------------------
 * Many independent chains. bamg_setup_batched sets up chain i from A[i],
 * geom[i] (geom may be NULL: no geometry for any chain) and opt[i]. The
 * chains run concurrently on nstreams library streams (0 = 4), largest
 * first, each stream served by its own host thread; the caller's stream
 * is joined to them on entry and on return, so work enqueued on it
 * afterwards sees every result. A failing chain does not fail the batch:
 * its status is kept (bamg_batch_status) and it is skipped by the solve.
 * Returns BAMG_OK when the batch object was created. */
typedef struct bamg_batch bamg_batch;
bamg_status bamg_setup_batched(int32_t nchains, const bamg_csr *A, const bamg_geometry *geom,
                               const bamg_options *opt, const bamg_allocator *alloc,
                               int32_t nstreams, void *hip_stream, bamg_batch **out);
/* Setup status of chain i and its handle (NULL if the setup failed); the
 * handle stays owned by the batch. */
bamg_status bamg_batch_status(const bamg_batch *b, int32_t i, bamg_status *setup_status,
                              bamg_handle **handle);
/* bamg_gmres_solve for every chain that was set up: x[i] device FP64 of
 * chain i's length; infos and statuses (host, nchains entries each;
 * statuses nullable) receive each chain's result. Returns BAMG_OK if all
 * chains converged, BAMG_NOT_CONVERGED if any did not or failed.
 *
 * Chains run in one persistent launch on the caller's stream, or by
 * bamg_gmres_solve on the library streams, both at once. In the launch each
 * workgroup takes the next chain (largest first) and runs its GMRES(m)
 * (Section 6) with V-cycle preconditioning (Section 3) to the stopping
 * test of Section 7 with workgroup barriers only; its arithmetic and
 * summation orders are those of bamg_gmres_solve on the same handle, so
 * every chain's x, iteration count and residual equal that call's bit for
 * bit, whichever way it ran. The launch takes chains with a V-cycle (or no
 * preconditioner), restart <= 32 and no learned iteration fallback, and
 * under the default BAMG_BATCH_AUTO only those of at most 5000 states
 * (larger ones are faster per chain on the streams); BAMG_BATCH_PERSISTENT
 * gives it every chain it can take, BAMG_BATCH_STREAMS none. The call
 * returns when every result is written. infos[i].t_solve_ms is the chain's
 * own time (inside the launch, or its call's). */
bamg_status bamg_gmres_solve_batched(bamg_batch *b, double *const *x, int32_t restart,
                                     double tol, int32_t max_iters, bamg_solve_info *infos,
                                     bamg_status *statuses, void *hip_stream);
enum { BAMG_BATCH_AUTO = 0, BAMG_BATCH_PERSISTENT = 1, BAMG_BATCH_STREAMS = 2 };
/* Choose how bamg_gmres_solve_batched runs (BAMG_BATCH_*). BAMG_E_ARG for
 * an unknown value. */
bamg_status bamg_batch_set_solver(bamg_batch *b, int32_t solver);
void bamg_batch_destroy(bamg_batch *b);

/* Create a network from BAMG_MLP_NPARAMS FP32 parameters (host memory,
 * copied) on the current device. Adam moments start at zero. */
bamg_status bamg_mlp_create(const float *params, bamg_mlp **out);
/* Copy the current FP32 parameters to host memory (BAMG_MLP_NPARAMS). */
bamg_status bamg_mlp_get_params(const bamg_mlp *m, float *params);
void bamg_mlp_destroy(bamg_mlp *m);
/* Y = MLP(X) for npts points: X device FP32 npts x 96, Y device FP32
 * npts x 8. mode 0 = FP32 (the training arithmetic), 1 = BF16 MFMA (the
 * inference path used by the setup). */
bamg_status bamg_mlp_forward(const bamg_mlp *m, const float *X, int64_t npts, float *Y,
                             int32_t mode, void *hip_stream);
/* Loss and gradient over npts points (device FP32 X npts x 96, targets T
 * and mask M npts x 8):
 *   loss = 1/(2 npts) sum_p sum_t M_pt (MLP(X_p)_t - T_pt)^2
 * *loss (host) in FP64; grad (device FP32, BAMG_MLP_NPARAMS, same order
 * as the parameters). FP32 arithmetic, fixed summation order. */
bamg_status bamg_mlp_loss_grad(const bamg_mlp *m, const float *X, const float *T,
                               const float *M, int64_t npts, double *loss, float *grad,
                               void *hip_stream);
/* bamg_mlp_loss_grad for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving or training loops, harnesses that
 * forbid hipMalloc): the same inputs, outputs and kernels, with the
 * per-point activations, the gradient partials and the loss sum held in one
 * fixed device array of the library (64 MiB per GPU, held until the process
 * ends) instead of fresh allocations. At most BAMG_MLP_NOALLOC_MAX_POINTS
 * points per call (else BAMG_E_ARG, nothing enqueued). Every call on one GPU
 * uses that GPU's array: calls that overlap on one GPU (different streams or
 * threads without ordering) race and must not be made. The call synchronises
 * hip_stream to return *loss. */
#define BAMG_MLP_NOALLOC_MAX_POINTS 60000
bamg_status bamg_mlp_loss_grad_noalloc(const bamg_mlp *m, const float *X, const float *T,
                                       const float *M, int64_t npts, double *loss, float *grad,
                                       void *hip_stream);
/* Adam training (beta1 0.9, beta2 0.999, eps 1e-8) on the loss above with
 * mini-batches of `batch` consecutive points, `epochs` passes in the given
 * order. loss_per_epoch (host, epochs entries, nullable) receives the mean
 * batch loss of each epoch. */
bamg_status bamg_mlp_train(bamg_mlp *m, const float *X, const float *T, const float *M,
                           int64_t npts, int32_t batch, int32_t epochs, float lr,
                           double *loss_per_epoch, void *hip_stream);
/* Training data of a handle set up with learned = BAMG_LEARNED_RECORD:
 * for level l (< levels - 1), the cycle-1 features of its F points
 * (ascending state index) and their final P rows (weights in J_i order,
 * zero-padded to 8) with a mask of the valid entries. Training targets for
 * the corrections are T - X[:, 80:88]. X, T, M are device
 * FP32 buffers of nF x 96, nF x 8, nF x 8, or all NULL to query *nF. */
bamg_status bamg_harvest(const bamg_handle *h, int32_t level, float *X, float *T, float *M,
                         int64_t *nF, void *hip_stream);
/* Points whose P row the MLP supplied and rows that fell back to the exact
 * LS fit, summed over levels (learned = BAMG_LEARNED_USE). */
bamg_status bamg_learned_stats(const bamg_handle *h, int64_t *mlp_rows, int64_t *fallback_rows);

/* Static description of a status code. */
const char *bamg_status_string(bamg_status s);

/* Text of the last error on this thread (empty if none). */
const char *bamg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
