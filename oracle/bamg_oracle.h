/*
 * Plain FP64 CPU oracle of bootstrap-AMG preconditioned GMRES for the
 * stationary vector of an irreducible Markov chain (Brannick, Kahl,
 * Sokolovic, "An adaptively constructed algebraic multigrid preconditioner
 * for irreducible Markov chains").
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the HIP path; it
 * shares no code with it. Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. The product path never
 * calls it.
 *
 * It is deliberately slow and simple: serial loops, fixed summation order,
 * dense accumulators, textbook dense linear algebra (Cholesky, Householder
 * QR, one-sided Jacobi SVD). Every function cites the passage it follows.
 *
 * Conventions: A is given in CSR by destination state (row i holds a_ij =
 * p_ji, Section 2), 0-based int32 indices, FP64 values. Vectors of r test
 * vectors are n x r row-major.
 */
#ifndef BAMG_ORACLE_H
#define BAMG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_NOT_CONVERGED = 1,
  ORC_E_ARG = -1,
  ORC_E_NOT_STOCHASTIC = -2,
  ORC_E_REDUCIBLE = -3,
  ORC_E_BAD_DIAG = -4,
  ORC_E_COARSE = -5,
  ORC_E_BREAKDOWN = -6,
  ORC_E_NOMEM = -9
};

enum { ORC_COARSEN_GEOM = 0, ORC_COARSEN_MIS = 1, ORC_COARSEN_CR = 2 };
enum { ORC_SMOOTH_JACOBI = 0, ORC_SMOOTH_KACZMARZ = 1 };

typedef struct {
  int32_t r;            /* number of test vectors per side (Section 4.1) */
  int32_t setup_cycles; /* 1 = BAMG, 2 = BAMG^2 (Section 7) */
  int32_t nu_pre, nu_post, nu_setup; /* smoothing steps (Section 7) */
  double omega;         /* Jacobi damping (Section 7: 0.7) */
  int32_t max_interp;   /* c: cap on |J_i| (Section 4.1) */
  int32_t max_levels;
  int32_t coarse_max;   /* stop coarsening once n_l <= coarse_max */
  int32_t coarsening;   /* ORC_COARSEN_GEOM, ORC_COARSEN_MIS or ORC_COARSEN_CR */
  int32_t geom_kind;    /* 1 = 1-D line, 2 = 2-D grid (index iy*nx+ix) */
  int32_t nx, ny;
  uint64_t seed;
  int32_t smoother;     /* ORC_SMOOTH_JACOBI or ORC_SMOOTH_KACZMARZ */
  int32_t interp_rule;  /* 0 plain LS, 1 active set (no negative weights) */
  int32_t record_features; /* keep cycle-1 MLP features of the F points */
  int32_t cycle;        /* preconditioning cycle: ORC_CYCLE_V, _W or _F (Section 3) */
  int32_t mu;           /* passes of the inner loop of Algorithm 1 per level visit */
  int32_t restriction;  /* 0 = LS fit with 1^T Q = 1^T (Section 5), 1 = simple averaging */
  /* compatible relaxation (coarsening = ORC_COARSEN_CR, reading R-CR) */
  double cr_theta;      /* target F-relaxation rate: stop once a round's rate is at most this */
  double cr_beta;       /* candidates: F points with |e_i| >= cr_beta * max |e| */
  int32_t cr_sweeps;    /* F-relaxation sweeps per round */
  int32_t cr_rounds;    /* at most this many rounds */
} orc_options;

enum { ORC_CYCLE_V = 0, ORC_CYCLE_W = 1, ORC_CYCLE_F = 2 };

typedef struct {
  int32_t iterations, restarts, converged;
  double rel_residual, x_min;
} orc_info;

typedef struct orc_ctx orc_ctx;

void orc_default_options(orc_options *o);

/* Validate A, build the hierarchy and run the bootstrap setup cycles
 * (Algorithm 1, Sections 4-5). */
int orc_setup(int64_t n, const int32_t *rp, const int32_t *ci, const double *a,
              const orc_options *opt, orc_ctx **out);
void orc_destroy(orc_ctx *c);

int orc_num_levels(const orc_ctx *c);

/* Compatible-relaxation C/F splitting (reading R-CR) of the operator B
 * (CSR with values, diagonal stored) on the symmetrised graph G (no
 * diagonal): cf[i] = 1 for C, 0 for F. rates (rounds entries, nullable)
 * receives each round's F-relaxation rate; *nrounds the rounds run. */
int orc_cr(int n, const int32_t *brp, const int32_t *bci, const double *bv, const int32_t *grp,
           const int32_t *gci, uint64_t seed, int level, double theta, double beta, int sweeps,
           int rounds, double omega, int32_t *cf, double *rates, int32_t *nrounds);
/* Threads of the OpenMP row loops from now on (n >= 1; any count gives the
 * same results); returns the previous count. */
int orc_set_threads(int n);
/* dims: [n, nc, nnzB, nnzM, nnzP, nnzQ(coarse rows, == nnzP)] */
int orc_level_dims(const orc_ctx *c, int l, int64_t dims[6]);
/* what: 0 = B_l, 1 = B_l^T, 2 = M_l, 3 = N_l, 4 = P_l (fine rows),
 *       5 = Q_l (coarse rows), 6 = Q_l^T (fine rows, P_l's pattern). */
int orc_level_csr(const orc_ctx *c, int l, int what, int32_t *rp, int32_t *ci, double *v);
int orc_level_cf(const orc_ctx *c, int l, int32_t *cf, int32_t *cidx);
int orc_level_vectors(const orc_ctx *c, int l, double *U, double *V);
int orc_sigma(const orc_ctx *c, double *sigma);
int orc_x0(const orc_ctx *c, double *x0);
int orc_coarse_pinv(const orc_ctx *c, double *bdag); /* n_L x n_L row-major */
int orc_complexity(const orc_ctx *c, double *oc, double *og);

/* One V-cycle from a zero initial guess: x = C b (Section 6); the cycle
 * type of the options (V, W or F). */
int orc_vcycle(const orc_ctx *c, const double *b, double *x);
/* One cycle of the given type (ORC_CYCLE_*) on level 0 for B x = b: from
 * x = 0 if x_zero, else from the x passed in. */
int orc_cycle(const orc_ctx *c, int type, const double *b, double *x, int x_zero);
/* Apply one smoothing sweep on level l: x <- S_l(x, b). */
int orc_smooth(const orc_ctx *c, int l, const double *b, double *x);
/* Left-preconditioned GMRES(m) on C B e = -C B x0 (Section 6); stops when
 * ||Bx||_2/||x||_2 < tol; x is returned scaled to 1^T x = 1. */
int orc_gmres(const orc_ctx *c, double *x, int32_t m, double tol, int32_t maxit,
              int32_t use_x0, int32_t precondition, orc_info *info);

/* Learned interpolation (an addition to the paper): the 96 features of each
 * F point of level l as recorded in setup cycle 1 (record_features = 1), and
 * the final P rows (zero-padded to 8) with their mask. nF receives the
 * number of F points; X, T, M (nF x 96, nF x 8, nF x 8) may be NULL. */
int orc_harvest(const orc_ctx *c, int l, int64_t *nF, double *X, double *T, double *M);

/* Building blocks exposed for the pins. */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double orc_uniform_pm1(uint64_t seed, uint64_t side, uint64_t k, uint64_t i);
/* Weighted LS for one interpolation row (eq. ls_interpolation): G is r x m
 * row-major (G[k*m+t] = v_k at the t-th interpolation point), g[k] = v_k at
 * the fine point, w[k] the weights. Result p[m]. */
int orc_ls_row(int r, int m, const double *G, const double *g, const double *w, double *p);
/* Same with the sum-to-one constraint of Section 5, rows k >= 1 only. */
int orc_ls_row_sum1(int r, int m, const double *G, const double *g, const double *w, double *q);
/* Interpolation weights of one F point as the setup fits them: rule 0 =
 * plain weighted LS over all m points (eq. ls_interpolation), rule 1 =
 * R-ACT (while a weight is negative, the point with the most negative
 * weight is dropped and the fit redone, at least one point stays). sum1 = 1
 * takes the constrained Q-column fit of Section 5 instead (rows k >= 1,
 * weights sum to one). Same G, g, w layout as orc_ls_row. */
int orc_fit_point(int rule, int r, int m, const double *G, const double *g, const double *w,
                  int sum1, double *p);
/* The generalized Rayleigh quotient of eq. singular_value for one pair
 * (u, v) of length n, with B, M, N in CSR. */
int orc_rayleigh_sigma(int n, const int32_t *brp, const int32_t *bci, const double *bv,
                       const int32_t *mrp, const int32_t *mci, const double *mv,
                       const int32_t *nrp, const int32_t *nci, const double *nv,
                       const double *u, const double *v, double *sigma);
/* Dense generalized singular triplets of (B, M, N), eq. generalized_eigenvalue:
 * all n values ascending, U, V n x n column-major. */
int orc_gsvd(int n, const double *B, const double *M, const double *N,
             double *sigma, double *U, double *V);
/* Dense SVD by one-sided Jacobi: B = U diag(s) V^T, s unsorted per column. */
int orc_svd_jacobi(int n, const double *B, double *s, double *U, double *V);
/* Greedy maximal independent set on a symmetric pattern (no diagonal). */
int orc_mis(int n, const int32_t *rp, const int32_t *ci, uint64_t seed, int level,
            int32_t *cf);
/* Distance-2 greedy row colouring used by the Kaczmarz smoother. */
int orc_row_colouring(int n, const int32_t *rp, const int32_t *ci, const int32_t *crp,
                      const int32_t *cci, int32_t *colour);

#ifdef __cplusplus
}
#endif
#endif
