// C ABI of the library (include/bamg.h): argument checks, error translation
// (no exception crosses the boundary), device memory ownership.
#include <chrono>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <cmath>

#include "bamg_internal.h"

namespace bamg {

static thread_local std::string g_last_error;

void fail(bamg_status code, const std::string &msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char *what, const char *file, int line) {
  if (e == hipSuccess) return;
  const bamg_status code = (e == hipErrorOutOfMemory) ? BAMG_E_NOMEM : BAMG_E_DEVICE;
  throw Error{code, std::string(what) + ": " + hipGetErrorString(e) + " at " + file + ":" +
                        std::to_string(line)};
}

static void *device_alloc(Pool &pool, size_t bytes) {
  void *p = nullptr;
  if (pool.custom) {
    p = pool.a.alloc(pool.a.ctx, bytes, (void *)pool.s);
    if (!p) throw Error{BAMG_E_NOMEM, "caller allocator returned NULL"};
  } else {
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error{BAMG_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    }
  }
  return p;
}

static void free_one(Pool &pool, void *p) {
  if (pool.custom)
    pool.a.free(pool.a.ctx, p, (void *)pool.s);
  else
    (void)hipFree(p);
}

// Small requests are carved out of 32 MiB chunks (256-byte aligned); large
// ones get their own allocation. Only the latter are ever freed early.
void *Pool::raw(size_t bytes) {
  constexpr size_t kChunk = size_t(32) << 20, kAlign = 256;
  bytes = (bytes + kAlign - 1) / kAlign * kAlign;
  if (bytes >= kChunk / 4) {
    void *p = device_alloc(*this, bytes);
    live.push_back(p);
    return p;
  }
  if (bytes > chunk_left) {
    chunk_cur = static_cast<char *>(device_alloc(*this, kChunk));
    live.push_back(chunk_cur);
    chunks.push_back(chunk_cur);
    chunk_left = kChunk;
  }
  void *p = chunk_cur;
  chunk_cur += bytes;
  chunk_left -= bytes;
  return p;
}

void Pool::release(void *p) { deferred.push_back(p); }

void Pool::flush() {
  if (deferred.empty()) return;
  (void)hipStreamSynchronize(s);
  for (void *p : deferred) {
    for (size_t i = 0; i < live.size(); ++i)
      if (live[i] == p) {
        bool is_chunk = false;
        for (void *c : chunks) is_chunk |= (c == p);
        if (is_chunk) break;  // first carve of a chunk: keep the chunk
        live[i] = live.back();
        live.pop_back();
        free_one(*this, p);
        break;
      }
  }
  deferred.clear();
}

// Pinned blocks are recycled through a process-wide free list rather than
// freed, so a handle made per solve does not pay for pinning memory (nor a
// free that may synchronise the device); they last until the process ends.
namespace {
std::mutex g_pin_mu;
std::vector<int *> g_pin_free;
}  // namespace

int *Pool::pinned() {
  if (!hpin) {
    std::lock_guard<std::mutex> g(g_pin_mu);
    if (!g_pin_free.empty()) {
      hpin = g_pin_free.back();
      g_pin_free.pop_back();
    }
  }
  if (!hpin) HIPCHK(hipHostMalloc((void **)&hpin, sizeof(int) * kPinnedInts, hipHostMallocDefault));
  return hpin;
}

void Pool::release_all() {
  (void)hipStreamSynchronize(s);
  if (hpin) {
    std::lock_guard<std::mutex> g(g_pin_mu);
    g_pin_free.push_back(hpin);
    hpin = nullptr;
  }
  for (void *p : live) free_one(*this, p);
  live.clear();
  deferred.clear();
  chunks.clear();
  chunk_cur = nullptr;
  chunk_left = 0;
}

// record one profiling event (start or stop of a bracketed run of launches)
void profile_mark(bamg_handle *h, hipStream_t s, bool start) {
  if (start && h->prof_used + 2 > h->prof_ev.size()) {
    const size_t old = h->prof_ev.size(), grow = old ? old : 1024;
    h->prof_ev.resize(old + grow);
    for (size_t i = old; i < h->prof_ev.size(); ++i) HIPCHK(hipEventCreate(&h->prof_ev[i]));
  }
  HIPCHK(hipEventRecord(h->prof_ev[h->prof_used++], s));
  h->prof_stream = s;
}

}  // namespace bamg

// Wait for the validation work on the auxiliary stream and release it.
void bamg_handle::join_validation(bool wait_main) {
  if (!aux) return;
  (void)hipStreamSynchronize(aux);
  if (wait_main) (void)hipStreamSynchronize(pool.s);
  (void)hipEventDestroy(aux_ready);
  (void)hipEventDestroy(aux_done);
  (void)hipStreamDestroy(aux);
  aux = nullptr;
  aux_ready = aux_done = nullptr;
}

void bamg_handle::search_more() {
  if (!vdeferred || !aux || !vqueues) return;
  vdeferred = false;
  vlevels = bamg::reach_more(lv[0].B, lv[0].Bt, vvisited, vqueues, vflag, vlevels, aux);
}

int bamg_handle::finish_validation() {
  if (!aux) return vstatus;
  join_validation(true);
  vstatus = validation_result();
  if (vvisited) pool.release(vvisited);
  if (vqueues) pool.release(vqueues);
  vvisited = nullptr;
  vqueues = nullptr;
  pool.flush();
  return vstatus;
}

// Outcome of the input validation (BAMG_OK when it was not requested).
int bamg_handle::validation_result() {
  if (!vflag) return BAMG_OK;
  try {
    // levels of the search beyond those enqueued with it, if it needs them
    if (vlevels > 0 && vqueues)
      bamg::reach_finish(lv[0].B, lv[0].Bt, vvisited, vqueues, vflag, vlevels, pool.s);
    vlevels = 0;
  } catch (...) {
    return BAMG_E_DEVICE;
  }
  int hv[4] = {0, 0, 0, 0};
  if (hipMemcpyAsync(hv, vflag, sizeof(hv), hipMemcpyDeviceToHost, pool.s) != hipSuccess ||
      hipStreamSynchronize(pool.s) != hipSuccess)
    return BAMG_E_DEVICE;
  return bamg::validation_status(hv, lv.empty() ? 0 : lv[0].n);
}

namespace bamg {

static bamg_status translate(const Error &e) {
  g_last_error = e.msg;
  return e.code;
}

}  // namespace bamg

using namespace bamg;

#define BAMG_TRY try {
#define BAMG_CATCH                                                                          \
  }                                                                                         \
  catch (const Error &e) {                                                                  \
    return translate(e);                                                                    \
  }                                                                                         \
  catch (const std::bad_alloc &) {                                                          \
    g_last_error = "host allocation failed";                                                \
    return BAMG_E_NOMEM;                                                                    \
  }                                                                                         \
  catch (...) {                                                                             \
    g_last_error = "unexpected exception";                                                  \
    return BAMG_E_DEVICE;                                                                   \
  }

extern "C" {

bamg_status bamg_default_options(bamg_options *o) {
  if (!o) return BAMG_E_ARG;
  std::memset(o, 0, sizeof(*o));
  o->r = 8;
  o->setup_cycles = 1;
  o->nu_pre = 3;
  o->nu_post = 3;
  o->nu_setup = 3;
  o->omega = 0.7;
  o->max_interp = 4;
  o->max_levels = 16;
  o->coarse_max = 289;
  o->coarsening = BAMG_COARSEN_GEOMETRIC;
  o->seed = 14024001ULL;
  o->smoother = BAMG_SMOOTH_JACOBI;
  o->precision = BAMG_PRECISION_FP64;
  o->interp_rule = 1;
  o->validate = 1;
  o->use_graph = 0;
  o->fuse_last_level = 1;
  o->cycle = BAMG_CYCLE_V;
  o->mu = 1;
  o->restriction = 0;
  o->cr_theta = 0.8;
  o->cr_beta = 0.7;
  o->cr_sweeps = 5;
  o->cr_rounds = 10;
  o->flexible = 0;
  return BAMG_OK;
}

const char *bamg_status_string(bamg_status s) {
  switch (s) {
    case BAMG_OK: return "ok";
    case BAMG_NOT_CONVERGED: return "not converged";
    case BAMG_E_ARG: return "invalid argument";
    case BAMG_E_NOT_STOCHASTIC: return "matrix is not column stochastic";
    case BAMG_E_REDUCIBLE: return "chain is reducible";
    case BAMG_E_BAD_DIAG: return "zero diagonal";
    case BAMG_E_COARSE: return "coarsest level solve failed";
    case BAMG_E_BREAKDOWN: return "GMRES breakdown";
    case BAMG_E_NONFINITE: return "non-finite value";
    case BAMG_E_DEVICE: return "HIP error";
    case BAMG_E_NOMEM: return "out of device memory";
    default: return "unknown status";
  }
}

const char *bamg_last_error(void) { return g_last_error.c_str(); }

static bamg_status check_options(const bamg_options *o) {
  if (o->r < 2 || o->r > 16) return BAMG_E_ARG;
  if (o->setup_cycles < 1 || o->setup_cycles > 16) return BAMG_E_ARG;
  if (o->nu_pre < 0 || o->nu_post < 0 || o->nu_setup < 0) return BAMG_E_ARG;
  if (o->nu_pre > 64 || o->nu_post > 64 || o->nu_setup > 256) return BAMG_E_ARG;
  if (!(o->omega > 0.0 && o->omega < 2.0)) return BAMG_E_ARG;
  if (o->max_interp < 1 || o->max_interp > 8) return BAMG_E_ARG;
  if (o->max_levels < 2 || o->max_levels > 32) return BAMG_E_ARG;
  if (o->coarse_max < 1 || o->coarse_max > 2048) return BAMG_E_ARG;
  if (o->smoother != BAMG_SMOOTH_JACOBI && o->smoother != BAMG_SMOOTH_KACZMARZ) return BAMG_E_ARG;
  if (o->precision != BAMG_PRECISION_FP64 && o->precision != BAMG_PRECISION_MIXED) return BAMG_E_ARG;
  if (o->interp_rule != 0 && o->interp_rule != 1) return BAMG_E_ARG;
  if (o->validate < 0 || o->validate > 3) return BAMG_E_ARG;
  if (o->cycle < BAMG_CYCLE_V || o->cycle > BAMG_CYCLE_NONE) return BAMG_E_ARG;
  if (o->mu < 1 || o->mu > 8) return BAMG_E_ARG;
  if (o->restriction != 0 && o->restriction != 1) return BAMG_E_ARG;
  if (o->profile_setup != 0 && o->profile_setup != 1) return BAMG_E_ARG;
  if (o->learned_max_iters < 0) return BAMG_E_ARG;
  if (o->coarsening < BAMG_COARSEN_GEOMETRIC || o->coarsening > BAMG_COARSEN_CR) return BAMG_E_ARG;
  if (!std::isfinite(o->cr_theta) || !(o->cr_beta >= 0.0 && o->cr_beta <= 1.0) ||
      o->cr_sweeps < 1 || o->cr_sweeps > 64 || o->cr_rounds < 0 || o->cr_rounds > 64)
    return BAMG_E_ARG;
  if (o->flexible != 0 && o->flexible != 1) return BAMG_E_ARG;
  if (o->learned < BAMG_LEARNED_OFF || o->learned > BAMG_LEARNED_RECORD) return BAMG_E_ARG;
  if (o->learned == BAMG_LEARNED_USE && !o->mlp) return BAMG_E_ARG;
  return BAMG_OK;
}

bamg_status bamg_setup(const bamg_csr *A, const bamg_geometry *geom, const bamg_options *opt,
                       const bamg_allocator *alloc, void *hip_stream, bamg_handle **out) {
  if (!A || !opt || !out || !A->row_ptr || !A->col_idx || !A->val) return BAMG_E_ARG;
  if (A->n < 2 || A->n > 0x7fffffffLL || A->nnz < 1 || A->nnz > 0x7fffffffLL) return BAMG_E_ARG;
  bamg_status st = check_options(opt);
  if (st != BAMG_OK) return st;
  if (geom && geom->kind != BAMG_GEOM_NONE) {
    if (geom->kind == BAMG_GEOM_GRID2D && (int64_t)geom->nx * geom->ny != A->n) return BAMG_E_ARG;
    if (geom->kind == BAMG_GEOM_LINE && geom->nx != A->n) return BAMG_E_ARG;
    if (geom->kind != BAMG_GEOM_GRID2D && geom->kind != BAMG_GEOM_LINE) return BAMG_E_ARG;
  }
  if (alloc && (!alloc->alloc || !alloc->free)) return BAMG_E_ARG;
  bamg_handle *h = new (std::nothrow) bamg_handle();
  if (!h) return BAMG_E_NOMEM;
  h->opt = *opt;
  h->prec = opt->precision == BAMG_PRECISION_MIXED ? 1 : 0;
  h->use_graph = opt->use_graph ? 1 : 0;
  h->last_fused = opt->fuse_last_level ? 1 : 0;
  h->pool.s = (hipStream_t)hip_stream;
  if (opt->profile_setup) h->prof_kernel = BAMG_PROFILE_COARSEST_SVD;
  if (alloc) {
    h->pool.a = *alloc;
    h->pool.custom = true;
  }
  const auto t0 = std::chrono::steady_clock::now();
  try {
    if (h->prec == 0)
      setup_all<double>(h, A, geom);
    else
      setup_all<float>(h, A, geom);
    if (h->prec != 0) {
      h->vb = h->pool.get<float>(h->lv[0].n);
      h->vx = h->pool.get<float>(h->lv[0].n);
    }
  } catch (const Error &e) {
    // an invalid input explains later failures: report the validation first
    h->join_validation(true);
    const int vst = e.code == BAMG_E_DEVICE || e.code == BAMG_E_NOMEM ? BAMG_OK
                                                                       : h->validation_result();
    h->pool.release_all();
    delete h;
    if (vst != BAMG_OK) return translate(Error{vst, "transition matrix rejected"});
    return translate(e);
  } catch (...) {
    h->join_validation(true);
    h->pool.release_all();
    delete h;
    g_last_error = "unexpected exception in setup";
    return BAMG_E_DEVICE;
  }
  h->t_setup_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h;
  return BAMG_OK;
}

bamg_status bamg_setup_from_levels(int32_t nlevels, const bamg_level_ops *levels,
                                   const double *coarse_pinv, const double *x0,
                                   const bamg_options *opt, const bamg_allocator *alloc,
                                   void *hip_stream, bamg_handle **out) {
  if (nlevels < 2 || nlevels > 32 || !levels || !coarse_pinv || !x0 || !opt || !out)
    return BAMG_E_ARG;
  if (opt->nu_pre < 0 || opt->nu_post < 0 || opt->nu_pre > 64 || opt->nu_post > 64 ||
      !(opt->omega > 0.0 && opt->omega < 2.0) ||
      (opt->smoother != BAMG_SMOOTH_JACOBI && opt->smoother != BAMG_SMOOTH_KACZMARZ) ||
      (opt->precision != BAMG_PRECISION_FP64 && opt->precision != BAMG_PRECISION_MIXED) ||
      opt->cycle < BAMG_CYCLE_V || opt->cycle > BAMG_CYCLE_NONE)
    return BAMG_E_ARG;
  if (alloc && (!alloc->alloc || !alloc->free)) return BAMG_E_ARG;
  bamg_handle *h = new (std::nothrow) bamg_handle();
  if (!h) return BAMG_E_NOMEM;
  h->opt = *opt;
  h->opt.learned = BAMG_LEARNED_OFF;
  h->opt.mlp = nullptr;
  h->imported = 1;
  h->prec = opt->precision == BAMG_PRECISION_MIXED ? 1 : 0;
  h->use_graph = opt->use_graph ? 1 : 0;
  h->last_fused = opt->fuse_last_level ? 1 : 0;
  h->pool.s = (hipStream_t)hip_stream;
  if (alloc) {
    h->pool.a = *alloc;
    h->pool.custom = true;
  }
  try {
    if (h->prec == 0)
      import_all<double>(h, nlevels, levels, coarse_pinv, x0);
    else
      import_all<float>(h, nlevels, levels, coarse_pinv, x0);
  } catch (const Error &e) {
    (void)hipStreamSynchronize(h->pool.s);
    h->pool.release_all();
    delete h;
    return translate(e);
  } catch (...) {
    (void)hipStreamSynchronize(h->pool.s);
    h->pool.release_all();
    delete h;
    g_last_error = "unexpected exception in bamg_setup_from_levels";
    return BAMG_E_DEVICE;
  }
  *out = h;
  return BAMG_OK;
}

// A validation still running beside the hierarchy (validate = 3) is joined
// when a computation on it ends; its failure replaces that result.
static bamg_status with_validation(bamg_handle *h, bamg_status st) {
  const int vst = h->finish_validation();
  if (vst != BAMG_OK) {
    g_last_error = "transition matrix rejected";
    return (bamg_status)vst;
  }
  return st;
}

static bamg_status vcycle_impl(bamg_handle *h, const void *b, void *x, int32_t dtype,
                               void *hip_stream);

bamg_status bamg_vcycle(bamg_handle *h, const void *b, void *x, int32_t dtype, void *hip_stream) {
  if (!h || !b || !x || b == x) return BAMG_E_ARG;
  if (dtype != BAMG_DTYPE_F64 && dtype != BAMG_DTYPE_F32) return BAMG_E_ARG;
  if (dtype == BAMG_DTYPE_F32 && h->prec == 0) return BAMG_E_ARG;
  return with_validation(h, vcycle_impl(h, b, x, dtype, hip_stream));
}

static bamg_status vcycle_impl(bamg_handle *h, const void *b, void *x, int32_t dtype,
                               void *hip_stream) {
  BAMG_TRY
  hipStream_t s = (hipStream_t)hip_stream;
  const int n = h->lv[0].n;
  if (h->prec == 0) {
    vcycle_run<double>(h, (const double *)b, (double *)x, s);
  } else if (dtype == BAMG_DTYPE_F32) {
    vcycle_run<float>(h, (const float *)b, (float *)x, s);
  } else {
    convert<double, float>((float *)h->vb, (const double *)b, n, s);
    vcycle_run<float>(h, (const float *)h->vb, (float *)h->vx, s);
    convert<float, double>((double *)x, (const float *)h->vx, n, s);
  }
  return BAMG_OK;
  BAMG_CATCH
}

namespace {

__global__ void k_identity_minus(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                 const double *__restrict__ bv, double *__restrict__ av) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) av[k] = (ci[k] == i ? 1.0 : 0.0) - bv[k];
}

// The iteration fallback of the learned form: a hierarchy set up from the
// same chain (A = I - B, B's pattern and FP64 values) with the same options
// but exact LS fits replaces h's; the old one is freed.
void rebuild_exact(bamg_handle *h, hipStream_t s) {
  Level &L0 = h->lv[0];
  const int n = L0.n, nnz = L0.B.nnz;
  double *av = h->pool.get<double>(nnz);
  k_identity_minus<<<ceil_div(n, 256), 256, 0, s>>>(n, L0.B.rp, L0.B.ci, h->B64, av);
  LAUNCHCHK();
  bamg_csr A{n, nnz, L0.B.rp, L0.B.ci, av, 1};
  bamg_geometry g{L0.gkind, L0.nx, L0.gkind == BAMG_GEOM_GRID2D ? L0.ny : 0};
  if (g.kind == BAMG_GEOM_LINE) g.nx = n;
  bamg_options o = h->opt;
  o.learned = BAMG_LEARNED_OFF;
  o.mlp = nullptr;
  o.validate = 0;  // the chain was validated by the first setup
  o.profile_setup = 0;
  bamg_handle *h2 = nullptr;
  const bamg_status st = bamg_setup(&A, g.kind ? &g : nullptr, &o,
                                    h->pool.custom ? &h->pool.a : nullptr, s, &h2);
  if (st != BAMG_OK) fail(st, "rebuilding the hierarchy with exact LS fits failed");
  h2->t_setup_ms += h->t_setup_ms;
  std::swap(*h, *h2);
  bamg_destroy(h2);  // the learned hierarchy (and B's arrays A borrowed)
}

}  // namespace

static bamg_status gmres_impl(bamg_handle *h, void *x, int32_t restart, double tol,
                              int32_t max_iters, int32_t use_x0, bamg_solve_info *info,
                              void *hip_stream);

// Learned-row counts of the hierarchy a solve ended on; a read that fails
// leaves them 0 (the solve's own status is what the caller gets).
static void learned_counts(const bamg_handle *h, hipStream_t s, bamg_solve_info *inf) {
  inf->mlp_rows = inf->ls_fallbacks = 0;
  if (!h->lcount) return;
  int c[2] = {0, 0};
  if (hipMemcpyAsync(c, h->lcount, sizeof(c), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return;
  inf->mlp_rows = c[0];
  inf->ls_fallbacks = c[1];
}

bamg_status bamg_gmres_solve(bamg_handle *h, void *x, int32_t restart, double tol,
                             int32_t max_iters, int32_t use_x0, bamg_solve_info *info,
                             void *hip_stream) {
  if (!h || !x || restart < 1 || restart > 255 || max_iters < 0 || !(tol > 0.0)) return BAMG_E_ARG;
  return with_validation(h, gmres_impl(h, x, restart, tol, max_iters, use_x0, info, hip_stream));
}

static bamg_status gmres_impl(bamg_handle *h, void *x, int32_t restart, double tol,
                              int32_t max_iters, int32_t use_x0, bamg_solve_info *info,
                              void *hip_stream) {
  BAMG_TRY
  hipStream_t s = (hipStream_t)hip_stream;
  bamg_solve_info local{};
  bamg_solve_info *inf = info ? info : &local;
  const bool fb = h->opt.learned == BAMG_LEARNED_USE && h->opt.learned_max_iters > 0 &&
                  !h->imported && h->opt.learned_max_iters < max_iters;
  const int first = fb ? h->opt.learned_max_iters : max_iters;
  bool fell_back = false;
  for (int part = 0; part < 2; ++part) {
    hipStream_t keep = h->pool.s;
    h->pool.s = s;
    bool more = false;
    bamg_solve_info cur{};
    try {
      gmres_run(h, (double *)x, restart, tol, part == 0 ? first : max_iters - first,
                part == 0 ? use_x0 : 1, &cur, s);
    } catch (const Error &e) {
      h->pool.s = keep;
      if (e.code != BAMG_NOT_CONVERGED || !fb || part == 1) {
        if (part == 1) {  // report the whole solve with the status of its second part
          cur.iterations += inf->iterations;
          cur.restarts += inf->restarts;
          cur.t_solve_ms += inf->t_solve_ms;
        }
        cur.setup_cycles = h->opt.setup_cycles;
        cur.mlp_fallback = fell_back ? 1 : 0;
        cur.t_setup_ms = h->t_setup_ms;
        *inf = cur;
        if (e.code == BAMG_NOT_CONVERGED) learned_counts(h, s, inf);
        throw;
      }
      more = true;
    }
    h->pool.s = keep;
    if (part == 1) {
      cur.iterations += inf->iterations;
      cur.restarts += inf->restarts;
      cur.t_solve_ms += inf->t_solve_ms;
    }
    *inf = cur;
    if (!more) break;
    // the rebuilt handle replaces this one: settle a validation still running
    const int vst = h->finish_validation();
    if (vst != BAMG_OK) fail(vst, "transition matrix rejected");
    rebuild_exact(h, s);
    fell_back = true;
  }
  inf->setup_cycles = h->opt.setup_cycles;
  inf->mlp_fallback = fell_back ? 1 : 0;
  inf->t_setup_ms = h->t_setup_ms;
  learned_counts(h, s, inf);
  return BAMG_OK;
  BAMG_CATCH
}

bamg_status bamg_set_cycle(bamg_handle *h, int32_t cycle) {
  if (!h || cycle < BAMG_CYCLE_V || cycle > BAMG_CYCLE_NONE) return BAMG_E_ARG;
  if (h->opt.cycle != cycle && h->vc_exec) {
    (void)hipGraphExecDestroy(h->vc_exec);  // captured with the old shape
    h->vc_exec = nullptr;
  }
  h->opt.cycle = cycle;
  return BAMG_OK;
}

bamg_status bamg_hierarchy_info(const bamg_handle *h, int32_t *levels, int64_t *n_l,
                                int64_t *nnz_l, double *oc, double *og) {
  if (!h) return BAMG_E_ARG;
  if (levels) *levels = h->L;
  double sb = 0, sn = 0;
  for (int l = 0; l < h->L; ++l) {
    if (n_l) n_l[l] = h->lv[l].n;
    if (nnz_l) nnz_l[l] = h->lv[l].B.nnz;
    sb += h->lv[l].B.nnz;
    sn += h->lv[l].n;
  }
  if (oc) *oc = sb / h->lv[0].B.nnz;
  if (og) *og = sn / h->lv[0].n;
  return BAMG_OK;
}

static bool level_pick(const bamg_handle *h, int l, int what, const Csr **A, const void **v) {
  if (l < 0 || l >= h->L || what < 0 || what > 6) return false;
  if (h->imported && (what == 1 || what == 2 || what == 3 || what == 6)) return false;
  const Level &L = h->lv[l];
  if (what >= 4 && l == h->L - 1) return false;
  switch (what) {
    case 0: *A = &L.B; *v = L.Bv; break;
    case 1: *A = &L.Bt; *v = L.Btv; break;
    case 2: *A = &L.M; *v = L.Mv; break;
    case 3: *A = &L.M; *v = L.Nv; break;
    case 4: *A = &L.P; *v = L.Pv; break;
    case 5: *A = &L.Pc; *v = L.Qv; break;
    default: *A = &L.P; *v = L.Qtv; break;
  }
  return true;
}

bamg_status bamg_level_nnz(const bamg_handle *h, int32_t l, int32_t what, int64_t *rows,
                           int64_t *nnz) {
  if (!h) return BAMG_E_ARG;
  const Csr *A;
  const void *v;
  if (!level_pick(h, l, what, &A, &v)) return BAMG_E_ARG;
  if (rows) *rows = A->nr;
  if (nnz) *nnz = A->nnz;
  return BAMG_OK;
}

bamg_status bamg_level_csr(const bamg_handle *h, int32_t l, int32_t what, int32_t *row_ptr,
                           int32_t *col_idx, double *val) {
  if (!h) return BAMG_E_ARG;
  const Csr *A;
  const void *v;
  if (!level_pick(h, l, what, &A, &v)) return BAMG_E_ARG;
  BAMG_TRY
  if (row_ptr) HIPCHK(hipMemcpy(row_ptr, A->rp, sizeof(int) * (A->nr + 1), hipMemcpyDeviceToHost));
  if (col_idx) HIPCHK(hipMemcpy(col_idx, A->ci, sizeof(int) * A->nnz, hipMemcpyDeviceToHost));
  if (val) {
    if (h->prec == 0) {
      HIPCHK(hipMemcpy(val, v, sizeof(double) * A->nnz, hipMemcpyDeviceToHost));
    } else {
      std::vector<float> tmp(A->nnz);
      HIPCHK(hipMemcpy(tmp.data(), v, sizeof(float) * A->nnz, hipMemcpyDeviceToHost));
      for (int i = 0; i < A->nnz; ++i) val[i] = tmp[i];
    }
  }
  return BAMG_OK;
  BAMG_CATCH
}

bamg_status bamg_level_cf(const bamg_handle *h, int32_t l, int32_t *cf, int32_t *cidx) {
  if (!h || h->imported || l < 0 || l >= h->L - 1) return BAMG_E_ARG;
  BAMG_TRY
  const Level &L = h->lv[l];
  if (cf) HIPCHK(hipMemcpy(cf, L.cf, sizeof(int) * L.n, hipMemcpyDeviceToHost));
  if (cidx) HIPCHK(hipMemcpy(cidx, L.cidx, sizeof(int) * L.n, hipMemcpyDeviceToHost));
  return BAMG_OK;
  BAMG_CATCH
}

bamg_status bamg_level_vectors(const bamg_handle *h, int32_t l, double *U, double *V) {
  if (!h || h->imported || l < 0 || l >= h->L) return BAMG_E_ARG;
  BAMG_TRY
  const Level &L = h->lv[l];
  const size_t nr = (size_t)L.n * h->opt.r;
  for (int side = 0; side < 2; ++side) {
    double *dst = side ? V : U;
    const void *src = side ? L.V : L.U;
    if (!dst) continue;
    if (h->prec == 0) {
      HIPCHK(hipMemcpy(dst, src, sizeof(double) * nr, hipMemcpyDeviceToHost));
    } else {
      std::vector<float> tmp(nr);
      HIPCHK(hipMemcpy(tmp.data(), src, sizeof(float) * nr, hipMemcpyDeviceToHost));
      for (size_t i = 0; i < nr; ++i) dst[i] = tmp[i];
    }
  }
  return BAMG_OK;
  BAMG_CATCH
}

bamg_status bamg_sigma(const bamg_handle *h, double *sigma) {
  if (!h || !sigma) return BAMG_E_ARG;
  BAMG_TRY
  HIPCHK(hipMemcpy(sigma, h->sigma, sizeof(double) * h->opt.r, hipMemcpyDeviceToHost));
  return BAMG_OK;
  BAMG_CATCH
}

bamg_status bamg_x0(const bamg_handle *h, void *x_device, void *hip_stream) {
  if (!h || !x_device) return BAMG_E_ARG;
  BAMG_TRY
  hipStream_t s = (hipStream_t)hip_stream;
  HIPCHK(hipMemcpyAsync(x_device, h->x0, sizeof(double) * h->lv[0].n, hipMemcpyDeviceToDevice, s));
  return BAMG_OK;
  BAMG_CATCH
}

bamg_status bamg_coarse_pinv(const bamg_handle *h, double *bdag) {
  if (!h || !bdag) return BAMG_E_ARG;
  BAMG_TRY
  const int n = h->lv[h->L - 1].n;
  HIPCHK(hipMemcpy(bdag, h->bdag, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToHost));
  return BAMG_OK;
  BAMG_CATCH
}

bamg_status bamg_vcycle_bytes(const bamg_handle *h, double *bytes) {
  if (!h || !bytes) return BAMG_E_ARG;
  const double s = h->prec ? 4.0 : 8.0;
  const int nu1 = h->opt.nu_pre, nu2 = h->opt.nu_post;
  double tot = 0.0;
  for (int l = 0; l + 1 < h->L; ++l) {
    const Level &L = h->lv[l];
    const double n = L.n, nnz = L.B.nnz, nc = h->lv[l + 1].n, np = L.P.nnz, nq = L.Pc.nnz;
    const double sweep = nnz * (s + 4) + 4 * (n + 1) + 4 * s * n;
    const double first = 3 * s * n;
    const double resid = nnz * (s + 4) + 4 * (n + 1) + 3 * s * n;
    const double restr = nq * (s + 4) + 4 * (nc + 1) + s * (n + nc);
    const double prol = np * (s + 4) + 4 * (n + 1) + s * (nc + 2 * n);
    const int sweeps = (nu1 > 0 ? nu1 - 1 : 0) + nu2;
    tot += sweeps * sweep + (nu1 > 0 ? first : 0) + resid + restr + prol;
  }
  const double nL = h->lv[h->L - 1].n;
  tot += 8.0 * nL * nL + 2 * s * nL;
  *bytes = tot;
  return BAMG_OK;
}

bamg_status bamg_level_lanes(const bamg_handle *h, int32_t l, int32_t *lanes) {
  if (!h || !lanes || l < 0 || l >= h->L) return BAMG_E_ARG;
  const Level &L = h->lv[l];
  *lanes = L.lanes > 0 ? L.lanes : sweep_lanes_default(L.n, L.B.nnz);
  return BAMG_OK;
}

bamg_status bamg_level_set_lanes(bamg_handle *h, int32_t l, int32_t lanes) {
  if (!h || l < 0 || l >= h->L - 1) return BAMG_E_ARG;
  if (lanes != 1 && lanes != 2 && lanes != 4) return BAMG_E_ARG;
  if (h->vc_exec) return BAMG_E_ARG;  // a captured V-cycle keeps its launches
  h->lv[l].lanes = lanes;
  return BAMG_OK;
}

bamg_status bamg_level_threads(const bamg_handle *h, int32_t l, int32_t *threads) {
  if (!h || !threads || l < 0 || l >= h->L - 1) return BAMG_E_ARG;
  *threads = h->lv[l].threads > 0 ? h->lv[l].threads : 256;
  return BAMG_OK;
}

bamg_status bamg_level_set_threads(bamg_handle *h, int32_t l, int32_t threads) {
  if (!h || l < 0 || l >= h->L - 1) return BAMG_E_ARG;
  if (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024)
    return BAMG_E_ARG;
  if (h->vc_exec) return BAMG_E_ARG;  // a captured V-cycle keeps its launches
  h->lv[l].threads = threads;
  return BAMG_OK;
}

bamg_status bamg_kernel_profile_begin(bamg_handle *h, int32_t kernel) {
  if (!h || kernel != BAMG_PROFILE_FINEST_SWEEP) return BAMG_E_ARG;
  h->prof_kernel = kernel;
  h->prof_used = 0;
  h->prof_bytes = 0.0;
  h->prof_launches = 0;
  return BAMG_OK;
}

bamg_status bamg_kernel_profile_end(bamg_handle *h, int64_t *launches, double *ms_total,
                                    double *bytes_total) {
  if (!h) return BAMG_E_ARG;
  BAMG_TRY
  double ms = 0.0;
  if (h->prof_used) HIPCHK(hipStreamSynchronize(h->prof_stream));
  for (size_t i = 0; i + 1 < h->prof_used; i += 2) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, h->prof_ev[i], h->prof_ev[i + 1]));
    ms += t;
  }
  if (launches) *launches = (int64_t)h->prof_launches;
  if (ms_total) *ms_total = ms;
  if (bytes_total) *bytes_total = h->prof_bytes;
  h->prof_kernel = -1;
  h->prof_used = 0;
  return BAMG_OK;
  BAMG_CATCH
}

bamg_status bamg_mlp_create(const float *params, bamg_mlp **out) {
  if (!params || !out) return BAMG_E_ARG;
  bamg_mlp *m = new (std::nothrow) bamg_mlp();
  if (!m) return BAMG_E_NOMEM;
  const size_t pb = sizeof(float) * BAMG_MLP_NPARAMS;
  try {
    HIPCHK(hipMalloc(&m->p, pb));
    HIPCHK(hipMalloc(&m->m, pb));
    HIPCHK(hipMalloc(&m->v, pb));
    HIPCHK(hipMalloc(&m->wb, sizeof(__bf16) * (BAMG_MLP_HIDDEN * BAMG_MLP_IN +
                                               BAMG_MLP_HIDDEN * BAMG_MLP_HIDDEN +
                                               16 * BAMG_MLP_HIDDEN)));
    HIPCHK(hipMemcpy(m->p, params, pb, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(m->m, 0, pb));
    HIPCHK(hipMemset(m->v, 0, pb));
    mlp_refresh_bf16(m, nullptr);
    HIPCHK(hipDeviceSynchronize());
  } catch (const Error &e) {
    bamg_mlp_destroy(m);
    return translate(e);
  }
  *out = m;
  return BAMG_OK;
}

bamg_status bamg_mlp_get_params(const bamg_mlp *m, float *params) {
  if (!m || !params) return BAMG_E_ARG;
  BAMG_TRY
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(params, m->p, sizeof(float) * BAMG_MLP_NPARAMS, hipMemcpyDeviceToHost));
  return BAMG_OK;
  BAMG_CATCH
}

void bamg_mlp_destroy(bamg_mlp *m) {
  if (!m) return;
  void *ps[] = {m->p, m->m, m->v, m->wb};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  delete m;
}

bamg_status bamg_mlp_forward(const bamg_mlp *m, const float *X, int64_t npts, float *Y,
                             int32_t mode, void *hip_stream) {
  if (!m || npts < 0 || (npts > 0 && (!X || !Y)) || (mode != 0 && mode != 1)) return BAMG_E_ARG;
  BAMG_TRY
  mlp_forward(m, X, (long)npts, Y, mode, (hipStream_t)hip_stream);
  return BAMG_OK;
  BAMG_CATCH
}

bamg_status bamg_mlp_loss_grad(const bamg_mlp *m, const float *X, const float *T,
                               const float *M, int64_t npts, double *loss, float *grad,
                               void *hip_stream) {
  if (!m || !X || !T || !M || npts < 1 || !loss || !grad) return BAMG_E_ARG;
  BAMG_TRY
  *loss = mlp_loss_grad(m, X, T, M, (long)npts, grad, (hipStream_t)hip_stream);
  return BAMG_OK;
  BAMG_CATCH
}

bamg_status bamg_mlp_loss_grad_noalloc(const bamg_mlp *m, const float *X, const float *T,
                                       const float *M, int64_t npts, double *loss, float *grad,
                                       void *hip_stream) {
  if (!m || !X || !T || !M || npts < 1 || !loss || !grad) return BAMG_E_ARG;
  BAMG_TRY
  *loss = mlp_loss_grad_noalloc(m, X, T, M, (long)npts, grad, (hipStream_t)hip_stream);
  return BAMG_OK;
  BAMG_CATCH
}

bamg_status bamg_mlp_train(bamg_mlp *m, const float *X, const float *T, const float *M,
                           int64_t npts, int32_t batch, int32_t epochs, float lr,
                           double *loss_per_epoch, void *hip_stream) {
  if (!m || !X || !T || !M || npts < 1 || batch < 1 || epochs < 0 || !(lr > 0.f))
    return BAMG_E_ARG;
  BAMG_TRY
  mlp_train(m, X, T, M, (long)npts, batch, epochs, lr, loss_per_epoch, (hipStream_t)hip_stream);
  return BAMG_OK;
  BAMG_CATCH
}

bamg_status bamg_harvest(const bamg_handle *h, int32_t level, float *X, float *T, float *M,
                         int64_t *nF, void *hip_stream) {
  if (!h || !nF || level < 0 || level >= h->L - 1) return BAMG_E_ARG;
  const Level &L = h->lv[level];
  if (h->opt.learned != BAMG_LEARNED_RECORD || L.nF < 0) return BAMG_E_ARG;
  *nF = L.nF;
  if (!X && !T && !M) return BAMG_OK;
  if (!X || !T || !M) return BAMG_E_ARG;
  BAMG_TRY
  hipStream_t s = (hipStream_t)hip_stream;
  if (L.nF > 0) {
    HIPCHK(hipMemcpyAsync(X, L.feat, sizeof(float) * (size_t)L.nF * BAMG_MLP_IN,
                          hipMemcpyDeviceToDevice, s));
    if (h->prec == 0)
      mlp_targets<double>(L, (const double *)L.Pv, T, M, s);
    else
      mlp_targets<float>(L, (const float *)L.Pv, T, M, s);
  }
  return BAMG_OK;
  BAMG_CATCH
}

bamg_status bamg_learned_stats(const bamg_handle *h, int64_t *mlp_rows, int64_t *fallback_rows) {
  if (!h || !mlp_rows || !fallback_rows) return BAMG_E_ARG;
  int c[2] = {0, 0};
  BAMG_TRY
  if (h->lcount) {
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(c, h->lcount, sizeof(c), hipMemcpyDeviceToHost));
  }
  *mlp_rows = c[0];
  *fallback_rows = c[1];
  return BAMG_OK;
  BAMG_CATCH
}

void bamg_destroy(bamg_handle *h) {
  if (!h) return;
  h->join_validation(true);  // the search may still use the handle's memory
  for (hipEvent_t e : h->prof_ev) (void)hipEventDestroy(e);
  if (h->vc_exec) (void)hipGraphExecDestroy(h->vc_exec);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  h->pool.release_all();
  if (h->hred) (void)hipHostFree(h->hred);
  for (hipEvent_t e : h->gm_ev)
    if (e) (void)hipEventDestroy(e);
  delete h;
}

}  // extern "C"
