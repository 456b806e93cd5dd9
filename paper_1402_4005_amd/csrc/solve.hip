// Host orchestration of the solve phase: the V-cycle preconditioner
// (Sections 3 and 6) and GMRES(m) on the residual equation (Section 6) with
// the stopping test of Section 7.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "bamg_internal.h"
#include "device_common.h"

namespace bamg {

namespace {

// y = z + A x (the prolongation written into the other smoothing buffer)
template <class T>
__global__ void k_spmv_add_into(int nr, const int *__restrict__ rp, const int *__restrict__ ci,
                                const T *__restrict__ val, const T *__restrict__ x,
                                const T *__restrict__ z, T *__restrict__ y) {
  int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= nr) return;
  T s = 0;
  for (int a = rp[i]; a < rp[i + 1]; ++a) s += val[a] * x[ci[a]];
  y[i] = z[i] + s;
}

template <class T>
void smooth_steps(bamg_handle *h, Level &L, const T *b, T *x, int steps, bool from_zero,
                  hipStream_t s) {
  if (steps <= 0) {
    if (from_zero) fill<T>(x, (T)0, L.n, s);
    return;
  }
  if (h->opt.smoother == BAMG_SMOOTH_KACZMARZ) {
    if (from_zero) fill<T>(x, (T)0, L.n, s);
    for (int it = 0; it < steps; ++it)
      for (size_t c = 0; c + 1 < L.offB.size(); ++c)
        kaczmarz_colour<T>(L.B, (const T *)L.Bv, (const T *)L.rowinvB, L.ordB + L.offB[c],
                           L.offB[c + 1] - L.offB[c], b, x, s);
    return;
  }
  // weighted Jacobi, ping-pong between x and the level's spare buffer so the
  // last step lands in x
  const T om = (T)h->opt.omega;
  T *spare = (T *)L.tb;
  T *cur = x, *oth = spare;
  if (from_zero) {
    // the first two sweeps in one kernel (one if only one is asked for)
    const int done = steps >= 2 ? 2 : 1;
    T *first = ((steps - done) % 2 == 0) ? x : spare;
    if (done == 2)
      jacobi2_from_zero<T>(L.B, (const T *)L.Bv, (const T *)L.dinv, om, b, first, L.lanes, s,
                        L.threads);
    else
      jacobi<T>(L.B, (const T *)L.Bv, (const T *)L.dinv, om, b, nullptr, first, L.lanes, s,
                L.threads);
    cur = first;
    oth = first == x ? spare : x;
    steps -= done;
  } else if (steps % 2 == 1) {
    // odd count from x: the caller provided x in the spare buffer instead
    cur = spare;
    oth = x;
  }
  // profiled: one event pair around the run of back-to-back sweeps
  const bool prof = h->prof_kernel == BAMG_PROFILE_FINEST_SWEEP && &L == &h->lv[0] && steps > 0;
  if (prof) profile_mark(h, s, true);
  for (int it = 0; it < steps; ++it) {
    jacobi<T>(L.B, (const T *)L.Bv, (const T *)L.dinv, om, b, cur, oth, L.lanes, s, L.threads);
    std::swap(cur, oth);
  }
  if (prof) {
    profile_mark(h, s, false);
    const double sz = sizeof(T);
    h->prof_bytes += steps * ((double)L.B.nnz * (sz + 4) + 4.0 * (L.n + 1) + 4.0 * sz * L.n);
    h->prof_launches += steps;
  }
}

// One cycle of shape `type` on level l for B_l x = b (Section 3): from
// x = 0 when x_zero, else from the x passed in. Pre-smoothing, residual,
// restriction by Q, the coarse correction (one cycle of the same shape on
// level l + 1 from zero; a W-cycle a second one from the first's result, an
// F-cycle a V-cycle from it), interpolation by P, post-smoothing. On the
// coarsest level: x = B_L^+ b, or x + B_L^+ (b - B_L x) from a guess.
template <class T>
void cycle_level(bamg_handle *h, int l, int type, const T *b, T *x, bool x_zero,
                 hipStream_t s) {
  Level &L = h->lv[l];
  if (l == h->L - 1) {
    if (x_zero) {
      coarse_gemv<T>(h->bdag, L.n, b, x, s);
    } else {
      spmv<T>(L.B, (const T *)L.Bv, x, (T *)L.rb, b, 1, 0, s);  // r = b - B x
      coarse_gemv<T>(h->bdag, L.n, (const T *)L.rb, x, s, 1);   // x += B^+ r
    }
    return;
  }
  if (x_zero && type == BAMG_CYCLE_V && vcycle_last_level<T>(h, l, b, x, s))
    return;
  Level &C = h->lv[l + 1];
  const int nu1 = h->opt.nu_pre, nu2 = h->opt.nu_post;
  const bool jac = h->opt.smoother != BAMG_SMOOTH_KACZMARZ;
  if (!x_zero && jac && nu1 % 2 == 1)  // an odd count from a guess starts in the spare buffer
    HIPCHK(hipMemcpyAsync(L.tb, x, sizeof(T) * L.n, hipMemcpyDeviceToDevice, s));
  smooth_steps<T>(h, L, b, x, nu1, x_zero, s);
  spmv<T>(L.B, (const T *)L.Bv, x, (T *)L.rb, b, 1, L.lanes, s, L.threads);  // r = b - B x
  spmv<T>(L.Pc, (const T *)L.Qv, (const T *)L.rb, (T *)C.bb, nullptr, 0,
          transfer_lanes(L.Pc.nr, L.Pc.nnz), s);  // b_c = Q r
  cycle_level<T>(h, l + 1, type, (const T *)C.bb, (T *)C.xb, true, s);
  if (type == BAMG_CYCLE_W)
    cycle_level<T>(h, l + 1, BAMG_CYCLE_W, (const T *)C.bb, (T *)C.xb, false, s);
  else if (type == BAMG_CYCLE_F)
    cycle_level<T>(h, l + 1, BAMG_CYCLE_V, (const T *)C.bb, (T *)C.xb, false, s);
  if (jac && nu2 % 2 == 1) {
    // spare = x + P x_c, then an odd number of sweeps ends in x
    k_spmv_add_into<T><<<ceil_div(L.n, 256), 256, 0, s>>>(L.n, L.P.rp, L.P.ci, (const T *)L.Pv,
                                                          (const T *)C.xb, x, (T *)L.tb);
    LAUNCHCHK();
  } else {
    spmv<T>(L.P, (const T *)L.Pv, (const T *)C.xb, x, nullptr, 2, transfer_lanes(L.P.nr, L.P.nnz),
            s);  // x += P x_c
  }
  smooth_steps<T>(h, L, b, x, nu2, false, s);
}

}  // namespace

template <class T>
void vcycle_run(bamg_handle *h, const T *b, T *x, hipStream_t s) {
  if (h->opt.cycle == BAMG_CYCLE_NONE) {
    HIPCHK(hipMemcpyAsync(x, b, sizeof(T) * h->lv[0].n, hipMemcpyDeviceToDevice, s));
    return;
  }
  cycle_level<T>(h, 0, h->opt.cycle, b, x, true, s);
}
template void vcycle_run<double>(bamg_handle *, const double *, double *, hipStream_t);
template void vcycle_run<float>(bamg_handle *, const float *, float *, hipStream_t);

// C applied to an FP64 vector (FP32 inside for a mixed-precision handle)
static void precondition(bamg_handle *h, const double *b, double *x, hipStream_t s) {
  if (h->prec == 0) {
    vcycle_run<double>(h, b, x, s);
    return;
  }
  const int n = h->lv[0].n;
  convert<double, float>((float *)h->vb, b, n, s);
  vcycle_run<float>(h, (const float *)h->vb, (float *)h->vx, s);
  convert<float, double>(x, (const float *)h->vx, n, s);
}

// C applied to the fixed input buffer h->vcin, result in h->gw. The launch
// sequence of one V-cycle (about ten kernels per level) is captured once
// into a HIP graph and replayed, which removes per-launch host overhead.
static void precondition_fixed(bamg_handle *h, hipStream_t s) {
  if (!h->use_graph || h->prof_kernel >= 0) {
    precondition(h, h->vcin, h->gw, s);
    return;
  }
  if (!h->vc_exec) {
    // captured on a library stream (the caller's may be the null stream,
    // which cannot be captured), launched on the caller's stream
    if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = h->cap_stream;
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    hipGraph_t g = nullptr;
    try {
      precondition(h, h->vcin, h->gw, cs);
    } catch (...) {
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHK(hipStreamEndCapture(cs, &g));
    const hipError_t e = hipGraphInstantiate(&h->vc_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
  }
  HIPCHK(hipGraphLaunch(h->vc_exec, s));
}

__global__ void k_krylov_start(const double *__restrict__ h1, double *__restrict__ g, int m,
                               double *__restrict__ flags) {
  if (threadIdx.x != 0) return;
  const double beta = sqrt(h1[0]);
  for (int i = 0; i <= m; ++i) g[i] = 0.0;
  g[0] = beta;
  flags[3] = beta > 0.0 ? 1.0 / beta : 0.0;
  flags[8] = beta;
}

int gmres_blocks(int n) { return std::min(kRedBlocks, std::max(1, ceil_div(n, 256))); }

void gmres_buffers(bamg_handle *h, int m) {
  Pool &pool = h->pool;
  const int n = h->lv[0].n;
  const int nblk = gmres_blocks(n);
  if (h->gm_m != m) {
    // (re)allocate Krylov storage; old buffers stay with the pool until destroy
    h->gV = pool.get<double>((size_t)(m + 1) * n);
    h->gBV = pool.get<double>((size_t)m * n);
    h->gw = pool.get<double>(n);
    h->gx0 = pool.get<double>(n);
    h->gbx0 = pool.get<double>(n);
    h->gH = pool.get<double>((size_t)(m + 1) * m + 4 * (m + 2) + 64);
    h->gZ = h->opt.flexible ? pool.get<double>((size_t)m * n) : nullptr;
    h->gsc = pool.get<double>((size_t)(m + 2) * nblk * 2 + 2 * nblk + 16);
    if (h->prec != 0) {
      h->vb = pool.get<float>(n);
      h->vx = pool.get<float>(n);
    }
    if (!h->hred) {
      // mapped and coherent: the residual kernel writes each iteration's
      // flags here directly, the host reads them after that iteration's event
      HIPCHK(hipHostMalloc((void **)&h->hred, sizeof(double) * 32,
                           hipHostMallocMapped | hipHostMallocCoherent));
      HIPCHK(hipHostGetDevicePointer((void **)&h->hred_dev, h->hred, 0));
    }
    for (hipEvent_t &e : h->gm_ev)
      if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (!h->vcin) h->vcin = pool.get<double>(n);
    if (h->vc_exec) {
      (void)hipGraphExecDestroy(h->vc_exec);  // it wrote into the old gw
      h->vc_exec = nullptr;
    }
    h->gm_m = m;
  }
}

void gmres_run(bamg_handle *h, double *x, int m, double tol, int maxit, int use_x0,
               bamg_solve_info *info, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  Pool &pool = h->pool;
  Level &L0 = h->lv[0];
  const int n = L0.n;
  const int nblk = gmres_blocks(n);
  gmres_buffers(h, m);
  double *H = h->gH;
  double *cs = H + (size_t)(m + 1) * m, *sn = cs + (m + 2), *g = sn + (m + 2), *y = g + (m + 2);
  double *flags = y + (m + 2);  // 16 values
  double *part = h->gsc;                          // (m+2) * nblk: multi-dot partials
  double *part2 = part + (size_t)(m + 2) * nblk;  // nblk: |w|^2 partials
  double *part3 = part2 + nblk;                   // 2 nblk: residual-check partials
  double *coef = pool.get<double>(4 * (size_t)(m + 2));
  double *c1 = coef, *c2 = coef + (m + 2);  // the two Gram-Schmidt passes
  double *yring = coef + 2 * (m + 2);       // y of the last two iterations

  if (use_x0)
    HIPCHK(hipMemcpyAsync(h->gx0, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  else
    HIPCHK(hipMemcpyAsync(h->gx0, h->x0, sizeof(double) * n, hipMemcpyDeviceToDevice, s));

  const Csr &B = L0.B;
  const int lanes = L0.lanes, threads = L0.threads;
  const bool flex = h->opt.flexible != 0;
  double *hf = h->hred;
  auto read_flags = [&]() {
    HIPCHK(hipMemcpyAsync(hf, flags, sizeof(double) * 16, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  };

  // initial test on x0
  spmv<double>(B, h->B64, h->gx0, h->gbx0, nullptr, 0, lanes, s, threads);
  residual_check_partials(h->gx0, h->gbx0, h->gV, h->gBV, c1, n, 0, part3, nblk, s);
  residual_check_finalize(part3, nblk, tol, flags, nullptr, s);
  read_flags();
  int it = 0, restarts = 0, breakdowns = 0, conv = hf[0] != 0.0;
  double rel = hf[2];
  bamg_status st = BAMG_OK;
  while (!conv && it < maxit) {
    spmv<double>(B, h->B64, h->gx0, h->gbx0, nullptr, 0, lanes, s, threads);  // B x0
    if (flex) {
      negate_copy(h->gbx0, h->gw, n, s);  // r0 = -B x0
    } else {
      negate_copy(h->gbx0, h->vcin, n, s);  // r0 = -B x0
      precondition_fixed(h, s);             // z = C r0
    }
    multi_dot(h->gV, n, 0, h->gw, part, nblk, s);
    finalize_multi(part, nblk, 1, c1, s);
    k_krylov_start<<<1, 64, 0, s>>>(c1, g, m, flags);
    LAUNCHCHK();
    scale_vec(h->gw, flags + 3, h->gV, n, s);  // v_0 = z / beta (flexible: r0 / beta)
    int used = 0;
    bool broke = false;
    // Iteration j is enqueued with its status flags written by the residual
    // kernel into a mapped pinned slot and its y into a ring slot; the host
    // reads them only after iteration j + 1 is enqueued, so the device never
    // waits for the host between iterations. Stopping at j discards the work of j + 1 (it writes only
    // basis vector j + 2, the Hessenberg column j + 1 and the other y slot).
    // v_{j+1} = w / h_{j+1,j} is written by iteration j + 1's product
    // kernel, which is the first to read it.
    auto enqueue = [&](int j) {
      double *vj = h->gV + (size_t)j * n, *bvj = h->gBV + (size_t)j * n;
      if (flex) {
        // flexible: z_j = C v_j kept, w = B z_j (kept too, for the true residual)
        double *zj = h->gZ + (size_t)j * n;
        if (j > 0) scale_vec(h->gw, flags + 3, vj, n, s);  // v_j = w / h_{j,j-1}
        precondition(h, vj, zj, s);
        spmv_dual(B, h->B64, zj, bvj, h->gw, lanes, s, threads);
      } else if (j == 0) {
        spmv_dual(B, h->B64, vj, bvj, h->vcin, lanes, s, threads);  // B v_0
      } else {
        spmv_dual_scaled(B, h->B64, h->gw, flags + 3, vj, bvj, h->vcin, lanes, s,
                         threads);  // v_j, B v_j
      }
      if (!flex) precondition_fixed(h, s);  // w = C B v_j
      // Gram-Schmidt, twice; the first update and the second pass's dots in one kernel
      multi_dot(h->gV, n, j + 1, h->gw, part, nblk, s);
      finalize_multi(part, nblk, j + 2, c1, s);  // c1[0..j], c1[j+1] = |w|^2
      if (!multi_axpy_dot(h->gV, n, j + 1, c1, h->gw, part, nblk, s)) {
        multi_axpy_norm(h->gV, n, j + 1, c1, h->gw, part2, nblk, s);
        multi_dot(h->gV, n, j + 1, h->gw, part, nblk, s);
      }
      finalize_multi(part, nblk, j + 1, c2, s);
      multi_axpy_norm(h->gV, n, j + 1, c2, h->gw, part2, nblk, s);
      // y goes straight to this iteration's ring slot
      double *ys = yring + (size_t)(j & 1) * (m + 2);
      gmres_arnoldi_update(H, cs, sn, g, ys, c1, c2, part2, nblk, nullptr, j, m, flags, s);
      residual_check_partials(h->gx0, h->gbx0, flex ? h->gZ : h->gV, h->gBV, ys, n, j + 1, part3,
                              nblk, s);
      residual_check_finalize(part3, nblk, tol, flags, h->hred_dev + 16 * (j & 1), s);
      HIPCHK(hipEventRecord(h->gm_ev[j & 1], s));
    };
    auto finished = [&](int j) {  // true: stop after iteration j
      HIPCHK(hipEventSynchronize(h->gm_ev[j & 1]));
      const double *f = hf + 16 * (j & 1);
      ++it;
      used = j + 1;
      rel = f[2];
      if (!std::isfinite(rel)) {
        st = BAMG_E_NONFINITE;
        return true;
      }
      if (f[0] != 0.0) {
        conv = 1;
        return true;
      }
      if (f[1] != 0.0) {
        broke = true;
        return true;
      }
      return false;
    };
    if (it < maxit) {
      enqueue(0);
      for (int j = 0;; ++j) {
        const bool more = j + 1 < m && it + 1 < maxit;
        if (more) enqueue(j + 1);
        if (finished(j) || !more) break;
      }
    }
    if (used > 0)
      update_iterate(h->gx0, flex ? h->gZ : h->gV, yring + (size_t)((used - 1) & 1) * (m + 2), n,
                     used, s);
    if (st != BAMG_OK) break;
    if (broke && !conv && ++breakdowns >= 2) {
      st = BAMG_E_BREAKDOWN;
      break;
    }
    if (!conv) ++restarts;
  }
  // scale to 1^T x = 1
  normalize_sum(h->gx0, n, part, nblk, flags, s);
  HIPCHK(hipMemcpyAsync(x, h->gx0, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  read_flags();
  if (info) {
    info->iterations = it;
    info->restarts = restarts;
    info->converged = conv;
    info->breakdowns = breakdowns;
    info->rel_residual = rel;
    info->x_min = hf[5];
    info->t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  pool.release(coef);
  pool.flush();
  if (st != BAMG_OK) fail(st, "GMRES failed");
  if (!conv) throw Error{BAMG_NOT_CONVERGED, "iteration cap reached"};
}

}  // namespace bamg
