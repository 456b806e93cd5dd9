// Interpolation-weight MLP (96 -> 64 -> 64 -> 8, ReLU): an addition to the
// method, not part of the paper. The setup can take the F rows of P in its
// first bootstrap cycle from the network instead of from the least-squares
// fit of eq. ls_interpolation, keeping the exact fit for any row where the
// network's weights give an LS objective above twice the optimum.
//
// The network's outputs are corrections added to the exact LS row, which is
// also one of its inputs.
//
// Kernels:
//  * k_mlp_infer      inference on MFMA (v_mfma_f32_16x16x32_bf16): one wave
//                     per 16 points, weights in LDS as BF16, FP32 accumulate;
//  * k_mlp_point      FP32 forward and backward of one point per thread;
//  * k_mlp_wgrad      weight gradients as fixed-order sums over the batch;
//  * k_adam, k_mlp_bf16  the optimiser step and the BF16 weight copy;
//  * k_mlp_features   the 96 inputs of each F point;
//  * k_mlp_select     MLP row or exact LS row, by the objective test.
#include <mutex>
#include <string>

#include "bamg_internal.h"
#include "device_common.h"

namespace bamg {

constexpr int kIn = BAMG_MLP_IN, kHid = BAMG_MLP_HIDDEN, kOut = BAMG_MLP_OUT;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid,
              oW3 = oB2 + kHid, oB3 = oW3 + kOut * kHid, kNPar = oB3 + kOut;
static_assert(kNPar == BAMG_MLP_NPARAMS, "parameter layout");
// BF16 copy: W1 | W2 | W3 padded to 16 rows (rows 8..15 zero)
constexpr int bW1 = 0, bW2 = bW1 + kHid * kIn, bW3 = bW2 + kHid * kHid, kNBf = bW3 + 16 * kHid;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ inference
// Lane l of a wave holds, for v_mfma_f32_16x16x32_bf16: A row l % 16 and
// k = 8 (l / 16) + 0..7; B column l % 16 and the same k; D column l % 16 and
// rows 4 (l / 16) + 0..3.
constexpr int kInferWaves = 4;

__global__ void __launch_bounds__(kInferWaves * kWave)
    k_mlp_infer(const __bf16 *__restrict__ wb, const float *__restrict__ par,
                const float *__restrict__ X, long npts, float *__restrict__ Y) {
  __shared__ __attribute__((aligned(16))) __bf16 w[kNBf];
  __shared__ float bias[kHid + kHid + kOut];
  __shared__ __attribute__((aligned(16))) __bf16 hs[kInferWaves][2][16 * kHid];
  for (int e = threadIdx.x; e < kNBf; e += blockDim.x) w[e] = wb[e];
  for (int e = threadIdx.x; e < kHid; e += blockDim.x) {
    bias[e] = par[oB1 + e];
    bias[kHid + e] = par[oB2 + e];
  }
  for (int e = threadIdx.x; e < kOut; e += blockDim.x) bias[2 * kHid + e] = par[oB3 + e];
  __syncthreads();
  const int wv = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int row = l % 16, kq = 8 * (l / 16), rq = 4 * (l / 16);
  const long p0 = ((long)blockIdx.x * kInferWaves + wv) * 16;
  const long pr = p0 + row;  // the point whose A row this lane loads
  __bf16 *h1 = hs[wv][0], *h2 = hs[wv][1];
  // layer 1: [16 x 96] x [96 x 64]
  f32x4 acc[4];
  for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < kIn / 32; ++ks) {
    bf16x8 a;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      a[e] = (__bf16)(pr < npts ? X[pr * kIn + 32 * ks + kq + e] : 0.f);
    for (int nb = 0; nb < 4; ++nb) {
      const bf16x8 b = *(const bf16x8 *)&w[bW1 + (16 * nb + row) * kIn + 32 * ks + kq];
      acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nb], 0, 0, 0);
    }
  }
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = 16 * nb + row;
      h1[(rq + e) * kHid + j] = (__bf16)fmaxf(acc[nb][e] + bias[j], 0.f);
    }
  __syncthreads();
  // layer 2: [16 x 64] x [64 x 64]
  for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < kHid / 32; ++ks) {
    const bf16x8 a = *(const bf16x8 *)&h1[row * kHid + 32 * ks + kq];
    for (int nb = 0; nb < 4; ++nb) {
      const bf16x8 b = *(const bf16x8 *)&w[bW2 + (16 * nb + row) * kHid + 32 * ks + kq];
      acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nb], 0, 0, 0);
    }
  }
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = 16 * nb + row;
      h2[(rq + e) * kHid + j] = (__bf16)fmaxf(acc[nb][e] + bias[kHid + j], 0.f);
    }
  __syncthreads();
  // layer 3: [16 x 64] x [64 x 16] (columns 8..15 are zero padding)
  f32x4 o = {0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < kHid / 32; ++ks) {
    const bf16x8 a = *(const bf16x8 *)&h2[row * kHid + 32 * ks + kq];
    const bf16x8 b = *(const bf16x8 *)&w[bW3 + row * kHid + 32 * ks + kq];
    o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, o, 0, 0, 0);
  }
  if (row < kOut)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const long p = p0 + rq + e;
      if (p < npts) Y[p * kOut + row] = o[e] + bias[2 * kHid + row];
    }
}

// ------------------------------------------------------------ training
// One point per thread: forward in FP32; with targets, the backward pass to
// the hidden layers. Stores h1, h2 (post-ReLU), dh1, dh2 (pre-activation
// gradients) and dy for the weight gradients, and the scaled point loss.
constexpr int kPointThreads = 128;

__global__ void __launch_bounds__(kPointThreads)
    k_mlp_point(const float *__restrict__ par, const float *__restrict__ X,
                const float *__restrict__ T, const float *__restrict__ M, long npts, float scale,
                float *__restrict__ H1, float *__restrict__ H2, float *__restrict__ D1,
                float *__restrict__ D2, float *__restrict__ DY, float *__restrict__ Y,
                double *__restrict__ ploss) {
  __shared__ float w[kNPar];
  for (int e = threadIdx.x; e < kNPar; e += blockDim.x) w[e] = par[e];
  __syncthreads();
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  float x[kIn], a1[kHid], a2[kHid], y[kOut];
  for (int i = 0; i < kIn; ++i) x[i] = X[p * kIn + i];
  for (int o = 0; o < kHid; ++o) {
    float s = w[oB1 + o];
    for (int i = 0; i < kIn; ++i) s += w[oW1 + o * kIn + i] * x[i];
    a1[o] = s;
  }
  for (int o = 0; o < kHid; ++o) {
    float s = w[oB2 + o];
    for (int q = 0; q < kHid; ++q) s += w[oW2 + o * kHid + q] * fmaxf(a1[q], 0.f);
    a2[o] = s;
  }
  for (int t = 0; t < kOut; ++t) {
    float s = w[oB3 + t];
    for (int o = 0; o < kHid; ++o) s += w[oW3 + t * kHid + o] * fmaxf(a2[o], 0.f);
    y[t] = s;
  }
  if (Y)
    for (int t = 0; t < kOut; ++t) Y[p * kOut + t] = y[t];
  if (!T) return;
  float dy[kOut];
  double lp = 0.0;
  for (int t = 0; t < kOut; ++t) {
    const float m = M[p * kOut + t], d = y[t] - T[p * kOut + t];
    dy[t] = m * d * scale;
    lp += 0.5 * (double)m * (double)d * (double)d;
    DY[p * kOut + t] = dy[t];
  }
  ploss[p] = lp * (double)scale;
  float d2[kHid];
  for (int o = 0; o < kHid; ++o) {
    float s = 0.f;
    for (int t = 0; t < kOut; ++t) s += w[oW3 + t * kHid + o] * dy[t];
    d2[o] = a2[o] > 0.f ? s : 0.f;
    D2[p * kHid + o] = d2[o];
    H2[p * kHid + o] = fmaxf(a2[o], 0.f);
  }
  for (int q = 0; q < kHid; ++q) {
    float s = 0.f;
    for (int o = 0; o < kHid; ++o) s += w[oW2 + o * kHid + q] * d2[o];
    D1[p * kHid + q] = a1[q] > 0.f ? s : 0.f;
    H1[p * kHid + q] = fmaxf(a1[q], 0.f);
  }
}

// gradient entry e = sum over the batch, in point order
__global__ void __launch_bounds__(256)
    k_mlp_wgrad(const float *__restrict__ X, const float *__restrict__ H1,
                const float *__restrict__ H2, const float *__restrict__ D1,
                const float *__restrict__ D2, const float *__restrict__ DY, long npts,
                float *__restrict__ G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kNPar) return;
  float g = 0.f;
  if (e < oB1) {
    const int o = e / kIn, i = e % kIn;
    for (long p = 0; p < npts; ++p) g += D1[p * kHid + o] * X[p * kIn + i];
  } else if (e < oW2) {
    const int o = e - oB1;
    for (long p = 0; p < npts; ++p) g += D1[p * kHid + o];
  } else if (e < oB2) {
    const int o = (e - oW2) / kHid, q = (e - oW2) % kHid;
    for (long p = 0; p < npts; ++p) g += D2[p * kHid + o] * H1[p * kHid + q];
  } else if (e < oW3) {
    const int o = e - oB2;
    for (long p = 0; p < npts; ++p) g += D2[p * kHid + o];
  } else if (e < oB3) {
    const int t = (e - oW3) / kHid, o = (e - oW3) % kHid;
    for (long p = 0; p < npts; ++p) g += DY[p * kOut + t] * H2[p * kHid + o];
  } else {
    const int t = e - oB3;
    for (long p = 0; p < npts; ++p) g += DY[p * kOut + t];
  }
  G[e] = g;
}

__global__ void k_adam(float *__restrict__ par, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int n, float lr, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mi = b1 * m[e] + (1.f - b1) * g[e];
  const float vi = b2 * v[e] + (1.f - b2) * g[e] * g[e];
  m[e] = mi;
  v[e] = vi;
  par[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_mlp_bf16(const float *__restrict__ par, __bf16 *__restrict__ wb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kNBf) return;
  float x;
  if (e < bW2)
    x = par[oW1 + e];
  else if (e < bW3)
    x = par[oW2 + (e - bW2)];
  else
    x = (e - bW3) < kOut * kHid ? par[oW3 + (e - bW3)] : 0.f;
  wb[e] = (__bf16)x;  // round to nearest even
}

__global__ void k_sum_double(const double *__restrict__ x, long n, double *__restrict__ out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (long i = threadIdx.x; i < n; i += 256) s += x[i];
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) *out = s;
}

// ------------------------------------------------------------ features
template <class T>
__global__ void k_mlp_features(int nF, const int *__restrict__ fpts, int r,
                               const int *__restrict__ prp, const int *__restrict__ pci,
                               const int *__restrict__ cpts, const T *__restrict__ V,
                               const double *__restrict__ wv, const int *__restrict__ brp,
                               const int *__restrict__ bci, const T *__restrict__ bv,
                               const T *__restrict__ Pv, float *__restrict__ F) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nF) return;
  const int i = fpts[f];
  const int a0 = prp[i], m = min(prp[i + 1] - a0, kOut);
  int J[kOut];
  for (int t = 0; t < kOut; ++t) J[t] = t < m ? cpts[pci[a0 + t]] : -1;
  float *o = F + (size_t)f * kIn;
  double S = 0.0;
  for (int k = 0; k < 8; ++k) {
    const double sw = k < r ? sqrt(wv[k]) : 0.0;
    double a = k < r ? fabs(sw * (double)V[(size_t)i * r + k]) : 0.0;
    S = fmax(S, a);
    for (int t = 0; t < m; ++t)
      if (k < r) S = fmax(S, fabs(sw * (double)V[(size_t)J[t] * r + k]));
  }
  if (!(S > 0.0)) S = 1.0;
  for (int k = 0; k < 8; ++k) {
    const double sw = k < r ? sqrt(wv[k]) : 0.0;
    o[9 * k] = k < r ? (float)(sw * (double)V[(size_t)i * r + k] / S) : 0.f;
    for (int t = 0; t < kOut; ++t)
      o[9 * k + 1 + t] = (k < r && t < m) ? (float)(sw * (double)V[(size_t)J[t] * r + k] / S) : 0.f;
  }
  double bii = 1.0;
  for (int a = brp[i]; a < brp[i + 1]; ++a)
    if (bci[a] == i) bii = (double)bv[a];
  if (bii == 0.0) bii = 1.0;
  for (int t = 0; t < kOut; ++t) {
    double bij = 0.0;
    if (t < m)
      for (int a = brp[i]; a < brp[i + 1]; ++a)
        if (bci[a] == J[t]) bij = (double)bv[a];
    o[72 + t] = (float)(bij / bii);
    o[80 + t] = t < m ? (float)Pv[a0 + t] : 0.f;
    o[88 + t] = t < m ? 1.f : 0.f;
  }
}

// LS objective sum_k w_k (v_i - sum_t p_t v_{j_t})^2 of the MLP row (the
// exact row in Pv plus the network's correction) against the exact row; the
// MLP row replaces it if within 2x.
template <class T>
__global__ void k_mlp_select(int nF, const int *__restrict__ fpts, int r,
                             const int *__restrict__ prp, const int *__restrict__ pci,
                             const int *__restrict__ cpts, const T *__restrict__ V,
                             const double *__restrict__ wv, const float *__restrict__ Y,
                             T *__restrict__ Pv, int *__restrict__ counts) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  bool take = false;
  const bool active = f < nF;
  if (active) {
    const int i = fpts[f];
    const int a0 = prp[i], m = min(prp[i + 1] - a0, kOut);
    int J[kOut];
    double pl[kOut], pm[kOut];
    for (int t = 0; t < m; ++t) {
      J[t] = cpts[pci[a0 + t]];
      pl[t] = (double)Pv[a0 + t];
      pm[t] = pl[t] + (double)Y[(size_t)f * kOut + t];
    }
    double jm = 0.0, jl = 0.0;
    for (int k = 0; k < r; ++k) {
      double em = (double)V[(size_t)i * r + k], el = em;
      for (int t = 0; t < m; ++t) {
        const double vj = (double)V[(size_t)J[t] * r + k];
        em -= pm[t] * vj;
        el -= pl[t] * vj;
      }
      jm += wv[k] * em * em;
      jl += wv[k] * el * el;
    }
    take = jm <= 2.0 * jl;
    if (take)
      for (int t = 0; t < m; ++t) Pv[a0 + t] = (T)pm[t];
  }
  // one counter update per wave
  const unsigned long long bt = __ballot(active && take), bf = __ballot(active && !take);
  if ((threadIdx.x % kWave) == 0) {
    if (bt) atomicAdd(&counts[0], (int)__popcll(bt));
    if (bf) atomicAdd(&counts[1], (int)__popcll(bf));
  }
}

__global__ void k_flag_f(int n, const int *__restrict__ cf, int *__restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = cf[i] ? 0 : 1;
}

__global__ void k_scatter_f(int n, const int *__restrict__ cf, const int *__restrict__ pos,
                            int *__restrict__ fpts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !cf[i]) fpts[pos[i]] = i;
}

// P rows of the F points as targets (zero-padded) and the mask
template <class T>
__global__ void k_mlp_targets(int nF, const int *__restrict__ fpts, const int *__restrict__ prp,
                              const T *__restrict__ Pv, float *__restrict__ Tg,
                              float *__restrict__ Mk) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nF) return;
  const int i = fpts[f];
  const int a0 = prp[i], m = min(prp[i + 1] - a0, kOut);
  for (int t = 0; t < kOut; ++t) {
    Tg[(size_t)f * kOut + t] = t < m ? (float)Pv[a0 + t] : 0.f;
    Mk[(size_t)f * kOut + t] = t < m ? 1.f : 0.f;
  }
}

// ------------------------------------------------------------ host side
void mlp_refresh_bf16(bamg_mlp *m, hipStream_t s) {
  k_mlp_bf16<<<ceil_div(kNBf, 256), 256, 0, s>>>(m->p, m->wb);
  LAUNCHCHK();
}

void mlp_forward(const bamg_mlp *m, const float *X, long npts, float *Y, int mode, hipStream_t s) {
  if (npts <= 0) return;
  if (mode == 1) {
    const long waves = (npts + 15) / 16;
    k_mlp_infer<<<ceil_div(waves, kInferWaves), kInferWaves * kWave, 0, s>>>(m->wb, m->p, X,
                                                                            npts, Y);
  } else {
    k_mlp_point<<<ceil_div(npts, kPointThreads), kPointThreads, 0, s>>>(
        m->p, X, nullptr, nullptr, npts, 1.f, nullptr, nullptr, nullptr, nullptr, nullptr, Y,
        nullptr);
  }
  LAUNCHCHK();
}

// scratch for one batch of up to `cap` points
struct MlpScratch {
  float *H1, *H2, *D1, *D2, *DY, *G;
  double *pl, *lsum;
};

static MlpScratch mlp_scratch(long cap) {
  MlpScratch w{};
  const size_t hb = sizeof(float) * (size_t)cap * kHid;
  HIPCHK(hipMalloc(&w.H1, hb));
  HIPCHK(hipMalloc(&w.H2, hb));
  HIPCHK(hipMalloc(&w.D1, hb));
  HIPCHK(hipMalloc(&w.D2, hb));
  HIPCHK(hipMalloc(&w.DY, sizeof(float) * (size_t)cap * kOut));
  HIPCHK(hipMalloc(&w.G, sizeof(float) * kNPar));
  HIPCHK(hipMalloc(&w.pl, sizeof(double) * (size_t)cap));
  HIPCHK(hipMalloc(&w.lsum, sizeof(double)));
  return w;
}

static void mlp_scratch_free(MlpScratch &w) {
  void *ps[] = {w.H1, w.H2, w.D1, w.D2, w.DY, w.G, w.pl, w.lsum};
  for (void *p : ps)
    if (p) (void)hipFree(p);
}

// loss (sum of scaled point losses) into w.lsum and gradient into w.G
static void mlp_batch_grad(const bamg_mlp *m, const float *X, const float *T, const float *M,
                           long npts, MlpScratch &w, hipStream_t s) {
  const float scale = 1.f / (float)npts;
  k_mlp_point<<<ceil_div(npts, kPointThreads), kPointThreads, 0, s>>>(
      m->p, X, T, M, npts, scale, w.H1, w.H2, w.D1, w.D2, w.DY, nullptr, w.pl);
  LAUNCHCHK();
  k_mlp_wgrad<<<ceil_div(kNPar, 256), 256, 0, s>>>(X, w.H1, w.H2, w.D1, w.D2, w.DY, npts, w.G);
  LAUNCHCHK();
  k_sum_double<<<1, 256, 0, s>>>(w.pl, npts, w.lsum);
  LAUNCHCHK();
}

double mlp_loss_grad(const bamg_mlp *m, const float *X, const float *T, const float *M, long npts,
                     float *grad, hipStream_t s) {
  MlpScratch w = mlp_scratch(npts);
  double loss = 0.0;
  try {
    mlp_batch_grad(m, X, T, M, npts, w, s);
    HIPCHK(hipMemcpyAsync(grad, w.G, sizeof(float) * kNPar, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(&loss, w.lsum, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  } catch (...) {
    mlp_scratch_free(w);
    throw;
  }
  mlp_scratch_free(w);
  return loss;
}

// ---------------------------------------------------------------- no-alloc
// Scratch of the loss/gradient for callers that cannot allocate device
// memory: one fixed array per GPU, held until the process ends and shared by
// every call on that GPU (the last call's contents stay; every kernel below
// writes its part in full before it is read, so nothing needs clearing).
// Host code never passes the array's name to a kernel: its device address
// is looked up once per device and kept in g_scratch_ptr.
constexpr long kNoAllocPoints = BAMG_MLP_NOALLOC_MAX_POINTS;
constexpr size_t kNoAllocBytes = size_t(64) << 20;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

constexpr size_t round256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kHidBytes = round256(sizeof(float) * (size_t)kNoAllocPoints * kHid);
constexpr size_t kDyBytes = round256(sizeof(float) * (size_t)kNoAllocPoints * kOut);
constexpr size_t kGBytes = round256(sizeof(float) * kNPar);
constexpr size_t kPlBytes = round256(sizeof(double) * (size_t)kNoAllocPoints);
static_assert(4 * kHidBytes + kDyBytes + kGBytes + kPlBytes + 256 <= kNoAllocBytes,
              "no-alloc scratch too small for its maximum point count");

// device address of this GPU's scratch array (looked up on the first call
// made with the device current)
char *scratch_base() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(BAMG_E_DEVICE, "device ordinal above 63");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  return static_cast<char *>(g_scratch_ptr[dev]);
}
}  // namespace

double mlp_loss_grad_noalloc(const bamg_mlp *m, const float *X, const float *T, const float *M,
                             long npts, float *grad, hipStream_t s) {
  if (npts < 1 || npts > kNoAllocPoints)
    fail(BAMG_E_ARG, "npts above the no-allocation maximum of " +
                         std::to_string(kNoAllocPoints) + " points");
  char *b = scratch_base();
  MlpScratch w{};
  w.H1 = reinterpret_cast<float *>(b);
  w.H2 = reinterpret_cast<float *>(b + kHidBytes);
  w.D1 = reinterpret_cast<float *>(b + 2 * kHidBytes);
  w.D2 = reinterpret_cast<float *>(b + 3 * kHidBytes);
  w.DY = reinterpret_cast<float *>(b + 4 * kHidBytes);
  w.G = reinterpret_cast<float *>(b + 4 * kHidBytes + kDyBytes);
  w.pl = reinterpret_cast<double *>(b + 4 * kHidBytes + kDyBytes + kGBytes);
  w.lsum = reinterpret_cast<double *>(b + 4 * kHidBytes + kDyBytes + kGBytes + kPlBytes);
  double loss = 0.0;
  mlp_batch_grad(m, X, T, M, npts, w, s);
  HIPCHK(hipMemcpyAsync(grad, w.G, sizeof(float) * kNPar, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(&loss, w.lsum, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return loss;
}

void mlp_train(bamg_mlp *m, const float *X, const float *T, const float *M, long npts, int batch,
               int epochs, float lr, double *loss_per_epoch, hipStream_t s) {
  MlpScratch w = mlp_scratch(batch);
  try {
    for (int ep = 0; ep < epochs; ++ep) {
      double tot = 0.0;
      int nb = 0;
      for (long b0 = 0; b0 < npts; b0 += batch) {
        const long nbp = std::min<long>(batch, npts - b0);
        mlp_batch_grad(m, X + b0 * kIn, T + b0 * kOut, M + b0 * kOut, nbp, w, s);
        ++m->step;
        const float c1 = 1.f - powf(0.9f, (float)m->step), c2 = 1.f - powf(0.999f, (float)m->step);
        k_adam<<<ceil_div(kNPar, 256), 256, 0, s>>>(m->p, m->m, m->v, w.G, kNPar, lr, c1, c2);
        LAUNCHCHK();
        if (loss_per_epoch) {
          double l = 0.0;
          HIPCHK(hipMemcpyAsync(&l, w.lsum, sizeof(double), hipMemcpyDeviceToHost, s));
          HIPCHK(hipStreamSynchronize(s));
          tot += l;
        }
        ++nb;
      }
      if (loss_per_epoch) loss_per_epoch[ep] = nb ? tot / nb : 0.0;
    }
    mlp_refresh_bf16(m, s);
    HIPCHK(hipStreamSynchronize(s));
  } catch (...) {
    mlp_scratch_free(w);
    throw;
  }
  mlp_scratch_free(w);
}

// F points of a level in ascending order (computed once per level)
void level_fpoints(bamg_handle *h, Level &L, hipStream_t s) {
  if (L.fpts) return;
  int *cnt = h->pool.get<int>(L.n);
  int *pos = h->pool.get<int>(L.n + 1);
  k_flag_f<<<ceil_div(L.n, 256), 256, 0, s>>>(L.n, L.cf, cnt);
  LAUNCHCHK();
  scan_counts(h->pool, cnt, pos, L.n, s);
  L.nF = read_int(pos + L.n, s);
  L.fpts = h->pool.get<int>(L.nF > 0 ? L.nF : 1);
  k_scatter_f<<<ceil_div(L.n, 256), 256, 0, s>>>(L.n, L.cf, pos, L.fpts);
  LAUNCHCHK();
  h->pool.release(cnt);
  h->pool.release(pos);
}

template <class T>
void mlp_features(const Level &L, int r, const T *V, const double *wv, const T *Pv, float *F,
                  hipStream_t s) {
  if (L.nF <= 0) return;
  k_mlp_features<T><<<ceil_div(L.nF, 128), 128, 0, s>>>(L.nF, L.fpts, r, L.P.rp, L.P.ci, L.cpts,
                                                        V, wv, L.B.rp, L.B.ci, (const T *)L.Bv,
                                                        Pv, F);
  LAUNCHCHK();
}

template <class T>
void mlp_select(const Level &L, int r, const T *V, const double *wv, const float *Y, T *Pv,
                int *counts, hipStream_t s) {
  if (L.nF <= 0) return;
  k_mlp_select<T><<<ceil_div(L.nF, 128), 128, 0, s>>>(L.nF, L.fpts, r, L.P.rp, L.P.ci, L.cpts, V,
                                                      wv, Y, Pv, counts);
  LAUNCHCHK();
}

template <class T>
void mlp_targets(const Level &L, const T *Pv, float *Tg, float *Mk, hipStream_t s) {
  if (L.nF <= 0) return;
  k_mlp_targets<T><<<ceil_div(L.nF, 128), 128, 0, s>>>(L.nF, L.fpts, L.P.rp, Pv, Tg, Mk);
  LAUNCHCHK();
}

#define INST(T)                                                                              \
  template void mlp_features<T>(const Level &, int, const T *, const double *, const T *,  \
                                float *, hipStream_t);                                       \
  template void mlp_select<T>(const Level &, int, const T *, const double *, const float *, \
                              T *, int *, hipStream_t);                                      \
  template void mlp_targets<T>(const Level &, const T *, float *, float *, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace bamg
