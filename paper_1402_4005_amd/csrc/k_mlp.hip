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
//  * k_mlp_tile       FP32 forward and backward of 64 points on FP32 MFMA;
//  * k_mlp_wgrad_mfma weight gradients as batch products on FP32 MFMA;
//  * k_adam, k_mlp_bf16  the optimiser step and the BF16 weight copy;
//  * k_mlp_features   the 96 inputs of each F point (recorded for training);
//  * k_mlp_apply      features, inference and the objective test (MLP row or
//                     exact LS row) of 16 F points per wave, in one launch.
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

// ------------------------------------------------------------ training on MFMA
// FP32 matrix-core products (v_mfma_f32_16x16x4f32: FP32 operands, FP32
// accumulation) for the forward and backward passes and the weight
// gradients. D (16 x 16) += A B over k in [0, K), K a multiple of 4: lane l
// supplies A[l % 16][k + l / 16] and B[k + l / 16][l % 16] and holds
// D[4 (l / 16) + r][l % 16] in acc[r].
template <class FA, class FB>
__device__ __forceinline__ f32x4 mfma32(int K, FA a, FB b, f32x4 acc, int k0 = 0, int kstep = 4) {
  const int l = threadIdx.x % kWave;
  for (int k = k0; k < K; k += kstep)
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a(l % 16, k + l / 16), b(k + l / 16, l % 16), acc,
                                               0, 0, 0);
  return acc;
}

// 64 points per workgroup (4 waves, wave w owns points 16 w .. 16 w + 15):
// a1 = x W1^T + b1, a2 = relu(a1) W2^T + b2, y = relu(a2) W3^T + b3; with
// targets dy = m (y - t) scale, d2 = (dy W3) [a2 > 0], d1 = (d2 W2) [a1 > 0].
// Stores what k_mlp_wgrad_mfma needs (h1, h2 post-ReLU, d1, d2, dy) and the
// scaled point losses. Dynamic LDS: mlp_tile_lds().
constexpr int kTileP = 64, kXs = kIn + 1, kHs = kHid + 1, kYs = kOut + 1;
static size_t mlp_tile_lds() {
  return sizeof(float) * ((size_t)kNPar + kTileP * kXs + 3 * kTileP * kHs + kTileP * kYs);
}

__global__ void __launch_bounds__(256)
    k_mlp_tile(const float *__restrict__ par, const float *__restrict__ X,
               const float *__restrict__ T, const float *__restrict__ M, long npts, float scale,
               float *__restrict__ H1, float *__restrict__ H2, float *__restrict__ D1,
               float *__restrict__ D2, float *__restrict__ DY, float *__restrict__ Y,
               double *__restrict__ ploss) {
  extern __shared__ float sm[];
  float *w = sm;                        // parameters, as in memory
  float *xs = w + kNPar;                // 64 x 96 inputs
  float *a1 = xs + kTileP * kXs;        // 64 x 64 pre-activations of layer 1
  float *a2 = a1 + kTileP * kHs;        // layer 2
  float *d2 = a2 + kTileP * kHs;        // 64 x 64 gradient of a2
  float *yv = d2 + kTileP * kHs;        // 64 x 8 outputs, then dy
  const long p0 = (long)blockIdx.x * kTileP;
  const int t = threadIdx.x, wv = t / kWave, ln = t % kWave;
  for (int e = t; e < kNPar; e += 256) w[e] = par[e];
  for (int e = t; e < kTileP * kIn; e += 256) {
    const int r = e / kIn, i = e % kIn;
    xs[r * kXs + i] = p0 + r < npts ? X[(p0 + r) * kIn + i] : 0.f;
  }
  __syncthreads();
  const int pr = 16 * wv;  // this wave's point rows
  auto store = [&](float *dst, int ld, int cj, f32x4 acc, auto f) {
    for (int r = 0; r < 4; ++r) {
      const int row = pr + 4 * (ln / 16) + r, col = 16 * cj + ln % 16;
      dst[row * ld + col] = f(acc[r], col);
    }
  };
  // layer 1
  for (int cj = 0; cj < kHid / 16; ++cj) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma32(kIn, [&](int i, int k) { return xs[(pr + i) * kXs + k]; },
                 [&](int k, int j) { return w[oW1 + (16 * cj + j) * kIn + k]; }, acc);
    store(a1, kHs, cj, acc, [&](float v, int c) { return v + w[oB1 + c]; });
  }
  __syncthreads();
  // layer 2
  for (int cj = 0; cj < kHid / 16; ++cj) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma32(kHid, [&](int i, int k) { return fmaxf(a1[(pr + i) * kHs + k], 0.f); },
                 [&](int k, int j) { return w[oW2 + (16 * cj + j) * kHid + k]; }, acc);
    store(a2, kHs, cj, acc, [&](float v, int c) { return v + w[oB2 + c]; });
  }
  __syncthreads();
  // output layer (columns 8..15 of the tile are zero)
  {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma32(kHid, [&](int i, int k) { return fmaxf(a2[(pr + i) * kHs + k], 0.f); },
                 [&](int k, int j) { return j < kOut ? w[oW3 + j * kHid + k] : 0.f; }, acc);
    for (int r = 0; r < 4; ++r) {
      const int row = pr + 4 * (ln / 16) + r, col = ln % 16;
      if (col < kOut) yv[row * kYs + col] = acc[r] + w[oB3 + col];
    }
  }
  __syncthreads();
  if (Y)
    for (int e = t; e < kTileP * kOut; e += 256) {
      const int r = e / kOut, c = e % kOut;
      if (p0 + r < npts) Y[(p0 + r) * kOut + c] = yv[r * kYs + c];
    }
  if (!T) return;
  if (t < kTileP) {
    const long p = p0 + t;
    double lp = 0.0;
    for (int c = 0; c < kOut; ++c) {
      float dy = 0.f;
      if (p < npts) {
        const float m = M[p * kOut + c], d = yv[t * kYs + c] - T[p * kOut + c];
        dy = m * d * scale;
        lp += 0.5 * (double)m * (double)d * (double)d;
        DY[p * kOut + c] = dy;
      }
      yv[t * kYs + c] = dy;
    }
    if (p < npts) ploss[p] = lp * (double)scale;
  }
  __syncthreads();
  // d2 = (dy W3) [a2 > 0]: K = 8
  for (int cj = 0; cj < kHid / 16; ++cj) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma32(kOut, [&](int i, int k) { return yv[(pr + i) * kYs + k]; },
                 [&](int k, int j) { return w[oW3 + k * kHid + 16 * cj + j]; }, acc);
    for (int r = 0; r < 4; ++r) {
      const int row = pr + 4 * (ln / 16) + r, col = 16 * cj + ln % 16;
      const float av = a2[row * kHs + col], dv = av > 0.f ? acc[r] : 0.f;
      d2[row * kHs + col] = dv;
      if (p0 + row < npts) {
        D2[(p0 + row) * kHid + col] = dv;
        H2[(p0 + row) * kHid + col] = fmaxf(av, 0.f);
      }
    }
  }
  __syncthreads();
  // d1 = (d2 W2) [a1 > 0]
  for (int cj = 0; cj < kHid / 16; ++cj) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma32(kHid, [&](int i, int k) { return d2[(pr + i) * kHs + k]; },
                 [&](int k, int j) { return w[oW2 + k * kHid + 16 * cj + j]; }, acc);
    for (int r = 0; r < 4; ++r) {
      const int row = pr + 4 * (ln / 16) + r, col = 16 * cj + ln % 16;
      const float av = a1[row * kHs + col];
      if (p0 + row < npts) {
        D1[(p0 + row) * kHid + col] = av > 0.f ? acc[r] : 0.f;
        H1[(p0 + row) * kHid + col] = fmaxf(av, 0.f);
      }
    }
  }
}

// Weight gradients as products over the batch, one workgroup per 16 x 16
// tile of a gradient matrix; wave w takes the groups of four points 4 w,
// 4 w + 16, ... and the four partial tiles are added in wave order, so the
// result does not depend on timing:
// G_W1 = D1^T X (24 tiles), G_W2 = D2^T H1 (16), G_W3 = DY^T H2 (4, rows 8..15
// padding), and the bias gradients as products with a ones column (4 + 4 +
// 1 tiles, column 0 kept).
constexpr int kGradTiles = 24 + 16 + 4 + 9;

constexpr int kGradWaves = 4;

__global__ void __launch_bounds__(kGradWaves * kWave)
    k_mlp_wgrad_mfma(const float *__restrict__ X, const float *__restrict__ H1,
                     const float *__restrict__ H2, const float *__restrict__ D1,
                     const float *__restrict__ D2, const float *__restrict__ DY, long npts,
                     float *__restrict__ G) {
  __shared__ f32x4 part[kGradWaves][kWave];
  const int tile = blockIdx.x, wv = threadIdx.x / kWave, ln = threadIdx.x % kWave;
  const int K = (int)((npts + 3) / 4) * 4, k0 = 4 * wv, ks = 4 * kGradWaves;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  auto pt = [&](int k) { return (long)k < npts; };
  int kind, ti, tj;
  if (tile < 24) {
    kind = 0, ti = tile / 6, tj = tile % 6;
    acc = mfma32(K, [&](int i, int k) { return pt(k) ? D1[(long)k * kHid + 16 * ti + i] : 0.f; },
                 [&](int k, int j) { return pt(k) ? X[(long)k * kIn + 16 * tj + j] : 0.f; }, acc, k0, ks);
  } else if (tile < 40) {
    kind = 1, ti = (tile - 24) / 4, tj = (tile - 24) % 4;
    acc = mfma32(K, [&](int i, int k) { return pt(k) ? D2[(long)k * kHid + 16 * ti + i] : 0.f; },
                 [&](int k, int j) { return pt(k) ? H1[(long)k * kHid + 16 * tj + j] : 0.f; },
                 acc, k0, ks);
  } else if (tile < 44) {
    kind = 2, ti = 0, tj = tile - 40;
    acc = mfma32(
        K, [&](int i, int k) { return pt(k) && i < kOut ? DY[(long)k * kOut + i] : 0.f; },
        [&](int k, int j) { return pt(k) ? H2[(long)k * kHid + 16 * tj + j] : 0.f; }, acc, k0, ks);
  } else {
    // bias tiles: 44..47 -> b1 rows, 48..51 -> b2 rows, 52 -> b3
    kind = 3 + (tile - 44) / 4;
    ti = (tile - 44) % 4;
    tj = 0;
    const float *Dm = tile < 48 ? D1 : tile < 52 ? D2 : DY;
    const int ld = tile < 52 ? kHid : kOut, nr = tile < 52 ? 16 : kOut;
    const int r0 = tile < 52 ? 16 * ti : 0;
    acc = mfma32(K, [&](int i, int k) { return pt(k) && i < nr ? Dm[(long)k * ld + r0 + i] : 0.f; },
                 [&](int k, int j) { return pt(k) && j == 0 ? 1.f : 0.f; }, acc, k0, ks);
  }
  part[wv][ln] = acc;
  __syncthreads();
  if (wv != 0) return;
  for (int q = 1; q < kGradWaves; ++q) acc += part[q][ln];
  for (int r = 0; r < 4; ++r) {
    const int i = 4 * (ln / 16) + r, j = ln % 16;
    const float v = acc[r];
    if (kind == 0)
      G[oW1 + (16 * ti + i) * kIn + 16 * tj + j] = v;
    else if (kind == 1)
      G[oW2 + (16 * ti + i) * kHid + 16 * tj + j] = v;
    else if (kind == 2) {
      if (i < kOut) G[oW3 + i * kHid + 16 * tj + j] = v;
    } else if (j == 0) {
      if (kind == 3) G[oB1 + 16 * ti + i] = v;
      else if (kind == 4) G[oB2 + 16 * ti + i] = v;
      else if (i < kOut) G[oB3 + i] = v;
    }
  }
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
// The 96 inputs of F point f (state fpts[f]) into o[0 .. 95]: the weighted
// test-vector values at the point and its coarse neighbours (scaled by
// their largest magnitude), the stencil ratios b_ij / b_ii, the exact LS row
// and the neighbour mask.
template <class T>
__device__ __forceinline__ void mlp_point_features(
    int f, const int *__restrict__ fpts, int r, const int *__restrict__ prp,
    const int *__restrict__ pci, const int *__restrict__ cpts, const T *__restrict__ V,
    const double *__restrict__ wv, const int *__restrict__ brp, const int *__restrict__ bci,
    const T *__restrict__ bv, const T *__restrict__ Pv, float *__restrict__ o) {
  const int i = fpts[f];
  const int a0 = prp[i], m = min(prp[i + 1] - a0, kOut);
  int J[kOut];
  for (int t = 0; t < kOut; ++t) J[t] = t < m ? cpts[pci[a0 + t]] : -1;
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

template <class T>
__global__ void k_mlp_features(int nF, const int *__restrict__ fpts, int r,
                               const int *__restrict__ prp, const int *__restrict__ pci,
                               const int *__restrict__ cpts, const T *__restrict__ V,
                               const double *__restrict__ wv, const int *__restrict__ brp,
                               const int *__restrict__ bci, const T *__restrict__ bv,
                               const T *__restrict__ Pv, float *__restrict__ F) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nF) return;
  mlp_point_features<T>(f, fpts, r, prp, pci, cpts, V, wv, brp, bci, bv, Pv, F + (size_t)f * kIn);
}

// LS objective sum_k w_k (v_i - sum_t p_t v_{j_t})^2 of the MLP row (the
// exact row in Pv plus the network's correction y) against the exact row;
// the MLP row replaces it if within 2x. Returns whether it did.
template <class T>
__device__ __forceinline__ bool mlp_point_select(int f, const int *__restrict__ fpts, int r,
                                                 const int *__restrict__ prp,
                                                 const int *__restrict__ pci,
                                                 const int *__restrict__ cpts,
                                                 const T *__restrict__ V,
                                                 const double *__restrict__ wv,
                                                 const float *__restrict__ y,
                                                 T *__restrict__ Pv) {
  const int i = fpts[f];
  const int a0 = prp[i], m = min(prp[i + 1] - a0, kOut);
  int J[kOut];
  double pl[kOut], pm[kOut];
  for (int t = 0; t < m; ++t) {
    J[t] = cpts[pci[a0 + t]];
    pl[t] = (double)Pv[a0 + t];
    pm[t] = pl[t] + (double)y[t];
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
  const bool take = jm <= 2.0 * jl;
  if (take)
    for (int t = 0; t < m; ++t) Pv[a0 + t] = (T)pm[t];
  return take;
}

// The features of one point by four lanes: part g (0..3) writes the entries
// of test vectors k = 2g, 2g + 1 and of neighbours t = 2g, 2g + 1; every
// entry is formed by the same operations as mlp_point_features (the scale
// S is a maximum, combined across the four lanes exactly), so the row is
// the same bit for bit. The four lanes of a point are l, l ^ 16, l ^ 32 and
// l ^ 48 of one wave; `valid` is uniform across them.
template <class T>
__device__ __forceinline__ void mlp_point_features4(
    int f, bool valid, int g, const int *__restrict__ fpts, int r, const int *__restrict__ prp,
    const int *__restrict__ pci, const int *__restrict__ cpts, const T *__restrict__ V,
    const double *__restrict__ wv, const int *__restrict__ brp, const int *__restrict__ bci,
    const T *__restrict__ bv, const T *__restrict__ Pv, float *__restrict__ o) {
  int i = 0, a0 = 0, m = 0;
  int J[kOut];
  double S = 0.0;
  if (valid) {
    i = fpts[f];
    a0 = prp[i];
    m = min(prp[i + 1] - a0, kOut);
    for (int t = 0; t < kOut; ++t) J[t] = t < m ? cpts[pci[a0 + t]] : -1;
    for (int k = 2 * g; k < 2 * g + 2; ++k) {
      const double sw = k < r ? sqrt(wv[k]) : 0.0;
      double a = k < r ? fabs(sw * (double)V[(size_t)i * r + k]) : 0.0;
      S = fmax(S, a);
      for (int t = 0; t < m; ++t)
        if (k < r) S = fmax(S, fabs(sw * (double)V[(size_t)J[t] * r + k]));
    }
  }
  S = fmax(S, __shfl_xor(S, 16, kWave));
  S = fmax(S, __shfl_xor(S, 32, kWave));
  if (!valid) return;
  if (!(S > 0.0)) S = 1.0;
  for (int k = 2 * g; k < 2 * g + 2; ++k) {
    const double sw = k < r ? sqrt(wv[k]) : 0.0;
    o[9 * k] = k < r ? (float)(sw * (double)V[(size_t)i * r + k] / S) : 0.f;
    for (int t = 0; t < kOut; ++t)
      o[9 * k + 1 + t] = (k < r && t < m) ? (float)(sw * (double)V[(size_t)J[t] * r + k] / S) : 0.f;
  }
  double bii = 1.0;
  for (int a = brp[i]; a < brp[i + 1]; ++a)
    if (bci[a] == i) bii = (double)bv[a];
  if (bii == 0.0) bii = 1.0;
  for (int t = 2 * g; t < 2 * g + 2; ++t) {
    double bij = 0.0;
    if (t < m)
      for (int a = brp[i]; a < brp[i + 1]; ++a)
        if (bci[a] == J[t]) bij = (double)bv[a];
    o[72 + t] = (float)(bij / bii);
    o[80 + t] = t < m ? (float)Pv[a0 + t] : 0.f;
    o[88 + t] = t < m ? 1.f : 0.f;
  }
}

// The objective test of one point by four lanes: part g forms the residuals
// em, el of test vectors 2g, 2g + 1 as mlp_point_select does; part 0 then
// adds the terms w_k e_k^2 in the order k = 0 .. r - 1 and writes the row.
// Returns the decision in every lane of the point.
template <class T>
__device__ __forceinline__ bool mlp_point_select4(int f, bool valid, int g,
                                                  const int *__restrict__ fpts, int r,
                                                  const int *__restrict__ prp,
                                                  const int *__restrict__ pci,
                                                  const int *__restrict__ cpts,
                                                  const T *__restrict__ V,
                                                  const double *__restrict__ wv,
                                                  const float *__restrict__ y,
                                                  T *__restrict__ Pv) {
  int i = 0, a0 = 0, m = 0;
  int J[kOut];
  double pl[kOut], pm[kOut];
  double em[2] = {0.0, 0.0}, el[2] = {0.0, 0.0};
  if (valid) {
    i = fpts[f];
    a0 = prp[i];
    m = min(prp[i + 1] - a0, kOut);
    for (int t = 0; t < m; ++t) {
      J[t] = cpts[pci[a0 + t]];
      pl[t] = (double)Pv[a0 + t];
      pm[t] = pl[t] + (double)y[t];
    }
    for (int q = 0; q < 2; ++q) {
      const int k = 2 * g + q;
      if (k >= r) continue;
      double e1 = (double)V[(size_t)i * r + k], e2 = e1;
      for (int t = 0; t < m; ++t) {
        const double vj = (double)V[(size_t)J[t] * r + k];
        e1 -= pm[t] * vj;
        e2 -= pl[t] * vj;
      }
      em[q] = e1;
      el[q] = e2;
    }
  }
  // part 0 gathers the residuals of k = 0 .. 7 from the four parts
  double ems[8], els[8];
  const int lane = threadIdx.x % kWave, base = lane % 16;
#pragma unroll
  for (int gg = 0; gg < 4; ++gg)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      ems[2 * gg + q] = __shfl(em[q], base + 16 * gg, kWave);
      els[2 * gg + q] = __shfl(el[q], base + 16 * gg, kWave);
    }
  bool take = false;
  if (valid && g == 0) {
    double jm = 0.0, jl = 0.0;
    for (int k = 0; k < r; ++k) {
      jm += wv[k] * ems[k] * ems[k];
      jl += wv[k] * els[k] * els[k];
    }
    take = jm <= 2.0 * jl;
    if (take)
      for (int t = 0; t < m; ++t) Pv[a0 + t] = (T)pm[t];
  }
  return __shfl((int)take, base, kWave) != 0;
}

// The learned F rows of one level in one launch: each wave takes 16 F
// points, forms their features in LDS (four lanes per point), runs the
// network on them as k_mlp_infer does (the same BF16 operands and MFMA
// order) and applies the objective test to its outputs (four lanes per
// point again), so the 96 inputs and 8 outputs of a point never pass through
// memory; the results are those of k_mlp_features, k_mlp_infer and the test
// one after the other. A point reads and writes only its own row of P, so
// the points of a launch are independent. The hidden layers and the outputs
// reuse the feature rows' LDS once layer 1 has read them. counts[0] /
// counts[1]: points that took the network's / kept the exact row.
template <class T>
__global__ void __launch_bounds__(kInferWaves * kWave)
    k_mlp_apply(const __bf16 *__restrict__ wb, const float *__restrict__ par, int nF,
                const int *__restrict__ fpts, int r, const int *__restrict__ prp,
                const int *__restrict__ pci, const int *__restrict__ cpts,
                const T *__restrict__ V, const double *__restrict__ wv,
                const int *__restrict__ brp, const int *__restrict__ bci,
                const T *__restrict__ bv, T *__restrict__ Pv, int *__restrict__ counts) {
  static_assert(kOut == 8, "four lanes of two test vectors and two neighbours each");
  __shared__ __attribute__((aligned(16))) __bf16 w[kNBf];
  __shared__ float bias[kHid + kHid + kOut];
  // per wave: 16 feature rows (6 KB); later h1 | h2 (2 KB each, BF16) and
  // the 16 outputs (512 B) in the same space
  __shared__ __attribute__((aligned(16))) float xs[kInferWaves][16 * kIn];
  for (int e = threadIdx.x; e < kNBf; e += blockDim.x) w[e] = wb[e];
  for (int e = threadIdx.x; e < kHid; e += blockDim.x) {
    bias[e] = par[oB1 + e];
    bias[kHid + e] = par[oB2 + e];
  }
  for (int e = threadIdx.x; e < kOut; e += blockDim.x) bias[2 * kHid + e] = par[oB3 + e];
  const int wv_ = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const long p0 = ((long)blockIdx.x * kInferWaves + wv_) * 16;
  float *X = xs[wv_];
  const int q = l % 16, g = l / 16;
  const bool valid = p0 + q < nF;
  mlp_point_features4<T>((int)(p0 + q), valid, g, fpts, r, prp, pci, cpts, V, wv, brp, bci, bv,
                         Pv, X + q * kIn);
  __syncthreads();
  const int row = l % 16, kq = 8 * (l / 16), rq = 4 * (l / 16);
  const long pr = p0 + row;  // the point whose A row this lane loads
  __bf16 *h1 = reinterpret_cast<__bf16 *>(X), *h2 = h1 + 16 * kHid;
  float *ys = X + 16 * kHid;  // after h1 | h2 (2 x 16 x 64 BF16 = 16 x 64 floats)
  // layer 1: [16 x 96] x [96 x 64]; every lane's A operands are in
  // registers before the wave's first MFMA, so h1 may overwrite the rows
  f32x4 acc[4];
  for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 a1[kIn / 32];
#pragma unroll
  for (int ks = 0; ks < kIn / 32; ++ks)
#pragma unroll
    for (int e = 0; e < 8; ++e)
      a1[ks][e] = (__bf16)(pr < nF ? X[row * kIn + 32 * ks + kq + e] : 0.f);
  __syncthreads();
#pragma unroll
  for (int ks = 0; ks < kIn / 32; ++ks)
    for (int nb = 0; nb < 4; ++nb) {
      const bf16x8 b = *(const bf16x8 *)&w[bW1 + (16 * nb + row) * kIn + 32 * ks + kq];
      acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[ks], b, acc[nb], 0, 0, 0);
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
    for (int e = 0; e < 4; ++e) ys[(rq + e) * kOut + row] = o[e] + bias[2 * kHid + row];
  __syncthreads();
  const bool take = mlp_point_select4<T>((int)(p0 + q), valid, g, fpts, r, prp, pci, cpts, V, wv,
                                         ys + q * kOut, Pv);
  // one counter update per wave (the point's part-0 lanes)
  const unsigned long long bt = __ballot(valid && g == 0 && take);
  const unsigned long long bf = __ballot(valid && g == 0 && !take);
  if (l == 0) {
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

static void mlp_tile_attr() {
  static const bool done = [] {
    return hipFuncSetAttribute((const void *)k_mlp_tile,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)mlp_tile_lds()) == hipSuccess;
  }();
  if (!done) fail(BAMG_E_DEVICE, "k_mlp_tile: dynamic LDS size not accepted");
}

void mlp_forward(const bamg_mlp *m, const float *X, long npts, float *Y, int mode, hipStream_t s) {
  if (npts <= 0) return;
  if (mode == 1) {
    const long waves = (npts + 15) / 16;
    k_mlp_infer<<<ceil_div(waves, kInferWaves), kInferWaves * kWave, 0, s>>>(m->wb, m->p, X,
                                                                            npts, Y);
  } else {
    mlp_tile_attr();
    k_mlp_tile<<<ceil_div(npts, kTileP), 256, mlp_tile_lds(), s>>>(
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
  mlp_tile_attr();
  k_mlp_tile<<<ceil_div(npts, kTileP), 256, mlp_tile_lds(), s>>>(
      m->p, X, T, M, npts, scale, w.H1, w.H2, w.D1, w.D2, w.DY, nullptr, w.pl);
  LAUNCHCHK();
  k_mlp_wgrad_mfma<<<kGradTiles, kGradWaves * kWave, 0, s>>>(X, w.H1, w.H2, w.D1, w.D2, w.DY, npts, w.G);
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
void mlp_apply(const Level &L, int r, const T *V, const double *wv, const bamg_mlp *m, T *Pv,
               int *counts, hipStream_t s) {
  if (L.nF <= 0) return;
  const long waves = ((long)L.nF + 15) / 16;
  k_mlp_apply<T><<<ceil_div(waves, kInferWaves), kInferWaves * kWave, 0, s>>>(
      m->wb, m->p, L.nF, L.fpts, r, L.P.rp, L.P.ci, L.cpts, V, wv, L.B.rp, L.B.ci,
      (const T *)L.Bv, Pv, counts);
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
  template void mlp_apply<T>(const Level &, int, const T *, const double *, const bamg_mlp *,  \
                             T *, int *, hipStream_t);                                         \
  template void mlp_targets<T>(const Level &, const T *, float *, float *, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace bamg
