// Device helpers shared by the kernels of the HIP library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bamg {

constexpr int kWave = 64;

// Philox-4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 64x64 -> 128-bit products with the round multipliers, key bumped by the
// Weyl constants between rounds. Returns the first output word.
__device__ __forceinline__ uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t c2,
                                                 uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return c0;
}

// [-1, 1) from the top 53 bits; every step is exact in FP64.
__device__ __forceinline__ double uniform_pm1(uint64_t seed, uint64_t side, uint64_t k,
                                              uint64_t i) {
  const uint64_t w = philox_word0(i, k, side, 0, seed, 0);
  const double u = (double)(w >> 11) * 0x1.0p-53;
  return 2.0 * u - 1.0;
}

// Sum over a group of `width` consecutive lanes (width a power of two <= 64).
template <class X>
__device__ __forceinline__ X group_sum(X v, int width) {
  for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, width);
  return v;
}

// Three group sums at once: the same butterfly as group_sum for each value
// (bit-identical results), with the three shuffle chains interleaved so
// their latencies overlap.
template <class X>
__device__ __forceinline__ void group_sum3(X &a, X &b, X &c, int width) {
  for (int off = width >> 1; off > 0; off >>= 1) {
    const X ta = __shfl_xor(a, off, width), tb = __shfl_xor(b, off, width),
            tc = __shfl_xor(c, off, width);
    a += ta;
    b += tb;
    c += tc;
  }
}

// The dispatcher hands workgroup b to XCD b % 8. Renumbering so that XCD x
// owns one contiguous range of logical blocks keeps neighbouring rows (and
// the vector entries they gather) in one XCD's L2 instead of all eight.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  const int q = nblocks / kXcds, r = nblocks % kXcds;
  const int x = b % kXcds, k = b / kXcds;
  return x * q + (x < r ? x : r) + k;
}

// Block-wide sum of one FP64 value per thread; result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = group_sum(v, kWave);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / kWave; ++i) r += sh[i];
  __syncthreads();
  return r;
}

}  // namespace bamg
