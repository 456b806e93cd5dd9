// Row sums of CSR matrices shared by the one-kernel-per-step sparse
// kernels and the batched persistent solve, so both form every row's sum in
// the same order.
#pragma once

#include "device_common.h"

namespace bamg {

// A lane's share of a CSR row, sum over k = k0, k0 + LPR, ... < e of
// val[k] * g(ci[k]), added in that order. U = 4 entries per round: their
// indices and values are loaded first, then the four gathers, so a short
// row costs one dependent round trip instead of a chain of them (8 per
// round raises the register count past what full occupancy allows, and is
// slower). Positions past the row end load the row's last entry again (no
// branches around the loads, so all of them are in flight together) and
// are not added.
template <class T, int LPR, class G>
__device__ __forceinline__ T lane_dot(int k0, int e, const int *__restrict__ ci,
                                      const T *__restrict__ val, G g) {
  constexpr int U = 4;
  T sum = 0;
  for (int k = k0; k < e; k += U * LPR) {
    int c[U];
    T v[U], xv[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int kk = min(k + j * LPR, e - 1);
      c[j] = ci[kk];
      v[j] = val[kk];
    }
#pragma unroll
    for (int j = 0; j < U; ++j) xv[j] = g(c[j]);
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (k + j * LPR < e) sum += v[j] * xv[j];
  }
  return sum;
}

// The sum of a CSR row, sum over k in [rs, e) of val[k] * g(ci[k]), in one
// fixed order whatever the number LPR <= 4 of lanes sharing the row, so
// results do not depend on the lanes a tuner picks: entry k goes to partial
// (k - rs) mod 4, each partial adds its entries in ascending order, and the
// four partials are combined as (p0+p1)+(p2+p3). Lane `lane` of the group
// holds the partials lane, lane + LPR, ...; a level of the combining tree is
// a cross-lane shuffle when the two partials sit in different lanes and a
// register add otherwise (both lanes of a shuffle form the same sum:
// addition is commutative). Every lane of the group returns the row sum.
// Loads as in lane_dot: U = 4 entries per round, indices and values first,
// then the gathers. Four partials keep every sweep kernel at full occupancy
// (eight took the one-lane sweep from 42 to 65 VGPRs).
constexpr int kCanon = 4;

template <class T, int LPR, class G>
__device__ __forceinline__ T row_dot(int rs, int e, int lane, const int *__restrict__ ci,
                                     const T *__restrict__ val, G g) {
  static_assert(LPR >= 1 && LPR <= kCanon, "canonical row sums take at most 4 lanes");
  constexpr int R = kCanon / LPR, U = 4, PH = R > U ? R / U : 1;
  T acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0;
  for (int k = rs + lane; k < e; k += PH * U * LPR) {
#pragma unroll
    for (int ph = 0; ph < PH; ++ph) {
      const int kp = k + ph * U * LPR;
      if (ph == 0 || kp < e) {
        int c[U];
        T v[U], xv[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
          const int kk = min(kp + j * LPR, e - 1);
          c[j] = ci[kk];
          v[j] = val[kk];
        }
#pragma unroll
        for (int j = 0; j < U; ++j) xv[j] = g(c[j]);
#pragma unroll
        for (int j = 0; j < U; ++j)
          if (kp + j * LPR < e) acc[(ph * U + j) % R] += v[j] * xv[j];
      }
    }
  }
#pragma unroll
  for (int st = 1; st < kCanon; st <<= 1) {
    if (st < LPR) {
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = acc[r] + __shfl_xor(acc[r], st, LPR);
    } else {
      const int step = st / LPR;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if ((r & step) == 0 && r + step < R) acc[r] = acc[r] + acc[r + step];
    }
  }
  return acc[0];
}

// Row sum for any LPR: the canonical order up to 4 lanes; wider groups (an
// SpMV whose lanes follow from the row length alone, such as the coarsest
// level's residual in a W-cycle) add their lanes' shares by a butterfly.
template <class T, int LPR, class G>
__device__ __forceinline__ T row_sum(int rs, int e, int lane, const int *__restrict__ ci,
                                     const T *__restrict__ val, G g) {
  if constexpr (LPR <= kCanon) {
    return row_dot<T, LPR>(rs, e, lane, ci, val, g);
  } else {
    return group_sum(lane_dot<T, LPR>(rs + lane, e, ci, val, g), LPR);
  }
}

// Weighted-Jacobi row updates (Section 3): the first sweep from x = 0 and a
// sweep from x_r, given the row sum of A x.
template <class T>
__device__ __forceinline__ T jacobi_first(T omega, T dr, T br) {
  return omega * dr * br;
}
template <class T>
__device__ __forceinline__ T jacobi_next(T xr, T omega, T dr, T br, T sum) {
  return xr + omega * dr * (br - sum);
}

}  // namespace bamg
