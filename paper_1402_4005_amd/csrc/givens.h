// Givens rotations of GMRES's Hessenberg update (Section 6), with every
// fused multiply-add written out: an expression such as c a + s b can be
// contracted around either product, and the compiler's choice may differ
// from kernel to kernel, so the per-step and the batched solves both call
// these and round identically.
#pragma once

#include <hip/hip_runtime.h>

namespace bamg {

// (a, b) <- (c a + s b, -s a + c b)
__device__ __forceinline__ void givens_apply(double c, double s, double &a, double &b) {
  const double a2 = fma(c, a, s * b);
  const double b2 = fma(-s, a, c * b);
  a = a2;
  b = b2;
}

// sqrt(a^2 + b^2), the entry that remains after the rotation zeroing b
__device__ __forceinline__ double givens_norm(double a, double b) { return sqrt(fma(a, a, b * b)); }

}  // namespace bamg
