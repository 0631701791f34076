// Coefficient updates shared by the build and the fit kernels: rounding FP32 to BF16 storage, and
// one Adam step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "common.hpp"

namespace pws {

// FP32 -> BF16 bits, round to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// One Adam update (Kingma and Ba, Algorithm 1) of a coefficient p with gradient g and moments m, v:
//     m <- b1 m + (1 - b1) g,   v <- b2 v + (1 - b2) g^2,
//     p <- p - s m / (sqrt(v) r + eps),   s = lr / (1 - b1^t),  r = 1 / sqrt(1 - b2^t),
// the bias corrections of step t folded into s and r on the host; in the precision T of the moments.
template <typename T> struct AdamCoef {
  T b1, c1, b2, c2, step_size, inv_sqrt_bc2, eps;   // c1 = 1 - b1, c2 = 1 - b2
};

template <typename T>
inline AdamCoef<T> adam_coef(double lr, double b1, double b2, double eps, int step) {
  const double bc1 = 1.0 - std::pow(b1, step), bc2 = 1.0 - std::pow(b2, step);
  return AdamCoef<T>{(T)b1, (T)(1.0 - b1), (T)b2, (T)(1.0 - b2), (T)(lr / bc1), (T)(1.0 / std::sqrt(bc2)), (T)eps};
}

template <typename T>
__device__ __forceinline__ void adam_update(const AdamCoef<T>& k, T g, T& p, T& m, T& v) {
  m = fmaa(k.b1, m, k.c1 * g);
  v = fmaa(k.b2, v, k.c2 * (g * g));
  p = p - k.step_size * (m / fmaa(sqrt(v), k.inv_sqrt_bc2, k.eps));
}

}  // namespace pws
