// Shared host/device helpers of the pwspline library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pwspline.h"

namespace pws {

// ---------------------------------------------------------------- host-side errors
int fail(int code, const char* fmt, ...);          // records the message, returns code
int hip_fail(hipError_t err, const char* what);    // SPL_EHIP with the HIP error string
void clear_error();
int check_desc(const spl_desc* d);                 // desc_init was run and fields are consistent

// ---------------------------------------------------------------- vector types
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

// Geometry of one periodic table, passed by value to kernels.
struct Geom {
  double ainv[9];    // s = ainv . r (crystal coordinates)
  double jac[9];     // J[i][c] = N_i ainv[i][c]
  double metric[6];  // M00 M11 M22 M01 M02 M12 of M = J J^T
  int32_t n[3];      // grid points per axis
  int32_t o_pad;     // orbital stride of a table row
  int64_t s0, s1;    // row strides (elements) of the first and second grid index
};

Geom make_geom(const spl_desc* d);

// Accumulator type: FP64 tables accumulate in FP64, FP32 and BF16 tables in FP32.
template <typename TS> struct Acc { using type = float; };
template <> struct Acc<double> { using type = double; };

// ---------------------------------------------------------------- device helpers
// Every fused multiply-add in device code is written out (the library is built with
// -ffp-contract=off), so all kernels sharing a code path round identically.
__host__ __device__ __forceinline__ double fmaa(double a, double b, double c) { return __builtin_fma(a, b, c); }
__host__ __device__ __forceinline__ float fmaa(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Reduced coordinates (Sec. II, Eq. reducedcoordinate): s = a^-1 r folded into [0,1),
// u = N s, i0 = floor(u), t = u - i0.  Always FP64.  A non-finite point returns false
// with i0 = 0, t = 0 so every later index stays inside the table.  Host and device: the
// host build serves a CPU check of the indices over adversarial positions.
__host__ __device__ __forceinline__ bool reduce_point(const Geom& g, double r0, double r1, double r2,
                                                      int i0[3], double t[3]) {
  bool ok = __builtin_isfinite(r0) && __builtin_isfinite(r1) && __builtin_isfinite(r2);
  if (!ok) { r0 = 0.0; r1 = 0.0; r2 = 0.0; }
  double s[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s[i] = fmaa(g.ainv[3 * i + 2], r2, fmaa(g.ainv[3 * i + 1], r1, g.ainv[3 * i] * r0));
    ok = ok && __builtin_isfinite(s[i]);    // a finite position can still overflow here
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double si = ok ? s[i] - floor(s[i]) : 0.0;   // in [0, 1]
    const double u = (double)g.n[i] * si;              // in [0, N]
    const double fl = floor(u);
    int k = (int)fl;
    double ti = u - fl;
    if (k >= g.n[i]) k -= g.n[i];                      // s or u rounded up to the cell edge
    if (k < 0 || k >= g.n[i]) { k = 0; ti = 0.0; }     // unreachable; keeps every index inside the table
    i0[i] = k;
    t[i] = ti;
  }
  return ok;
}

// Cubic B-spline weights for the rows i0-1, i0, i0+1, i0+2 at reduced coordinate t in [0,1),
// standard normalization (sum 1): (1-t)^3/6, (3t^3 - 6t^2 + 4)/6, (-3t^3 + 3t^2 + 3t + 1)/6, t^3/6,
// with first and second derivatives in t.
template <typename A>
__device__ __forceinline__ void bspline_weights(A t, A w[4], A dw[4], A d2w[4]) {
  const A s = A(1) - t;
  const A t2 = t * t;
  const A sixth = A(1) / A(6);
  w[0] = sixth * (s * s * s);
  w[1] = sixth * fmaa(t2, fmaa(A(3), t, A(-6)), A(4));
  w[2] = sixth * fmaa(t2, fmaa(A(-3), t, A(3)), fmaa(A(3), t, A(1)));
  w[3] = sixth * (t2 * t);
  dw[0] = A(-0.5) * (s * s);
  dw[1] = A(0.5) * (t * fmaa(A(3), t, A(-4)));
  dw[2] = A(0.5) * fmaa(t, fmaa(A(-3), t, A(2)), A(1));
  dw[3] = A(0.5) * t2;
  d2w[0] = s;
  d2w[1] = fmaa(A(3), t, A(-2));
  d2w[2] = fmaa(A(-3), t, A(1));
  d2w[3] = t;
}

template <typename A>
__device__ __forceinline__ void bspline_values(A t, A w[4]) {
  const A s = A(1) - t;
  const A t2 = t * t;
  const A sixth = A(1) / A(6);
  w[0] = sixth * (s * s * s);
  w[1] = sixth * fmaa(t2, fmaa(A(3), t, A(-6)), A(4));
  w[2] = sixth * fmaa(t2, fmaa(A(-3), t, A(3)), fmaa(A(3), t, A(1)));
  w[3] = sixth * (t2 * t);
}

// Cubic Lagrange weights for the rows i0-1, i0, i0+1, i0+2 at reduced coordinate t in [0,1)
// (App. A, Eq. lagrangebasis): -t(t-1)(t-2)/6, (t+1)(t-1)(t-2)/2, -(t+1)t(t-2)/2, (t+1)t(t-1)/6.
template <typename A>
__device__ __forceinline__ void lagrange_values(A t, A w[4]) {
  const A tp = t + A(1), tm = t - A(1), tm2 = t - A(2);
  const A sixth = A(1) / A(6);
  w[0] = -sixth * (t * tm * tm2);
  w[1] = A(0.5) * (tp * tm * tm2);
  w[2] = A(-0.5) * (tp * t * tm2);
  w[3] = sixth * (tp * t * tm);
}

// pp-spline basis (App. A, Eq. pp-splinebasis) at reduced coordinate t in [0,1), in the order
// (grid point i0, value), (i0, second derivative), (i0+1, value), (i0+1, second derivative):
// 1 - t, -t^3/6 + t^2/2 - t/3, t, t^3/6 - t/6; with first and second derivatives in t.
template <typename A>
__device__ __forceinline__ void pp_values(A t, A w[4]) {
  const A sixth = A(1) / A(6);
  w[0] = A(1) - t;
  w[1] = t * fmaa(t, fmaa(-sixth, t, A(0.5)), A(-1) / A(3));
  w[2] = t;
  w[3] = sixth * (t * fmaa(t, t, A(-1)));
}

template <typename A>
__device__ __forceinline__ void pp_weights(A t, A w[4], A dw[4], A d2w[4]) {
  pp_values<A>(t, w);
  const A sixth = A(1) / A(6);
  dw[0] = A(-1);
  dw[1] = fmaa(t, fmaa(A(-0.5), t, A(1)), A(-1) / A(3));
  dw[2] = A(1);
  dw[3] = fmaa(A(0.5), t * t, -sixth);
  d2w[0] = A(0);
  d2w[1] = A(1) - t;
  d2w[2] = A(0);
  d2w[3] = t;
}

// Four-term dot product in a fixed order: w0 x0 + w1 x1 + w2 x2 + w3 x3.
template <typename A>
__device__ __forceinline__ A dot4(const A w[4], A x0, A x1, A x2, A x3) {
  return fmaa(w[3], x3, fmaa(w[2], x2, fmaa(w[1], x1, w[0] * x0)));
}

// Spread the low 10 bits of x to every third bit (one coordinate of a 3D Morton index).
__device__ __forceinline__ uint32_t spread3(uint32_t x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

// Row indices i0-1 .. i0+2 modulo n (n >= 4, 0 <= i0 < n).
__host__ __device__ __forceinline__ void wrap4(int i0, int n, int idx[4]) {
  idx[0] = (i0 == 0) ? n - 1 : i0 - 1;
  idx[1] = i0;
  idx[2] = (i0 + 1 >= n) ? i0 + 1 - n : i0 + 1;
  idx[3] = (i0 + 2 >= n) ? i0 + 2 - n : i0 + 2;
}

// Load VEC = 16 / sizeof(TS) consecutive stored coefficients as accumulator values.
template <typename TS> struct Row16;

template <> struct Row16<double> {
  static constexpr int VEC = 2;
  __device__ __forceinline__ static void load(const double* p, double x[2]) {
    const d2v v = *reinterpret_cast<const d2v*>(p);
    x[0] = v.x; x[1] = v.y;
  }
};

template <> struct Row16<float> {
  static constexpr int VEC = 4;
  __device__ __forceinline__ static void load(const float* p, float x[4]) {
    const f4v v = *reinterpret_cast<const f4v*>(p);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  }
};

// BF16 is stored as raw 16-bit patterns; widening to FP32 is a 16-bit shift.
template <> struct Row16<uint16_t> {
  static constexpr int VEC = 8;
  __device__ __forceinline__ static void load(const uint16_t* p, float x[8]) {
    const u4v v = *reinterpret_cast<const u4v*>(p);
    x[0] = __uint_as_float(v.x << 16); x[1] = __uint_as_float(v.x & 0xffff0000u);
    x[2] = __uint_as_float(v.y << 16); x[3] = __uint_as_float(v.y & 0xffff0000u);
    x[4] = __uint_as_float(v.z << 16); x[5] = __uint_as_float(v.z & 0xffff0000u);
    x[6] = __uint_as_float(v.w << 16); x[7] = __uint_as_float(v.w & 0xffff0000u);
  }
};

// Output element type: FP64 for FP64 tables, FP32 otherwise.
template <typename TS> struct Out { using type = float; };
template <> struct Out<double> { using type = double; };

}  // namespace pws
