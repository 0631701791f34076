// Forward evaluation kernels: orbital values, gradients and Laplacians through the periodic
// tricubic B-spline (App. A, Eq. b-splineapproximation; chain rule of Sec. II), and the other
// representations the paper compares: cubic Lagrange interpolation of grid values (App. A,
// Eq. lagrangeinterpolation3) and separate interpolants of the gradient and the Laplacian
// (Sec. III A, Fig. 1), for real orbitals and for Bloch orbitals exp(i k.r) u(r) (Sec. I).
//
// Mapping.  A group of G lanes (G a power of two, 2..256) owns one point; lane c of the group
// owns the orbital chunks c, c+G, c+2G, ... where a chunk is OPL consecutive orbitals (one
// vector load of OPL stored coefficients per table row).  The orbital index is innermost in
// the table, so the G lanes of a group read contiguous bytes of each of the 64 rows of the
// point's 4x4x4 block: every load is coalesced.  The reduced coordinate and the 36 one-
// dimensional weights of a point are computed once per group (wave-uniform when G >= 64).
//
// Contraction.  Separable, innermost grid axis first: for each of the 16 (l, m) row pairs the
// 4 coefficients along the third axis are reduced with (b, b', b'') of t_3; those partial sums
// are folded with the second axis' weights into six sums for the current l, and those with
// the first axis' weights into the ten reduced derivatives (value, 3 first, 6 second): about
// 340 FMA per orbital instead of 640.  The chain rule then gives Cartesian derivatives.
//
// Memory-level parallelism.  The loop over the first grid axis is kept rolled: one iteration
// contracts the 16 rows of one slab (l fixed) while the 16 loads of the next slab are in flight
// (a second register buffer, when a lane's slab is at most 16 bytes per row), with a register
// budget that leaves room for at least one more wave per SIMD.
// No matrix cores: the work is a gather followed by a short dot product, bound by memory.
//
// pp-spline tables (App. A, Piecewise-polynomial-form splines) hold 8 numbers per grid point; a
// point reads the 2x2x2 corners of its cell, which is again a 4x4x4 arrangement of 64 rows per
// orbital (per axis: corner i0 or i0+1, times value or second derivative), so the same contraction
// serves with the pp basis and corner addressing.
//
// Variants.  MODE_SEP reads five tables (orbital, d/dx, d/dy, d/dz, Laplacian) by value, with
// B-spline or Lagrange weights.  Bloch orbitals keep (Re u, Im u) in adjacent columns, so a lane
// with an even OPL holds whole pairs; after the contraction the product rule and the phase
// exp(i k.r) (FP64 argument, unfolded position) turn them into the orbital's complex outputs.
#pragma once
#include "common.hpp"

namespace pws {

struct EvalArgs {
  Geom g;
  const void* table;
  const double* pos;
  void* v;
  void* grad;
  void* lap;
  int32_t n_pts;
  int32_t n_orb;      // columns of an output row (stored real columns: 2 per Bloch orbital)
  int32_t n_chunks;   // ceil(n_orb / OPL): chunks holding at least one real column
  int32_t vec_store;  // n_orb % OPL == 0 and outputs 16-byte aligned: whole-vector stores
  int64_t tab_stride; // elements of one table: table q (separate Laplacian, gradients) starts at q * tab_stride
  double k[3];        // crystal momentum of Bloch orbitals (Bloch variants only)
  const int32_t* perm;  // locality order of the points (sorted evaluation), or null: point q is perm[q]
  int32_t per_xcd;      // with perm: tiles per XCD (workgroup b takes tile (b mod 8) * per_xcd + b / 8)
  int32_t lanes;        // batched launches with per-item shapes: lanes per point of this item (8 .. 256)
};

enum { MODE_V = 0, MODE_VGL = 1, MODE_VGL_SEPLAP = 2, MODE_SEP = 3 };
// variant bits of a kernel: Lagrange weights instead of B-spline, Bloch phase, pp-spline layout, and
// no slab prefetch (FP64 instances for cache-resident gathers: the sorted call)
enum { VAR_LAGRANGE = 1, VAR_BLOCH = 2, VAR_PP = 4, VAR_NOPF = 8 };

// ---------------------------------------------------------------- loads of OPL stored values
template <typename TS, int OPL> struct RowN;

template <> struct RowN<double, 1> {
  __device__ __forceinline__ static void load(const double* p, double x[1]) { x[0] = *p; }
};
template <> struct RowN<double, 2> {
  __device__ __forceinline__ static void load(const double* p, double x[2]) {
    const d2v v = *reinterpret_cast<const d2v*>(p);
    x[0] = v.x; x[1] = v.y;
  }
};
template <> struct RowN<float, 1> {
  __device__ __forceinline__ static void load(const float* p, float x[1]) { x[0] = *p; }
};
template <> struct RowN<float, 2> {
  __device__ __forceinline__ static void load(const float* p, float x[2]) {
    const f2v v = *reinterpret_cast<const f2v*>(p);
    x[0] = v.x; x[1] = v.y;
  }
};
template <> struct RowN<float, 4> {
  __device__ __forceinline__ static void load(const float* p, float x[4]) {
    const f4v v = *reinterpret_cast<const f4v*>(p);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  }
};
// BF16 is stored as raw 16-bit patterns; widening to FP32 is a 16-bit shift.
__device__ __forceinline__ void bf16x2(uint32_t w, float& lo, float& hi) {
  lo = __uint_as_float(w << 16);
  hi = __uint_as_float(w & 0xffff0000u);
}
template <> struct RowN<uint16_t, 2> {
  __device__ __forceinline__ static void load(const uint16_t* p, float x[2]) {
    bf16x2(*reinterpret_cast<const uint32_t*>(p), x[0], x[1]);
  }
};
typedef uint32_t u2v __attribute__((ext_vector_type(2)));
template <> struct RowN<uint16_t, 4> {
  __device__ __forceinline__ static void load(const uint16_t* p, float x[4]) {
    const u2v v = *reinterpret_cast<const u2v*>(p);
    bf16x2(v.x, x[0], x[1]);
    bf16x2(v.y, x[2], x[3]);
  }
};
template <> struct RowN<uint16_t, 8> {
  __device__ __forceinline__ static void load(const uint16_t* p, float x[8]) {
    const u4v v = *reinterpret_cast<const u4v*>(p);
    bf16x2(v.x, x[0], x[1]);
    bf16x2(v.y, x[2], x[3]);
    bf16x2(v.z, x[4], x[5]);
    bf16x2(v.w, x[6], x[7]);
  }
};

// ---------------------------------------------------------------- stores of OPL outputs
// Whole-vector stores only when the vector lies inside the n_orb real orbitals of the row;
// otherwise element by element with the tail masked (outputs are unpadded [.][n_orb]).
template <typename O, int OPL>
__device__ __forceinline__ void store_out(O* dst, const O (&x)[OPL], int o, int n_orb, bool vec_ok) {
  if (vec_ok && o + OPL <= n_orb) {
    if constexpr (sizeof(O) == 8 && OPL == 2) {
      __builtin_nontemporal_store(d2v{x[0], x[1]}, reinterpret_cast<d2v*>(dst + o));
      return;
    } else if constexpr (sizeof(O) == 4 && OPL == 2) {
      __builtin_nontemporal_store(f2v{x[0], x[1]}, reinterpret_cast<f2v*>(dst + o));
      return;
    } else if constexpr (sizeof(O) == 4 && OPL == 4) {
      __builtin_nontemporal_store(f4v{x[0], x[1], x[2], x[3]}, reinterpret_cast<f4v*>(dst + o));
      return;
    } else if constexpr (sizeof(O) == 4 && OPL == 8) {
      __builtin_nontemporal_store(f4v{x[0], x[1], x[2], x[3]}, reinterpret_cast<f4v*>(dst + o));
      __builtin_nontemporal_store(f4v{x[4], x[5], x[6], x[7]}, reinterpret_cast<f4v*>(dst + o + 4));
      return;
    }
  }
#pragma unroll
  for (int j = 0; j < OPL; ++j)
    if (o + j < n_orb) __builtin_nontemporal_store(x[j], dst + o + j);
}

template <typename A>
__device__ __forceinline__ A pick4(int l, A a0, A a1, A a2, A a3) {
  return l == 0 ? a0 : (l == 1 ? a1 : (l == 2 ? a2 : a3));
}

// Element offset of the first-axis slab l of a point's block: row ix[l] of the B-spline block, or
// the pp-spline's precomputed corner-and-kind offset xo[l].
template <bool PP>
__device__ __forceinline__ int64_t slab_offset(int l, const int ix[4], const int64_t xo[4], int64_t s0) {
  if constexpr (PP) return pick4(l, xo[0], xo[1], xo[2], xo[3]);
  else return (int64_t)pick4(l, ix[0], ix[1], ix[2], ix[3]) * s0;
}

// Software prefetch of the next first-axis slab: while slab l is contracted, the 16 loads of slab
// l+1 are already in flight (a second register buffer, copied over at the end of the iteration).
// It pays where the gather waits on HBM: FP64 tables (measured: +6% on the 113 MB Si table, +3% on
// the 1.8 GB MgO table).  For FP32/BF16 tables, and for gathers served from cache (the sorted call),
// the second buffer costs more in occupancy than it gains, so each slab is loaded at the top of its
// iteration instead.
template <typename A, int VAR> struct Prefetch {
  static constexpr bool on = sizeof(A) == 8 && (VAR & VAR_NOPF) == 0;
};

// The 16 rows (m, n) of first-axis slab l of a point's block, OPL columns from `tab`.
template <typename TS, int OPL, typename A, bool PP>
__device__ __forceinline__ void load_slab(const TS* __restrict__ tab, int l, const int ix[4], const int64_t xo[4],
                                          const int64_t ry[4], const int64_t rz[4], int64_t s0,
                                          A (&r)[4][4][OPL]) {
  const TS* slab = tab + slab_offset<PP>(l, ix, xo, s0);
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) RowN<TS, OPL>::load(slab + ry[m] + rz[n], r[m][n]);
}

template <typename A, int OPL>
__device__ __forceinline__ void copy_slab(A (&dst)[4][4][OPL], const A (&src)[4][4][OPL]) {
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int j = 0; j < OPL; ++j) dst[m][n][j] = src[m][n][j];
}

// Value of one table at a point for OPL consecutive columns: sum_lmn w_l w_m w_n beta_lmn.
// `tab` points at the column o of table row 0; the first-axis loop stays rolled (16 loads per
// slab, plus the next slab's 16 with the prefetch).
template <typename TS, int OPL, typename A, bool PP, bool PF>
__device__ __forceinline__ void value_pass(const TS* __restrict__ tab, const int ix[4], const int64_t xo[4],
                                           const int64_t ry[4], const int64_t rz[4], int64_t s0, const A wx[4],
                                           const A wy[4], const A wz[4], A out[OPL]) {
#pragma unroll
  for (int j = 0; j < OPL; ++j) out[j] = A(0);
  A r[4][4][OPL], nx[4][4][OPL];
  if constexpr (PF) load_slab<TS, OPL, A, PP>(tab, 0, ix, xo, ry, rz, s0, r);
#pragma unroll 1
  for (int l = 0; l < 4; ++l) {
    if constexpr (PF) {
      if (l < 3) load_slab<TS, OPL, A, PP>(tab, l + 1, ix, xo, ry, rz, s0, nx);
    } else {
      load_slab<TS, OPL, A, PP>(tab, l, ix, xo, ry, rz, s0, r);
    }
    const A xw = pick4(l, wx[0], wx[1], wx[2], wx[3]);
#pragma unroll
    for (int j = 0; j < OPL; ++j) {
      A q = A(0);
#pragma unroll
      for (int m = 0; m < 4; ++m) q = fmaa(wy[m], dot4(wz, r[m][0][j], r[m][1][j], r[m][2][j], r[m][3][j]), q);
      out[j] = fmaa(xw, q, out[j]);
    }
    if constexpr (PF) copy_slab<A, OPL>(r, nx);
  }
}

// (re, im) <- (c + i s)(re + i im) for every pair (2i, 2i+1) of x.
template <typename A, int OPL>
__device__ __forceinline__ void phase_pairs(A c, A s, A (&x)[OPL]) {
#pragma unroll
  for (int j = 0; j < OPL; j += 2) {
    const A re = x[j], im = x[j + 1];
    x[j] = fmaa(c, re, -(s * im));
    x[j + 1] = fmaa(s, re, c * im);
  }
}

template <typename O, typename A, int OPL>
__device__ __forceinline__ void to_out(const A (&x)[OPL], bool ok, O (&y)[OPL]) {
#pragma unroll
  for (int j = 0; j < OPL; ++j) y[j] = ok ? (O)x[j] : (O)__builtin_nan("");
}

// All outputs of point p (0 <= p < a.n_pts) for the orbital chunks of lane `lane` of its group.
template <typename TS, int MODE, int G, int OPL, int VAR>
__device__ __forceinline__ void eval_point(const EvalArgs& a, const int p, const int lane) {
  using A = typename Acc<TS>::type;
  using O = typename Out<TS>::type;
  constexpr bool LAGR = (VAR & VAR_LAGRANGE) != 0;
  constexpr bool BLOCH = (VAR & VAR_BLOCH) != 0;
  constexpr bool PP = (VAR & VAR_PP) != 0;
  constexpr bool PF = Prefetch<A, VAR>::on;
  constexpr bool DERIV = MODE == MODE_VGL || MODE == MODE_VGL_SEPLAP;
  static_assert(!(LAGR && DERIV), "Lagrange tables are read by value only");
  static_assert(!(PP && (LAGR || MODE == MODE_SEP)), "pp-spline tables: B-spline function, no separate gradients");
  static_assert(!BLOCH || OPL % 2 == 0, "Bloch orbitals need whole (re, im) pairs per lane");
  constexpr int NQ = (MODE == MODE_VGL) ? 10 : 4;
  const TS* __restrict__ tab = static_cast<const TS*>(a.table);
  const bool vec_ok = a.vec_store != 0;

  const double r0 = a.pos[3 * (int64_t)p], r1 = a.pos[3 * (int64_t)p + 1], r2 = a.pos[3 * (int64_t)p + 2];
  int i0[3];
  double t[3];
  const bool ok = reduce_point(a.g, r0, r1, r2, i0, t);
  int ix[4], iy[4], iz[4];
  wrap4(i0[0], a.g.n[0], ix);
  wrap4(i0[1], a.g.n[1], iy);
  wrap4(i0[2], a.g.n[2], iz);
  int64_t xo[4], ry[4], rz[4];
  if constexpr (PP) {
    // corners i0 = idx[1] and i0 + 1 = idx[2] per axis; the 8 numbers of a grid point are rows
    // q = 4 (kx - 1) + 2 (ky - 1) + (kz - 1) of o_pad elements each
    const int64_t op = a.g.o_pad;
    xo[0] = (int64_t)ix[1] * a.g.s0;
    xo[1] = xo[0] + 4 * op;
    xo[2] = (int64_t)ix[2] * a.g.s0;
    xo[3] = xo[2] + 4 * op;
    ry[0] = (int64_t)iy[1] * a.g.s1;
    ry[1] = ry[0] + 2 * op;
    ry[2] = (int64_t)iy[2] * a.g.s1;
    ry[3] = ry[2] + 2 * op;
    rz[0] = (int64_t)iz[1] * 8 * op;
    rz[1] = rz[0] + op;
    rz[2] = (int64_t)iz[2] * 8 * op;
    rz[3] = rz[2] + op;
  } else {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      xo[m] = 0;
      ry[m] = (int64_t)iy[m] * a.g.s1;
      rz[m] = (int64_t)iz[m] * a.g.o_pad;
    }
  }

  A ph_c = A(1), ph_s = A(0);   // exp(i k.r), Bloch variants
  if constexpr (BLOCH) {
    double sn, cs;
    sincos(fmaa(a.k[2], r2, fmaa(a.k[1], r1, a.k[0] * r0)), &sn, &cs);
    ph_c = (A)cs;
    ph_s = (A)sn;
  }

  A wx[4], wy[4], wz[4], dwx[4], dwy[4], dwz[4], d2wx[4], d2wy[4], d2wz[4];
  if constexpr (!DERIV) {
    if constexpr (LAGR) {
      lagrange_values<A>((A)t[0], wx);
      lagrange_values<A>((A)t[1], wy);
      lagrange_values<A>((A)t[2], wz);
    } else if constexpr (PP) {
      pp_values<A>((A)t[0], wx);
      pp_values<A>((A)t[1], wy);
      pp_values<A>((A)t[2], wz);
    } else {
      bspline_values<A>((A)t[0], wx);
      bspline_values<A>((A)t[1], wy);
      bspline_values<A>((A)t[2], wz);
    }
  } else if constexpr (PP) {
    pp_weights<A>((A)t[0], wx, dwx, d2wx);
    pp_weights<A>((A)t[1], wy, dwy, d2wy);
    pp_weights<A>((A)t[2], wz, dwz, d2wz);
  } else {
    bspline_weights<A>((A)t[0], wx, dwx, d2wx);
    bspline_weights<A>((A)t[1], wy, dwy, d2wy);
    bspline_weights<A>((A)t[2], wz, dwz, d2wz);
  }

  O* vout = static_cast<O*>(a.v) + (int64_t)p * a.n_orb;
  O* gout = static_cast<O*>(a.grad) + (int64_t)p * 3 * a.n_orb;
  O* lout = static_cast<O*>(a.lap) + (int64_t)p * a.n_orb;
  for (int c = lane; c < a.n_chunks; c += G) {
    const int o = c * OPL;
    if constexpr (MODE == MODE_V) {
      A val[OPL];
      value_pass<TS, OPL, A, PP, PF>(tab + o, ix, xo, ry, rz, a.g.s0, wx, wy, wz, val);
      if constexpr (BLOCH) phase_pairs<A, OPL>(ph_c, ph_s, val);
      O ov[OPL];
      to_out<O, A, OPL>(val, ok, ov);
      store_out<O, OPL>(vout, ov, o, a.n_orb, vec_ok);
    } else if constexpr (MODE == MODE_SEP) {
      // orbital, three Cartesian gradient components and Laplacian, each its own table
      A val[5][OPL];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        value_pass<TS, OPL, A, false, PF>(tab + q * a.tab_stride + o, ix, xo, ry, rz, a.g.s0, wx, wy, wz, val[q]);
        if constexpr (BLOCH) phase_pairs<A, OPL>(ph_c, ph_s, val[q]);
      }
      O y[OPL];
      to_out<O, A, OPL>(val[0], ok, y);
      store_out<O, OPL>(vout, y, o, a.n_orb, vec_ok);
      to_out<O, A, OPL>(val[1], ok, y);
      store_out<O, OPL>(gout, y, o, a.n_orb, vec_ok);
      to_out<O, A, OPL>(val[2], ok, y);
      store_out<O, OPL>(gout + a.n_orb, y, o, a.n_orb, vec_ok);
      to_out<O, A, OPL>(val[3], ok, y);
      store_out<O, OPL>(gout + 2 * a.n_orb, y, o, a.n_orb, vec_ok);
      to_out<O, A, OPL>(val[4], ok, y);
      store_out<O, OPL>(lout, y, o, a.n_orb, vec_ok);
    } else {
      // reduced derivatives: 0 V, 1-3 first, 4 xx, 5 yy, 6 zz, 7 xy, 8 xz, 9 yz
      A acc[NQ][OPL];
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int j = 0; j < OPL; ++j) acc[q][j] = A(0);

      A r[4][4][OPL], nx[4][4][OPL];
      if constexpr (PF) load_slab<TS, OPL, A, PP>(tab + o, 0, ix, xo, ry, rz, a.g.s0, r);
#pragma unroll 1
      for (int l = 0; l < 4; ++l) {
        if constexpr (PF) {
          if (l < 3) load_slab<TS, OPL, A, PP>(tab + o, l + 1, ix, xo, ry, rz, a.g.s0, nx);
        } else {
          load_slab<TS, OPL, A, PP>(tab + o, l, ix, xo, ry, rz, a.g.s0, r);
        }

        const A xw = pick4(l, wx[0], wx[1], wx[2], wx[3]);
        const A xd = pick4(l, dwx[0], dwx[1], dwx[2], dwx[3]);
        const A xdd = pick4(l, d2wx[0], d2wx[1], d2wx[2], d2wx[3]);
#pragma unroll
        for (int j = 0; j < OPL; ++j) {
          // second-axis sums for this l: s0 = sum wy a0, s1 = sum dwy a0, s2 = sum d2wy a0,
          //                              s3 = sum wy a1, s4 = sum dwy a1, s5 = sum wy a2
          A s0 = A(0), s1 = A(0), s2 = A(0), s3 = A(0), s4 = A(0), s5 = A(0);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const A a0 = dot4(wz, r[m][0][j], r[m][1][j], r[m][2][j], r[m][3][j]);
            const A a1 = dot4(dwz, r[m][0][j], r[m][1][j], r[m][2][j], r[m][3][j]);
            s0 = fmaa(wy[m], a0, s0);
            s1 = fmaa(dwy[m], a0, s1);
            s3 = fmaa(wy[m], a1, s3);
            if constexpr (MODE == MODE_VGL) {
              const A a2 = dot4(d2wz, r[m][0][j], r[m][1][j], r[m][2][j], r[m][3][j]);
              s2 = fmaa(d2wy[m], a0, s2);
              s4 = fmaa(dwy[m], a1, s4);
              s5 = fmaa(wy[m], a2, s5);
            }
          }
          acc[0][j] = fmaa(xw, s0, acc[0][j]);
          acc[1][j] = fmaa(xd, s0, acc[1][j]);
          acc[2][j] = fmaa(xw, s1, acc[2][j]);
          acc[3][j] = fmaa(xw, s3, acc[3][j]);
          if constexpr (MODE == MODE_VGL) {
            acc[4][j] = fmaa(xdd, s0, acc[4][j]);
            acc[5][j] = fmaa(xw, s2, acc[5][j]);
            acc[6][j] = fmaa(xw, s5, acc[6][j]);
            acc[7][j] = fmaa(xd, s1, acc[7][j]);
            acc[8][j] = fmaa(xd, s3, acc[8][j]);
            acc[9][j] = fmaa(xw, s4, acc[9][j]);
          }
        }
        if constexpr (PF) copy_slab<A, OPL>(r, nx);
      }

      A lacc[OPL];
      if constexpr (MODE == MODE_VGL_SEPLAP) {
        // Laplacian = value of the separate Laplacian spline (same block, value weights)
        value_pass<TS, OPL, A, PP, PF>(tab + a.tab_stride + o, ix, xo, ry, rz, a.g.s0, wx, wy, wz, lacc);
      }
      // chain rule (Sec. II): grad = J^T grad_t, lap = sum_ij M_ij H_ij
      const A j00 = (A)a.g.jac[0], j01 = (A)a.g.jac[1], j02 = (A)a.g.jac[2];
      const A j10 = (A)a.g.jac[3], j11 = (A)a.g.jac[4], j12 = (A)a.g.jac[5];
      const A j20 = (A)a.g.jac[6], j21 = (A)a.g.jac[7], j22 = (A)a.g.jac[8];
      A av[OPL], ax[OPL], ay[OPL], az[OPL], al[OPL];
#pragma unroll
      for (int j = 0; j < OPL; ++j) {
        const A g0 = acc[1][j], g1 = acc[2][j], g2 = acc[3][j];
        if constexpr (MODE == MODE_VGL) {
          const A diag = fmaa((A)a.g.metric[2], acc[6][j], fmaa((A)a.g.metric[1], acc[5][j], (A)a.g.metric[0] * acc[4][j]));
          const A off = fmaa((A)a.g.metric[5], acc[9][j], fmaa((A)a.g.metric[4], acc[8][j], (A)a.g.metric[3] * acc[7][j]));
          al[j] = fmaa(A(2), off, diag);
        } else {
          al[j] = lacc[j];
        }
        av[j] = acc[0][j];
        ax[j] = fmaa(j20, g2, fmaa(j10, g1, j00 * g0));
        ay[j] = fmaa(j21, g2, fmaa(j11, g1, j01 * g0));
        az[j] = fmaa(j22, g2, fmaa(j12, g1, j02 * g0));
      }
      if constexpr (BLOCH) {
        // product rule for phi = e u (e = exp(i k.r)): grad phi = e (grad u + i k u),
        // lap phi = e (lap u + 2 i k.grad u - |k|^2 u), or e w with a separate Laplacian table
        const A k0 = (A)a.k[0], k1 = (A)a.k[1], k2 = (A)a.k[2];
        const A kk = (A)fmaa(a.k[2], a.k[2], fmaa(a.k[1], a.k[1], a.k[0] * a.k[0]));
#pragma unroll
        for (int j = 0; j < OPL; j += 2) {
          const A ur = av[j], ui = av[j + 1];
          if constexpr (MODE == MODE_VGL) {
            const A kgr = fmaa(k2, az[j], fmaa(k1, ay[j], k0 * ax[j]));
            const A kgi = fmaa(k2, az[j + 1], fmaa(k1, ay[j + 1], k0 * ax[j + 1]));
            al[j] = fmaa(-kk, ur, fmaa(A(-2), kgi, al[j]));
            al[j + 1] = fmaa(-kk, ui, fmaa(A(2), kgr, al[j + 1]));
          }
          ax[j] = fmaa(-k0, ui, ax[j]);
          ax[j + 1] = fmaa(k0, ur, ax[j + 1]);
          ay[j] = fmaa(-k1, ui, ay[j]);
          ay[j + 1] = fmaa(k1, ur, ay[j + 1]);
          az[j] = fmaa(-k2, ui, az[j]);
          az[j + 1] = fmaa(k2, ur, az[j + 1]);
        }
        phase_pairs<A, OPL>(ph_c, ph_s, av);
        phase_pairs<A, OPL>(ph_c, ph_s, ax);
        phase_pairs<A, OPL>(ph_c, ph_s, ay);
        phase_pairs<A, OPL>(ph_c, ph_s, az);
        phase_pairs<A, OPL>(ph_c, ph_s, al);
      }
      O y[OPL];
      to_out<O, A, OPL>(av, ok, y);
      store_out<O, OPL>(vout, y, o, a.n_orb, vec_ok);
      to_out<O, A, OPL>(ax, ok, y);
      store_out<O, OPL>(gout, y, o, a.n_orb, vec_ok);
      to_out<O, A, OPL>(ay, ok, y);
      store_out<O, OPL>(gout + a.n_orb, y, o, a.n_orb, vec_ok);
      to_out<O, A, OPL>(az, ok, y);
      store_out<O, OPL>(gout + 2 * a.n_orb, y, o, a.n_orb, vec_ok);
      to_out<O, A, OPL>(al, ok, y);
      store_out<O, OPL>(lout, y, o, a.n_orb, vec_ok);
    }
  }
}

// One launch over one table: groups of G lanes, one point per group.  With a permutation (sorted
// evaluation) the points are taken in its order, and workgroups, which the hardware hands to the 8
// XCDs in turn, are remapped so that each XCD walks a contiguous stretch of that order.
template <typename TS, int MODE, int G, int OPL, int VAR>
__global__ __launch_bounds__(256) void k_eval(EvalArgs a) {
  constexpr int GPB = 256 / G;
  const int b = (int)blockIdx.x;
  const int64_t tile = a.perm ? (int64_t)(b & 7) * a.per_xcd + (b >> 3) : (int64_t)b;
  const int64_t q = tile * GPB + (int)threadIdx.x / G;
  if (q >= a.n_pts) return;
  int p = a.perm ? a.perm[q] : (int)q;
  if constexpr (G >= 64) p = __builtin_amdgcn_readfirstlane(p);
  eval_point<TS, MODE, G, OPL, VAR>(a, p, (int)threadIdx.x % G);
}

// ---------------------------------------------------------------- batched persistent launch
// Many tables and point sets in one launch.  The work list is implicit: item j owns tiles
// [tile_start[j], tile_start[j+1]), a tile being the 256 / G points one workgroup covers in one
// pass.  Workgroups take tiles from a device counter until it passes n_tiles, so the launch is
// load-balanced however uneven the items are; every workgroup leaves the loop once the counter
// is exhausted.  Items are ordered by decreasing cost per tile on the host (largest first).  With a
// permutation per item (sorted plans) each item's points are taken in locality order.
struct BatchArgs {
  const EvalArgs* items;      // device array [n_items]
  const int32_t* tile_start;  // device array [n_items + 1], exclusive prefix of tiles per item
  int32_t* counter;           // device int, zeroed by k_batch_reset before each launch
  int32_t n_items;
  int32_t n_tiles;
};

// One tile of a batched launch: 256 / G points of item `a`, G lanes per point; rel is the tile's
// index within the item.
template <typename TS, int MODE, int G, int OPL>
__device__ __forceinline__ void batch_tile(const EvalArgs& a, int rel) {
  int p = rel * (256 / G) + (int)threadIdx.x / G;
  if (p < a.n_pts) {
    if (a.perm) p = a.perm[p];                         // the item's points in locality order
    if constexpr (G >= 64) p = __builtin_amdgcn_readfirstlane(p);
    eval_point<TS, MODE, G, OPL, 0>(a, p, (int)threadIdx.x % G);
  }
}

// The next tile of a persistent launch and its item (the last item whose first tile <= tile), or
// tile >= n_tiles when the work is done.  Uniform over the workgroup.
__device__ __forceinline__ int batch_next(const BatchArgs& b, int32_t* s_tile, int* item) {
  if (threadIdx.x == 0) *s_tile = atomicAdd(b.counter, 1);
  __syncthreads();
  const int tile = __builtin_amdgcn_readfirstlane(*s_tile);
  __syncthreads();                                   // s_tile is rewritten next iteration
  int lo = 0, hi = b.n_items - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.tile_start[mid] <= tile) lo = mid;
    else hi = mid - 1;
  }
  *item = lo;
  return tile;
}

template <typename TS, int MODE, int G, int OPL>
__global__ __launch_bounds__(256) void k_eval_batch(BatchArgs b) {
  __shared__ int32_t s_tile;
  for (;;) {
    int lo;
    const int tile = batch_next(b, &s_tile, &lo);
    if (tile >= b.n_tiles) break;                      // uniform: the whole workgroup leaves
    batch_tile<TS, MODE, G, OPL>(b.items[lo], tile - b.tile_start[lo]);
  }
}

// The same persistent launch with every item's own lanes per point (EvalArgs::lanes) and a common
// OPL: items with few orbitals take short lane groups and more points per tile.  Every shape runs
// the same per-point arithmetic, so each item's outputs equal the single-system kernel's at its
// shape, bit for bit.
template <typename TS, int MODE, int OPL>
__global__ __launch_bounds__(256) void k_eval_batch_multi(BatchArgs b) {
  __shared__ int32_t s_tile;
  for (;;) {
    int lo;
    const int tile = batch_next(b, &s_tile, &lo);
    if (tile >= b.n_tiles) break;
    const EvalArgs& a = b.items[lo];
    const int rel = tile - b.tile_start[lo];
    switch (__builtin_amdgcn_readfirstlane(a.lanes)) {
      case 8: batch_tile<TS, MODE, 8, OPL>(a, rel); break;
      case 16: batch_tile<TS, MODE, 16, OPL>(a, rel); break;
      case 32: batch_tile<TS, MODE, 32, OPL>(a, rel); break;
      case 64: batch_tile<TS, MODE, 64, OPL>(a, rel); break;
      case 128: batch_tile<TS, MODE, 128, OPL>(a, rel); break;
      case 256: batch_tile<TS, MODE, 256, OPL>(a, rel); break;
      default: break;                                  // not reachable: the plan validates every shape
    }
  }
}

typedef void (*EvalKernel)(EvalArgs);
typedef void (*BatchKernel)(BatchArgs);

// g = 0: per-item lanes per point (k_eval_batch_multi)
template <typename TS, int MODE, int OPL>
inline BatchKernel pick_batch_g(int g) {
  switch (g) {
    case 0: return k_eval_batch_multi<TS, MODE, OPL>;
    case 8: return k_eval_batch<TS, MODE, 8, OPL>;
    case 16: return k_eval_batch<TS, MODE, 16, OPL>;
    case 32: return k_eval_batch<TS, MODE, 32, OPL>;
    case 64: return k_eval_batch<TS, MODE, 64, OPL>;
    case 128: return k_eval_batch<TS, MODE, 128, OPL>;
    case 256: return k_eval_batch<TS, MODE, 256, OPL>;
    default: return nullptr;
  }
}

template <typename TS, int MODE, int OPL, int VAR>
inline EvalKernel pick_g(int g) {
  if constexpr ((VAR & VAR_BLOCH) != 0 && OPL % 2 != 0) {
    (void)g;
    return nullptr;                        // Bloch pairs need an even number of columns per lane
  } else {
    switch (g) {
      case 2: return k_eval<TS, MODE, 2, OPL, VAR>;
      case 4: return k_eval<TS, MODE, 4, OPL, VAR>;
      case 8: return k_eval<TS, MODE, 8, OPL, VAR>;
      case 16: return k_eval<TS, MODE, 16, OPL, VAR>;
      case 32: return k_eval<TS, MODE, 32, OPL, VAR>;
      case 64: return k_eval<TS, MODE, 64, OPL, VAR>;
      case 128: return k_eval<TS, MODE, 128, OPL, VAR>;
      case 256: return k_eval<TS, MODE, 256, OPL, VAR>;
      default: return nullptr;
    }
  }
}

// orbitals per lane offered per storage dtype: loads of 8 or 16 bytes (FP64), 4-16 (FP32),
// 4-16 (BF16); the default is the middle entry
template <typename TS> struct OplSet;
template <> struct OplSet<double> { static constexpr int lo = 1, mid = 2, hi = 2; };
template <> struct OplSet<float> { static constexpr int lo = 1, mid = 2, hi = 4; };
template <> struct OplSet<uint16_t> { static constexpr int lo = 2, mid = 4, hi = 8; };

template <typename TS, int MODE, int VAR>
inline EvalKernel pick_opl(int g, int opl) {
  if (opl == OplSet<TS>::lo) return pick_g<TS, MODE, OplSet<TS>::lo, VAR>(g);
  if (opl == OplSet<TS>::mid) return pick_g<TS, MODE, OplSet<TS>::mid, VAR>(g);
  if (opl == OplSet<TS>::hi) return pick_g<TS, MODE, OplSet<TS>::hi, VAR>(g);
  return nullptr;
}

template <typename TS, int MODE>
inline BatchKernel pick_batch_opl(int g, int opl);

// Real B-spline tables, values or VGL from derivatives (with or without a separate Laplacian).
template <typename TS>
inline EvalKernel pick_mode(int mode, int g, int opl) {
  switch (mode) {
    case MODE_V: return pick_opl<TS, MODE_V, 0>(g, opl);
    case MODE_VGL: return pick_opl<TS, MODE_VGL, 0>(g, opl);
    case MODE_VGL_SEPLAP: return pick_opl<TS, MODE_VGL_SEPLAP, 0>(g, opl);
    default: return nullptr;
  }
}

// Everything else: Lagrange weights, five separate tables, Bloch orbitals, pp-spline layout, and the
// FP64 instances without prefetch (real and Bloch B-spline tables, for the sorted call).
template <typename TS>
inline EvalKernel pick_mode_variant(int mode, int var, int g, int opl) {
  if (var & VAR_NOPF) {
    if constexpr (sizeof(TS) == 8) {
      const int v = var & ~VAR_NOPF;
      if (v == 0) {
        if (mode == MODE_V) return pick_opl<TS, MODE_V, VAR_NOPF>(g, opl);
        if (mode == MODE_VGL) return pick_opl<TS, MODE_VGL, VAR_NOPF>(g, opl);
        if (mode == MODE_VGL_SEPLAP) return pick_opl<TS, MODE_VGL_SEPLAP, VAR_NOPF>(g, opl);
      } else if (v == VAR_BLOCH) {
        if (mode == MODE_V) return pick_opl<TS, MODE_V, VAR_NOPF | VAR_BLOCH>(g, opl);
        if (mode == MODE_VGL) return pick_opl<TS, MODE_VGL, VAR_NOPF | VAR_BLOCH>(g, opl);
        if (mode == MODE_VGL_SEPLAP) return pick_opl<TS, MODE_VGL_SEPLAP, VAR_NOPF | VAR_BLOCH>(g, opl);
      }
    }
    return nullptr;
  }
  if (mode == MODE_SEP) {
    switch (var) {
      case 0: return pick_opl<TS, MODE_SEP, 0>(g, opl);
      case VAR_LAGRANGE: return pick_opl<TS, MODE_SEP, VAR_LAGRANGE>(g, opl);
      case VAR_BLOCH: return pick_opl<TS, MODE_SEP, VAR_BLOCH>(g, opl);
      case VAR_BLOCH | VAR_LAGRANGE: return pick_opl<TS, MODE_SEP, VAR_BLOCH | VAR_LAGRANGE>(g, opl);
      default: return nullptr;
    }
  }
  if (mode == MODE_V) {
    switch (var) {
      case VAR_LAGRANGE: return pick_opl<TS, MODE_V, VAR_LAGRANGE>(g, opl);
      case VAR_BLOCH: return pick_opl<TS, MODE_V, VAR_BLOCH>(g, opl);
      case VAR_BLOCH | VAR_LAGRANGE: return pick_opl<TS, MODE_V, VAR_BLOCH | VAR_LAGRANGE>(g, opl);
      case VAR_PP: return pick_opl<TS, MODE_V, VAR_PP>(g, opl);
      case VAR_PP | VAR_BLOCH: return pick_opl<TS, MODE_V, VAR_PP | VAR_BLOCH>(g, opl);
      default: return nullptr;
    }
  }
  const bool lap = mode == MODE_VGL_SEPLAP;
  switch (var) {
    case VAR_BLOCH:
      return lap ? pick_opl<TS, MODE_VGL_SEPLAP, VAR_BLOCH>(g, opl) : pick_opl<TS, MODE_VGL, VAR_BLOCH>(g, opl);
    case VAR_PP:
      return lap ? pick_opl<TS, MODE_VGL_SEPLAP, VAR_PP>(g, opl) : pick_opl<TS, MODE_VGL, VAR_PP>(g, opl);
    case VAR_PP | VAR_BLOCH:
      return lap ? pick_opl<TS, MODE_VGL_SEPLAP, VAR_PP | VAR_BLOCH>(g, opl)
                 : pick_opl<TS, MODE_VGL, VAR_PP | VAR_BLOCH>(g, opl);
    default: return nullptr;
  }
}

template <typename TS, int MODE>
inline BatchKernel pick_batch_opl(int g, int opl) {
  if (opl == OplSet<TS>::lo) return pick_batch_g<TS, MODE, OplSet<TS>::lo>(g);
  if (opl == OplSet<TS>::mid) return pick_batch_g<TS, MODE, OplSet<TS>::mid>(g);
  if (opl == OplSet<TS>::hi) return pick_batch_g<TS, MODE, OplSet<TS>::hi>(g);
  return nullptr;
}

template <typename TS>
inline BatchKernel pick_batch_mode(int mode, int g, int opl) {
  return mode == MODE_VGL ? pick_batch_opl<TS, MODE_VGL>(g, opl) : pick_batch_opl<TS, MODE_VGL_SEPLAP>(g, opl);
}

}  // namespace pws
