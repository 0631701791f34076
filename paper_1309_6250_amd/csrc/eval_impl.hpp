// Forward evaluation kernels: orbital values, gradients and Laplacians through the periodic
// tricubic B-spline (App. A, Eq. b-splineapproximation; chain rule of Sec. II).
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
// issues the 16 row loads of one slab (l fixed) before using them, so each wave keeps 16
// vector loads in flight with a register budget that leaves room for several waves per SIMD.
// No matrix cores: the work is a gather followed by a short dot product, bound by memory.
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
  int32_t n_orb;
  int32_t n_chunks;   // ceil(n_orb / OPL): chunks holding at least one real orbital
  int32_t vec_store;  // n_orb % OPL == 0 and outputs 16-byte aligned: whole-vector stores
  int64_t lap_off;    // element offset of the separate Laplacian table
};

enum { MODE_V = 0, MODE_VGL = 1, MODE_VGL_SEPLAP = 2 };

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

// All outputs of point p (0 <= p < a.n_pts) for the orbital chunks of lane `lane` of its group.
template <typename TS, int MODE, int G, int OPL>
__device__ __forceinline__ void eval_point(const EvalArgs& a, const int p, const int lane) {
  using A = typename Acc<TS>::type;
  using O = typename Out<TS>::type;
  constexpr int NQ = (MODE == MODE_V) ? 1 : (MODE == MODE_VGL ? 10 : 4);
  const TS* __restrict__ tab = static_cast<const TS*>(a.table);
  const bool vec_ok = a.vec_store != 0;

  int i0[3];
  double t[3];
  const bool ok = reduce_point(a.g, a.pos[3 * (int64_t)p], a.pos[3 * (int64_t)p + 1], a.pos[3 * (int64_t)p + 2],
                               i0, t);
  int ix[4], iy[4], iz[4];
  wrap4(i0[0], a.g.n[0], ix);
  wrap4(i0[1], a.g.n[1], iy);
  wrap4(i0[2], a.g.n[2], iz);
  int64_t ry[4], rz[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    ry[m] = (int64_t)iy[m] * a.g.s1;
    rz[m] = (int64_t)iz[m] * a.g.o_pad;
  }

  A wx[4], wy[4], wz[4], dwx[4], dwy[4], dwz[4], d2wx[4], d2wy[4], d2wz[4];
  if constexpr (MODE == MODE_V) {
    bspline_values<A>((A)t[0], wx);
    bspline_values<A>((A)t[1], wy);
    bspline_values<A>((A)t[2], wz);
  } else {
    bspline_weights<A>((A)t[0], wx, dwx, d2wx);
    bspline_weights<A>((A)t[1], wy, dwy, d2wy);
    bspline_weights<A>((A)t[2], wz, dwz, d2wz);
  }

  O* vout = static_cast<O*>(a.v) + (int64_t)p * a.n_orb;
  for (int c = lane; c < a.n_chunks; c += G) {
    const int o = c * OPL;
    // reduced derivatives: 0 V, 1-3 first, 4 xx, 5 yy, 6 zz, 7 xy, 8 xz, 9 yz
    A acc[NQ][OPL];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int j = 0; j < OPL; ++j) acc[q][j] = A(0);

#pragma unroll 1
    for (int l = 0; l < 4; ++l) {
      const TS* slab = tab + (int64_t)pick4(l, ix[0], ix[1], ix[2], ix[3]) * a.g.s0 + o;
      A r[4][4][OPL];
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) RowN<TS, OPL>::load(slab + ry[m] + rz[n], r[m][n]);

      const A xw = pick4(l, wx[0], wx[1], wx[2], wx[3]);
      if constexpr (MODE == MODE_V) {
#pragma unroll
        for (int j = 0; j < OPL; ++j) {
          A q = A(0);
#pragma unroll
          for (int m = 0; m < 4; ++m) q = fmaa(wy[m], dot4(wz, r[m][0][j], r[m][1][j], r[m][2][j], r[m][3][j]), q);
          acc[0][j] = fmaa(xw, q, acc[0][j]);
        }
      } else {
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
      }
    }

    if constexpr (MODE == MODE_V) {
      O ov[OPL];
#pragma unroll
      for (int j = 0; j < OPL; ++j) ov[j] = ok ? (O)acc[0][j] : (O)__builtin_nan("");
      store_out<O, OPL>(vout, ov, o, a.n_orb, vec_ok);
    } else {
      A lacc[OPL];
#pragma unroll
      for (int j = 0; j < OPL; ++j) lacc[j] = A(0);
      if constexpr (MODE == MODE_VGL_SEPLAP) {
        // Laplacian = value of the separate Laplacian spline (same block, value weights)
#pragma unroll 1
        for (int l = 0; l < 4; ++l) {
          const TS* slab = tab + a.lap_off + (int64_t)pick4(l, ix[0], ix[1], ix[2], ix[3]) * a.g.s0 + o;
          A r[4][4][OPL];
#pragma unroll
          for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) RowN<TS, OPL>::load(slab + ry[m] + rz[n], r[m][n]);
          const A xw = pick4(l, wx[0], wx[1], wx[2], wx[3]);
#pragma unroll
          for (int j = 0; j < OPL; ++j) {
            A q = A(0);
#pragma unroll
            for (int m = 0; m < 4; ++m) q = fmaa(wy[m], dot4(wz, r[m][0][j], r[m][1][j], r[m][2][j], r[m][3][j]), q);
            lacc[j] = fmaa(xw, q, lacc[j]);
          }
        }
      }
      // chain rule (Sec. II): grad = J^T grad_t, lap = sum_ij M_ij H_ij
      const A j00 = (A)a.g.jac[0], j01 = (A)a.g.jac[1], j02 = (A)a.g.jac[2];
      const A j10 = (A)a.g.jac[3], j11 = (A)a.g.jac[4], j12 = (A)a.g.jac[5];
      const A j20 = (A)a.g.jac[6], j21 = (A)a.g.jac[7], j22 = (A)a.g.jac[8];
      O ov[OPL], gx[OPL], gy[OPL], gz[OPL], lv[OPL];
      const O nan = (O)__builtin_nan("");
#pragma unroll
      for (int j = 0; j < OPL; ++j) {
        const A g0 = acc[1][j], g1 = acc[2][j], g2 = acc[3][j];
        A lp;
        if constexpr (MODE == MODE_VGL) {
          const A diag = fmaa((A)a.g.metric[2], acc[6][j], fmaa((A)a.g.metric[1], acc[5][j], (A)a.g.metric[0] * acc[4][j]));
          const A off = fmaa((A)a.g.metric[5], acc[9][j], fmaa((A)a.g.metric[4], acc[8][j], (A)a.g.metric[3] * acc[7][j]));
          lp = fmaa(A(2), off, diag);
        } else {
          lp = lacc[j];
        }
        ov[j] = ok ? (O)acc[0][j] : nan;
        gx[j] = ok ? (O)fmaa(j20, g2, fmaa(j10, g1, j00 * g0)) : nan;
        gy[j] = ok ? (O)fmaa(j21, g2, fmaa(j11, g1, j01 * g0)) : nan;
        gz[j] = ok ? (O)fmaa(j22, g2, fmaa(j12, g1, j02 * g0)) : nan;
        lv[j] = ok ? (O)lp : nan;
      }
      O* gout = static_cast<O*>(a.grad) + (int64_t)p * 3 * a.n_orb;
      O* lout = static_cast<O*>(a.lap) + (int64_t)p * a.n_orb;
      store_out<O, OPL>(vout, ov, o, a.n_orb, vec_ok);
      store_out<O, OPL>(gout, gx, o, a.n_orb, vec_ok);
      store_out<O, OPL>(gout + a.n_orb, gy, o, a.n_orb, vec_ok);
      store_out<O, OPL>(gout + 2 * a.n_orb, gz, o, a.n_orb, vec_ok);
      store_out<O, OPL>(lout, lv, o, a.n_orb, vec_ok);
    }
  }
}

// One launch over one table: groups of G lanes, one point per group.
template <typename TS, int MODE, int G, int OPL>
__global__ __launch_bounds__(256) void k_eval(EvalArgs a) {
  constexpr int GPB = 256 / G;
  int p = (int)blockIdx.x * GPB + (int)threadIdx.x / G;
  if constexpr (G >= 64) p = __builtin_amdgcn_readfirstlane(p);
  if (p >= a.n_pts) return;
  eval_point<TS, MODE, G, OPL>(a, p, (int)threadIdx.x % G);
}

// ---------------------------------------------------------------- batched persistent launch
// Many tables and point sets in one launch.  The work list is implicit: item j owns tiles
// [tile_start[j], tile_start[j+1]), a tile being the 256 / G points one workgroup covers in one
// pass.  Workgroups take tiles from a device counter until it passes n_tiles, so the launch is
// load-balanced however uneven the items are; every workgroup leaves the loop once the counter
// is exhausted.  Items are ordered by decreasing cost per tile on the host (largest first).
struct BatchArgs {
  const EvalArgs* items;      // device array [n_items]
  const int32_t* tile_start;  // device array [n_items + 1], exclusive prefix of tiles per item
  int32_t* counter;           // device int, zeroed by k_batch_reset before each launch
  int32_t n_items;
  int32_t n_tiles;
};

template <typename TS, int MODE, int G, int OPL>
__global__ __launch_bounds__(256) void k_eval_batch(BatchArgs b) {
  constexpr int GPB = 256 / G;
  __shared__ int32_t s_tile;
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(b.counter, 1);
    __syncthreads();
    const int tile = __builtin_amdgcn_readfirstlane(s_tile);
    __syncthreads();                                   // s_tile is rewritten next iteration
    if (tile >= b.n_tiles) break;                      // uniform: the whole workgroup leaves
    int lo = 0, hi = b.n_items - 1;                    // last item whose first tile <= tile
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (b.tile_start[mid] <= tile) lo = mid;
      else hi = mid - 1;
    }
    const EvalArgs& a = b.items[lo];
    int p = (tile - b.tile_start[lo]) * GPB + (int)threadIdx.x / G;
    if constexpr (G >= 64) p = __builtin_amdgcn_readfirstlane(p);
    if (p < a.n_pts) eval_point<TS, MODE, G, OPL>(a, p, (int)threadIdx.x % G);
  }
}

typedef void (*EvalKernel)(EvalArgs);
typedef void (*BatchKernel)(BatchArgs);

template <typename TS, int MODE, int OPL>
inline BatchKernel pick_batch_g(int g) {
  switch (g) {
    case 8: return k_eval_batch<TS, MODE, 8, OPL>;
    case 16: return k_eval_batch<TS, MODE, 16, OPL>;
    case 32: return k_eval_batch<TS, MODE, 32, OPL>;
    case 64: return k_eval_batch<TS, MODE, 64, OPL>;
    case 128: return k_eval_batch<TS, MODE, 128, OPL>;
    case 256: return k_eval_batch<TS, MODE, 256, OPL>;
    default: return nullptr;
  }
}

template <typename TS, int MODE, int OPL>
inline EvalKernel pick_g(int g) {
  switch (g) {
    case 2: return k_eval<TS, MODE, 2, OPL>;
    case 4: return k_eval<TS, MODE, 4, OPL>;
    case 8: return k_eval<TS, MODE, 8, OPL>;
    case 16: return k_eval<TS, MODE, 16, OPL>;
    case 32: return k_eval<TS, MODE, 32, OPL>;
    case 64: return k_eval<TS, MODE, 64, OPL>;
    case 128: return k_eval<TS, MODE, 128, OPL>;
    case 256: return k_eval<TS, MODE, 256, OPL>;
    default: return nullptr;
  }
}

// orbitals per lane offered per storage dtype: loads of 8 or 16 bytes (FP64), 4-16 (FP32),
// 4-16 (BF16); the default is the middle entry
template <typename TS> struct OplSet;
template <> struct OplSet<double> { static constexpr int lo = 1, mid = 2, hi = 2; };
template <> struct OplSet<float> { static constexpr int lo = 1, mid = 2, hi = 4; };
template <> struct OplSet<uint16_t> { static constexpr int lo = 2, mid = 4, hi = 8; };

template <typename TS, int MODE>
inline EvalKernel pick_opl(int g, int opl) {
  if (opl == OplSet<TS>::lo) return pick_g<TS, MODE, OplSet<TS>::lo>(g);
  if (opl == OplSet<TS>::mid) return pick_g<TS, MODE, OplSet<TS>::mid>(g);
  if (opl == OplSet<TS>::hi) return pick_g<TS, MODE, OplSet<TS>::hi>(g);
  return nullptr;
}

template <typename TS, int MODE>
inline BatchKernel pick_batch_opl(int g, int opl);

template <typename TS>
inline EvalKernel pick_mode(int mode, int g, int opl) {
  switch (mode) {
    case MODE_V: return pick_opl<TS, MODE_V>(g, opl);
    case MODE_VGL: return pick_opl<TS, MODE_VGL>(g, opl);
    default: return pick_opl<TS, MODE_VGL_SEPLAP>(g, opl);
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
