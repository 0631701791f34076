// Forward evaluation: orbital values, gradients and Laplacians through the periodic
// tricubic B-spline (App. A, Eq. b-splineapproximation; chain rule of Sec. II).
//
// Mapping.  A group of G lanes (G a power of two, 1..256) owns one point; lane c of the
// group owns the orbital chunks c, c+G, c+2G, ... where a chunk is the 16 bytes of
// stored coefficients one vector load brings in (2 FP64, 4 FP32 or 8 BF16 orbitals).
// Because the orbital index is innermost in the table, the G lanes of a group read
// contiguous bytes of each of the 64 rows of the point's 4x4x4 block: every load is
// coalesced.  The reduced coordinate and the 36 one-dimensional weights of a point are
// computed once per group and held in registers (wave-uniform when G >= 64).
//
// Contraction.  Separable, the innermost grid axis first: for each of the 16 (l, m) row
// pairs, the 4 coefficients along the third axis are reduced with (b, b', b'') of t_3;
// those three partial sums are folded with the second axis' weights into six sums per
// l, and those with the first axis' weights into the ten reduced derivatives
// (value, 3 first, 6 second).  About 340 FMA per orbital instead of 640.  The chain
// rule then gives the Cartesian gradient and Laplacian.  No matrix cores: the work is a
// gather followed by a short dot product, bound by memory bandwidth.
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
  int32_t n_chunks;   // o_pad / VEC
  int32_t vec_store;  // n_orb % VEC == 0: outputs can be written as whole vectors
  int64_t lap_off;    // element offset of the separate Laplacian table
};

enum { MODE_V = 0, MODE_VGL = 1, MODE_VGL_SEPLAP = 2 };

template <typename O, int VEC>
__device__ __forceinline__ void store_vec(O* dst, const O (&x)[VEC], int o, int n_orb, bool vec_ok) {
  if (vec_ok) {
    if constexpr (sizeof(O) * VEC == 16 && sizeof(O) == 8) {
      __builtin_nontemporal_store(d2v{x[0], x[1]}, reinterpret_cast<d2v*>(dst + o));
      return;
    } else if constexpr (sizeof(O) == 4 && VEC == 4) {
      __builtin_nontemporal_store(f4v{x[0], x[1], x[2], x[3]}, reinterpret_cast<f4v*>(dst + o));
      return;
    } else if constexpr (sizeof(O) == 4 && VEC == 8) {
      __builtin_nontemporal_store(f4v{x[0], x[1], x[2], x[3]}, reinterpret_cast<f4v*>(dst + o));
      __builtin_nontemporal_store(f4v{x[4], x[5], x[6], x[7]}, reinterpret_cast<f4v*>(dst + o + 4));
      return;
    }
  }
#pragma unroll
  for (int j = 0; j < VEC; ++j)
    if (o + j < n_orb) __builtin_nontemporal_store(x[j], dst + o + j);
}

template <typename TS, int MODE, int G, int PPL>
__global__ __launch_bounds__(256) void k_eval(EvalArgs a) {
  using A = typename Acc<TS>::type;
  using O = typename Out<TS>::type;
  constexpr int VEC = Row16<TS>::VEC;
  constexpr int GPB = 256 / G;
  const int grp = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  const TS* __restrict__ tab = static_cast<const TS*>(a.table);
  const bool vec_ok = a.vec_store != 0;

#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    int p = ((int)blockIdx.x * PPL + k) * GPB + grp;
    if constexpr (G >= 64) p = __builtin_amdgcn_readfirstlane(p);
    if (p >= a.n_pts) return;

    int i0[3];
    double t[3];
    const bool ok = reduce_point(a.g, a.pos[3 * (int64_t)p], a.pos[3 * (int64_t)p + 1],
                                 a.pos[3 * (int64_t)p + 2], i0, t);
    int ix[4], iy[4], iz[4];
    wrap4(i0[0], a.g.n[0], ix);
    wrap4(i0[1], a.g.n[1], iy);
    wrap4(i0[2], a.g.n[2], iz);
    int64_t rx[4], ry[4], rz[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      rx[l] = (int64_t)ix[l] * a.g.s0;
      ry[l] = (int64_t)iy[l] * a.g.s1;
      rz[l] = (int64_t)iz[l] * a.g.o_pad;
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
      const int o = c * VEC;
      if constexpr (MODE == MODE_V) {
        A val[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) val[j] = A(0);
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          A q[VEC];
#pragma unroll
          for (int j = 0; j < VEC; ++j) q[j] = A(0);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const TS* rp = tab + rx[l] + ry[m] + o;
            A r[4][VEC];
#pragma unroll
            for (int n = 0; n < 4; ++n) Row16<TS>::load(rp + rz[n], r[n]);
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
              const A a0 = wz[0] * r[0][j] + wz[1] * r[1][j] + wz[2] * r[2][j] + wz[3] * r[3][j];
              q[j] += wy[m] * a0;
            }
          }
#pragma unroll
          for (int j = 0; j < VEC; ++j) val[j] += wx[l] * q[j];
        }
        O ov[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) ov[j] = ok ? (O)val[j] : (O)__builtin_nan("");
        store_vec<O, VEC>(vout, ov, o, a.n_orb, vec_ok);
      } else {
        // reduced derivatives: 0 V, 1-3 first, 4 xx, 5 yy, 6 zz, 7 xy, 8 xz, 9 yz
        constexpr int NQ = (MODE == MODE_VGL) ? 10 : 4;
        A acc[NQ][VEC];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int j = 0; j < VEC; ++j) acc[q][j] = A(0);
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          // y-stage sums for this l: s0 = sum wy a0, s1 = sum dwy a0, s2 = sum d2wy a0,
          //                          s3 = sum wy a1, s4 = sum dwy a1, s5 = sum wy a2
          A s[6][VEC];
#pragma unroll
          for (int q = 0; q < 6; ++q)
#pragma unroll
            for (int j = 0; j < VEC; ++j) s[q][j] = A(0);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const TS* rp = tab + rx[l] + ry[m] + o;
            A r[4][VEC];
#pragma unroll
            for (int n = 0; n < 4; ++n) Row16<TS>::load(rp + rz[n], r[n]);
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
              const A a0 = wz[0] * r[0][j] + wz[1] * r[1][j] + wz[2] * r[2][j] + wz[3] * r[3][j];
              const A a1 = dwz[0] * r[0][j] + dwz[1] * r[1][j] + dwz[2] * r[2][j] + dwz[3] * r[3][j];
              s[0][j] += wy[m] * a0;
              s[1][j] += dwy[m] * a0;
              s[3][j] += wy[m] * a1;
              if constexpr (MODE == MODE_VGL) {
                const A a2 = d2wz[0] * r[0][j] + d2wz[1] * r[1][j] + d2wz[2] * r[2][j] + d2wz[3] * r[3][j];
                s[2][j] += d2wy[m] * a0;
                s[4][j] += dwy[m] * a1;
                s[5][j] += wy[m] * a2;
              }
            }
          }
#pragma unroll
          for (int j = 0; j < VEC; ++j) {
            acc[0][j] += wx[l] * s[0][j];
            acc[1][j] += dwx[l] * s[0][j];
            acc[2][j] += wx[l] * s[1][j];
            acc[3][j] += wx[l] * s[3][j];
            if constexpr (MODE == MODE_VGL) {
              acc[4][j] += d2wx[l] * s[0][j];
              acc[5][j] += wx[l] * s[2][j];
              acc[6][j] += wx[l] * s[5][j];
              acc[7][j] += dwx[l] * s[1][j];
              acc[8][j] += dwx[l] * s[3][j];
              acc[9][j] += wx[l] * s[4][j];
            }
          }
        }
        A lacc[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) lacc[j] = A(0);
        if constexpr (MODE == MODE_VGL_SEPLAP) {
          // Laplacian = value of the separate Laplacian spline (same block, value weights)
          const TS* ltab = tab + a.lap_off;
#pragma unroll
          for (int l = 0; l < 4; ++l) {
            A q[VEC];
#pragma unroll
            for (int j = 0; j < VEC; ++j) q[j] = A(0);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const TS* rp = ltab + rx[l] + ry[m] + o;
              A r[4][VEC];
#pragma unroll
              for (int n = 0; n < 4; ++n) Row16<TS>::load(rp + rz[n], r[n]);
#pragma unroll
              for (int j = 0; j < VEC; ++j)
                q[j] += wy[m] * (wz[0] * r[0][j] + wz[1] * r[1][j] + wz[2] * r[2][j] + wz[3] * r[3][j]);
            }
#pragma unroll
            for (int j = 0; j < VEC; ++j) lacc[j] += wx[l] * q[j];
          }
        }
        // chain rule (Sec. II): grad = J^T grad_t, lap = sum_ij M_ij H_ij
        const A j00 = (A)a.g.jac[0], j01 = (A)a.g.jac[1], j02 = (A)a.g.jac[2];
        const A j10 = (A)a.g.jac[3], j11 = (A)a.g.jac[4], j12 = (A)a.g.jac[5];
        const A j20 = (A)a.g.jac[6], j21 = (A)a.g.jac[7], j22 = (A)a.g.jac[8];
        O ov[VEC], gx[VEC], gy[VEC], gz[VEC], lv[VEC];
        const O nan = (O)__builtin_nan("");
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
          const A g0 = acc[1][j], g1 = acc[2][j], g2 = acc[3][j];
          A lp;
          if constexpr (MODE == MODE_VGL) {
            lp = (A)a.g.metric[0] * acc[4][j] + (A)a.g.metric[1] * acc[5][j] + (A)a.g.metric[2] * acc[6][j] +
                 A(2) * ((A)a.g.metric[3] * acc[7][j] + (A)a.g.metric[4] * acc[8][j] +
                         (A)a.g.metric[5] * acc[9][j]);
          } else {
            lp = lacc[j];
          }
          ov[j] = ok ? (O)acc[0][j] : nan;
          gx[j] = ok ? (O)(j00 * g0 + j10 * g1 + j20 * g2) : nan;
          gy[j] = ok ? (O)(j01 * g0 + j11 * g1 + j21 * g2) : nan;
          gz[j] = ok ? (O)(j02 * g0 + j12 * g1 + j22 * g2) : nan;
          lv[j] = ok ? (O)lp : nan;
        }
        O* gout = static_cast<O*>(a.grad) + (int64_t)p * 3 * a.n_orb;
        O* lout = static_cast<O*>(a.lap) + (int64_t)p * a.n_orb;
        store_vec<O, VEC>(vout, ov, o, a.n_orb, vec_ok);
        store_vec<O, VEC>(gout, gx, o, a.n_orb, vec_ok);
        store_vec<O, VEC>(gout + a.n_orb, gy, o, a.n_orb, vec_ok);
        store_vec<O, VEC>(gout + 2 * a.n_orb, gz, o, a.n_orb, vec_ok);
        store_vec<O, VEC>(lout, lv, o, a.n_orb, vec_ok);
      }
    }
  }
}

}  // namespace pws


namespace pws {

typedef void (*EvalKernel)(EvalArgs);

template <typename TS, int MODE, int PPL>
inline EvalKernel pick_g(int g) {
  switch (g) {
    case 1: return k_eval<TS, MODE, 1, PPL>;
    case 2: return k_eval<TS, MODE, 2, PPL>;
    case 4: return k_eval<TS, MODE, 4, PPL>;
    case 8: return k_eval<TS, MODE, 8, PPL>;
    case 16: return k_eval<TS, MODE, 16, PPL>;
    case 32: return k_eval<TS, MODE, 32, PPL>;
    case 64: return k_eval<TS, MODE, 64, PPL>;
    case 128: return k_eval<TS, MODE, 128, PPL>;
    case 256: return k_eval<TS, MODE, 256, PPL>;
    default: return nullptr;
  }
}

template <typename TS, int MODE>
inline EvalKernel pick(int g, int ppl) {
  switch (ppl) {
    case 1: return pick_g<TS, MODE, 1>(g);
    case 2: return pick_g<TS, MODE, 2>(g);
    default: return nullptr;
  }
}

template <typename TS>
inline EvalKernel pick_mode(int mode, int g, int ppl) {
  switch (mode) {
    case MODE_V: return pick<TS, MODE_V>(g, ppl);
    case MODE_VGL: return pick<TS, MODE_VGL>(g, ppl);
    default: return pick<TS, MODE_VGL_SEPLAP>(g, ppl);
  }
}

}  // namespace pws
