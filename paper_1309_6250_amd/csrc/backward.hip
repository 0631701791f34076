// spline_eval_vgl_backward: adjoint of the forward evaluation.
//
// The outputs V, grad V, lap V of a point are linear in the 64 coefficients of its block
// (App. A, Eq. b-splineapproximation, with the chain rule of Sec. II).  Given the
// gradients of a scalar loss with respect to them (gV, gG[3], gL), per orbital:
//
//   coefficients:  d beta(l,m,n) += gV w + gt . grad_t w + sum_ij C_ij d2_ij w
//        with gt = J gG (reduced-space cotangent of the gradient) and C_ij = M_ij gL
//        (2 M_ij off the diagonal): the exact transpose of the forward gather, done as a
//        separable scatter (x weights, then y, then z) and hardware FP atomics into the
//        caller's gradient table (L2 resolves collisions between points).
//   positions:     d pos = J^T q,  q_k = gV d_k V + sum_i gt_i H_ik + gL T_k,
//        T_k = sum_ij M_ij d3_ijk V (the piecewise-constant third derivative of the cubic
//        basis, -1 3 -3 1), or with a separate Laplacian spline the reduced gradient of
//        that spline.  q is summed over the orbitals of a point across its lane group
//        (LDS reduction), then one lane applies J^T and writes gpos.
//
// Mapping.  A lane group of G lanes owns a point.  Lane c of the group owns the orbitals
// c, c + G, ..., c + (OPL-1) G of each chunk of G*OPL orbitals: consecutive lanes hold
// consecutive orbitals, so every load and every atomic instruction of a wave covers whole
// contiguous cache lines of a table row (the scatter is bound by the number of line-sized
// atomic operations the memory side performs, so this matters more than vector width).
#include "common.hpp"

namespace pws {

struct BwdArgs {
  Geom g;
  const void* table;
  const double* pos;
  const void* gv;
  const void* ggrad;
  const void* glap;
  void* gtable;
  double* gpos;
  int32_t n_pts;
  int32_t n_orb;
  int32_t pad0_;
  int32_t pad1_;
  int64_t lap_off;
};

template <typename TS> struct Elem;
template <> struct Elem<double> {
  __device__ __forceinline__ static double load(const double* p) { return *p; }
};
template <> struct Elem<float> {
  __device__ __forceinline__ static float load(const float* p) { return *p; }
};
template <> struct Elem<uint16_t> {   // BF16 bits -> FP32
  __device__ __forceinline__ static float load(const uint16_t* p) { return __uint_as_float((uint32_t)*p << 16); }
};

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

template <typename A>
__device__ __forceinline__ A pick4b(int l, A a0, A a1, A a2, A a3) {
  return l == 0 ? a0 : (l == 1 ? a1 : (l == 2 ? a2 : a3));
}

template <typename TS, bool SEPLAP, int G, int OPL>
__global__ __launch_bounds__(256) void k_backward(BwdArgs a) {
  using A = typename Acc<TS>::type;
  using GO = typename Out<TS>::type;   // dtype of upstream gradients and of the gradient table
  constexpr int GPB = 256 / G;
  __shared__ double red[256][3];
  const int grp = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  const int p = (int)blockIdx.x * GPB + grp;
  const bool active = p < a.n_pts;
  double qs[3] = {0.0, 0.0, 0.0};
  bool ok = false;

  if (active) {
    int i0[3];
    double t[3];
    ok = reduce_point(a.g, a.pos[3 * (int64_t)p], a.pos[3 * (int64_t)p + 1], a.pos[3 * (int64_t)p + 2], i0,
                      t);
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
    bspline_weights<A>((A)t[0], wx, dwx, d2wx);
    bspline_weights<A>((A)t[1], wy, dwy, d2wy);
    bspline_weights<A>((A)t[2], wz, dwz, d2wz);
    const A d3w[4] = {A(-1), A(3), A(-3), A(1)};   // third derivative of the cubic basis (unit spacing)
    A jm[9], mt[6];
#pragma unroll
    for (int i = 0; i < 9; ++i) jm[i] = (A)a.g.jac[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) mt[i] = (A)a.g.metric[i];

    const TS* __restrict__ tab = static_cast<const TS*>(a.table);
    const GO* gvp = static_cast<const GO*>(a.gv);
    const GO* ggp = static_cast<const GO*>(a.ggrad);
    const GO* glp = static_cast<const GO*>(a.glap);
    GO* gtab = static_cast<GO*>(a.gtable);

    for (int cb = 0; cb < a.n_orb && ok; cb += G * OPL) {
      int oj[OPL];            // this lane's orbitals in the chunk
      bool inj[OPL];
#pragma unroll
      for (int j = 0; j < OPL; ++j) {
        oj[j] = cb + lane + j * G;
        inj[j] = oj[j] < a.n_orb;
      }
      A gV[OPL], gL[OPL], gt[3][OPL];
#pragma unroll
      for (int j = 0; j < OPL; ++j) {
        const bool in = inj[j];
        const int64_t po = (int64_t)p * a.n_orb + oj[j];
        const int64_t pg = (int64_t)p * 3 * a.n_orb + oj[j];
        gV[j] = (in && gvp) ? (A)gvp[po] : A(0);
        gL[j] = (in && glp) ? (A)glp[po] : A(0);
        const A g0 = (in && ggp) ? (A)ggp[pg] : A(0);
        const A g1 = (in && ggp) ? (A)ggp[pg + a.n_orb] : A(0);
        const A g2 = (in && ggp) ? (A)ggp[pg + 2 * a.n_orb] : A(0);
#pragma unroll
        for (int i = 0; i < 3; ++i) gt[i][j] = fmaa(jm[3 * i + 2], g2, fmaa(jm[3 * i + 1], g1, jm[3 * i] * g0));
      }

      // ---------------- d beta: separable scatter, transpose of the forward contraction
      if (gtab) {
#pragma unroll 1
        for (int l = 0; l < 4; ++l) {
          const A xw = pick4b(l, wx[0], wx[1], wx[2], wx[3]);
          const A xd = pick4b(l, dwx[0], dwx[1], dwx[2], dwx[3]);
          const A xdd = pick4b(l, d2wx[0], d2wx[1], d2wx[2], d2wx[3]);
          GO* slab = gtab + (int64_t)pick4b(l, ix[0], ix[1], ix[2], ix[3]) * a.g.s0;
          A e[6][OPL];
#pragma unroll
          for (int j = 0; j < OPL; ++j) {
            const A cl = SEPLAP ? A(0) : gL[j];
            e[0][j] = fmaa(mt[0] * cl, xdd, fmaa(gt[0][j], xd, gV[j] * xw));   // with wy wz
            e[1][j] = fmaa(A(2) * mt[3] * cl, xd, gt[1][j] * xw);              // with dwy wz
            e[2][j] = fmaa(A(2) * mt[4] * cl, xd, gt[2][j] * xw);              // with wy dwz
            e[3][j] = (mt[1] * cl) * xw;                                       // with d2wy wz
            e[4][j] = (mt[2] * cl) * xw;                                       // with wy d2wz
            e[5][j] = (A(2) * mt[5] * cl) * xw;                                // with dwy dwz
          }
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            A f0[OPL], f1[OPL], f2[OPL];
#pragma unroll
            for (int j = 0; j < OPL; ++j) {
              f0[j] = fmaa(e[3][j], d2wy[m], fmaa(e[1][j], dwy[m], e[0][j] * wy[m]));
              f1[j] = fmaa(e[5][j], dwy[m], e[2][j] * wy[m]);
              f2[j] = e[4][j] * wy[m];
            }
            GO* rp = slab + ry[m];
#pragma unroll
            for (int n = 0; n < 4; ++n) {
#pragma unroll
              for (int j = 0; j < OPL; ++j)
                if (inj[j])
                  atomic_add<GO>(rp + rz[n] + oj[j], (GO)fmaa(f2[j], d2wz[n], fmaa(f1[j], dwz[n], f0[j] * wz[n])));
            }
          }
        }
        if constexpr (SEPLAP) {
#pragma unroll 1
          for (int l = 0; l < 4; ++l) {
            const A xw = pick4b(l, wx[0], wx[1], wx[2], wx[3]);
            GO* slab = gtab + a.lap_off + (int64_t)pick4b(l, ix[0], ix[1], ix[2], ix[3]) * a.g.s0;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              GO* rp = slab + ry[m];
              const A xy = xw * wy[m];
#pragma unroll
              for (int n = 0; n < 4; ++n) {
                const A w = xy * wz[n];
#pragma unroll
                for (int j = 0; j < OPL; ++j)
                  if (inj[j]) atomic_add<GO>(rp + rz[n] + oj[j], (GO)(gL[j] * w));
              }
            }
          }
        }
      }

      // ---------------- d pos: reduced derivatives up to third order
      if (a.gpos) {
        A dg[3][OPL], dh[6][OPL], dt[3][OPL];   // grad_t, Hessian (xx yy zz xy xz yz), T
#pragma unroll
        for (int j = 0; j < OPL; ++j) {
#pragma unroll
          for (int i = 0; i < 3; ++i) { dg[i][j] = A(0); dt[i][j] = A(0); }
#pragma unroll
          for (int i = 0; i < 6; ++i) dh[i][j] = A(0);
        }
#pragma unroll 1
        for (int l = 0; l < 4; ++l) {
          const A xw = pick4b(l, wx[0], wx[1], wx[2], wx[3]);
          const A xd = pick4b(l, dwx[0], dwx[1], dwx[2], dwx[3]);
          const A xdd = pick4b(l, d2wx[0], d2wx[1], d2wx[2], d2wx[3]);
          const A xddd = pick4b(l, d3w[0], d3w[1], d3w[2], d3w[3]);
          const TS* slab = tab + (int64_t)pick4b(l, ix[0], ix[1], ix[2], ix[3]) * a.g.s0;
          // second-axis sums B(b,c) = sum_m d^b wy * (sum_n d^c wz beta):
          // 0 (0,0) 1 (1,0) 2 (2,0) 3 (3,0) 4 (0,1) 5 (1,1) 6 (2,1) 7 (0,2) 8 (1,2) 9 (0,3)
          A B[10][OPL];
#pragma unroll
          for (int q = 0; q < 10; ++q)
#pragma unroll
            for (int j = 0; j < OPL; ++j) B[q][j] = A(0);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const TS* rp = slab + ry[m];
            A r[4][OPL];
#pragma unroll
            for (int n = 0; n < 4; ++n)
#pragma unroll
              for (int j = 0; j < OPL; ++j) r[n][j] = inj[j] ? (A)Elem<TS>::load(rp + rz[n] + oj[j]) : A(0);
#pragma unroll
            for (int j = 0; j < OPL; ++j) {
              const A z0 = dot4(wz, r[0][j], r[1][j], r[2][j], r[3][j]);
              const A z1 = dot4(dwz, r[0][j], r[1][j], r[2][j], r[3][j]);
              const A z2 = dot4(d2wz, r[0][j], r[1][j], r[2][j], r[3][j]);
              B[0][j] = fmaa(wy[m], z0, B[0][j]);
              B[1][j] = fmaa(dwy[m], z0, B[1][j]);
              B[2][j] = fmaa(d2wy[m], z0, B[2][j]);
              B[4][j] = fmaa(wy[m], z1, B[4][j]);
              B[5][j] = fmaa(dwy[m], z1, B[5][j]);
              B[7][j] = fmaa(wy[m], z2, B[7][j]);
              if constexpr (!SEPLAP) {
                const A z3 = dot4(d3w, r[0][j], r[1][j], r[2][j], r[3][j]);
                B[3][j] = fmaa(d3w[m], z0, B[3][j]);
                B[6][j] = fmaa(d2wy[m], z1, B[6][j]);
                B[8][j] = fmaa(dwy[m], z2, B[8][j]);
                B[9][j] = fmaa(wy[m], z3, B[9][j]);
              }
            }
          }
#pragma unroll
          for (int j = 0; j < OPL; ++j) {
            dg[0][j] = fmaa(xd, B[0][j], dg[0][j]);
            dg[1][j] = fmaa(xw, B[1][j], dg[1][j]);
            dg[2][j] = fmaa(xw, B[4][j], dg[2][j]);
            dh[0][j] = fmaa(xdd, B[0][j], dh[0][j]);
            dh[1][j] = fmaa(xw, B[2][j], dh[1][j]);
            dh[2][j] = fmaa(xw, B[7][j], dh[2][j]);
            dh[3][j] = fmaa(xd, B[1][j], dh[3][j]);
            dh[4][j] = fmaa(xd, B[4][j], dh[4][j]);
            dh[5][j] = fmaa(xw, B[5][j], dh[5][j]);
            if constexpr (!SEPLAP) {
              const A xxx = xddd * B[0][j], yyy = xw * B[3][j], zzz = xw * B[9][j];
              const A xxy = xdd * B[1][j], xxz = xdd * B[4][j], xyy = xd * B[2][j];
              const A yyz = xw * B[6][j], xzz = xd * B[7][j], yzz = xw * B[8][j];
              const A xyz = xd * B[5][j];
              dt[0][j] += fmaa(A(2), fmaa(mt[5], xyz, fmaa(mt[4], xxz, mt[3] * xxy)),
                               fmaa(mt[2], xzz, fmaa(mt[1], xyy, mt[0] * xxx)));
              dt[1][j] += fmaa(A(2), fmaa(mt[5], yyz, fmaa(mt[4], xyz, mt[3] * xyy)),
                               fmaa(mt[2], yzz, fmaa(mt[1], yyy, mt[0] * xxy)));
              dt[2][j] += fmaa(A(2), fmaa(mt[5], yzz, fmaa(mt[4], xzz, mt[3] * xyz)),
                               fmaa(mt[2], zzz, fmaa(mt[1], yyz, mt[0] * xxz)));
            }
          }
        }
        if constexpr (SEPLAP) {
          // T = reduced gradient of the separate Laplacian spline
#pragma unroll 1
          for (int l = 0; l < 4; ++l) {
            const A xw = pick4b(l, wx[0], wx[1], wx[2], wx[3]);
            const A xd = pick4b(l, dwx[0], dwx[1], dwx[2], dwx[3]);
            const TS* slab = tab + a.lap_off + (int64_t)pick4b(l, ix[0], ix[1], ix[2], ix[3]) * a.g.s0;
            A b0[OPL], b1[OPL], b4[OPL];
#pragma unroll
            for (int j = 0; j < OPL; ++j) { b0[j] = A(0); b1[j] = A(0); b4[j] = A(0); }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const TS* rp = slab + ry[m];
              A r[4][OPL];
#pragma unroll
              for (int n = 0; n < 4; ++n)
#pragma unroll
                for (int j = 0; j < OPL; ++j) r[n][j] = inj[j] ? (A)Elem<TS>::load(rp + rz[n] + oj[j]) : A(0);
#pragma unroll
              for (int j = 0; j < OPL; ++j) {
                const A z0 = dot4(wz, r[0][j], r[1][j], r[2][j], r[3][j]);
                const A z1 = dot4(dwz, r[0][j], r[1][j], r[2][j], r[3][j]);
                b0[j] = fmaa(wy[m], z0, b0[j]);
                b1[j] = fmaa(dwy[m], z0, b1[j]);
                b4[j] = fmaa(wy[m], z1, b4[j]);
              }
            }
#pragma unroll
            for (int j = 0; j < OPL; ++j) {
              dt[0][j] = fmaa(xd, b0[j], dt[0][j]);
              dt[1][j] = fmaa(xw, b1[j], dt[1][j]);
              dt[2][j] = fmaa(xw, b4[j], dt[2][j]);
            }
          }
        }
        // q_k = gV g_k + sum_i gt_i H_ik + gL T_k, summed over this lane's orbitals
#pragma unroll
        for (int j = 0; j < OPL; ++j) {
          const A h00 = dh[0][j], h11 = dh[1][j], h22 = dh[2][j], h01 = dh[3][j], h02 = dh[4][j], h12 = dh[5][j];
          const A q0 = fmaa(gL[j], dt[0][j], fmaa(gt[2][j], h02, fmaa(gt[1][j], h01, fmaa(gt[0][j], h00, gV[j] * dg[0][j]))));
          const A q1 = fmaa(gL[j], dt[1][j], fmaa(gt[2][j], h12, fmaa(gt[1][j], h11, fmaa(gt[0][j], h01, gV[j] * dg[1][j]))));
          const A q2 = fmaa(gL[j], dt[2][j], fmaa(gt[2][j], h22, fmaa(gt[1][j], h12, fmaa(gt[0][j], h02, gV[j] * dg[2][j]))));
          qs[0] += (double)q0;
          qs[1] += (double)q1;
          qs[2] += (double)q2;
        }
      }
    }
  }

  if (a.gpos) {
    red[threadIdx.x][0] = qs[0];
    red[threadIdx.x][1] = qs[1];
    red[threadIdx.x][2] = qs[2];
    __syncthreads();
    if (active && lane == 0) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int i = 0; i < G; ++i) {
        s0 += red[threadIdx.x + i][0];
        s1 += red[threadIdx.x + i][1];
        s2 += red[threadIdx.x + i][2];
      }
      double* out = a.gpos + 3 * (int64_t)p;
      if (ok) {
        const double* J = a.g.jac;
        out[0] = fmaa(J[6], s2, fmaa(J[3], s1, J[0] * s0));
        out[1] = fmaa(J[7], s2, fmaa(J[4], s1, J[1] * s0));
        out[2] = fmaa(J[8], s2, fmaa(J[5], s1, J[2] * s0));
      } else {
        out[0] = out[1] = out[2] = __builtin_nan("");
      }
    }
  }
}

typedef void (*BwdKernel)(BwdArgs);

template <typename TS, bool SEPLAP, int OPL>
static BwdKernel pick_bwd_g(int g) {
  switch (g) {
    case 4: return k_backward<TS, SEPLAP, 4, OPL>;
    case 16: return k_backward<TS, SEPLAP, 16, OPL>;
    default: return k_backward<TS, SEPLAP, 64, OPL>;
  }
}

template <typename TS, bool SEPLAP>
static BwdKernel pick_bwd(int g, int opl) {
  return opl == 1 ? pick_bwd_g<TS, SEPLAP, 1>(g) : pick_bwd_g<TS, SEPLAP, 2>(g);
}

int vec_of(int dtype);

int launch_backward(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, const void* gv,
                    const void* ggrad, const void* glap, void* gtable, double* gpos, hipStream_t stream) {
  if (n_pts == 0 || (!gtable && !gpos)) return SPL_OK;
  BwdArgs a;
  a.g = make_geom(d);
  a.table = table;
  a.pos = pos;
  a.gv = gv;
  a.ggrad = ggrad;
  a.glap = glap;
  a.gtable = gtable;
  a.gpos = gpos;
  a.n_pts = (int32_t)n_pts;
  a.n_orb = d->n_orb;
  a.pad0_ = 0;
  a.pad1_ = 0;
  a.lap_off = d->table_elems;
  // lanes per point: 4, 16 or 64 (enough to cover the orbitals); orbitals per lane: 1 for FP64
  // tables, up to 2 otherwise (more would cost occupancy); further orbitals loop over chunks
  const int g = d->n_orb <= 4 ? 4 : (d->n_orb <= 16 ? 16 : 64);
  const int need = (d->n_orb + g - 1) / g;
  const int opl = (d->dtype == SPL_F64 || need <= 1) ? 1 : 2;
  BwdKernel k;
  if (d->dtype == SPL_F64) k = d->has_lap ? pick_bwd<double, true>(g, opl) : pick_bwd<double, false>(g, opl);
  else if (d->dtype == SPL_F32) k = d->has_lap ? pick_bwd<float, true>(g, opl) : pick_bwd<float, false>(g, opl);
  else k = d->has_lap ? pick_bwd<uint16_t, true>(g, opl) : pick_bwd<uint16_t, false>(g, opl);
  const int64_t per_block = 256 / g;
  const dim3 grid((unsigned)((n_pts + per_block - 1) / per_block));
  hipLaunchKernelGGL(k, grid, dim3(256), 0, stream, a);
  return hip_fail(hipGetLastError(), "backward launch");
}

}  // namespace pws
