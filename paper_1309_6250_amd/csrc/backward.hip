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
// A lane group of G lanes owns a point, as in the forward kernel.
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
  int32_t n_chunks;
  int32_t pad_;
  int64_t lap_off;
};

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

template <typename TS, bool SEPLAP, int G>
__global__ __launch_bounds__(256) void k_backward(BwdArgs a) {
  using A = typename Acc<TS>::type;
  using GO = typename Out<TS>::type;   // dtype of upstream gradients and of the gradient table
  constexpr int VEC = Row16<TS>::VEC;
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
    int64_t rx[4], ry[4], rz[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      rx[l] = (int64_t)ix[l] * a.g.s0;
      ry[l] = (int64_t)iy[l] * a.g.s1;
      rz[l] = (int64_t)iz[l] * a.g.o_pad;
    }
    A wx[4], wy[4], wz[4], dwx[4], dwy[4], dwz[4], d2wx[4], d2wy[4], d2wz[4];
    bspline_weights<A>((A)t[0], wx, dwx, d2wx);
    bspline_weights<A>((A)t[1], wy, dwy, d2wy);
    bspline_weights<A>((A)t[2], wz, dwz, d2wz);
    const A d3w[4] = {A(-1), A(3), A(-3), A(1)};
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

    for (int c = lane; c < a.n_chunks && ok; c += G) {
      const int o = c * VEC;
      A gV[VEC], gL[VEC], gt[3][VEC];
#pragma unroll
      for (int j = 0; j < VEC; ++j) {
        const bool in = o + j < a.n_orb;
        const int64_t po = (int64_t)p * a.n_orb + o + j;
        const int64_t pg = (int64_t)p * 3 * a.n_orb + o + j;
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
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          A e[6][VEC];
#pragma unroll
          for (int j = 0; j < VEC; ++j) {
            const A cl = SEPLAP ? A(0) : gL[j];
            e[0][j] = fmaa(mt[0] * cl, d2wx[l], fmaa(gt[0][j], dwx[l], gV[j] * wx[l]));   // with wy wz
            e[1][j] = fmaa(A(2) * mt[3] * cl, dwx[l], gt[1][j] * wx[l]);                  // with dwy wz
            e[2][j] = fmaa(A(2) * mt[4] * cl, dwx[l], gt[2][j] * wx[l]);                  // with wy dwz
            e[3][j] = (mt[1] * cl) * wx[l];                                               // with d2wy wz
            e[4][j] = (mt[2] * cl) * wx[l];                                               // with wy d2wz
            e[5][j] = (A(2) * mt[5] * cl) * wx[l];                                        // with dwy dwz
          }
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            A f0[VEC], f1[VEC], f2[VEC];
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
              f0[j] = fmaa(e[3][j], d2wy[m], fmaa(e[1][j], dwy[m], e[0][j] * wy[m]));
              f1[j] = fmaa(e[5][j], dwy[m], e[2][j] * wy[m]);
              f2[j] = e[4][j] * wy[m];
            }
            GO* rp = gtab + rx[l] + ry[m] + o;
#pragma unroll
            for (int n = 0; n < 4; ++n) {
#pragma unroll
              for (int j = 0; j < VEC; ++j)
                if (o + j < a.n_orb)
                  atomic_add<GO>(rp + rz[n] + j, (GO)fmaa(f2[j], d2wz[n], fmaa(f1[j], dwz[n], f0[j] * wz[n])));
            }
          }
        }
        if constexpr (SEPLAP) {
          GO* ltab = gtab + a.lap_off;
#pragma unroll
          for (int l = 0; l < 4; ++l)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              GO* rp = ltab + rx[l] + ry[m] + o;
#pragma unroll
              for (int n = 0; n < 4; ++n) {
                const A w = wx[l] * wy[m] * wz[n];
#pragma unroll
                for (int j = 0; j < VEC; ++j)
                  if (o + j < a.n_orb) atomic_add<GO>(rp + rz[n] + j, (GO)(gL[j] * w));
              }
            }
        }
      }

      // ---------------- d pos: reduced derivatives up to third order
      if (a.gpos) {
        A dg[3][VEC], dh[6][VEC], dt[3][VEC];   // grad_t, Hessian (xx yy zz xy xz yz), T
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
#pragma unroll
          for (int i = 0; i < 3; ++i) { dg[i][j] = A(0); dt[i][j] = A(0); }
#pragma unroll
          for (int i = 0; i < 6; ++i) dh[i][j] = A(0);
        }
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          // y-stage sums B(b,c) = sum_m d^b wy * (sum_n d^c wz beta):
          // 0 (0,0) 1 (1,0) 2 (2,0) 3 (3,0) 4 (0,1) 5 (1,1) 6 (2,1) 7 (0,2) 8 (1,2) 9 (0,3)
          A B[10][VEC];
#pragma unroll
          for (int q = 0; q < 10; ++q)
#pragma unroll
            for (int j = 0; j < VEC; ++j) B[q][j] = A(0);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const TS* rp = tab + rx[l] + ry[m] + o;
            A r[4][VEC];
#pragma unroll
            for (int n = 0; n < 4; ++n) Row16<TS>::load(rp + rz[n], r[n]);
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
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
          for (int j = 0; j < VEC; ++j) {
            dg[0][j] = fmaa(dwx[l], B[0][j], dg[0][j]);
            dg[1][j] = fmaa(wx[l], B[1][j], dg[1][j]);
            dg[2][j] = fmaa(wx[l], B[4][j], dg[2][j]);
            dh[0][j] = fmaa(d2wx[l], B[0][j], dh[0][j]);
            dh[1][j] = fmaa(wx[l], B[2][j], dh[1][j]);
            dh[2][j] = fmaa(wx[l], B[7][j], dh[2][j]);
            dh[3][j] = fmaa(dwx[l], B[1][j], dh[3][j]);
            dh[4][j] = fmaa(dwx[l], B[4][j], dh[4][j]);
            dh[5][j] = fmaa(wx[l], B[5][j], dh[5][j]);
            if constexpr (!SEPLAP) {
              const A xxx = d3w[l] * B[0][j], yyy = wx[l] * B[3][j], zzz = wx[l] * B[9][j];
              const A xxy = d2wx[l] * B[1][j], xxz = d2wx[l] * B[4][j], xyy = dwx[l] * B[2][j];
              const A yyz = wx[l] * B[6][j], xzz = dwx[l] * B[7][j], yzz = wx[l] * B[8][j];
              const A xyz = dwx[l] * B[5][j];
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
          const TS* ltab = tab + a.lap_off;
#pragma unroll
          for (int l = 0; l < 4; ++l) {
            A b0[VEC], b1[VEC], b4[VEC];
#pragma unroll
            for (int j = 0; j < VEC; ++j) { b0[j] = A(0); b1[j] = A(0); b4[j] = A(0); }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const TS* rp = ltab + rx[l] + ry[m] + o;
              A r[4][VEC];
#pragma unroll
              for (int n = 0; n < 4; ++n) Row16<TS>::load(rp + rz[n], r[n]);
#pragma unroll
              for (int j = 0; j < VEC; ++j) {
                const A z0 = dot4(wz, r[0][j], r[1][j], r[2][j], r[3][j]);
                const A z1 = dot4(dwz, r[0][j], r[1][j], r[2][j], r[3][j]);
                b0[j] = fmaa(wy[m], z0, b0[j]);
                b1[j] = fmaa(dwy[m], z0, b1[j]);
                b4[j] = fmaa(wy[m], z1, b4[j]);
              }
            }
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
              dt[0][j] = fmaa(dwx[l], b0[j], dt[0][j]);
              dt[1][j] = fmaa(wx[l], b1[j], dt[1][j]);
              dt[2][j] = fmaa(wx[l], b4[j], dt[2][j]);
            }
          }
        }
        // q_k = gV g_k + sum_i gt_i H_ik + gL T_k, summed over this lane's orbitals
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
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

template <typename TS, bool SEPLAP>
static BwdKernel pick_bwd(int g) {
  switch (g) {
    case 1: return k_backward<TS, SEPLAP, 1>;
    case 2: return k_backward<TS, SEPLAP, 2>;
    case 4: return k_backward<TS, SEPLAP, 4>;
    case 8: return k_backward<TS, SEPLAP, 8>;
    case 16: return k_backward<TS, SEPLAP, 16>;
    case 32: return k_backward<TS, SEPLAP, 32>;
    case 64: return k_backward<TS, SEPLAP, 64>;
    case 128: return k_backward<TS, SEPLAP, 128>;
    default: return k_backward<TS, SEPLAP, 256>;
  }
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
  a.n_chunks = d->o_pad / vec_of(d->dtype);
  a.pad_ = 0;
  a.lap_off = d->table_elems;
  int g = 1;
  while (g < a.n_chunks && g < 64) g <<= 1;
  BwdKernel k;
  if (d->dtype == SPL_F64) k = d->has_lap ? pick_bwd<double, true>(g) : pick_bwd<double, false>(g);
  else if (d->dtype == SPL_F32) k = d->has_lap ? pick_bwd<float, true>(g) : pick_bwd<float, false>(g);
  else k = d->has_lap ? pick_bwd<uint16_t, true>(g) : pick_bwd<uint16_t, false>(g);
  const int64_t per_block = 256 / g;
  const dim3 grid((unsigned)((n_pts + per_block - 1) / per_block));
  hipLaunchKernelGGL(k, grid, dim3(256), 0, stream, a);
  return hip_fail(hipGetLastError(), "backward launch");
}

}  // namespace pws
