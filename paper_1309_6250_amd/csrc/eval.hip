// Dispatch of the forward-evaluation kernels (the kernels live in eval_impl.hpp and are
// instantiated per storage dtype in eval_f64.hip, eval_f32.hip and eval_bf16.hip).
#include "eval_impl.hpp"

namespace pws {

EvalKernel pick_eval_f64(int mode, int g, int opl);
EvalKernel pick_eval_f32(int mode, int g, int opl);
EvalKernel pick_eval_bf16(int mode, int g, int opl);
EvalKernel pick_evalx_f64(int mode, int var, int g, int opl);
EvalKernel pick_evalx_f32(int mode, int var, int g, int opl);
EvalKernel pick_evalx_bf16(int mode, int var, int g, int opl);

// coefficients per 16-byte vector (the padding quantum of a table row)
int vec_of(int dtype) { return dtype == SPL_F64 ? 2 : dtype == SPL_F32 ? 4 : 8; }

// orbitals-per-lane choices of the forward kernels, per storage dtype: {lo, mid, hi}
void opl_set(int dtype, int out[3]) {
  if (dtype == SPL_F64) { out[0] = 1; out[1] = 2; out[2] = 2; }
  else if (dtype == SPL_F32) { out[0] = 1; out[1] = 2; out[2] = 4; }
  else { out[0] = 2; out[1] = 4; out[2] = 8; }
}

bool tile_valid(int dtype, const int32_t tile[2]) {
  const int g = tile[0], opl = tile[1];
  int set[3];
  opl_set(dtype, set);
  return g >= 2 && g <= 256 && (g & (g - 1)) == 0 && (opl == set[0] || opl == set[1] || opl == set[2]);
}

// A tile is valid for a descriptor when it is valid for its dtype and, for Bloch orbitals,
// gives every lane whole (re, im) pairs.
bool tile_valid_for(const spl_desc* d, const int32_t tile[2]) {
  return tile_valid(d->dtype, tile) && (!d->bloch || tile[1] % 2 == 0);
}

// Kernel arguments of one forward evaluation of one table with orbitals-per-lane `opl`.
void fill_eval_args(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v, void* grad,
                    void* lap, int values_only, int opl, EvalArgs* a) {
  a->g = make_geom(d);
  a->table = table;
  a->pos = pos;
  a->v = v;
  a->grad = grad;
  a->lap = lap;
  a->n_pts = (int32_t)n_pts;
  a->n_orb = d->n_col;
  a->n_chunks = (d->n_col + opl - 1) / opl;   // loads stay inside the row: o_pad is a multiple of opl
  // whole-vector stores need n_col % OPL == 0 and 16-byte aligned outputs
  const bool al = ((uintptr_t)v & 15) == 0 && (values_only || (((uintptr_t)grad & 15) == 0 &&
                                                               ((uintptr_t)lap & 15) == 0));
  a->vec_store = (d->n_col % opl) == 0 && al;
  a->tab_stride = d->table_elems;
  for (int c = 0; c < 3; ++c) a->k[c] = d->kvec[c];
  a->perm = nullptr;
  a->per_xcd = 0;
}

// Kernel of one forward evaluation of descriptor d (nullptr if the tile has none).  cached: the
// gather is expected to be served from cache (sorted call), so FP64 B-spline tables take the
// instances without slab prefetch.
EvalKernel eval_kernel_for(const spl_desc* d, int values_only, const int32_t tile[2], int cached) {
  const int mode = values_only ? MODE_V : (d->sep_grad ? MODE_SEP : (d->has_lap ? MODE_VGL_SEPLAP : MODE_VGL));
  int var = (d->basis == SPL_LAGRANGE ? VAR_LAGRANGE : 0) | (d->basis == SPL_PPSPLINE ? VAR_PP : 0) |
            (d->bloch ? VAR_BLOCH : 0);
  if (cached && d->dtype == SPL_F64 && mode != MODE_SEP && (var == 0 || var == VAR_BLOCH)) var |= VAR_NOPF;
  if (var == 0 && mode != MODE_SEP) {
    if (d->dtype == SPL_F64) return pick_eval_f64(mode, tile[0], tile[1]);
    if (d->dtype == SPL_F32) return pick_eval_f32(mode, tile[0], tile[1]);
    return pick_eval_bf16(mode, tile[0], tile[1]);
  }
  if (d->dtype == SPL_F64) return pick_evalx_f64(mode, var, tile[0], tile[1]);
  if (d->dtype == SPL_F32) return pick_evalx_f32(mode, var, tile[0], tile[1]);
  return pick_evalx_bf16(mode, var, tile[0], tile[1]);
}

// Launch one forward evaluation.  values_only: 1 values, 0 VGL (derivatives, separate Laplacian or
// five separate tables, as the descriptor says).
int launch_eval(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v, void* grad,
                void* lap, int values_only, const int32_t tile[2], hipStream_t stream) {
  if (n_pts == 0) return SPL_OK;
  if (!tile_valid_for(d, tile)) return fail(SPL_EINVAL, "invalid tile shape (%d, %d)", tile[0], tile[1]);
  EvalArgs a;
  fill_eval_args(d, table, n_pts, pos, v, grad, lap, values_only, tile[1], &a);
  EvalKernel k = eval_kernel_for(d, values_only, tile, 0);
  if (!k) return fail(SPL_EINVAL, "invalid tile shape (%d, %d)", tile[0], tile[1]);
  const int64_t per_block = 256 / tile[0];
  const dim3 grid((unsigned)((n_pts + per_block - 1) / per_block));
  hipLaunchKernelGGL(k, grid, dim3(256), 0, stream, a);
  return hip_fail(hipGetLastError(), "evaluation launch");
}

}  // namespace pws
