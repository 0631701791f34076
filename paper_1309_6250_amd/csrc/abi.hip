// C ABI of the pwspline library: descriptors, argument checks, error reporting and the
// dispatch of the build, forward and backward entry points declared in pwspline.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "cells.hpp"
#include "internal.hpp"

namespace pws {

static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t err, const char* what) {
  if (err == hipSuccess) return SPL_OK;
  return fail(SPL_EHIP, "%s: %s", what, hipGetErrorString(err));
}

void clear_error() { g_last_error.clear(); }

static int elem_bytes_of(int dtype) { return dtype == SPL_F64 ? 8 : dtype == SPL_F32 ? 4 : 2; }

Geom make_geom(const spl_desc* d) {
  Geom g;
  memcpy(g.ainv, d->ainv, sizeof(g.ainv));
  memcpy(g.jac, d->jac, sizeof(g.jac));
  memcpy(g.metric, d->metric, sizeof(g.metric));
  for (int i = 0; i < 3; ++i) g.n[i] = d->grid[i];
  g.o_pad = d->o_pad;
  g.s1 = (int64_t)d->grid[2] * d->o_pad * (d->basis == SPL_PPSPLINE ? 8 : 1);
  g.s0 = (int64_t)d->grid[1] * g.s1;
  return g;
}

static int derive(spl_desc* d) {
  if (!d) return fail(SPL_EINVAL, "descriptor is NULL");
  if (d->dtype != SPL_F64 && d->dtype != SPL_F32 && d->dtype != SPL_BF16)
    return fail(SPL_EDTYPE, "unknown dtype %d", d->dtype);
  for (int i = 0; i < 3; ++i)
    if (d->grid[i] < 4 || d->grid[i] > 1024)
      return fail(SPL_EGRID, "grid[%d] = %d outside [4, 1024]", i, d->grid[i]);
  if (d->n_orb < 1) return fail(SPL_EINVAL, "n_orb = %d < 1", d->n_orb);
  if (d->n_orb > (1 << 29)) return fail(SPL_EINVAL, "n_orb = %d too large", d->n_orb);
  if (d->has_lap != 0 && d->has_lap != 1) return fail(SPL_EINVAL, "has_lap must be 0 or 1");
  if (d->sep_grad != 0 && d->sep_grad != 1) return fail(SPL_EINVAL, "sep_grad must be 0 or 1");
  if (d->bloch != 0 && d->bloch != 1) return fail(SPL_EINVAL, "bloch must be 0 or 1");
  if (d->basis != SPL_BSPLINE && d->basis != SPL_LAGRANGE && d->basis != SPL_PPSPLINE)
    return fail(SPL_EINVAL, "unknown basis %d", d->basis);
  if (d->basis == SPL_PPSPLINE && d->sep_grad) return fail(SPL_EINVAL, "pp-spline tables take no separate gradients");
  if (d->reserved != 0) return fail(SPL_EINVAL, "reserved must be 0");
  if (d->sep_grad && !d->has_lap) return fail(SPL_EINVAL, "sep_grad needs has_lap (five tables)");
  if (d->basis == SPL_LAGRANGE && !d->sep_grad)
    return fail(SPL_EINVAL, "Lagrange tables have no continuous derivatives: set sep_grad and has_lap");
  for (int c = 0; c < 3; ++c) {
    if (!isfinite(d->kvec[c])) return fail(SPL_EINVAL, "kvec has a non-finite entry");
    if (!d->bloch && d->kvec[c] != 0.0) return fail(SPL_EINVAL, "kvec must be zero unless bloch = 1");
  }
  for (int i = 0; i < 9; ++i)
    if (!isfinite(d->lattice[i])) return fail(SPL_EINVAL, "lattice has a non-finite entry");
  // a = lattice^T (columns = lattice vectors); ainv = a^-1 = (lattice^-1)^T
  const double* L = d->lattice;
  const double c00 = L[4] * L[8] - L[5] * L[7], c01 = L[5] * L[6] - L[3] * L[8], c02 = L[3] * L[7] - L[4] * L[6];
  const double det = L[0] * c00 + L[1] * c01 + L[2] * c02;
  double scale = 0.0;
  for (int i = 0; i < 9; ++i) scale = fmax(scale, fabs(L[i]));
  if (!(fabs(det) > 1e-12 * scale * scale * scale) || !isfinite(det))
    return fail(SPL_EINVAL, "lattice is singular (det = %g)", det);
  // inverse of L (row-major): Linv[i][j] = cof[j][i] / det
  double cof[9];
  cof[0] = c00; cof[1] = c01; cof[2] = c02;
  cof[3] = L[2] * L[7] - L[1] * L[8]; cof[4] = L[0] * L[8] - L[2] * L[6]; cof[5] = L[1] * L[6] - L[0] * L[7];
  cof[6] = L[1] * L[5] - L[2] * L[4]; cof[7] = L[2] * L[3] - L[0] * L[5]; cof[8] = L[0] * L[4] - L[1] * L[3];
  double linv[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) linv[3 * i + j] = cof[3 * j + i] / det;
  // ainv = (Linv)^T
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) d->ainv[3 * i + j] = linv[3 * j + i];
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < 3; ++c) d->jac[3 * i + c] = (double)d->grid[i] * d->ainv[3 * i + c];
  double m[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      m[3 * i + j] = d->jac[3 * i] * d->jac[3 * j] + d->jac[3 * i + 1] * d->jac[3 * j + 1] +
                     d->jac[3 * i + 2] * d->jac[3 * j + 2];
  d->metric[0] = m[0]; d->metric[1] = m[4]; d->metric[2] = m[8];
  d->metric[3] = m[1]; d->metric[4] = m[2]; d->metric[5] = m[5];
  d->elem_bytes = elem_bytes_of(d->dtype);
  d->n_col = d->n_orb * (1 + d->bloch);
  d->n_tables = 1 + d->has_lap + 3 * d->sep_grad;
  const int per16 = 16 / d->elem_bytes;
  d->o_pad = (d->n_col + per16 - 1) / per16 * per16;
  const int64_t pts = (int64_t)d->grid[0] * d->grid[1] * d->grid[2];
  d->table_elems = pts * d->o_pad * (d->basis == SPL_PPSPLINE ? 8 : 1);
  d->table_bytes = d->n_tables * d->table_elems * d->elem_bytes;
  d->work_bytes = pts * d->n_col * 8;
  d->gtable_bytes = d->n_tables * d->table_elems * (d->dtype == SPL_F64 ? 8 : 4);
  return SPL_OK;
}

int check_desc(const spl_desc* d) {
  if (!d) return fail(SPL_EINVAL, "descriptor is NULL");
  spl_desc tmp = *d;
  const int rc = derive(&tmp);
  if (rc) return rc;
  if (tmp.o_pad != d->o_pad || tmp.table_elems != d->table_elems || tmp.table_bytes != d->table_bytes ||
      tmp.elem_bytes != d->elem_bytes || tmp.n_col != d->n_col || tmp.n_tables != d->n_tables ||
      memcmp(tmp.jac, d->jac, sizeof(tmp.jac)) != 0)
    return fail(SPL_EINVAL, "descriptor not initialized by spline_desc_init (or modified since)");
  return SPL_OK;
}

static bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

// ---------------------------------------------------------------- tile cache
static std::mutex g_tune_mu;
static std::map<std::string, std::pair<int, int>> g_tune;
static bool g_tune_loaded = false;

static std::string tune_key(const spl_desc* d) {
  char buf[128];
  snprintf(buf, sizeof(buf), "v3:%d:%d:%d:%d:%d:%d:%d:%d:%d", d->dtype, d->has_lap, d->o_pad, d->grid[0],
           d->grid[1], d->grid[2], d->basis, d->sep_grad, d->bloch);
  return buf;
}

static void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = getenv("PWSPLINE_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char key[128];
  int g, opl;
  while (fscanf(f, "%127s %d %d", key, &g, &opl) == 3) g_tune[key] = {g, opl};
  fclose(f);
}

static void tune_store_locked(const std::string& key, int g, int opl) {
  g_tune[key] = {g, opl};
  const char* path = getenv("PWSPLINE_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %d\n", key.c_str(), g, opl);
  fclose(f);
}

int vec_of(int dtype);
void opl_set(int dtype, int out[3]);
bool tile_valid(int dtype, const int32_t tile[2]);

// Default launch shape: the middle orbitals-per-lane choice, and enough lanes per point to
// cover a table row in one pass (at most 256).
void default_tile(const spl_desc* d, int32_t tile[2]) {
  int set[3];
  opl_set(d->dtype, set);
  const int chunks = d->o_pad / set[1];
  int g = 2;
  while (g < chunks && g < 256) g <<= 1;
  tile[0] = g;
  tile[1] = set[1];
}

void tile_for(const spl_desc* d, int32_t tile[2]) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(tune_key(d));
  if (it != g_tune.end()) {
    tile[0] = it->second.first;
    tile[1] = it->second.second;
    if (tile_valid_for(d, tile)) return;
  }
  default_tile(d, tile);
}

int launch_eval(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v, void* grad,
                void* lap, int values_only, const int32_t tile[2], hipStream_t stream);
int launch_backward(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, const void* gv,
                    const void* ggrad, const void* glap, void* gtable, double* gpos, hipStream_t stream);
int build_one(const spl_desc* d, const double* vals, void* table, double* work, hipStream_t stream);
int cast_one(const spl_desc* d, const double* vals, void* table, hipStream_t stream);
int build_one_pp(const spl_desc* d, const double* vals, void* table, double* work, hipStream_t stream);
int sorted_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes);
int64_t smoothing_work_bytes(const spl_desc* d);
int build_smoothing(const spl_desc* d, int64_t n_g, const int32_t* miller, const double* coef, void* table,
                    void* work, hipStream_t stream);
int launch_backward_sorted(const spl_desc* d, int64_t n_pts, const double* pos, const void* gv, const void* ggrad,
                           const void* glap, void* gtable, void* work, int64_t work_bytes, bool reuse,
                           hipStream_t stream);

int check_eval_args(const spl_desc* d, const void* table, int64_t n_pts, const double* pos) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (n_pts < 0 || n_pts > 0x7fffffffLL) return fail(SPL_EINVAL, "n_pts = %lld outside [0, 2^31)", (long long)n_pts);
  if (n_pts == 0) return SPL_OK;
  if (!table) return fail(SPL_EINVAL, "table is NULL");
  if (!pos) return fail(SPL_EINVAL, "pos is NULL");
  if (!aligned(table, 16)) return fail(SPL_EINVAL, "table must be 16-byte aligned");
  if (!aligned(pos, 8)) return fail(SPL_EINVAL, "pos must be 8-byte aligned");
  return SPL_OK;
}

static int out_align_ok(const spl_desc* d, const void* p) {
  return aligned(p, d->dtype == SPL_F64 ? 8 : 4);
}

int check_vgl_outputs(const spl_desc* d, const void* v, const void* grad, const void* lap) {
  if (!v || !grad || !lap) return fail(SPL_EINVAL, "v, grad and lap must be non-NULL");
  if (!out_align_ok(d, v) || !out_align_ok(d, grad) || !out_align_ok(d, lap))
    return fail(SPL_EINVAL, "output not aligned to its element size");
  return SPL_OK;
}

}  // namespace pws

using namespace pws;

extern "C" {

int spline_version(void) { return 10300; }

const char* spline_last_error(void) { return g_last_error.c_str(); }

int spline_desc_init(spl_desc* d) {
  clear_error();
  return derive(d);
}

int spline_build(const spl_desc* d, const double* grid_vals, const double* lap_vals, void* table, void* work,
                 void* stream) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (d->basis == SPL_LAGRANGE || d->sep_grad)
    return fail(SPL_EINVAL, "Lagrange or separate-gradient descriptors are built with spline_build_tables");
  if (!grid_vals || !table || !work) return fail(SPL_EINVAL, "grid_vals, table and work must be non-NULL");
  if (d->has_lap && !lap_vals) return fail(SPL_EINVAL, "has_lap = 1 needs lap_vals");
  if (!d->has_lap && lap_vals) return fail(SPL_EINVAL, "lap_vals given but has_lap = 0");
  if (!aligned(grid_vals, 8) || !aligned(work, 8) || !aligned(table, 16) || (lap_vals && !aligned(lap_vals, 8)))
    return fail(SPL_EINVAL, "misaligned buffer (grid values/work need 8 bytes, table 16)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto one = d->basis == SPL_PPSPLINE ? build_one_pp : build_one;
  if ((rc = one(d, grid_vals, table, static_cast<double*>(work), s))) return rc;
  if (d->has_lap) {
    char* lt = static_cast<char*>(table) + d->table_elems * d->elem_bytes;
    if ((rc = one(d, lap_vals, lt, static_cast<double*>(work), s))) return rc;
  }
  return SPL_OK;
}

int spline_build_tables(const spl_desc* d, const double* vals, void* table, void* work, void* stream) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  const bool lagr = d->basis == SPL_LAGRANGE;
  if (!vals || !table || (!lagr && !work)) return fail(SPL_EINVAL, "vals, table and (B-spline) work must be non-NULL");
  if (!aligned(vals, 8) || !aligned(table, 16) || (work && !aligned(work, 8)))
    return fail(SPL_EINVAL, "misaligned buffer (grid values/work need 8 bytes, table 16)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t per_vals = (int64_t)d->grid[0] * d->grid[1] * d->grid[2] * d->n_col;
  for (int t = 0; t < d->n_tables; ++t) {
    const double* v = vals + t * per_vals;
    void* dst = static_cast<char*>(table) + t * d->table_elems * d->elem_bytes;
    double* w = static_cast<double*>(work);
    if ((rc = lagr ? cast_one(d, v, dst, s)
                   : (d->basis == SPL_PPSPLINE ? build_one_pp(d, v, dst, w, s) : build_one(d, v, dst, w, s))))
      return rc;
  }
  return SPL_OK;
}

int spline_smoothing_work_bytes(const spl_desc* d, int64_t* bytes) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (!bytes) return fail(SPL_EINVAL, "bytes is NULL");
  *bytes = smoothing_work_bytes(d);
  return SPL_OK;
}

int spline_build_smoothing(const spl_desc* d, int64_t n_g, const int32_t* miller, const double* coef, void* table,
                           void* work, void* stream) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (d->basis != SPL_BSPLINE) return fail(SPL_EINVAL, "smoothing coefficients are B-spline coefficients");
  if (n_g < 1 || n_g > 0x7fffffffLL) return fail(SPL_EINVAL, "n_g = %lld outside [1, 2^31)", (long long)n_g);
  if ((double)n_g * d->n_orb > 9.0e18) return fail(SPL_EINVAL, "too many coefficients");
  if (!miller || !coef || !table || !work) return fail(SPL_EINVAL, "miller, coef, table and work must be non-NULL");
  if (!aligned(miller, 4) || !aligned(coef, 16) || !aligned(table, 16) || !aligned(work, 256))
    return fail(SPL_EINVAL, "misaligned buffer (miller 4, coef 16, table 16, work 256 bytes)");
  return build_smoothing(d, n_g, miller, coef, table, work, static_cast<hipStream_t>(stream));
}

int spline_eval_v(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v, void* stream) {
  clear_error();
  int rc = check_eval_args(d, table, n_pts, pos);
  if (rc || n_pts == 0) return rc;
  if (!v) return fail(SPL_EINVAL, "v is NULL");
  if (!out_align_ok(d, v)) return fail(SPL_EINVAL, "output not aligned to its element size");
  int32_t tile[2];
  tile_for(d, tile);
  // the values-only kernel keeps the VGL tile's lane grouping
  return launch_eval(d, table, n_pts, pos, v, nullptr, nullptr, 1, tile, static_cast<hipStream_t>(stream));
}

int spline_eval_vgl_tile(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v,
                         void* grad, void* lap, const int32_t tile[2], void* stream) {
  clear_error();
  int rc = check_eval_args(d, table, n_pts, pos);
  if (rc || n_pts == 0) return rc;
  if ((rc = check_vgl_outputs(d, v, grad, lap))) return rc;
  if (!tile || !tile_valid_for(d, tile)) return fail(SPL_EINVAL, "invalid tile");
  return launch_eval(d, table, n_pts, pos, v, grad, lap, 0, tile, static_cast<hipStream_t>(stream));
}

int spline_eval_vgl(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v, void* grad,
                    void* lap, void* stream) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  int32_t tile[2];
  tile_for(d, tile);
  return spline_eval_vgl_tile(d, table, n_pts, pos, v, grad, lap, tile, stream);
}

int spline_tile_for(const spl_desc* d, int64_t n_pts, int32_t tile_out[2]) {
  clear_error();
  (void)n_pts;
  int rc = check_desc(d);
  if (rc) return rc;
  if (!tile_out) return fail(SPL_EINVAL, "tile_out is NULL");
  tile_for(d, tile_out);
  return SPL_OK;
}

int spline_autotune(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v, void* grad,
                    void* lap, void* stream, int32_t tile_out[2]) {
  clear_error();
  int rc = check_eval_args(d, table, n_pts, pos);
  if (rc) return rc;
  if (!v || !grad || !lap || !tile_out) return fail(SPL_EINVAL, "outputs and tile_out must be non-NULL");
  if (n_pts == 0) return fail(SPL_EINVAL, "autotuning needs n_pts > 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int set[3];
  opl_set(d->dtype, set);
  hipEvent_t e0, e1;
  if ((rc = hip_fail(hipEventCreate(&e0), "hipEventCreate"))) return rc;
  if ((rc = hip_fail(hipEventCreate(&e1), "hipEventCreate"))) { hipEventDestroy(e0); return rc; }
  float best = 1e30f;
  int32_t best_tile[2] = {0, 0};
  for (int k = 0; k < 3 && !rc; ++k) {
    const int opl = set[k];
    if (k > 0 && opl == set[k - 1]) continue;
    if (d->bloch && opl % 2 != 0) continue;       // Bloch lanes hold whole (re, im) pairs
    const int chunks = d->o_pad / opl;
    int gmax = 2;
    while (gmax < chunks && gmax < 256) gmax <<= 1;
    for (int g = (gmax >= 4 ? 4 : 2); g <= gmax && !rc; g <<= 1) {
      const int32_t tile[2] = {g, opl};
      if ((rc = launch_eval(d, table, n_pts, pos, v, grad, lap, 0, tile, s))) break;   // warm-up
      float times[3];
      for (int r = 0; r < 3 && !rc; ++r) {
        hipEventRecord(e0, s);
        rc = launch_eval(d, table, n_pts, pos, v, grad, lap, 0, tile, s);
        hipEventRecord(e1, s);
        if (!rc) rc = hip_fail(hipEventSynchronize(e1), "hipEventSynchronize");
        if (!rc) rc = hip_fail(hipEventElapsedTime(&times[r], e0, e1), "hipEventElapsedTime");
      }
      if (rc) break;
      float lo = times[0] < times[1] ? times[0] : times[1];
      float hi = times[0] < times[1] ? times[1] : times[0];
      const float med = times[2] < lo ? lo : (times[2] > hi ? hi : times[2]);
      if (med < best) { best = med; best_tile[0] = g; best_tile[1] = opl; }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    tune_store_locked(tune_key(d), best_tile[0], best_tile[1]);
  }
  tile_out[0] = best_tile[0];
  tile_out[1] = best_tile[1];
  // leave valid outputs computed with the chosen tile
  if ((rc = launch_eval(d, table, n_pts, pos, v, grad, lap, 0, best_tile, s))) return rc;
  return hip_fail(hipStreamSynchronize(s), "hipStreamSynchronize");
}

int spline_sorted_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (!bytes) return fail(SPL_EINVAL, "bytes is NULL");
  if (n_pts < 0 || n_pts > 0x7fffffffLL) return fail(SPL_EINVAL, "n_pts = %lld outside [0, 2^31)", (long long)n_pts);
  *bytes = 0;
  return n_pts == 0 ? SPL_OK : sorted_eval_work_bytes(d, n_pts, bytes);
}

int spline_eval_vgl_sorted(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v,
                           void* grad, void* lap, const int32_t* tile, void* work, int64_t work_bytes, void* stream) {
  clear_error();
  int rc = check_eval_args(d, table, n_pts, pos);
  if (rc) return rc;
  if (n_pts == 0) return SPL_OK;
  if ((rc = check_vgl_outputs(d, v, grad, lap))) return rc;
  if (!work) return fail(SPL_EINVAL, "work is NULL (size from spline_sorted_work_bytes)");
  if (!aligned(work, 256)) return fail(SPL_EINVAL, "workspace must be 256-byte aligned");
  int32_t t[2];
  if (tile) {
    t[0] = tile[0];
    t[1] = tile[1];
  } else {
    tile_for(d, t);
  }
  if (!tile_valid_for(d, t)) return fail(SPL_EINVAL, "invalid tile");
  return launch_eval_sorted(d, table, n_pts, pos, v, grad, lap, 0, t, work, work_bytes,
                            static_cast<hipStream_t>(stream));
}

int spline_backward_work_bytes(const spl_desc* d, int64_t n_pts, int32_t flags, int64_t* bytes) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (!bytes) return fail(SPL_EINVAL, "bytes is NULL");
  if (n_pts < 0 || n_pts > 0x7fffffffLL) return fail(SPL_EINVAL, "n_pts = %lld outside [0, 2^31)", (long long)n_pts);
  if (flags & ~(SPL_DETERMINISTIC | SPL_REUSE_SORT)) return fail(SPL_EINVAL, "unknown flags 0x%x", flags);
  if (d->basis != SPL_BSPLINE || d->sep_grad || d->bloch)
    return fail(SPL_EUNSUPPORTED, "the adjoint covers real B-spline tables without separate gradients");
  *bytes = 0;
  if (!(flags & SPL_DETERMINISTIC) || n_pts == 0) return SPL_OK;
  return sorted_work_bytes(d, n_pts, bytes);
}

int spline_cells_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (!bytes || n_pts < 0 || n_pts > 0x7fffffffLL) return fail(SPL_EINVAL, "bytes is NULL or n_pts out of range");
  if (n_pts == 0) {
    *bytes = 0;
    return SPL_OK;
  }
  return cells_eval_work_bytes(d, n_pts, bytes);
}

int spline_eval_vgl_cells(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v,
                          void* grad, void* lap, int32_t flags, void* work, int64_t work_bytes, void* stream) {
  clear_error();
  int rc = check_eval_args(d, table, n_pts, pos);
  if (rc) return rc;
  if (flags & ~SPL_REUSE_SORT) return fail(SPL_EINVAL, "unknown flags 0x%x", flags);
  if (d->basis != SPL_BSPLINE || d->sep_grad || d->bloch)
    return fail(SPL_EUNSUPPORTED, "the cell-wise evaluation covers real B-spline tables without separate gradients");
  if (n_pts == 0) return SPL_OK;
  if (!v && !grad && !lap) return fail(SPL_EINVAL, "no output requested");
  for (const void* o : {static_cast<const void*>(v), static_cast<const void*>(grad), static_cast<const void*>(lap)})
    if (o && !out_align_ok(d, o)) return fail(SPL_EINVAL, "output not aligned to its element size");
  if (!work) return fail(SPL_EINVAL, "work is NULL (size from spline_cells_work_bytes)");
  if (!aligned(work, 256)) return fail(SPL_EINVAL, "workspace must be 256-byte aligned");
  return launch_eval_cells(d, table, n_pts, pos, v, grad, lap, work, work_bytes, (flags & SPL_REUSE_SORT) != 0,
                           static_cast<hipStream_t>(stream), nullptr);
}

int spline_fit_terms_cells(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, const void* t_v,
                           double w_v, void* g_v, const void* t_lap, double w_lap, void* g_lap, double* loss,
                           int32_t flags, void* work, int64_t work_bytes, void* stream) {
  clear_error();
  int rc = check_eval_args(d, table, n_pts, pos);
  if (rc) return rc;
  if (flags & ~SPL_REUSE_SORT) return fail(SPL_EINVAL, "unknown flags 0x%x", flags);
  if (d->basis != SPL_BSPLINE || d->sep_grad || d->bloch)
    return fail(SPL_EUNSUPPORTED, "the fit terms cover real B-spline tables without separate gradients");
  if (!isfinite(w_v) || !isfinite(w_lap)) return fail(SPL_EINVAL, "weight is not finite");
  if (!t_v != !g_v || !t_lap != !g_lap) return fail(SPL_EINVAL, "a term needs both its target and its gradient");
  if (!t_v && !t_lap) return fail(SPL_EINVAL, "no term requested");
  if (n_pts == 0) return SPL_OK;
  for (const void* o : {t_v, static_cast<const void*>(g_v), t_lap, static_cast<const void*>(g_lap)})
    if (o && !out_align_ok(d, o)) return fail(SPL_EINVAL, "target or gradient not aligned to its element size");
  if (!loss || (uintptr_t)loss % 8) return fail(SPL_EINVAL, "loss is NULL or not 8-byte aligned");
  if (!work) return fail(SPL_EINVAL, "work is NULL (size from spline_cells_work_bytes)");
  if (!aligned(work, 256)) return fail(SPL_EINVAL, "workspace must be 256-byte aligned");
  FitTerms fit{t_v, w_v, t_lap, w_lap, loss};
  return launch_eval_cells(d, table, n_pts, pos, g_v, nullptr, g_lap, work, work_bytes,
                           (flags & SPL_REUSE_SORT) != 0, static_cast<hipStream_t>(stream), &fit);
}

int spline_fit_gradient_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (!bytes || n_pts < 0 || n_pts > 0x7fffffffLL) return fail(SPL_EINVAL, "bytes is NULL or n_pts out of range");
  if (n_pts == 0) {
    *bytes = 0;
    return SPL_OK;
  }
  return fit_gradient_work_bytes(d, n_pts, bytes);
}

int spline_fit_gradient_cells(const spl_desc* d, const void* table, int64_t n_pts, const double* pos,
                              const void* t_v, double w_v, const void* t_lap, double w_lap, void* gtable,
                              double* loss, int32_t flags, void* work, int64_t work_bytes, void* stream) {
  clear_error();
  int rc = check_eval_args(d, table, n_pts, pos);
  if (rc) return rc;
  if (flags & ~SPL_REUSE_SORT) return fail(SPL_EINVAL, "unknown flags 0x%x", flags);
  if (d->basis != SPL_BSPLINE || d->sep_grad || d->bloch)
    return fail(SPL_EUNSUPPORTED, "the fit gradient covers real B-spline tables without separate gradients");
  if (!isfinite(w_v) || !isfinite(w_lap)) return fail(SPL_EINVAL, "weight is not finite");
  if (!t_v || !t_lap) return fail(SPL_EINVAL, "the one-pass fit gradient needs both targets");
  if (n_pts == 0) return SPL_OK;
  for (const void* o : {t_v, t_lap})
    if (!out_align_ok(d, o)) return fail(SPL_EINVAL, "target not aligned to its element size");
  if (!gtable || !aligned(gtable, d->dtype == SPL_F64 ? 8 : 4)) return fail(SPL_EINVAL, "gtable is NULL or misaligned");
  if (!loss || (uintptr_t)loss % 8) return fail(SPL_EINVAL, "loss is NULL or not 8-byte aligned");
  if (!work) return fail(SPL_EINVAL, "work is NULL (size from spline_fit_gradient_work_bytes)");
  if (!aligned(work, 256)) return fail(SPL_EINVAL, "workspace must be 256-byte aligned");
  return launch_fit_gradient(d, table, n_pts, pos, t_v, w_v, t_lap, w_lap, gtable, loss, work, work_bytes,
                             (flags & SPL_REUSE_SORT) != 0, static_cast<hipStream_t>(stream));
}

int spline_eval_vgl_backward(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, const void* gv,
                             const void* ggrad, const void* glap, void* gtable, double* gpos, int32_t flags,
                             void* work, int64_t work_bytes, void* stream) {
  clear_error();
  int rc = check_eval_args(d, table, n_pts, pos);
  if (rc) return rc;
  if (flags & ~(SPL_DETERMINISTIC | SPL_REUSE_SORT)) return fail(SPL_EINVAL, "unknown flags 0x%x", flags);
  if ((flags & SPL_REUSE_SORT) && !(flags & SPL_DETERMINISTIC))
    return fail(SPL_EINVAL, "SPL_REUSE_SORT needs SPL_DETERMINISTIC");
  if (d->basis != SPL_BSPLINE || d->sep_grad || d->bloch)
    return fail(SPL_EUNSUPPORTED, "the adjoint covers real B-spline tables without separate gradients");
  if (n_pts == 0) return SPL_OK;
  if (gtable && !aligned(gtable, d->dtype == SPL_F64 ? 8 : 4)) return fail(SPL_EINVAL, "gtable misaligned");
  if (gpos && !aligned(gpos, 8)) return fail(SPL_EINVAL, "gpos misaligned");
  for (const void* g : {gv, ggrad, glap})
    if (g && !out_align_ok(d, g)) return fail(SPL_EINVAL, "upstream gradient misaligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!(flags & SPL_DETERMINISTIC))
    return launch_backward(d, table, n_pts, pos, gv, ggrad, glap, gtable, gpos, s);
  if (gtable) {
    if (!work) return fail(SPL_EINVAL, "SPL_DETERMINISTIC needs a workspace (spline_backward_work_bytes)");
    if (!aligned(work, 256)) return fail(SPL_EINVAL, "workspace must be 256-byte aligned");
    if ((rc = launch_backward_sorted(d, n_pts, pos, gv, ggrad, glap, gtable, work, work_bytes,
                                     (flags & SPL_REUSE_SORT) != 0, s)))
      return rc;
  }
  // the position gradient is deterministic as computed (fixed-order reduction per point)
  return gpos ? launch_backward(d, table, n_pts, pos, gv, ggrad, glap, nullptr, gpos, s) : SPL_OK;
}

}  // extern "C"
