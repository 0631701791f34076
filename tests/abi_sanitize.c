/* Host-side driver for the C ABI's argument validation, built against a library whose
 * validation units carry AddressSanitizer and UndefinedBehaviorSanitizer instrumentation.
 * Every call here is rejected (or is a no-op) before anything reaches a GPU, so it runs on a
 * machine without one.  Exit status 0: every return code was as documented and no sanitizer
 * report fired (reports abort the process). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "pwspline.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
  if (got != want) {
    fprintf(stderr, "%s: returned %d, expected %d (%s)\n", what, got, want, spline_last_error());
    ++failures;
  }
  /* the message is always a valid, terminated string */
  if (strlen(spline_last_error()) > 4096) {
    fprintf(stderr, "%s: oversized error message\n", what);
    ++failures;
  }
}

static spl_desc make(int n1, int n2, int n3, int n_orb, int dtype, int has_lap) {
  spl_desc d;
  memset(&d, 0, sizeof d);
  const double lat[9] = {7.0, 0.4, -0.3, 1.1, 6.2, 0.5, -0.6, 0.9, 8.3};
  memcpy(d.lattice, lat, sizeof lat);
  d.grid[0] = n1;
  d.grid[1] = n2;
  d.grid[2] = n3;
  d.n_orb = n_orb;
  d.dtype = dtype;
  d.has_lap = has_lap;
  return d;
}

int main(void) {
  void* fake = (void*)(uintptr_t)4096; /* never dereferenced: validation fails first */
  const double* fpos = (const double*)fake;
  int32_t tile[2];
  int64_t bytes = 0;

  /* descriptors: the valid ones of every representation, then every rejected field */
  spl_desc d = make(8, 8, 8, 5, SPL_F64, 0);
  expect(spline_desc_init(&d), SPL_OK, "desc f64");
  spl_desc d32 = make(9, 10, 11, 37, SPL_F32, 1);
  expect(spline_desc_init(&d32), SPL_OK, "desc f32 lap");
  spl_desc dbf = make(12, 12, 12, 130, SPL_BF16, 0);
  expect(spline_desc_init(&dbf), SPL_OK, "desc bf16");
  spl_desc dl = make(8, 8, 8, 4, SPL_F32, 1);
  dl.basis = SPL_LAGRANGE;
  dl.sep_grad = 1;
  expect(spline_desc_init(&dl), SPL_OK, "desc lagrange");
  spl_desc dp = make(8, 8, 8, 4, SPL_F64, 0);
  dp.basis = SPL_PPSPLINE;
  expect(spline_desc_init(&dp), SPL_OK, "desc pp");
  spl_desc db = make(8, 8, 8, 3, SPL_F32, 0);
  db.bloch = 1;
  db.kvec[0] = 0.3;
  expect(spline_desc_init(&db), SPL_OK, "desc bloch");
  spl_desc big = make(1024, 1024, 1024, 1, SPL_BF16, 0);
  expect(spline_desc_init(&big), SPL_OK, "desc largest grid");

  expect(spline_desc_init(NULL), SPL_EINVAL, "desc NULL");
  spl_desc bad = make(3, 8, 8, 5, SPL_F64, 0);
  expect(spline_desc_init(&bad), SPL_EGRID, "desc N < 4");
  bad = make(8, 8, 1025, 5, SPL_F64, 0);
  expect(spline_desc_init(&bad), SPL_EGRID, "desc N > 1024");
  bad = make(8, 8, 8, 0, SPL_F64, 0);
  expect(spline_desc_init(&bad), SPL_EINVAL, "desc n_orb 0");
  bad = make(8, 8, 8, 5, 7, 0);
  expect(spline_desc_init(&bad), SPL_EDTYPE, "desc dtype");
  bad = make(8, 8, 8, 5, SPL_F64, 0);
  memset(bad.lattice, 0, sizeof bad.lattice);
  expect(spline_desc_init(&bad), SPL_EINVAL, "desc singular lattice");
  bad = make(8, 8, 8, 5, SPL_F64, 0);
  bad.lattice[4] = NAN;
  expect(spline_desc_init(&bad), SPL_EINVAL, "desc NaN lattice");
  bad = make(8, 8, 8, 5, SPL_F64, 0);
  bad.reserved = 1;
  expect(spline_desc_init(&bad), SPL_EINVAL, "desc reserved");
  bad = make(8, 8, 8, 5, SPL_F64, 0);
  bad.kvec[1] = 0.5;
  expect(spline_desc_init(&bad), SPL_EINVAL, "desc k without bloch");
  bad = make(8, 8, 8, 5, SPL_F64, 0);
  bad.basis = SPL_LAGRANGE;
  expect(spline_desc_init(&bad), SPL_EINVAL, "desc lagrange without separate tables");
  bad = make(8, 8, 8, 5, SPL_F64, 0);
  bad.basis = 3;
  expect(spline_desc_init(&bad), SPL_EINVAL, "desc basis");

  /* a descriptor changed after init is refused everywhere */
  spl_desc moved = d;
  moved.grid[0] = 9;
  expect(spline_eval_vgl(&moved, fake, 10, fpos, fake, fake, fake, NULL), SPL_EINVAL, "modified desc");

  /* evaluation */
  expect(spline_eval_vgl(&d, NULL, 10, fpos, fake, fake, fake, NULL), SPL_EINVAL, "eval NULL table");
  expect(spline_eval_vgl(&d, fake, 10, NULL, fake, fake, fake, NULL), SPL_EINVAL, "eval NULL pos");
  expect(spline_eval_vgl(&d, fake, 10, fpos, NULL, fake, fake, NULL), SPL_EINVAL, "eval NULL v");
  expect(spline_eval_vgl(&d, fake, -1, fpos, fake, fake, fake, NULL), SPL_EINVAL, "eval n < 0");
  expect(spline_eval_vgl(&d, fake, (int64_t)1 << 31, fpos, fake, fake, fake, NULL), SPL_EINVAL, "eval n too large");
  expect(spline_eval_vgl(&d, (void*)((char*)fake + 8), 10, fpos, fake, fake, fake, NULL), SPL_EINVAL,
         "eval misaligned table");
  expect(spline_eval_vgl(&d, NULL, 0, NULL, NULL, NULL, NULL, NULL), SPL_OK, "eval n == 0");
  expect(spline_eval_v(&d, fake, 10, fpos, NULL, NULL), SPL_EINVAL, "eval_v NULL v");
  tile[0] = 3;
  tile[1] = 1;
  expect(spline_eval_vgl_tile(&d, fake, 10, fpos, fake, fake, fake, tile, NULL), SPL_EINVAL, "tile lanes");
  tile[0] = 64;
  tile[1] = 3;
  expect(spline_eval_vgl_tile(&d, fake, 10, fpos, fake, fake, fake, tile, NULL), SPL_EINVAL, "tile orbitals");
  tile[0] = 8;
  tile[1] = 1;
  expect(spline_eval_vgl_tile(&db, fake, 10, fpos, fake, fake, fake, tile, NULL), SPL_EINVAL, "bloch odd tile");
  expect(spline_tile_for(&d32, 1000, tile), SPL_OK, "tile_for");
  expect(spline_tile_for(&d32, 1000, NULL), SPL_EINVAL, "tile_for NULL");

  /* sorted evaluation */
  expect(spline_eval_vgl_sorted(&d, fake, 10, fpos, fake, fake, fake, NULL, NULL, 0, NULL), SPL_EINVAL,
         "sorted NULL work");
  expect(spline_eval_vgl_sorted(&d, fake, 10, fpos, fake, fake, fake, NULL, (char*)fake + 8, 1 << 20, NULL),
         SPL_EINVAL, "sorted misaligned work");
  expect(spline_eval_vgl_sorted(&d, NULL, 0, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL), SPL_OK, "sorted n == 0");
  expect(spline_sorted_work_bytes(&d, 0, &bytes), SPL_OK, "sorted work bytes");

  /* cell-wise forward */
  expect(spline_cells_work_bytes(&d, 0, &bytes), SPL_OK, "cells work bytes");
  expect(spline_eval_vgl_cells(&d, fake, 10, fpos, NULL, NULL, NULL, 0, fake, 1 << 20, NULL), SPL_EINVAL,
         "cells no output");
  expect(spline_eval_vgl_cells(&d, fake, 10, fpos, fake, NULL, NULL, 0, NULL, 0, NULL), SPL_EINVAL, "cells NULL work");
  expect(spline_eval_vgl_cells(&dp, fake, 10, fpos, fake, NULL, NULL, 0, fake, 1 << 20, NULL), SPL_EUNSUPPORTED,
         "cells pp");
  expect(spline_eval_vgl_cells(&d, fake, 10, fpos, fake, NULL, NULL, 5, fake, 1 << 20, NULL), SPL_EINVAL,
         "cells flags");
  expect(spline_eval_vgl_backward(&d, fake, 10, fpos, NULL, NULL, NULL, fake, NULL, SPL_REUSE_SORT, fake, 1 << 20,
                                  NULL), SPL_EINVAL, "reuse without deterministic");

  /* fit terms from the cell-wise forward */
  expect(spline_fit_terms_cells(&d, fake, 10, fpos, fake, 1.0, NULL, NULL, 0.0, NULL, fake, 0, fake, 1 << 20, NULL),
         SPL_EINVAL, "fit terms target without gradient");
  expect(spline_fit_terms_cells(&d, fake, 10, fpos, NULL, 1.0, NULL, NULL, 0.0, NULL, fake, 0, fake, 1 << 20, NULL),
         SPL_EINVAL, "fit terms no term");
  expect(spline_fit_terms_cells(&d, fake, 10, fpos, fake, 1.0, fake, NULL, 0.0, NULL, NULL, 0, fake, 1 << 20, NULL),
         SPL_EINVAL, "fit terms NULL loss");
  expect(spline_fit_terms_cells(&d, fake, 10, fpos, fake, 1.0, fake, NULL, 0.0, NULL, fake, 0, NULL, 0, NULL),
         SPL_EINVAL, "fit terms NULL work");
  expect(spline_fit_terms_cells(&dp, fake, 10, fpos, fake, 1.0, fake, NULL, 0.0, NULL, fake, 0, fake, 1 << 20, NULL),
         SPL_EUNSUPPORTED, "fit terms pp");
  expect(spline_fit_terms_cells(&d, fake, 0, fpos, fake, 1.0, fake, NULL, 0.0, NULL, fake, 0, NULL, 0, NULL), SPL_OK,
         "fit terms n == 0");

  /* the fit's data terms and their gradient in one pass */
  expect(spline_fit_gradient_work_bytes(&d, 0, &bytes), SPL_OK, "fit gradient work bytes");
  expect(spline_fit_gradient_work_bytes(&d, 10, NULL), SPL_EINVAL, "fit gradient work bytes NULL");
  expect(spline_fit_gradient_cells(&d, fake, 10, fpos, NULL, 1.0, fake, 1.0, fake, fake, 0, fake, 1 << 20, NULL),
         SPL_EINVAL, "fit gradient without value target");
  expect(spline_fit_gradient_cells(&d, fake, 10, fpos, fake, 1.0, fake, 1.0, NULL, fake, 0, fake, 1 << 20, NULL),
         SPL_EINVAL, "fit gradient NULL gtable");
  expect(spline_fit_gradient_cells(&d, fake, 10, fpos, fake, 1.0, fake, 1.0, fake, NULL, 0, fake, 1 << 20, NULL),
         SPL_EINVAL, "fit gradient NULL loss");
  expect(spline_fit_gradient_cells(&d, fake, 10, fpos, fake, 1.0, fake, 1.0, fake, fake, 0, NULL, 0, NULL),
         SPL_EINVAL, "fit gradient NULL work");
  expect(spline_fit_gradient_cells(&d, fake, 10, fpos, fake, 0.0 / 0.0, fake, 1.0, fake, fake, 0, fake, 1 << 20,
                                   NULL), SPL_EINVAL, "fit gradient NaN weight");
  expect(spline_fit_gradient_cells(&d, fake, 10, fpos, fake, 1.0, fake, 1.0, fake, fake, 4, fake, 1 << 20, NULL),
         SPL_EINVAL, "fit gradient unknown flag");
  expect(spline_fit_gradient_cells(&dp, fake, 10, fpos, fake, 1.0, fake, 1.0, fake, fake, 0, fake, 1 << 20, NULL),
         SPL_EUNSUPPORTED, "fit gradient pp");
  expect(spline_fit_gradient_cells(&d, fake, 0, fpos, fake, 1.0, fake, 1.0, fake, fake, 0, NULL, 0, NULL), SPL_OK,
         "fit gradient n == 0");

  /* the element-wise Adam step */
  expect(spline_adam_step(SPL_F32, 0, NULL, NULL, NULL, NULL, 0.1, 0.9, 0.999, 1e-8, 1, NULL), SPL_OK, "adam n == 0");
  expect(spline_adam_step(7, 10, fake, fake, fake, fake, 0.1, 0.9, 0.999, 1e-8, 1, NULL), SPL_EDTYPE, "adam dtype");
  expect(spline_adam_step(SPL_F32, -1, fake, fake, fake, fake, 0.1, 0.9, 0.999, 1e-8, 1, NULL), SPL_EINVAL,
         "adam n < 0");
  expect(spline_adam_step(SPL_F32, 10, fake, NULL, fake, fake, 0.1, 0.9, 0.999, 1e-8, 1, NULL), SPL_EINVAL,
         "adam NULL grad");
  expect(spline_adam_step(SPL_F64, 10, (char*)fake + 4, fake, fake, fake, 0.1, 0.9, 0.999, 1e-8, 1, NULL), SPL_EINVAL,
         "adam misaligned param");
  expect(spline_adam_step(SPL_F32, 10, fake, fake, fake, fake, 0.1, -0.1, 0.999, 1e-8, 1, NULL), SPL_EINVAL,
         "adam negative beta1");
  expect(spline_adam_step(SPL_F32, 10, fake, fake, fake, fake, 0.1, 0.9, 0.999, 1e-8, 0, NULL), SPL_EINVAL,
         "adam step 0");

  /* build */
  expect(spline_build(&d, fake, fake, fake, fake, NULL), SPL_EINVAL, "build lap values without lap table");
  expect(spline_build(&d32, fake, NULL, fake, fake, NULL), SPL_EINVAL, "build lap table without values");
  expect(spline_build(&d, NULL, NULL, fake, fake, NULL), SPL_EINVAL, "build NULL values");
  expect(spline_build(&dl, fake, NULL, fake, fake, NULL), SPL_EINVAL, "build lagrange");
  expect(spline_build_tables(&d, NULL, fake, fake, NULL), SPL_EINVAL, "build_tables NULL values");
  expect(spline_smoothing_work_bytes(&d, &bytes), SPL_OK, "smoothing work bytes");
  expect(spline_build_smoothing(&dl, 4, fake, fake, fake, fake, NULL), SPL_EINVAL, "smoothing lagrange");
  expect(spline_build_smoothing(&d, -1, fake, fake, fake, fake, NULL), SPL_EINVAL, "smoothing n_g < 0");

  /* adjoint */
  expect(spline_eval_vgl_backward(&d, fake, 10, fpos, NULL, NULL, NULL, fake, NULL, 8, NULL, 0, NULL), SPL_EINVAL,
         "backward flags");
  expect(spline_eval_vgl_backward(&d, fake, 10, fpos, NULL, NULL, NULL, fake, NULL, SPL_DETERMINISTIC, NULL, 0, NULL),
         SPL_EINVAL, "backward workspace");
  expect(spline_eval_vgl_backward(&dp, fake, 10, fpos, NULL, NULL, NULL, fake, NULL, 0, NULL, 0, NULL),
         SPL_EUNSUPPORTED, "backward pp");
  expect(spline_backward_work_bytes(&d, 10, 0, &bytes), SPL_OK, "backward work bytes");
  expect(spline_backward_work_bytes(&d, 10, 4, &bytes), SPL_EINVAL, "backward work bytes flags");

  /* misfit */
  expect(spline_misfit_work_bytes(&d32, 100, &bytes), SPL_OK, "misfit work bytes");
  expect(spline_misfit(&d32, 0, NULL, NULL, 1.0, NULL, NULL, NULL, 0, NULL), SPL_OK, "misfit n == 0");
  expect(spline_misfit(&d32, 10, fake, fake, NAN, fake, (double*)fake, fake, bytes, NULL), SPL_EINVAL, "misfit NaN w");
  expect(spline_misfit(&d32, 10, fake, NULL, 1.0, fake, (double*)fake, fake, bytes, NULL), SPL_EINVAL, "misfit NULL t");
  expect(spline_misfit(&d32, 10, fake, fake, 1.0, fake, (double*)fake, fake, bytes - 8, NULL), SPL_EINVAL,
         "misfit short work");
  expect(spline_misfit(&d, 10, (char*)fake + 4, fake, 1.0, fake, (double*)fake, fake, bytes, NULL), SPL_EINVAL,
         "misfit misaligned");

  /* smoothness penalty */
  expect(spline_smoothness_penalty(&d32, fake, 1.0, NULL, (double*)fake, fake, bytes, NULL), SPL_EINVAL,
         "penalty NULL gtable");
  expect(spline_smoothness_penalty(&d32, fake, INFINITY, fake, (double*)fake, fake, bytes, NULL), SPL_EINVAL,
         "penalty inf w");
  expect(spline_smoothness_penalty(&dp, fake, 1.0, fake, (double*)fake, fake, bytes, NULL), SPL_EUNSUPPORTED,
         "penalty pp");

  /* batched plans */
  void* plan = fake;
  expect(spline_batch_plan_create(NULL, 1, NULL, NULL, &plan), SPL_EINVAL, "plan NULL items");
  spl_item item;
  memset(&item, 0, sizeof item);
  item.d = &dp;
  item.table = fake;
  item.n_pts = 4;
  item.pos = fpos;
  item.v = item.grad = item.lap = fake;
  expect(spline_batch_plan_create(&item, 1, NULL, NULL, &plan), SPL_EUNSUPPORTED, "plan pp item");
  expect(spline_batch_plan_sort(NULL, 1, NULL), SPL_EINVAL, "plan sort NULL");
  expect(spline_batch_plan_get_tiles(NULL, tile), SPL_EINVAL, "plan get tiles NULL");
  expect(spline_batch_plan_set_tiles(NULL, tile, NULL), SPL_EINVAL, "plan set tiles NULL");

  /* the sorted evaluation without allocation: rejected arguments, and no points (a no-op) */
  expect(spline_eval_vgl_sorted_noalloc(NULL, fake, 4, fpos, fake, fake, fake, NULL, NULL), SPL_EINVAL,
         "noalloc NULL desc");
  expect(spline_eval_vgl_sorted_noalloc(&d, NULL, 4, fpos, fake, fake, fake, NULL, NULL), SPL_EINVAL,
         "noalloc NULL table");
  expect(spline_eval_vgl_sorted_noalloc(&d, fake, -1, fpos, fake, fake, fake, NULL, NULL), SPL_EINVAL,
         "noalloc negative n_pts");
  expect(spline_eval_vgl_sorted_noalloc(&d, fake, 4, fpos, NULL, fake, fake, NULL, NULL), SPL_EINVAL,
         "noalloc NULL output");
  expect(spline_eval_vgl_sorted_noalloc(&d, fake, 0, fpos, fake, fake, fake, NULL, NULL), SPL_OK, "noalloc no points");

  /* read-rate probe */
  expect(spline_stream_read(NULL, 16, fake, NULL), SPL_EINVAL, "stream NULL buf");
  expect(spline_stream_read(fake, 16, NULL, NULL), SPL_EINVAL, "stream NULL sink");
  expect(spline_stream_read(fake, 15, fake, NULL), SPL_EINVAL, "stream size not a multiple of 16");
  expect(spline_stream_read(fake, -16, fake, NULL), SPL_EINVAL, "stream negative size");
  expect(spline_stream_read((const void*)(uintptr_t)4104, 16, fake, NULL), SPL_EINVAL, "stream misaligned buf");
  expect(spline_stream_read(fake, 16, (void*)(uintptr_t)4098, NULL), SPL_EINVAL, "stream misaligned sink");
  expect(spline_stream_read(NULL, 0, NULL, NULL), SPL_OK, "stream zero bytes");

  if (spline_version() <= 0) {
    fprintf(stderr, "version\n");
    ++failures;
  }
  if (failures) {
    fprintf(stderr, "%d unexpected results\n", failures);
    return 1;
  }
  printf("all validation paths returned as documented\n");
  return 0;
}
