// Host build of the coordinate reduction and block indexing that every forward and adjoint
// kernel runs per point (reduce_point, wrap4 in csrc/common.hpp), for a CPU check over
// adversarial positions.  The geometry comes from the library itself (spline_desc_init,
// pws::make_geom).
//
// stdin:  lattice (9 doubles, rows a_i) grid (3 ints) o_pad_min (int) pp (0/1) n_pts
//         then n_pts lines of 3 positions written as C99 hex floats
// stdout: per point "ok i0 i1 i2 t0 t1 t2 rows_in_range" (t as hex floats)
// rows_in_range is 1 when all 64 row offsets of the point's block (16 runs of 4 rows; for a
// pp-spline table the 2x2x2 corners and their 8 numbers) lie inside the table.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "common.hpp"

int main() {
  spl_desc d;
  memset(&d, 0, sizeof d);
  int pp = 0, opad_min = 0;
  long n_pts = 0;
  for (int i = 0; i < 9; ++i)
    if (scanf("%la", &d.lattice[i]) != 1) return 2;
  if (scanf("%d %d %d %d %d %ld", &d.grid[0], &d.grid[1], &d.grid[2], &opad_min, &pp, &n_pts) != 6) return 2;
  d.n_orb = opad_min;
  d.dtype = SPL_F64;
  d.basis = pp ? SPL_PPSPLINE : SPL_BSPLINE;
  if (spline_desc_init(&d) != SPL_OK) {
    fprintf(stderr, "desc: %s\n", spline_last_error());
    return 3;
  }
  const pws::Geom g = pws::make_geom(&d);
  const int64_t rows_total = (int64_t)g.n[0] * g.s0;          // elements of one table
  for (long p = 0; p < n_pts; ++p) {
    double r[3];
    if (scanf("%la %la %la", &r[0], &r[1], &r[2]) != 3) return 2;
    int i0[3] = {-7, -7, -7};
    double t[3] = {-1.0, -1.0, -1.0};
    const bool ok = pws::reduce_point(g, r[0], r[1], r[2], i0, t);
    int ix[4], iy[4], iz[4];
    pws::wrap4(i0[0], g.n[0], ix);
    pws::wrap4(i0[1], g.n[1], iy);
    pws::wrap4(i0[2], g.n[2], iz);
    bool in_range = true;
    const int64_t op = g.o_pad;
    for (int l = 0; l < 4; ++l)
      for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) {
          int64_t off;
          if (pp) {
            // corner (i0 + (l >> 1)) on each axis, number 4 (l & 1) + 2 (m & 1) + (n & 1)
            off = (int64_t)ix[1 + (l >> 1)] * g.s0 + (int64_t)iy[1 + (m >> 1)] * g.s1 +
                  (int64_t)iz[1 + (n >> 1)] * 8 * op + (4 * (l & 1) + 2 * (m & 1) + (n & 1)) * op;
          } else {
            off = (int64_t)ix[l] * g.s0 + (int64_t)iy[m] * g.s1 + (int64_t)iz[n] * op;
          }
          if (off < 0 || off + op > rows_total) in_range = false;
        }
    printf("%d %d %d %d %a %a %a %d\n", ok ? 1 : 0, i0[0], i0[1], i0[2], t[0], t[1], t[2], in_range ? 1 : 0);
  }
  return 0;
}
