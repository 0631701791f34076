/*
 * pwspline.h -- periodic tricubic B-spline orbitals on AMD Instinct MI355X (gfx950).
 *
 * The method: single-particle orbitals given as planewave sums are replaced by
 * cubic B-splines on a uniform periodic real-space grid (Parker, Umrigar, Alfe,
 * Hennig, Wilkins, "Comparison of polynomial approximations to speed up
 * planewave-based quantum Monte Carlo calculations", arXiv:1309.6250).  Every
 * evaluation of an orbital, its gradient and its Laplacian at a point reads the
 * 4x4x4 block of coefficients around the point (Sec. III B) and contracts it
 * with tensor-product basis weights (App. A, Eq. b-splineapproximation); the
 * Cartesian derivatives follow from the chain rule through the reduced
 * coordinates (Sec. II, Eq. reducedcoordinate and the Coordinates paragraph).
 *
 * Conventions used by every entry point
 *   - Pointers named "device" are HIP device pointers; everything else is host.
 *     The caller owns every buffer.  No entry point below allocates device
 *     memory except spline_batch_plan_create and spline_autotune (documented).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *     enqueued asynchronously on it; nothing synchronizes with the host unless
 *     stated.  Faults inside a kernel surface at the caller's next synchronize.
 *   - Return values: SPL_OK (0) or a negative SPL_E* code.  All argument checks
 *     happen before anything is enqueued; on failure nothing is enqueued and
 *     spline_last_error() describes the problem (thread-local, never NULL).
 *     No entry point aborts or throws.
 *   - Lattice: lattice[3*i + c] is Cartesian component c (bohr) of lattice vector
 *     a_i, i.e. ROWS are lattice vectors.  The paper's matrix a has them as
 *     columns, so crystal coordinates are s = a^-1 r with a = lattice^T.
 *   - Coefficient table layout: [N1][N2][N3][o_pad], orbital index innermost and
 *     zero-padded to o_pad, in the storage dtype.  With has_lap, a second table of
 *     the same shape (the separate Laplacian spline) follows the first; with
 *     sep_grad, five tables follow one another (see spl_desc).
 *   - Representations (App. A): cubic B-splines (default) or cubic Lagrange
 *     interpolation of grid values; the gradient and the Laplacian are either
 *     derivatives of the orbital's interpolant or interpolants of their own grid
 *     values (the paper's "separate" or direct approximations, Sec. III A, Fig. 1).
 *   - Bloch orbitals (Sec. I): phi(r) = exp(i k.r) u(r) with u periodic and complex.
 *     Each orbital occupies two adjacent real columns (Re u, Im u) of every table,
 *     and every output is complex, stored as (re, im) pairs: v [n_pts][n_orb][2],
 *     grad [n_pts][3][n_orb][2], lap [n_pts][n_orb][2].  The phase uses the
 *     unfolded Cartesian position.
 *   - Basis normalization: the standard cubic B-spline (values 1/6, 2/3, 1/6 at
 *     the knots; the 64 weights of a point sum to 1).  The paper's basis is this
 *     one times 3/2 per axis (its constant C = 3/2, App. A); the spline function
 *     is identical, stored coefficients differ by the factor (3/2)^3.
 *   - Positions are FP64 Cartesian [n_pts][3], anywhere in R^3 (folded into the
 *     cell).  A point with a non-finite coordinate yields NaN outputs.
 *   - Outputs are FP64 for SPL_F64 tables and FP32 for SPL_F32 / SPL_BF16 tables
 *     (whose arithmetic is FP32; reduced coordinates are always FP64).
 */
#ifndef PWSPLINE_H
#define PWSPLINE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* storage dtype of coefficient tables */
enum { SPL_F64 = 0, SPL_F32 = 1, SPL_BF16 = 2 };

/* status codes */
enum {
  SPL_OK = 0,
  SPL_EINVAL = -1,       /* bad argument: NULL required pointer, n_orb < 1, n_pts < 0, singular lattice ... */
  SPL_EGRID = -2,        /* grid size outside [4, 1024] on some axis */
  SPL_EDTYPE = -3,       /* unknown dtype */
  SPL_ENOMEM = -4,       /* a library-owned allocation failed (batch plans, autotuning only) */
  SPL_EHIP = -5,         /* a HIP runtime call or launch failed; message holds the HIP error string */
  SPL_EUNSUPPORTED = -6  /* valid request that this build does not implement */
};

/* flags of spline_eval_vgl_backward (and SPL_REUSE_SORT of spline_eval_vgl_cells) */
enum {
  SPL_DETERMINISTIC = 1,  /* cell-sorted, bitwise-reproducible coefficient gradient */
  SPL_REUSE_SORT = 2      /* the workspace already holds the cell sort of these same points (same
                             descriptor, n_pts and pos), made by an earlier spline_eval_vgl_cells or
                             deterministic spline_eval_vgl_backward call: skip sorting.  A workspace
                             that holds something else gives wrong results, never an access outside
                             the caller's arrays (every index read from it is bounded) */
};

/* basis of the interpolant (spl_desc.basis) */
enum { SPL_BSPLINE = 0, SPL_LAGRANGE = 1, SPL_PPSPLINE = 2 };

/*
 * Descriptor of one coefficient table.  The caller fills the first block and
 * calls spline_desc_init, which validates it and fills the derived block.
 * Plain data: it may be copied freely; entry points read it on the host.
 */
typedef struct spl_desc {
  /* --- set by the caller --- */
  double  lattice[9];     /* rows = lattice vectors a_i, bohr */
  int32_t grid[3];        /* N_1, N_2, N_3: grid points along a_1, a_2, a_3 (need not be equal, Sec. II Grid) */
  int32_t n_orb;          /* number of orbitals (>= 1) */
  int32_t dtype;          /* SPL_F64 / SPL_F32 / SPL_BF16 */
  int32_t has_lap;        /* 1: a separate Laplacian spline follows the orbital table (Sec. III A) */
  int32_t basis;          /* SPL_BSPLINE (App. A, B-splines); SPL_LAGRANGE (App. A, Lagrange
                             interpolation: the table holds grid values; needs sep_grad, since the
                             Lagrange interpolant has no continuous derivatives); SPL_PPSPLINE (App. A,
                             piecewise-polynomial form of the same interpolating spline: 8 numbers per
                             grid point, [N1][N2][N3][8][o_pad] per table; no sep_grad) */
  int32_t sep_grad;       /* 1: separate gradient tables too (needs has_lap): five tables in the order
                             orbital, d/dx, d/dy, d/dz (Cartesian), Laplacian, each read by value */
  int32_t bloch;          /* 1: Bloch orbitals exp(i k.r) u(r) (Sec. I); n_orb counts complex orbitals */
  int32_t reserved;       /* must be 0 */
  double  kvec[3];        /* k, Cartesian, 1/bohr; must be all zero unless bloch */
  /* --- derived by spline_desc_init --- */
  double  ainv[9];        /* a^-1 (row-major): s = ainv . r */
  double  jac[9];         /* J[i][c] = N_i ainv[i][c] = d u_i / d r_c, u = grid units */
  double  metric[6];      /* M = J J^T as M00 M11 M22 M01 M02 M12 */
  int32_t o_pad;          /* orbital stride of a table row: n_orb rounded up to 16 bytes of storage */
  int32_t elem_bytes;     /* 8 / 4 / 2 */
  int64_t table_elems;    /* N1*N2*N3*o_pad (x8 for SPL_PPSPLINE): elements of ONE table */
  int64_t table_bytes;    /* bytes of the full table buffer: n_tables * table_elems * elem_bytes */
  int64_t work_bytes;     /* bytes of the FP64 workspace spline_build needs: N1*N2*N3*n_col*8 */
  int64_t gtable_bytes;   /* bytes of a coefficient-gradient buffer: n_tables * table_elems * (8 or 4) */
  int32_t n_tables;       /* 1 + has_lap + 3 sep_grad */
  int32_t n_col;          /* real columns of a table row: n_orb, or 2 n_orb (Re u, Im u) with bloch */
} spl_desc;

/*
 * Validate the caller block of *d and fill the derived block.  Host only,
 * enqueues nothing.  Errors: d == NULL, n_orb < 1, non-finite or singular lattice
 * -> SPL_EINVAL; any N_i outside [4, 1024] -> SPL_EGRID; unknown dtype ->
 * SPL_EDTYPE; has_lap, sep_grad or bloch not 0/1, unknown basis, reserved != 0,
 * sep_grad without has_lap, SPL_LAGRANGE without sep_grad, SPL_PPSPLINE with sep_grad, a
 * non-finite kvec, or a nonzero kvec without bloch -> SPL_EINVAL.  N_i >= 4 keeps the four rows of a
 * point's block distinct along each axis.
 */
int spline_desc_init(spl_desc* d);

/*
 * Interpolating B-spline coefficients from grid values (App. A, Interpolating
 * B-spline coefficients).  The coefficients solve (B_1 x B_2 x B_3) beta = f, each
 * B_d periodic tridiagonal with corner elements (rows 1/6, 4/6, 1/6); solved in
 * three stages, one axis at a time, in FP64, then rounded once (to nearest even,
 * via FP32 for BF16) into the storage dtype.
 *   grid_vals  device, FP64 [N1][N2][N3][n_col]: orbital values at r = a (i/N1, j/N2, k/N3)
 *              (with bloch: (Re u, Im u) per orbital)
 *   lap_vals   device, FP64, same shape: grid values of the planewave Laplacian
 *              (the input of the separate Laplacian spline; with bloch its periodic part
 *              exp(-i k.r) lap phi); must be NULL iff !has_lap
 *   table      device, d->table_bytes, written completely (padding zeroed)
 *   work       device, d->work_bytes of scratch FP64, contents undefined afterwards
 * grid_vals and lap_vals are not modified.  None of the buffers may overlap.
 * SPL_PPSPLINE: the same solve kept in FP64, then the 8 numbers of every grid point (the value,
 * second and mixed derivatives of the spline at the knot in grid units, Eq. pp-splinecoefficients3),
 * each the coefficients filtered along every axis by the knot weights (1, 4, 1)/6 or (1, -2, 1).
 * For SPL_LAGRANGE or sep_grad descriptors use spline_build_tables (-> SPL_EINVAL here).
 */
int spline_build(const spl_desc* d, const double* grid_vals, const double* lap_vals,
                 void* table, void* work, void* stream);

/*
 * All n_tables tables of a descriptor from their grid values, stacked:
 *   vals   device, FP64 [n_tables][N1][N2][N3][n_col]: the orbital, then (sep_grad) the
 *          Cartesian gradient components x, y, z, then (has_lap) the Laplacian, each sampled
 *          at r = a (i/N1, j/N2, k/N3) (with bloch: periodic parts, (re, im) per orbital)
 *   table  device, d->table_bytes, written completely (padding zeroed)
 *   work   device, d->work_bytes of scratch FP64 (unused for SPL_LAGRANGE, may be NULL then)
 * SPL_BSPLINE and SPL_PPSPLINE tables are built as in spline_build; SPL_LAGRANGE tables are the
 * grid values themselves, rounded once into the storage dtype (App. A, Eq. lagrangeinterpolation3).
 * vals is not modified.
 */
int spline_build_tables(const spl_desc* d, const double* vals, void* table, void* work, void* stream);

/*
 * Smoothing (Fourier-matched) B-spline coefficients from planewave coefficients (App. A,
 * "Smoothing B-spline coefficients", Eq. b-splinecoefficients):
 *   beta(r_lmn) = sum_G (c_G / gamma_G) exp(i G . r_lmn),  r_lmn = a (l/N1, m/N2, n/N3),
 * with gamma_G = prod_m sinc^4(theta_m / 2), theta_m = 2 pi n_m / N_m (the Fourier transform of
 * one standard-normalized tensor-product basis function), so the spline's fundamental Fourier
 * components equal c_G.  With has_lap, the second table uses (-|G|^2) c_G.
 *   n_g     number of planewaves, 1 <= n_g < 2^31
 *   miller  device, int32 [n_g][3]: Miller indices n of G = 2 pi lattice^-1 n
 *   coef    device, FP64 [n_orb][n_g][2]: complex coefficients (re, im), conjugate-symmetric
 *           in G for real orbitals (the real part of the sum is stored); with bloch, the
 *           coefficients of u (no symmetry; real and imaginary parts are stored)
 *   table   device, d->table_bytes, written completely (padding zeroed)
 *   work    device, spline_smoothing_work_bytes() bytes, 256-byte aligned, scratch
 * The tables after the first hold the smoothing splines of the gradient's periodic parts,
 * coefficients i (k+G)_c c_G (sep_grad), and of the Laplacian's, -|k+G|^2 c_G (has_lap).
 * SPL_LAGRANGE and SPL_PPSPLINE descriptors -> SPL_EINVAL.  The grid must give every G its own Fourier bin
 * (N_i > 2 max |n_i|); planewaves that share a bin are added.  Computed in FP64 by separable
 * inverse DFTs, rounded once into the storage dtype.
 */
int spline_build_smoothing(const spl_desc* d, int64_t n_g, const int32_t* miller, const double* coef,
                           void* table, void* work, void* stream);

/* Workspace bytes of spline_build_smoothing: one complex FP64 grid [N1][N2][N3][n_orb] plus
 * twiddle tables.  Host only. */
int spline_smoothing_work_bytes(const spl_desc* d, int64_t* bytes);

/*
 * Orbital values phi_o(r_p) (App. A, Eq. b-splineapproximation) at n_pts points.
 *   table  device, as written by spline_build
 *   pos    device, FP64 [n_pts][3]
 *   v      device, [n_pts][n_col] (FP64 for SPL_F64 tables, else FP32)
 * SPL_LAGRANGE tables use the Lagrange weights (App. A, Eq. lagrangeinterpolation3), SPL_PPSPLINE
 * tables the 2x2x2 corners and the pp basis (Eq. pp-splineinterpolation3); Bloch orbitals are
 * multiplied by exp(i k.r).  n_pts == 0 is a no-op.
 */
int spline_eval_v(const spl_desc* d, const void* table, int64_t n_pts, const double* pos,
                  void* v, void* stream);

/*
 * Values, Cartesian gradients and Laplacians (VGL) of every orbital at n_pts points.
 * Gradient: grad phi = J^T grad_t phi; Laplacian: sum_ij M_ij d2 phi / dt_i dt_j with
 * the full metric M (off-diagonal terms for non-orthogonal cells), or, with has_lap,
 * the value of the separate Laplacian spline; with sep_grad every output is the value of
 * its own table.  Bloch orbitals (phase e = exp(i k.r)): V = e u, grad = e (grad u + i k u),
 * lap = e (lap u + 2 i k.grad u - |k|^2 u), or e w with a separate Laplacian table of the
 * periodic part w, and e g_c for separate gradient tables.
 *   v     device, [n_pts][n_col]
 *   grad  device, [n_pts][3][n_col]
 *   lap   device, [n_pts][n_col]
 * (FP64 for SPL_F64 tables, else FP32.)  All three are required.
 */
int spline_eval_vgl(const spl_desc* d, const void* table, int64_t n_pts, const double* pos,
                    void* v, void* grad, void* lap, void* stream);

/*
 * Same as spline_eval_vgl with an explicit launch shape: tile[0] = lanes that
 * share one point (2, 4, ..., 256), tile[1] = consecutive orbitals per lane (one
 * vector load per table row): 1 or 2 for SPL_F64, 1, 2 or 4 for SPL_F32, 2, 4 or 8
 * for SPL_BF16; with bloch only the even choices (a lane holds whole (re, im) pairs).
 * Used by the autotuner and tests; results are identical for every valid tile.
 * Invalid tile -> SPL_EINVAL.
 */
int spline_eval_vgl_tile(const spl_desc* d, const void* table, int64_t n_pts, const double* pos,
                         void* v, void* grad, void* lap, const int32_t tile[2], void* stream);

/*
 * spline_eval_vgl with the points evaluated in locality order: the same outputs, bitwise, in the
 * caller's point order.  Points arrive spread over the whole cell, so consecutive points rarely
 * share rows of the table, although each row belongs to the blocks of 64 n_pts / (N1 N2 N3)
 * points on average (Sec. III B: every evaluation reads its 4x4x4 block).  Here a counting sort
 * puts the points into buckets of cells numbered along a Morton curve (at most 2^18 buckets;
 * larger grids group 2^k cells per axis), and the forward kernel runs through that permutation
 * with each XCD taking a contiguous stretch of the curve, so neighbouring points share their rows
 * in L2 and the Infinity Cache.  The sort runs on `stream` inside the call; the order within a
 * bucket may differ between calls, the outputs do not.
 *   tile       NULL = the tile spline_eval_vgl would use, else as in spline_eval_vgl_tile
 *   work       device workspace, 256-byte aligned, at least spline_sorted_work_bytes() bytes,
 *              contents undefined afterwards
 * Every representation a descriptor can describe is accepted.  Allocates nothing.
 */
int spline_eval_vgl_sorted(const spl_desc* d, const void* table, int64_t n_pts, const double* pos,
                           void* v, void* grad, void* lap, const int32_t* tile,
                           void* work, int64_t work_bytes, void* stream);

/* Workspace size (bytes) of spline_eval_vgl_sorted for n_pts points (bucket of each point, bucket
 * counts and offsets, permutation, the scan's scratch).  Host only; may query the current HIP device. */
int spline_sorted_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes);

/*
 * spline_eval_vgl_sorted for callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same computation and outputs, bit for bit, with the
 * workspace taken from a static device array of the library (16 MiB per device, held until the process
 * ends) instead of a caller buffer.  Calls no allocating routine; the first call on a device looks up
 * that device's copy of the array.  All arguments as for spline_eval_vgl_sorted (no work, work_bytes).
 * Limit: the workspace of n_pts points must fit in 16 MiB, about 1.8 million points; more ->
 * SPL_EINVAL before anything is enqueued (use spline_eval_vgl_sorted).  Every call on a device shares
 * that device's array and leaves it dirty: calls that overlap on one device (other streams, other host
 * threads) race and must be serialized by the caller.
 */
int spline_eval_vgl_sorted_noalloc(const spl_desc* d, const void* table, int64_t n_pts, const double* pos,
                                   void* v, void* grad, void* lap, const int32_t* tile, void* stream);

/*
 * Values, gradients and Laplacians as spline_eval_vgl, computed cell by cell: the points are
 * sorted by grid cell (stable radix sort), and for the points of one cell the outputs are a dense
 * product of their 64 row weights with the cell's 4x4x4 block (Eq. b-splineapproximation with
 * the chain rule of Sec. II), done on the matrix cores with each block read once per cell.  For
 * point sets with several points per cell (fits, dense sampling); QMC walkers rarely share cells.
 * The outputs equal spline_eval_vgl's up to the order of summation, in the caller's point order.
 *   v, grad, lap  device, as for spline_eval_vgl; each may be NULL to skip it (not all three)
 *   flags         0 or SPL_REUSE_SORT
 *   work          device workspace, 256-byte aligned, at least spline_cells_work_bytes() bytes; it
 *                 holds the cell sort afterwards (a deterministic spline_eval_vgl_backward of the same
 *                 points may reuse it, given spline_backward_work_bytes() bytes)
 * Non-finite points get NaN.  Real B-spline tables only (with or without a separate Laplacian
 * table); other descriptors -> SPL_EUNSUPPORTED.  Allocates nothing.
 */
int spline_eval_vgl_cells(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v,
                          void* grad, void* lap, int32_t flags, void* work, int64_t work_bytes, void* stream);

/* Workspace bytes of spline_eval_vgl_cells and spline_fit_terms_cells for n_pts points (the sort's
 * keys, runs and point records, one FP64 partial sum per cell and 16 orbitals).  Host only; may
 * query the current HIP device. */
int spline_cells_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes);

/*
 * The data terms of the least-squares fit (spline_misfit) computed straight from the cell-wise
 * evaluation, so values and Laplacians never pass through memory: for the n_pts fit points,
 * with y_v, y_lap the values and Laplacians spline_eval_vgl_cells would write,
 *   g_v    = 2 w_v (y_v - t_v),        g_lap = 2 w_lap (y_lap - t_lap)     (OVERWRITTEN)
 *   *loss += w_v sum (y_v - t_v)^2 + w_lap sum (y_lap - t_lap)^2           (ACCUMULATED)
 *   t_v, g_v      device, [n_pts][n_orb] of the output type (FP64 for SPL_F64, else FP32), the
 *                 caller's point order; both NULL to leave out the value term
 *   t_lap, g_lap  likewise for the Laplacian term (at least one term is required)
 *   w_v, w_lap    the terms' weights, finite
 *   loss          device, one FP64
 *   flags, work   as for spline_eval_vgl_cells (the workspace holds the cell sort afterwards)
 * g equals what spline_misfit makes of spline_eval_vgl_cells' outputs bit for bit (the residuals
 * are the same numbers in the output type); the loss is summed in FP64 per cell and 16 orbitals
 * and then in a fixed order, so it is reproducible bit for bit and agrees with spline_misfit's to
 * rounding.  A non-finite point gets NaN gradients and makes the loss NaN.  Errors as for
 * spline_eval_vgl_cells, plus: a target without its gradient or the reverse, no term, non-finite
 * weight, NULL or misaligned loss -> SPL_EINVAL.  Allocates nothing.
 */
int spline_fit_terms_cells(const spl_desc* d, const void* table, int64_t n_pts, const double* pos,
                           const void* t_v, double w_v, void* g_v, const void* t_lap, double w_lap,
                           void* g_lap, double* loss, int32_t flags, void* work, int64_t work_bytes,
                           void* stream);

/*
 * The data terms of the least-squares fit and their coefficient gradient in one pass: for the
 * n_pts fit points, with y_v, y_lap the values and Laplacians of the table there,
 *   *loss  += w_v sum (y_v - t_v)^2 + w_lap sum (y_lap - t_lap)^2                (ACCUMULATED)
 *   gtable += d/dtable of those two sums                                            (ACCUMULATED)
 * that is, spline_fit_terms_cells followed by spline_eval_vgl_backward (SPL_DETERMINISTIC) of its
 * upstream gradients, with the same results bit for bit (for a lattice with orthogonal vectors the
 * same numbers: the vanishing mixed terms of the Laplacian are skipped, so an exact zero may differ
 * in sign), but the upstream gradients are never stored: each batch of a cell's points is
 * evaluated, compared with its targets and multiplied back on the matrix cores in one kernel.  (The fit's regression counterpart of the smoothing spline of
 * App. A; the adjoint is the transpose of Eq. b-splineapproximation.)
 *   t_v, t_lap   device, FP32 [n_pts][n_orb] in the caller's point order (both required)
 *   w_v, w_lap   the terms' weights, finite
 *   gtable       device, d->gtable_bytes, FP32 [N1][N2][N3][o_pad]; padding columns are never written
 *   loss         device, one FP64
 *   flags        SPL_REUSE_SORT: the workspace holds the cell sort of these points, with its cells'
 *                point ranges, from an earlier call of this function (the layout differs from
 *                spline_cells_work_bytes')
 *   work         device, 256-byte aligned, spline_fit_gradient_work_bytes() bytes
 * Supported: FP32 B-spline tables without a separate Laplacian table, at least 2.5 points per cell
 * on average, and the table and each target array under 2 GiB; otherwise SPL_EUNSUPPORTED (use
 * spline_fit_terms_cells and spline_eval_vgl_backward).  A non-finite point contributes nothing to
 * gtable and makes the loss NaN.  Other errors as for spline_fit_terms_cells.  Allocates nothing.
 */
int spline_fit_gradient_cells(const spl_desc* d, const void* table, int64_t n_pts, const double* pos,
                              const void* t_v, double w_v, const void* t_lap, double w_lap, void* gtable,
                              double* loss, int32_t flags, void* work, int64_t work_bytes, void* stream);

/* Workspace bytes of spline_fit_gradient_cells for n_pts points (the cell sort, each cell's point
 * range, the brick regions and the loss partial sums).  Host only; may query the current HIP device. */
int spline_fit_gradient_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes);


/*
 * Adjoint of spline_eval_vgl: given dL/dv, dL/dgrad, dL/dlap of a scalar loss L,
 *   gtable += dL/dtable   (the transpose of the 64-coefficient gather, periodic wrap)
 *   gpos    = dL/dpos     (through grad, Hessian and gradient of the Laplacian)
 *   gv, ggrad, glap  device, same layouts and dtypes as the forward outputs; each may be
 *                    NULL (treated as zero)
 *   gtable           device, d->gtable_bytes: [(1+has_lap)][N1][N2][N3][o_pad], FP64 for
 *                    SPL_F64 tables, else FP32; ACCUMULATED into (zero it first for a plain
 *                    gradient); may be NULL to skip; padding columns are never written
 *   gpos             device, FP64 [n_pts][3], OVERWRITTEN; may be NULL to skip
 *   flags            0: the coefficient gradient is summed with hardware float atomics (order
 *                    of summation not reproducible; no workspace); SPL_DETERMINISTIC: points are
 *                    sorted by grid cell and every sum is formed in a fixed order on the matrix
 *                    cores: under 2.5 points per cell, each tile of 4x4x4 table rows sums the
 *                    points of the cells whose blocks reach it and adds the sum once; at 2.5
 *                    or more, the cells' blocks are summed per brick of 2x2x2 cells and gathered
 *                    per table row: bitwise reproducible, and the faster of the two at every
 *                    density measured
 *                    SPL_REUSE_SORT (with SPL_DETERMINISTIC): the workspace already holds the
 *                    cell sort of these points
 *   work, work_bytes device workspace for SPL_DETERMINISTIC, 256-byte aligned, at least
 *                    spline_backward_work_bytes() bytes; holds the cell sort afterwards; may be
 *                    NULL (0 bytes) without that flag
 * The position gradient is deterministic either way.  Points with non-finite coordinates
 * contribute nothing to gtable and get NaN in gpos.  Descriptors with basis, sep_grad or
 * bloch set -> SPL_EUNSUPPORTED (the adjoint covers the real B-spline forms).
 */
int spline_eval_vgl_backward(const spl_desc* d, const void* table, int64_t n_pts, const double* pos,
                             const void* gv, const void* ggrad, const void* glap,
                             void* gtable, double* gpos, int32_t flags,
                             void* work, int64_t work_bytes, void* stream);

/* Workspace size (bytes) spline_eval_vgl_backward needs for n_pts points and `flags` (0 without
 * SPL_DETERMINISTIC).  With it: the sort's keys, runs and point records, every cell's point range
 * (12 bytes per cell), and, when 2 n_pts >= 5 N1 N2 N3 and they fit in 4 GiB, the regions of the
 * bricks of 2x2x2 cells (ceil(N1/2) ceil(N2/2) ceil(N3/2) 125 o_pad gradient values).
 * Host only; may query the current HIP device. */
int spline_backward_work_bytes(const spl_desc* d, int64_t n_pts, int32_t flags, int64_t* bytes);

/*
 * Data term of the least-squares fit of coefficients to orbital samples, the regression
 * counterpart of App. A's smoothing spline that exercises the adjoint: for n outputs y of
 * spline_eval_vgl (values or Laplacians at the fit points) and their targets t,
 *   *loss += w sum_i (y_i - t_i)^2,      g_i = 2 w (y_i - t_i)  (the upstream gradient of that
 *                                        term, input to spline_eval_vgl_backward).
 *   n     number of output values (n_pts n_col for a whole output array); 0 is a no-op
 *   y, t  device, n values of the descriptor's output type (FP64 for SPL_F64, else FP32)
 *   w     the term's weight, finite (a mean over the outputs passes 1/n times its weight)
 *   g     device, n values, OVERWRITTEN; may be y itself
 *   loss  device, one FP64, ACCUMULATED into
 *   work  device, spline_misfit_work_bytes() bytes, 8-byte aligned (partial sums)
 * Residuals are formed in the output type, their squares and sums in FP64 in a fixed order,
 * so *loss is reproducible bit for bit.  Errors: NULL pointer, n < 0, non-finite w, short work,
 * misaligned pointer -> SPL_EINVAL.  Allocates nothing.
 */
int spline_misfit(const spl_desc* d, int64_t n, const void* y, const void* t, double w, void* g, double* loss,
                  void* work, int64_t work_bytes, void* stream);

/*
 * Smoothness penalty of the same fit: with D the periodic second difference along one grid axis
 * (beta_{i-1} - 2 beta_i + beta_{i+1}), over the orbital table's real orbitals o < n_orb,
 *   *loss  += w sum over the 3 axes, the grid points and the orbitals of (D beta)^2
 *   gtable += 2 w sum over the axes of D (D beta)   (the gradient; D is symmetric under the wrap)
 *   table   device, as written by spline_build (real B-spline; other descriptors -> SPL_EUNSUPPORTED)
 *   w       the penalty's weight, finite
 *   gtable  device, the gradient table of spline_eval_vgl_backward; its orbital table is
 *           ACCUMULATED into, padding columns untouched
 *   loss    device, one FP64, ACCUMULATED into
 *   work    device, spline_misfit_work_bytes() bytes, 8-byte aligned
 * Computed in FP64 whatever the storage type; the sum is reduced in a fixed order (bitwise
 * reproducible).  Errors: NULL pointer, non-finite w, short work, misalignment -> SPL_EINVAL.
 */
int spline_smoothness_penalty(const spl_desc* d, const void* table, double w, void* gtable, double* loss,
                              void* work, int64_t work_bytes, void* stream);

/* Workspace bytes of spline_misfit (a fixed number of FP64 partial sums).  Host only. */
int spline_misfit_work_bytes(const spl_desc* d, int64_t n, int64_t* bytes);

/*
 * One Adam step (Kingma and Ba, Algorithm 1) on n stored coefficients, element by element:
 *   m = beta1 m + (1 - beta1) g,   v = beta2 v + (1 - beta2) g^2,
 *   param -= lr / (1 - beta1^step) m / (sqrt(v) / sqrt(1 - beta2^step) + eps)
 * in the precision of the moments: FP64 for SPL_F64, FP32 for SPL_F32 and SPL_BF16 (BF16 parameters
 * are widened and rounded back to nearest even).  The fit's optimizer.
 *   dtype        SPL_F64, SPL_F32 or SPL_BF16 (the table's)
 *   param        device, n values of the table's storage type, UPDATED
 *   grad, m, v   device, n values of the moment type (FP64 for SPL_F64, else FP32); m, v UPDATED
 *                (zero before step 1)
 *   lr, beta1, beta2, eps, step   finite lr; 0 <= beta1, beta2 < 1; eps > 0; step >= 1
 * n = 0 is a no-op.  Errors: unknown dtype -> SPL_EDTYPE; n < 0, arguments out of range, NULL or
 * misaligned pointers -> SPL_EINVAL.  Allocates nothing.
 */
int spline_adam_step(int32_t dtype, int64_t n, void* param, const void* grad, void* m, void* v, double lr,
                     double beta1, double beta2, double eps, int32_t step, void* stream);

/* ---------------------------------------------------------------------------
 * Batched evaluation: many independent systems (tables of different sizes and
 * orbital counts, point sets of different sizes) in ONE persistent launch.
 * All items of a plan share one storage dtype.
 */
typedef struct spl_item {
  const spl_desc* d;      /* host pointer, read during plan creation only */
  const void* table;      /* device */
  int64_t n_pts;
  const double* pos;      /* device [n_pts][3] */
  void* v;                /* device outputs, as for spline_eval_vgl */
  void* grad;
  void* lap;
} spl_item;

/*
 * Build a plan: copies per-item parameters and the work list of (item, point tile) pairs
 * to device memory the plan owns (this call allocates, once, and synchronizes `stream`).
 * Items are reordered internally by decreasing work per tile; outputs go to each item's
 * own buffers.  All items must share dtype and has_lap, and be real B-spline tables
 * without sep_grad (others -> SPL_EUNSUPPORTED).  tile: NULL = the tuned (or
 * default) shape of the heaviest item, else as in spline_eval_vgl_tile with tile[0] in
 * 8..256.  On success *plan is set.  The item buffers must outlive the plan.
 * Errors: any item failing the checks of spline_eval_vgl -> that code, prefixed with the
 * item index; allocation failure -> SPL_ENOMEM.
 */
int spline_batch_plan_create(const spl_item* items, int32_t n_items, const int32_t* tile,
                             void* stream, void** plan);

/* One persistent launch over the plan's whole work list: a counter-reset kernel then the
 * persistent kernel, whose workgroups take point tiles from a device counter until none
 * remain.  Graph-capturable (no memset, no allocation).  One launch of a plan at a time:
 * concurrent launches of the same plan share its counter and race. */
int spline_batch_eval_vgl(void* plan, void* stream);

/* Capture spline_batch_eval_vgl into a HIP graph owned by the plan (on first use, on a
 * private stream of default priority) and launch that graph on `stream`.  Later calls
 * replay the same graph; changing the plan's tile drops it. */
int spline_batch_graph_launch(void* plan, void* stream);

/* Choose the plan's tile shapes by timing on `stream` (synchronizes): every common shape (lanes per
 * point 8..256 x the dtype's orbitals-per-lane choices) with whole persistent launches, then, for
 * each orbitals-per-lane choice, per-item shapes (each item's lanes per point the fastest for that
 * item alone, timed with the single-system kernel on its own buffers) again as whole launches.  The
 * fastest is kept in the plan; tile_out gets the common shape, or (0, orbitals per lane) when items
 * keep their own lanes per point (spline_batch_plan_get_tiles lists them).  Every shape gives the same
 * outputs bit for bit; they are overwritten with valid results. */
int spline_batch_autotune(void* plan, void* stream, int32_t tile_out[2]);

/* Each item's tile shape in the caller's item order: tiles_out[2 j] = lanes per point of item j,
 * tiles_out[2 j + 1] = orbitals per lane (common to all items).  Host only. */
int spline_batch_plan_get_tiles(void* plan, int32_t* tiles_out);

/* Give each item its own lanes per point: tiles[2 j], tiles[2 j + 1] as above, in the caller's item
 * order (a power of two in 8..256; one orbitals-per-lane value for all items, valid for the dtype).
 * Synchronizes `stream` (uploads the plan's records); drops the captured graph.  Errors: NULL plan
 * or tiles, an invalid shape, or differing orbitals per lane -> SPL_EINVAL. */
int spline_batch_plan_set_tiles(void* plan, const int32_t* tiles, void* stream);

/* Evaluate the plan's points in locality order (enable = 1) or in their given order (0, the
 * default).  Sorted launches first counting-sort every item's points into buckets of its cells
 * numbered along a Morton curve (at most 2^15 per item), as spline_eval_vgl_sorted does for one
 * system, then run the persistent kernel through each item's permutation; outputs are bitwise the
 * same.  The first enable allocates the plan-owned sort state (per-point buckets and permutation,
 * bucket counts and offsets, scan scratch) and synchronizes `stream`; toggling drops the captured
 * graph.  Sorted launches stay graph-capturable.  Errors: NULL plan or enable not 0/1 ->
 * SPL_EINVAL; allocation failure -> SPL_ENOMEM. */
int spline_batch_plan_sort(void* plan, int32_t enable, void* stream);

/* Release a plan and everything it owns (synchronizes the device first). */
void spline_batch_plan_destroy(void* plan);

/* Work counters of a plan: number of tiles and of (point, orbital) evaluations. */
int spline_batch_plan_info(void* plan, int64_t* n_tiles, int64_t* n_evals);

/*
 * Time the tile shapes of spline_eval_vgl_tile on the caller's buffers (lanes per point from 4
 * up to one row per pass, every orbitals-per-lane choice)
 * (each several times, HIP events on `stream`; synchronizes), keep the fastest in
 * the process-wide cache keyed by (dtype, has_lap, o_pad, grid), and return it in
 * tile_out[0..1].  The outputs are overwritten with valid results.  If the
 * environment variable PWSPLINE_TUNE_CACHE names a file, the cache is also
 * appended there and read back at first use.
 */
int spline_autotune(const spl_desc* d, const void* table, int64_t n_pts, const double* pos,
                    void* v, void* grad, void* lap, void* stream, int32_t tile_out[2]);

/* Tile shape spline_eval_vgl would use for this descriptor (cache hit or default). */
int spline_tile_for(const spl_desc* d, int64_t n_pts, int32_t tile_out[2]);

/*
 * Read-rate probe (measurement aid, not part of the method): reads `bytes` bytes of `buf` once, as a
 * linear stream of 16-byte loads spread over the whole device, and writes nothing but (practically
 * never) 4 bytes at `sink`.  Timed by the caller, it gives the achievable read bandwidth of device
 * memory, the ceiling for the gather of Sec. III B, which reads and hardly writes.
 *   buf    device, 16-byte aligned; bytes a multiple of 16 (0: no-op)
 *   sink   device, 4 bytes, 4-byte aligned
 * Errors: negative or unaligned sizes, NULL or misaligned pointers -> SPL_EINVAL; launch -> SPL_EHIP.
 */
int spline_stream_read(const void* buf, int64_t bytes, void* sink, void* stream);

/* Human-readable description of the last error on this thread ("" if none). */
const char* spline_last_error(void);

/* Library version (major*10000 + minor*100 + patch). */
int spline_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PWSPLINE_H */
