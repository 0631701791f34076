"""GPU parity of the HIP library against the FP64 oracle (small and ragged cases).

Tolerances (normwise = max|err| / max|ref| per quantity; elementwise bounds use the
oracle's sum over the 64 terms of |weight| * |coefficient|, a standard dot-product
rounding bound):
  * kernel parity, same stored table on both sides: |err| <= 2 * 64 * u_acc * sum|w||beta|
    with u_acc = 2^-53 (FP64 tables) or 2^-24 (FP32 / BF16 tables, FP32 arithmetic), plus
    the movement allowed by rounding of the grid coordinate u on either side (derivative
    one order higher times |delta u|, oracle.evaluate.coordinate_error_bound);
  * build parity (FP64): <= 1e-13 * max|beta|; storage casts: within one unit in the last
    place of the storage type and identical for >= 99.9% of coefficients (the two FP64
    builds differ by rounding, which can move a value across a rounding boundary);
  * end to end against the FP64 oracle: normwise <= 1e-10 (FP64), <= 1e-5 (FP32), and for
    BF16 <= 5e-3 (value), 1e-2 (gradient), 5e-2 (Laplacian from derivatives), 5e-3
    (separate Laplacian spline).
"""
import numpy as np
import pytest
import torch

import paper_1309_6250_amd as P
from oracle import build as obuild, evaluate as oeval, quantize as oq, adjoint as oadj
from workloads import config, make_system
from workloads.configs import A_MGO, cubic
from gpu_helpers import (say, to_dev, table_from_oracle, gpu_build, gpu_vgl, normwise, assert_elementwise,
                         host_table, coordinate_rounding, U_ACC, DEV)

pytestmark = pytest.mark.gpu

SKEW = np.array([[7.0, 0.4, -0.3], [1.1, 6.2, 0.5], [-0.6, 0.9, 8.3]])


def special_points(lattice, grid, rng, n=64):
    n_ = np.array(grid)
    k = rng.integers(0, n_, size=(n // 4, 3))
    on_grid = (k / n_) @ lattice                                   # exactly on knots
    far = rng.uniform(-3, 3, size=(n // 4, 3)) @ lattice           # anywhere in R^3
    edges = np.array([[-1e-300, 0.0, 0.0], [0.0, -1e-17, 5e-324]]) @ np.eye(3)
    planes = ((rng.integers(0, n_, size=(n // 4, 3)) + rng.choice([0.0, 0.5], size=(n // 4, 3))) / n_) @ lattice
    return np.concatenate([on_grid, far, edges, planes])


def off_knots(lattice, grid, pos, eps=1e-9):
    """Points farther than eps (grid units) from every knot plane: there the position gradient of
    the Laplacian (a third derivative, piecewise constant across knots) is single-valued."""
    _, t, ok = oeval.reduced_coordinates(lattice, grid, pos)
    return ok & np.all((t > eps) & (t < 1 - eps), axis=1)


def small_cases():
    """(name, lattice, grid values f, lap values or None, positions)."""
    out = []
    w = config(0)
    s = w.system
    rng = np.random.default_rng(100)
    out.append(("si-fcc-16", s.lattice, s.grid_values(), None,
                np.concatenate([w.positions(), special_points(s.lattice, s.grid, rng)])))
    s5 = config(5).system
    out.append(("al-fcc-16", s5.lattice, s5.grid_values(), None, config(5).positions()[:1000]))
    # ragged: unequal grid, orbital count not a multiple of any vector width, skewed cell
    rs = make_system("ragged", SKEW, (5, 7, 9), 3, 1.6, 2.0, (5, 5))
    out.append(("ragged-5x7x9-o3", SKEW, rs.grid_values(), None,
                np.concatenate([rs.positions(777), special_points(SKEW, (5, 7, 9), rng)])))
    # MgO-like rock-salt cell with a separate Laplacian spline, 37 orbitals (ragged tail)
    ms = make_system("mgo-small", cubic(2 * A_MGO), (20, 20, 20), 37, 3.2, 8.0, (9, 9))
    out.append(("mgo-20-o37-lap", ms.lattice, ms.grid_values(), ms.grid_laplacian(), ms.positions(1500)))
    return out


CASES = small_cases()
CASE_IDS = [c[0] for c in CASES]


@pytest.fixture(scope="module", params=range(len(CASES)), ids=CASE_IDS)
def case(request):
    name, lattice, f, lf, pos = CASES[request.param]
    beta = obuild.build_interp(f)
    lbeta = None if lf is None else obuild.build_interp(lf)
    return dict(name=name, lattice=lattice, f=f, lf=lf, pos=pos, beta=beta, lbeta=lbeta)


def _desc(c, dtype):
    n_orb = c["f"].shape[3]
    return P.spline_desc_init(c["lattice"], c["f"].shape[:3], n_orb, dtype, has_lap=c["lf"] is not None)


def test_build_fp64_matches_oracle(case):
    d = _desc(case, "f64")
    tab = gpu_build(d, case["f"], case["lf"])
    got = host_table(d, tab)
    beta = case["beta"]
    assert np.abs(got[0] - beta).max() <= 1e-13 * np.abs(beta).max()
    if case["lbeta"] is not None:
        assert np.abs(got[1] - case["lbeta"]).max() <= 1e-13 * np.abs(case["lbeta"]).max()
    pad = tab.double().cpu().numpy()[..., d.n_orb:]
    assert pad.size == 0 or np.all(pad == 0.0)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_build_storage_cast(case, dtype):
    d = _desc(case, dtype)
    tab = gpu_build(d, case["f"], case["lf"])
    got = host_table(d, tab)
    tables = [case["beta"]] + ([case["lbeta"]] if case["lbeta"] is not None else [])
    for k, beta in enumerate(tables):
        ref = oq.quantized(beta, dtype)
        ulp = (2.0**-23 if dtype == "f32" else 2.0**-7) * np.abs(ref)
        diff = np.abs(got[k] - ref)
        assert np.all(diff <= ulp + 1e-300)
        assert np.mean(diff == 0) >= 0.999
    pad = tab.float().cpu().numpy()[..., d.n_orb:]
    assert pad.size == 0 or np.all(pad == 0.0)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_eval_kernel_parity_same_table(case, dtype):
    """Same stored coefficients on both sides: isolates the kernel's arithmetic."""
    d = _desc(case, dtype)
    tab = table_from_oracle(d, case["beta"], dtype, case["lbeta"])
    bq = oq.quantized(case["beta"], dtype)
    lq = None if case["lbeta"] is None else oq.quantized(case["lbeta"], dtype)
    pos = case["pos"]
    v, g, l = gpu_vgl(d, tab, pos)
    rv, rg, rl = oeval.eval_vgl(bq, case["lattice"], pos, lap_beta=lq)
    bv, bg, bl = oeval.eval_abs_bound(bq, case["lattice"], pos, lap_beta=lq)
    cv, cg, cl = oeval.coordinate_error_bound(bq, case["lattice"], pos,
                                              coordinate_rounding(d, case["lattice"], pos, dtype), lap_beta=lq)
    fac = 2 * 64 * U_ACC[dtype]
    ok = np.isfinite(rv[:, 0])
    out_round = 0.0 if dtype == "f64" else 2.0**-24       # FP32 outputs round once more
    assert_elementwise(v[ok], rv[ok], bv[ok] + cv[ok] / (fac + out_round), fac + out_round, "V")
    assert_elementwise(g[ok], rg[ok], bg[ok] + cg[ok] / (fac + out_round), fac + out_round, "grad")
    assert_elementwise(l[ok], rl[ok], bl[ok] + cl[ok] / (fac + out_round), fac + out_round, "lap")
    assert np.isnan(v[~ok]).all() and np.isnan(g[~ok]).all() and np.isnan(l[~ok]).all()


GATES = {"f64": (1e-10, 1e-10, 1e-10, 1e-10), "f32": (1e-5, 1e-5, 1e-5, 1e-5),
         "bf16": (5e-3, 1e-2, 5e-2, 5e-3)}


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_end_to_end_against_fp64_oracle(case, dtype):
    """GPU build + GPU eval against the oracle's FP64 build + eval of the same grid values."""
    d = _desc(case, dtype)
    tab = gpu_build(d, case["f"], case["lf"])
    pos = case["pos"]
    v, g, l = gpu_vgl(d, tab, pos)
    rv, rg, rl = oeval.eval_vgl(case["beta"], case["lattice"], pos, lap_beta=case["lbeta"])
    gv, gg, gd, gs = GATES[dtype]
    assert normwise(v, rv) <= gv
    assert normwise(g, rg) <= gg
    assert normwise(l, rl) <= (gs if case["lbeta"] is not None else gd)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_all_tiles_give_identical_results(case, dtype):
    d = _desc(case, dtype)
    tab = table_from_oracle(d, case["beta"], dtype, case["lbeta"])
    pos = case["pos"][:700]
    opls = {"f64": (1, 2), "f32": (1, 2, 4), "bf16": (2, 4, 8)}[dtype]
    ref = gpu_vgl(d, tab, pos, tile=(2, opls[0]))
    for g in (2, 4, 16, 64, 256):
        for opl in opls:
            out = gpu_vgl(d, tab, pos, tile=(g, opl))
            for a, b in zip(out, ref):
                np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_eval_v_matches_oracle(case, dtype):
    d = _desc(case, dtype)
    tab = table_from_oracle(d, case["beta"], dtype, case["lbeta"])
    pos = case["pos"]
    say("spline_eval_v", case["name"], dtype)
    v = P.spline_eval_v(d, tab, to_dev(pos))
    torch.cuda.synchronize()
    v = v.double().cpu().numpy()
    bq = oq.quantized(case["beta"], dtype)
    rv = oeval.eval_v(bq, case["lattice"], pos)
    bv, _, _ = oeval.eval_abs_bound(bq, case["lattice"], pos)
    cv, _, _ = oeval.coordinate_error_bound(bq, case["lattice"], pos, coordinate_rounding(d, case["lattice"], pos, dtype))
    ok = np.isfinite(rv[:, 0])
    fac = 2 * 64 * U_ACC[dtype] + (0 if dtype == "f64" else 2.0**-24)
    assert_elementwise(v[ok], rv[ok], bv[ok] + cv[ok] / fac, fac, "V")
    vgl = gpu_vgl(d, tab, pos)
    np.testing.assert_array_equal(v[ok], vgl[0][ok])


def test_nonfinite_points_and_empty_input():
    c = CASES[0]
    d = P.spline_desc_init(c[1], c[2].shape[:3], c[2].shape[3], "f64")
    tab = gpu_build(d, c[2])
    pos = np.array([[np.nan, 0, 0], [1.0, 2.0, 3.0], [np.inf, -np.inf, 0], [0, 0, np.nan]])
    v, g, l = gpu_vgl(d, tab, pos)
    assert np.isnan(v[[0, 2, 3]]).all() and np.isnan(g[[0, 2, 3]]).all() and np.isnan(l[[0, 2, 3]]).all()
    assert np.isfinite(v[1]).all()
    say("empty input")
    empty = torch.empty((0, 3), dtype=torch.float64, device=DEV)
    v0, g0, l0 = P.spline_eval_vgl(d, tab, empty)
    torch.cuda.synchronize()
    assert v0.shape == (0, d.n_orb)


def test_largest_grid_axis():
    # grid axis at the 1024 limit (build stage with the smallest LDS tile) and a 1-orbital table
    rng = np.random.default_rng(101)
    lat = np.diag([40.0, 3.0, 3.5])
    f = rng.standard_normal((1024, 4, 5, 1))
    beta = obuild.build_interp(f)
    d = P.spline_desc_init(lat, (1024, 4, 5), 1, "f64")
    tab = gpu_build(d, f)
    assert np.abs(host_table(d, tab)[0] - beta).max() <= 1e-13 * np.abs(beta).max()
    pos = rng.uniform(-50, 50, size=(300, 3))
    v, g, l = gpu_vgl(d, tab, pos)
    rv, rg, rl = oeval.eval_vgl(beta, lat, pos)
    assert normwise(v, rv) < 1e-12 and normwise(g, rg) < 1e-12 and normwise(l, rl) < 1e-12


# ------------------------------------------------------------------ backward
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("which", ["all", "value-only", "no-grad"])
def test_backward_matches_oracle(case, dtype, which):
    d = _desc(case, dtype)
    tab = table_from_oracle(d, case["beta"], dtype, case["lbeta"])
    bq = oq.quantized(case["beta"], dtype)
    lq = None if case["lbeta"] is None else oq.quantized(case["lbeta"], dtype)
    rng = np.random.default_rng(102)
    pos = case["pos"]
    keep = np.all(np.isfinite(pos), axis=1)
    # stay off the knots: the third derivative (position gradient of the Laplacian) jumps there
    pos = pos[keep][:600]
    n, o = pos.shape[0], d.n_orb
    gv = rng.standard_normal((n, o))
    gg = None if which == "value-only" else rng.standard_normal((n, 3, o))
    gl = None if which in ("value-only",) else rng.standard_normal((n, o))
    if which == "no-grad":
        gg = None
    od = torch.float64 if dtype == "f64" else torch.float32
    say("spline_eval_vgl_backward", case["name"], dtype, which)
    gtab, gpos = P.spline_eval_vgl_backward(d, tab, to_dev(pos), to_dev(gv, od),
                                            None if gg is None else to_dev(gg, od),
                                            None if gl is None else to_dev(gl, od))
    torch.cuda.synchronize()
    rb, rlb, rp = oadj.vgl_backward(bq, case["lattice"], pos, gv, gg, gl, lap_beta=lq)
    got = gtab.double().cpu().numpy()[..., :o]
    tol = 1e-12 if dtype == "f64" else 2e-5
    assert normwise(got[0], rb) <= tol
    if rlb is not None:
        if np.any(rlb != 0):
            assert normwise(got[1], rlb) <= tol
        else:                                   # no Laplacian upstream gradient: nothing reaches that table
            assert np.all(got[1] == 0.0)
    # position gradients: compared off the knot planes, where the third derivative is single-valued
    gp = gpos.cpu().numpy()
    smooth = off_knots(case["lattice"], d.grid, pos)
    assert normwise(gp[smooth], rp[smooth]) <= (1e-10 if dtype == "f64" else 1e-4)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_backward_position_gradient_on_knots(dtype):
    """Points on a knot plane and within 1e-9 grid units of one.  The position gradient of the
    Laplacian term uses the third derivative, which jumps across a knot plane, so at such a point
    the gradient has two one-sided values: the oracle's on either side (1e-11 grid units away, where
    the continuous terms have not moved measurably).  The GPU must match one of them per component
    (the side its own rounding of the grid coordinate picks); points off the plane by 1e-9 must
    match the side they lie on."""
    rng = np.random.default_rng(107)
    grid = (7, 6, 8)
    n_orb = 5
    n = np.array(grid)
    beta = rng.standard_normal(grid + (n_orb,))
    d = P.spline_desc_init(SKEW, grid, n_orb, dtype)
    tab = table_from_oracle(d, beta, dtype)
    bq = oq.quantized(beta, dtype)
    m = 240
    cells = rng.integers(0, n, size=(m, 3))
    u = cells + rng.uniform(0.2, 0.8, size=(m, 3))
    axis = rng.integers(0, 3, size=m)
    offset = np.choose(np.arange(m) % 3, [0.0, 1e-9, -1e-9])
    u[np.arange(m), axis] = cells[np.arange(m), axis] + offset
    pos = (u / n) @ SKEW
    gv = rng.standard_normal((m, n_orb))
    gg = rng.standard_normal((m, 3, n_orb))
    gl = rng.standard_normal((m, n_orb))
    od = torch.float64 if dtype == "f64" else torch.float32
    say("position gradient on knot planes", dtype)
    _, gpos = P.spline_eval_vgl_backward(d, tab, to_dev(pos), to_dev(gv, od), to_dev(gg, od), to_dev(gl, od))
    torch.cuda.synchronize()
    gp = gpos.cpu().numpy()
    step = np.zeros((m, 3))
    step[np.arange(m), axis] = 1e-11
    side = []
    for sgn in (-1.0, 1.0):
        _, _, rp = oadj.vgl_backward(bq, SKEW, ((u + sgn * step) / n) @ SKEW, gv, gg, gl)
        side.append(rp)
    scale = np.abs(np.concatenate(side)).max()
    tol = (1e-10 if dtype == "f64" else 1e-4) * scale
    near = [np.abs(gp - r) <= tol for r in side]
    on_plane = offset == 0.0
    assert np.all((near[0] | near[1])[on_plane])
    assert np.all(near[0][offset < 0]) and np.all(near[1][offset > 0])
    # the two sides do differ on the plane (the test would be empty otherwise)
    assert np.abs(side[0] - side[1])[on_plane].max() > 100 * tol


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n_orb", [1, 3, 4, 8, 12])
def test_no_writes_past_outputs(dtype, n_orb):
    """Outputs live at the front of larger buffers whose tails hold a sentinel: every tile and
    both entry points must leave the tails untouched (padding chunks are never stored)."""
    rng = np.random.default_rng(103)
    grid = (6, 5, 7)
    beta = rng.standard_normal(grid + (n_orb,))
    d = P.spline_desc_init(SKEW, grid, n_orb, dtype)
    tab = table_from_oracle(d, beta, dtype)
    n = 37
    pos = to_dev(rng.uniform(-5, 5, size=(n, 3)))
    od = torch.float64 if dtype == "f64" else torch.float32
    guard = 64
    opls = {"f64": (1, 2), "f32": (1, 2, 4), "bf16": (2, 4, 8)}[dtype]
    for g in (2, 8, 64):
        for opl in opls:
            say("guard band", dtype, n_orb, g, opl)
            bufs = [torch.full((k * n * n_orb + guard,), 7.25, dtype=od, device=DEV) for k in (1, 3, 1)]
            v, gr, lp = (bufs[0][:n * n_orb].view(n, n_orb), bufs[1][:3 * n * n_orb].view(n, 3, n_orb),
                         bufs[2][:n * n_orb].view(n, n_orb))
            P.spline_eval_vgl(d, tab, pos, v, gr, lp, tile=(g, opl))
            torch.cuda.synchronize()
            for b, k in zip(bufs, (1, 3, 1)):
                assert torch.all(b[k * n * n_orb:] == 7.25)
            assert torch.isfinite(v).all() and torch.isfinite(gr).all() and torch.isfinite(lp).all()
    vb = torch.full((n * n_orb + guard,), 7.25, dtype=od, device=DEV)
    P.spline_eval_v(d, tab, pos, vb[:n * n_orb].view(n, n_orb))
    torch.cuda.synchronize()
    assert torch.all(vb[n * n_orb:] == 7.25)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_backward_deterministic_matches_oracle_and_repeats(case, dtype):
    """SPL_DETERMINISTIC: cell-sorted accumulation (row tiles, or bricks for the 2.9 points per cell of
    the ragged case) with ragged tails (5, 7, 9 cells per axis there), non-finite points; equal to the
    oracle and bitwise equal across runs."""
    d = _desc(case, dtype)
    tab = table_from_oracle(d, case["beta"], dtype, case["lbeta"])
    bq = oq.quantized(case["beta"], dtype)
    lq = None if case["lbeta"] is None else oq.quantized(case["lbeta"], dtype)
    rng = np.random.default_rng(104)
    pos = case["pos"][:900]
    n, o = pos.shape[0], d.n_orb
    gv, gg, gl = rng.standard_normal((n, o)), rng.standard_normal((n, 3, o)), rng.standard_normal((n, o))
    od = torch.float64 if dtype == "f64" else torch.float32
    args = (to_dev(gv, od), to_dev(gg, od), to_dev(gl, od))
    say("deterministic backward", case["name"], dtype)
    runs = []
    for _ in range(3):
        gt, gp = P.spline_eval_vgl_backward(d, tab, to_dev(pos), *args, flags=P.SPL_DETERMINISTIC)
        torch.cuda.synchronize()
        runs.append((gt.clone(), gp.clone()))
    for gt, gp in runs[1:]:
        assert torch.equal(gt, runs[0][0])
        assert torch.equal(torch.nan_to_num(gp, nan=7.0), torch.nan_to_num(runs[0][1], nan=7.0))
    rb, rlb, rp = oadj.vgl_backward(bq, case["lattice"], pos, gv, gg, gl, lap_beta=lq)
    got = runs[0][0].double().cpu().numpy()[..., :o]
    tol = 1e-12 if dtype == "f64" else 2e-5
    assert normwise(got[0], rb) <= tol
    if rlb is not None:
        assert normwise(got[1], rlb) <= tol
    pad = runs[0][0].double().cpu().numpy()[..., o:]
    assert pad.size == 0 or np.all(pad == 0.0)
    ok = np.all(np.isfinite(pos), axis=1)
    gp = runs[0][1].cpu().numpy()
    assert np.isnan(gp[~ok]).all()
    smooth = ok & off_knots(case["lattice"], d.grid, pos)
    assert normwise(gp[smooth], rp[smooth]) <= (1e-10 if dtype == "f64" else 1e-4)


def test_backward_deterministic_many_points_per_cell():
    """Clustered points (about 60 per occupied cell): sorted accumulation equals the atomic form."""
    rng = np.random.default_rng(105)
    grid = (8, 8, 12)
    beta = rng.standard_normal(grid + (33,))
    d = P.spline_desc_init(SKEW, grid, 33, "f64")
    tab = table_from_oracle(d, beta, "f64")
    centers = rng.uniform(0, 1, size=(40, 3))
    s = (centers[rng.integers(0, 40, 6000)] + rng.normal(0, 0.01, size=(6000, 3))) % 1.0
    pos = s @ SKEW
    gv = rng.standard_normal((6000, 33))
    say("deterministic backward, clustered points")
    a, _ = P.spline_eval_vgl_backward(d, tab, to_dev(pos), to_dev(gv), want_pos=False, flags=P.SPL_DETERMINISTIC)
    b, _ = P.spline_eval_vgl_backward(d, tab, to_dev(pos), to_dev(gv), want_pos=False)
    torch.cuda.synchronize()
    rb, _, _ = oadj.vgl_backward(beta, SKEW, pos, gv)
    assert normwise(a.cpu().numpy()[0, ..., :33], rb) < 1e-12
    assert normwise(b.cpu().numpy()[0, ..., :33], rb) < 1e-12


@pytest.mark.parametrize("n_orb", [37, 70])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_backward_deterministic_row_tiles(dtype, n_orb):
    """Under 2.5 points per cell the deterministic adjoint forms each tile of 4 x 4 x 4 table rows from
    the points of the cells whose blocks reach it: axes of 4 and 6 cells (the window is the whole axis;
    6 leaves a last tile of 2 rows) and of 19 (a window of 7 of them; a last tile of 3 rows), clustered
    points so that some windows hold several batches of 32 points and some tiles receive none, every
    upstream term with the separate Laplacian table, a non-finite point, and orbital counts that leave
    waves of a workgroup partly or wholly past the last orbital.  Oracle parity and a bitwise repeat."""
    rng = np.random.default_rng(113)
    grid = (4, 6, 19)
    n = 2 * int(np.prod(grid))                          # 2 points per cell on average: the row-tile form
    beta = rng.standard_normal(grid + (n_orb,))
    lbeta = rng.standard_normal(grid + (n_orb,))
    d = P.spline_desc_init(SKEW, grid, n_orb, dtype, has_lap=True)
    tab = table_from_oracle(d, beta, dtype, lbeta)
    bq, lq = oq.quantized(beta, dtype), oq.quantized(lbeta, dtype)
    centers = np.array([[0.1, 0.2, 0.1], [0.6, 0.7, 0.15], [0.3, 0.4, 0.2]])
    s = (centers[rng.integers(0, 3, n)] + rng.normal(0, 0.05, size=(n, 3))) % 1.0
    pos = s @ SKEW
    pos[5] = np.nan
    i0, _, ok = oeval.reduced_coordinates(SKEW, grid, pos)
    # points of each tile's window: cells within -2 .. +4 of the tile's first row along every axis
    win = []
    for tx in range(0, grid[0], 4):
        for ty in range(0, grid[1], 4):
            for tz in range(0, grid[2], 4):
                near = np.ones(n, bool)
                for ax, t0 in enumerate((tx, ty, tz)):
                    near &= ((i0[:, ax] - (t0 - 2)) % grid[ax]) <= 6 if grid[ax] >= 7 else True
                win.append(int((near & ok).sum()))
    assert max(win) > 2 * 32 and min(win) == 0
    gv, gg, gl = rng.standard_normal((n, n_orb)), rng.standard_normal((n, 3, n_orb)), rng.standard_normal((n, n_orb))
    od = torch.float64 if dtype == "f64" else torch.float32
    args = (to_dev(gv, od), to_dev(gg, od), to_dev(gl, od))
    say("deterministic backward, row tiles", dtype, n_orb)
    runs = []
    for _ in range(2):
        gt, _ = P.spline_eval_vgl_backward(d, tab, to_dev(pos), *args, want_pos=False, flags=P.SPL_DETERMINISTIC)
        torch.cuda.synchronize()
        runs.append(gt.clone())
    assert torch.equal(runs[0], runs[1])
    rb, rlb, _ = oadj.vgl_backward(bq, SKEW, pos[ok], gv[ok], gg[ok], gl[ok], lap_beta=lq)
    got = runs[0].double().cpu().numpy()
    tol = 1e-12 if dtype == "f64" else 2e-5
    assert normwise(got[0, ..., :n_orb], rb) <= tol
    assert normwise(got[1, ..., :n_orb], rlb) <= tol
    assert np.all(got[..., n_orb:] == 0.0)


@pytest.mark.parametrize("n_orb", [37, 38])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_backward_deterministic_dense_path(dtype, n_orb):
    """At 2.5 or more points per cell the deterministic adjoint sums the cell blocks of every brick of
    2 x 2 x 2 cells into a 5 x 5 x 5-row region in the workspace and gathers the regions per table row
    (not per row tile): oracle parity with the separate Laplacian table and every upstream term, an
    odd or even orbital count, a ragged grid (odd cell counts leave partial bricks; 5 cells wrap a region onto
    itself), repeatable bit for bit.  An even orbital count takes FP32's paired columns."""
    rng = np.random.default_rng(107)
    grid, n = (6, 5, 7), 2000
    beta = rng.standard_normal(grid + (n_orb,))
    lbeta = rng.standard_normal(grid + (n_orb,))
    d = P.spline_desc_init(SKEW, grid, n_orb, dtype, has_lap=True)
    tab = table_from_oracle(d, beta, dtype, lbeta)
    bq, lq = oq.quantized(beta, dtype), oq.quantized(lbeta, dtype)
    pos = rng.uniform(-3, 3, size=(n, 3)) @ SKEW / 3.0
    pos[17] = np.nan                                    # a non-finite point contributes nothing
    gv, gg, gl = rng.standard_normal((n, n_orb)), rng.standard_normal((n, 3, n_orb)), rng.standard_normal((n, n_orb))
    od = torch.float64 if dtype == "f64" else torch.float32
    args = (to_dev(gv, od), to_dev(gg, od), to_dev(gl, od))
    nb = P.spline_backward_work_bytes(d, n, P.SPL_DETERMINISTIC)
    n_bricks = np.prod([(k + 1) // 2 for k in grid])
    assert nb >= n_bricks * 125 * d.o_pad * (8 if dtype == "f64" else 4)   # the region workspace
    say("deterministic backward, dense path", dtype)
    runs = []
    for _ in range(2):
        gt, _ = P.spline_eval_vgl_backward(d, tab, to_dev(pos), *args, want_pos=False, flags=P.SPL_DETERMINISTIC)
        torch.cuda.synchronize()
        runs.append(gt.clone())
    assert torch.equal(runs[0], runs[1])
    ok = np.all(np.isfinite(pos), axis=1)
    rb, rlb, _ = oadj.vgl_backward(bq, SKEW, pos[ok], gv[ok], gg[ok], gl[ok], lap_beta=lq)
    got = runs[0].double().cpu().numpy()
    tol = 1e-12 if dtype == "f64" else 2e-5
    assert normwise(got[0, ..., :n_orb], rb) <= tol
    assert normwise(got[1, ..., :n_orb], rlb) <= tol
    assert np.all(got[..., n_orb:] == 0.0)


@pytest.mark.parametrize("n_orb", [45, 46])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_backward_dense_value_and_laplacian_terms(dtype, n_orb):
    """The fit's term set (value and Laplacian upstream gradients, derivative Laplacian) on the dense
    path, whose row weights are fixed at compile time: clustered points, so that some cells hold
    several batches of 32 points and many cells and whole bricks hold none; oracle parity and a
    bitwise repeat.  An even orbital count takes FP32's paired columns (two adjacent orbitals per
    lane), with a partly filled last group of orbitals."""
    rng = np.random.default_rng(109)
    grid = (10, 8, 9)
    beta = rng.standard_normal(grid + (n_orb,))
    d = P.spline_desc_init(SKEW, grid, n_orb, dtype)
    tab = table_from_oracle(d, beta, dtype)
    bq = oq.quantized(beta, dtype)
    centers = rng.uniform(0, 1, size=(6, 3))
    n = 4 * int(np.prod(grid))                          # 4 points per cell on average: the dense path
    s = (centers[rng.integers(0, 6, n)] + rng.normal(0, 0.04, size=(n, 3))) % 1.0
    pos = s @ SKEW
    i0, _, _ = oeval.reduced_coordinates(SKEW, grid, pos)
    per_cell = np.bincount(np.ravel_multi_index(i0.T, grid), minlength=int(np.prod(grid)))
    bricks = [(k + 1) // 2 for k in grid]
    per_brick = np.bincount(np.ravel_multi_index((i0 // 2).T, bricks), minlength=int(np.prod(bricks)))
    assert per_cell.max() > 2 * 32 and (per_brick == 0).any()
    gv, gl = rng.standard_normal((n, n_orb)), rng.standard_normal((n, n_orb))
    od = torch.float64 if dtype == "f64" else torch.float32
    say("deterministic backward, dense path, value and Laplacian terms", dtype)
    runs = []
    for _ in range(2):
        gt, _ = P.spline_eval_vgl_backward(d, tab, to_dev(pos), to_dev(gv, od), None, to_dev(gl, od), want_pos=False,
                                           flags=P.SPL_DETERMINISTIC)
        torch.cuda.synchronize()
        runs.append(gt.clone())
    assert torch.equal(runs[0], runs[1])
    rb, _, _ = oadj.vgl_backward(bq, SKEW, pos, gv, None, gl)
    got = runs[0].double().cpu().numpy()
    assert normwise(got[0, ..., :n_orb], rb) <= (1e-12 if dtype == "f64" else 2e-5)
    assert np.all(got[..., n_orb:] == 0.0)
