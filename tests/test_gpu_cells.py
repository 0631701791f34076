"""spline_eval_vgl_cells: the forward evaluation cell by cell on the matrix cores, against the
per-point kernel (spline_eval_vgl) and the FP64 oracle, on dense and sparse point sets."""
import math

import numpy as np
import pytest
import torch

import paper_1309_6250_amd as P
from oracle import evaluate as oeval, quantize as oq
from workloads import config
from gpu_helpers import say, to_dev, table_from_oracle, normwise, DEV

pytestmark = pytest.mark.gpu

SKEW = np.array([[7.0, 0.4, -0.3], [1.1, 6.2, 0.5], [-0.6, 0.9, 8.3]])
TOL = {"f64": 1e-12, "f32": 3e-6, "bf16": 3e-6}      # against the per-point kernel (other summation order)


def _case(grid, n_orb, n, dtype, has_lap, seed):
    rng = np.random.default_rng(seed)
    beta = rng.standard_normal(grid + (n_orb,))
    lbeta = rng.standard_normal(grid + (n_orb,)) if has_lap else None
    d = P.spline_desc_init(SKEW, grid, n_orb, dtype, has_lap=has_lap)
    tab = table_from_oracle(d, beta, dtype, lbeta)
    pos = rng.uniform(-1.5, 1.5, size=(n, 3)) @ SKEW
    return d, tab, pos, beta, lbeta


@pytest.mark.parametrize("has_lap", [False, True], ids=["lap-from-derivatives", "lap-table"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape", [((6, 5, 7), 37, 2000), ((16, 16, 16), 20, 300)], ids=["dense", "sparse"])
def test_cells_match_per_point_kernel(shape, dtype, has_lap):
    grid, n_orb, n = shape
    d, tab, pos, _, _ = _case(grid, n_orb, n, dtype, has_lap, 110)
    pos[5] = np.nan
    pos[n - 3] = [1e300, 0.0, 0.0]
    x = to_dev(pos)
    say("cells forward", grid, n_orb, n, dtype, has_lap)
    rv, rg, rl = P.spline_eval_vgl(d, tab, x)
    v, g, l = P.spline_eval_vgl_cells(d, tab, x)
    torch.cuda.synchronize()
    bad = ~np.all(np.isfinite(pos), axis=1)      # a huge finite coordinate folds into the cell like any other
    for got, ref in ((v, rv), (g, rg), (l, rl)):
        got, ref = got.double().cpu().numpy(), ref.double().cpu().numpy()
        assert np.isnan(got[bad]).all()
        assert normwise(got[~bad], ref[~bad]) <= TOL[dtype]


@pytest.mark.parametrize("outputs", ["v", "l", "vl", "g"])
def test_cells_skip_outputs(outputs):
    d, tab, pos, _, _ = _case((6, 5, 7), 37, 1500, "f32", False, 111)
    x = to_dev(pos)
    say("cells forward, outputs", outputs)
    rv, rg, rl = P.spline_eval_vgl(d, tab, x)
    v, g, l = P.spline_eval_vgl_cells(d, tab, x, outputs=outputs)
    torch.cuda.synchronize()
    for key, got, ref in (("v", v, rv), ("g", g, rg), ("l", l, rl)):
        if key in outputs:
            assert normwise(got.double().cpu().numpy(), ref.double().cpu().numpy()) <= TOL["f32"]
        else:
            assert got is None


def test_cells_match_oracle():
    d, tab, pos, beta, _ = _case((6, 5, 7), 37, 1200, "f64", False, 112)
    say("cells forward against the oracle")
    v, g, l = P.spline_eval_vgl_cells(d, tab, to_dev(pos))
    torch.cuda.synchronize()
    ov, og, ol = oeval.eval_vgl(beta, SKEW, pos)
    assert normwise(v.cpu().numpy(), ov) < 1e-12
    assert normwise(g.cpu().numpy(), og) < 1e-12
    assert normwise(l.cpu().numpy(), ol) < 1e-12


@pytest.mark.parametrize("has_lap", [False, True], ids=["lap-from-derivatives", "lap-table"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_cells_match_oracle_elementwise(dtype, has_lap):
    """Kernel parity of the matrix-core forward against the oracle on the same stored (quantized)
    table, element by element: |err| <= 2 * 64 * u_acc * sum |w| |beta| plus the movement allowed by
    rounding of the grid coordinate (the per-point kernel's bound; oracle.evaluate.eval_abs_bound)."""
    from gpu_helpers import assert_elementwise, coordinate_rounding, U_ACC
    d, tab, pos, beta, lbeta = _case((6, 5, 7), 37, 1200, dtype, has_lap, 115)
    say("cells forward against the oracle, elementwise", dtype, has_lap)
    v, g, l = P.spline_eval_vgl_cells(d, tab, to_dev(pos))
    torch.cuda.synchronize()
    bq = oq.quantized(beta, dtype)
    lq = None if lbeta is None else oq.quantized(lbeta, dtype)
    ref = oeval.eval_vgl(bq, SKEW, pos, lap_beta=lq)
    bnd = oeval.eval_abs_bound(bq, SKEW, pos, lap_beta=lq)
    crd = oeval.coordinate_error_bound(bq, SKEW, pos, coordinate_rounding(d, SKEW, pos, dtype), lap_beta=lq)
    fac = 2 * 64 * U_ACC[dtype] + (0.0 if dtype == "f64" else 2.0**-24)
    for name, got, r, b, c in zip(("V", "grad", "lap"), (v, g, l), ref, bnd, crd):
        assert_elementwise(got.double().cpu().numpy(), r, b + c / fac, fac, name)


@pytest.mark.timeout(600)
def test_cells_at_fit_size():
    """10^6 points in 32^3 cells (FP32): value and Laplacian against the per-point kernel."""
    w = config(4)
    s = w.system
    x = to_dev(w.positions())
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f32")
    tab = P.spline_build(d, to_dev(s.grid_values()))
    say("cells forward at 1e6 points")
    v, _, l = P.spline_eval_vgl_cells(d, tab, x, outputs="vl")
    rv, _, rl = P.spline_eval_vgl(d, tab, x)
    torch.cuda.synchronize()
    assert normwise(v.double().cpu().numpy(), rv.double().cpu().numpy()) < 3e-6
    assert normwise(l.double().cpu().numpy(), rl.double().cpu().numpy()) < 3e-6


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_cells_smallest_grid_and_all_nonfinite(dtype):
    """N = 4 along two axes (a cell's block then covers the whole axis): cell-wise forward against
    the per-point kernel and the oracle; the deterministic adjoint's dense form against the oracle;
    a call whose points are all non-finite gives NaN everywhere and adds nothing."""
    from oracle import adjoint as oadj
    d, tab, pos, beta, _ = _case((4, 5, 4), 9, 800, dtype, False, 113)
    x = to_dev(pos)
    say("cells on a 4x5x4 grid", dtype)
    rv, rg, rl = P.spline_eval_vgl(d, tab, x)
    v, g, l = P.spline_eval_vgl_cells(d, tab, x)
    torch.cuda.synchronize()
    for got, ref in ((v, rv), (g, rg), (l, rl)):
        assert normwise(got.double().cpu().numpy(), ref.double().cpu().numpy()) <= TOL[dtype]
    if dtype == "f64":
        ov, og, ol = oeval.eval_vgl(beta, SKEW, pos)
        assert normwise(v.cpu().numpy(), ov) < 1e-12 and normwise(l.cpu().numpy(), ol) < 1e-12
    rng = np.random.default_rng(114)
    gv = rng.standard_normal((pos.shape[0], 9))
    od = torch.float64 if dtype == "f64" else torch.float32
    gt, _ = P.spline_eval_vgl_backward(d, tab, x, to_dev(gv, od), want_pos=False, flags=P.SPL_DETERMINISTIC)
    torch.cuda.synchronize()
    rb, _, _ = oadj.vgl_backward(oq.quantized(beta, dtype), SKEW, pos, gv)
    assert normwise(gt.double().cpu().numpy()[0, ..., :9], rb) <= (1e-12 if dtype == "f64" else 2e-5)
    bad = to_dev(np.full((50, 3), np.nan))
    v, g, l = P.spline_eval_vgl_cells(d, tab, bad)
    gt, _ = P.spline_eval_vgl_backward(d, tab, bad, torch.ones((50, 9), dtype=od, device=DEV), want_pos=False,
                                       flags=P.SPL_DETERMINISTIC)
    torch.cuda.synchronize()
    assert torch.isnan(v).all() and torch.isnan(g).all() and torch.isnan(l).all()
    assert torch.count_nonzero(gt) == 0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sort_reuse_is_bitwise(dtype):
    """SPL_REUSE_SORT: the forward and the deterministic adjoint on a workspace that already holds
    the cell sort of the same points (made by either call) give the same bits as with a fresh sort,
    in the dense and in the sparse adjoint form."""
    od = torch.float64 if dtype == "f64" else torch.float32
    for grid, n in (((6, 5, 7), 2000), ((16, 16, 16), 300)):
        d, tab, pos, _, _ = _case(grid, 37, n, dtype, True, 115)
        pos[7] = np.nan
        x = to_dev(pos)
        rng = np.random.default_rng(116)
        gv, gl = to_dev(rng.standard_normal((n, 37)), od), to_dev(rng.standard_normal((n, 37)), od)
        say("sort reuse", grid, n, dtype)
        nb = max(P.spline_cells_work_bytes(d, n), P.spline_backward_work_bytes(d, n, P.SPL_DETERMINISTIC))
        work = torch.empty(nb, dtype=torch.uint8, device=DEV)
        fresh_f = P.spline_eval_vgl_cells(d, tab, x)
        fresh_b, _ = P.spline_eval_vgl_backward(d, tab, x, gv, None, gl, want_pos=False, flags=P.SPL_DETERMINISTIC)
        P.spline_eval_vgl_cells(d, tab, x, work=work)                       # sorts into work
        reuse_b, _ = P.spline_eval_vgl_backward(d, tab, x, gv, None, gl, want_pos=False, work=work,
                                                flags=P.SPL_DETERMINISTIC | P.SPL_REUSE_SORT)
        reuse_f = P.spline_eval_vgl_cells(d, tab, x, work=work, flags=P.SPL_REUSE_SORT)
        torch.cuda.synchronize()
        assert torch.equal(reuse_b, fresh_b)
        for a, b in zip(reuse_f, fresh_f):
            assert torch.equal(torch.nan_to_num(a, nan=3.0), torch.nan_to_num(b, nan=3.0))


@pytest.mark.parametrize("terms", ["vl", "v", "l"])
@pytest.mark.parametrize("has_lap", [False, True], ids=["lap-from-derivatives", "lap-table"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape", [((6, 5, 7), 37, 2000), ((16, 16, 16), 20, 300)], ids=["dense", "sparse"])
def test_fit_terms_match_forward_then_misfit(shape, dtype, has_lap, terms):
    """spline_fit_terms_cells against the two-pass form (cell-wise forward, then spline_misfit on
    each output): the gradients 2 w (y - t) bit for bit, the loss (accumulated into) to FP64
    summation accuracy, and the loss itself repeatable bit for bit, also on a reused sort."""
    grid, n_orb, n = shape
    d, tab, pos, _, _ = _case(grid, n_orb, n, dtype, has_lap, 117)
    x = to_dev(pos)
    od = torch.float64 if dtype == "f64" else torch.float32
    rng = np.random.default_rng(118)
    tv = to_dev(rng.standard_normal((n, n_orb)), od) if "v" in terms else None
    tl = to_dev(3.0 * rng.standard_normal((n, n_orb)), od) if "l" in terms else None
    wv, wl = 0.37, 0.011
    say("fit terms", grid, n_orb, n, dtype, has_lap, terms)
    v, _, l = P.spline_eval_vgl_cells(d, tab, x, outputs=terms)
    ref_loss = torch.full((1,), 1.5, dtype=torch.float64, device=DEV)
    rgv = P.spline_misfit(d, v, tv, wv, ref_loss) if tv is not None else None
    rgl = P.spline_misfit(d, l, tl, wl, ref_loss) if tl is not None else None
    nb = P.spline_cells_work_bytes(d, n)
    work = torch.empty(nb, dtype=torch.uint8, device=DEV)
    loss = torch.full((1,), 1.5, dtype=torch.float64, device=DEV)
    gv, gl, _ = P.spline_fit_terms_cells(d, tab, x, tv, wv, tl, wl, loss=loss, work=work)
    loss2 = torch.full((1,), 1.5, dtype=torch.float64, device=DEV)
    gv2, gl2, _ = P.spline_fit_terms_cells(d, tab, x, tv, wv, tl, wl, loss=loss2, work=work, flags=P.SPL_REUSE_SORT)
    torch.cuda.synchronize()
    for got, got2, ref in ((gv, gv2, rgv), (gl, gl2, rgl)):
        if ref is None:
            assert got is None and got2 is None
        else:
            assert torch.equal(got, ref) and torch.equal(got2, ref)
    assert abs(float(loss) - float(ref_loss)) <= 1e-13 * float(ref_loss)
    assert float(loss) == float(loss2)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fit_terms_against_oracle(dtype):
    """The loss of spline_fit_terms_cells against the oracle's values and Laplacians: w_v sum
    (V - t_v)^2 + w_lap sum (lap - t_lap)^2 with V and lap evaluated in FP64 from the table the
    kernel reads (within the output type's rounding of each residual)."""
    d, tab, pos, beta, _ = _case((6, 5, 7), 37, 1500, dtype, False, 119)
    n = pos.shape[0]
    rng = np.random.default_rng(120)
    ov, _, ol = oeval.eval_vgl(oq.quantized(beta, dtype), SKEW, pos)
    t_v = ov + 0.1 * rng.standard_normal(ov.shape)
    t_l = ol + 0.5 * rng.standard_normal(ol.shape)
    od = torch.float64 if dtype == "f64" else torch.float32
    nd = np.float64 if dtype == "f64" else np.float32
    wv, wl = 0.7, 0.05
    say("fit terms against the oracle", dtype)
    gv, gl, loss = P.spline_fit_terms_cells(d, tab, to_dev(pos), to_dev(t_v, od), wv, to_dev(t_l, od), wl)
    torch.cuda.synchronize()
    tv, tl = t_v.astype(nd).astype(np.float64), t_l.astype(nd).astype(np.float64)
    ref = wv * np.sum((ov - tv) ** 2) + wl * np.sum((ol - tl) ** 2)
    tol = 1e-11 if dtype == "f64" else 1e-5
    assert abs(float(loss) - ref) <= tol * ref
    assert normwise(gv.double().cpu().numpy(), 2 * wv * (ov - tv)) <= tol
    assert normwise(gl.double().cpu().numpy(), 2 * wl * (ol - tl)) <= tol


def test_fit_terms_nonfinite_points():
    """A non-finite point: its gradient rows are NaN and the loss is NaN; all points non-finite
    likewise; the finite points' gradients are unaffected."""
    d, tab, pos, _, _ = _case((6, 5, 7), 9, 700, "f32", False, 121)
    pos[11] = [np.inf, 0.0, 0.0]
    x = to_dev(pos)
    rng = np.random.default_rng(122)
    tv = to_dev(rng.standard_normal((700, 9)), torch.float32)
    say("fit terms, non-finite points")
    gv, _, loss = P.spline_fit_terms_cells(d, tab, x, tv, 1.0)
    v, _, _ = P.spline_eval_vgl_cells(d, tab, x, outputs="v")
    rl = torch.zeros(1, dtype=torch.float64, device=DEV)
    rg = P.spline_misfit(d, v, tv, 1.0, rl)
    bad = to_dev(np.full((40, 3), np.nan))
    tb = torch.zeros((40, 9), dtype=torch.float32, device=DEV)
    gb, _, lb = P.spline_fit_terms_cells(d, tab, bad, tb, 1.0)
    torch.cuda.synchronize()
    assert torch.isnan(gv[11]).all() and math.isnan(float(loss))
    keep = torch.ones(700, dtype=torch.bool)
    keep[11] = False
    assert torch.equal(gv[keep.to(DEV)], rg[keep.to(DEV)])
    assert torch.isnan(gb).all() and math.isnan(float(lb))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_cells_outputs_at_odd_offsets(dtype):
    """Outputs (and the fit terms' targets and gradients) one element past an 8-byte boundary, with
    an even orbital count: the same bits as aligned buffers (the kernel then stores value by value
    instead of in pairs)."""
    n, n_orb = 1500, 20
    d, tab, pos, _, _ = _case((6, 5, 7), n_orb, n, dtype, False, 123)
    x = to_dev(pos)
    m = n * n_orb

    def odd(k=1):
        return torch.empty(k * m + 1, dtype=torch.float32, device=DEV)[1:]
    say("cells forward, outputs at odd offsets", dtype)
    v, g, l = P.spline_eval_vgl_cells(d, tab, x)
    vo, go, lo = odd(), odd(3), odd()
    P.spline_eval_vgl_cells(d, tab, x, vo, go, lo)
    rng = np.random.default_rng(124)
    tv = to_dev(rng.standard_normal((n, n_orb)), torch.float32)
    tl = to_dev(rng.standard_normal((n, n_orb)), torch.float32)
    gv, gl, loss = P.spline_fit_terms_cells(d, tab, x, tv, 0.5, tl, 0.25)
    tvo, tlo = odd(), odd()
    tvo.copy_(tv.reshape(-1))
    tlo.copy_(tl.reshape(-1))
    gvo, glo = odd(), odd()
    _, _, loss_o = P.spline_fit_terms_cells(d, tab, x, tvo, 0.5, tlo, 0.25, g_v=gvo, g_lap=glo)
    torch.cuda.synchronize()
    assert vo.data_ptr() % 8 == 4
    for a, b in ((v, vo), (g, go), (l, lo), (gv, gvo), (gl, glo)):
        assert torch.equal(a.reshape(-1), b)
    assert float(loss) == float(loss_o)


def _fit_gradient_reference(d, tab, x, tv, wv, tl, wl, loss0, gtable0):
    """spline_fit_terms_cells, then the deterministic adjoint of its upstream gradients."""
    loss = torch.full((1,), loss0, dtype=torch.float64, device=DEV)
    gv, gl, _ = P.spline_fit_terms_cells(d, tab, x, tv, wv, tl, wl, loss=loss)
    gt = gtable0.clone()
    P.spline_eval_vgl_backward(d, tab, x, gv, None, gl, gt, None, want_pos=False, flags=P.SPL_DETERMINISTIC)
    return gt, loss


@pytest.mark.parametrize("n_orb", [45, 70, 128])
def test_fit_gradient_one_pass_equals_terms_then_adjoint(n_orb):
    """spline_fit_gradient_cells (forward, misfit and adjoint of each batch in one kernel) against
    spline_fit_terms_cells followed by the deterministic adjoint: the coefficient gradient and the
    loss, both accumulated into, bit for bit; again on a reused sort.  Clustered points, so cells hold
    up to several batches of 32 and many cells and bricks none; a ragged grid; 45 orbitals leave a
    partial orbital group, 70 a wave without one."""
    rng = np.random.default_rng(131)
    grid = (10, 8, 9)
    beta = rng.standard_normal(grid + (n_orb,))
    d = P.spline_desc_init(SKEW, grid, n_orb, "f32")
    tab = table_from_oracle(d, beta, "f32")
    centers = rng.uniform(0, 1, size=(6, 3))
    n = 4 * int(np.prod(grid))
    pos = ((centers[rng.integers(0, 6, n)] + rng.normal(0, 0.05, size=(n, 3))) % 1.0) @ SKEW
    x = to_dev(pos)
    tv = to_dev(rng.standard_normal((n, n_orb)), torch.float32)
    tl = to_dev(5.0 * rng.standard_normal((n, n_orb)), torch.float32)
    wv, wl = 0.37, 0.011
    g0 = to_dev(rng.standard_normal(P.table_shape(d)), torch.float32)
    say("one-pass fit gradient", grid, n_orb, n)
    rgt, rloss = _fit_gradient_reference(d, tab, x, tv, wv, tl, wl, 0.25, g0)
    work = torch.empty(P.spline_fit_gradient_work_bytes(d, n), dtype=torch.uint8, device=DEV)
    outs = []
    for flags in (0, P.SPL_REUSE_SORT):
        gt = g0.clone()
        loss = torch.full((1,), 0.25, dtype=torch.float64, device=DEV)
        P.spline_fit_gradient_cells(d, tab, x, tv, wv, tl, wl, gtable=gt, loss=loss, work=work, flags=flags)
        outs.append((gt, loss))
    torch.cuda.synchronize()
    for gt, loss in outs:
        assert torch.equal(gt, rgt)
        assert float(loss) == float(rloss)


@pytest.mark.timeout(600)
def test_fit_gradient_one_pass_at_fit_size():
    """The 64-atom fit workload (10^6 points, 128 orbitals, 32^3 FP32 table): one pass equals fit terms
    then adjoint bit for bit, gradient and loss, over four calls (fresh and reused sort)."""
    w = config(4)
    s = w.system
    x = to_dev(w.positions())
    n = x.shape[0]
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f32")
    tab = P.spline_build(d, to_dev(s.grid_values()))
    g = torch.Generator(device=DEV).manual_seed(132)
    tv = torch.randn((n, s.n_orb), device=DEV, generator=g)
    tl = 10.0 * torch.randn((n, s.n_orb), device=DEV, generator=g)
    g0 = torch.zeros(P.table_shape(d), dtype=torch.float32, device=DEV)
    say("one-pass fit gradient at fit size")
    rgt, rloss = _fit_gradient_reference(d, tab, x, tv, 1.0, tl, 1e-3, 0.0, g0)
    work = torch.empty(P.spline_fit_gradient_work_bytes(d, n), dtype=torch.uint8, device=DEV)
    for flags in (0, P.SPL_REUSE_SORT, P.SPL_REUSE_SORT, 0):    # repeated, on a fresh and a reused sort
        gt, loss = P.spline_fit_gradient_cells(d, tab, x, tv, 1.0, tl, 1e-3, work=work, flags=flags)
        torch.cuda.synchronize()
        assert torch.equal(gt, rgt)
        assert float(loss) == float(rloss)


def test_fit_gradient_one_pass_nonfinite_and_unsupported():
    """A non-finite point makes the loss NaN and leaves the gradient equal to the two-kernel path's;
    FP64 tables, a separate Laplacian table and sparse points are refused with SPL_EUNSUPPORTED."""
    rng = np.random.default_rng(133)
    grid, n_orb, n = (6, 5, 7), 33, 1500
    d = P.spline_desc_init(SKEW, grid, n_orb, "f32")
    tab = table_from_oracle(d, rng.standard_normal(grid + (n_orb,)), "f32")
    pos = rng.uniform(0, 1, size=(n, 3)) @ SKEW
    pos[7] = [np.nan, 0.0, 0.0]
    x = to_dev(pos)
    tv = to_dev(rng.standard_normal((n, n_orb)), torch.float32)
    tl = to_dev(rng.standard_normal((n, n_orb)), torch.float32)
    g0 = torch.zeros(P.table_shape(d), dtype=torch.float32, device=DEV)
    say("one-pass fit gradient, non-finite point and refusals")
    rgt, rloss = _fit_gradient_reference(d, tab, x, tv, 1.0, tl, 0.5, 0.0, g0)
    gt, loss = P.spline_fit_gradient_cells(d, tab, x, tv, 1.0, tl, 0.5)
    torch.cuda.synchronize()
    assert math.isnan(float(loss)) and math.isnan(float(rloss))
    assert torch.equal(gt, rgt)
    for dd, nn in ((P.spline_desc_init(SKEW, grid, n_orb, "f64"), n),
                   (P.spline_desc_init(SKEW, grid, n_orb, "f32", has_lap=True), n), (d, 100)):
        od = torch.float64 if dd.dtype == P.SPL_F64 else torch.float32
        tt = torch.zeros((nn, n_orb), dtype=od, device=DEV)
        with pytest.raises(P.SplineError) as err:
            P.spline_fit_gradient_cells(dd, P.new_table(dd), x[:nn], tt, 1.0, tt, 1.0)
        assert err.value.code == P.SPL_EUNSUPPORTED



ORTHO = np.diag([7.0, 6.2, 8.3])    # orthogonal, axis-aligned lattice vectors: the metric is exactly diagonal


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_diagonal_metric_forms_against_oracle(dtype):
    """An orthorhombic cell along the Cartesian axes (the metric's and the Jacobian's off-diagonal
    entries exactly 0) takes the forms that skip their products: the cell-wise forward of V and lap and
    of all five outputs against the oracle's values; the deterministic adjoint of value and Laplacian
    upstream values, and of all five, at dense points (bricks) and at sparse points (row tiles),
    against the oracle's adjoint; and (FP32) the one-pass fit gradient against the oracle's loss and
    gradient, and against the fit terms followed by the adjoint (equal values).  A ragged grid and an
    odd orbital count."""
    from oracle import adjoint as oadj
    rng = np.random.default_rng(151)
    grid, n_orb, n = (6, 5, 7), 37, 2000
    beta = rng.standard_normal(grid + (n_orb,))
    d = P.spline_desc_init(ORTHO, grid, n_orb, dtype)
    assert d.metric[3] == 0.0 and d.metric[4] == 0.0 and d.metric[5] == 0.0
    assert all(d.jac[i] == 0.0 for i in (1, 2, 3, 5, 6, 7))
    tab = table_from_oracle(d, beta, dtype)
    bq = oq.quantized(beta, dtype)
    pos = rng.uniform(-3, 3, size=(n, 3)) @ ORTHO / 3.0
    x = to_dev(pos)
    od = torch.float64 if dtype == "f64" else torch.float32
    nd = np.float64 if dtype == "f64" else np.float32
    gv, gg, gl = rng.standard_normal((n, n_orb)), rng.standard_normal((n, 3, n_orb)), rng.standard_normal((n, n_orb))
    tol = 1e-12 if dtype == "f64" else 2e-5
    from gpu_helpers import assert_elementwise, coordinate_rounding, U_ACC
    ov, og, ol = oeval.eval_vgl(bq, ORTHO, pos)
    bnd = oeval.eval_abs_bound(bq, ORTHO, pos)
    crd = oeval.coordinate_error_bound(bq, ORTHO, pos, coordinate_rounding(d, ORTHO, pos, dtype))
    fac = 2 * 64 * U_ACC[dtype] + (0.0 if dtype == "f64" else 2.0**-24)
    for outputs in ("vl", "vgl"):                    # the cell-wise forward's diagonal forms, element by element
        say("diagonal metric: cell-wise forward", dtype, outputs)
        outs = P.spline_eval_vgl_cells(d, tab, x, outputs=outputs)
        torch.cuda.synchronize()
        for name, got, r, b, c in zip(("V", "grad", "lap"), outs, (ov, og, ol), bnd, crd):
            if got is not None:
                assert_elementwise(got.double().cpu().numpy(), r, b + c / fac, fac, name)
    for m in (n, 300):                               # 9.5 and 1.4 points per cell: bricks, row tiles
        for with_grad in (False, True):
            say("diagonal metric: deterministic adjoint", dtype, m, "points", "all terms" if with_grad else "V and L")
            gt, _ = P.spline_eval_vgl_backward(d, tab, x[:m], to_dev(gv[:m], od),
                                               to_dev(gg[:m], od) if with_grad else None, to_dev(gl[:m], od),
                                               want_pos=False, flags=P.SPL_DETERMINISTIC)
            torch.cuda.synchronize()
            rb, _, _ = oadj.vgl_backward(bq, ORTHO, pos[:m], gv[:m], gg[:m] if with_grad else None, gl[:m])
            assert normwise(gt.double().cpu().numpy()[0, ..., :n_orb], rb) <= tol
    if dtype == "f64":
        return
    t_v = (ov + 0.1 * rng.standard_normal(ov.shape)).astype(nd)
    t_l = (ol + 0.5 * rng.standard_normal(ol.shape)).astype(nd)
    wv, wl = 0.7, 0.05
    say("diagonal metric: one-pass fit gradient")
    tv, tl = to_dev(t_v, od), to_dev(t_l, od)
    gt1, loss = P.spline_fit_gradient_cells(d, tab, x, tv, wv, tl, wl)
    rgt, rloss = _fit_gradient_reference(d, tab, x, tv, wv, tl, wl, 0.0, torch.zeros_like(gt1))
    torch.cuda.synchronize()
    rv, rl = ov - t_v.astype(np.float64), ol - t_l.astype(np.float64)
    ref = wv * np.sum(rv ** 2) + wl * np.sum(rl ** 2)
    assert abs(float(loss) - ref) <= 1e-5 * ref
    rg, _, _ = oadj.vgl_backward(bq, ORTHO, pos, 2 * wv * rv, None, 2 * wl * rl)
    assert normwise(gt1.double().cpu().numpy()[0, ..., :n_orb], rg) <= 2e-5
    assert torch.equal(gt1, rgt)
    assert float(loss) == float(rloss)

# ---------------------------------------------------------------- the fit's Adam step
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_adam_step_matches_torch_adam(dtype):
    """spline_adam_step against torch.optim.Adam in FP64 on the CPU (the same hyperparameters), over
    three steps whose gradients differ in scale: an FP64 table to 1e-12 of its largest coefficient,
    FP32 to 2e-6, and BF16 coefficients (rounded back to BF16 every step, moments in FP32) to four
    units of their last place."""
    rng = np.random.default_rng(141)
    shape = (5, 6, 7, 16)
    p0 = rng.standard_normal(shape)
    grads = [rng.standard_normal(shape) * 10.0 ** k for k in (0, -2, 1)]
    lr, b1, b2, eps = 0.05, 0.9, 0.999, 1e-8
    ref = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([ref], lr=lr, betas=(b1, b2), eps=eps, foreach=False)
    store = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    mom = torch.float64 if dtype == "f64" else torch.float32
    p = torch.tensor(p0).to(store).to(DEV)
    m = torch.zeros(shape, dtype=mom, device=DEV)
    v = torch.zeros_like(m)
    say("Adam step", dtype)
    for k, g in enumerate(grads, 1):
        ref.grad = torch.tensor(g)
        opt.step()
        P.spline_adam_step(p, torch.tensor(g).to(mom).to(DEV), m, v, lr, k, beta1=b1, beta2=b2, eps=eps)
    torch.cuda.synchronize()
    got, want = p.double().cpu(), ref.detach()
    tol = {"f64": 1e-12, "f32": 2e-6, "bf16": 4 * 2.0 ** -8}[dtype]
    assert float((got - want).abs().max()) <= tol * float(want.abs().max())
