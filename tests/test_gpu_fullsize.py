"""Parity at the benchmark's full sizes and launch configuration (autotuned tiles).

The GPU evaluates whole workloads; the oracle recomputes a seeded sample of 256 points for a strided
set of orbitals that spans every column (every 7th and the last: all residues modulo the lanes'
orbital chunks, and every part of a tile's width; the interpolating build is independent per
orbital, so the oracle builds only those).
Where the oracle cannot follow (sums over 10^6 points), properties that hold at any size are
checked instead: the adjoint identity <g, J db> = <J^T g, db>, and batched = single-system.
"""
import numpy as np
import pytest
import torch

import paper_1309_6250_amd as P
from oracle import build as obuild, evaluate as oeval, quantize as oq
from workloads import config, batched_systems, make_system
from workloads.configs import A_MGO, cubic
from gpu_helpers import say, to_dev, normwise, DEV

pytestmark = pytest.mark.gpu

GATES = {"f64": (1e-10, 1e-10, 1e-10, 1e-10), "f32": (1e-5, 1e-5, 1e-5, 1e-5), "bf16": (5e-3, 1e-2, 5e-2, 5e-3)}


def _sample(n, k=256, seed=1309):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=k, replace=False))


def _columns(n_orb, stride=7):
    """Orbitals compared with the oracle: every `stride`-th and the last."""
    return np.unique(np.r_[np.arange(0, n_orb, stride), n_orb - 1])


def _take(out, idx, cols, dtype=np.float64):
    """The sampled points' outputs (V, grad, lap) for the columns `cols`, on the host."""
    it = torch.as_tensor(idx, device=DEV)
    v, g, l = (t.index_select(0, it).cpu().numpy() for t in out)
    return [v[:, cols].astype(dtype), g[:, :, cols].astype(dtype), l[:, cols].astype(dtype)]


@pytest.fixture(scope="module")
def si64():
    w = config(1)
    s = w.system
    f = s.grid_values()
    pos = w.positions()
    return dict(s=s, f=f, pos=pos, f_dev=to_dev(f), pos_dev=to_dev(pos))


@pytest.fixture(scope="module")
def mgo96():
    w = config(2)
    s = w.system
    f = s.grid_values()
    lf = s.grid_laplacian()
    pos = w.positions()
    return dict(s=s, f=f, lf=lf, pos=pos, f_dev=to_dev(f), lf_dev=to_dev(lf), pos_dev=to_dev(pos))


def _run_and_check(c, dtype, has_lap):
    s = c["s"]
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, dtype, has_lap=has_lap)
    say("full size", s.name, dtype, has_lap)
    tab = P.spline_build(d, c["f_dev"], c["lf_dev"] if has_lap else None)
    out = P.spline_eval_vgl(d, tab, c["pos_dev"])
    tile = P.spline_autotune(d, tab, c["pos_dev"], *out)           # the bench's launch shape
    out = P.spline_eval_vgl(d, tab, c["pos_dev"], *out, tile=tile)
    torch.cuda.synchronize()
    idx = _sample(c["pos"].shape[0])
    cols = _columns(s.n_orb)
    pos = c["pos"][idx]
    beta = obuild.build_interp(np.ascontiguousarray(c["f"][..., cols]))
    lbeta = obuild.build_interp(np.ascontiguousarray(c["lf"][..., cols])) if has_lap else None
    ref = oeval.eval_vgl(beta, s.lattice, pos, lap_beta=lbeta)
    got = _take(out, idx, cols)
    gv, gg, gd, gs = GATES[dtype]
    assert normwise(got[0], ref[0]) <= gv
    assert normwise(got[1], ref[1]) <= gg
    assert normwise(got[2], ref[2]) <= (gs if has_lap else gd)
    return d, tab, out


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_si64_full_size(si64, dtype):
    _run_and_check(si64, dtype, False)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype,has_lap", [("f64", False), ("f32", False), ("bf16", False),
                                           ("f64", True), ("f32", True), ("bf16", True)])
def test_mgo96_full_size(mgo96, dtype, has_lap):
    _run_and_check(mgo96, dtype, has_lap)


@pytest.mark.timeout(600)
def test_adjoint_identity_at_fit_size():
    """10^6 points, 128 orbitals, 32^3 grid (FP64 table): <g, J db> = <J^T g, db>."""
    w = config(4)
    s = w.system
    pos = to_dev(w.positions())
    n = pos.shape[0]
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f64")
    g = torch.Generator(device=DEV).manual_seed(404)
    db = torch.randn(P.table_shape(d), dtype=torch.float64, device=DEV, generator=g)
    db[..., s.n_orb:] = 0
    gv = torch.randn((n, s.n_orb), dtype=torch.float64, device=DEV, generator=g)
    gg = torch.randn((n, 3, s.n_orb), dtype=torch.float64, device=DEV, generator=g)
    gl = torch.randn((n, s.n_orb), dtype=torch.float64, device=DEV, generator=g)
    say("adjoint identity at 1e6 points")
    v, gr, lp = P.spline_eval_vgl(d, db, pos)
    lhs = float((v * gv).sum() + (gr * gg).sum() + (lp * gl).sum())
    gt, _ = P.spline_eval_vgl_backward(d, db, pos, gv, gg, gl, want_pos=False)
    rhs = float((gt * db).sum())
    torch.cuda.synchronize()
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs), (lhs, rhs)


@pytest.mark.timeout(600)
def test_batched_48_systems_full_size():
    """All 48 uneven systems in one persistent launch equal per-system launches bitwise (same tile),
    and a sample of three systems matches the oracle."""
    systems = batched_systems()
    items, host = [], []
    say("building the 48 batched systems")
    for j, w in enumerate(systems):
        s = w.system
        f = s.grid_values()
        d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f32")
        tab = P.spline_build(d, to_dev(f))
        pos_h = w.positions()
        pos = to_dev(pos_h)
        n = pos_h.shape[0]
        items.append((d, tab, pos, torch.empty((n, s.n_orb), device=DEV), torch.empty((n, 3, s.n_orb), device=DEV),
                      torch.empty((n, s.n_orb), device=DEV)))
        host.append((s, f if j < 3 else None, pos_h))
    plan = P.BatchPlan(items)
    tile = plan.autotune()
    say("batched graph launch", tile)
    plan.run_graph()
    torch.cuda.synchronize()
    for (d, tab, pos, v, g, l) in items:
        rv, rg, rl = P.spline_eval_vgl(d, tab, pos, tile=tile)
        assert torch.equal(v, rv) and torch.equal(g, rg) and torch.equal(l, rl)
    say("sorted batched graph launch", tile)
    plan.sort(True)
    for (d, tab, pos, v, g, l) in items:
        v.fill_(1.5)
    plan.run_graph()
    torch.cuda.synchronize()
    for (d, tab, pos, v, g, l) in items:
        rv, rg, rl = P.spline_eval_vgl(d, tab, pos, tile=tile)
        assert torch.equal(v, rv) and torch.equal(g, rg) and torch.equal(l, rl)
    for (d, tab, pos, v, g, l), (s, f, pos_h) in zip(items[:3], host[:3]):
        idx = _sample(pos_h.shape[0], k=min(256, pos_h.shape[0]))
        cols = _columns(s.n_orb)
        beta = obuild.build_interp(np.ascontiguousarray(f[..., cols]))
        rv, rg, rl = oeval.eval_vgl(beta, s.lattice, pos_h[idx])
        assert normwise(v.double().cpu().numpy()[idx][:, cols], rv) < 1e-5
        assert normwise(g.double().cpu().numpy()[idx][:, :, cols], rg) < 1e-5
        assert normwise(l.double().cpu().numpy()[idx][:, cols], rl) < 1e-5
    plan.close()


@pytest.mark.timeout(600)
def test_deterministic_adjoint_at_fit_size():
    """10^6 points (FP32 table): the cell-sorted gradient is reproducible bit for bit over four calls
    (each with a fresh workspace) and agrees with the atomic form to FP32 summation accuracy."""
    w = config(4)
    s = w.system
    pos = to_dev(w.positions())
    n = pos.shape[0]
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f32")
    tab = P.spline_build(d, to_dev(s.grid_values()))
    g = torch.Generator(device=DEV).manual_seed(405)
    gv = torch.randn((n, s.n_orb), device=DEV, generator=g)
    gl = torch.randn((n, s.n_orb), device=DEV, generator=g)
    say("deterministic adjoint at 1e6 points")
    runs = [P.spline_eval_vgl_backward(d, tab, pos, gv, None, gl, want_pos=False, flags=P.SPL_DETERMINISTIC)[0]
            for _ in range(4)]
    c, _ = P.spline_eval_vgl_backward(d, tab, pos, gv, None, gl, want_pos=False)
    torch.cuda.synchronize()
    for b in runs[1:]:
        assert torch.equal(runs[0], b)
    assert normwise(runs[0].double().cpu().numpy(), c.double().cpu().numpy()) < 1e-5


@pytest.mark.timeout(600)
@pytest.mark.parametrize("terms", ["value-laplacian", "gradient"])
def test_deterministic_adjoint_upstream_arrays_over_2gib(terms):
    """Upstream arrays of 2 GiB or more: the dense path's brick kernel addresses them with 64-bit
    offsets instead of buffer loads.  FP32 table, 16^3 cells, 48 orbitals; 12 x 10^6 points with value
    and Laplacian terms (2.3 GB each), or 4 x 10^6 with the three gradient terms (one 2.3 GB array):
    bitwise repeatable, and equal to the atomic form to FP32 summation accuracy (which, with about
    2 x 10^5 contributions per table row, is looser than at the fit's 2 x 10^3)."""
    s = make_system("large-upstream", cubic(16 * 0.43), (16, 16, 16), 48, 4.0, 2.0, (1309, 6250, 77))
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f32")
    tab = P.spline_build(d, to_dev(s.grid_values()))
    n = 12_000_000 if terms == "value-laplacian" else 4_000_000
    g = torch.Generator(device=DEV).manual_seed(406)
    pos = (torch.rand((n, 3), device=DEV, generator=g, dtype=torch.float64) @ to_dev(s.lattice))
    if terms == "value-laplacian":
        up = (torch.randn((n, s.n_orb), device=DEV, generator=g), None,
              torch.randn((n, s.n_orb), device=DEV, generator=g))
    else:
        up = (None, torch.randn((n, 3, s.n_orb), device=DEV, generator=g), None)
    big = max(t.numel() * 4 for t in up if t is not None)
    assert big >= 2 ** 31
    say("deterministic adjoint, upstream arrays over 2 GiB", terms)
    a, _ = P.spline_eval_vgl_backward(d, tab, pos, *up, want_pos=False, flags=P.SPL_DETERMINISTIC)
    b, _ = P.spline_eval_vgl_backward(d, tab, pos, *up, want_pos=False, flags=P.SPL_DETERMINISTIC)
    c, _ = P.spline_eval_vgl_backward(d, tab, pos, *up, want_pos=False)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # two FP32 sums of about 64 n / 16^3 random contributions per row, in different orders: their
    # rounding errors grow like the square root of that count
    per_row = 64 * n / 16 ** 3
    assert normwise(a.double().cpu().numpy(), c.double().cpu().numpy()) < 8 * 2.0 ** -24 * np.sqrt(per_row)


@pytest.mark.timeout(600)
def test_deterministic_adjoint_sparse_upstream_arrays_over_2gib():
    """The row-tile form (under 2.5 points per cell) with upstream arrays of 2 GiB or more: 64-bit
    offsets instead of buffer loads.  FP32, the MgO-like 96^3 grid with 256 orbitals, 2.1 x 10^6 points
    (2.4 per cell), value and Laplacian terms of 2.15 GB each.  The gradient does not depend on the table, so it
    stays zero.  Bitwise repeatable, and equal to the atomic form to FP32 summation accuracy."""
    grid, n_orb, n = (96, 96, 96), 256, 2_100_000
    lattice = cubic(2.0 * A_MGO)
    d = P.spline_desc_init(lattice, grid, n_orb, "f32")
    tab = P.new_table(d).zero_()
    g = torch.Generator(device=DEV).manual_seed(407)
    pos = torch.rand((n, 3), device=DEV, generator=g, dtype=torch.float64) @ to_dev(lattice)
    gv = torch.randn((n, n_orb), device=DEV, generator=g)
    gl = torch.randn((n, n_orb), device=DEV, generator=g)
    assert gv.numel() * 4 >= 2 ** 31 and 2 * n < 5 * int(np.prod(grid))
    say("deterministic adjoint, row tiles, upstream arrays over 2 GiB")
    a, _ = P.spline_eval_vgl_backward(d, tab, pos, gv, None, gl, want_pos=False, flags=P.SPL_DETERMINISTIC)
    b, _ = P.spline_eval_vgl_backward(d, tab, pos, gv, None, gl, want_pos=False, flags=P.SPL_DETERMINISTIC)
    c, _ = P.spline_eval_vgl_backward(d, tab, pos, gv, None, gl, want_pos=False)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    per_row = 64 * n / np.prod(grid)
    assert normwise(a.double().cpu().numpy(), c.double().cpu().numpy()) < 8 * 2.0 ** -24 * np.sqrt(per_row)


# ---------------------------------------------------------------- the other representations at full size
@pytest.fixture(scope="module")
def twist():
    w = config(7)
    s = w.system
    f = s.grid_values()                      # periodic parts u, complex
    pos = w.positions()
    return dict(s=s, f=f, pos=pos, f_dev=to_dev(f, torch.complex128), pos_dev=to_dev(pos))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_bloch_twist_full_size(twist, dtype):
    """128 complex orbitals at the zone-corner twist on config 1's cell, autotuned tile."""
    from oracle import bloch as obl
    s = twist["s"]
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, dtype, kvec=s.k)
    say("full size Bloch", s.name, dtype)
    tab = P.spline_build(d, twist["f_dev"])
    out = P.spline_eval_vgl(d, tab, twist["pos_dev"])
    tile = P.spline_autotune(d, tab, twist["pos_dev"], *out)
    out = P.spline_eval_vgl(d, tab, twist["pos_dev"], *out, tile=tile)
    torch.cuda.synchronize()
    cols = _columns(s.n_orb)
    idx = _sample(twist["pos"].shape[0])
    u = twist["f"][..., cols]
    beta = obuild.build_interp(np.ascontiguousarray(u.real)) + 1j * obuild.build_interp(np.ascontiguousarray(u.imag))
    ref = obl.eval_bloch_vgl(beta, s.lattice, s.k, twist["pos"][idx])
    got = _take(out, idx, cols, np.complex128)
    gv, gg, gd, _ = GATES[dtype]
    assert normwise(got[0], ref[0]) <= gv
    assert normwise(got[1], ref[1]) <= gg
    assert normwise(got[2], ref[2]) <= gd


@pytest.fixture(scope="module")
def mgo96_grad(mgo96):
    return mgo96["s"].grid_gradient()        # [3][96^3][256]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("basis", ["bspline", "lagrange"])
def test_mgo96_separate_tables_full_size(mgo96, mgo96_grad, basis):
    """Five separate FP32 tables (orbital, gradient, Laplacian) of all 256 orbitals on the 96^3 grid:
    the bench's separate-table forms, autotuned tile; sampled against the oracle."""
    from oracle import separate as osep
    s = mgo96["s"]
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f32", has_lap=True, sep_grad=True, basis=basis)
    say("full size separate tables", s.name, basis)
    vals = torch.stack([mgo96["f_dev"]] + [to_dev(g) for g in mgo96_grad] + [mgo96["lf_dev"]])
    tab = P.spline_build_tables(d, vals)
    del vals
    out = P.spline_eval_vgl(d, tab, mgo96["pos_dev"])
    tile = P.spline_autotune(d, tab, mgo96["pos_dev"], *out)
    out = P.spline_eval_vgl(d, tab, mgo96["pos_dev"], *out, tile=tile)
    torch.cuda.synchronize()
    cols = _columns(s.n_orb)
    grids = [mgo96["f"], *mgo96_grad, mgo96["lf"]]
    grids = [np.ascontiguousarray(g[..., cols]) for g in grids]
    tabs = [obuild.build_interp(g) for g in grids] if basis == "bspline" else grids
    idx = _sample(mgo96["pos"].shape[0])
    ref = osep.eval_separate(tabs, s.lattice, mgo96["pos"][idx], basis)
    got = _take(out, idx, cols)
    for g, r in zip(got, ref):
        assert normwise(g, r) <= 1e-5


@pytest.mark.timeout(600)
def test_mgo96_pp_full_size(mgo96):
    """pp-spline form of all 256 orbitals on the 96^3 grid (FP32, 8 numbers per grid point): the
    bench's pp form at its autotuned tile, sampled against the oracle's pp build and evaluation."""
    from oracle import ppspline as opp
    s = mgo96["s"]
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f32", basis="pp")
    say("full size pp-spline", s.name)
    tab = P.spline_build(d, mgo96["f_dev"])
    out = P.spline_eval_vgl(d, tab, mgo96["pos_dev"])
    tile = P.spline_autotune(d, tab, mgo96["pos_dev"], *out)
    out = P.spline_eval_vgl(d, tab, mgo96["pos_dev"], *out, tile=tile)
    torch.cuda.synchronize()
    cols = _columns(s.n_orb)
    sig = opp.build_pp(np.ascontiguousarray(mgo96["f"][..., cols]))
    idx = _sample(mgo96["pos"].shape[0])
    ref = opp.eval_pp_vgl(sig, s.lattice, mgo96["pos"][idx])
    got = _take(out, idx, cols)
    for g, r in zip(got, ref):
        assert normwise(g, r) <= 1e-5


@pytest.mark.timeout(600)
def test_fused_fit_matches_autograd_form_at_fit_size():
    """At 10^6 points the fused fit path (forward, misfit kernels, adjoint) and the autograd form
    (SplineVGL + tensor ops) give the same loss and coefficient gradient to FP32 accuracy."""
    from paper_1309_6250_amd.fit import FitProblem, make_loss
    w = config(4)
    s = w.system
    pos = to_dev(w.positions())
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f32")
    tab = P.spline_build(d, to_dev(s.grid_values()))
    g = torch.Generator(device=DEV).manual_seed(406)
    v_t = torch.randn((pos.shape[0], s.n_orb), device=DEV, generator=g, dtype=torch.float64)
    l_t = 30.0 * torch.randn((pos.shape[0], s.n_orb), device=DEV, generator=g, dtype=torch.float64)
    say("fused fit against autograd at 1e6 points")
    prob = FitProblem(d, pos, v_t, l_t, lam=1e-3)
    loss, grad = prob.loss_and_grad(tab)
    beta = tab.clone().requires_grad_(True)
    ref = make_loss(d, pos, v_t, l_t, lam=1e-3)(beta)
    ref.backward()
    torch.cuda.synchronize()
    assert abs(float(loss) - float(ref.detach())) <= 1e-6 * abs(float(ref.detach()))
    assert normwise(grad.double().cpu().numpy(), beta.grad.double().cpu().numpy()) < 1e-5
