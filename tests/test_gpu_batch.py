"""Batched persistent launch (one launch over many uneven systems) and its HIP-graph replay.

Parity: for the same tile shape the batched kernel runs the same per-point arithmetic as the
single-system kernel, so outputs must be bitwise equal; the single-system kernel is itself
checked against the FP64 oracle (test_gpu_parity), and a sample is rechecked here.
"""
import numpy as np
import pytest
import torch

import paper_1309_6250_amd as P
from oracle import build as obuild, evaluate as oeval, quantize as oq
from workloads import make_system, batched_systems
from workloads.configs import cubic, BATCH_SPACING
from gpu_helpers import say, to_dev, table_from_oracle, normwise, DEV

pytestmark = pytest.mark.gpu

SPECS = [  # (orbitals, grid, points)
    (3, (6, 7, 8), 301), (17, (10, 10, 10), 0), (32, (12, 9, 14), 1), (64, (16, 16, 16), 2049),
    (100, (8, 12, 10), 777), (256, (14, 14, 14), 1500), (40, (24, 24, 24), 64),
]


def make_items(dtype, has_lap, seed=200):
    rng = np.random.default_rng(seed)
    items, refs = [], []
    for k, (n_orb, grid, n_pts) in enumerate(SPECS):
        lat = cubic(grid[0] * 0.5) + np.diag([0.0, 0.3 * k, -0.2 * k])
        beta = rng.standard_normal(grid + (n_orb,))
        lbeta = rng.standard_normal(grid + (n_orb,)) if has_lap else None
        d = P.spline_desc_init(lat, grid, n_orb, dtype, has_lap=has_lap)
        tab = table_from_oracle(d, beta, dtype, lbeta)
        pos_h = rng.uniform(-10, 10, size=(n_pts, 3))
        pos = to_dev(pos_h)
        od = torch.float64 if dtype == "f64" else torch.float32
        v = torch.full((n_pts, n_orb), np.nan, dtype=od, device=DEV)
        g = torch.full((n_pts, 3, n_orb), np.nan, dtype=od, device=DEV)
        l = torch.full((n_pts, n_orb), np.nan, dtype=od, device=DEV)
        items.append((d, tab, pos, v, g, l))
        refs.append((lat, beta, lbeta, pos_h))
    return items, refs


def single(items, tile):
    out = []
    for d, tab, pos, *_ in items:
        if pos.shape[0] == 0:
            out.append(None)
            continue
        out.append([x.clone() for x in P.spline_eval_vgl(d, tab, pos, tile=tile)])
    torch.cuda.synchronize()
    return out


def assert_same(items, ref):
    for (d, tab, pos, v, g, l), r in zip(items, ref):
        if r is None:
            continue
        for a, b in zip((v, g, l), r):
            assert torch.equal(a, b), (d.n_orb, tuple(d.grid))


@pytest.mark.parametrize("dtype,has_lap", [("f64", False), ("f32", False), ("bf16", False), ("f32", True)])
def test_batch_equals_single_system_kernel(dtype, has_lap):
    items, refs = make_items(dtype, has_lap)
    opl = {"f64": 2, "f32": 4, "bf16": 4}[dtype]
    for tile in ((8, opl), (32, opl), (128, opl)):
        say("batch", dtype, has_lap, tile)
        plan = P.BatchPlan(items, tile=tile)
        n_tiles, n_evals = plan.info()
        assert n_evals == sum(s[0] * s[2] for s in SPECS)
        plan.run()
        torch.cuda.synchronize()
        assert_same(items, single(items, tile))
        plan.close()


def test_batch_matches_oracle_sample():
    items, refs = make_items("f64", False, seed=201)
    plan = P.BatchPlan(items)
    say("batch f64 default tile")
    plan.run()
    torch.cuda.synchronize()
    for (d, tab, pos, v, g, l), (lat, beta, lbeta, pos_h) in zip(items, refs):
        if pos_h.shape[0] == 0:
            continue
        idx = np.arange(0, pos_h.shape[0], max(1, pos_h.shape[0] // 40))
        rv, rg, rl = oeval.eval_vgl(beta, lat, pos_h[idx])
        assert normwise(v.cpu().numpy()[idx], rv) < 1e-12
        assert normwise(g.cpu().numpy()[idx], rg) < 1e-12
        assert normwise(l.cpu().numpy()[idx], rl) < 1e-12
    plan.close()


def test_graph_replays_match_eager():
    """Replay the captured graph several times with eager work and synchronizations in between;
    every replay must reproduce the eager result (outputs are cleared before each replay)."""
    items, _ = make_items("f32", False, seed=202)
    plan = P.BatchPlan(items, tile=(32, 2))
    say("batch eager reference")
    plan.run()
    torch.cuda.synchronize()
    ref = [[x.clone() for x in it[3:]] for it in items]
    for rep in range(4):
        for it in items:
            for x in it[3:]:
                x.fill_(np.nan)                     # eager work between replays
        torch.cuda.synchronize()
        say("graph replay", rep)
        plan.run_graph()
        torch.cuda.synchronize()
        for it, r in zip(items, ref):
            for a, b in zip(it[3:], r):
                assert torch.equal(a, b)
        _ = torch.ones(1000, device=DEV).sum().item()   # unrelated eager kernel + sync
    plan.close()


def test_batch_autotune_picks_valid_tile_and_keeps_results():
    """The autotuned shape is a common one, or (0, orbitals per lane) when the items keep their own lanes
    per point (whichever timed fastest): every item's listed shape is valid, and each item's outputs equal
    the single-system kernel's at that item's shape, bit for bit."""
    items, _ = make_items("bf16", False, seed=203)
    plan = P.BatchPlan(items)
    say("batch autotune")
    g, opl = plan.autotune()
    lanes = (8, 16, 32, 64, 128, 256)
    assert opl in (2, 4, 8) and (g == 0 or g in lanes)
    tiles = plan.tiles()
    assert all(t[0] in lanes and t[1] == opl for t in tiles)
    if g:
        assert all(t[0] == g for t in tiles)
    for it in items:
        for x in it[3:]:
            x.fill_(np.nan)
    plan.run()
    torch.cuda.synchronize()
    ref = [single([it], t)[0] for it, t in zip(items, tiles)]
    assert_same(items, ref)
    plan.close()


def test_batch_rejects_mixed_dtypes():
    a, _ = make_items("f32", False, seed=204)
    b, _ = make_items("f64", False, seed=205)
    with pytest.raises(P.SplineError) as ei:
        P.BatchPlan([a[0], b[3]])
    assert ei.value.code == P.SPL_EINVAL


def test_batched_workload_subset_against_oracle():
    """The first systems of the uneven 48-system workload (fewer walkers), built on the GPU."""
    systems = batched_systems(scale=0.05)[:5]
    items, hosts = [], []
    for w in systems:
        s = w.system
        f = s.grid_values()
        d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f32")
        tab = P.spline_build(d, to_dev(f))
        pos_h = w.positions()
        pos = to_dev(pos_h)
        v = torch.empty((pos_h.shape[0], s.n_orb), dtype=torch.float32, device=DEV)
        g = torch.empty((pos_h.shape[0], 3, s.n_orb), dtype=torch.float32, device=DEV)
        l = torch.empty_like(v)
        items.append((d, tab, pos, v, g, l))
        hosts.append((s, f, pos_h))
    plan = P.BatchPlan(items)
    say("config-3 subset batch")
    plan.run_graph()
    torch.cuda.synchronize()
    for (d, tab, pos, v, g, l), (s, f, pos_h) in zip(items, hosts):
        idx = np.arange(0, pos_h.shape[0], max(1, pos_h.shape[0] // 32))
        beta = obuild.build_interp(f)
        rv, rg, rl = oeval.eval_vgl(beta, s.lattice, pos_h[idx])
        assert normwise(v.double().cpu().numpy()[idx], rv) < 1e-5
        assert normwise(g.double().cpu().numpy()[idx], rg) < 1e-5
        assert normwise(l.double().cpu().numpy()[idx], rl) < 1e-5
    plan.close()


@pytest.mark.parametrize("dtype,has_lap", [("f64", False), ("f32", True), ("bf16", False)])
def test_sorted_batch_equals_single_system_kernel(dtype, has_lap):
    """Sorted plans (points in locality order per item) give the same outputs bitwise; the option can
    be switched off and on again."""
    items, refs = make_items(dtype, has_lap, seed=206)
    items[0][2][5] = float("nan")                      # a non-finite point in one item
    opl = {"f64": 2, "f32": 4, "bf16": 4}[dtype]
    for tile in ((8, opl), (64, opl)):
        say("sorted batch", dtype, has_lap, tile)
        plan = P.BatchPlan(items, tile=tile)
        ref = single(items, tile)
        for enable in (True, False, True):
            for it in items:
                for x in it[3:]:
                    x.fill_(1234.5)
            plan.sort(enable)
            plan.run()
            torch.cuda.synchronize()
            for (d, tab, pos, v, g, l), r in zip(items, ref):
                if r is None:
                    continue
                for a, b in zip((v, g, l), r):
                    assert torch.equal(torch.nan_to_num(a, nan=7.0), torch.nan_to_num(b, nan=7.0))
        plan.close()


def test_sorted_batch_graph_replays_match_eager():
    items, _ = make_items("f32", False, seed=207)
    plan = P.BatchPlan(items, tile=(32, 2))
    plan.sort(True)
    say("sorted batch eager reference")
    plan.run()
    torch.cuda.synchronize()
    ref = [[x.clone() for x in it[3:]] for it in items]
    assert_same(items, single(items, (32, 2)))
    for rep in range(4):
        for it in items:
            for x in it[3:]:
                x.fill_(np.nan)
        torch.cuda.synchronize()
        say("sorted graph replay", rep)
        plan.run_graph()
        torch.cuda.synchronize()
        for it, r in zip(items, ref):
            for a, b in zip(it[3:], r):
                assert torch.equal(a, b)
        _ = torch.ones(1000, device=DEV).sum().item()
    plan.close()


@pytest.mark.parametrize("dtype,has_lap", [("f64", False), ("f32", False), ("bf16", False), ("f32", True)])
def test_per_item_tiles_equal_single_system_kernel(dtype, has_lap):
    """Items with their own lanes per point in one persistent launch (eager and graph replay, in the
    given order and in locality order): each item's outputs equal the single-system kernel's at that
    item's shape, bit for bit.  Also after the autotuner picks the shapes."""
    items, _ = make_items(dtype, has_lap, seed=205)
    opl = {"f64": 2, "f32": 4, "bf16": 4}[dtype]
    lanes = [8, 16, 32, 64, 128, 256, 8]
    shapes = [(g, opl) for g in lanes]
    plan = P.BatchPlan(items)
    plan.set_tiles(shapes)
    assert plan.tiles() == shapes
    ref = [None if pos.shape[0] == 0 else [x.clone() for x in P.spline_eval_vgl(d, tab, pos, tile=t)]
           for (d, tab, pos, *_), t in zip(items, shapes)]
    torch.cuda.synchronize()
    for how in ("eager", "graph", "sorted graph"):
        for (_, _, _, v, g, l) in items:
            v.fill_(np.nan), g.fill_(np.nan), l.fill_(np.nan)
        say("per-item tiles", dtype, has_lap, how)
        if how == "sorted graph":
            plan.sort(True)
        if how == "eager":
            plan.run()
        else:
            plan.run_graph()
        torch.cuda.synchronize()
        assert plan.tiles() == shapes
        assert_same(items, ref)
    say("batch autotune with per-item shapes", dtype, has_lap)
    plan.autotune()
    chosen = plan.tiles()
    assert len({t[1] for t in chosen}) == 1
    for (_, _, _, v, g, l) in items:
        v.fill_(np.nan), g.fill_(np.nan), l.fill_(np.nan)
    plan.run_graph()
    torch.cuda.synchronize()
    assert_same(items, [None if pos.shape[0] == 0 else [x.clone() for x in P.spline_eval_vgl(d, tab, pos, tile=t)]
                        for (d, tab, pos, *_), t in zip(items, chosen)])
    with pytest.raises(P.SplineError):
        plan.set_tiles([(8, opl)] * (len(items) - 1) + [(8, 1 if opl != 1 else 2)])      # mixed orbitals per lane
    with pytest.raises(P.SplineError):
        plan.set_tiles([(4, opl)] * len(items))                                         # fewer than 8 lanes
    plan.close()
