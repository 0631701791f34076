"""Locality-ordered evaluation (spline_eval_vgl_sorted): the same outputs, bitwise, as
spline_eval_vgl at the same tile, in the caller's point order, whatever the point order; and
against the FP64 oracle directly."""
import numpy as np
import pytest
import torch

import paper_1309_6250_amd as P
from oracle import build as obuild, evaluate as oeval
from workloads import config, make_system
from gpu_helpers import say, to_dev, normwise, table_from_oracle, DEV

pytestmark = pytest.mark.gpu

SKEW = np.array([[7.0, 0.4, -0.3], [1.1, 6.2, 0.5], [-0.6, 0.9, 8.3]])


def _points(s, n, seed):
    rng = np.random.default_rng(seed)
    pos = s.positions(n)
    clustered = pos[:1] + rng.normal(scale=0.05, size=(97, 3))          # many points in a few cells
    far = pos[:5] + np.array([4.0, -9.0, 2.0]) @ s.lattice
    out = np.concatenate([pos, clustered, far, -pos[5:11]])
    out[17] = [np.nan, 1.0, 2.0]
    out[n + 3] = [1.0, np.inf, 2.0]
    return out


def _same(a, b):
    return all(torch.equal(torch.nan_to_num(x, nan=12345.0), torch.nan_to_num(y, nan=12345.0)) for x, y in zip(a, b))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("lap", [False, True])
def test_sorted_equals_unsorted_bitwise(dtype, lap):
    s = make_system("sorted-skew", SKEW, (10, 9, 11), 13, 2.2, 2.0, (45, 1))
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, dtype, has_lap=lap)
    table = P.spline_build(d, to_dev(s.grid_values()), to_dev(s.grid_laplacian()) if lap else None)
    pos = to_dev(_points(s, 1500, 46))
    opls = {"f64": (1, 2), "f32": (1, 2, 4), "bf16": (2, 4, 8)}[dtype]
    for g in (2, 8, 32, 256):
        for opl in opls:
            say("sorted vs unsorted", dtype, lap, g, opl)
            a = P.spline_eval_vgl(d, table, pos, tile=(g, opl))
            b = P.spline_eval_vgl_sorted(d, table, pos, tile=(g, opl))
            torch.cuda.synchronize()
            assert _same(a, b), (g, opl)
    c = P.spline_eval_vgl_sorted(d, table, pos)                           # default tile
    torch.cuda.synchronize()
    assert _same(P.spline_eval_vgl(d, table, pos), c)


def test_sorted_matches_oracle_and_edge_cases():
    w = config(0)
    s = w.system
    f = s.grid_values()
    beta = obuild.build_interp(f)
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f64")
    table = table_from_oracle(d, beta, "f64")
    pos = _points(s, 900, 47)
    say("sorted vs oracle")
    got = [x.cpu().numpy() for x in P.spline_eval_vgl_sorted(d, table, to_dev(pos))]
    ref = oeval.eval_vgl(beta, s.lattice, pos)
    for g, r in zip(got, ref):
        assert np.array_equal(np.isnan(g), np.isnan(r))
        assert normwise(np.nan_to_num(g), np.nan_to_num(r)) <= 1e-12
    # empty input, and a workspace that is too small
    empty = torch.empty((0, 3), dtype=torch.float64, device=DEV)
    out = P.spline_eval_vgl_sorted(d, table, empty)
    assert all(o.shape[0] == 0 for o in out)
    small = torch.empty(16, dtype=torch.uint8, device=DEV)
    with pytest.raises(ValueError):
        P.spline_eval_vgl_sorted(d, table, to_dev(pos), work=small)
    v, g, l = P.spline_eval_vgl(d, table, to_dev(pos))
    rc = P.lib().spline_eval_vgl_sorted(P.api.ctypes.byref(d), P.api._ptr(table), len(pos), P.api._ptr(to_dev(pos)),
                                        P.api._ptr(v), P.api._ptr(g), P.api._ptr(l), None, P.api._ptr(small), 16,
                                        None)
    assert rc == P.SPL_EINVAL
    assert P.spline_sorted_work_bytes(d, 10**6) >= 8 * 10**6          # bucket and slot of every point


@pytest.mark.timeout(600)
@pytest.mark.parametrize("key,dtype", [(1, "f64"), (2, "f64"), (2, "bf16")])
def test_sorted_full_size_equals_unsorted(key, dtype):
    """Full workloads (65 536 points; Si 48^3 x 128 and MgO-like 96^3 x 256) at the tiles the bench
    uses: the locality-ordered call reproduces spline_eval_vgl bitwise."""
    w = config(key)
    s = w.system
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, dtype)
    table = P.spline_build(d, to_dev(s.grid_values()))
    pos = to_dev(w.positions())
    say("full size sorted", s.name, dtype)
    a = P.spline_eval_vgl(d, table, pos)
    tile = P.spline_autotune(d, table, pos, *a)
    a = P.spline_eval_vgl(d, table, pos, tile=tile)
    b = P.spline_eval_vgl_sorted(d, table, pos, tile=tile)
    torch.cuda.synchronize()
    assert _same(a, b)


@pytest.mark.parametrize("kind", ["pp", "pp_lap", "sep_bspline", "sep_lagrange", "bloch", "bloch_lap", "bloch_pp"])
@pytest.mark.parametrize("dtype", ["f64", "bf16"])
def test_sorted_equals_unsorted_for_every_representation(kind, dtype):
    bloch = kind.startswith("bloch")
    s = make_system("sorted-var", SKEW, (10, 9, 11), 5, 2.0, 2.0, (45, 2),
                    kvec=(0.21, -0.13, 0.33) if bloch else None)
    cdt = torch.complex128 if bloch else torch.float64
    kv = s.k if bloch else None
    if kind.startswith("sep"):
        d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, dtype, has_lap=True, sep_grad=True,
                               basis=kind.split("_")[1])
        grids = [s.grid_values()] + list(s.grid_gradient()) + [s.grid_laplacian()]
        table = P.spline_build_tables(d, [to_dev(g, cdt) for g in grids])
    else:
        lap = kind.endswith("lap")
        d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, dtype, has_lap=lap,
                               basis="pp" if "pp" in kind else "bspline", kvec=kv)
        table = P.spline_build(d, to_dev(s.grid_values(), cdt), to_dev(s.grid_laplacian(), cdt) if lap else None)
    pos = to_dev(_points(s, 700, 48))
    opls = {"f64": (1, 2), "bf16": (2, 4, 8)}[dtype]
    for g in (4, 64):
        for opl in opls:
            if bloch and opl % 2:
                continue
            say("sorted vs unsorted", kind, dtype, g, opl)
            a = P.spline_eval_vgl(d, table, pos, tile=(g, opl))
            b = P.spline_eval_vgl_sorted(d, table, pos, tile=(g, opl))
            torch.cuda.synchronize()
            if bloch:
                a, b = [torch.view_as_real(x) for x in a], [torch.view_as_real(x) for x in b]
            assert _same(a, b), (kind, g, opl)
