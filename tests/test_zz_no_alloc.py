"""spline_eval_vgl_sorted_noalloc: the locality-ordered evaluation with its workspace in the
library's static device scratch, for callers that cannot allocate.  Through the C ABI its outputs
equal spline_eval_vgl_sorted's (caller workspace) bit for bit, on two calls in a row, the second
with fewer points (the scratch keeps the first call's contents), for every storage dtype and with a
separate Laplacian table; a point count beyond the scratch is rejected before anything runs."""
import numpy as np
import pytest
import torch

import paper_1309_6250_amd as P
from workloads import make_system
from gpu_helpers import say, to_dev, DEV

pytestmark = pytest.mark.gpu

SKEW = np.array([[7.0, 0.4, -0.3], [1.1, 6.2, 0.5], [-0.6, 0.9, 8.3]])


def noalloc(desc, table, pos, tile=None):
    """The entry point through the C ABI, with outputs allocated here (the entry point allocates nothing)."""
    n = pos.shape[0]
    v, g, l = P.api._outputs(desc, n, pos.device, None, None, None)
    return P.spline_eval_vgl_sorted_noalloc(desc, table, pos, v, g, l, tile=tile)


def _same(a, b):
    return all(torch.equal(torch.nan_to_num(x, nan=12345.0), torch.nan_to_num(y, nan=12345.0)) for x, y in zip(a, b))


def _points(s, n, seed):
    rng = np.random.default_rng(seed)
    pos = s.positions(n)
    clustered = pos[:1] + rng.normal(scale=0.05, size=(97, 3))
    out = np.concatenate([pos, clustered, -pos[5:11]])
    out[17] = [np.nan, 1.0, 2.0]
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("lap", [False, True])
def test_noalloc_equals_sorted_on_two_calls(dtype, lap):
    s = make_system("noalloc-skew", SKEW, (10, 9, 11), 13, 2.2, 2.0, (45, 7))
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, dtype, has_lap=lap)
    table = P.spline_build(d, to_dev(s.grid_values()), to_dev(s.grid_laplacian()) if lap else None)
    big = to_dev(_points(s, 6000, 51))
    small = to_dev(_points(s, 700, 52))
    for name, pos in (("first call", big), ("second call, fewer points", small)):
        for tile in (None, (8, 2 if dtype == "bf16" else 1)):
            say("noalloc", name, dtype, lap, tile, pos.shape[0])
            got = noalloc(d, table, pos, tile)
            ref = P.spline_eval_vgl_sorted(d, table, pos, tile=tile)
            torch.cuda.synchronize()
            assert _same(got, ref), (name, tile)


def test_noalloc_full_population_and_limit():
    """A QMC population of 65 536 points fits the scratch; 2.5 million points do not and are
    rejected before anything is enqueued."""
    s = make_system("noalloc-cube", np.eye(3) * 12.0, (24, 24, 24), 40, 2.5, 2.0, (45, 8))
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f32")
    table = P.spline_build(d, to_dev(s.grid_values()))
    pos = to_dev(s.positions(65536))
    say("noalloc full population")
    got = noalloc(d, table, pos)
    ref = P.spline_eval_vgl_sorted(d, table, pos)
    torch.cuda.synchronize()
    assert _same(got, ref)
    too_many = torch.zeros((2_500_000, 3), dtype=torch.float64, device=DEV)
    with pytest.raises(P.SplineError) as exc:
        noalloc(d, table, too_many)
    assert exc.value.code == P.SPL_EINVAL and "static scratch" in str(exc.value)
    # the library still works afterwards, and the scratch serves a smaller call again
    again = noalloc(d, table, pos[:1000].contiguous())
    ref2 = P.spline_eval_vgl_sorted(d, table, pos[:1000].contiguous())
    torch.cuda.synchronize()
    assert _same(again, ref2)
