"""Smoothing (Fourier-matched) build on the GPU against the oracle's FFT construction, and its
accuracy against the planewave orbitals compared with the interpolating build."""
import numpy as np
import pytest
import torch

import paper_1309_6250_amd as P
from oracle import smoothing as osm, build as obuild, evaluate as oeval, pw as opw, quantize as oq
from workloads import config, make_system
from workloads.configs import cubic, A_MGO
from gpu_helpers import say, to_dev, host_table, normwise, DEV

pytestmark = pytest.mark.gpu

SKEW = np.array([[7.0, 0.4, -0.3], [1.1, 6.2, 0.5], [-0.6, 0.9, 8.3]])


def systems():
    return [config(0).system,
            make_system("smooth-skew", SKEW, (10, 12, 14), 5, 2.0, 2.0, (31, 1)),
            make_system("smooth-mgo", cubic(2 * A_MGO), (24, 24, 24), 12, 4.0, 8.0, (31, 2)),
            # an axis longer than 192 points: that stage takes the per-line kernel, the others the matrix cores
            make_system("smooth-long", np.diag([40.0, 5.0, 5.0]), (200, 6, 6), 3, 2.0, 2.0, (31, 3)),
            # more orbitals than one 32-wide tile of the coefficient scatter, the last tile partial (70 = 2 x 32
            # + 6), and several hundred planewaves
            make_system("smooth-wide", SKEW, (12, 12, 14), 70, 2.6, 2.0, (31, 4))]


def _gpu_smoothing(s, dtype, has_lap):
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, dtype, has_lap=has_lap)
    say("spline_build_smoothing", s.name, dtype, has_lap)
    tab = P.spline_build_smoothing(d, torch.from_numpy(s.miller.astype(np.int32)).to(DEV),
                                   torch.from_numpy(s.coef).to(DEV))
    torch.cuda.synchronize()
    return d, tab


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("has_lap", [False, True])
def test_smoothing_table_matches_oracle(k, has_lap):
    s = systems()[k]
    assert s.nyquist_ok()
    d, tab = _gpu_smoothing(s, "f64", has_lap)
    got = host_table(d, tab)
    ref = osm.build_smoothing(s.miller, s.coef, s.grid)
    assert np.abs(got[0] - ref).max() <= 1e-12 * np.abs(ref).max()
    if has_lap:
        g2 = np.einsum("ij,ij->i", s.gvecs, s.gvecs)
        lref = osm.build_smoothing(s.miller, s.coef * (-g2)[None, :], s.grid)
        assert np.abs(got[1] - lref).max() <= 1e-12 * np.abs(lref).max()
    pad = tab.double().cpu().numpy()[..., s.n_orb:]
    assert pad.size == 0 or np.all(pad == 0.0)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_smoothing_storage_cast(dtype):
    s = systems()[1]
    d, tab = _gpu_smoothing(s, dtype, False)
    ref = oq.quantized(osm.build_smoothing(s.miller, s.coef, s.grid), dtype)
    got = host_table(d, tab)[0]
    ulp = (2.0**-23 if dtype == "f32" else 2.0**-7) * np.abs(ref)
    diff = np.abs(got - ref)
    assert np.all(diff <= ulp + 1e-300) and np.mean(diff == 0) >= 0.999


def test_smoothing_more_accurate_than_interpolation():
    """RMAE of value and gradient against the planewave sum: the Fourier-matched spline beats the
    interpolating one (the paper's finding, on the synthetic MgO-like orbitals)."""
    s = systems()[2]
    pos = s.positions(2000)
    vp, gp, lp = opw.pw_vgl(s.gvecs, s.coef, pos)
    d, tab_s = _gpu_smoothing(s, "f64", False)
    tab_i = P.spline_build(d, to_dev(s.grid_values()))
    x = to_dev(pos)
    outs_s = [t.cpu().numpy() for t in P.spline_eval_vgl(d, tab_s, x)]
    outs_i = [t.cpu().numpy() for t in P.spline_eval_vgl(d, tab_i, x)]
    torch.cuda.synchronize()
    rmae = lambda a, b: np.abs(a - b).mean() / np.abs(b).mean()
    es = [rmae(a, b) for a, b in zip(outs_s, (vp, gp, lp))]
    ei = [rmae(a, b) for a, b in zip(outs_i, (vp, gp, lp))]
    assert es[0] < ei[0] and es[1] < ei[1], (es, ei)
