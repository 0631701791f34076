"""Pins of the oracle's adjoint (transpose of the evaluation) and of the fit loss gradient."""
import numpy as np

from oracle import build, evaluate, adjoint, fit

SKEW = np.array([[7.0, 0.4, -0.3], [1.1, 6.2, 0.5], [-0.6, 0.9, 8.3]])


def _setup(seed, grid=(6, 7, 8), n_orb=3, n_pts=40, interior=True):
    rng = np.random.default_rng(seed)
    beta = build.build_interp(rng.standard_normal(grid + (n_orb,)))
    cells = rng.integers(0, np.array(grid), size=(n_pts, 3))
    lo, hi = (0.2, 0.8) if interior else (0.0, 1.0)
    u = cells + rng.uniform(lo, hi, size=(n_pts, 3))
    pos = (u / np.array(grid)) @ SKEW + rng.integers(-1, 2, size=(n_pts, 1)) * SKEW[1]
    gv = rng.standard_normal((n_pts, n_orb))
    gg = rng.standard_normal((n_pts, 3, n_orb))
    gl = rng.standard_normal((n_pts, n_orb))
    return rng, beta, pos, gv, gg, gl


def _dot(outs, gv, gg, gl):
    v, g, lap = outs
    return np.sum(v * gv) + np.sum(g * gg) + np.sum(lap * gl)


def test_adjoint_dot_product_identity():
    rng, beta, pos, gv, gg, gl = _setup(20, interior=False)
    gbeta, _, _ = adjoint.vgl_backward(beta, SKEW, pos, gv, gg, gl)
    dbeta = rng.standard_normal(beta.shape)
    lhs = _dot(evaluate.eval_vgl(dbeta, SKEW, pos), gv, gg, gl)      # <g, J dbeta> (forward is linear)
    rhs = np.sum(gbeta * dbeta)                                        # <J^T g, dbeta>
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_dot_product_identity_separate_laplacian():
    rng, beta, pos, gv, gg, gl = _setup(21, interior=False)
    lap_beta = rng.standard_normal(beta.shape)
    gbeta, glb, _ = adjoint.vgl_backward(beta, SKEW, pos, gv, gg, gl, lap_beta=lap_beta)
    db = rng.standard_normal(beta.shape)
    dl = rng.standard_normal(beta.shape)
    lhs = _dot(evaluate.eval_vgl(db, SKEW, pos, lap_beta=dl), gv, gg, gl)
    rhs = np.sum(gbeta * db) + np.sum(glb * dl)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _fd_positions(beta, pos, gv, gg, gl, lap_beta=None, d=1e-5):
    out = np.zeros((pos.shape[0], 3))
    for a in range(3):
        e = np.zeros(3)
        e[a] = d
        fp = evaluate.eval_vgl(beta, SKEW, pos + e, lap_beta=lap_beta)
        fm = evaluate.eval_vgl(beta, SKEW, pos - e, lap_beta=lap_beta)
        # per-point objective: sum_o g . out, differentiated point by point
        for k, (x, y) in enumerate(zip(fp, fm)):
            w = (gv, gg, gl)[k]
            out[:, a] += (np.sum((x - y) * w, axis=tuple(range(1, x.ndim)))) / (2 * d)
    return out


def test_position_gradient_finite_difference():
    _, beta, pos, gv, gg, gl = _setup(22)
    _, _, gpos = adjoint.vgl_backward(beta, SKEW, pos, gv, gg, gl)
    fd = _fd_positions(beta, pos, gv, gg, gl)
    np.testing.assert_allclose(gpos, fd, atol=1e-6 * np.abs(fd).max())


def test_position_gradient_finite_difference_separate_laplacian():
    rng, beta, pos, gv, gg, gl = _setup(23)
    lap_beta = build.build_interp(rng.standard_normal(beta.shape))
    _, _, gpos = adjoint.vgl_backward(beta, SKEW, pos, gv, gg, gl, lap_beta=lap_beta)
    fd = _fd_positions(beta, pos, gv, gg, gl, lap_beta=lap_beta)
    np.testing.assert_allclose(gpos, fd, atol=1e-6 * np.abs(fd).max())


def test_backward_with_missing_upstream_terms():
    _, beta, pos, gv, gg, gl = _setup(24)
    a = adjoint.vgl_backward(beta, SKEW, pos, gv=gv)
    b = adjoint.vgl_backward(beta, SKEW, pos, gv=gv, ggrad=np.zeros_like(gg), glap=np.zeros_like(gl))
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[2], b[2])


def test_nonfinite_points_contribute_nothing():
    _, beta, pos, gv, gg, gl = _setup(25)
    pos = pos.copy()
    pos[3] = np.nan
    gb, _, gp = adjoint.vgl_backward(beta, SKEW, pos, gv, gg, gl)
    keep = np.ones(pos.shape[0], bool)
    keep[3] = False
    gb2, _, gp2 = adjoint.vgl_backward(beta, SKEW, pos[keep], gv[keep], gg[keep], gl[keep])
    np.testing.assert_allclose(gb, gb2, atol=1e-13)
    assert np.isnan(gp[3]).all() and np.isfinite(gp[keep]).all()


def test_fit_loss_gradient_finite_difference():
    rng, beta, pos, _, _, _ = _setup(26, grid=(5, 5, 6), n_orb=2, n_pts=60, interior=False)
    v_pw = rng.standard_normal((pos.shape[0], 2))
    l_pw = 10 * rng.standard_normal((pos.shape[0], 2))
    w_v, w_l = fit.weights_from_targets(v_pw, l_pw)
    loss, grad = fit.loss_and_grad(beta, SKEW, pos, v_pw, l_pw, w_v, w_l, lam=0.3)
    d = 1e-6
    for _ in range(8):
        idx = tuple(rng.integers(0, s) for s in beta.shape)
        bp = beta.copy()
        bp[idx] += d
        bm = beta.copy()
        bm[idx] -= d
        fd = (fit.loss_and_grad(bp, SKEW, pos, v_pw, l_pw, w_v, w_l, 0.3)[0]
              - fit.loss_and_grad(bm, SKEW, pos, v_pw, l_pw, w_v, w_l, 0.3)[0]) / (2 * d)
        assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(fd)), (fd, grad[idx])
