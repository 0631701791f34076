"""Bloch orbitals phi(r) = exp(i k.r) u(r) with a lattice-periodic u (Sec. I, Bloch functions).

The periodic part u is complex; its real and imaginary parts are two ordinary periodic
interpolants (any of the representations of App. A).  The orbital's derivatives follow from
the product rule:

    grad phi = e^{ik.r} (grad u + i k u)
    lap phi  = e^{ik.r} (lap u + 2 i k.grad u - |k|^2 u)

When the Laplacian is approximated separately, its table interpolates the periodic part of the
orbital's Laplacian, w = e^{-ik.r} lap phi (for planewave coefficients c_G of u,
w = sum_G -|k+G|^2 c_G e^{iG.r}), and lap phi = e^{ik.r} w.  With separate gradient tables
the same holds per Cartesian component: grad_a phi = e^{ik.r} g_a, g_a = sum_G i(k+G)_a c_G e^{iG.r}.
The phase uses the unfolded Cartesian position r.
"""
import numpy as np

from . import evaluate, separate, ppspline


def pw_bloch_vgl(gvecs, coef, kvec, pos, chunk=256):
    """Direct planewave sums of phi = sum_G c_G e^{i(k+G).r}, its gradient and Laplacian (complex).

    Returns v [P,O], grad [P,3,O], lap [P,O], complex128."""
    q = np.asarray(gvecs, dtype=np.float64) + np.asarray(kvec, dtype=np.float64)
    cv = np.asarray(coef, dtype=np.complex128).T
    pos = np.asarray(pos, dtype=np.float64)
    q2 = np.einsum("ij,ij->i", q, q)
    n_pts, n_orb = pos.shape[0], cv.shape[1]
    v = np.empty((n_pts, n_orb), dtype=np.complex128)
    grad = np.empty((n_pts, 3, n_orb), dtype=np.complex128)
    lap = np.empty((n_pts, n_orb), dtype=np.complex128)
    for p0 in range(0, n_pts, chunk):
        e = np.exp(1j * (pos[p0:p0 + chunk] @ q.T))
        v[p0:p0 + chunk] = e @ cv
        for a in range(3):
            grad[p0:p0 + chunk, a] = e @ ((1j * q[:, a])[:, None] * cv)
        lap[p0:p0 + chunk] = e @ ((-q2)[:, None] * cv)
    return v, grad, lap


def phase(kvec, pos):
    """e^{ik.r} per point, [P] complex."""
    return np.exp(1j * (np.asarray(pos, dtype=np.float64) @ np.asarray(kvec, dtype=np.float64)))


def _complex_vgl(beta, lattice, pos, lap_beta=None, form="bspline"):
    """V, grad, lap of a complex-coefficient spline: real and imaginary parts evaluated apart."""
    beta = np.asarray(beta)
    lre = None if lap_beta is None else np.ascontiguousarray(np.real(lap_beta))
    lim = None if lap_beta is None else np.ascontiguousarray(np.imag(lap_beta))
    if form == "bspline":
        re = evaluate.eval_vgl(np.ascontiguousarray(beta.real), lattice, pos, lap_beta=lre)
        im = evaluate.eval_vgl(np.ascontiguousarray(beta.imag), lattice, pos, lap_beta=lim)
    elif form == "pp":
        re = ppspline.eval_pp_vgl(np.ascontiguousarray(beta.real), lattice, pos, lap_sigma=lre)
        im = ppspline.eval_pp_vgl(np.ascontiguousarray(beta.imag), lattice, pos, lap_sigma=lim)
    else:
        raise ValueError(form)
    return tuple(a + 1j * b for a, b in zip(re, im))


def eval_bloch_vgl(beta, lattice, kvec, pos, lap_beta=None, form="bspline"):
    """Bloch orbital from complex spline coefficients of u: B-spline coefficients beta
    [N1][N2][N3][O], or with form="pp" the pp-spline numbers [N1][N2][N3][8][O].

    Without lap_beta the Laplacian comes from second derivatives of u; with it (complex
    coefficients of w) from w's value.  Returns complex V [P,O], grad [P,3,O], lap [P,O]."""
    k = np.asarray(kvec, dtype=np.float64)
    u, gu, lu = _complex_vgl(beta, lattice, pos, lap_beta, form)
    e = phase(k, pos)[:, None]
    v = e * u
    grad = e[:, None, :] * (gu + 1j * k[None, :, None] * u[:, None, :])
    if lap_beta is None:
        kdotg = np.einsum("a,pao->po", k, gu)
        lap = e * (lu + 2j * kdotg - (k @ k) * u)
    else:
        lap = e * lu
    return v, grad, lap


def eval_bloch_v(beta, lattice, kvec, pos):
    """Values of the Bloch orbitals, complex [P,O]."""
    beta = np.asarray(beta)
    u = (evaluate.eval_v(np.ascontiguousarray(beta.real), lattice, pos)
         + 1j * evaluate.eval_v(np.ascontiguousarray(beta.imag), lattice, pos))
    return phase(kvec, pos)[:, None] * u


def eval_bloch_separate(tables, lattice, kvec, pos, basis="bspline"):
    """Bloch orbital from five complex separate tables (u, g_x, g_y, g_z, w); see the module docstring."""
    re = separate.eval_separate([np.ascontiguousarray(np.real(t)) for t in tables], lattice, pos, basis)
    im = separate.eval_separate([np.ascontiguousarray(np.imag(t)) for t in tables], lattice, pos, basis)
    e = phase(kvec, pos)[:, None]
    v, g, l = (a + 1j * b for a, b in zip(re, im))
    return e * v, e[:, None, :] * g, e * l
