"""Planewave orbitals by direct summation (Sec. I, Eq. pw_orbital).

phi_o(r)       = sum_G c_{o,G} exp(i G.r)
grad phi_o(r)  = sum_G (i G) c_{o,G} exp(i G.r)
lap phi_o(r)   = sum_G (-|G|^2) c_{o,G} exp(i G.r)

Real parts are returned; for real orbitals (c_{-G} = conj c_G) the imaginary
parts vanish up to rounding.  This is the O(N_G) per-point cost that the spline
representation replaces.
"""
import numpy as np


def pw_vgl(gvecs, coef, pos, chunk=256):
    """Value, gradient and Laplacian of every orbital at every point.

    gvecs [N_G,3] (1/bohr), coef [O,N_G] complex, pos [P,3] (bohr).
    Returns v [P,O], grad [P,3,O], lap [P,O], all float64.
    """
    gvecs = np.asarray(gvecs, dtype=np.float64)
    coef = np.asarray(coef, dtype=np.complex128)
    pos = np.asarray(pos, dtype=np.float64)
    n_pts, n_orb = pos.shape[0], coef.shape[0]
    g2 = np.einsum("ij,ij->i", gvecs, gvecs)
    cv = coef.T                                            # [N_G, O]
    cg = [(1j * gvecs[:, a])[:, None] * cv for a in range(3)]
    cl = (-g2)[:, None] * cv
    v = np.empty((n_pts, n_orb))
    grad = np.empty((n_pts, 3, n_orb))
    lap = np.empty((n_pts, n_orb))
    for p0 in range(0, n_pts, chunk):
        r = pos[p0:p0 + chunk]
        e = np.exp(1j * (r @ gvecs.T))                     # [p, N_G]
        v[p0:p0 + chunk] = (e @ cv).real
        for a in range(3):
            grad[p0:p0 + chunk, a] = (e @ cg[a]).real
        lap[p0:p0 + chunk] = (e @ cl).real
    return v, grad, lap


def pw_value(gvecs, coef, pos, chunk=256):
    """Orbital values only, [P,O]."""
    gvecs = np.asarray(gvecs, dtype=np.float64)
    cv = np.asarray(coef, dtype=np.complex128).T
    pos = np.asarray(pos, dtype=np.float64)
    out = np.empty((pos.shape[0], cv.shape[1]))
    for p0 in range(0, pos.shape[0], chunk):
        e = np.exp(1j * (pos[p0:p0 + chunk] @ gvecs.T))
        out[p0:p0 + chunk] = (e @ cv).real
    return out
