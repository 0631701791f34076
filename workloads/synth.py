"""Seeded planewave orbitals, their grid samples, and electron positions.

Conventions
-----------
* ``lattice`` is a 3x3 array whose ROW i is the lattice vector a_i in bohr.
  The paper's matrix a (Sec. II, Coordinates paragraph) has the lattice vectors
  as columns, so a = lattice.T and crystal coordinates are s = a^-1 r.
* A reciprocal vector is G = 2*pi * a^-T ... written per Miller triple n as
  G = 2*pi * inv(lattice) @ n, so that G.r = 2*pi n.s for r = a s.
* Orbital phi_o(r) = sum_G c_{o,G} exp(i G.r) (Eq. pw_orbital, Gamma point).
  Real orbitals: c_{-G} = conj(c_G); c_0 is real.
* Bloch orbitals at crystal momentum k (Sec. I): phi_o(r) = exp(i k.r) u_o(r) with the
  periodic part u_o(r) = sum_G c_{o,G} exp(i G.r), planewaves |k + G| < Gcut.  The
  coefficients have no symmetry: Re and Im of every c_G are independent
  N(0, exp(-|k+G|^2/decay)/2), drawn as standard_normal((n_orb, 2 N_G)) with columns
  (2g, 2g+1) = (Re, Im) of the g-th G in lexicographic Miller order.
* Grid samples are always of periodic functions: u itself, the periodic part of the
  orbital's gradient, sum_G i(k+G) c_G e^{iG.r}, and of its Laplacian,
  sum_G -|k+G|^2 c_G e^{iG.r} (k = 0 for Gamma orbitals, whose samples are real).
* Coefficient draw: E|c_G|^2 = exp(-|G|^2 / decay).  On the half space
  H = {n : first nonzero Miller index > 0}, Re and Im are independent
  N(0, exp(-|G|^2/decay)/2); the partner -n gets the conjugate; c_0 ~ N(0, 1).
  Draw order: one array standard_normal((n_orb, 1 + 2*|H|)); column 0 is c_0,
  columns 1+2h and 2+2h are (Re, Im) of the h-th member of H in lexicographic
  Miller order.
* Random streams: SeedSequence(seed_key).spawn(2) -> (coefficients, positions).

Nothing here evaluates a spline; grid samples come from numpy's inverse FFT,
which is exact for any grid because every e^{iG.r} is sampled at the grid points
without approximation (several G falling into one FFT bin add up).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BOHR_PER_ANGSTROM = 1.0 / 0.529177210903


def gvectors(lattice: np.ndarray, gcut: float, kvec=None):
    """All reciprocal-lattice vectors with |k + G| < gcut (strict; k = 0 by default),
    lexicographic in (n1, n2, n3).

    Returns (miller [N_G, 3] int64, gvecs [N_G, 3] float64).
    """
    lattice = np.asarray(lattice, dtype=np.float64)
    k = np.zeros(3) if kvec is None else np.asarray(kvec, dtype=np.float64)
    inv = np.linalg.inv(lattice)            # columns of inv are b_j / (2 pi)
    reach = gcut + float(np.linalg.norm(k))
    nmax = [int(math.ceil(reach * np.linalg.norm(lattice[i]) / (2.0 * math.pi))) for i in range(3)]
    r = [np.arange(-m, m + 1, dtype=np.int64) for m in nmax]
    n = np.stack(np.meshgrid(*r, indexing="ij"), axis=-1).reshape(-1, 3)   # lexicographic
    g = 2.0 * math.pi * (n.astype(np.float64) @ inv.T)
    q = g + k
    keep = np.einsum("ij,ij->i", q, q) < gcut * gcut
    return n[keep], g[keep]


def draw_coefficients(miller: np.ndarray, gvecs: np.ndarray, n_orb: int, decay: float,
                      rng: np.random.Generator) -> np.ndarray:
    """Complex coefficients c[o, G] of real (Gamma-point) orbitals; see the module docstring."""
    miller = np.asarray(miller)
    n_g = miller.shape[0]
    first_nz = np.zeros(n_g, dtype=np.int64)
    for ax in (2, 1, 0):                       # first nonzero index, scanning n1, n2, n3
        nz = miller[:, ax] != 0
        first_nz = np.where(nz, miller[:, ax], first_nz)
    half = np.nonzero(first_nz > 0)[0]
    zero = np.nonzero(np.all(miller == 0, axis=1))[0]
    index = {tuple(m): i for i, m in enumerate(miller.tolist())}
    partner = np.array([index[(-m[0], -m[1], -m[2])] for m in miller[half].tolist()], dtype=np.int64)

    z = rng.standard_normal((n_orb, 1 + 2 * half.size))
    c = np.zeros((n_orb, n_g), dtype=np.complex128)
    if zero.size:
        c[:, zero[0]] = z[:, 0]
    g2 = np.einsum("ij,ij->i", gvecs[half], gvecs[half])
    scale = np.sqrt(np.exp(-g2 / decay) / 2.0)
    c[:, half] = (z[:, 1::2] + 1j * z[:, 2::2]) * scale
    c[:, partner] = np.conj(c[:, half])
    return c


def draw_bloch_coefficients(gvecs: np.ndarray, kvec, n_orb: int, decay: float,
                            rng: np.random.Generator) -> np.ndarray:
    """Complex coefficients c[o, G] of the periodic parts of Bloch orbitals; see the module docstring."""
    q = np.asarray(gvecs, dtype=np.float64) + np.asarray(kvec, dtype=np.float64)
    q2 = np.einsum("ij,ij->i", q, q)
    z = rng.standard_normal((n_orb, 2 * q.shape[0]))
    scale = np.sqrt(np.exp(-q2 / decay) / 2.0)
    return (z[:, 0::2] + 1j * z[:, 1::2]) * scale


def _grid_from_coef(miller, coef, grid, chunk=16, out=None, keep_complex=False):
    n1, n2, n3 = (int(v) for v in grid)
    n_orb = coef.shape[0]
    if out is None:
        out = np.empty((n1, n2, n3, n_orb), dtype=np.complex128 if keep_complex else np.float64)
    bins = np.ravel_multi_index(tuple((np.asarray(miller) % np.array([n1, n2, n3])).T), (n1, n2, n3))
    total = n1 * n2 * n3
    for o0 in range(0, n_orb, chunk):
        nc = min(chunk, n_orb - o0)
        spec = np.zeros((nc, total), dtype=np.complex128)
        np.add.at(spec, (np.arange(nc)[:, None], bins[None, :]), coef[o0:o0 + nc])
        x = np.fft.ifftn(spec.reshape(nc, n1, n2, n3), axes=(1, 2, 3))
        x *= total
        out[..., o0:o0 + nc] = np.moveaxis(x if keep_complex else x.real, 0, -1)
    return out


def sample_grid(miller, coef, grid, out=None):
    """phi_o at r_ijk = a (i/N1, j/N2, k/N3): array [N1][N2][N3][n_orb] float64, orbital innermost."""
    return _grid_from_coef(miller, coef, grid, out=out)


def sample_grid_laplacian(miller, gvecs, coef, grid, out=None):
    """Grid samples of the planewave Laplacian, sum_G (-|G|^2) c_G e^{iG.r} (input of a separate Laplacian spline)."""
    g2 = np.einsum("ij,ij->i", gvecs, gvecs)
    return _grid_from_coef(miller, coef * (-g2)[None, :], grid, out=out)


def draw_positions(lattice, n_pts: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform points in the cell: s ~ U[0,1)^3, r = a s (row form r = s @ lattice).  [n_pts][3] float64."""
    s = rng.random((int(n_pts), 3))
    return s @ np.asarray(lattice, dtype=np.float64)


@dataclasses.dataclass
class System:
    """One periodic cell with its planewave orbitals (everything the generator knows about it)."""
    name: str
    lattice: np.ndarray          # [3,3], rows a_i, bohr
    grid: tuple                  # (N1, N2, N3)
    n_orb: int
    gcut: float
    decay: float
    seed_key: tuple
    kvec: tuple = None           # crystal momentum (1/bohr) of Bloch orbitals; None = real Gamma orbitals
    miller: np.ndarray = None
    gvecs: np.ndarray = None
    coef: np.ndarray = None

    def __post_init__(self):
        self.lattice = np.asarray(self.lattice, dtype=np.float64)
        self.grid = tuple(int(v) for v in self.grid)
        ss = np.random.SeedSequence(list(self.seed_key))
        self._ss_coef, self._ss_pos = ss.spawn(2)
        if self.kvec is not None:
            self.kvec = tuple(float(v) for v in self.kvec)
        if self.miller is None:
            rng = np.random.Generator(np.random.PCG64(self._ss_coef))
            self.miller, self.gvecs = gvectors(self.lattice, self.gcut, self.kvec)
            if self.kvec is None:
                self.coef = draw_coefficients(self.miller, self.gvecs, self.n_orb, self.decay, rng)
            else:
                self.coef = draw_bloch_coefficients(self.gvecs, self.kvec, self.n_orb, self.decay, rng)

    @property
    def bloch(self) -> bool:
        return self.kvec is not None

    @property
    def k(self) -> np.ndarray:
        """Crystal momentum as an array (zeros for Gamma orbitals)."""
        return np.zeros(3) if self.kvec is None else np.asarray(self.kvec, dtype=np.float64)

    @property
    def qvecs(self) -> np.ndarray:
        """k + G for every planewave: the wavevectors of the orbital's planewaves."""
        return self.gvecs + self.k

    @property
    def n_g(self) -> int:
        return int(self.miller.shape[0])

    def nyquist_ok(self) -> bool:
        """Grid resolves every G without aliasing: N_i > 2 max|n_i|."""
        return all(self.grid[i] > 2 * int(np.abs(self.miller[:, i]).max()) for i in range(3))

    def grid_values(self, out=None) -> np.ndarray:
        """Samples of u (the orbital itself at Gamma): [N1][N2][N3][n_orb], complex for Bloch orbitals."""
        return _grid_from_coef(self.miller, self.coef, self.grid, out=out, keep_complex=self.bloch)

    def grid_laplacian(self, out=None) -> np.ndarray:
        """Samples of the periodic part of the orbital's Laplacian, sum_G -|k+G|^2 c_G e^{iG.r}."""
        q = self.qvecs
        q2 = np.einsum("ij,ij->i", q, q)
        return _grid_from_coef(self.miller, self.coef * (-q2)[None, :], self.grid, out=out,
                               keep_complex=self.bloch)

    def grid_gradient(self) -> np.ndarray:
        """Samples of the periodic part of the orbital's gradient, sum_G i(k+G) c_G e^{iG.r}:
        [3][N1][N2][N3][n_orb] (Cartesian component first), complex for Bloch orbitals."""
        q = self.qvecs
        return np.stack([_grid_from_coef(self.miller, self.coef * (1j * q[:, a])[None, :], self.grid,
                                         keep_complex=self.bloch) for a in range(3)])

    def positions(self, n_pts: int) -> np.ndarray:
        return draw_positions(self.lattice, n_pts, np.random.Generator(np.random.PCG64(self._ss_pos)))


def make_system(name, lattice, grid, n_orb, gcut, decay, seed_key, kvec=None) -> System:
    return System(name=name, lattice=lattice, grid=grid, n_orb=n_orb, gcut=gcut, decay=decay,
                  seed_key=tuple(seed_key), kvec=kvec)
