"""Named synthetic workloads shaped like the paper's Si, Al and MgO cells.

The paper's orbitals are DFT Gamma-point orbitals of diamond Si, fcc Al and
rock-salt MgO (Sec. III); none are available, so seeded planewave orbitals with
a Gaussian spectral decay stand in for them, on cells of the same shape.

  0  Si fcc primitive cell (a = 5.43 A), 4 orbitals, Gcut 4 1/bohr, 16^3 grid,
     8 electrons x 1 walker + 4096 uniform points (small case).
  1  64-atom Si 2x2x2 conventional cubic cell, 128 orbitals, Gcut 4, 48^3 grid,
     256 walkers x 256 electrons.
  2  MgO-like 2x2x2 rock-salt cubic cell (a = 4.21 A), 256 orbitals, Gcut 8 with
     the slower decay exp(-|G|^2/8), 96^3 grid, separate Laplacian table,
     512 walkers x 128 electrons.
  3  48 independent cubic cells of uneven size (see batched_systems).
  4  as 1 but a 32^3 grid and 10^6 fit points (smoothing fit).
  5  Al fcc primitive cell (a = 4.05 A), 4 orbitals, 16^3 grid (Al-like variant of 0).
  6  Bloch orbitals at the L point, k = (pi/a)(1,1,1), of the Si fcc primitive cell of 0:
     4 complex orbitals, 16^3 grid, 8 + 4096 points (small case).
  7  Bloch orbitals in config 1's cell at the supercell zone-corner twist k = (pi/L)(1,1,1),
     L = 2a: 128 complex orbitals, 48^3 grid, 256 walkers x 256 electrons.
  8  64-atom Al-like cell at the scale of 1: the fcc primitive cell (a = 4.05 A) repeated
     4x4x4 along its own (non-orthogonal) lattice vectors, 3 valence electrons per atom,
     so 96 orbitals and 192 electrons; Gcut 4, 50^3 grid (spacing 0.43 bohr, as in 1),
     256 walkers x 192 electrons.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .synth import BOHR_PER_ANGSTROM, System, make_system

SEED = (1309, 6250)
A_SI = 5.43 * BOHR_PER_ANGSTROM
A_MGO = 4.21 * BOHR_PER_ANGSTROM
A_AL = 4.05 * BOHR_PER_ANGSTROM
BATCH_SPACING = 2.0 * A_SI / 48.0          # config 1's grid spacing, reused by the batched cells


def fcc_primitive(a):
    return 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])


def cubic(length):
    return length * np.eye(3)


@dataclasses.dataclass
class Workload:
    key: int
    system: System
    n_walkers: int
    n_elec: int
    dtypes: tuple
    has_lap: bool
    extra_points: int = 0

    @property
    def n_pts(self) -> int:
        return self.n_walkers * self.n_elec + self.extra_points

    def positions(self) -> np.ndarray:
        return self.system.positions(self.n_pts)


CONFIGS = {
    0: dict(name="si-fcc-prim-16", lattice=lambda: fcc_primitive(A_SI), grid=(16, 16, 16), n_orb=4,
            gcut=4.0, decay=2.0, walkers=1, elec=8, extra=4096, dtypes=("f64",), has_lap=False),
    1: dict(name="si64-cubic-48", lattice=lambda: cubic(2.0 * A_SI), grid=(48, 48, 48), n_orb=128,
            gcut=4.0, decay=2.0, walkers=256, elec=256, extra=0, dtypes=("f64", "f32"), has_lap=False),
    2: dict(name="mgo-rocksalt-96", lattice=lambda: cubic(2.0 * A_MGO), grid=(96, 96, 96), n_orb=256,
            gcut=8.0, decay=8.0, walkers=512, elec=128, extra=0, dtypes=("f64", "f32", "bf16"),
            has_lap=True),
    4: dict(name="si64-cubic-32-fit", lattice=lambda: cubic(2.0 * A_SI), grid=(32, 32, 32), n_orb=128,
            gcut=4.0, decay=2.0, walkers=1, elec=1_000_000, extra=0, dtypes=("f32",), has_lap=False),
    5: dict(name="al-fcc-prim-16", lattice=lambda: fcc_primitive(A_AL), grid=(16, 16, 16), n_orb=4,
            gcut=4.0, decay=2.0, walkers=1, elec=8, extra=4096, dtypes=("f64",), has_lap=False),
    6: dict(name="si-fcc-prim-16-L", lattice=lambda: fcc_primitive(A_SI), grid=(16, 16, 16), n_orb=4,
            gcut=4.0, decay=2.0, walkers=1, elec=8, extra=4096, dtypes=("f64",), has_lap=False,
            kvec=lambda: (np.pi / A_SI) * np.ones(3)),
    7: dict(name="si64-cubic-48-twist", lattice=lambda: cubic(2.0 * A_SI), grid=(48, 48, 48), n_orb=128,
            gcut=4.0, decay=2.0, walkers=256, elec=256, extra=0, dtypes=("f64", "f32"), has_lap=False,
            kvec=lambda: (np.pi / (2.0 * A_SI)) * np.ones(3)),
    8: dict(name="al64-fcc-4x4x4-50", lattice=lambda: 4.0 * fcc_primitive(A_AL), grid=(50, 50, 50), n_orb=96,
            gcut=4.0, decay=2.0, walkers=256, elec=192, extra=0, dtypes=("f64", "f32", "bf16"), has_lap=False),
}


def config(key: int) -> Workload:
    """The named single-system workload ``key`` (0, 1, 2, 4, 5, 6, 7 or 8)."""
    c = CONFIGS[key]
    kvec = c["kvec"]() if "kvec" in c else None
    sysm = make_system(c["name"], c["lattice"](), c["grid"], c["n_orb"], c["gcut"], c["decay"],
                       SEED + (key,), kvec=kvec)
    return Workload(key=key, system=sysm, n_walkers=c["walkers"], n_elec=c["elec"],
                    dtypes=c["dtypes"], has_lap=c["has_lap"], extra_points=c["extra"])


def batched_systems(n_systems: int = 48, scale: float = 1.0):
    """Config 3: uneven systems drawn from SeedSequence(1309, 6250, 3).

    Per system j: orbitals ~ U{32..256}, cubic grid N ~ U{24..64} with cell
    length N * BATCH_SPACING, walkers ~ U{16..512}, electrons ~ U{64..256};
    Gcut 4, decay 2; its orbitals and positions come from SeedSequence(1309, 6250, 3, j).
    ``scale`` < 1 shrinks walker counts (for fast tests) without changing the rest.
    Returns a list of Workload.
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(SEED + (3,)))))
    n_orb = rng.integers(32, 257, size=n_systems)
    n_grid = rng.integers(24, 65, size=n_systems)
    walkers = rng.integers(16, 513, size=n_systems)
    elec = rng.integers(64, 257, size=n_systems)
    out = []
    for j in range(n_systems):
        n = int(n_grid[j])
        sysm = make_system(f"batch-{j}", cubic(n * BATCH_SPACING), (n, n, n), int(n_orb[j]), 4.0, 2.0,
                           SEED + (3, j))
        w = max(1, int(round(int(walkers[j]) * scale)))
        out.append(Workload(key=3, system=sysm, n_walkers=w, n_elec=int(elec[j]), dtypes=("f32",),
                            has_lap=False))
    return out
