"""CPU check of the per-point indexing that every kernel runs (coordinate reduction, Sec. II
Eq. reducedcoordinate; the four wrapped rows per axis of App. A Eq. b-splineapproximation).

tests/index_check.hip includes the library's own reduce_point and wrap4 (host and device
functions) and takes the geometry from the built library (spline_desc_init, make_geom).  It is
built here for the host with AddressSanitizer and UndefinedBehaviorSanitizer and driven over
adversarial positions: far images (up to 1e300), tiny negatives that round the crystal
coordinate up to the cell edge, exact grid planes and their neighbours one ulp away, signed
zeros, subnormals and non-finite values, on grids of 4 to 1024 points per axis.  Every index
must lie in [0, N), every t in [0, 1), every one of the 64 block rows inside the table, and
(i0, t) must agree with the oracle's reduced coordinates up to the rounding of s.
"""
import glob
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import evaluate

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1309_6250_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
LIB = os.path.join(PKG, "libpwspline.so")

SKEW = np.array([[7.0, 0.4, -0.3], [1.1, 6.2, 0.5], [-0.6, 0.9, 8.3]])
FCC = 5.1306 * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
CUBE = np.diag([20.5224] * 3)


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    runtime = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not shutil.which(HIPCC) or not os.path.exists(LIB) or not runtime:
        pytest.skip("needs hipcc, the built library and the host ASan runtime")
    out = str(tmp_path_factory.mktemp("idx") / "index_check")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-shared-libsan",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           os.path.join(ROOT, "tests", "index_check.hip"), "-o", out,
           f"-L{PKG}", "-lpwspline", f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{os.path.dirname(runtime[0])}"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    return out


def run_check(exe, lattice, grid, pos, pp=False):
    lines = [" ".join(float(x).hex() for x in np.asarray(lattice, dtype=np.float64).reshape(-1)),
             f"{grid[0]} {grid[1]} {grid[2]} 1 {int(pp)} {len(pos)}"]
    lines += [" ".join(float(x).hex() for x in p) for p in pos]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
    rows = [ln.split() for ln in res.stdout.strip().splitlines()]
    assert len(rows) == len(pos)
    ok = np.array([int(r[0]) for r in rows], dtype=bool)
    i0 = np.array([[int(x) for x in r[1:4]] for r in rows])
    t = np.array([[float.fromhex(x) for x in r[4:7]] for r in rows])
    in_range = np.array([int(r[7]) for r in rows], dtype=bool)
    return ok, i0, t, in_range


def adversarial_points(lattice, grid, seed):
    rng = np.random.default_rng(seed)
    n = np.asarray(grid)
    s = [rng.uniform(-50, 50, size=(400, 3))]                             # far images
    # exact grid planes (crystal coordinate k/N, k = 0..N, so the far edge is included) and the
    # neighbouring doubles one ulp on either side
    k = rng.integers(0, n + 1, size=(300, 3))
    planes = k / n
    s += [planes, np.nextafter(planes, -np.inf), np.nextafter(planes, np.inf)]
    s += [np.full((1, 3), -1e-300), np.full((1, 3), -5e-324), np.full((1, 3), 5e-324), np.full((1, 3), -0.0),
          np.full((1, 3), 1.0 - 2.0**-53), np.full((1, 3), -2.0**-53), np.full((1, 3), 2.0**52 + 0.5)]
    s = np.concatenate(s)
    pos = [s @ lattice]
    # Cartesian extremes, as given
    ext = np.array([[1e300, -1e300, 1e300], [-1e300, 1e300, 3.0], [1e308, 1e308, 1e308], [-1e308, 1.0, 2.0],
                    [1e-300, -1e-300, 0.0], [-0.0, -0.0, -0.0], [np.nan, 0.0, 0.0], [0.0, np.inf, 0.0],
                    [0.0, 0.0, -np.inf], [2.0**60, -2.0**61, 2.0**62]])
    pos.append(ext)
    # one ulp below every lattice vector's image of the origin
    pos.append(np.nextafter(lattice, -np.inf))
    pos.append(-np.nextafter(np.zeros((3, 3)), np.inf))
    return np.concatenate(pos)


CASES = [(SKEW, (4, 4, 4)), (SKEW, (1024, 5, 7)), (FCC, (16, 16, 16)), (CUBE, (4, 1024, 1024)), (CUBE, (48, 48, 48))]


@pytest.mark.parametrize("lattice,grid", CASES)
@pytest.mark.parametrize("pp", [False, True])
def test_indices_in_range_and_match_oracle(checker, lattice, grid, pp):
    pos = adversarial_points(lattice, grid, seed=sum(grid) + int(pp))
    ok, i0, t, in_range = run_check(checker, lattice, grid, pos, pp)
    n = np.asarray(grid)
    assert in_range.all()
    assert np.all((i0 >= 0) & (i0 < n)) and np.all((t >= 0) & (t < 1))
    assert np.all(i0[~ok] == 0) and np.all(t[~ok] == 0)
    ri0, rt, rok = evaluate.reduced_coordinates(lattice, grid, pos)
    # Cartesian inputs too large for the crystal coordinates may overflow in one route and
    # not the other; every other point agrees on finiteness
    huge = np.abs(np.nan_to_num(pos, nan=0.0, posinf=0.0, neginf=0.0)).max(axis=1) > 1e307
    assert np.array_equal(ok[~huge], rok[~huge])
    both = ok & rok
    # the rounding of s = a^-1 r: a few ulps of sum_j |a^-1_ij| |r_j| (not of |s_i|, which
    # cancellation can make far smaller), times N in grid units
    safe = np.where(both[:, None], pos, 0.0)
    sabs = np.abs(np.linalg.inv(np.asarray(lattice).T)) @ np.abs(safe).T
    tol = 16 * n * np.spacing(np.maximum(sabs.T, 1.0)) + 1e-15
    du = (i0 + t) - (ri0 + rt)                                   # in grid units
    du = (du + n / 2) % n - n / 2                                # across the periodic wrap
    bad = both[:, None] & (np.abs(du) > tol)
    assert not bad.any(), (pos[bad.any(axis=1)][:5], i0[bad.any(axis=1)][:5], ri0[bad.any(axis=1)][:5])
    # where the two routes round to the same cell, t agrees to the same tolerance
    same = both[:, None] & (i0 == ri0)
    assert np.all(np.abs(t - rt)[same] <= tol[same])


def test_edge_cases_exact(checker):
    """Points whose result is fixed exactly: the origin, a tiny negative coordinate (its
    fold rounds to 1.0, so the index wraps to 0 with t = 0), and an exact lattice vector."""
    grid = (8, 9, 10)
    pos = np.array([[0.0, 0.0, 0.0], [-1e-300, -1e-300, -1e-300], CUBE[0], CUBE[0] + CUBE[1] + CUBE[2], [-0.0] * 3])
    ok, i0, t, in_range = run_check(checker, CUBE, grid, pos)
    assert ok.all() and in_range.all()
    assert np.all(i0 == 0) and np.all(t == 0)
