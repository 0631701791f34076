#!/usr/bin/env python3
"""Orbital-VGL throughput of the periodic B-spline library on one MI355X.

A step is one VGL sweep (value, gradient and Laplacian of every orbital at every point of one
walker population) through spline_eval_vgl.  The headline workload is the MgO-like rock-salt cell:
256 orbitals on a 96^3 grid, 512 walkers x 128 electrons, FP64 coefficient table (1.8 GB, far
beyond the 256 MB Infinity Cache, so the gather is served by HBM).  Inputs (table and positions)
are resident in HBM before timing starts.

The last stdout line is one compact JSON record (under 4 KB): the headline, its roofline, the
FP32 / BF16 forms' speedups at their measured error, the CPU oracle baseline.  Everything else
goes to a detail file (--detail, default gpurun_out/bench_detail.json):
  forms     every precision form (FP64 / FP32 / BF16 tables, with and without a separate Laplacian
            spline) on the MgO-like cell; five separate tables (B-spline or Lagrange) and the
            pp-spline form there; the Si-like and Al-like 64-atom cells and Bloch orbitals at a
            twist (tables that fit the Infinity Cache: their fractions of the HBM peak are
            "effective"); the locality-ordered (sorted) call of each, also effective;
  rows      spline_build, spline_eval_v, the adjoint, the batched persistent launch, the fit
            (200 Adam steps and the exact optimum by conjugate gradients), the smoothing build,
            the paper's comparison of methods, and the read and copy ceilings of device memory.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick] [--only FORM] [--detail PATH]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MALL_BYTES = 256 << 20          # Infinity Cache: tables at or below this size are largely cache-served
METRIC = "orbital-VGL evals/sec + % HBM peak, FP64 vs FP32/BF16 at stated error"
# FP64 operations of one orbital-VGL in the forward kernel: per first-axis slab, 4 x (three 4-term dot
# products = 12 FMA, six second-axis FMA) + 10 first-axis FMA = 82 FMA, times 4 slabs, plus the chain
# rule (9 FMA for the gradient, 7 for the Laplacian): 344 FMA = 688 flops
FLOPS_PER_EVAL = 688
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ("paper_1309_6250_amd/csrc/eval_impl.hpp", "paper_1309_6250_amd/csrc/common.hpp")
STORE_BYTES = {"f64": 8, "f32": 4, "bf16": 2}
# Adam on the fit: step size relative to the rms of the interpolating table, and its schedule
FIT_LR = 0.1
FIT_SCHEDULE = "cosine"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def bytes_per_eval(dtype, n_tables=1, cols=1):
    """Algorithmic HBM bytes of one orbital-VGL: 64 coefficients of each table read (1; 2 with a
    separate Laplacian; 5 with separate gradients) plus 5 outputs, per stored column (2 for a Bloch
    orbital's real and imaginary parts); positions add 24 bytes per point."""
    out = 8 if dtype == "f64" else 4
    return cols * (64 * STORE_BYTES[dtype] * n_tables + 5 * out)


def time_launches(fn, steps, warmup):
    """Average ms per call of fn() over `steps` calls, HIP events on torch's current stream
    (the stream the library launches on), bracketed by device synchronizations."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def normwise(a, b):
    import numpy as np
    return float(np.nanmax(np.abs(a - b)) / np.nanmax(np.abs(b)))


class Workload:
    """One single-system workload: host inputs at construction, device copies on upload()."""

    def __init__(self, key, lap=False):
        from workloads import config
        self.key = key
        self.w = config(key)
        s = self.w.system
        self.s = s
        t0 = time.time()
        self.f_host = s.grid_values()
        self.lf_host = s.grid_laplacian() if lap else None
        self.pos_host = self.w.positions()
        log(f"config {key} ({s.name}) host inputs in {time.time() - t0:.1f} s")

    def upload(self):
        import torch
        self.f = torch.from_numpy(self.f_host).cuda()          # complex128 for Bloch orbitals
        self.lf = None if self.lf_host is None else torch.from_numpy(self.lf_host).cuda()
        self.pos = torch.from_numpy(self.pos_host).cuda()
        torch.cuda.synchronize()
        return self

    def describe(self, dtype, has_lap):
        s = self.s
        out = {"workload": s.name, "n_orb": s.n_orb, "grid": list(s.grid), "walkers": self.w.n_walkers,
               "electrons": self.w.n_elec, "points": int(self.pos.shape[0]), "table": dtype,
               "separate_laplacian": bool(has_lap), "lattice_bohr": [round(x, 6) for x in s.lattice.reshape(-1)]}
        if s.bloch:
            out["kvec_per_bohr"] = [round(x, 8) for x in s.k]
        return out


def frac_key(table_bytes):
    """Key of a form's algorithmic-bandwidth fraction of the HBM peak: "frac_hbm_peak" where the tables
    exceed the Infinity Cache (the gather is served by HBM), "effective_frac_hbm_peak" where they fit
    in it (rows come partly from the cache, and the figure may pass 1)."""
    return "frac_hbm_peak" if table_bytes > MALL_BYTES else "effective_frac_hbm_peak"


def run_form(wl, dtype, has_lap, steps, warmup, tune=True, tile=None, sep=None, fields=None, basis="bspline"):
    """Build, autotune (or take `tile`) and time one form; returns (record, desc, table, outputs).

    sep: None (derivatives of the orbital table, plus a separate Laplacian table with has_lap; basis
    "bspline" or its piecewise-polynomial form "pp") or "bspline" / "lagrange" (five separate tables
    built from `fields`, the stacked device grid values).  Bloch orbitals follow from the workload's
    crystal momentum."""
    import torch
    import paper_1309_6250_amd as P
    s = wl.s
    kvec = s.k if s.bloch else None
    if sep:
        d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, dtype, has_lap=True, sep_grad=True, basis=sep, kvec=kvec)
    else:
        d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, dtype, has_lap=has_lap, kvec=kvec, basis=basis)
    work = None if sep == "lagrange" else torch.empty(d.work_bytes // 8, dtype=torch.float64, device="cuda")
    table = P.new_table(d)
    if sep:
        build_ms = time_launches(lambda: P.spline_build_tables(d, fields, table, work), 1, 1)
    else:
        build_ms = time_launches(lambda: P.spline_build(d, wl.f, wl.lf if has_lap else None, table, work), 1, 1)
    outs = P.spline_eval_vgl(d, table, wl.pos, tile=tile)
    if tile is None:
        tile = P.spline_autotune(d, table, wl.pos, *outs) if tune else P.spline_tile_for(d)
    ms = time_launches(lambda: P.spline_eval_vgl(d, table, wl.pos, *outs, tile=tile), steps, warmup)
    n_pts, n_orb = wl.pos.shape[0], s.n_orb
    evals = n_pts * n_orb
    alg = evals * bytes_per_eval(dtype, d.n_tables, 2 if s.bloch else 1) + 24 * n_pts
    rec = {
        "evals_per_s": evals / (ms * 1e-3),
        "ms_per_sweep": ms,
        "alg_bytes_per_sweep": alg,
        "alg_GBps": alg / (ms * 1e-3) / 1e9,
        frac_key(d.table_bytes): alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "tile": list(tile),
        "table_bytes": int(d.table_bytes),
        "build_ms": build_ms,
    }
    del work
    return rec, d, table, outs


OPLS = {"f64": (1, 2), "f32": (1, 2, 4), "bf16": (2, 4, 8)}


def sorted_form(wl, d, table, outs, dtype, steps, warmup, tile=None):
    """The same evaluation through spline_eval_vgl_sorted: a counting sort of the points into Morton
    buckets of cells and the permuted kernel, all inside every timed call.  The tile is the fastest of a sweep (three timed
    calls each).  alg_GBps counts each point's 64 rows as if read from memory, as for the other
    forms; rows reused from L2 or the Infinity Cache can take it past the HBM peak."""
    import torch
    import paper_1309_6250_amd as P
    n_pts = int(wl.pos.shape[0])
    work = torch.empty(P.spline_sorted_work_bytes(d, n_pts), dtype=torch.uint8, device="cuda")
    if tile is None:
        best = None
        for opl in OPLS[dtype]:
            if d.bloch and opl % 2:
                continue                       # Bloch lanes hold whole (re, im) pairs
            for g in (4, 8, 16, 32, 64, 128, 256):
                ms = time_launches(lambda: P.spline_eval_vgl_sorted(d, table, wl.pos, *outs, work=work, tile=(g, opl)),
                                   3, 1)
                if best is None or ms < best[0]:
                    best = (ms, (g, opl))
        tile = best[1]
    ms = time_launches(lambda: P.spline_eval_vgl_sorted(d, table, wl.pos, *outs, work=work, tile=tile), steps, warmup)
    evals = n_pts * d.n_orb
    alg = evals * bytes_per_eval(dtype, d.n_tables, 2 if d.bloch else 1) + 24 * n_pts
    return {"evals_per_s": evals / (ms * 1e-3), "ms_per_sweep": ms, "alg_bytes_per_sweep": alg,
            "alg_GBps": alg / (ms * 1e-3) / 1e9,
            "effective_frac_hbm_peak": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "tile": list(tile), "table_bytes": int(d.table_bytes),
            "note": "spline_eval_vgl_sorted; the sort of the points runs inside every timed call; rows shared "
                    "by neighbouring points come from L2 and the Infinity Cache, so the fraction is effective"}


def grid_fields_gpu(system, chunk=16):
    """Fixture for the five-table forms: grid samples of the orbital (u for Bloch orbitals), of the
    periodic parts of its gradient, sum_G i(k+G) c_G e^{iG.r}, and of its Laplacian,
    sum_G -|k+G|^2 c_G e^{iG.r}, by inverse FFTs on the GPU (input generation, never timed).
    Returns FP64 [5][N1][N2][N3][n_col] on the device."""
    import numpy as np
    import torch
    s = system
    n1, n2, n3 = s.grid
    total = n1 * n2 * n3
    q = torch.from_numpy(s.qvecs).cuda()
    mults = [torch.ones(s.n_g, dtype=torch.complex128, device="cuda")]
    mults += [(1j * q[:, a]).to(torch.complex128) for a in range(3)]
    mults.append((-(q * q).sum(1)).to(torch.complex128))
    bins = torch.from_numpy(np.ravel_multi_index(tuple((s.miller % np.array(s.grid)).T), s.grid)).cuda()
    coef = torch.from_numpy(s.coef).cuda()
    n_col = s.n_orb * (2 if s.bloch else 1)
    out = torch.empty((5, n1, n2, n3, n_col), dtype=torch.float64, device="cuda")
    for t, m in enumerate(mults):
        for o0 in range(0, s.n_orb, chunk):
            nc = min(chunk, s.n_orb - o0)
            spec = torch.zeros((nc, total), dtype=torch.complex128, device="cuda")
            spec.index_add_(1, bins, coef[o0:o0 + nc] * m[None, :])
            x = (torch.fft.ifftn(spec.view(nc, n1, n2, n3), dim=(1, 2, 3)) * total).permute(1, 2, 3, 0)
            if s.bloch:
                out[t, ..., 2 * o0:2 * (o0 + nc)] = torch.view_as_real(x.contiguous()).reshape(n1, n2, n3, 2 * nc)
            else:
                out[t, ..., o0:o0 + nc] = x.real
    torch.cuda.synchronize()
    return out


def _host(t):
    import numpy as np
    return t.cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


def accuracy(wl, dtype, form, outs, n_sample=1024, n_orb_ref=None):
    """Errors of the GPU outputs on a seeded sample of points (all orbitals unless n_orb_ref is given):
    against the planewave sum (the representation's own approximation error) and, for FP32/BF16
    tables, against the FP64 table's outputs of the same representation `form` (the storage and
    arithmetic error).  The FP64 form must be measured first; its agreement with the FP64 oracle is
    what the parity tests check (and the headline's parity sample below)."""
    import numpy as np
    import torch
    idx = parity_sample(wl.pos_host.shape[0], n_sample)
    k = wl.s.n_orb if n_orb_ref is None else min(n_orb_ref, wl.s.n_orb)
    cache = wl.__dict__.setdefault("_accuracy_cache", {})
    if "pw" not in cache:
        x = wl.pos[torch.from_numpy(idx).cuda()].contiguous()
        cache["pw"] = planewave_vgl_gpu(wl.s, x, k)
    pwref = cache["pw"]
    got = [_host(outs[0])[idx, :k], _host(outs[1])[idx, :, :k], _host(outs[2])[idx, :k]]
    if dtype == "f64":
        cache[("f64", form)] = got
    f64 = cache.get(("f64", form))
    res = {}
    for j, (name, g, p) in enumerate(zip(("V", "grad", "lap"), got, pwref)):
        r = {"normwise_vs_planewave": normwise(g, p),
             "rmae_vs_planewave": float(np.abs(g - p).mean() / np.abs(p).mean())}
        if dtype != "f64" and f64 is not None:
            r["normwise_vs_fp64_table"] = normwise(g, f64[j])
            r["maxabs_vs_fp64_table"] = float(np.abs(g - f64[j]).max())
        res[name] = r
    res["sample"] = f"{n_sample} seeded points x {'all ' if k == wl.s.n_orb else 'first '}{k} orbitals"
    return res


def planewave_vgl_gpu(system, x, k, chunk=256):
    """Value, gradient and Laplacian of the first k planewave orbitals (Eq. pw_orbital; Bloch
    orbitals sum over k+G) at the points x (device, [n][3]), by direct summation over the
    planewaves in complex128 on the GPU: the exact function the representations approximate.
    Returns numpy arrays [n][k], [n][3][k], [n][k] (complex for Bloch orbitals, else real)."""
    import numpy as np
    import torch
    q = torch.from_numpy(system.qvecs).cuda()                       # [N_G][3]
    c = torch.from_numpy(system.coef[:k]).cuda()                    # [k][N_G]
    cv = c.t().contiguous()
    cg = [(1j * q[:, a][None, :] * c).t().contiguous() for a in range(3)]
    cl = (-(q * q).sum(1)[None, :] * c).t().contiguous()
    outs = [[], [], []]
    for p0 in range(0, x.shape[0], chunk):
        e = torch.exp(1j * (x[p0:p0 + chunk] @ q.t()))              # [n][N_G]
        v = e @ cv
        grad = torch.stack([e @ cg[a] for a in range(3)], 1)
        lap = e @ cl
        if not system.bloch:
            v, grad, lap = v.real, grad.real, lap.real
        for lst, t in zip(outs, (v, grad, lap)):
            lst.append(_host(t))
    return tuple(np.concatenate(lst) for lst in outs)


def _cores(max_workers=16):
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return max(1, min(max_workers, cores))      # never more than the box's 16-core share


def parity_sample(n_pts, n_sample=1024):
    """Seeded sample of point indices shared by the accuracy figures and the oracle parity check."""
    import numpy as np
    return np.sort(np.random.default_rng(1309).choice(n_pts, size=n_sample, replace=False))


def cpu_baseline(wl, n_sample=32768, max_workers=16):
    """The FP64 oracle (eval_vgl on the oracle's own interpolating table) on the host cores, over a
    seeded sample of the workload's points (its first n_sample points: the positions are already
    uniform random) and all its orbitals, split across forked worker processes.  Also returns the
    oracle's outputs on the parity sample, for the GPU outputs to be compared with."""
    import multiprocessing as mp
    import numpy as np
    from oracle import build as obuild, evaluate as oeval
    global _CPU_BETA, _CPU_LAT, _CPU_POS
    t0 = time.time()
    _CPU_BETA = obuild.build_interp(wl.f_host)
    _CPU_LAT = wl.s.lattice
    _CPU_POS = wl.pos_host[:n_sample]
    build_s = time.time() - t0
    workers = _cores(max_workers)
    n = _CPU_POS.shape[0]
    bounds = np.linspace(0, n, workers + 1).astype(int)
    ctx = mp.get_context("fork")
    t0 = time.time()
    with ctx.Pool(workers) as pool:
        pool.map(_cpu_worker, [(int(bounds[i]), int(bounds[i + 1])) for i in range(workers)])
    wall = time.time() - t0
    evals = n * wl.s.n_orb
    idx = parity_sample(wl.pos_host.shape[0])
    ref = oeval.eval_vgl(_CPU_BETA, _CPU_LAT, wl.pos_host[idx])
    _CPU_BETA = None
    return ({"value": evals / wall, "unit": "orbital-VGL evals/s", "cores": workers, "kind": "oracle",
             "sample": f"first {n} of the {wl.pos_host.shape[0]} points x all {wl.s.n_orb} orbitals of {wl.s.name} "
                       f"(FP64 table), {workers} processes, {wall:.1f} s wall ({workers * wall:.0f} core-s); oracle build "
                       f"{build_s:.0f} s not included",
             "wall_s": wall}, (idx, ref))


_CPU_BETA = _CPU_LAT = _CPU_POS = None
_CPU_JOB = None


def cpu_context(wl, n_pw=512, max_workers=16):
    """Host-side context in the same kind of pool: the direct planewave sum of every orbital on the
    headline cell (the O(N_G) per orbital-VGL work the splines replace)."""
    import multiprocessing as mp
    import numpy as np
    global _CPU_JOB
    workers = _cores(max_workers)
    s = wl.s
    _CPU_JOB = (s.gvecs, s.coef, wl.pos_host[:n_pw])
    bounds = np.linspace(0, n_pw, workers + 1).astype(int)
    t0 = time.time()
    with mp.get_context("fork").Pool(workers) as pool:
        pool.map(_cpu_pw_worker, [(int(bounds[i]), int(bounds[i + 1])) for i in range(workers)])
    wall = time.time() - t0
    _CPU_JOB = None
    return {"planewave_sum_vgl": {"evals_per_s": n_pw * s.n_orb / wall, "cores": workers, "n_g": int(s.n_g),
                                  "sample": f"{n_pw} points x {s.n_orb} orbitals of {s.name}", "wall_s": wall}}


def _cpu_pw_worker(rng_):
    from threadpoolctl import threadpool_limits
    from oracle import pw as opw
    a, b = rng_
    with threadpool_limits(1):
        opw.pw_vgl(_CPU_JOB[0], _CPU_JOB[1], _CPU_JOB[2][a:b])
    return b - a


def _cpu_worker(rng_):
    from threadpoolctl import threadpool_limits
    from oracle import evaluate as oeval
    with threadpool_limits(1):
        a, b = rng_
        oeval.eval_vgl(_CPU_BETA, _CPU_LAT, _CPU_POS[a:b])
    return rng_[1] - rng_[0]


def oracle_parity(outs, parity, dtype):
    """Normwise error of GPU outputs against the oracle's FP64 outputs on the parity sample."""
    idx, ref = parity
    got = [_host(outs[0])[idx], _host(outs[1])[idx], _host(outs[2])[idx]]
    return {name: normwise(g, r) for name, g, r in zip(("V", "grad", "lap"), got, ref)}


def traffic_for(form_key, tile):
    """Measured HBM bytes per launch from the committed rocprof counter summary for this form at this
    tile, or None when the counters were taken at another tile or the kernel sources changed since."""
    try:
        with open(PROFILE_TRAFFIC) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = data.get("forms", {}).get(f"{form_key}@{tile[0]},{tile[1]}")
    if not ent or ent.get("kernel_hash") != kernel_hash():
        return None
    return ent.get("bytes_per_launch")


def rows_measurements(wl1, steps, warmup):
    """The other entry points of the path, timed on the Si workload."""
    import torch
    import paper_1309_6250_amd as P
    out = {}
    s = wl1.s
    n_pts = wl1.pos.shape[0]
    # spline_build (three-stage cyclic solves): each stage reads and writes the FP64 grid once
    for dtype in ("f64", "f32"):
        d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, dtype)
        work = torch.empty(d.work_bytes // 8, dtype=torch.float64, device="cuda")
        table = P.new_table(d)
        ms = time_launches(lambda: P.spline_build(d, wl1.f, None, table, work), max(3, steps // 4), 1)
        pts = s.grid[0] * s.grid[1] * s.grid[2]
        alg = 5 * pts * s.n_orb * 8 + pts * d.o_pad * STORE_BYTES[dtype]
        out[f"spline_build_{dtype}"] = {"ms": ms, "alg_GBps": alg / (ms * 1e-3) / 1e9,
                                        "note": "3 stages: read+write FP64 twice, read FP64 + write table once"}
    # spline_eval_v
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f64")
    table = P.spline_build(d, wl1.f)
    v = P.spline_eval_v(d, table, wl1.pos)
    ms = time_launches(lambda: P.spline_eval_v(d, table, wl1.pos, v), steps, warmup)
    alg = n_pts * s.n_orb * (64 * 8 + 8) + 24 * n_pts
    out["spline_eval_v_f64"] = {"ms": ms, "evals_per_s": n_pts * s.n_orb / (ms * 1e-3),
                                "alg_GBps": alg / (ms * 1e-3) / 1e9}
    # adjoint (FP32 table, all three upstream gradients)
    d32 = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f32")
    t32 = P.spline_build(d32, wl1.f)
    g = torch.Generator(device="cuda").manual_seed(7)
    gv = torch.randn((n_pts, s.n_orb), device="cuda", generator=g)
    gg = torch.randn((n_pts, 3, s.n_orb), device="cuda", generator=g)
    gl = torch.randn((n_pts, s.n_orb), device="cuda", generator=g)
    gt = P.new_gtable(d32)
    gp = torch.empty((n_pts, 3), dtype=torch.float64, device="cuda")
    for name, flags in (("atomic", 0), ("deterministic", P.SPL_DETERMINISTIC)):
        ms = time_launches(lambda: P.spline_eval_vgl_backward(d32, t32, wl1.pos, gv, gg, gl, gt, gp, flags=flags),
                           max(3, steps // 4), 1)
        out[f"spline_eval_vgl_backward_f32_{name}"] = {
            "ms": ms, "evals_per_s": n_pts * s.n_orb / (ms * 1e-3), "workload": s.name,
            "note": "all three upstream terms; d pos by the per-point gather, d table by "
                    + ("atomic scatter-add" if not flags else "the cell-sorted matrix-core sums")}
    return out


def planewave_targets_gpu(system, pos, chunk=16384):
    """Fixture for the fit: value and Laplacian of the planewave orbitals (Eq. pw_orbital) at the fit
    points, as dense complex matmuls on the GPU.  Input generation only, outside every timed region."""
    import torch
    g = torch.from_numpy(system.gvecs).cuda()
    c = torch.from_numpy(system.coef).cuda()                       # [O, N_G] complex128
    g2 = (g * g).sum(1)
    cv = c.t().contiguous()
    cl = (c * (-g2)[None, :]).t().contiguous()
    n = pos.shape[0]
    v = torch.empty((n, system.n_orb), dtype=torch.float64, device="cuda")
    lap = torch.empty_like(v)
    for p0 in range(0, n, chunk):
        e = torch.exp(1j * (pos[p0:p0 + chunk] @ g.t()))
        v[p0:p0 + chunk] = (e @ cv).real
        lap[p0:p0 + chunk] = (e @ cl).real
    return v, lap


def fit_rows(steps, warmup, adam_steps=200, cg_iters=400):
    """Differentiation form on the fit workload (128 orbitals, 32^3 FP32 table, 10^6 points): the
    adjoint in both summation modes, the fit's terms, 200 Adam steps of the least-squares fit from the
    interpolating spline, and the fit's exact optimum (conjugate gradients on the same loss, FP64
    table) that the Adam steps approach."""
    import torch
    import paper_1309_6250_amd as P
    from paper_1309_6250_amd.fit import fit_adam, fit_optimum_cg
    from workloads import config
    w = config(4)
    s = w.system
    pos = torch.from_numpy(w.positions()).cuda()
    n = pos.shape[0]
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f32")
    table = P.spline_build(d, torch.from_numpy(s.grid_values()).cuda())
    g = torch.Generator(device="cuda").manual_seed(11)
    gv = torch.randn((n, s.n_orb), device="cuda", generator=g)
    gl = torch.randn((n, s.n_orb), device="cuda", generator=g)
    gt = P.new_gtable(d)
    out = {}
    for name, flags in (("atomic", 0), ("deterministic", P.SPL_DETERMINISTIC)):
        ms = time_launches(lambda: P.spline_eval_vgl_backward(d, table, pos, gv, None, gl, gt, None, want_pos=False,
                                                              flags=flags), max(3, steps // 4), 1)
        out[f"spline_eval_vgl_backward_fit_{name}"] = {
            "ms": ms, "evals_per_s": n * s.n_orb / (ms * 1e-3), "points": n, "n_orb": s.n_orb, "grid": list(s.grid)}
    # the forward on the fit's dense points: per-point kernel (sorted call) against the cell-wise one
    cw = torch.empty(max(1, P.spline_cells_work_bytes(d, n)), dtype=torch.uint8, device="cuda")
    sw = torch.empty(max(1, P.spline_sorted_work_bytes(d, n)), dtype=torch.uint8, device="cuda")
    outs = P.spline_eval_vgl(d, table, pos)
    ms_sorted = time_launches(lambda: P.spline_eval_vgl_sorted(d, table, pos, *outs, work=sw), max(3, steps // 4), 1)
    ms_vgl = time_launches(lambda: P.spline_eval_vgl_cells(d, table, pos, *outs, work=cw), max(3, steps // 4), 1)
    ms_vl = time_launches(lambda: P.spline_eval_vgl_cells(d, table, pos, outs[0], None, outs[2], outputs="vl",
                                                          work=cw), max(3, steps // 4), 1)
    out["spline_eval_vgl_cells_fit_f32"] = {
        "ms_vl": ms_vl, "ms_vgl": ms_vgl, "ms_sorted_per_point_vgl": ms_sorted,
        "evals_per_s_vl": n * s.n_orb / (ms_vl * 1e-3), "points": n, "n_orb": s.n_orb, "grid": list(s.grid),
        "note": "matrix-core products of each cell's block with its points' row weights (30 points per cell)"}
    del outs, sw
    v_t, lap_t = planewave_targets_gpu(s, pos)
    # the misfit kernel alone: one pass over outputs and targets (12 B per FP32 value)
    od = P.OUT_TORCH[d.dtype]
    y = torch.randn((n, s.n_orb), device="cuda", generator=g, dtype=od)
    t = v_t.to(od)
    gm = torch.empty_like(y)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    mw = torch.empty(P.spline_misfit_work_bytes(d, y.numel()), dtype=torch.uint8, device="cuda")
    ms = time_launches(lambda: P.spline_misfit(d, y, t, 1.0, loss, g=gm, work=mw), max(3, steps // 4), 1)
    out["spline_misfit_f32"] = {"ms": ms, "values": y.numel(),
                                "alg_GBps": 12 * y.numel() / (ms * 1e-3) / 1e9}
    del y, t, gm
    # the misfit of V and lap formed inside the cell-wise forward, against forward + two misfit passes;
    # both on the cell sort the fit keeps (SPL_REUSE_SORT), as in every fit step after the first
    tv, tl = v_t.to(od), lap_t.to(od)
    yv, yl = torch.empty_like(tv), torch.empty_like(tl)
    P.spline_eval_vgl_cells(d, table, pos, yv, None, yl, outputs="vl", work=cw)
    reuse = P.SPL_REUSE_SORT

    def two_pass():
        P.spline_eval_vgl_cells(d, table, pos, yv, None, yl, outputs="vl", work=cw, flags=reuse)
        P.spline_misfit(d, yv, tv, 1.0, loss, g=yv, work=mw)
        P.spline_misfit(d, yl, tl, 1.0, loss, g=yl, work=mw)
    ms_two = time_launches(two_pass, max(3, steps // 4), 1)
    ms_fused = time_launches(lambda: P.spline_fit_terms_cells(d, table, pos, tv, 1.0, tl, 1.0, g_v=yv, g_lap=yl,
                                                              loss=loss, work=cw, flags=reuse), max(3, steps // 4), 1)
    out["spline_fit_terms_cells_fit_f32"] = {
        "ms": ms_fused, "ms_forward_then_misfit": ms_two, "points": n, "n_orb": s.n_orb,
        "note": "V and lap misfit gradients and loss from the cell-wise forward, sort reused"}
    # the fit's loss terms and their coefficient gradient: fit terms then the deterministic adjoint
    # (one workspace, one sort), against the one pass (forward, misfit and adjoint in one kernel)
    ww = torch.empty(max(P.spline_cells_work_bytes(d, n), P.spline_backward_work_bytes(d, n, P.SPL_DETERMINISTIC)),
                     dtype=torch.uint8, device="cuda")
    fw = torch.empty(P.spline_fit_gradient_work_bytes(d, n), dtype=torch.uint8, device="cuda")
    gtab = P.new_gtable(d)
    P.spline_fit_terms_cells(d, table, pos, tv, 1.0, tl, 1.0, g_v=yv, g_lap=yl, loss=loss, work=ww)
    P.spline_fit_gradient_cells(d, table, pos, tv, 1.0, tl, 1.0, gtable=gtab, loss=loss, work=fw)

    def terms_then_adjoint():
        P.spline_fit_terms_cells(d, table, pos, tv, 1.0, tl, 1.0, g_v=yv, g_lap=yl, loss=loss, work=ww, flags=reuse)
        P.spline_eval_vgl_backward(d, table, pos, yv, None, yl, gtab, None, want_pos=False,
                                   flags=P.SPL_DETERMINISTIC | reuse, work=ww)
    ms_pair = time_launches(terms_then_adjoint, max(3, steps // 4), 1)
    ms_one = time_launches(lambda: P.spline_fit_gradient_cells(d, table, pos, tv, 1.0, tl, 1.0, gtable=gtab, loss=loss,
                                                               work=fw, flags=reuse), max(3, steps // 4), 1)
    out["spline_fit_gradient_cells_fit_f32"] = {
        "ms": ms_one, "ms_terms_then_adjoint": ms_pair, "points": n, "n_orb": s.n_orb,
        "note": "loss terms of V and lap and their coefficient gradient; one pass: forward, misfit and adjoint of "
                "each batch of points in one kernel (the same bits as the two kernels), sort reused"}
    del tv, tl, yv, yl, cw, ww, fw, gtab
    rms = float(torch.sqrt(torch.mean(table.double() ** 2)))
    lr = FIT_LR * rms
    fit_adam(d, table, pos, v_t, lap_t, steps=2, lam=1e-3, lr=lr)     # untimed: first-use allocations
    torch.cuda.synchronize()
    t0 = time.time()
    fitted, losses = fit_adam(d, table, pos, v_t, lap_t, steps=adam_steps, lam=1e-3, lr=lr, schedule=FIT_SCHEDULE)
    torch.cuda.synchronize()
    wall = time.time() - t0
    # the optimum of the same loss, by conjugate gradients from the same start (FP64 table)
    d64 = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f64")
    t64 = P.spline_build(d64, torch.from_numpy(s.grid_values()).cuda())
    t0 = time.time()
    opt64, loss_opt, cg_done, cg_res = fit_optimum_cg(d64, t64, pos, v_t, lap_t, lam=1e-3, iters=cg_iters, rtol=1e-8)
    torch.cuda.synchronize()
    cg_s = time.time() - t0
    # held-out points: error of the interpolating start and of the fitted table against the planewaves
    hold = torch.from_numpy(w.system.positions(n + 4096)[n:]).cuda()
    hv, hl = planewave_targets_gpu(s, hold)
    res = {}
    for tag, dd, tab in (("interpolating", d, table), ("adam", d, fitted.contiguous()), ("optimum", d64, opt64)):
        v, _, lap = P.spline_eval_vgl(dd, tab, hold)
        res[tag] = {"rmae_V": float((v.double() - hv).abs().mean() / hv.abs().mean()),
                    "rmae_lap": float((lap.double() - hl).abs().mean() / hl.abs().mean())}
    out["smoothing_fit_adam_f32"] = {"adam_steps": adam_steps, "ms_per_step": 1e3 * wall / adam_steps,
                                     "loss_step0": losses[0], "loss_last": losses[-1], "loss_optimum": loss_opt,
                                     "gap_closed": (losses[0] - losses[-1]) / (losses[0] - loss_opt),
                                     "lr": lr, "lr_over_rms_table": FIT_LR, "schedule": FIT_SCHEDULE,
                                     "optimum": {"method": "conjugate gradients on the same loss, FP64 table",
                                                 "iterations": cg_done, "relative_residual": cg_res, "s": cg_s},
                                     "lambda": 1e-3, "deterministic_gradient": True, "heldout": res,
                                     "note": "per step: spline_fit_gradient_cells (cell-wise forward, misfit of V "
                                             "and lap, and adjoint in one pass) and the smoothness penalty on the "
                                             "cell sort of the first step; the library's Adam update "
                                             "(spline_adam_step) of the 16.8 MB table and its moments; after 2 "
                                             "untimed steps"}
    return out


def memory_ceilings():
    """Achievable bandwidth of device memory, for context: a linear read-only stream of 4 GiB
    (spline_stream_read: the ceiling for a kernel that reads and hardly writes, like the gather) and a
    plain device-to-device copy of 2 GiB (reads and writes)."""
    import torch
    import paper_1309_6250_amd as P
    src = torch.ones(1 << 29, dtype=torch.float64, device="cuda")           # 4 GiB
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    ms_read = time_launches(lambda: P.spline_stream_read(src, sink), 10, 2)
    read_bytes = src.numel() * 8
    half = src[: 1 << 28]
    dst = torch.empty_like(half)
    ms_copy = time_launches(lambda: dst.copy_(half), 10, 2)
    del src, dst, half
    return {"stream_read": {"bytes": read_bytes, "ms": ms_read, "GBps": read_bytes / (ms_read * 1e-3) / 1e9},
            "copy": {"bytes_per_copy": 2 * (1 << 31), "ms": ms_copy, "GBps": 2 * (1 << 31) / (ms_copy * 1e-3) / 1e9}}


def smoothing_rows(wl2):
    """Fourier-matched build on the MgO-like cell and the paper's comparison of methods on the synthetic
    orbitals: RMAE against the planewave sum of value, gradient and Laplacian for the interpolating and
    the smoothing spline, each with the Laplacian from derivatives and from a separate spline (FP64)."""
    import numpy as np
    import torch
    import paper_1309_6250_amd as P
    s = wl2.s
    d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f64", has_lap=True)
    miller = torch.from_numpy(s.miller.astype(np.int32)).cuda()
    coef = torch.from_numpy(s.coef).cuda()
    work = torch.empty(P.spline_smoothing_work_bytes(d), dtype=torch.uint8, device="cuda")
    tab_s = P.new_table(d)
    ms = time_launches(lambda: P.spline_build_smoothing(d, miller, coef, tab_s, work), 1, 1)
    del work
    tab_i = P.spline_build(d, wl2.f, wl2.lf)
    idx = parity_sample(wl2.pos_host.shape[0])
    k = s.n_orb
    d_nolap = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f64")
    x = wl2.pos[torch.from_numpy(idx).cuda()].contiguous()
    cache = wl2.__dict__.setdefault("_accuracy_cache", {})
    if "pw" not in cache:
        cache["pw"] = planewave_vgl_gpu(s, x, k)
    vp, gp, lp = cache["pw"]
    out = {"spline_build_smoothing_f64_lap_ms": ms, "sample": f"{len(idx)} seeded points x all {k} orbitals"}
    rmae = lambda a, b: float(np.abs(a - b).mean() / np.abs(b).mean())
    for name, tab in (("interpolating", tab_i), ("smoothing", tab_s)):
        v, g, l = [t.cpu().numpy() for t in P.spline_eval_vgl(d_nolap, tab[:1].contiguous(), x)]
        _, _, ls = [t.cpu().numpy() for t in P.spline_eval_vgl(d, tab, x)]
        out[name] = {"rmae_V": rmae(v[:, :k], vp), "rmae_grad": rmae(g[:, :, :k], gp),
                     "rmae_lap_derivative": rmae(l[:, :k], lp), "rmae_lap_separate": rmae(ls[:, :k], lp)}
    del tab_s, tab_i
    return out


def method_comparison_row(wl2, fields, k=16, n_sample=1024):
    """The paper's comparison of representations (Fig. 1) on the synthetic MgO-like orbitals: RMAE
    against the planewave sum of the orbital and of direct approximations of its gradient and
    Laplacian (five separate tables each) for Lagrange interpolation, interpolating B-splines and
    smoothing B-splines (FP64 tables of the first k orbitals, n_sample seeded points)."""
    import numpy as np
    import torch
    import paper_1309_6250_amd as P
    s = wl2.s
    sub = fields[..., :k].contiguous()
    idx = parity_sample(wl2.pos_host.shape[0], n_sample)
    x = wl2.pos[torch.from_numpy(idx).cuda()].contiguous()
    ref = planewave_vgl_gpu(s, x, k)
    miller = torch.from_numpy(s.miller.astype(np.int32)).cuda()
    coef = torch.from_numpy(np.ascontiguousarray(s.coef[:k])).cuda()
    rmae = lambda a, b: float(np.abs(a - b).mean() / np.abs(b).mean())
    out = {"sample": f"{n_sample} points x first {k} orbitals, FP64 tables, five separate tables each"}
    for name in ("lagrange", "interpolating_bspline", "smoothing_bspline"):
        d = P.spline_desc_init(s.lattice, s.grid, k, "f64", has_lap=True, sep_grad=True,
                               basis="lagrange" if name == "lagrange" else "bspline")
        if name == "smoothing_bspline":
            tab = P.spline_build_smoothing(d, miller, coef)
        else:
            tab = P.spline_build_tables(d, sub)
        got = [_host(t) for t in P.spline_eval_vgl(d, tab, x)]
        out[name] = {q: rmae(g, r) for q, g, r in zip(("rmae_V", "rmae_grad", "rmae_lap"), got, ref)}
        del tab
    del sub
    return out


def batched_row(steps, warmup):
    """48 uneven systems (orbitals 32-256, grids 24^3-64^3, 16-512 walkers x 64-256 electrons),
    FP32 tables built on the GPU, all VGL evaluations in one persistent launch replayed from a
    HIP graph, tile chosen by the batch autotuner."""
    import torch
    import paper_1309_6250_amd as P
    from workloads import batched_systems
    t0 = time.time()
    items, table_bytes = [], 0
    for w in batched_systems():
        s = w.system
        f = torch.from_numpy(s.grid_values()).cuda()
        d = P.spline_desc_init(s.lattice, s.grid, s.n_orb, "f32")
        tab = P.spline_build(d, f)
        del f
        pos = torch.from_numpy(w.positions()).cuda()
        n = pos.shape[0]
        items.append((d, tab, pos, torch.empty((n, s.n_orb), device="cuda"),
                      torch.empty((n, 3, s.n_orb), device="cuda"), torch.empty((n, s.n_orb), device="cuda")))
        table_bytes += d.table_bytes
    torch.cuda.synchronize()
    log(f"batched workload: {len(items)} systems ready in {time.time() - t0:.1f} s")
    plan = P.BatchPlan(items)
    tile = plan.autotune()
    item_tiles = plan.tiles()
    n_tiles, n_evals = plan.info()
    ms = time_launches(plan.run_graph, steps, warmup)
    ms_eager = time_launches(plan.run, steps, warmup)
    alg = sum(it[2].shape[0] * it[0].n_orb * bytes_per_eval("f32") + 24 * it[2].shape[0] for it in items)
    # the same plan with every item's points in locality order (sort inside every launch), retuned
    plan.sort(True)
    tile_s = plan.autotune()
    ms_sorted = time_launches(plan.run_graph, steps, warmup)
    plan.close()
    lanes = sorted({t[0] for t in item_tiles})
    return {"systems": len(items), "evals_per_launch": n_evals, "tiles": n_tiles, "tile": list(tile),
            "per_item_lanes": lanes if tile[0] == 0 else None,
            "shapes": "one shape for all items" if tile[0] != 0 else
                      f"per-item lanes per point {lanes}, {tile[1]} orbitals per lane",
            "ms_graph": ms, "ms_eager": ms_eager, "evals_per_s": n_evals / (ms * 1e-3),
            "alg_GBps": alg / (ms * 1e-3) / 1e9,
            "effective_frac_hbm_peak": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "table_bytes": table_bytes, "largest_item_table_bytes": max(it[0].table_bytes for it in items),
            "note": "every item's table is smaller than the Infinity Cache, so the fraction is effective",
            "sorted": {"tile": list(tile_s), "ms_graph": ms_sorted, "evals_per_s": n_evals / (ms_sorted * 1e-3),
                       "speedup": ms / ms_sorted,
                       "note": "spline_batch_plan_sort: counting sort of every item's points inside each launch"}}


def _gpu_ready():
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    import paper_1309_6250_amd as P
    P.lib()
    return torch


def compact_line(line, limit=4000):
    """The final stdout record, kept under `limit` bytes: optional keys are dropped, last first."""
    text = json.dumps(line)
    for key in ("rows", "effective", "cpu_context", "precision_forms"):
        if len(text) <= limit:
            break
        line.pop(key, None)
        text = json.dumps(line)
    return text


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="headline only: no extra forms, rows or CPU baseline")
    ap.add_argument("--only", default=None,
                    help="time only one form, e.g. c2-f32, c2-bf16-lap, c2-f32-sep-lagrange, c2-f64-pp, "
                         "c7-f64-bloch or c8-f32, 'fit' for the differentiation rows or 'c1-adjoint' for the "
                         "adjoint at QMC density (for profiling runs)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tile", default=None, help="with --only: fixed tile 'G,OPL' instead of autotuning")
    ap.add_argument("--detail", default=os.path.join("gpurun_out", "bench_detail.json"),
                    help="where the full record (every form and row) is written")
    ap.add_argument("--fit-steps", type=int, default=200, help="Adam steps of the fit row")
    ap.add_argument("--cg-iters", type=int, default=400, help="conjugate-gradient iterations of the fit's optimum")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (scales memory counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the evaluation shards by points with no communication, "
              "so N GPUs would run N independent copies of this workload. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        torch = _gpu_ready()
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")      # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of 1 GiB (1073741824 bytes read + written each)")
        del src, dst

    if args.only == "fit":
        # differentiation form only (for profiling runs): adjoint in both modes, misfit, Adam fit
        _gpu_ready()
        print(json.dumps({"only": "fit", **fit_rows(args.steps, args.warmup, args.fit_steps, args.cg_iters)}),
              flush=True)
        return

    if args.only == "c1-adjoint":
        # the adjoint at QMC density only (for profiling runs): the Si-like cell's 65 536 points,
        # atomic and deterministic forms, together with the other rows of that cell
        wl1 = Workload(1)
        _gpu_ready()
        wl1.upload()
        print(json.dumps({"only": "c1-adjoint", **rows_measurements(wl1, args.steps, args.warmup)}), flush=True)
        return

    if args.only and args.only.endswith("-sorted"):
        # locality-ordered call only (for profiling runs: the sorted kernel's launches alone)
        import paper_1309_6250_amd as P
        key, dtype, *rest = args.only[:-len("-sorted")].split("-")
        lap = bool(rest and rest[0] == "lap")
        wl = Workload(int(key[1:]), lap=lap)
        _gpu_ready()
        wl.upload()
        s_ = wl.s
        d = P.spline_desc_init(s_.lattice, s_.grid, s_.n_orb, dtype, has_lap=lap)
        table = P.spline_build(d, wl.f, wl.lf if lap else None)
        outs = P.spline_eval_vgl(d, table, wl.pos)
        tile = None if args.tile is None else tuple(int(x) for x in args.tile.split(","))
        rec = sorted_form(wl, d, table, outs, dtype, args.steps, args.warmup, tile=tile)
        print(json.dumps({"only": args.only, **rec}), flush=True)
        return

    if args.only:
        key, dtype, *rest = args.only.split("-")
        lap = bool(rest and rest[0] == "lap")
        sep = rest[1] if rest and rest[0] == "sep" else None
        basis = "pp" if rest and rest[0] == "pp" else "bspline"
        wl = Workload(int(key[1:]), lap=lap)
        _gpu_ready()
        wl.upload()
        fields = grid_fields_gpu(wl.s) if sep else None
        tile = None if args.tile is None else tuple(int(x) for x in args.tile.split(","))
        rec, *_ = run_form(wl, dtype, lap or bool(sep), args.steps, args.warmup, tile=tile, sep=sep, fields=fields,
                           basis=basis)
        print(json.dumps({"only": args.only, **rec}), flush=True)
        return

    # ---------------------------------------------------------------- host leg (before the GPU is touched)
    wl2 = Workload(2, lap=True)
    cpu = cpu_more = parity = None
    if not args.quick and not args.no_cpu:
        cpu, parity = cpu_baseline(wl2)
        log(f"cpu baseline: {cpu['value']:.3e} evals/s on {cpu['cores']} processes ({cpu['wall_s']:.1f} s)")
        cpu_more = cpu_context(wl2)
        log(f"cpu context: planewave sum {cpu_more['planewave_sum_vgl']['evals_per_s']:.3e} evals/s")

    # ---------------------------------------------------------------- headline: MgO-like cell, FP64 table
    torch = _gpu_ready()
    import paper_1309_6250_amd as P
    wl2.upload()
    head, d2, t2, o2 = run_form(wl2, "f64", False, args.steps, args.warmup)
    log(f"headline c2-f64: {head['ms_per_sweep']:.3f} ms, {head['evals_per_s']:.3e} evals/s, "
        f"{head['alg_GBps']:.0f} GB/s algorithmic ({100 * head['frac_hbm_peak']:.1f}% of HBM peak)")
    n_pts = int(wl2.pos.shape[0])
    forms = {"c2-f64": head}
    rows = {}
    head["accuracy"] = accuracy(wl2, "f64", "derivative", o2)
    if parity is not None:
        head["vs_oracle"] = oracle_parity(o2, parity, "f64")
    per_launch = head["alg_bytes_per_sweep"]
    traffic = traffic_for("c2-f64", head["tile"])
    roofline = {"bound": "hbm", "achieved": head["alg_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": head["alg_GBps"] / HBM_PEAK_GBS, "traffic": traffic,
                "traffic_source": "not measured in this run: rocprofv3 FETCH_SIZE + WRITE_SIZE per launch from "
                                  "profiles/traffic.json at this tile, scaled by a 1 GiB copy; null when taken at "
                                  "another tile or the kernel sources changed since",
                "kernel": "k_eval (spline_eval_vgl, FP64 table, VGL)", "tile": head["tile"],
                "alg_bytes_per_launch": per_launch,
                "per_unit": "552 B per orbital-VGL (64 x 8 B coefficients + 5 x 8 B outputs) + 24 B per point",
                "kernel_hash": kernel_hash()}
    flops = FLOPS_PER_EVAL * n_pts * wl2.s.n_orb
    roofline["valu_frac_fp64"] = flops / (head["ms_per_sweep"] * 1e-3) / 1e12 / 78.6
    if not args.quick:
        forms["c2-f64-sorted"] = sorted_form(wl2, d2, t2, o2, "f64", args.steps, args.warmup)
        log(f"c2-f64-sorted: {forms['c2-f64-sorted']['evals_per_s']:.3e} evals/s (effective)")
    del t2, o2
    torch.cuda.empty_cache()

    # ---------------------------------------------------------------- precision forms on the same cell
    f64_rate = {False: head["evals_per_s"]}
    precision = {}
    for lap in (False, True):
        for dtype in ("f64", "f32", "bf16"):
            if dtype == "f64" and not lap:
                continue
            if args.quick and lap:
                continue
            rec, d, t, o = run_form(wl2, dtype, lap, args.steps, args.warmup)
            rec["accuracy"] = accuracy(wl2, dtype, "separate_lap" if lap else "derivative", o)
            name = f"c2-{dtype}" + ("-lap" if lap else "")
            if dtype == "f64":
                f64_rate[lap] = rec["evals_per_s"]
            rec["speedup_vs_f64"] = rec["evals_per_s"] / f64_rate[lap]
            if parity is not None and not lap:
                rec["vs_oracle"] = oracle_parity(o, parity, dtype)
            rec["traffic"] = traffic_for(name, rec["tile"])
            forms[name] = rec
            log(f"{name}: {rec['evals_per_s']:.3e} evals/s, {rec['alg_GBps']:.0f} GB/s "
                f"({100 * rec['frac_hbm_peak']:.1f}% of HBM peak)")
            if not args.quick and (not lap or dtype != "bf16"):
                forms[name + "-sorted"] = sorted_form(wl2, d, t, o, dtype, args.steps, args.warmup)
                log(f"{name}-sorted: {forms[name + '-sorted']['evals_per_s']:.3e} evals/s (effective)")
            del t, o
            torch.cuda.empty_cache()
            err = rec["accuracy"]
            key = "normwise_vs_fp64_table"
            precision[dtype + ("-lap" if lap else "")] = {
                "evals_per_s": rec["evals_per_s"], "speedup_vs_f64": rec["speedup_vs_f64"],
                "frac_hbm_peak": round(rec["frac_hbm_peak"], 4),
                "err_vs_fp64": None if dtype == "f64" else {q: float(f"{err[q][key]:.2e}") for q in ("V", "grad", "lap")}}

    if not args.quick:
        rows["memory_ceilings"] = memory_ceilings()
        log(f"read stream {rows['memory_ceilings']['stream_read']['GBps']:.0f} GB/s, "
            f"copy {rows['memory_ceilings']['copy']['GBps']:.0f} GB/s")
        rows["smoothing_vs_interpolating_mgo96"] = smoothing_rows(wl2)
        torch.cuda.empty_cache()
        # the representations the paper compares, with direct approximations of the gradient and the
        # Laplacian: five separate tables of B-spline coefficients or of Lagrange grid values
        fields = grid_fields_gpu(wl2.s)
        rows["method_comparison_mgo96"] = method_comparison_row(wl2, fields)
        log("method comparison: " + ", ".join(f"{k}: lap {v['rmae_lap']:.2e}" for k, v in
                                              rows["method_comparison_mgo96"].items() if isinstance(v, dict)))
        for basis in ("bspline", "lagrange"):
            for dtype in ("f64", "f32"):
                rec, d, t, o = run_form(wl2, dtype, True, args.steps, args.warmup, sep=basis, fields=fields)
                name = f"c2-{dtype}-sep-{basis}"
                rec["accuracy"] = accuracy(wl2, dtype, "separate_" + basis, o)
                rec["traffic"] = traffic_for(name, rec["tile"])
                forms[name] = rec
                log(f"{name}: {rec['evals_per_s']:.3e} evals/s, {rec['alg_GBps']:.0f} GB/s "
                    f"({100 * rec['frac_hbm_peak']:.1f}% of HBM peak)")
                if dtype == "f32":
                    forms[name + "-sorted"] = sorted_form(wl2, d, t, o, dtype, args.steps, args.warmup)
                del t, o
                torch.cuda.empty_cache()
        del fields
        torch.cuda.empty_cache()
        # the same interpolating spline in piecewise-polynomial form: 8 numbers per grid point, the
        # 2x2x2 corners of a point's cell (8 contiguous runs of 8 rows instead of 16 runs of 4)
        for dtype in ("f64", "f32"):
            rec, d, t, o = run_form(wl2, dtype, False, args.steps, args.warmup, basis="pp")
            name = f"c2-{dtype}-pp"
            rec["accuracy"] = accuracy(wl2, dtype, "pp", o)
            rec["traffic"] = traffic_for(name, rec["tile"])
            forms[name] = rec
            log(f"{name}: {rec['evals_per_s']:.3e} evals/s, {rec['alg_GBps']:.0f} GB/s "
                f"({100 * rec['frac_hbm_peak']:.1f}% of HBM peak)")
            if dtype == "f32":
                forms[name + "-sorted"] = sorted_form(wl2, d, t, o, dtype, args.steps, args.warmup)
            del t, o
            torch.cuda.empty_cache()
        wl2.f = wl2.lf = None
        torch.cuda.empty_cache()

        # ------------------------------------------------------------ cells whose tables fit the cache
        for key, bloch in ((1, False), (8, False), (7, True)):
            wl = Workload(key).upload()
            for dtype in ("f64", "f32", "bf16"):
                if bloch and dtype == "bf16":
                    continue
                rec, d, t, o = run_form(wl, dtype, False, args.steps, args.warmup)
                name = f"c{key}-{dtype}" + ("-bloch" if bloch else "")
                rec["accuracy"] = accuracy(wl, dtype, "bloch" if bloch else "derivative", o)
                rec["traffic"] = traffic_for(name, rec["tile"])
                if dtype == "f64":
                    base = rec["evals_per_s"]
                rec["speedup_vs_f64"] = rec["evals_per_s"] / base
                forms[name] = rec
                log(f"{name} ({wl.s.name}): {rec['evals_per_s']:.3e} evals/s, {rec['alg_GBps']:.0f} GB/s (effective)")
                forms[name + "-sorted"] = sorted_form(wl, d, t, o, dtype, args.steps, args.warmup)
                del t, o
                torch.cuda.empty_cache()
            if key == 1:
                rows.update(rows_measurements(wl, args.steps, args.warmup))
            del wl
            torch.cuda.empty_cache()

        rows["batched_persistent_graph_f32"] = batched_row(args.steps, args.warmup)
        log(f"batched: {rows['batched_persistent_graph_f32']['evals_per_s']:.3e} evals/s, sorted "
            f"{rows['batched_persistent_graph_f32']['sorted']['evals_per_s']:.3e}")
        torch.cuda.empty_cache()
        rows.update(fit_rows(args.steps, args.warmup))
        fr = rows["smoothing_fit_adam_f32"]
        log(f"fit: {fr['ms_per_step']:.2f} ms per Adam step, loss {fr['loss_step0']:.5e} -> {fr['loss_last']:.5e} "
            f"(optimum {fr['loss_optimum']:.5e}, {100 * fr['gap_closed']:.0f}% of the gap)")
        torch.cuda.empty_cache()

    ms = head["ms_per_sweep"]
    detail = {"headline": "c2-f64", "config": wl2.describe("f64", False), "roofline": roofline,
              "cpu_baseline": cpu, "cpu_context": cpu_more, "forms": forms, "rows": rows}
    try:
        os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
        with open(args.detail, "w") as fh:
            json.dump(detail, fh, indent=1)
    except OSError as exc:
        log(f"could not write {args.detail}: {exc}")
    cfg = wl2.describe("f64", False)
    cfg.pop("lattice_bohr", None)
    cfg.update({"table_bytes": int(head["table_bytes"]), "tile": head["tile"]})
    line = {
        "metric": METRIC,
        "value": head["evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded planewave orbitals of an MgO-like cell, uniform random electron positions)",
        "config": cfg,
        "hbm_frac": roofline["frac"],
        "roofline": {k: roofline[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic",
                                                "traffic_source", "kernel", "per_unit")},
        "accuracy_fp64": {"vs_oracle": head.get("vs_oracle"),
                          "vs_planewave": {q: float(f"{head['accuracy'][q]['normwise_vs_planewave']:.2e}")
                                           for q in ("V", "grad", "lap")},
                          "sample": head["accuracy"]["sample"]},
        "precision_forms": precision,
        "cpu_baseline": None if cpu is None else {k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample")},
        "detail": args.detail,
    }
    if cpu is not None:
        line["gpu_over_cpu"] = head["evals_per_s"] / cpu["value"]
    if rows:
        line["rows"] = {"stream_read_GBps": rows["memory_ceilings"]["stream_read"]["GBps"],
                        "fit_loss_step0_last_optimum": [fr["loss_step0"], fr["loss_last"], fr["loss_optimum"]],
                        "fit_ms_per_adam_step": fr["ms_per_step"],
                        "batched_evals_per_s": rows["batched_persistent_graph_f32"]["evals_per_s"]}
        line["effective"] = {k: forms[k]["evals_per_s"] for k in ("c1-f64", "c8-f64", "c1-f64-sorted", "c2-f64-sorted")
                             if k in forms}
    print(compact_line(line), flush=True)


if __name__ == "__main__":
    main()
