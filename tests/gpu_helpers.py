"""Shared helpers of the GPU parity tests (compare the HIP library with the FP64 oracle)."""
import sys

import numpy as np
import torch

import paper_1309_6250_amd as P
from oracle import build as obuild, evaluate as oeval, quantize as oq

DEV = "cuda:0"
U_ACC = {"f64": 2.0**-53, "f32": 2.0**-24, "bf16": 2.0**-24}     # accumulation precision per table dtype


def say(*args):
    """Name the case before each GPU step (flushed), so a failed run shows where it was."""
    print("[gpu]", *args, file=sys.stderr, flush=True)


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def table_from_oracle(desc, beta, dtype, lap_beta=None):
    """Upload oracle coefficients as a device table of the storage dtype (padding zeroed)."""
    n1, n2, n3, n_orb = beta.shape
    arr = np.zeros((1 + desc.has_lap, n1, n2, n3, desc.o_pad))
    arr[0, ..., :n_orb] = beta
    if lap_beta is not None:
        arr[1, ..., :n_orb] = lap_beta
    if dtype == "f64":
        return to_dev(arr)
    if dtype == "f32":
        return to_dev(oq.to_f32(arr), torch.float32)
    bits = oq.to_bf16_bits(arr)
    return torch.from_numpy(bits.view(np.int16)).to(DEV).view(torch.bfloat16)


def oracle_table_values(beta, dtype):
    """The FP64 values the kernel sees after storage in ``dtype``."""
    return oq.quantized(beta, dtype)


def gpu_build(desc, f, lap_f=None):
    say("spline_build", tuple(desc.grid), desc.n_orb, desc.dtype, desc.has_lap)
    gv = to_dev(f)
    lv = None if lap_f is None else to_dev(lap_f)
    table = P.spline_build(desc, gv, lv)
    torch.cuda.synchronize()
    return table


def gpu_vgl(desc, table, pos, tile=None):
    say("spline_eval_vgl", tuple(desc.grid), desc.n_orb, desc.dtype, desc.has_lap, len(pos), tile)
    out = P.spline_eval_vgl(desc, table, to_dev(pos), tile=tile)
    torch.cuda.synchronize()
    return [x.double().cpu().numpy() for x in out]


def normwise(a, b):
    return float(np.nanmax(np.abs(a - b)) / np.nanmax(np.abs(b)))


def assert_elementwise(got, ref, bound, factor, name):
    """|got - ref| <= factor * bound elementwise (bound = sum |w||beta| from the oracle)."""
    err = np.abs(got - ref)
    lim = factor * bound + 1e-300
    bad = err > lim
    if bad.any():
        i = np.argmax(err / lim)
        raise AssertionError(f"{name}: {bad.sum()} elements over the bound; worst err {err.flat[i]:.3e} "
                             f"vs bound {lim.flat[i]:.3e}")


def coordinate_rounding(desc, lattice, pos, dtype):
    """Per point and axis, a bound on |delta u| from rounding in the coordinate reduction on
    either side (s = a^-1 r in FP64: a few roundings relative to sum_j |ainv_ij r_j|, then
    u = N s), plus the FP32 rounding of t when the table arithmetic is FP32."""
    ainv = np.abs(np.array(desc.ainv).reshape(3, 3))
    mag = np.abs(np.nan_to_num(pos)) @ ainv.T + 1.0
    du = 8 * 2.0**-53 * np.array(desc.grid)[None, :] * mag
    if dtype != "f64":
        du = du + 2.0**-24
    return du


def host_table(desc, table):
    """Device table -> FP64 numpy [(1+has_lap), N1, N2, N3, n_orb] (padding dropped)."""
    t = table.float() if table.dtype == torch.bfloat16 else table
    return t.double().cpu().numpy()[..., :desc.n_orb]
