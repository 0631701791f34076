"""Python binding of the pwspline C ABI: the same entry points, taking torch tensors.

Only argument marshalling happens here (device pointers, sizes, the current HIP
stream); every step of the computation runs in the library's HIP kernels.  All
tensors must live on the GPU and be contiguous.
"""
import ctypes

import torch

from ._lib import (SplDesc, SplItem, check, lib, SPL_F64, SPL_F32, SPL_BF16, SPL_BSPLINE, SPL_LAGRANGE,
                   SPL_PPSPLINE)

DTYPES = {"f64": SPL_F64, "f32": SPL_F32, "bf16": SPL_BF16}
BASES = {"bspline": SPL_BSPLINE, "lagrange": SPL_LAGRANGE, "pp": SPL_PPSPLINE}
STORE_TORCH = {SPL_F64: torch.float64, SPL_F32: torch.float32, SPL_BF16: torch.bfloat16}
OUT_TORCH = {SPL_F64: torch.float64, SPL_F32: torch.float32, SPL_BF16: torch.float32}


def _dtype_code(dtype):
    if isinstance(dtype, str):
        return DTYPES[dtype]
    return int(dtype)


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need(t, name, dtype, numel=None, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


def spline_desc_init(lattice, grid, n_orb, dtype="f64", has_lap=False, basis="bspline", sep_grad=False, kvec=None):
    """Validated descriptor (ctypes struct) of one coefficient table set.

    basis: "bspline", "lagrange" (needs sep_grad and has_lap) or "pp" (the interpolating spline in
    piecewise-polynomial form, 8 numbers per grid point); sep_grad: five
    tables (orbital, gradient x/y/z, Laplacian) read by value; kvec: crystal momentum (1/bohr)
    of Bloch orbitals exp(i k.r) u(r), whose n_orb complex orbitals take two columns each.
    """
    d = SplDesc()
    lat = [float(x) for x in torch.as_tensor(lattice, dtype=torch.float64).reshape(-1).tolist()]
    if len(lat) != 9:
        raise ValueError("lattice must be 3x3")
    for i in range(9):
        d.lattice[i] = lat[i]
    g = [int(x) for x in grid]
    if len(g) != 3:
        raise ValueError("grid must have 3 entries")
    for i in range(3):
        d.grid[i] = g[i]
    d.n_orb = int(n_orb)
    d.dtype = _dtype_code(dtype)
    d.has_lap = 1 if has_lap else 0
    d.basis = BASES[basis] if isinstance(basis, str) else int(basis)
    d.sep_grad = 1 if sep_grad else 0
    if kvec is not None:
        k = [float(x) for x in torch.as_tensor(kvec, dtype=torch.float64).reshape(-1).tolist()]
        if len(k) != 3:
            raise ValueError("kvec must have 3 entries")
        d.bloch = 1
        for i in range(3):
            d.kvec[i] = k[i]
    check(lib().spline_desc_init(ctypes.byref(d)), "spline_desc_init")
    return d


def table_shape(desc):
    if desc.basis == SPL_PPSPLINE:
        return (desc.n_tables, desc.grid[0], desc.grid[1], desc.grid[2], 8, desc.o_pad)
    return (desc.n_tables, desc.grid[0], desc.grid[1], desc.grid[2], desc.o_pad)


def _real_columns(desc, t, name):
    """Bloch inputs may be given as complex tensors [..., n_orb]; the ABI takes (re, im) columns."""
    if t is not None and t.is_complex():
        if not desc.bloch:
            raise TypeError(f"{name} is complex but the descriptor has no Bloch orbitals")
        return torch.view_as_real(t.contiguous()).reshape(*t.shape[:-1], 2 * t.shape[-1])
    return t


def new_table(desc, device="cuda"):
    return torch.empty(table_shape(desc), dtype=STORE_TORCH[desc.dtype], device=device)


def new_gtable(desc, device="cuda"):
    return torch.zeros(table_shape(desc), dtype=OUT_TORCH[desc.dtype], device=device)


def spline_build(desc, grid_vals, lap_vals=None, table=None, work=None, stream=None):
    """Interpolating coefficients from FP64 grid values [N1][N2][N3][n_orb] (device; complex128
    or (re, im) columns for Bloch orbitals)."""
    pts = desc.grid[0] * desc.grid[1] * desc.grid[2]
    grid_vals = _real_columns(desc, grid_vals, "grid_vals")
    lap_vals = _real_columns(desc, lap_vals, "lap_vals")
    _need(grid_vals, "grid_vals", torch.float64, pts * desc.n_col)
    if lap_vals is not None:
        _need(lap_vals, "lap_vals", torch.float64, pts * desc.n_col)
    if table is None:
        table = new_table(desc, grid_vals.device)
    _need(table, "table", STORE_TORCH[desc.dtype], desc.table_elems * desc.n_tables)
    if work is None:
        work = torch.empty(pts * desc.n_col, dtype=torch.float64, device=grid_vals.device)
    _need(work, "work", torch.float64, pts * desc.n_col)
    check(lib().spline_build(ctypes.byref(desc), _ptr(grid_vals), _ptr(lap_vals), _ptr(table), _ptr(work),
                             _stream(stream)), "spline_build")
    return table


def spline_build_tables(desc, vals, table=None, work=None, stream=None):
    """All tables of a descriptor from stacked FP64 grid values [n_tables][N1][N2][N3][n_orb]
    (orbital, gradient x/y/z with sep_grad, Laplacian with has_lap; device; complex128 or
    (re, im) columns for Bloch orbitals).  A list of per-table tensors is stacked first."""
    if isinstance(vals, (list, tuple)):
        vals = torch.stack(list(vals))
    vals = _real_columns(desc, vals, "vals")
    pts = desc.grid[0] * desc.grid[1] * desc.grid[2]
    _need(vals, "vals", torch.float64, desc.n_tables * pts * desc.n_col)
    if table is None:
        table = new_table(desc, vals.device)
    _need(table, "table", STORE_TORCH[desc.dtype], desc.table_elems * desc.n_tables)
    if work is None and desc.basis == SPL_BSPLINE:
        work = torch.empty(pts * desc.n_col, dtype=torch.float64, device=vals.device)
    if work is not None:
        _need(work, "work", torch.float64, pts * desc.n_col)
    check(lib().spline_build_tables(ctypes.byref(desc), _ptr(vals), _ptr(table), _ptr(work), _stream(stream)),
          "spline_build_tables")
    return table


def spline_smoothing_work_bytes(desc):
    out = ctypes.c_int64()
    check(lib().spline_smoothing_work_bytes(ctypes.byref(desc), ctypes.byref(out)), "spline_smoothing_work_bytes")
    return out.value


def spline_build_smoothing(desc, miller, coef, table=None, work=None, stream=None):
    """Fourier-matched coefficients from planewave coefficients.

    miller: int32 [n_g, 3] (device); coef: complex128 [n_orb, n_g] (device).
    """
    _need(miller, "miller", torch.int32)
    _need(coef, "coef", torch.complex128)
    n_g = miller.shape[0]
    if miller.shape != (n_g, 3) or coef.shape != (desc.n_orb, n_g):
        raise ValueError("miller must be [n_g, 3] and coef [n_orb, n_g]")
    if table is None:
        table = new_table(desc, coef.device)
    _need(table, "table", STORE_TORCH[desc.dtype], desc.table_elems * desc.n_tables)
    nbytes = spline_smoothing_work_bytes(desc)
    if work is None:
        work = torch.empty(nbytes, dtype=torch.uint8, device=coef.device)
    if work.numel() * work.element_size() < nbytes:
        raise ValueError(f"work must hold {nbytes} bytes")
    check(lib().spline_build_smoothing(ctypes.byref(desc), int(n_g), _ptr(miller), _ptr(coef), _ptr(table),
                                       _ptr(work), _stream(stream)), "spline_build_smoothing")
    return table


def _outputs(desc, n_pts, device, v, grad, lap, values_only=False):
    """Real output buffers [.][n_col] (Bloch outputs given as complex tensors are viewed as
    (re, im) columns)."""
    od = OUT_TORCH[desc.dtype]
    v, grad, lap = (_real_columns(desc, t, n) for t, n in ((v, "v"), (grad, "grad"), (lap, "lap")))
    if v is None:
        v = torch.empty((n_pts, desc.n_col), dtype=od, device=device)
    _need(v, "v", od, n_pts * desc.n_col)
    if values_only:
        return v, None, None
    if grad is None:
        grad = torch.empty((n_pts, 3, desc.n_col), dtype=od, device=device)
    if lap is None:
        lap = torch.empty((n_pts, desc.n_col), dtype=od, device=device)
    _need(grad, "grad", od, 3 * n_pts * desc.n_col)
    _need(lap, "lap", od, n_pts * desc.n_col)
    return v, grad, lap


def _as_complex(desc, t):
    """Bloch outputs as complex tensors [..., n_orb] viewing the (re, im) columns."""
    if t is None or not desc.bloch:
        return t
    return torch.view_as_complex(t.view(*t.shape[:-1], desc.n_orb, 2))


def _check_inputs(desc, table, pos):
    _need(table, "table", STORE_TORCH[desc.dtype], desc.table_elems * desc.n_tables)
    _need(pos, "pos", torch.float64)
    if pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("pos must be [n_pts, 3]")
    return pos.shape[0]


def spline_eval_v(desc, table, pos, v=None, stream=None):
    n = _check_inputs(desc, table, pos)
    v, _, _ = _outputs(desc, n, pos.device, v, None, None, values_only=True)
    check(lib().spline_eval_v(ctypes.byref(desc), _ptr(table), n, _ptr(pos), _ptr(v), _stream(stream)),
          "spline_eval_v")
    return _as_complex(desc, v)


def spline_eval_vgl(desc, table, pos, v=None, grad=None, lap=None, stream=None, tile=None):
    n = _check_inputs(desc, table, pos)
    v, grad, lap = _outputs(desc, n, pos.device, v, grad, lap)
    if tile is None:
        check(lib().spline_eval_vgl(ctypes.byref(desc), _ptr(table), n, _ptr(pos), _ptr(v), _ptr(grad), _ptr(lap),
                                    _stream(stream)), "spline_eval_vgl")
    else:
        t = (ctypes.c_int32 * 2)(int(tile[0]), int(tile[1]))
        check(lib().spline_eval_vgl_tile(ctypes.byref(desc), _ptr(table), n, _ptr(pos), _ptr(v), _ptr(grad),
                                         _ptr(lap), t, _stream(stream)), "spline_eval_vgl_tile")
    return _as_complex(desc, v), _as_complex(desc, grad), _as_complex(desc, lap)


def spline_sorted_work_bytes(desc, n_pts):
    out = ctypes.c_int64()
    check(lib().spline_sorted_work_bytes(ctypes.byref(desc), int(n_pts), ctypes.byref(out)), "spline_sorted_work_bytes")
    return out.value


def spline_eval_vgl_sorted(desc, table, pos, v=None, grad=None, lap=None, work=None, tile=None, stream=None):
    """spline_eval_vgl with the points evaluated in Morton order of their cells (same outputs, in
    the caller's order).  `work` (uint8 device tensor of spline_sorted_work_bytes bytes) is
    allocated if not given; pass one to keep allocation out of repeated calls."""
    n = _check_inputs(desc, table, pos)
    v, grad, lap = _outputs(desc, n, pos.device, v, grad, lap)
    nbytes = spline_sorted_work_bytes(desc, n)
    if work is None:
        work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=pos.device)
    if work.numel() * work.element_size() < nbytes:
        raise ValueError(f"work must hold {nbytes} bytes")
    t = None if tile is None else (ctypes.c_int32 * 2)(int(tile[0]), int(tile[1]))
    check(lib().spline_eval_vgl_sorted(ctypes.byref(desc), _ptr(table), n, _ptr(pos), _ptr(v), _ptr(grad), _ptr(lap),
                                       t, _ptr(work), int(work.numel() * work.element_size()), _stream(stream)),
          "spline_eval_vgl_sorted")
    return _as_complex(desc, v), _as_complex(desc, grad), _as_complex(desc, lap)


def spline_eval_vgl_sorted_noalloc(desc, table, pos, v, grad, lap, tile=None, stream=None):
    """spline_eval_vgl_sorted with the library's static device scratch as workspace: allocates
    nothing, so the outputs v, grad, lap must be given.  Calls that overlap on one device race."""
    n = _check_inputs(desc, table, pos)
    if v is None or grad is None or lap is None:
        raise ValueError("spline_eval_vgl_sorted_noalloc allocates nothing: pass v, grad and lap")
    v, grad, lap = _outputs(desc, n, pos.device, v, grad, lap)
    t = None if tile is None else (ctypes.c_int32 * 2)(int(tile[0]), int(tile[1]))
    check(lib().spline_eval_vgl_sorted_noalloc(ctypes.byref(desc), _ptr(table), n, _ptr(pos), _ptr(v), _ptr(grad),
                                               _ptr(lap), t, _stream(stream)), "spline_eval_vgl_sorted_noalloc")
    return _as_complex(desc, v), _as_complex(desc, grad), _as_complex(desc, lap)


def spline_cells_work_bytes(desc, n_pts):
    out = ctypes.c_int64()
    check(lib().spline_cells_work_bytes(ctypes.byref(desc), int(n_pts), ctypes.byref(out)), "spline_cells_work_bytes")
    return out.value


def spline_eval_vgl_cells(desc, table, pos, v=None, grad=None, lap=None, outputs="vgl", work=None, flags=0,
                          stream=None):
    """spline_eval_vgl computed cell by cell on the matrix cores (for several points per cell).
    `outputs` names the ones wanted ('v', 'g', 'l' in any combination); returns (v, grad, lap) with
    None for the others.  Equal to spline_eval_vgl up to the order of summation.  flags:
    SPL_REUSE_SORT when `work` already holds the cell sort of these same points."""
    n = _check_inputs(desc, table, pos)
    od = OUT_TORCH[desc.dtype]
    dev = pos.device
    o = desc.n_orb
    if "v" in outputs and v is None:
        v = torch.empty((n, o), dtype=od, device=dev)
    if "g" in outputs and grad is None:
        grad = torch.empty((n, 3, o), dtype=od, device=dev)
    if "l" in outputs and lap is None:
        lap = torch.empty((n, o), dtype=od, device=dev)
    for name, t, k in (("v", v, 1), ("grad", grad, 3), ("lap", lap, 1)):
        if t is not None:
            _need(t, name, od, k * n * o)
    nbytes = spline_cells_work_bytes(desc, n)
    if work is None:
        work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    if work.numel() * work.element_size() < nbytes:
        raise ValueError(f"work must hold {nbytes} bytes")
    check(lib().spline_eval_vgl_cells(ctypes.byref(desc), _ptr(table), n, _ptr(pos), _ptr(v), _ptr(grad), _ptr(lap),
                                      int(flags), _ptr(work), int(work.numel() * work.element_size()), _stream(stream)),
          "spline_eval_vgl_cells")
    return v, grad, lap


def spline_fit_terms_cells(desc, table, pos, t_v=None, w_v=1.0, t_lap=None, w_lap=1.0, g_v=None, g_lap=None,
                           loss=None, work=None, flags=0, stream=None):
    """The misfit of values and Laplacians against targets t_v, t_lap ([n_pts, n_orb], output type)
    straight from the cell-wise evaluation: returns (g_v, g_lap, loss) with g = 2 w (y - t) (None for
    a term without a target) and loss (a one-element FP64 device tensor, zero if not given)
    accumulated into.  flags: SPL_REUSE_SORT when `work` already holds the cell sort of these same
    points."""
    n = _check_inputs(desc, table, pos)
    od = OUT_TORCH[desc.dtype]
    dev = pos.device
    o = desc.n_orb
    if t_v is not None and g_v is None:
        g_v = torch.empty((n, o), dtype=od, device=dev)
    if t_lap is not None and g_lap is None:
        g_lap = torch.empty((n, o), dtype=od, device=dev)
    for name, t in (("t_v", t_v), ("g_v", g_v), ("t_lap", t_lap), ("g_lap", g_lap)):
        if t is not None:
            _need(t, name, od, n * o)
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
    _need(loss, "loss", torch.float64, 1)
    nbytes = spline_cells_work_bytes(desc, n)
    if work is None:
        work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    if work.numel() * work.element_size() < nbytes:
        raise ValueError(f"work must hold {nbytes} bytes")
    check(lib().spline_fit_terms_cells(ctypes.byref(desc), _ptr(table), n, _ptr(pos), _ptr(t_v), float(w_v),
                                       _ptr(g_v), _ptr(t_lap), float(w_lap), _ptr(g_lap), _ptr(loss), int(flags),
                                       _ptr(work), int(work.numel() * work.element_size()), _stream(stream)),
          "spline_fit_terms_cells")
    return g_v, g_lap, loss


def spline_fit_gradient_work_bytes(desc, n_pts):
    out = ctypes.c_int64()
    check(lib().spline_fit_gradient_work_bytes(ctypes.byref(desc), int(n_pts), ctypes.byref(out)),
          "spline_fit_gradient_work_bytes")
    return out.value


def spline_fit_gradient_cells(desc, table, pos, t_v, w_v, t_lap, w_lap, gtable=None, loss=None, work=None, flags=0,
                              stream=None):
    """The fit's value and Laplacian misfit and its coefficient gradient in one pass: returns
    (gtable, loss), both accumulated into (fresh zeros if not given); the same bits as
    spline_fit_terms_cells followed by the deterministic spline_eval_vgl_backward (for orthogonal
    lattice vectors the same numbers, an exact zero possibly of the other sign).  FP32 tables,
    dense points (SPL_EUNSUPPORTED otherwise).  flags: SPL_REUSE_SORT when `work` already holds this
    function's cell sort of these same points."""
    n = _check_inputs(desc, table, pos)
    od = OUT_TORCH[desc.dtype]
    dev = pos.device
    for name, t in (("t_v", t_v), ("t_lap", t_lap)):
        _need(t, name, od, n * desc.n_orb)
    if gtable is None:
        gtable = new_gtable(desc)
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
    _need(loss, "loss", torch.float64, 1)
    nbytes = spline_fit_gradient_work_bytes(desc, n)
    if work is None:
        work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    if work.numel() * work.element_size() < nbytes:
        raise ValueError(f"work must hold {nbytes} bytes")
    check(lib().spline_fit_gradient_cells(ctypes.byref(desc), _ptr(table), n, _ptr(pos), _ptr(t_v), float(w_v),
                                          _ptr(t_lap), float(w_lap), _ptr(gtable), _ptr(loss), int(flags), _ptr(work),
                                          int(work.numel() * work.element_size()), _stream(stream)),
          "spline_fit_gradient_cells")
    return gtable, loss


def spline_adam_step(param, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """One Adam step on a table (or any array of its storage type): param, m and v are updated in
    place.  param FP64, FP32 or BF16; grad, m, v FP64 for an FP64 param, else FP32."""
    codes = {torch.float64: SPL_F64, torch.float32: SPL_F32, torch.bfloat16: SPL_BF16}
    if not isinstance(param, torch.Tensor) or param.dtype not in codes:
        raise TypeError("param must be an FP64, FP32 or BF16 torch tensor")
    dtype = codes[param.dtype]
    _need(param, "param", param.dtype, None)
    for name, t in (("grad", grad), ("m", m), ("v", v)):
        _need(t, name, OUT_TORCH[dtype], param.numel())
    check(lib().spline_adam_step(int(dtype), param.numel(), _ptr(param), _ptr(grad), _ptr(m), _ptr(v), float(lr),
                                 float(beta1), float(beta2), float(eps), int(step), _stream(stream)),
          "spline_adam_step")
    return param


def spline_eval_vgl_backward(desc, table, pos, gv=None, ggrad=None, glap=None, gtable=None, gpos=None,
                             want_table=True, want_pos=True, flags=0, stream=None, work=None):
    """Returns (gtable, gpos).  gtable is accumulated into (a fresh zero table if not given).
    work: uint8 device tensor of spline_backward_work_bytes bytes (allocated if not given)."""
    n = _check_inputs(desc, table, pos)
    od = OUT_TORCH[desc.dtype]
    for name, g, numel in (("gv", gv, n * desc.n_orb), ("ggrad", ggrad, 3 * n * desc.n_orb),
                           ("glap", glap, n * desc.n_orb)):
        if g is not None:
            _need(g, name, od, numel)
    if want_table and gtable is None:
        gtable = new_gtable(desc, pos.device)
    if gtable is not None:
        _need(gtable, "gtable", od, desc.table_elems * desc.n_tables)
    if want_pos and gpos is None:
        gpos = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    if gpos is not None:
        _need(gpos, "gpos", torch.float64, 3 * n)
    nbytes = spline_backward_work_bytes(desc, n, flags)
    if not nbytes:
        work = None
    elif work is None:
        work = torch.empty(nbytes, dtype=torch.uint8, device=pos.device)     # caller-owned workspace
    elif work.numel() * work.element_size() < nbytes:
        raise ValueError(f"work must hold {nbytes} bytes")
    check(lib().spline_eval_vgl_backward(ctypes.byref(desc), _ptr(table), n, _ptr(pos), _ptr(gv), _ptr(ggrad),
                                         _ptr(glap), _ptr(gtable), _ptr(gpos), int(flags), _ptr(work),
                                         0 if work is None else int(work.numel() * work.element_size()),
                                         _stream(stream)),
          "spline_eval_vgl_backward")
    return gtable, gpos


def spline_backward_work_bytes(desc, n_pts, flags=0):
    out = ctypes.c_int64()
    check(lib().spline_backward_work_bytes(ctypes.byref(desc), int(n_pts), int(flags), ctypes.byref(out)),
          "spline_backward_work_bytes")
    return out.value


def spline_misfit_work_bytes(desc, n):
    out = ctypes.c_int64()
    check(lib().spline_misfit_work_bytes(ctypes.byref(desc), int(n), ctypes.byref(out)), "spline_misfit_work_bytes")
    return out.value


def spline_misfit(desc, y, t, w, loss, g=None, work=None, stream=None):
    """loss (FP64 device scalar) += w sum (y - t)^2; returns g = 2 w (y - t) (written into `g`,
    which may be `y` itself, or a new tensor).  y, t: the descriptor's output dtype, same size."""
    od = OUT_TORCH[desc.dtype]
    n = y.numel()
    _need(y, "y", od, n)
    _need(t, "t", od, n)
    _need(loss, "loss", torch.float64, 1)
    if g is None:
        g = torch.empty_like(y)
    _need(g, "g", od, n)
    if work is None:
        work = torch.empty(spline_misfit_work_bytes(desc, n), dtype=torch.uint8, device=y.device)
    check(lib().spline_misfit(ctypes.byref(desc), n, _ptr(y), _ptr(t), float(w), _ptr(g), _ptr(loss), _ptr(work),
                              int(work.numel() * work.element_size()), _stream(stream)), "spline_misfit")
    return g


def spline_smoothness_penalty(desc, table, w, loss, gtable=None, work=None, stream=None):
    """loss (FP64 device scalar) += w sum (D beta)^2 over axes, grid points and real orbitals of the
    orbital table; gtable (allocated as zeros if not given) += its gradient.  Returns gtable."""
    if gtable is None:
        gtable = new_gtable(desc, table.device)
    _need(table, "table", None)
    _need(gtable, "gtable", OUT_TORCH[desc.dtype], desc.table_elems * desc.n_tables)
    _need(loss, "loss", torch.float64, 1)
    if work is None:
        work = torch.empty(spline_misfit_work_bytes(desc, 0), dtype=torch.uint8, device=table.device)
    check(lib().spline_smoothness_penalty(ctypes.byref(desc), _ptr(table), float(w), _ptr(gtable), _ptr(loss),
                                          _ptr(work), int(work.numel() * work.element_size()), _stream(stream)),
          "spline_smoothness_penalty")
    return gtable


def spline_stream_read(buf, sink, stream=None):
    """Read-rate probe: reads every byte of the contiguous device tensor `buf` (its size a multiple of
    16 bytes) once; `sink` is a device tensor of at least 4 bytes that is (practically) never written."""
    _need(buf, "buf", None)
    _need(sink, "sink", None)
    if sink.numel() * sink.element_size() < 4:
        raise ValueError("sink must hold at least 4 bytes")
    check(lib().spline_stream_read(_ptr(buf), int(buf.numel() * buf.element_size()), _ptr(sink), _stream(stream)),
          "spline_stream_read")


def spline_autotune(desc, table, pos, v=None, grad=None, lap=None, stream=None):
    n = _check_inputs(desc, table, pos)
    v, grad, lap = _outputs(desc, n, pos.device, v, grad, lap)
    t = (ctypes.c_int32 * 2)()
    check(lib().spline_autotune(ctypes.byref(desc), _ptr(table), n, _ptr(pos), _ptr(v), _ptr(grad), _ptr(lap),
                                _stream(stream), t), "spline_autotune")
    return (t[0], t[1])


def spline_tile_for(desc, n_pts=0):
    t = (ctypes.c_int32 * 2)()
    check(lib().spline_tile_for(ctypes.byref(desc), int(n_pts), t), "spline_tile_for")
    return (t[0], t[1])


class BatchPlan:
    """One persistent launch over many systems (spline_batch_* entry points).

    items: list of (desc, table, pos, v, grad, lap) with device tensors.  The
    tensors must stay alive as long as the plan does.
    """

    def __init__(self, items, tile=None, stream=None):
        self._keep = list(items)
        self._descs = [it[0] for it in items]
        arr = (SplItem * len(items))()
        for k, (desc, table, pos, v, grad, lap) in enumerate(items):
            _check_inputs(desc, table, pos)
            _outputs(desc, pos.shape[0], pos.device, v, grad, lap)
            arr[k].d = ctypes.pointer(self._descs[k])
            arr[k].table = table.data_ptr()
            arr[k].n_pts = pos.shape[0]
            arr[k].pos = pos.data_ptr()
            arr[k].v = v.data_ptr()
            arr[k].grad = grad.data_ptr()
            arr[k].lap = lap.data_ptr()
        self._items = arr
        plan = ctypes.c_void_p()
        t = None if tile is None else (ctypes.c_int32 * 2)(int(tile[0]), int(tile[1]))
        check(lib().spline_batch_plan_create(arr, len(items), t, _stream(stream), ctypes.byref(plan)),
              "spline_batch_plan_create")
        self._plan = plan

    def run(self, stream=None):
        check(lib().spline_batch_eval_vgl(self._plan, _stream(stream)), "spline_batch_eval_vgl")

    def run_graph(self, stream=None):
        check(lib().spline_batch_graph_launch(self._plan, _stream(stream)), "spline_batch_graph_launch")

    def autotune(self, stream=None):
        t = (ctypes.c_int32 * 2)()
        check(lib().spline_batch_autotune(self._plan, _stream(stream), t), "spline_batch_autotune")
        return (t[0], t[1])

    def tiles(self):
        """Each item's (lanes per point, orbitals per lane), in the order the items were given."""
        t = (ctypes.c_int32 * (2 * len(self._descs)))()
        check(lib().spline_batch_plan_get_tiles(self._plan, t), "spline_batch_plan_get_tiles")
        return [(t[2 * j], t[2 * j + 1]) for j in range(len(self._descs))]

    def set_tiles(self, tiles, stream=None):
        """Give item j the shape tiles[j] = (lanes per point, orbitals per lane); one orbitals per lane for all."""
        flat = (ctypes.c_int32 * (2 * len(self._descs)))(*[int(x) for t in tiles for x in t])
        check(lib().spline_batch_plan_set_tiles(self._plan, flat, _stream(stream)), "spline_batch_plan_set_tiles")

    def sort(self, enable=True, stream=None):
        """Evaluate the points in locality order from now on (same outputs); allocates once."""
        check(lib().spline_batch_plan_sort(self._plan, 1 if enable else 0, _stream(stream)), "spline_batch_plan_sort")

    def info(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        check(lib().spline_batch_plan_info(self._plan, ctypes.byref(a), ctypes.byref(b)), "spline_batch_plan_info")
        return a.value, b.value

    def close(self):
        if getattr(self, "_plan", None):
            lib().spline_batch_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
