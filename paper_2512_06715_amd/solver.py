"""Python front end of libpdhg: a Problem owns one handle and its workspace.

Every step of the solve runs in the HIP library; this module only moves
arguments across the C ABI.  PyTorch provides the device workspace and the
stream.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib as L

OPTION_NAMES = [f for f, _ in L.PdhgOpts._fields_]


def default_opts(**overrides) -> L.PdhgOpts:
    o = L.PdhgOpts()
    L.load().pdhg_default_opts(ctypes.byref(o))
    for k, v in overrides.items():
        if k not in OPTION_NAMES:
            raise KeyError(f"unknown option {k}")
        if k == "precision" and isinstance(v, str):
            v = {"fp64": L.PDHG_FP64, "mixed": L.PDHG_MIXED}[v]
        setattr(o, k, v)
    return o


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


class Problem:
    """An LP set up on the GPU.

    `lp` has attributes m, n, row_ptr, col_idx, val, row_kind, b, c, l, u
    (numpy arrays: host input, or torch CUDA tensors with device=True) and
    optionally obj_offset, a constant added to the reported objectives.
    """

    def __init__(self, lp, device: bool = False, stream=None, **opts):
        import torch
        lib = L.load()
        self.m, self.n = int(lp.m), int(lp.n)
        self.device = device
        if device:
            arrs = dict(row_ptr=lp.row_ptr, col_idx=lp.col_idx, val=lp.val,
                        row_kind=lp.row_kind, b=lp.b, c=lp.c, l=lp.l, u=lp.u)
            nnz = int(arrs["col_idx"].numel())
        else:
            arrs = dict(row_ptr=_host(lp.row_ptr, np.int32), col_idx=_host(lp.col_idx, np.int32),
                        val=_host(lp.val, np.float64), row_kind=_host(lp.row_kind, np.uint8),
                        b=_host(lp.b, np.float64), c=_host(lp.c, np.float64),
                        l=_host(lp.l, np.float64), u=_host(lp.u, np.float64))
            nnz = int(len(arrs["col_idx"]))
        self._keep = arrs
        self.nnz = nnz
        self._lp = L.PdhgLP(self.m, self.n, nnz, *[_ptr(arrs[k]) for k in
                            ("row_ptr", "col_idx", "val", "row_kind", "b", "c", "l", "u")],
                            float(getattr(lp, "obj_offset", 0.0)), 1 if device else 0)
        self.opts = default_opts(**opts)
        nbytes = ctypes.c_size_t()
        L.check(lib.pdhg_workspace_bytes(ctypes.byref(self._lp), ctypes.byref(self.opts),
                                         ctypes.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device="cuda")
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        L.check(lib.pdhg_setup(ctypes.byref(self._lp), ctypes.byref(self.opts),
                               ctypes.c_void_p(self.workspace.data_ptr()),
                               self.workspace_bytes, ctypes.c_void_p(stream.cuda_stream),
                               ctypes.byref(h)))
        self.handle = h
        self._keep = None if not device else arrs

    def solve(self, x0=None, y0=None, out=None):
        """Returns (x, y, info dict); numpy arrays for host problems."""
        lib = L.load()
        if self.device:
            import torch
            x = torch.empty(self.n, dtype=torch.float64, device="cuda") if out is None else out[0]
            y = torch.empty(self.m, dtype=torch.float64, device="cuda") if out is None else out[1]
        else:
            x = np.zeros(self.n) if out is None else out[0]
            y = np.zeros(self.m) if out is None else out[1]
            x0 = None if x0 is None else _host(x0, np.float64)
            y0 = None if y0 is None else _host(y0, np.float64)
        info = L.PdhgInfo()
        L.check(lib.pdhg_solve(self.handle, _ptr(x0), _ptr(y0), _ptr(x), _ptr(y),
                               ctypes.byref(info)))
        return x, y, info.as_dict()

    def polish(self, x, y, tol: float = 1e-8, max_iter: int = 0, omega: float = 0.0):
        """Feasibility polishing of (x, y): returns (x', y', info dict) with the
        combined point's measures on the original problem (pdhg_polish)."""
        lib = L.load()
        if self.device:
            import torch
            xo = torch.empty(self.n, dtype=torch.float64, device="cuda")
            yo = torch.empty(self.m, dtype=torch.float64, device="cuda")
        else:
            x, y = _host(x, np.float64), _host(y, np.float64)
            xo, yo = np.zeros(self.n), np.zeros(self.m)
        info = L.PdhgInfo()
        L.check(lib.pdhg_polish(self.handle, _ptr(x), _ptr(y), float(tol), int(max_iter),
                                float(omega), _ptr(xo), _ptr(yo), ctypes.byref(info)))
        return xo, yo, info.as_dict()

    def export_setup(self) -> dict:
        lib = L.load()
        out = dict(var_kind=np.zeros(self.n, np.uint8), colptr=np.zeros(self.n + 1, np.int32),
                   rowidx=np.zeros(self.nnz, np.int32), valT=np.zeros(self.nnz),
                   val_s=np.zeros(self.nnz), Dr=np.zeros(self.m), Dc=np.zeros(self.n))
        L.check(lib.pdhg_export_setup(self.handle, *[_ptr(out[k]) for k in
                                      ("var_kind", "colptr", "rowidx", "valT", "val_s", "Dr", "Dc")]))
        return out

    def export_fp32(self) -> dict:
        """The FP32 copies of the mixed-precision path (caller's order)."""
        lib = L.load()
        out = dict(val_s=np.zeros(self.nnz, np.float32), valT=np.zeros(self.nnz, np.float32),
                   b=np.zeros(self.m, np.float32), c=np.zeros(self.n, np.float32),
                   l=np.zeros(self.n, np.float32), u=np.zeros(self.n, np.float32))
        L.check(lib.pdhg_export_fp32(self.handle, *[_ptr(out[k]) for k in
                                     ("val_s", "valT", "b", "c", "l", "u")]))
        return out

    def spmv(self, x, transpose: bool = False) -> np.ndarray:
        lib = L.load()
        x = _host(x, np.float64)
        out = np.zeros(self.n if transpose else self.m)
        L.check(lib.pdhg_spmv(self.handle, 1 if transpose else 0, _ptr(x), _ptr(out)))
        return out

    def update(self, b=None, c=None):
        """Replace b and/or c (original space) of the set-up problem."""
        lib = L.load()
        if not self.device:
            b = None if b is None else _host(b, np.float64)
            c = None if c is None else _host(c, np.float64)
        L.check(lib.pdhg_update(self.handle, _ptr(b), _ptr(c)))

    def backward(self, grad_value: float = 1.0):
        """Gradient of c'x_K of the last unrolled solve w.r.t. (b, c), times grad_value."""
        lib = L.load()
        if self.device:
            import torch
            gb = torch.empty(self.m, dtype=torch.float64, device="cuda")
            gc = torch.empty(self.n, dtype=torch.float64, device="cuda")
        else:
            gb, gc = np.zeros(self.m), np.zeros(self.n)
        L.check(lib.pdhg_backward(self.handle, float(grad_value), _ptr(gb), _ptr(gc)))
        return gb, gc

    def partition(self) -> dict:
        """The SpMV partition in use (chosen by the autotuner or the options)."""
        out = (ctypes.c_int * 7)()
        L.check(L.load().pdhg_get_partition(self.handle, out))
        return dict(tiles_per_block=out[0], direct=out[1], long_seg=out[2], long_segments=out[3],
                    compact=out[4], stream_nt_fp64=out[5], stream_nt_fp32=out[6])

    def time_kernels(self, attempts: int = 200) -> dict:
        """Average ms per launch of the attempt kernels, timed with HIP events."""
        lib = L.load()
        ms = (ctypes.c_double * 4)()
        L.check(lib.pdhg_time_kernels(self.handle, int(attempts), ms))
        return dict(primal=ms[0], dual=ms[1], control=ms[2], attempt=ms[3])

    def time_kernels_cold(self, attempts: int = 50, flush_bytes: int = 1 << 30) -> dict:
        """time_kernels with the L2 and Infinity Cache flushed before each attempt
        (a read of a flush_bytes device buffer)."""
        import torch
        lib = L.load()
        ms = (ctypes.c_double * 4)()
        buf = torch.zeros(flush_bytes // 8, dtype=torch.float64, device="cuda")
        L.check(lib.pdhg_time_kernels_cold(self.handle, int(attempts),
                                           ctypes.c_void_p(buf.data_ptr()), int(flush_bytes), ms))
        del buf
        return dict(primal=ms[0], dual=ms[1], control=ms[2], attempt=ms[3])

    def time_spmv_merge(self, attempts: int = 200) -> dict:
        """Average ms of the merge-path SpMV on this problem's scaled matrices in
        its iteration precision: A'y (`transpose`) and A x (`forward`)."""
        import torch
        lib = L.load()
        nb = ctypes.c_size_t()
        L.check(lib.pdhg_spmv_merge_workspace_bytes(self.n, self.nnz, ctypes.byref(nb)))
        na = ctypes.c_size_t()
        L.check(lib.pdhg_spmv_merge_workspace_bytes(self.m, self.nnz, ctypes.byref(na)))
        ws = torch.empty(nb.value + na.value + 256, dtype=torch.uint8, device="cuda")
        base = (ws.data_ptr() + 255) & ~255
        ms = (ctypes.c_double * 2)()
        L.check(lib.pdhg_time_spmv_merge(self.handle, int(attempts), ctypes.c_void_p(base),
                                         nb.value + na.value, ms))
        del ws
        return dict(transpose=ms[0], forward=ms[1])

    def close(self):
        if getattr(self, "handle", None):
            L.load().pdhg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def implied_bounds(problem):
    """(lo, hi): the implied bounds the dual bound uses (caller's order)."""
    lo = np.zeros(problem.n)
    hi = np.zeros(problem.n)
    L.check(L.load().pdhg_implied_bounds(problem.handle, _ptr(lo), _ptr(hi)))
    return lo, hi


def locality_order(lp):
    """(row_order, col_order) of the relabelling pdhg_setup applies with
    reorder=1 (host computation, no GPU)."""
    rp = np.ascontiguousarray(lp.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(lp.col_idx, dtype=np.int32)
    ro = np.empty(lp.m, dtype=np.int32)
    co = np.empty(lp.n, dtype=np.int32)
    L.check(L.load().pdhg_locality_order(lp.m, lp.n, rp.ctypes.data, ci.ctypes.data,
                                         ro.ctypes.data, co.ctypes.data))
    return ro, co


def solve(lp, x0=None, y0=None, **opts):
    p = Problem(lp, **opts)
    try:
        return p.solve(x0, y0)
    finally:
        p.close()


class MergeSpmv:
    """Merge-path SpMV y = A x on device CSR tensors (int32 row_ptr and
    col_idx, float64 or float32 values): the plan is made once here, then
    each call launches on the current torch stream."""

    def __init__(self, row_ptr, col_idx, val, n: int):
        import torch
        lib = L.load()
        self.m = int(row_ptr.numel()) - 1
        self.n = int(n)
        self.nnz = int(col_idx.numel())
        if val.dtype not in (torch.float64, torch.float32) or int(val.numel()) != self.nnz:
            raise ValueError("val must be float64 or float32 with one entry per nonzero")
        self.dtype = val.dtype
        self.rp, self.ci, self.val = row_ptr, col_idx, val
        nb = ctypes.c_size_t()
        L.check(lib.pdhg_spmv_merge_workspace_bytes(self.m, self.nnz, ctypes.byref(nb)))
        self.ws_bytes = int(nb.value)
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device="cuda")
        self.ws = (self._ws.data_ptr() + 255) & ~255
        stream = torch.cuda.current_stream().cuda_stream
        L.check(lib.pdhg_spmv_merge_plan(self.m, self.n, self.nnz, _ptr(row_ptr), _ptr(col_idx),
                                         ctypes.c_void_p(self.ws), self.ws_bytes,
                                         ctypes.c_void_p(stream)))

    def __call__(self, x, out=None):
        import torch
        lib = L.load()
        if x.dtype != self.dtype or int(x.numel()) != self.n:
            raise ValueError("x must match the matrix's dtype and column count")
        y = torch.empty(self.m, dtype=self.dtype, device="cuda") if out is None else out
        fn = lib.pdhg_spmv_merge_f64 if self.dtype == torch.float64 else lib.pdhg_spmv_merge_f32
        stream = torch.cuda.current_stream().cuda_stream
        L.check(fn(self.m, self.nnz, _ptr(self.rp), _ptr(self.ci), _ptr(self.val), _ptr(x),
                   _ptr(y), ctypes.c_void_p(self.ws), self.ws_bytes, ctypes.c_void_p(stream)))
        return y


def solve_batch(problems, instances, stream=None, static=False):
    """Solve many instances in one batched run.

    problems: list of Problem (the bases; same precision).
    instances: list of dicts with key 'base' (index into problems) and optional
    'b', 'c', 'l', 'u' (original-space overrides), 'fix_idx', 'fix_val'
    (variables fixed to a value), 'x0', 'y0' (warm start), 'omega0',
    'eta0' (initial primal weight and step size, scaled space; 0 or absent:
    the defaults) and 'hold_omega' (attempts during which the primal weight
    keeps its initial value).  Host problems take numpy arrays, device problems torch
    CUDA tensors.  Returns a list of (x, y, info dict).

    static=True calls pdhg_solve_batch_static: no workspace is allocated; the
    library's fixed device scratch array (64 MiB) holds the batch.
    """
    import torch
    lib = L.load()
    H = (ctypes.c_void_p * len(problems))(*[p.handle for p in problems])
    keep = []
    arr = (L.PdhgInstance * len(instances))()
    outs = []
    for k, d in enumerate(instances):
        bi = int(d["base"])
        # an out-of-range base is passed through so the library rejects it
        base = problems[bi] if 0 <= bi < len(problems) else problems[0]

        def conv(a, dt):
            if a is None:
                return None
            if base.device:
                return a
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a
        fi = conv(d.get("fix_idx"), np.int32)
        fv = conv(d.get("fix_val"), np.float64)
        nfix = 0 if fi is None else int(fi.numel() if base.device else len(fi))
        arr[k] = L.PdhgInstance(bi, _ptr(conv(d.get("b"), np.float64)),
                                _ptr(conv(d.get("c"), np.float64)),
                                _ptr(conv(d.get("l"), np.float64)),
                                _ptr(conv(d.get("u"), np.float64)), _ptr(fi), _ptr(fv), nfix,
                                _ptr(conv(d.get("x0"), np.float64)),
                                _ptr(conv(d.get("y0"), np.float64)),
                                float(d.get("omega0", 0.0)), float(d.get("eta0", 0.0)),
                                int(d.get("hold_omega", 0)))
        if base.device:
            x = torch.empty(base.n, dtype=torch.float64, device="cuda")
            y = torch.empty(base.m, dtype=torch.float64, device="cuda")
        else:
            x = np.zeros(base.n)
            y = np.zeros(base.m)
        outs.append((x, y))
    X = (ctypes.c_void_p * len(instances))(*[_ptr(o[0]).value for o in outs])
    Y = (ctypes.c_void_p * len(instances))(*[_ptr(o[1]).value for o in outs])
    infos = (L.PdhgInfo * len(instances))()
    if static:
        L.check(lib.pdhg_solve_batch_static(H, len(problems), arr, len(instances), X, Y, infos))
    else:
        nb = ctypes.c_size_t()
        L.check(lib.pdhg_batch_workspace_bytes(H, len(problems), arr, len(instances),
                                               ctypes.byref(nb)))
        ws = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
        L.check(lib.pdhg_solve_batch(H, len(problems), arr, len(instances),
                                     ctypes.c_void_p(ws.data_ptr()), int(nb.value), X, Y, infos))
        del ws
    return [(outs[k][0], outs[k][1], infos[k].as_dict()) for k in range(len(instances))]
