"""ctypes declarations of the C ABI in include/pdhg.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# PDHG_LIB points the loader at another build of the same sources (the
# host-sanitizer build of the tests); there is no fallback either way
LIB_PATH = os.environ.get("PDHG_LIB", os.path.join(_HERE, "libpdhg.so"))

PDHG_OK = 0
ERRORS = {-1: "PDHG_ERR_ARG", -2: "PDHG_ERR_CSR", -3: "PDHG_ERR_BOUNDS",
          -4: "PDHG_ERR_NONFINITE", -5: "PDHG_ERR_OOM", -6: "PDHG_ERR_HIP",
          -7: "PDHG_ERR_STATE"}
STATUS = {1: "OPTIMAL", 2: "ITER_LIMIT", 3: "TIME_LIMIT", 4: "NUMERICAL", 5: "PRIMAL_INFEASIBLE",
          6: "DUAL_INFEASIBLE"}
PDHG_FP64, PDHG_MIXED = 0, 1

c_i64 = ctypes.c_int64
c_dbl = ctypes.c_double
c_int = ctypes.c_int
vp = ctypes.c_void_p


class PdhgLP(ctypes.Structure):
    _fields_ = [("m", c_i64), ("n", c_i64), ("nnz", c_i64),
                ("row_ptr", vp), ("col_idx", vp), ("val", vp), ("row_kind", vp),
                ("b", vp), ("c", vp), ("l", vp), ("u", vp), ("obj_offset", c_dbl),
                ("on_device", c_int)]


class PdhgOpts(ctypes.Structure):
    _fields_ = [("tol", c_dbl), ("max_iter", c_i64), ("time_limit_s", c_dbl),
                ("precision", c_int), ("eval_period", c_int), ("step_mode", c_int),
                ("fixed_eta", c_dbl), ("fixed_omega", c_dbl), ("scaling_iters", c_int),
                ("pock_chambolle", c_int), ("restart", c_int), ("use_average", c_int),
                ("unroll_iters", c_i64), ("checkpoint_every", c_i64), ("use_graph", c_int),
                ("verbose", c_int), ("polish_tol", c_dbl), ("pw_update", c_int),
                ("pw_theta", c_dbl), ("tiles_per_block", c_int), ("autotune", c_int),
                ("spmv_direct", c_int), ("long_seg", c_int), ("reorder", c_int),
                ("compact_index", c_int), ("infeas_every", c_int),
                ("polish_pw_update", c_int), ("fp32_stall_evals", c_int),
                ("dinf_tol", c_dbl), ("batch_pack", c_int),
                ("stream_nt", c_int), ("polish_fp32_matrix", c_int)]


class PdhgInfo(ctypes.Structure):
    _fields_ = [("status", c_int), ("which", c_int), ("attempts", c_i64),
                ("accepted", c_i64), ("restarts", c_i64), ("attempts_fp32", c_i64),
                ("primal_obj", c_dbl), ("dual_obj", c_dbl), ("rel_primal", c_dbl),
                ("rel_dual", c_dbl), ("rel_gap", c_dbl), ("rel_kkt", c_dbl),
                ("eta", c_dbl), ("omega", c_dbl), ("setup_s", c_dbl), ("solve_s", c_dbl),
                ("dual_bound", c_dbl)]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


class PdhgInstance(ctypes.Structure):
    _fields_ = [("base", ctypes.c_int32), ("b", vp), ("c", vp), ("l", vp), ("u", vp),
                ("fix_idx", vp), ("fix_val", vp), ("n_fix", c_i64), ("x0", vp), ("y0", vp),
                ("omega0", c_dbl), ("eta0", c_dbl), ("hold_omega", c_i64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "pdhg_default_opts": (None, [ctypes.POINTER(PdhgOpts)]),
    "pdhg_workspace_bytes": (c_int, [ctypes.POINTER(PdhgLP), ctypes.POINTER(PdhgOpts),
                                     ctypes.POINTER(ctypes.c_size_t)]),
    "pdhg_setup": (c_int, [ctypes.POINTER(PdhgLP), ctypes.POINTER(PdhgOpts), vp,
                           ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
    "pdhg_solve": (c_int, [vp, vp, vp, vp, vp, ctypes.POINTER(PdhgInfo)]),
    "pdhg_batch_workspace_bytes": (c_int, [ctypes.POINTER(vp), c_int,
                                           ctypes.POINTER(PdhgInstance), c_int,
                                           ctypes.POINTER(ctypes.c_size_t)]),
    "pdhg_solve_batch": (c_int, [ctypes.POINTER(vp), c_int, ctypes.POINTER(PdhgInstance),
                                 c_int, vp, ctypes.c_size_t, ctypes.POINTER(vp),
                                 ctypes.POINTER(vp), ctypes.POINTER(PdhgInfo)]),
    "pdhg_export_fp32": (c_int, [vp, vp, vp, vp, vp, vp, vp]),
    "pdhg_polish": (c_int, [vp, vp, vp, c_dbl, c_i64, c_dbl, vp, vp, ctypes.POINTER(PdhgInfo)]),
    "pdhg_solve_batch_static": (c_int, [ctypes.POINTER(vp), c_int, ctypes.POINTER(PdhgInstance),
                                        c_int, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                        ctypes.POINTER(PdhgInfo)]),
    "pdhg_backward": (c_int, [vp, c_dbl, vp, vp]),
    "pdhg_update": (c_int, [vp, vp, vp]),
    "pdhg_destroy": (None, [vp]),
    "pdhg_last_error": (ctypes.c_char_p, []),
    "pdhg_export_setup": (c_int, [vp, vp, vp, vp, vp, vp, vp, vp]),
    "pdhg_spmv": (c_int, [vp, c_int, vp, vp]),
    "pdhg_time_kernels": (c_int, [vp, c_int, ctypes.POINTER(c_dbl)]),
    "pdhg_time_kernels_cold": (c_int, [vp, c_int, vp, ctypes.c_size_t, vp]),
    "pdhg_spmv_merge_workspace_bytes": (c_int, [c_i64, c_i64, ctypes.POINTER(ctypes.c_size_t)]),
    "pdhg_spmv_merge_plan": (c_int, [c_i64, c_i64, c_i64, vp, vp, vp, ctypes.c_size_t, vp]),
    "pdhg_spmv_merge_f64": (c_int, [c_i64, c_i64, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
    "pdhg_spmv_merge_f32": (c_int, [c_i64, c_i64, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
    "pdhg_time_spmv_merge": (c_int, [vp, c_int, vp, ctypes.c_size_t, vp]),
    "pdhg_get_partition": (c_int, [vp, ctypes.POINTER(c_int)]),
    "pdhg_locality_order": (c_int, [c_i64, c_i64, vp, vp, vp, vp]),
    "pdhg_implied_bounds": (c_int, [vp, vp, vp]),
}

_lib = None


class PdhgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def load():
    """Load libpdhg.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2512_06715_amd.build`")
        # torch's HIP runtime is loaded first, so the library binds to the
        # same one (loading the library before torch leaves two runtimes in
        # the process, and the second finds no device)
        import torch  # noqa: F401
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(rc: int):
    if rc != PDHG_OK:
        raise PdhgError(rc, load().pdhg_last_error().decode())
    return rc
