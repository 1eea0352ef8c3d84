"""FP64 CPU oracle for the PDHG LP solve.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark may use this package; the product path never
does.  It shares no code with the HIP library.

Contents
- `pdhg_oracle.c` (built to `liboracle.so` with gcc, FP contraction off):
  validation, bound kinds, transpose, power-of-two Ruiz/Pock-Chambolle
  scaling, the restarted adaptive PDHG (paper, "PDHG Background": the
  Chambolle-Pock updates plus the adaptive steps and restarts of the PDLP
  method it cites), an independent KKT checker and the unrolled PDHG with
  its forward-mode derivative.
- `csr_matvec`: the sparse product y = A x by its definition (numpy).
- `exact.py`: the LP optimum by definition on tiny problems (vertex
  enumeration), a dense bounded simplex, and HiGHS through scipy as a
  library LP solve.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdhg_oracle.c")
# ORACLE_LIB points the loader at another build of the same source (the
# sanitizer build of the tests)
_DEFAULT_LIB = os.path.join(_HERE, "liboracle.so")
_LIB = os.environ.get("ORACLE_LIB", _DEFAULT_LIB)
_SAN_LIB = os.path.join(_HERE, "liboracle_san.so")
_lib = None

ST_OPTIMAL, ST_ITER_LIMIT, ST_NUMERICAL = 1, 2, 4
VK_FREE, VK_LOWER, VK_UPPER, VK_BOXED, VK_FIXED = range(5)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no FP contraction, no fast-math)."""
    out = _DEFAULT_LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


def build_sanitized() -> str:
    """The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer,
    every finding fatal (for the sanitizer test; load it with ORACLE_LIB and
    gcc's libasan preloaded)."""
    if not os.path.exists(_SAN_LIB) or os.path.getmtime(_SAN_LIB) < os.path.getmtime(_SRC):
        tmp = _SAN_LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                               "-fno-fast-math", "-std=c11", "-fPIC", "-shared",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SAN_LIB)
    return _SAN_LIB


class _Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int64),
                ("eval_period", ctypes.c_int), ("step_mode", ctypes.c_int),
                ("fixed_eta", ctypes.c_double), ("ruiz_iters", ctypes.c_int),
                ("pock_chambolle", ctypes.c_int), ("restart", ctypes.c_int),
                ("use_average", ctypes.c_int), ("omega0", ctypes.c_double),
                ("pw_theta", ctypes.c_double), ("infeas_every", ctypes.c_int),
                ("ilo", ctypes.c_void_p), ("ihi", ctypes.c_void_p),
                ("dinf_eps", ctypes.c_double), ("trace", ctypes.c_void_p),
                ("trace_cap", ctypes.c_int64), ("term", ctypes.c_int)]

# fields of one evaluation record of pdhg(..., trace=N)
TRACE_FIELDS = ("k", "komega_cur", "komega_avg", "komega_last", "komega_prev", "restart",
                "cand_avg", "omega", "komega_new")


def lib():
    global _lib
    if _lib is None:
        if _LIB == _DEFAULT_LIB:
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.orc_validate.argtypes = [i64, i64] + [P] * 8
        L.orc_validate.restype = ctypes.c_int
        L.orc_var_kind.argtypes = [i64, P, P, P]
        L.orc_transpose.argtypes = [i64, i64, P, P, P, P, P, P]
        L.orc_scale.argtypes = [i64, i64, P, P, P, ctypes.c_int, ctypes.c_int, P, P]
        L.orc_pow2_sqrt.argtypes = [ctypes.c_double]
        L.orc_pow2_sqrt.restype = ctypes.c_double
        L.orc_kkt.argtypes = [i64, i64] + [P] * 11
        L.orc_power_norm.argtypes = [i64, i64, P, P, P, ctypes.c_int]
        L.orc_power_norm.restype = ctypes.c_double
        L.orc_pdhg.argtypes = [i64, i64] + [P] * 8 + [ctypes.POINTER(_Opts)] + [P] * 5
        L.orc_pdhg.restype = ctypes.c_int
        L.orc_unrolled.argtypes = ([i64, i64] + [P] * 8 +
                                   [ctypes.c_int, ctypes.c_int, i64, ctypes.c_double,
                                    ctypes.c_double] + [P] * 6)
        L.orc_unrolled.restype = ctypes.c_int
        L.orc_implied_bounds.argtypes = [i64, i64] + [P] * 5 + [ctypes.c_int, P, P]
        L.orc_implied_bounds.restype = i64
        L.orc_safe_bound.argtypes = [i64, i64] + [P] * 12
        L.orc_bound_repair.argtypes = [i64, i64] + [P] * 9
        L.orc_bound_repair.restype = i64
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _arrs(lp):
    rp = np.ascontiguousarray(lp.row_ptr, np.int32)
    ci = np.ascontiguousarray(lp.col_idx, np.int32)
    v = np.ascontiguousarray(lp.val, np.float64)
    kind = np.ascontiguousarray(lp.row_kind, np.uint8)
    f = lambda a: np.ascontiguousarray(a, np.float64)
    return rp, ci, v, kind, f(lp.b), f(lp.c), f(lp.l), f(lp.u)


def implied_bounds(lp, passes=64):
    """(lo, hi): l, u with infinite entries replaced where bound propagation
    over the rows finds a finite bound (widened to cover rounding)."""
    rp, ci, v, kind, b, c, l, u = _arrs(lp)
    lo, hi = l.copy(), u.copy()
    lib().orc_implied_bounds(lp.m, lp.n, _p(rp), _p(ci), _p(v), _p(kind), _p(b), int(passes),
                             _p(lo), _p(hi))
    return lo, hi


def bound_repair(lp, lo=None, hi=None):
    """(ylo, yhi): per row, the interval that keeps the reduced costs of its
    single-entry columns with an infinite bound sign-feasible (with a 2^-40
    relative margin), intersected with y >= 0 on >= rows.  lo, hi: the
    bounds the safe bound uses (default: the implied bounds)."""
    rp, ci, v, kind, b, c, l, u = _arrs(lp)
    if lo is None or hi is None:
        lo, hi = implied_bounds(lp)
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    ylo, yhi = np.empty(lp.m), np.empty(lp.m)
    lib().orc_bound_repair(lp.m, lp.n, _p(rp), _p(ci), _p(v), _p(kind), _p(c), _p(lo), _p(hi),
                           _p(ylo), _p(yhi))
    return ylo, yhi


def safe_bound(lp, y, lo=None, hi=None, repair=True) -> dict:
    """Weak-duality lower bound on the optimum from y (projected on >= rows
    and, with `repair`, clamped into the repair intervals), with the bounds
    lo, hi (default: the implied bounds)."""
    rp, ci, v, kind, b, c, l, u = _arrs(lp)
    if lo is None or hi is None:
        lo, hi = implied_bounds(lp)
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    ylo = yhi = None
    if repair:
        ylo, yhi = bound_repair(lp, lo, hi)
    out = np.zeros(5)
    lib().orc_safe_bound(lp.m, lp.n, _p(rp), _p(ci), _p(v), _p(kind), _p(b), _p(c), _p(lo),
                         _p(hi), _p(ylo), _p(yhi), _p(y), _p(out))
    return dict(bound=out[0], value=out[1], allowance=out[2], infinite_terms=int(out[3]),
                repaired_rows=int(out[4]))


def validate(lp) -> int:
    a = _arrs(lp)
    return lib().orc_validate(lp.m, lp.n, *[_p(x) for x in a])


def var_kind(l, u) -> np.ndarray:
    l = np.ascontiguousarray(l, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    out = np.zeros(len(l), np.uint8)
    lib().orc_var_kind(len(l), _p(l), _p(u), _p(out))
    return out


def transpose(m, n, row_ptr, col_idx, val):
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col_idx, np.int32)
    v = np.ascontiguousarray(val, np.float64)
    cp = np.zeros(n + 1, np.int32)
    ri = np.zeros(len(ci), np.int32)
    vt = np.zeros(len(ci), np.float64)
    lib().orc_transpose(m, n, _p(rp), _p(ci), _p(v), _p(cp), _p(ri), _p(vt))
    return cp, ri, vt


def csr_matvec(row_ptr, col_idx, val, x):
    """y = A x by definition: y_i = sum over row i's nonzeros of a_ik x_k, the
    products and the sum in FP64, in CSR order (the sparse product that both
    steps of the "PDHG Background" iteration apply).  Also returns
    s_i = sum_k |a_ik x_k|, which with the row length bounds the rounding of
    any summation order of the same products."""
    rp = np.asarray(row_ptr, np.int64)
    ci = np.asarray(col_idx, np.int64)
    prod = np.asarray(val, np.float64) * np.asarray(x, np.float64)[ci]
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    m = len(rp) - 1
    y = np.bincount(rows, weights=prod, minlength=m)
    s = np.bincount(rows, weights=np.abs(prod), minlength=m)
    return y, s


def pow2_sqrt(M: float) -> float:
    return lib().orc_pow2_sqrt(float(M))


def scale(lp, ruiz_iters=10, pock_chambolle=True):
    """Returns (scaled values of A, Dr, Dc) with A_scaled = diag(Dr) A diag(Dc)."""
    rp, ci, v, *_ = _arrs(lp)
    v = v.copy()
    Dr = np.zeros(lp.m)
    Dc = np.zeros(lp.n)
    lib().orc_scale(lp.m, lp.n, _p(rp), _p(ci), _p(v), int(ruiz_iters),
                    int(bool(pock_chambolle)), _p(Dr), _p(Dc))
    return v, Dr, Dc


KKT_FIELDS = ("rel_p", "rel_d", "rel_gap", "rel_kkt", "pobj", "dobj", "rp_norm",
              "rd_norm", "gap", "rp_inf", "rd_inf", "bound_viol", "cone_viol")


def kkt(lp, x, y) -> dict:
    """Independent KKT check of (x, y) on the original problem."""
    a = _arrs(lp)
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    out = np.zeros(len(KKT_FIELDS))
    lib().orc_kkt(lp.m, lp.n, *[_p(z) for z in a], _p(x), _p(y), _p(out))
    return dict(zip(KKT_FIELDS, out.tolist()))


def power_norm(m, n, row_ptr, col_idx, val, iters=50) -> float:
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col_idx, np.int32)
    v = np.ascontiguousarray(val, np.float64)
    return lib().orc_power_norm(m, n, _p(rp), _p(ci), _p(v), int(iters))


INFO_FIELDS = ("status", "attempts", "accepted", "restarts", "pobj", "dobj", "rel_p",
               "rel_d", "rel_gap", "rel_kkt", "eta", "omega", "which", "eta0", "omega0",
               "evaluations")


def pdhg(lp, tol=1e-4, max_iter=100000, eval_period=64, step_mode=0, fixed_eta=0.0,
         ruiz_iters=10, pock_chambolle=True, restart=True, use_average=True,
         omega0=0.0, pw_theta=0.5, x0=None, y0=None, infeas_every=4, dinf_eps=1e-8,
         trace=0, term=0):
    """Restarted PDHG in FP64.  Returns (x, y, info dict) in the original space.
    Every `infeas_every` evaluations (0: never) the current y is tested as a
    certificate of primal infeasibility over the implied bounds (status 5),
    then (dinf_eps > 0) the primal displacement since the last restart as a
    ray certifying dual infeasibility (status 6; x is then the ray).
    trace > 0 adds info["trace"]: the first `trace` evaluations that reached
    the restart decision, one dict of TRACE_FIELDS each.  term: the measure
    held to tol (0 relative KKT error, 1 primal residual, 2 dual residual)."""
    a = _arrs(lp)
    ilo = ihi = None
    if infeas_every > 0:
        ilo, ihi = implied_bounds(lp)
    o = _Opts(tol, int(max_iter), int(eval_period), int(step_mode), float(fixed_eta),
              int(ruiz_iters), int(bool(pock_chambolle)), int(bool(restart)),
              int(bool(use_average)), float(omega0), float(pw_theta), int(infeas_every),
              _p(ilo), _p(ihi), float(dinf_eps))
    o.term = int(term)
    tr = np.zeros((max(int(trace), 1), len(TRACE_FIELDS)))
    if trace > 0:
        o.trace = tr.ctypes.data_as(ctypes.c_void_p)
        o.trace_cap = int(trace)
    x = np.zeros(lp.n)
    y = np.zeros(lp.m)
    info = np.zeros(len(INFO_FIELDS))
    x0 = None if x0 is None else np.ascontiguousarray(x0, np.float64)
    y0 = None if y0 is None else np.ascontiguousarray(y0, np.float64)
    rc = lib().orc_pdhg(lp.m, lp.n, *[_p(z) for z in a], ctypes.byref(o), _p(x0), _p(y0),
                        _p(x), _p(y), _p(info))
    if rc != 0:
        raise RuntimeError(f"oracle pdhg failed: {rc}")
    d = dict(zip(INFO_FIELDS, info.tolist()))
    for k in ("status", "attempts", "accepted", "restarts", "which", "evaluations"):
        d[k] = int(d[k])
    if trace > 0:
        d["trace"] = [dict(zip(TRACE_FIELDS, r)) for r in tr[:min(d["evaluations"], int(trace))]]
    return x, y, d


def unrolled(lp, K, eta, omega, db=None, dc=None, ruiz_iters=10, pock_chambolle=True,
             return_xy=False):
    """Unrolled fixed-step PDHG: V = c'x_K and its derivative along (db, dc)."""
    a = _arrs(lp)
    V = ctypes.c_double()
    dV = ctypes.c_double()
    db = None if db is None else np.ascontiguousarray(db, np.float64)
    dc = None if dc is None else np.ascontiguousarray(dc, np.float64)
    x = np.zeros(lp.n) if return_xy else None
    y = np.zeros(lp.m) if return_xy else None
    lib().orc_unrolled(lp.m, lp.n, *[_p(z) for z in a], int(ruiz_iters),
                       int(bool(pock_chambolle)), int(K), float(eta), float(omega),
                       _p(db), _p(dc), ctypes.byref(V), ctypes.byref(dV), _p(x), _p(y))
    if return_xy:
        return V.value, dV.value, x, y
    return V.value, dV.value


def unrolled_step(lp, ruiz_iters=10, pock_chambolle=True, iters=50):
    """Fixed step of the unrolled mode: eta = 0.9/||A^||_2 and omega = ||c^||/||b^||."""
    v, Dr, Dc = scale(lp, ruiz_iters, pock_chambolle)
    nrm = power_norm(lp.m, lp.n, lp.row_ptr, lp.col_idx, v, iters)
    cs = Dc * lp.c
    bs = Dr * lp.b
    nc, nb = np.linalg.norm(cs), np.linalg.norm(bs)
    omega = nc / nb if (nc > 1e-10 and nb > 1e-10) else 1.0
    return 0.9 / nrm, omega
