"""The C ABI on the host: the library loads, exports every declared entry
point, and rejects bad input before touching a device (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2512_06715_amd import _lib as L
from paper_2512_06715_amd import ucgen

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "pdhg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdhg_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.SIGNATURES)


def test_default_opts():
    lib = L.load()
    o = L.PdhgOpts()
    lib.pdhg_default_opts(ctypes.byref(o))
    assert o.tol == 1e-4 and o.eval_period == 64 and o.scaling_iters == 10
    assert o.pock_chambolle == 1 and o.restart == 1 and o.use_average == 1
    assert o.step_mode == 0 and o.precision == L.PDHG_FP64 and o.pw_theta == 0.5
    assert o.reorder == 1 and o.compact_index == 1 and o.polish_pw_update == 1
    assert o.fp32_stall_evals == 300 and o.dinf_tol == 1e-8
    assert o.batch_pack == 0 and o.stream_nt == -1 and o.polish_fp32_matrix == 1


def _lp_struct(lp, obj_offset=0.0):
    arrs = [np.ascontiguousarray(lp.row_ptr, np.int32), np.ascontiguousarray(lp.col_idx, np.int32),
            np.ascontiguousarray(lp.val, np.float64), np.ascontiguousarray(lp.row_kind, np.uint8),
            np.ascontiguousarray(lp.b, np.float64), np.ascontiguousarray(lp.c, np.float64),
            np.ascontiguousarray(lp.l, np.float64), np.ascontiguousarray(lp.u, np.float64)]
    s = L.PdhgLP(lp.m, lp.n, len(lp.col_idx), *[a.ctypes.data_as(ctypes.c_void_p) for a in arrs],
                 obj_offset, 0)
    return s, arrs


def _setup_rc(lp, opts=None, obj_offset=0.0):
    lib = L.load()
    s, keep = _lp_struct(lp, obj_offset)
    o = L.PdhgOpts()
    lib.pdhg_default_opts(ctypes.byref(o))
    if opts:
        for k, v in opts.items():
            setattr(o, k, v)
    # no workspace: input checks come first, and a valid LP stops at the
    # workspace check (PDHG_ERR_OOM) before any device call
    h = ctypes.c_void_p()
    rc = lib.pdhg_setup(ctypes.byref(s), ctypes.byref(o), None, 0, None, ctypes.byref(h))
    return rc, lib.pdhg_last_error().decode()


def test_workspace_bytes_grows_with_size_and_precision():
    lib = L.load()
    out = []
    for name in ("uc14_t24", "uc1000_t48"):
        lp = ucgen.workload(name)
        s, keep = _lp_struct(lp)
        for prec in (L.PDHG_FP64, L.PDHG_MIXED):
            o = L.PdhgOpts()
            lib.pdhg_default_opts(ctypes.byref(o))
            o.precision = prec
            nb = ctypes.c_size_t()
            assert lib.pdhg_workspace_bytes(ctypes.byref(s), ctypes.byref(o), ctypes.byref(nb)) == 0
            out.append(nb.value)
    assert out[0] < out[1] < out[3] and out[0] < out[2]
    # FP64 bytes at least cover A and A' (12 bytes per nonzero each) and 16 vectors
    lp = ucgen.workload("uc1000_t48")
    assert out[2] >= 24 * lp.nnz + 8 * 16 * (lp.m + lp.n) // 2


@pytest.mark.parametrize("mutate,code", [
    (lambda lp: setattr(lp, "col_idx", np.where(np.arange(len(lp.col_idx)) == 1, lp.col_idx[0], lp.col_idx)), -2),
    (lambda lp: setattr(lp, "row_ptr", np.concatenate([[1], lp.row_ptr[1:]]).astype(np.int32)), -2),
    (lambda lp: setattr(lp, "row_kind", np.where(np.arange(lp.m) == 3, 2, lp.row_kind).astype(np.uint8)), -1),
    (lambda lp: setattr(lp, "l", np.where(np.arange(lp.n) == 0, 5.0, lp.l)), -3),
    (lambda lp: setattr(lp, "u", np.where(np.arange(lp.n) == 7, -np.inf, lp.u)), -3),
    (lambda lp: setattr(lp, "val", np.where(np.arange(len(lp.val)) == 9, np.inf, lp.val)), -4),
    (lambda lp: setattr(lp, "b", np.where(np.arange(lp.m) == 9, np.nan, lp.b)), -4),
    (lambda lp: setattr(lp, "c", np.where(np.arange(lp.n) == 2, np.nan, lp.c)), -4),
])
def test_setup_rejects_bad_input_on_host(mutate, code, oracle_mod):
    lp = ucgen.workload("uc14_t24").copy()
    mutate(lp)
    rc, msg = _setup_rc(lp)
    assert rc == code, msg
    assert msg
    assert oracle_mod.validate(lp) == code   # same category as the oracle


def test_setup_rejects_bad_options_and_small_workspace():
    lp = ucgen.workload("uc14_t24")
    assert _setup_rc(lp, dict(tol=0.0))[0] == -1
    assert _setup_rc(lp, dict(eval_period=0))[0] == -1
    assert _setup_rc(lp, dict(precision=7))[0] == -1
    assert _setup_rc(lp, dict(pw_theta=2.0))[0] == -1
    for bad in (dict(reorder=2), dict(compact_index=-1), dict(polish_pw_update=3),
                dict(fp32_stall_evals=-1), dict(dinf_tol=-1.0), dict(batch_pack=2),
                dict(stream_nt=2), dict(polish_fp32_matrix=-1)):
        rc, msg = _setup_rc(lp, bad)
        assert rc == -1 and list(bad)[0] in msg, (bad, msg)
    lib = L.load()
    s, keep = _lp_struct(lp)
    o = L.PdhgOpts()
    lib.pdhg_default_opts(ctypes.byref(o))
    buf = (ctypes.c_uint8 * 16)()
    h = ctypes.c_void_p()
    rc = lib.pdhg_setup(ctypes.byref(s), ctypes.byref(o), ctypes.cast(buf, ctypes.c_void_p), 16,
                        None, ctypes.byref(h))
    assert rc == -5


def test_shape_errors():
    lp = ucgen.workload("uc14_t24").copy()
    assert _setup_rc(lp)[0] == -5     # valid LP, no workspace
    assert _setup_rc(lp, obj_offset=-1e9)[0] == -5
    for bad in (float("nan"), float("inf")):
        rc, msg = _setup_rc(lp, obj_offset=bad)
        assert rc == -4 and "obj_offset" in msg
    lp.m = 0
    assert _setup_rc(lp)[0] == -1


def _lines_per_wave(rp, ci, elem=4, line=128, wave=64):
    """Distinct cache lines the lanes of one wave touch when 64 consecutive
    nonzeros gather the vector by their column index (the LDS-staged SpMV)."""
    L_ = np.asarray(ci, np.int64) * elem // line
    nw = (len(L_) + wave - 1) // wave
    pad = np.full(nw * wave, -1, np.int64)
    pad[:len(L_)] = L_
    pad = np.sort(pad.reshape(nw, wave), axis=1)
    return ((np.diff(pad, axis=1) != 0).sum(axis=1) + 1).sum() / nw


def test_locality_order_is_a_permutation_and_localises_gathers():
    import scipy.sparse as sp
    from paper_2512_06715_amd.solver import locality_order
    lp = ucgen.workload("uc1000_t48")
    ro, co = locality_order(lp)
    assert np.array_equal(np.sort(ro), np.arange(lp.m))
    assert np.array_equal(np.sort(co), np.arange(lp.n))
    ro2, co2 = locality_order(lp)  # deterministic
    assert np.array_equal(ro, ro2) and np.array_equal(co, co2)
    A = sp.csr_matrix((lp.val, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))
    P = A[ro][:, co].tocsr()
    P.sort_indices()
    for M0, M1 in ((A, P), (A.T.tocsr(), P.T.tocsr())):
        before = _lines_per_wave(M0.indptr, M0.indices)
        after = _lines_per_wave(M1.indptr, M1.indices)
        assert after < 0.6 * before, (before, after)


def test_locality_order_of_disconnected_and_empty_parts():
    from paper_2512_06715_amd.solver import locality_order
    # two blocks, an empty row and an empty column
    A = np.zeros((5, 6))
    A[0, 0] = A[0, 1] = A[1, 1] = 1.0
    A[3, 4] = A[4, 4] = A[4, 5] = 2.0
    lp = ucgen.dense_to_lp(A, np.zeros(5, np.uint8), np.ones(5), np.ones(6), np.zeros(6),
                           np.ones(6))
    ro, co = locality_order(lp)
    assert sorted(ro) == list(range(5)) and sorted(co) == list(range(6))


def test_locality_order_rejects_bad_csr():
    lib = L.load()
    rp = np.array([0, 2, 1], np.int32)
    ci = np.array([0, 1], np.int32)
    ro = np.empty(2, np.int32)
    co = np.empty(2, np.int32)
    rc = lib.pdhg_locality_order(2, 2, rp.ctypes.data, ci.ctypes.data, ro.ctypes.data,
                                 co.ctypes.data)
    assert rc == -2  # PDHG_ERR_CSR
    rp = np.array([0, 2, 2], np.int32)
    ci = np.array([1, 0], np.int32)  # not ascending
    rc = lib.pdhg_locality_order(2, 2, rp.ctypes.data, ci.ctypes.data, ro.ctypes.data,
                                 co.ctypes.data)
    assert rc == -2  # PDHG_ERR_CSR


def _c_struct_fields(name):
    """Field names of `typedef struct {...} name;` in the header, in order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    end = re.search(r"\}\s*" + name + r";", text).start()
    body = text[text.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        decl = re.sub(r"^(const\s+)?\w+\s*", "", decl)   # the type
        fields += [f.strip().lstrip("*").strip() for f in decl.split(",")]
    return fields


@pytest.mark.parametrize("cname,pytype", [("pdhg_lp", "PdhgLP"), ("pdhg_opts", "PdhgOpts"),
                                          ("pdhg_info", "PdhgInfo"),
                                          ("pdhg_instance", "PdhgInstance")])
def test_struct_layouts_match_the_header(cname, pytype, tmp_path):
    """Size and every field offset of the ABI structs, as a C compiler lays
    them out from the header, equal the binding's ctypes definitions."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    fields = _c_struct_fields(cname)
    src = tmp_path / "layout.c"
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pdhg.h"', "int main(void) {",
             f'  printf("size %zu\\n", sizeof({cname}));']
    lines += [f'  printf("{f} %zu\\n", offsetof({cname}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    py = getattr(L, pytype)
    assert [f[0] for f in py._fields_] == fields
    assert int(got["size"]) == ctypes.sizeof(py)
    for f in fields:
        assert int(got[f]) == getattr(py, f).offset, f
