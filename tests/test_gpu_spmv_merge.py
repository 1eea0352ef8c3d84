"""Merge-path SpMV (C ABI) against the oracle's y = A x by definition."""
import ctypes

import numpy as np
import pytest

from paper_2512_06715_amd import ucgen

pytestmark = pytest.mark.gpu

ITEMS = 2048  # merge-path items (row ends + nonzeros) per workgroup


def ragged_csr(seed, m, n, lens=None, long_rows=()):
    """Random CSR with row lengths 0-40, some rows empty, and long rows that
    span several workgroups' shares."""
    rng = np.random.default_rng(seed)
    if lens is None:
        lens = rng.integers(0, 41, m)
        lens[rng.random(m) < 0.1] = 0
        for r, k in long_rows:
            lens[r] = k
    lens = np.asarray(lens)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(n, int(k), replace=False)) if k else np.zeros(0, int)
                         for k in lens]).astype(np.int32)
    val = rng.standard_normal(int(rp[-1])) * 10.0 ** rng.integers(-2, 3, int(rp[-1]))
    x = rng.standard_normal(n)
    return rp, ci, val, x


def run_merge(rp, ci, val, x, n, dtype):
    import torch
    from paper_2512_06715_amd.solver import MergeSpmv
    t = dict(device="cuda")
    op = MergeSpmv(torch.tensor(rp, **t), torch.tensor(ci, **t),
                   torch.tensor(val, dtype=dtype, **t), n)
    xd = torch.tensor(x, dtype=dtype, **t)
    y1 = op(xd)
    y2 = op(xd)
    torch.cuda.synchronize()
    return y1.cpu().numpy(), y2.cpu().numpy()


def check(rp, ci, val, x, n, oracle_mod):
    import torch
    lens = np.diff(rp)
    for dtype, u in ((torch.float64, 2.0 ** -53), (torch.float32, 2.0 ** -24)):
        if dtype == torch.float32:
            # the FP32 kernel sees the FP32 casts; the reference is their exact product
            vr = val.astype(np.float32).astype(np.float64)
            xr = x.astype(np.float32).astype(np.float64)
        else:
            vr, xr = val, x
        y, y2 = run_merge(rp, ci, vr, xr, n, dtype)
        assert np.array_equal(y.view(np.uint8), y2.view(np.uint8)), "repeat differs"
        ref, sabs = oracle_mod.csr_matvec(rp, ci, vr, xr)
        # products rounded once each, sums in any order: (len + 1) u sum |a x|
        # (the reference's own FP64 error is below 2^-29 of that for FP32)
        bound = (lens + 1) * u * sabs * 1.0001 + 1e-300
        err = np.abs(y.astype(np.float64) - ref)
        bad = np.nonzero(err > bound)[0]
        assert bad.size == 0, (dtype, bad[:5], err[bad[:5]], bound[bad[:5]])
        assert np.all(y[lens == 0] == 0)


@pytest.mark.parametrize("seed", [0, 1])
def test_ragged_rows_several_workgroups(gpu, oracle_mod, seed):
    print("case merge ragged", seed, flush=True)
    rp, ci, val, x = ragged_csr(seed, 3000, 9000, long_rows=[(7, 5000), (1500, 2047), (2999, 8100)])
    check(rp, ci, val, x, 9000, oracle_mod)


@pytest.mark.parametrize("case", ["one_row", "no_nonzeros", "empty_then_long", "aligned",
                                  "single_entries", "one_workgroup"])
def test_edge_cases(gpu, oracle_mod, case):
    print("case merge edge", case, flush=True)
    n = 5000
    if case == "one_row":
        lens = [4500]
    elif case == "no_nonzeros":
        lens = [0] * 777
    elif case == "empty_then_long":
        lens = [0] * 3000 + [4096] + [0] * 5
    elif case == "aligned":
        # every row's items (row end + nonzeros) fill a workgroup's share exactly
        lens = [ITEMS - 1] * 2 + [ITEMS // 2 - 1] * 4
    elif case == "single_entries":
        lens = [1] * 10000
    else:
        lens = [3, 0, 5, 1]
    rp, ci, val, x = ragged_csr(11, len(lens), n, lens=lens)
    check(rp, ci, val, x, n, oracle_mod)


def test_paper_scale_matrix(gpu, oracle_mod):
    """A and its transpose of the 6717-bus, 96-period LP (2.03M x 3.22M, 7.19M
    nonzeros), every row against the oracle."""
    print("case merge uc6717", flush=True)
    lp = ucgen.workload("uc6717_t96")
    rng = np.random.default_rng(3)
    x = rng.standard_normal(lp.n)
    check(lp.row_ptr, lp.col_idx, lp.val, x, lp.n, oracle_mod)
    cp, ri, vt = oracle_mod.transpose(lp.m, lp.n, lp.row_ptr, lp.col_idx, lp.val)
    yv = rng.standard_normal(lp.m)
    check(cp, ri, vt, yv, lp.m, oracle_mod)


def test_plan_rejects_bad_structure(gpu):
    import torch
    from paper_2512_06715_amd import _lib
    from paper_2512_06715_amd.solver import MergeSpmv
    t = dict(device="cuda")
    rp = torch.tensor([0, 2, 1, 3], dtype=torch.int32, **t)      # decreasing
    ci = torch.tensor([0, 1, 2], dtype=torch.int32, **t)
    v = torch.ones(3, dtype=torch.float64, **t)
    with pytest.raises(_lib.PdhgError) as e:
        MergeSpmv(rp, ci, v, 4)
    assert e.value.code == -2  # PDHG_ERR_CSR
    rp = torch.tensor([0, 2, 3], dtype=torch.int32, **t)
    ci = torch.tensor([0, 9, 2], dtype=torch.int32, **t)         # column 9 of 4
    with pytest.raises(_lib.PdhgError) as e:
        MergeSpmv(rp, ci, v, 4)
    assert e.value.code == -2  # PDHG_ERR_CSR
    # a workspace below the plan's size
    lib = _lib.load()
    ci = torch.tensor([0, 1, 2], dtype=torch.int32, **t)
    op = MergeSpmv(rp, ci, v, 4)
    y = torch.empty(2, dtype=torch.float64, **t)
    x = torch.ones(4, dtype=torch.float64, **t)
    rc = lib.pdhg_spmv_merge_f64(2, 3, ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(ci.data_ptr()),
                                 ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(op.ws), 16, None)
    assert rc == -5  # PDHG_ERR_OOM


def test_timing_on_a_problem(gpu):
    """The handle's timing call runs both directions in the iteration precision."""
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc1000_t48")
    for prec in ("fp64", "mixed"):
        p = Problem(lp, precision=prec)
        t = p.time_spmv_merge(5)
        p.close()
        assert t["transpose"] > 0 and t["forward"] > 0, t
