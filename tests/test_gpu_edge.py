"""Degenerate shapes on the GPU against the oracle and HiGHS: a 1x1 LP, an
empty row and empty columns, every variable fixed, no nonzero at all,
duplicated rows, a free column with no entries."""
import numpy as np
import pytest

from edge_lps import CASES
from oracle import exact

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", list(CASES))
def test_edge_setup_and_first_attempt(gpu, oracle_mod, name):
    """Preprocessing bit for bit, and one attempt within 1e-12 of the oracle's."""
    from paper_2512_06715_amd.solver import Problem
    lp = CASES[name]()
    print("case edge setup", name, flush=True)
    p = Problem(lp, max_iter=1, tol=1e-12, use_graph=0)
    g = p.export_setup()
    x, y, info = p.solve()
    p.close()
    assert np.array_equal(g["var_kind"], oracle_mod.var_kind(lp.l, lp.u))
    vs, Dr, Dc = oracle_mod.scale(lp, 10, True)
    assert np.array_equal(g["val_s"].view(np.uint64), vs.view(np.uint64))
    assert np.array_equal(g["Dr"].view(np.uint64), Dr.view(np.uint64))
    assert np.array_equal(g["Dc"].view(np.uint64), Dc.view(np.uint64))
    cp, ri, vt = oracle_mod.transpose(lp.m, lp.n, lp.row_ptr, lp.col_idx, vs)
    assert np.array_equal(g["colptr"], cp) and np.array_equal(g["rowidx"], ri)
    xo, yo, io = oracle_mod.pdhg(lp, tol=1e-12, max_iter=1)
    assert info["attempts"] == io["attempts"] and info["accepted"] == io["accepted"]
    np.testing.assert_allclose(x, xo, rtol=1e-12, atol=1e-12 * (1 + np.abs(xo).max()))
    np.testing.assert_allclose(y, yo, rtol=1e-12, atol=1e-12 * (1 + np.abs(yo).max()))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-7), ("mixed", 1e-4)])
@pytest.mark.parametrize("name", list(CASES))
def test_edge_solve(gpu, oracle_mod, name, precision, tol):
    """The solve reaches its tolerance (the oracle's KKT checker), the
    objective matches HiGHS within the tolerance, and the safe bound is below
    the optimum."""
    from paper_2512_06715_amd.solver import Problem
    lp = CASES[name]()
    print("case edge solve", name, precision, flush=True)
    st, xh, opt, yh = exact.highs(lp)
    p = Problem(lp, tol=tol, precision=precision, max_iter=200000)
    x, y, info = p.solve()
    p.close()
    assert info["status"] == 1, info
    k = oracle_mod.kkt(lp, x, y)
    assert k["rel_kkt"] <= 1.001 * tol
    assert abs(k["pobj"] - opt) <= 10 * tol * (1 + abs(opt))
    assert info["dual_bound"] <= opt + 1e-12 * (1 + abs(opt))
