"""The seeded UC generator: sizes, determinism, canonical CSR, feasibility."""
import numpy as np
import pytest

from paper_2512_06715_amd import ucgen


@pytest.mark.parametrize("name", ["uc14_t24", "uc1000_t48", "uc2000_t24"])
def test_sizes_match_formulas(name):
    N, G, L, T, dt, seed = ucgen.WORKLOADS[name]
    lp = ucgen.workload(name)
    f = ucgen.size_formulas(N, G, L, T)
    assert (lp.n, lp.m, lp.nnz) == (f["n"], f["m"], f["nnz"])
    assert int((lp.row_kind == 0).sum()) == f["m_eq"]


def test_paper_scale_sizes():
    """The 6717-bus, 96-period case: formula sizes (the build itself takes ~1 s)."""
    f = ucgen.size_formulas(6717, 1100, 9000, 96)
    assert f == dict(n=3220992, m=2034728, m_eq=1614432, nnz=7188260)


def test_deterministic_by_seed():
    a = ucgen.workload("uc14_t24")
    b = ucgen.workload("uc14_t24")
    for k in ("row_ptr", "col_idx", "val", "row_kind", "b", "c", "l", "u"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    c = ucgen.workload("uc14_t24", seed=99)
    assert not np.array_equal(a.b, c.b)


def test_canonical_csr():
    lp = ucgen.workload("uc1000_t48")
    rp, ci = lp.row_ptr, lp.col_idx
    assert rp[0] == 0 and rp[-1] == len(ci)
    assert np.all(np.diff(rp) >= 1)
    for i in range(0, lp.m, 997):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)
    assert ci.min() >= 0 and ci.max() < lp.n
    assert np.all(np.isfinite(lp.val)) and np.all(lp.l <= lp.u)


def test_all_slack_point_is_feasible():
    for seed in range(3):
        lp = ucgen.random_uc(30, 8, 40, 6, 1.0, seed=seed)
        x = ucgen.all_slack_point(lp)
        ax = ucgen.scipy_csr(lp) @ x
        eq = lp.row_kind == 0
        assert np.allclose(ax[eq], lp.b[eq], rtol=0, atol=1e-9)
        assert np.all(ax[~eq] >= lp.b[~eq] - 1e-9)
        assert np.all(x >= lp.l) and np.all(x <= lp.u)
        # with commitments fixed (a branch-and-bound node) the spill slack keeps
        # the LP feasible; the exact solver confirms it
        from oracle import exact
        fixed = ucgen.fix_commitments(lp, seed=[3, seed])
        st, *_ = exact.highs(fixed)
        assert st == exact.OPTIMAL


def test_long_rows_are_reserve_rows():
    lp = ucgen.workload("uc14_t24")
    lens = np.diff(lp.row_ptr)
    G, T = 5, 24
    assert sorted(lens)[-T:] == [2 * G + 1] * T
    assert lens[lp.meta["res_rows"]].tolist() == [2 * G + 1] * T
