"""The weak-duality bound each solve reports, the implied bounds it uses, and
warm-started batches of branch-and-bound nodes."""
import numpy as np
import pytest

from oracle import exact
from paper_2512_06715_amd import ucgen

pytestmark = pytest.mark.gpu


def lps():
    from edge_lps import cancelling_row
    from test_gpu_parity import dense_column_lp
    return {"uc14_t24": ucgen.workload("uc14_t24"), "dense_cols": dense_column_lp(),
            "uc1000_t48": ucgen.workload("uc1000_t48"), "cancelling_row": cancelling_row()}


@pytest.mark.parametrize("name", ["uc14_t24", "dense_cols", "uc1000_t48", "cancelling_row"])
def test_implied_bounds_match_oracle(gpu, oracle_mod, name):
    from paper_2512_06715_amd.solver import Problem, implied_bounds
    lp = lps()[name]
    print("case implied bounds", name, flush=True)
    p = Problem(lp)
    lo, hi = implied_bounds(p)
    p.close()
    olo, ohi = oracle_mod.implied_bounds(lp)
    assert np.array_equal(lo.view(np.uint64), olo.view(np.uint64))
    assert np.array_equal(hi.view(np.uint64), ohi.view(np.uint64))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_dual_bound_with_cancelling_row(gpu, oracle_mod, precision):
    """The implied bound of x3 admits every feasible point although its row
    sum cancels, so the reported bound stays below the optimum -7e-3 (closed
    form) at any accuracy."""
    from paper_2512_06715_amd.solver import Problem, implied_bounds
    lp = lps()["cancelling_row"]
    print("case cancelling row", precision, flush=True)
    for iters in (1, 64, 100000):
        p = Problem(lp, tol=1e-6, precision=precision, max_iter=iters)
        x, y, info = p.solve()
        lo, hi = implied_bounds(p)
        p.close()
        assert lo[2] <= -7e-3
        assert info["dual_bound"] <= -7e-3, (iters, info)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["uc14_t24", "dense_cols"])
def test_dual_bound_valid_and_tight(gpu, oracle_mod, name, precision):
    """The reported bound never exceeds the optimum (HiGHS), equals the
    oracle's bound evaluated at the returned y up to the two rounding
    allowances, and is close to the optimum once the solve is accurate."""
    from paper_2512_06715_amd.solver import Problem
    lp = lps()[name]
    print("case dual bound", name, precision, flush=True)
    st, xh, opt, yh = exact.highs(lp)
    for tol in (1e-3, 1e-5):
        p = Problem(lp, tol=tol, precision=precision, max_iter=1000000)
        x, y, info = p.solve()
        p.close()
        assert info["status"] == 1
        db = info["dual_bound"]
        assert db <= opt, (tol, db, opt)
        ref = oracle_mod.safe_bound(lp, y)
        if np.isfinite(ref["bound"]):
            slack = ref["allowance"] * 4 + 1e-12 * abs(ref["value"])
            assert abs(db - ref["bound"]) <= slack, (db, ref)
        else:
            assert db == -np.inf
        if tol == 1e-5:
            assert np.isfinite(db) and opt - db <= 1e-3 * (1 + abs(opt)), (db, opt)
            print("bound gap at 1e-5:", (opt - db) / abs(opt), flush=True)


def test_warm_started_nodes_keep_valid_bounds(gpu, oracle_mod):
    """Children of a node (one commitment fixed to 0 and to 1) solved as one
    batch, warm-started from the parent's solution: every child's bound is
    below its own optimum, and warm starts do not cost more attempts than cold
    starts in total."""
    from paper_2512_06715_amd.solver import Problem, solve_batch
    lp = ucgen.workload("uc14_t24")
    print("case warm nodes", flush=True)
    p = Problem(lp, tol=1e-5, max_iter=400000)
    x, y, info = p.solve()
    ucols = lp.meta["u_cols"].ravel()
    frac = np.abs(x[ucols] - 0.5)
    picks = ucols[np.argsort(frac)[:3]]
    kids, lpk = [], []
    for j in picks:
        for v in (0.0, 1.0):
            kids.append(dict(base=0, fix_idx=np.array([j], np.int32), fix_val=np.array([v])))
            q = lp.copy()
            q.l[j] = q.u[j] = v
            lpk.append(q)
    warm = solve_batch([p], [dict(k, x0=x, y0=y) for k in kids])
    cold = solve_batch([p], kids)
    p.close()
    for k, (xk, yk, ik) in enumerate(warm):
        st, xh, opt, yh = exact.highs(lpk[k])
        assert ik["status"] == 1 and cold[k][2]["status"] == 1
        assert ik["dual_bound"] <= opt and cold[k][2]["dual_bound"] <= opt, k
        assert oracle_mod.kkt(lpk[k], xk, yk)["rel_kkt"] <= 1.001e-5
    assert sum(w[2]["attempts"] for w in warm) <= sum(c[2]["attempts"] for c in cold)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_dual_bound_finite_at_scale(gpu, oracle_mod, precision):
    """The 1000-bus, 48-period UC relaxation at tolerance 1e-4: its penalty
    slacks (single-entry columns without an upper bound) would make the plain
    bound -inf at an approximate y; with the repair the bound is finite, below
    the reference optimum, within 1e-3 of it, and equal to the oracle's bound
    at the returned y within the allowances."""
    import json
    import os
    from paper_2512_06715_amd.solver import Problem
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lp_refs.json")))
    opt = ref["uc1000_t48"]["objective"]
    lp = ucgen.workload("uc1000_t48")
    print("case bound at scale", precision, flush=True)
    p = Problem(lp, tol=1e-4, precision=precision)
    x, y, info = p.solve()
    p.close()
    assert info["status"] == 1
    db = info["dual_bound"]
    r = oracle_mod.safe_bound(lp, y)
    plain = oracle_mod.safe_bound(lp, y, repair=False)
    print("bound", db, "oracle", r["bound"], "repaired rows", r["repaired_rows"],
          "plain", plain["bound"], "gap", (opt - db) / abs(opt), flush=True)
    assert np.isfinite(db) and db <= opt + 1e-9 * abs(opt)
    assert (opt - db) <= 1e-3 * abs(opt)
    assert abs(db - r["bound"]) <= 4 * r["allowance"] + 1e-12 * abs(r["value"])
