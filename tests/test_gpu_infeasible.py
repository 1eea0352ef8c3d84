"""Certificates of primal infeasibility on the GPU (status 5), checked with
the oracle's Farkas sum at the returned y."""
import numpy as np
import pytest

from oracle import exact
from paper_2512_06715_amd import ucgen

pytestmark = pytest.mark.gpu


def farkas_value(oracle_mod, lp, y):
    q = lp.copy()
    q.c = np.zeros(lp.n)
    lo, hi = oracle_mod.implied_bounds(lp)
    return oracle_mod.safe_bound(q, y, lo, hi, repair=False)["bound"]


def infeasible_node():
    """The 14-bus relaxation without its penalty slacks, every unit of period
    5 switched off (HiGHS: infeasible)."""
    lp = ucgen.workload("uc14_t24")
    N, G, L = 14, 5, 20
    pos = np.arange(lp.n) % (4 * G + 3 * N + L + 1)
    q = lp.copy()
    q.u[pos >= 4 * G + N + L] = 0.0
    q.l[lp.meta["u_cols"][5]] = q.u[lp.meta["u_cols"][5]] = 0.0
    return q


def test_closed_form_and_toys(gpu, oracle_mod):
    """x >= 1 with x in [0, 1/2], and 20 random toys HiGHS calls infeasible:
    status 5 and a positive Farkas value at the returned y."""
    from paper_2512_06715_amd.solver import Problem
    lps = [ucgen.dense_to_lp(np.array([[1.0]]), np.array([1], np.uint8), np.array([1.0]),
                             np.array([1.0]), np.array([0.0]), np.array([0.5]))]
    rng = np.random.default_rng(7)
    while len(lps) < 21:
        m, n = int(rng.integers(1, 4)), int(rng.integers(1, 4))
        lp = ucgen.dense_to_lp(*ucgen.random_toy_lp(rng, m, n))
        if exact.highs(lp)[0] == exact.INFEASIBLE:
            lps.append(lp)
    print("case infeasible toys", flush=True)
    for t, lp in enumerate(lps):
        p = Problem(lp, tol=1e-8, max_iter=50000)
        x, y, info = p.solve()
        p.close()
        assert info["status"] == 5, (t, info)
        assert farkas_value(oracle_mod, lp, y) > 0.0, t


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_infeasible_uc_node(gpu, oracle_mod, precision):
    from paper_2512_06715_amd.solver import Problem
    q = infeasible_node()
    print("case infeasible node", precision, flush=True)
    p = Problem(q, tol=1e-6, precision=precision, max_iter=100000)
    x, y, info = p.solve()
    p.close()
    xo, yo, io = oracle_mod.pdhg(q, tol=1e-6, max_iter=100000)
    print("gpu attempts", info["attempts"], "oracle", io["attempts"], flush=True)
    assert info["status"] == 5 and io["status"] == 5
    assert farkas_value(oracle_mod, q, y) > 0.0


def test_infeasible_node_in_a_batch(gpu, oracle_mod):
    """An infeasible child (slacks and period 5's units fixed to 0) next to
    feasible ones: each instance gets its own status, the feasible ones their
    tolerance.  Fixings keep the base's implied bounds (they only shrink the
    feasible set), which the certificate needs for the free bus angles."""
    from paper_2512_06715_amd.solver import Problem, solve_batch
    lp = ucgen.workload("uc14_t24")
    q = infeasible_node()
    fixed = np.nonzero((q.l == q.u) & (lp.l != lp.u))[0].astype(np.int32)
    print("case infeasible in batch", len(fixed), flush=True)
    p = Problem(lp, tol=1e-4, max_iter=400000)
    insts = [dict(base=0), dict(base=0, fix_idx=fixed, fix_val=q.l[fixed]),
             dict(base=0, fix_idx=lp.meta["u_cols"][3].astype(np.int32),
                  fix_val=np.ones(5))]
    res = solve_batch([p], insts)
    p.close()
    print("statuses", [r[2]["status"] for r in res], "attempts", [r[2]["attempts"] for r in res],
          flush=True)
    assert [r[2]["status"] for r in res] == [1, 5, 1]
    assert farkas_value(oracle_mod, q, res[1][1]) > 0.0
    assert oracle_mod.kkt(lp, res[0][0], res[0][1])["rel_kkt"] <= 1.001e-4


def test_no_test_when_disabled(gpu):
    """infeas_every = 0 never reports infeasibility (the solve runs to its
    attempt limit)."""
    from paper_2512_06715_amd.solver import Problem
    p = Problem(infeasible_node(), tol=1e-6, max_iter=4096, infeas_every=0)
    print("case infeasibility test off", flush=True)
    x, y, info = p.solve()
    p.close()
    assert info["status"] == 2 and info["attempts"] == 4096


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_unbounded_toys(gpu, oracle_mod, precision):
    """The four closed-form unbounded LPs and ten random toys HiGHS calls
    unbounded end with status 6, as in the oracle, and the returned x is a ray
    that passes the exact check.  In mixed precision the FP32 phase hands
    over (stall or overflow) and the FP64 phase certifies."""
    from paper_2512_06715_amd.solver import Problem
    from ray_check import is_ray, random_unbounded_toys, unbounded_toys
    lps = unbounded_toys() + random_unbounded_toys(10)
    for t, lp in enumerate(lps):
        print("case unbounded toy", precision, t, flush=True)
        p = Problem(lp, tol=1e-8, precision=precision, max_iter=200000)
        x, y, info = p.solve()
        p.close()
        xo, yo, io = oracle_mod.pdhg(lp, tol=1e-8, max_iter=200000)
        assert io["status"] == 6 and is_ray(lp, xo)
        assert info["status"] == 6, (t, info)
        assert is_ray(lp, x), (t, x)
        print("attempts", info["attempts"], "fp32", info["attempts_fp32"], "oracle", io["attempts"],
              flush=True)


def test_batch_bounded_and_unbounded(gpu):
    """One batch over one matrix: min -x1 with x1 = x2 and 0 <= x <= 10
    (optimum -10), and the same LP without upper bounds through a per-instance
    override: statuses 1 and 6, the second with a valid ray."""
    from paper_2512_06715_amd.solver import Problem, solve_batch
    from ray_check import is_ray, unbounded_toys
    lp = unbounded_toys()[0].copy()
    lp.u[:] = 10.0
    print("case batch bounded + unbounded", flush=True)
    p = Problem(lp, tol=1e-8, max_iter=200000)
    res = solve_batch([p], [dict(base=0), dict(base=0, u=np.array([np.inf, np.inf]))])
    p.close()
    assert res[0][2]["status"] == 1 and abs(res[0][2]["primal_obj"] + 10.0) <= 1e-6, res[0][2]
    assert res[1][2]["status"] == 6, res[1][2]
    q = lp.copy()
    q.u[:] = np.inf
    assert is_ray(q, res[1][0])


def test_ray_test_skip_follows_the_costs(gpu):
    """min x1 with x1 = x2 and x >= 0 has c'x bounded below on its box, so
    the ray test is skipped for it (optimum 0).  A cost override in a batch
    (c = (-1, 0)) and an update of c on the handle each make it unbounded,
    and each turns the test back on: status 6 with a valid ray.  With the
    tolerance at 0 the test never runs and the unbounded copy does not end
    with status 6."""
    from paper_2512_06715_amd.solver import Problem, solve_batch
    from ray_check import is_ray, unbounded_toys
    lp = unbounded_toys()[0].copy()
    lp.c = np.array([1.0, 0.0])
    neg = lp.copy()
    neg.c = np.array([-1.0, 0.0])
    print("case ray-test skip", flush=True)
    p = Problem(lp, tol=1e-8, max_iter=20000)
    x, y, info = p.solve()
    assert info["status"] == 1 and abs(info["primal_obj"]) <= 1e-6, info
    res = solve_batch([p], [dict(base=0), dict(base=0, c=neg.c)])
    assert res[0][2]["status"] == 1 and res[1][2]["status"] == 6, (res[0][2], res[1][2])
    assert is_ray(neg, res[1][0])
    p.update(c=neg.c)
    x, y, info = p.solve()
    p.close()
    assert info["status"] == 6 and is_ray(neg, x), info
    q = Problem(neg, tol=1e-8, max_iter=20000, dinf_tol=0.0)
    x, y, info = q.solve()
    q.close()
    assert info["status"] != 6, info


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_unbounded_with_long_rows(gpu, oracle_mod, precision):
    """Rows longer than one lane's share of the ray test, summed by the whole
    wave: min -x0 with x0 equal to the mean of x1..x199 (a 200-entry row) and
    a >= row over all 1000 columns, x >= 0.  Unbounded along d = 1 on
    x0..x199: status 6 with a valid ray, as in the oracle."""
    from paper_2512_06715_amd.solver import Problem
    from ray_check import is_ray
    n = 1000
    A = np.zeros((2, n))
    A[0, 0] = 1.0
    A[0, 1:200] = -1.0 / 199.0
    A[1, :] = 1.0
    c = np.zeros(n)
    c[0] = -1.0
    lp = ucgen.dense_to_lp(A, np.array([0, 1], np.uint8), np.array([0.0, 1.0]), c,
                           np.zeros(n), np.full(n, np.inf))
    print("case unbounded long rows", precision, flush=True)
    xo, yo, io = oracle_mod.pdhg(lp, tol=1e-8, max_iter=200000)
    assert io["status"] == 6 and is_ray(lp, xo)
    p = Problem(lp, tol=1e-8, precision=precision, max_iter=200000)
    x, y, info = p.solve()
    p.close()
    assert info["status"] == 6, info
    assert is_ray(lp, x)
    print("attempts", info["attempts"], "oracle", io["attempts"], flush=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_farkas_repair_toy(gpu, oracle_mod, precision):
    """An infeasible toy whose proof needs y_2 = 0 exactly (two single-entry
    columns of row 2 lack a lower bound): the Farkas test clamps y into the
    repair intervals for c = 0, ends with status 5 and returns that y, whose
    value is positive, as in the oracle."""
    from paper_2512_06715_amd.solver import Problem
    from test_oracle_pins import farkas_repair_toy
    lp = farkas_repair_toy()
    print("case farkas repair toy", precision, flush=True)
    xo, yo, io = oracle_mod.pdhg(lp, tol=1e-8, max_iter=100000)
    assert io["status"] == 5
    p = Problem(lp, tol=1e-8, precision=precision, max_iter=100000)
    x, y, info = p.solve()
    p.close()
    assert info["status"] == 5, info
    assert y[1] == 0.0 and farkas_value(oracle_mod, lp, y) > 0.0, y
