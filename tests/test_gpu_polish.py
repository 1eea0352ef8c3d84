"""Feasibility polishing (pdhg_polish): two PDHG solves on the handle's
matrix, one for primal feasibility (c = 0, from x) and one for dual
feasibility (b = 0 and the finite bounds 0, from y), recombined.  Checked
against the oracle's PDHG on the same two LPs and, for its effect, by the
oracle's KKT checker and HiGHS's optimum."""
import json
import os

import numpy as np
import pytest

from paper_2512_06715_amd import ucgen

pytestmark = pytest.mark.gpu
REFS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lp_refs.json")))


def feasibility_lps(lp):
    """The two LPs the polish solves: c = 0; b = 0 with the finite bounds 0."""
    lpz = lp.copy()
    lpz.c = np.zeros(lp.n)
    lpd = lp.copy()
    lpd.b = np.zeros(lp.m)
    lpd.l = np.where(np.isfinite(lp.l), 0.0, lp.l)
    lpd.u = np.where(np.isfinite(lp.u), 0.0, lp.u)
    return lpz, lpd


@pytest.mark.parametrize("K,bound", [(16, 1e-11), (64, 1e-8)])
def test_polish_steps_match_oracle(gpu, oracle_mod, K, bound):
    """K attempts of each polishing solve from a fixed point, against the
    oracle's restarted PDHG on the same LPs from the same point: the primal
    step's x and the dual step's y entry by entry.  From a point this close
    to feasibility the step-size test divides tiny sums whose rounding
    depends on their order (a tree here, a loop in the oracle), so the
    trajectories part faster than a solve's: measured 7.4e-10 after 64."""
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc14_t24")
    print("case polish parity", flush=True)
    x, y, io = oracle_mod.pdhg(lp, tol=1e-4, max_iter=1000000)
    omega = io["omega"]
    lpz, lpd = feasibility_lps(lp)
    p = Problem(lp, tol=1e-4)
    xp, yp, info = p.polish(x, y, tol=1e-14, max_iter=K, omega=omega)
    p.close()
    assert info["attempts"] == 2 * K
    xo, _, i1 = oracle_mod.pdhg(lpz, tol=1e-14, max_iter=K, x0=x, omega0=omega, term=1,
                                infeas_every=0)
    _, yo, i2 = oracle_mod.pdhg(lpd, tol=1e-14, max_iter=K, y0=y, omega0=omega, term=2,
                                infeas_every=0)
    assert i1["attempts"] == i2["attempts"] == K
    for name, a, ref in (("x", xp, xo), ("y", yp, yo)):
        err = np.abs(a - ref) / (1 + np.abs(ref))
        j = int(np.argmax(err))
        print(name, "worst entry", err[j], flush=True)
        assert err[j] <= bound, (name, j, a[j], ref[j], err[j])


@pytest.mark.parametrize("name,precision", [("uc14_t24", "fp64"), ("uc1000_t48", "mixed")])
def test_polish_reduces_residuals(gpu, oracle_mod, name, precision):
    """From a solve at relative KKT 1e-5, polishing to a hundredth of the
    smaller of its relative primal and dual residuals lowers both at least
    100x (the oracle's checker on the returned point).  The polished pair
    then brackets the optimum (HiGHS): its dual objective below, its primal
    objective above up to its remaining infeasibility.  Fixing the primal
    residual can cost objective (here through penalty slacks), so the primal
    objective may move by more than the solve's tolerance; the bracket's
    width is reported."""
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload(name)
    ref = REFS[name]["objective"]
    print("case polish", name, precision, flush=True)
    p = Problem(lp, precision=precision, tol=1e-5, max_iter=5000000)
    x, y, info = p.solve()
    assert info["status"] == 1
    k0 = oracle_mod.kkt(lp, x, y)
    ptol = max(min(k0["rel_p"], k0["rel_d"]) / 100, 1e-12)
    xp, yp, pi = p.polish(x, y, tol=ptol, omega=info["omega"])
    p.close()
    k1 = oracle_mod.kkt(lp, xp, yp)
    print(f"before: rel_p {k0['rel_p']:.2e} rel_d {k0['rel_d']:.2e} gap {k0['rel_gap']:.2e} "
          f"obj {k0['pobj']:.10g}; polished to {ptol:.1e} in {pi['attempts']} attempts, "
          f"{pi['solve_s']:.2f}s: rel_p {k1['rel_p']:.2e} rel_d {k1['rel_d']:.2e} "
          f"gap {k1['rel_gap']:.2e} pobj {k1['pobj']:.10g} dobj {k1['dobj']:.10g}; "
          f"optimum {ref:.10g}", flush=True)
    assert k1["rel_p"] <= k0["rel_p"] / 100 and k1["rel_d"] <= k0["rel_d"] / 100
    assert abs(k1["rel_p"] - pi["rel_primal"]) <= 1e-6 * k1["rel_p"] + 1e-15
    assert k1["dobj"] <= ref * (1 + 1e-9) and pi["dual_bound"] <= ref
    assert k1["pobj"] >= ref * (1 - 1e-6)
