"""The seeded workloads at their stated accuracy, against references the
oracle package computed (tests/golden/lp_refs.json: HiGHS optima written by
tests/golden/make_refs.py)."""
import json
import os

import numpy as np
import pytest

from paper_2512_06715_amd import ucgen

pytestmark = pytest.mark.gpu
REFS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lp_refs.json")))


def test_uc1000_fp64_to_1e6(gpu, oracle_mod):
    """The mid-size LP (1000 buses, 200 units, 1400 lines, 48 periods) in
    plain FP64 to relative KKT 1e-6: the oracle's checker confirms the KKT
    error and the objective is within 1e-6 of HiGHS's optimum (measured
    5.7e-7 after 2.4M attempts)."""
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc1000_t48")
    ref = REFS["uc1000_t48"]["objective"]
    print("case uc1000 fp64 1e-6", flush=True)
    p = Problem(lp, precision="fp64", tol=1e-6, max_iter=4000000)
    x, y, info = p.solve()
    p.close()
    assert info["status"] == 1, info
    k = oracle_mod.kkt(lp, x, y)
    err = abs(k["pobj"] - ref) / abs(ref)
    print("attempts", info["attempts"], "kkt", k["rel_kkt"], "objective error", err, flush=True)
    assert k["rel_kkt"] <= 1.001e-6, k
    assert err <= 1e-6
    assert info["dual_bound"] <= ref
