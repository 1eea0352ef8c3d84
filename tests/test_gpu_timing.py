"""Timing entry points on handles in any state."""
import pytest

from paper_2512_06715_amd import ucgen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_time_kernels_before_any_solve(gpu, precision):
    """Setup leaves the iterate part of the control state unset; the timing
    call starts from the zero point itself, then a solve and a second timing
    still agree with the oracle-checked path."""
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc14_t24")
    print("case time_kernels fresh", precision, flush=True)
    p = Problem(lp, precision=precision, tol=1e-4, max_iter=400000)
    t = p.time_kernels(5)
    assert all(v > 0 for v in t.values()), t
    x, y, info = p.solve()
    assert info["status"] == 1
    t2 = p.time_kernels(5)
    assert all(v > 0 for v in t2.values()), t2
    p.close()
