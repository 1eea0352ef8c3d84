"""The no-allocation batched solve (pdhg_solve_batch_static, for callers that
cannot allocate) against the workspace batched solve (pdhg_solve_batch): the
same instances give the same results, on two calls in a row, the second with
a smaller batch, and sizes beyond the fixed scratch are rejected."""
import numpy as np
import pytest

from paper_2512_06715_amd import ucgen

pytestmark = pytest.mark.gpu


def node(lp, base, seed):
    v = ucgen.fix_commitments(lp, seed=seed, frac=0.1)
    return dict(base=base, fix_idx=v.meta["fix_idx"], fix_val=v.meta["fix_val"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_static_batch_matches_workspace_batch(gpu, oracle_mod, precision):
    from paper_2512_06715_amd.solver import Problem, solve_batch
    print("case no-allocation batch", precision, flush=True)
    a = ucgen.workload("uc14_t24")
    b = ucgen.random_uc(10, 4, 14, 12, 1.0, seed=21)
    probs = [Problem(a, tol=1e-4, precision=precision, max_iter=400000),
             Problem(b, tol=1e-4, precision=precision, max_iter=400000)]
    first = [node(a, 0, 500), node(b, 1, 601), node(a, 0, 502), node(b, 1, 603)]
    second = [first[2], dict(base=1)]
    for batch in (first, second):
        ref = solve_batch(probs, batch)
        got = solve_batch(probs, batch, static=True)
        for k, ((xr, yr, ir), (xg, yg, ig)) in enumerate(zip(ref, got)):
            assert ig["status"] == ir["status"] == 1, (k, ig, ir)
            assert ig["attempts"] == ir["attempts"], k
            assert np.array_equal(xg, xr) and np.array_equal(yg, yr), k
            assert ig["primal_obj"] == ir["primal_obj"] and ig["dual_bound"] == ir["dual_bound"]
            base = a if batch[k]["base"] == 0 else b
            lp = base.copy()
            if "fix_idx" in batch[k]:
                lp.l[batch[k]["fix_idx"]] = batch[k]["fix_val"]
                lp.u[batch[k]["fix_idx"]] = batch[k]["fix_val"]
            kk = oracle_mod.kkt(lp, xg, yg)
            assert kk["rel_kkt"] <= 1.001e-4, (k, kk)
    for p in probs:
        p.close()


def test_static_batch_rejects_sizes_beyond_its_scratch(gpu):
    from paper_2512_06715_amd import _lib
    from paper_2512_06715_amd.solver import Problem, solve_batch
    print("case no-allocation limits", flush=True)
    small = Problem(ucgen.workload("uc14_t24"), tol=1e-4)
    with pytest.raises(_lib.PdhgError) as e:
        solve_batch([small], [dict(base=0)] * 65, static=True)
    assert e.value.code == -5
    big = Problem(ucgen.workload("uc1000_t48"), tol=1e-4)
    with pytest.raises(_lib.PdhgError) as e:
        solve_batch([big], [dict(base=0)] * 4, static=True)
    assert e.value.code == -5
    # the array still serves a batch that fits
    (x, y, info), = solve_batch([small], [dict(base=0)], static=True)
    assert info["status"] == 1
    small.close()
    big.close()
