"""The node driver on the GPU: two levels of children of the 14-bus UC
relaxation, solved as warm-started batches, against HiGHS and the oracle."""
import numpy as np
import pytest

from oracle import exact
from paper_2512_06715_amd import ucgen

pytestmark = pytest.mark.gpu


def node_lp(lp, nd):
    q = lp.copy()
    q.l[nd.fix_idx] = nd.fix_val
    q.u[nd.fix_idx] = nd.fix_val
    return q


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_levels_of_nodes(gpu, oracle_mod, precision):
    """Root, its two children (most fractional commitment) and their four
    children: every node reaches its tolerance (oracle KKT), its safe bound
    is below its HiGHS optimum and within 1e-3 of it, children never beat
    their parent's optimum, and pruning against an incumbent drops only
    nodes whose optimum is above it."""
    from paper_2512_06715_amd import nodes as N
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc14_t24")
    ucols = lp.meta["u_cols"].ravel()
    print("case nodes", precision, flush=True)
    p = Problem(lp, tol=1e-5, precision=precision, max_iter=1000000)
    root = N.solve_nodes(p, [N.root()])[0]
    level1 = list(N.branch(root, int(N.most_fractional(root, ucols)[0])))
    N.solve_nodes(p, level1)
    level2 = [k for nd in level1 for k in N.branch(nd, int(N.most_fractional(nd, ucols)[0]))]
    N.solve_nodes(p, level2)
    p.close()
    opt = {}
    for nd in [root] + level1 + level2:
        st, xh, o, yh = exact.highs(node_lp(lp, nd))
        assert st == exact.OPTIMAL and nd.info["status"] == 1
        assert oracle_mod.kkt(node_lp(lp, nd), nd.x, nd.y)["rel_kkt"] <= 1.001e-5
        assert nd.bound <= o and o - nd.bound <= 1e-3 * (1 + abs(o)), (nd.fixed(), nd.bound, o)
        opt[id(nd)] = o
    for parent, kids in ((root, level1), (level1[0], level2[:2]), (level1[1], level2[2:])):
        for k in kids:
            assert opt[id(k)] >= opt[id(parent)] - 1e-9 * abs(opt[id(parent)])
    incumbent = float(np.median([opt[id(n)] for n in level2]))
    kept, cut = N.prune(level2, incumbent)
    assert all(opt[id(n)] > incumbent for n in cut)
    print("bounds", [round(n.bound, 3) for n in level2], "incumbent", incumbent,
          "pruned", len(cut), flush=True)


def test_batch_rejects_bad_weights(gpu):
    """omega0, eta0 must be finite and >= 0; the batch fails before any solve."""
    from paper_2512_06715_amd import _lib as L
    from paper_2512_06715_amd.solver import Problem, solve_batch
    p = Problem(ucgen.workload("uc14_t24"), tol=1e-3)
    print("case bad weights", flush=True)
    for bad in (dict(omega0=float("nan")), dict(eta0=-1.0), dict(omega0=float("inf")),
                dict(hold_omega=-1)):
        with pytest.raises(L.PdhgError):
            solve_batch([p], [dict(base=0, **bad)])
    x, y, info = solve_batch([p], [dict(base=0, omega0=3.0, eta0=0.5, hold_omega=200)])[0]
    p.close()
    assert info["status"] == 1


def test_nodes_on_a_device_resident_problem(gpu, oracle_mod):
    """The driver with the LP in device memory (fixings, warm starts and
    results as CUDA tensors): same statuses and bounds below HiGHS's optima."""
    import torch
    from paper_2512_06715_amd import nodes as N
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc14_t24")
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).cuda()

    class DevLP:
        m, n = lp.m, lp.n
        row_ptr = dev(lp.row_ptr, torch.int32)
        col_idx = dev(lp.col_idx, torch.int32)
        val = dev(lp.val, torch.float64)
        row_kind = dev(lp.row_kind, torch.uint8)
        b, c, l, u = (dev(a, torch.float64) for a in (lp.b, lp.c, lp.l, lp.u))
    print("case device-resident nodes", flush=True)
    p = Problem(DevLP, device=True, tol=1e-4, max_iter=400000)
    root = N.solve_nodes(p, [N.root()])[0]
    j = int(N.most_fractional(root, lp.meta["u_cols"].ravel())[0])
    kids = N.solve_nodes(p, list(N.branch(root, j)))
    p.close()
    for nd in [root] + kids:
        assert isinstance(nd.x, torch.Tensor) and nd.info["status"] == 1
        st, xh, opt, yh = exact.highs(node_lp(lp, nd))
        assert nd.bound <= opt
        x, y = nd.x.cpu().numpy(), nd.y.cpu().numpy()
        assert oracle_mod.kkt(node_lp(lp, nd), x, y)["rel_kkt"] <= 1.001e-4


def test_children_of_the_4224_bus_root(gpu, oracle_mod):
    """At the size of the batched workload: the 4224-bus, 48-period root in
    mixed precision, then the children of its two most fractional commitments
    (four nodes) as one warm-started batch on an FP64 handle.  Every child
    reaches 1e-4 by the oracle's checker, keeps its fixing, has a finite
    bound below its objective, and no child's objective lies far below the
    root's bound."""
    from paper_2512_06715_amd import nodes as N
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc4224_t48")
    ucols = lp.meta["u_cols"].ravel()
    print("case nodes uc4224", flush=True)
    p = Problem(lp, tol=1e-4, precision="mixed", max_iter=2000000)
    root = N.solve_nodes(p, [N.root()])[0]
    p.close()
    assert root.info["status"] == 1 and np.isfinite(root.bound)
    kids = [k for j in N.most_fractional(root, ucols, k=2) for k in N.branch(root, int(j))]
    q = Problem(lp, tol=1e-4, precision="fp64", max_iter=2000000)
    N.solve_nodes(q, kids, warm=True, weights=True)
    q.close()
    for k in kids:
        assert k.info["status"] == 1, k.info
        kk = oracle_mod.kkt(node_lp(lp, k), k.x, k.y)
        assert kk["rel_kkt"] <= 1.001e-4, kk
        assert np.array_equal(k.x[k.fix_idx], k.fix_val)
        assert np.isfinite(k.bound) and k.bound <= k.objective
        # a child's optimum is at least the root's; its reported objective,
        # within the tolerance of its own, cannot fall far below the root's bound
        assert k.objective >= root.bound - 2e-3 * abs(root.bound)
        print("child", k.fixed(), k.info["attempts"], k.objective, k.bound, flush=True)
