"""Host logic of the node driver (no GPU): children's fixings, warm starts,
the choice of the branching column and pruning by the safe bound."""
import numpy as np
import pytest

from paper_2512_06715_amd import nodes as N


def solved(fix_idx, fix_val, x, bound=0.0, obj=1.0):
    nd = N.Node(np.asarray(fix_idx, np.int32), np.asarray(fix_val, np.float64))
    nd.x, nd.y = np.asarray(x, float), np.zeros(2)
    nd.info = dict(dual_bound=bound, primal_obj=obj, omega=12.5, eta=0.75, attempts=640)
    return nd


def test_branch_adds_one_fixing_and_warm_starts_from_parent():
    p = solved([4], [1.0], [0.0, 0.3, 0.5, 0.9, 1.0])
    a, b = N.branch(p, 2)
    assert a.fixed() == {4: 1.0, 2: 0.0} and b.fixed() == {4: 1.0, 2: 1.0}
    assert a.depth == b.depth == 1
    assert a.x0 is p.x and b.y0 is p.y and not a.solved
    assert a.omega0 == b.omega0 == 12.5 and a.eta0 == b.eta0 == 0.75 and a.hold == b.hold == 640
    with pytest.raises(ValueError):
        N.branch(p, 4)                      # already fixed here
    with pytest.raises(ValueError):
        N.branch(N.root(), 0)               # unsolved parent


def test_most_fractional_skips_fixed_and_breaks_ties_by_index():
    p = solved([2], [1.0], [0.0, 0.45, 0.5, 0.55, 0.9, 0.5])
    assert N.most_fractional(p, [0, 1, 2, 3, 4, 5], k=1).tolist() == [5]
    assert N.most_fractional(p, [0, 1, 2, 3, 4, 5], k=3).tolist() == [5, 1, 3]
    assert N.most_fractional(p, [0, 4], k=5).tolist() == [4, 0]


def test_prune_uses_the_bound_strictly():
    ns = [solved([], [], [0.0], bound=b) for b in (1.0, 2.0, 3.0, -np.inf)]
    kept, cut = N.prune(ns, 2.0)
    assert [n.bound for n in kept] == [1.0, 2.0, -np.inf]
    assert [n.bound for n in cut] == [3.0]
    assert N.root().bound == -np.inf


def test_prune_drops_nodes_proved_infeasible():
    """A Farkas certificate (status 5) empties the subtree whatever the
    computed bound; an unbounded relaxation (status 6) keeps its -inf."""
    inf = solved([], [], [0.0], bound=-np.inf)
    inf.info["status"] = 5
    unb = solved([], [], [0.0], bound=-np.inf)
    unb.info["status"] = 6
    ok = solved([], [], [0.0], bound=1.0)
    ok.info["status"] = 1
    kept, cut = N.prune([inf, unb, ok], 1e30)
    assert [id(n) for n in cut] == [id(inf)] and [id(n) for n in kept] == [id(unb), id(ok)]
    assert inf.bound == np.inf and unb.bound == -np.inf and ok.bound == 1.0
