"""Batched solves: grouped launches over instances with per-instance state."""
import numpy as np
import pytest

from paper_2512_06715_amd import ucgen

pytestmark = pytest.mark.gpu


def node_variants(lp, count, seed0):
    out = []
    for k in range(count):
        v = ucgen.fix_commitments(lp, seed=[seed0, k])
        out.append(v)
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_standalone(gpu, oracle_mod, precision):
    from paper_2512_06715_amd.solver import Problem, solve_batch
    base_a = ucgen.random_uc(14, 5, 20, 6, 1.0, seed=21)
    base_b = ucgen.random_uc(10, 4, 14, 4, 1.0, seed=24)
    nodes = node_variants(base_a, 5, 3)
    print("case batch", precision, flush=True)
    opts = dict(tol=1e-6, max_iter=300000, precision=precision)
    pa, pb = Problem(base_a, **opts), Problem(base_b, **opts)
    insts = [dict(base=0)] + [dict(base=0, fix_idx=v.meta["fix_idx"], fix_val=v.meta["fix_val"])
                              for v in nodes] + [dict(base=1), dict(base=1, b=base_b.b * 1.05)]
    res = solve_batch([pa, pb], insts)
    pa.close()
    pb.close()
    lps = [base_a] + nodes + [base_b, base_b.copy()]
    lps[-1].b = base_b.b * 1.05
    for k, (x, y, info) in enumerate(res):
        lp = lps[k]
        assert info["status"] == 1, (k, info)
        kk = oracle_mod.kkt(lp, x, y)
        assert kk["rel_kkt"] <= 1.001e-6, (k, kk)
        # the same instance as a standalone problem: identical partition and
        # reduction order, so the FP64 path reproduces it bit for bit
        p = Problem(lp, **opts)
        xs, ys, info_s = p.solve()
        p.close()
        assert info_s["attempts"] == info["attempts"], k
        if precision == "fp64":
            assert np.array_equal(xs, x) and np.array_equal(ys, y), k
        else:
            np.testing.assert_allclose(x, xs, rtol=0, atol=1e-9 * (1 + np.abs(xs).max()))


def test_batch_rejects_bad_instances(gpu):
    from paper_2512_06715_amd import _lib
    from paper_2512_06715_amd.solver import Problem, solve_batch
    base = ucgen.random_uc(6, 3, 8, 4, 1.0, seed=5)
    p = Problem(base)
    with pytest.raises(_lib.PdhgError):
        solve_batch([p], [dict(base=1)])
    with pytest.raises(_lib.PdhgError):
        solve_batch([p], [dict(base=0, fix_idx=np.array([base.n + 5]), fix_val=np.array([1.0]))])
    p.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("count", [3, 11])
def test_shared_matrix_batch_matches_standalone(gpu, oracle_mod, precision, count):
    """Node variants of one LP (one shared matrix): the attempt kernels number
    their blocks tile-major so the instances' blocks of a tile share L2; the
    arithmetic is the one-instance kernels', so every instance reproduces its
    standalone solve bit for bit in FP64, also as the active set shrinks."""
    from paper_2512_06715_amd.solver import Problem, solve_batch
    base = ucgen.random_uc(14, 5, 20, 6, 1.0, seed=21)
    nodes = node_variants(base, count - 1, 7)
    print("case shared-matrix batch", precision, count, flush=True)
    opts = dict(tol=1e-6, max_iter=300000, precision=precision)
    p = Problem(base, **opts)
    insts = [dict(base=0)] + [dict(base=0, fix_idx=v.meta["fix_idx"], fix_val=v.meta["fix_val"])
                              for v in nodes]
    res = solve_batch([p], insts)
    p.close()
    for k, (x, y, info) in enumerate(res):
        lp = ([base] + nodes)[k]
        assert info["status"] == 1, (k, info)
        assert oracle_mod.kkt(lp, x, y)["rel_kkt"] <= 1.001e-6
        q = Problem(lp, **opts)
        xs, ys, info_s = q.solve()
        q.close()
        assert info_s["attempts"] == info["attempts"], k
        if precision == "fp64":
            assert np.array_equal(xs, x) and np.array_equal(ys, y), k
        else:
            np.testing.assert_allclose(x, xs, rtol=0, atol=1e-9 * (1 + np.abs(xs).max()))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("long_seg", [0, 4])
def test_pack_kernels_bit_identical(gpu, oracle_mod, precision, long_seg):
    """Shared-matrix instances walked four per workgroup (the pack kernels,
    the tile's structure loaded once) give the bits of one instance per
    workgroup: same products, same CSR-order sums, same partials.  Six
    instances make a full and a partial pack; a long-row threshold of 4
    sends thousands of rows and columns to the per-instance long path."""
    from paper_2512_06715_amd.solver import Problem, solve_batch
    base = ucgen.random_uc(14, 5, 20, 12, 1.0, seed=23)
    nodes = node_variants(base, 5, 9)
    print("case pack kernels", precision, long_seg, flush=True)
    insts = [dict(base=0)] + [dict(base=0, fix_idx=v.meta["fix_idx"], fix_val=v.meta["fix_val"])
                              for v in nodes]
    out = {}
    for pack in (1, 0):
        p = Problem(base, tol=1e-4, max_iter=400000, precision=precision, long_seg=long_seg,
                    batch_pack=pack)
        out[pack] = solve_batch([p], insts)
        p.close()
    for k in range(len(insts)):
        (x1, y1, i1), (x0, y0, i0) = out[1][k], out[0][k]
        assert i1["status"] == i0["status"] == 1, (k, i1, i0)
        assert i1["attempts"] == i0["attempts"] and i1["restarts"] == i0["restarts"], k
        assert np.array_equal(x1, x0) and np.array_equal(y1, y0), k
        lp = ([base] + nodes)[k]
        assert oracle_mod.kkt(lp, x1, y1)["rel_kkt"] <= 1.001e-4


def test_uc4224_variants_batch(gpu, oracle_mod):
    """Branch-and-bound variants of the 4224-bus, 48-period LP (a random 0-20%
    of the commitments fixed), in mixed precision to relative KKT 1e-4 in one
    batch: every instance reaches the tolerance by the oracle's checker and
    matches its standalone solve."""
    from paper_2512_06715_amd.solver import Problem, solve_batch
    lp = ucgen.workload("uc4224_t48")
    variants = [ucgen.fix_commitments(lp, seed=100 + k) for k in range(5)]
    print("case uc4224 variants", flush=True)
    opts = dict(tol=1e-4, max_iter=2000000, precision="mixed")
    p = Problem(lp, **opts)
    insts = [dict(base=0, fix_idx=v.meta["fix_idx"], fix_val=v.meta["fix_val"]) for v in variants]
    res = solve_batch([p], insts)
    for k, (x, y, info) in enumerate(res):
        assert info["status"] == 1, (k, info)
        kk = oracle_mod.kkt(variants[k], x, y)
        assert kk["rel_kkt"] <= 1.001e-4, (k, kk)
        (xs, ys, info_s), = solve_batch([p], [insts[k]])
        print(k, "attempts", info["attempts"], "alone", info_s["attempts"], flush=True)
        assert info_s["attempts"] == info["attempts"], k
        np.testing.assert_allclose(x, xs, rtol=0, atol=1e-9 * (1 + np.abs(xs).max()))
        np.testing.assert_allclose(y, ys, rtol=0, atol=1e-9 * (1 + np.abs(ys).max()))
    p.close()
