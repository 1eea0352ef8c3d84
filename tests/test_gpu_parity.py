"""GPU path against the FP64 oracle (calls go through the C ABI)."""
import numpy as np
import pytest

from paper_2512_06715_amd import ucgen

pytestmark = pytest.mark.gpu


def dense_column_lp(seed=7, m=300, n=120):
    """Random LP with one dense row and two dense columns (long-segment paths)."""
    rng = np.random.default_rng(seed)
    A = np.where(rng.random((m, n)) < 0.03, rng.standard_normal((m, n)), 0.0)
    A[5, :] = rng.standard_normal(n)          # dense row (> 64 entries)
    A[:, 3] = rng.standard_normal(m)          # dense columns
    A[:, 77] = rng.uniform(0.5, 2.0, m)
    x0 = rng.random(n)
    kind = (rng.random(m) < 0.5).astype(np.uint8)
    b = A @ x0 - kind * rng.random(m)
    c = rng.standard_normal(n)
    lo = np.zeros(n)
    hi = np.full(n, 2.0)
    hi[::7] = np.inf
    lo[::11] = -np.inf
    hi[::11] = np.inf
    return ucgen.dense_to_lp(A, kind, b, c, lo, hi)


def wide_tile_lp(seed=3, m=500, n=70000):
    """Sparse LP whose row tiles each join columns near 0 with columns near n
    (an index span above 65535 inside one 256-row tile)."""
    rng = np.random.default_rng(seed)
    rp, ci, vv = [0], [], []
    for i in range(m):
        cols = sorted({(i * 131) % n, (i * 131 + 7) % n, n - 1 - i})
        ci += cols
        vv += list(rng.uniform(0.5, 2.0, len(cols)))
        rp.append(len(ci))
    lp = ucgen.UCLP(m, n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(vv),
                    (rng.random(m) < 0.5).astype(np.uint8), np.zeros(m), rng.standard_normal(n),
                    np.zeros(n), np.ones(n), {})
    x0 = rng.random(n)
    lp.b = ucgen.scipy_csr(lp) @ x0 - lp.row_kind * rng.random(m)
    return lp


CASES = {
    "uc14_t24": lambda: ucgen.workload("uc14_t24"),
    "uc1000_t48": lambda: ucgen.workload("uc1000_t48"),
    "dense_cols": dense_column_lp,
}


@pytest.mark.parametrize("reorder", [1, 0])
@pytest.mark.parametrize("name", list(CASES))
def test_setup_bit_exact(gpu, oracle_mod, name, reorder):
    """The preprocessed problem, read back in the caller's order, is the
    oracle's bit for bit, whether or not the solver relabels it internally."""
    from paper_2512_06715_amd.solver import Problem
    lp = CASES[name]()
    print("case", name, "reorder", reorder, ucgen.describe(lp), flush=True)
    p = Problem(lp, reorder=reorder)
    g = p.export_setup()
    p.close()
    vk = oracle_mod.var_kind(lp.l, lp.u)
    assert np.array_equal(g["var_kind"], vk)
    vs, Dr, Dc = oracle_mod.scale(lp, 10, True)
    assert np.array_equal(g["val_s"].view(np.uint64), vs.view(np.uint64))
    assert np.array_equal(g["Dr"].view(np.uint64), Dr.view(np.uint64))
    assert np.array_equal(g["Dc"].view(np.uint64), Dc.view(np.uint64))
    cp, ri, vt = oracle_mod.transpose(lp.m, lp.n, lp.row_ptr, lp.col_idx, vs)
    assert np.array_equal(g["colptr"], cp)
    assert np.array_equal(g["rowidx"], ri)
    assert np.array_equal(g["valT"].view(np.uint64), vt.view(np.uint64))


@pytest.mark.parametrize("reorder", [1, 0])
@pytest.mark.parametrize("name", list(CASES))
def test_fp32_casts_bit_exact(gpu, oracle_mod, name, reorder):
    """The FP32 data of the mixed path are the round-to-nearest casts of the
    oracle's scaled FP64 values (numpy's float32 conversion), bit for bit, in
    the caller's order, for A, its transpose and b, c, l, u."""
    from paper_2512_06715_amd.solver import Problem
    lp = CASES[name]()
    print("case fp32 casts", name, reorder, flush=True)
    p = Problem(lp, precision="mixed", reorder=reorder)
    g = p.export_fp32()
    p.close()
    vs, Dr, Dc = oracle_mod.scale(lp, 10, True)
    cp, ri, vt = oracle_mod.transpose(lp.m, lp.n, lp.row_ptr, lp.col_idx, vs)
    f32 = lambda a: np.asarray(a, np.float64).astype(np.float32).view(np.uint32)
    assert np.array_equal(g["val_s"].view(np.uint32), f32(vs))
    assert np.array_equal(g["valT"].view(np.uint32), f32(vt))
    assert np.array_equal(g["b"].view(np.uint32), f32(Dr * lp.b))
    assert np.array_equal(g["c"].view(np.uint32), f32(Dc * lp.c))
    assert np.array_equal(g["l"].view(np.uint32), f32(lp.l / Dc))
    assert np.array_equal(g["u"].view(np.uint32), f32(lp.u / Dc))


@pytest.mark.parametrize("reorder", [1, 0])
@pytest.mark.parametrize("name", ["uc14_t24", "dense_cols"])
def test_one_attempt(gpu, oracle_mod, name, reorder):
    from paper_2512_06715_amd.solver import Problem
    lp = CASES[name]()
    print("case", name, "reorder", reorder, flush=True)
    p = Problem(lp, max_iter=1, tol=1e-12, use_graph=0, reorder=reorder)
    x, y, info = p.solve()
    p.close()
    xo, yo, io = oracle_mod.pdhg(lp, tol=1e-12, max_iter=1)
    assert info["attempts"] == 1 and io["attempts"] == 1
    assert info["accepted"] == io["accepted"]
    np.testing.assert_allclose(x, xo, rtol=1e-12, atol=1e-12 * (1 + np.abs(xo).max()))
    np.testing.assert_allclose(y, yo, rtol=1e-12, atol=1e-12 * (1 + np.abs(yo).max()))


# The adaptive-step iteration amplifies rounding differences (about tenfold
# per 40 attempts on these instances, the same under a 1e-15 perturbation of c
# in the oracle alone), so trajectories are compared over short horizons only;
# longer solves are compared by objective and KKT error.  Every entry is
# compared: |x_j - xo_j| <= bound (1 + |xo_j|), the same for y.  Measured
# worst entries: 1.7e-12 (uc14_t24, 64 attempts), 8.0e-12 (128), 1.2e-11
# (dense_cols, 64), 1.7e-7 (128, after a restart).
def assert_entrywise(a, ref, bound, what):
    err = np.abs(a - ref) / (1 + np.abs(ref))
    j = int(np.argmax(err))
    assert err[j] <= bound, (what, j, a[j], ref[j], err[j])


@pytest.mark.parametrize("name,iters,bound", [("uc14_t24", 64, 1e-10), ("uc14_t24", 128, 1e-9),
                                              ("dense_cols", 64, 1e-9), ("dense_cols", 128, 2e-6)])
def test_short_trajectory(gpu, oracle_mod, name, iters, bound):
    from paper_2512_06715_amd.solver import Problem
    lp = CASES[name]()
    print("case", name, iters, flush=True)
    p = Problem(lp, max_iter=iters, tol=1e-12)
    x, y, info = p.solve()
    p.close()
    xo, yo, io = oracle_mod.pdhg(lp, tol=1e-12, max_iter=iters)
    assert info["attempts"] == io["attempts"]
    assert info["restarts"] == io["restarts"]
    assert info["accepted"] == io["accepted"]
    assert_entrywise(x, xo, bound, "x")
    assert_entrywise(y, yo, bound, "y")
    k = oracle_mod.kkt(lp, x, y)
    assert abs(k["rel_kkt"] - info["rel_kkt"]) <= 1e-9 * max(1.0, k["rel_kkt"])


@pytest.mark.parametrize("part", [dict(spmv_direct=1), dict(long_seg=8), dict(tiles_per_block=3),
                                  dict(spmv_direct=1, long_seg=4, tiles_per_block=2)])
def test_partitions_agree(gpu, oracle_mod, part):
    """Every SpMV partition computes the same attempt (up to rounding) and
    solves to the same optimum."""
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.random_uc(14, 5, 20, 24, 1.0, seed=11)
    print("case partition", part, flush=True)
    p = Problem(lp, max_iter=1, tol=1e-12, use_graph=0, **part)
    x, y, info = p.solve()
    got = p.partition()
    p.close()
    for k, v in part.items():
        key = {"spmv_direct": "direct", "tiles_per_block": "tiles_per_block"}.get(k, k)
        assert got[key] == v
    xo, yo, io = oracle_mod.pdhg(lp, tol=1e-12, max_iter=1)
    np.testing.assert_allclose(x, xo, rtol=1e-12, atol=1e-12 * (1 + np.abs(xo).max()))
    np.testing.assert_allclose(y, yo, rtol=1e-12, atol=1e-12 * (1 + np.abs(yo).max()))
    p = Problem(lp, tol=1e-7, max_iter=400000, **part)
    x, y, info = p.solve()
    p.close()
    assert info["status"] == 1
    from oracle import exact
    _, _, ref, _ = exact.highs(lp)
    assert abs(info["primal_obj"] - ref) <= 1e-6 * abs(ref)


def test_autotune_picks_a_candidate(gpu, oracle_mod):
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc1000_t48")
    print("case autotune", flush=True)
    p = Problem(lp, autotune=1, tol=1e-4, precision="mixed")
    part = p.partition()
    assert part["tiles_per_block"] in (1, 2, 4)
    assert part["direct"] in (0, 1) and part["long_seg"] in (32, 64, 256)
    x, y, info = p.solve()
    p.close()
    assert info["status"] == 1
    assert oracle_mod.kkt(lp, x, y)["rel_kkt"] <= 1.001e-4
    print("autotuned partition", part, flush=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reorder_same_solution(gpu, oracle_mod, precision):
    """The internal relabelling changes rounding order only: both orders solve
    to the same optimum."""
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc1000_t48")
    print("case reorder", precision, flush=True)
    tol = 1e-4
    res = {}
    for r in (0, 1):
        p = Problem(lp, reorder=r, tol=tol, precision=precision)
        res[r] = p.solve()
        p.close()
        assert res[r][2]["status"] == 1
        k = oracle_mod.kkt(lp, res[r][0], res[r][1])
        assert k["rel_kkt"] <= tol * 1.001
    o0, o1 = res[0][2]["primal_obj"], res[1][2]["primal_obj"]
    assert abs(o0 - o1) <= 2 * tol * (1 + abs(o0))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_warm_start_in_callers_order(gpu, oracle_mod, precision):
    """Warm starts and results are in the caller's order: a solve started at
    an exact optimal vertex (HiGHS, KKT error ~1e-14) stops at the first
    evaluation, in either precision and with the internal relabelling on."""
    from oracle import exact
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc14_t24")
    print("case warm start", precision, flush=True)
    st, xo, _, yo = exact.highs(lp)
    assert st == exact.OPTIMAL and oracle_mod.kkt(lp, xo, yo)["rel_kkt"] < 1e-10
    p = Problem(lp, reorder=1, tol=1e-5, precision=precision)
    x, y, info = p.solve(x0=xo, y0=yo)
    p.close()
    assert info["status"] == 1 and info["attempts"] == 0
    assert np.abs(x - xo).max() <= 1e-6 * (1 + np.abs(xo).max())
    assert np.abs(y - yo).max() <= 1e-6 * (1 + np.abs(yo).max())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("part", [dict(), dict(spmv_direct=1), dict(long_seg=8, tiles_per_block=3)])
@pytest.mark.parametrize("name", ["uc14_t24", "dense_cols", "uc1000_t48"])
def test_compact_index_bit_identical(gpu, name, part, precision):
    """The 16-bit tile-relative structure changes only how indices are read:
    300 attempts (evaluations and restarts included) give bit-identical
    iterates with and without it."""
    from paper_2512_06715_amd.solver import Problem
    lp = CASES[name]()
    print("case compact", name, part, precision, flush=True)
    res = []
    for ci in (1, 0):
        p = Problem(lp, max_iter=300, tol=1e-12, precision=precision, compact_index=ci, **part)
        assert p.partition()["compact"] == ci
        x, y, info = p.solve()
        p.close()
        res.append((x, y, info))
    (x1, y1, i1), (x0, y0, i0) = res
    assert i1["attempts"] == i0["attempts"] and i1["accepted"] == i0["accepted"]
    assert np.array_equal(x1.view(np.uint64), x0.view(np.uint64))
    assert np.array_equal(y1.view(np.uint64), y0.view(np.uint64))


def test_compact_index_falls_back_on_wide_tiles(gpu, oracle_mod):
    """A tile whose indices span more than 65535 keeps the 32-bit structure,
    and the attempt still matches the oracle."""
    from paper_2512_06715_amd.solver import Problem
    lp = wide_tile_lp()
    print("case wide tiles", flush=True)
    p = Problem(lp, max_iter=4, tol=1e-12, reorder=0, use_graph=0)
    assert p.partition()["compact"] == 0
    x, y, info = p.solve()
    p.close()
    xo, yo, io = oracle_mod.pdhg(lp, tol=1e-12, max_iter=4)
    assert info["attempts"] == io["attempts"] == 4
    np.testing.assert_allclose(x, xo, rtol=1e-12, atol=1e-12 * (1 + np.abs(xo).max()))
    np.testing.assert_allclose(y, yo, rtol=1e-12, atol=1e-12 * (1 + np.abs(yo).max()))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_repeat_runs_bit_identical(gpu, precision):
    """Two runs of the same solve give the same bits.  With a low long-row
    threshold thousands of rows have workgroups of their own while their
    tiles' workgroups fold the running sums of the average; 300 attempts
    cover restarts to the average, which read those sums."""
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc1000_t48")
    print("case repeat", precision, flush=True)
    res = []
    for _ in range(2):
        p = Problem(lp, max_iter=300, tol=1e-12, precision=precision, long_seg=8)
        x, y, info = p.solve()
        p.close()
        res.append((x, y, info))
    assert res[0][2]["restarts"] >= 2
    assert res[0][2]["omega"] == res[1][2]["omega"]
    assert np.array_equal(res[0][0].view(np.uint64), res[1][0].view(np.uint64))
    assert np.array_equal(res[0][1].view(np.uint64), res[1][1].view(np.uint64))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_lds_and_per_row_partitions_bit_identical(gpu, precision):
    """Every product is rounded on its own (no multiply-add contraction), so
    the LDS-staged tiles and the per-row loops give the same bits: 300
    attempts with either partition, evaluations and restarts included."""
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc1000_t48")
    print("case lds vs per-row", precision, flush=True)
    res = []
    for direct in (0, 1):
        p = Problem(lp, max_iter=300, tol=1e-12, precision=precision, spmv_direct=direct)
        assert p.partition()["direct"] == direct
        res.append(p.solve())
        p.close()
    (x0, y0, i0), (x1, y1, i1) = res
    assert i0["attempts"] == i1["attempts"] and i0["accepted"] == i1["accepted"]
    assert np.array_equal(x0.view(np.uint64), x1.view(np.uint64))
    assert np.array_equal(y0.view(np.uint64), y1.view(np.uint64))


def test_objective_offset_is_reported_only(gpu):
    """A constant in the objective shifts the reported objectives and the dual
    bound by exactly that constant and changes nothing else: the same steps,
    the same bits of x and y, in a solve and in a batch."""
    from paper_2512_06715_amd.solver import Problem, solve_batch
    lp = ucgen.workload("uc14_t24")
    shifted = lp.copy()
    shifted.obj_offset = -1234.5
    print("case objective offset", flush=True)
    out = []
    for q in (lp, shifted):
        p = Problem(q, tol=1e-4, max_iter=400000)
        out.append(p.solve())
        (bx, by, bi), = solve_batch([p], [dict(base=0)])
        out.append((bx, by, bi))
        p.close()
    for (x0, y0, i0), (x1, y1, i1) in ((out[0], out[2]), (out[1], out[3])):
        assert i0["status"] == i1["status"] == 1
        assert i0["attempts"] == i1["attempts"]
        assert np.array_equal(x0, x1) and np.array_equal(y0, y1)
        for key in ("primal_obj", "dual_obj", "dual_bound"):
            assert i1[key] == i0[key] + shifted.obj_offset, key
        assert i1["rel_kkt"] == i0["rel_kkt"] and i1["rel_gap"] == i0["rel_gap"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_stream_load_policies_bit_identical(gpu, precision):
    """Non-temporal and ordinary stream loads read the same values: 300
    attempts with either policy give the same bits."""
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc1000_t48")
    print("case stream policy", precision, flush=True)
    res = []
    for nt in (0, 1):
        p = Problem(lp, max_iter=300, tol=1e-12, precision=precision, stream_nt=nt)
        part = p.partition()
        assert part["stream_nt_fp64"] == nt and part["stream_nt_fp32"] == nt
        res.append(p.solve())
        p.close()
    (x0, y0, i0), (x1, y1, i1) = res
    assert i0["attempts"] == i1["attempts"] and i0["accepted"] == i1["accepted"]
    assert np.array_equal(x0.view(np.uint64), x1.view(np.uint64))
    assert np.array_equal(y0.view(np.uint64), y1.view(np.uint64))
