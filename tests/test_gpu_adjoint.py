"""Adjoint of unrolled PDHG against the oracle's forward-mode derivative,
finite differences of the GPU's own unrolled map, and the autograd wrapper."""
import numpy as np
import pytest

from paper_2512_06715_amd import ucgen

pytestmark = pytest.mark.gpu


def setup_lp(oracle_mod, lp, K, C):
    from paper_2512_06715_amd.solver import Problem
    eta, omega = oracle_mod.unrolled_step(lp)
    p = Problem(lp, unroll_iters=K, checkpoint_every=C, fixed_eta=eta, fixed_omega=omega)
    return p, eta, omega


@pytest.mark.parametrize("dims,K,C", [((6, 3, 8, 6), 300, 50), ((14, 5, 20, 24), 1000, 64),
                                      ((14, 5, 20, 24), 37, 10)])
def test_adjoint_dot_product_with_oracle_jvp(gpu, oracle_mod, dims, K, C):
    lp = ucgen.random_uc(*dims, 1.0, seed=9)
    print("case adjoint", dims, K, C, flush=True)
    p, eta, omega = setup_lp(oracle_mod, lp, K, C)
    x, y, info = p.solve()
    gb, gc = p.backward(1.0)
    p.close()
    rng = np.random.default_rng(1)
    V_tot = 0.0
    for trial in range(3):
        db = rng.standard_normal(lp.m)
        dc = rng.standard_normal(lp.n)
        V, dV = oracle_mod.unrolled(lp, K, eta, omega, db, dc)
        lhs = gb @ db + gc @ dc
        assert abs(lhs - dV) <= 1e-9 * (1 + abs(dV)), (trial, lhs, dV)
        V_tot = V
    assert abs(info["primal_obj"] - V_tot) <= 1e-10 * (1 + abs(V_tot))


def test_adjoint_matches_gpu_finite_differences(gpu, oracle_mod):
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.random_uc(6, 3, 8, 6, 1.0, seed=9)
    K = 200
    p, eta, omega = setup_lp(oracle_mod, lp, K, 40)
    p.solve()
    gb, gc = p.backward(1.0)
    rng = np.random.default_rng(2)
    # directions away from the exact-zero entries, where the map has kinks
    db = rng.standard_normal(lp.m) * (lp.b != 0)
    dc = rng.standard_normal(lp.n) * (lp.c != 0)
    h = 1e-6
    vals = []
    for sgn in (1, -1):
        p.update(lp.b + sgn * h * db, lp.c + sgn * h * dc)
        _, _, info = p.solve()
        vals.append(info["primal_obj"])
    p.close()
    fd = (vals[0] - vals[1]) / (2 * h)
    assert abs(fd - (gb @ db + gc @ dc)) <= 1e-6 * (1 + abs(fd))


def test_backward_requires_unrolled_solve(gpu):
    from paper_2512_06715_amd import _lib
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.random_uc(6, 3, 8, 6, 1.0, seed=9)
    p = Problem(lp, unroll_iters=20)
    with pytest.raises(_lib.PdhgError):
        p.backward()
    p.solve()
    p.backward()
    p.update(lp.b)
    with pytest.raises(_lib.PdhgError):
        p.backward()
    p.close()


def test_autograd_load_and_cost(gpu, oracle_mod):
    import torch
    from paper_2512_06715_amd.autograd import OptimalCost, UCMaps
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.random_uc(14, 5, 20, 6, 1.0, seed=31)
    maps = UCMaps(lp)
    K = 400
    eta, omega = oracle_mod.unrolled_step(lp)
    p = Problem(lp, unroll_iters=K, checkpoint_every=50, fixed_eta=eta, fixed_omega=omega)
    load = torch.tensor(lp.meta["load"], dtype=torch.float64, requires_grad=True)
    cost = torch.tensor(lp.meta["gen_cost"], dtype=torch.float64, requires_grad=True)
    V = OptimalCost.apply(load, cost, p, maps)
    V.backward()
    # the same derivative through the oracle's forward mode, one direction each
    rng = np.random.default_rng(3)
    dD = rng.standard_normal(load.shape)
    dcost = rng.standard_normal(cost.shape)
    b1, c1 = maps.to_bc(lp.meta["load"] + dD, lp.meta["gen_cost"] + dcost)
    b0, c0 = maps.to_bc(lp.meta["load"], lp.meta["gen_cost"])
    Vo, dVo = oracle_mod.unrolled(lp, K, eta, omega, b1 - b0, c1 - c0)
    lhs = float((load.grad.numpy() * dD).sum() + (cost.grad.numpy() * dcost).sum())
    assert abs(lhs - dVo) <= 1e-9 * (1 + abs(dVo))
    assert abs(float(V.detach()) - Vo) <= 1e-10 * (1 + abs(Vo))
    p.close()
