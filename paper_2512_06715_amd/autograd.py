"""Differentiable optimal cost of the unit-commitment LP relaxation.

`OptimalCost.apply(load, cost, problem, uc)` runs the unrolled PDHG solve of
`problem` (a Problem set up with unroll_iters = K) after mapping the nodal
loads D[i, t] and the energy prices cost[g] into b and c, and returns
V = c'x_K.  Its backward calls the library's adjoint (pdhg_backward) and maps
dV/db, dV/dc back to the loads and prices:
    dV/dD[i, t]  = dV/db[bal(i, t)] + reserve_frac * dV/db[res(t)]
    dV/dcost[g]  = dt * sum_t dV/dc[p(g, t)]
"""
from __future__ import annotations

import numpy as np
import torch


class UCMaps:
    """Index maps between UC parameters and the LP vectors (from ucgen meta)."""

    def __init__(self, lp):
        meta = lp.meta
        self.bal = np.asarray(meta["bal_rows"])        # [T, N]
        self.res = np.asarray(meta["res_rows"])        # [T]
        self.pcols = np.asarray(meta["p_cols"])        # [T, G]
        self.dt = float(meta["dt"])
        self.rf = float(meta["reserve_frac"])
        self.b0 = np.asarray(lp.b, np.float64).copy()
        self.c0 = np.asarray(lp.c, np.float64).copy()

    def to_bc(self, load: np.ndarray, cost: np.ndarray):
        """load[N, T] (MW), cost[G] ($/MWh) -> (b, c)."""
        b = self.b0.copy()
        c = self.c0.copy()
        b[self.bal.T] = load
        b[self.res] = self.rf * load.sum(axis=0)
        c[self.pcols] = cost[None, :] * self.dt
        return b, c

    def grads(self, gb: np.ndarray, gc: np.ndarray):
        gload = gb[self.bal.T] + self.rf * gb[self.res][None, :]
        gcost = self.dt * gc[self.pcols].sum(axis=0)
        return gload, gcost


class OptimalCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, load, cost, problem, maps):
        b, c = maps.to_bc(load.detach().cpu().numpy(), cost.detach().cpu().numpy())
        problem.update(b, c)
        x, y, info = problem.solve()
        ctx.problem = problem
        ctx.maps = maps
        ctx.load_dtype, ctx.device = load.dtype, load.device
        return torch.tensor(info["primal_obj"], dtype=load.dtype, device=load.device)

    @staticmethod
    def backward(ctx, gV):
        gb, gc = ctx.problem.backward(float(gV))
        if isinstance(gb, torch.Tensor):
            gb, gc = gb.cpu().numpy(), gc.cpu().numpy()
        gload, gcost = ctx.maps.grads(gb, gc)
        t = lambda a: torch.as_tensor(a, dtype=ctx.load_dtype, device=ctx.device)
        return t(gload), t(gcost), None, None
