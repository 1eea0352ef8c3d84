"""Branch-and-bound node LPs on the GPU: the consumer of batched solves.

The paper puts the benefit of a GPU first-order method for the
unit-commitment MILP in faster bound estimation and tighter LP relaxation
bounds for branch and bound (abstract; Introduction, "Contribution"; Results
and Discussion, "PDHG Execution & Crossover Refinement").  A node of the
relaxed UC problem fixes some commitments u_{g,t} to 0 or 1 on top of the
base LP.  Here the children of
nodes are solved together in one batched run (one set of launches, the base
matrix shared), each started from its parent's point (x, y), and every
result carries a lower bound on the child's LP optimum that holds whatever
the accuracy of the returned duals (weak duality with implied variable
bounds, `pdhg_info.dual_bound`).  A node whose bound exceeds an incumbent's
objective can therefore be pruned exactly.

The search itself (node selection, incumbent heuristics, branching rules
beyond the most fractional commitment) belongs to the caller.  Warm-started
children may be solved on a mixed-precision or an FP64 handle of the same LP
at about the same cost (16 children of the 4224-bus root: 4.67 s in mixed
precision, 13.2k attempts mean, against 4.72 s and 10.2k in FP64).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .solver import solve_batch

PRIMAL_INFEASIBLE = 5   # pdhg_info.status of a proved-infeasible LP


@dataclasses.dataclass
class Node:
    """One node: columns fixed on top of the base LP (caller's order), the
    warm start it is solved from, and after solving its point and info."""
    fix_idx: np.ndarray
    fix_val: np.ndarray
    depth: int = 0
    x0: Optional[np.ndarray] = None
    y0: Optional[np.ndarray] = None
    omega0: float = 0.0   # parent's final primal weight and step size (0: defaults)
    eta0: float = 0.0
    hold: int = 0         # attempts the weight is held (the parent's attempt count)
    x: Optional[np.ndarray] = None
    y: Optional[np.ndarray] = None
    info: Optional[dict] = None

    @property
    def solved(self) -> bool:
        return self.info is not None

    @property
    def bound(self) -> float:
        """Lower bound on this node's LP optimum: -inf before solving, +inf
        when the solve proved the LP infeasible (a Farkas certificate: no
        feasible point, so its subtree is empty), else the safe bound."""
        if not self.info:
            return -np.inf
        if int(self.info.get("status", 0)) == PRIMAL_INFEASIBLE:
            return np.inf
        return float(self.info["dual_bound"])

    @property
    def objective(self) -> float:
        return float(self.info["primal_obj"]) if self.info else np.nan

    def fixed(self) -> dict:
        return dict(zip(self.fix_idx.tolist(), self.fix_val.tolist()))


def root() -> Node:
    return Node(np.zeros(0, np.int32), np.zeros(0, np.float64))


def branch(node: Node, col: int) -> Tuple[Node, Node]:
    """The two children of a solved node that fix column `col` to 0 and to 1,
    both warm-started from the node's point."""
    if not node.solved:
        raise ValueError("branch needs a solved node")
    if col in set(node.fix_idx.tolist()):
        raise ValueError(f"column {col} is already fixed at this node")
    kids = []
    for v in (0.0, 1.0):
        idx = np.append(node.fix_idx, np.int32(col)).astype(np.int32)
        val = np.append(node.fix_val, v).astype(np.float64)
        kids.append(Node(idx, val, node.depth + 1, x0=node.x, y0=node.y,
                         omega0=float(node.info.get("omega", 0.0)),
                         eta0=float(node.info.get("eta", 0.0)),
                         hold=int(node.info.get("attempts", 0))))
    return kids[0], kids[1]


def most_fractional(node: Node, cols: Sequence[int], k: int = 1) -> np.ndarray:
    """The k columns among `cols` (not fixed at the node) whose values in the
    node's solution are closest to 1/2; ties by column index."""
    if not node.solved:
        raise ValueError("most_fractional needs a solved node")
    cols = np.asarray(cols, dtype=np.int64)
    free = cols[~np.isin(cols, node.fix_idx)]
    x = _host(node.x)
    dist = np.abs(x[free] - 0.5)
    order = np.lexsort((free, dist))
    return free[order[:k]]


def solve_nodes(problem, nodes: List[Node], warm: bool = True,
                weights: bool = True) -> List[Node]:
    """Solve the nodes' LPs in one batched run on `problem` (a solver.Problem
    of the base LP).  With `warm`, each node starts from its x0, y0 when it
    has them; with `weights` also from its parent's step size and primal
    weight, the weight held for as many attempts as the parent took (near
    the optimum the restarts' weight updates see little primal movement and
    drive the weight up by a factor of about 1.5 per restart, stalling the
    primal iterate; past that budget the updates resume).  Fills x, y and
    info of every node and returns the list."""
    if not nodes:
        return nodes
    insts = []
    for nd in nodes:
        d = dict(base=0, fix_idx=_like(problem, nd.fix_idx, np.int32),
                 fix_val=_like(problem, nd.fix_val, np.float64))
        if warm and nd.x0 is not None and nd.y0 is not None:
            d["x0"] = _like(problem, nd.x0, np.float64)
            d["y0"] = _like(problem, nd.y0, np.float64)
            if weights:
                d["omega0"], d["eta0"], d["hold_omega"] = nd.omega0, nd.eta0, nd.hold
        insts.append(d)
    for nd, (x, y, info) in zip(nodes, solve_batch([problem], insts)):
        nd.x, nd.y, nd.info = x, y, info
    return nodes


def prune(nodes: Sequence[Node], incumbent: float) -> Tuple[List[Node], List[Node]]:
    """Split solved nodes into (kept, pruned): a node is pruned when its safe
    bound is above the incumbent's objective, so its subtree holds nothing
    better; a node proved infeasible always is (its bound is +inf)."""
    kept, cut = [], []
    for nd in nodes:
        (cut if nd.bound > incumbent else kept).append(nd)
    return kept, cut


def _host(a) -> np.ndarray:
    if isinstance(a, np.ndarray):
        return a
    return a.detach().cpu().numpy()


def _like(problem, a, dtype):
    """Array `a` in the form the problem's batch call takes (numpy for host
    problems, a CUDA tensor for device ones)."""
    if a is None:
        return None
    if not problem.device:
        return np.ascontiguousarray(_host(a), dtype=dtype)
    import torch
    tdt = torch.int32 if dtype == np.int32 else torch.float64
    if isinstance(a, np.ndarray):
        return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype)).to("cuda", tdt)
    return a.to("cuda", tdt).contiguous()
