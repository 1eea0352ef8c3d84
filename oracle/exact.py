"""The LP optimum by definition, for small problems.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The LP is   min c'x  s.t.  a_i'x = b_i (kind 0),  a_i'x >= b_i (kind 1),
            l <= x <= u.
- `vertex_enum`: brute force over the vertices (every choice of n linearly
  independent active constraints among the rows and finite bounds),
  for n, m <= 6 and every variable boxed.  The optimum of a bounded feasible LP
  is attained at a vertex, so this is the definition written out.
- `simplex`: a dense two-phase tableau simplex with Bland's rule (Bland's
  rule cannot cycle, which matters because these LPs are degenerate).
- `highs`: scipy's HiGHS, a library LP solve used as an independent reference.
Duals follow the Lagrangian c'x - y'(Ax - b): y free on equality rows and
y >= 0 on >= rows.
"""
from __future__ import annotations

import itertools

import numpy as np

OPTIMAL, INFEASIBLE, UNBOUNDED = "optimal", "infeasible", "unbounded"


def _dense(lp):
    A = np.zeros((lp.m, lp.n))
    for i in range(lp.m):
        s, e = lp.row_ptr[i], lp.row_ptr[i + 1]
        A[i, lp.col_idx[s:e]] = lp.val[s:e]
    return A


def vertex_enum(lp, tol=1e-9):
    """Minimum of c'x over the vertices of the feasible set (boxed variables)."""
    A = _dense(lp)
    m, n = A.shape
    if not (np.all(np.isfinite(lp.l)) and np.all(np.isfinite(lp.u))):
        raise ValueError("vertex enumeration needs every variable boxed")
    # candidate active constraints: (row vector, rhs, is_equality_row)
    cands = []
    for i in range(m):
        cands.append((A[i], lp.b[i], lp.row_kind[i] == 0))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cands.append((e, lp.l[j], False))
        cands.append((e, lp.u[j], False))
    # a vertex is a feasible point where n linearly independent constraints
    # hold with equality; equality rows are enforced by the feasibility test
    best, best_x = np.inf, None
    for rows in itertools.combinations(range(len(cands)), n):
        M = np.array([cands[k][0] for k in rows])
        r = np.array([cands[k][1] for k in rows])
        if np.linalg.matrix_rank(M, tol=1e-10) < n:
            continue
        x, *_ = np.linalg.lstsq(M, r, rcond=None)
        if np.max(np.abs(M @ x - r)) > 1e-8:
            continue
        ax = A @ x
        ok = np.all(x >= lp.l - tol) and np.all(x <= lp.u + tol)
        ok &= np.all(np.abs(ax - lp.b)[lp.row_kind == 0] <= tol * (1 + np.abs(lp.b[lp.row_kind == 0])))
        ok &= np.all((ax - lp.b)[lp.row_kind == 1] >= -tol * (1 + np.abs(lp.b[lp.row_kind == 1])))
        if ok:
            v = float(lp.c @ x)
            if v < best:
                best, best_x = v, x
    if best_x is None:
        return INFEASIBLE, None, np.inf
    return OPTIMAL, best_x, best


def simplex(lp, tol=1e-9, max_pivots=200000):
    """Two-phase dense tableau simplex with Bland's rule.

    Returns (status, x, objective, y).  Standard form: every variable is
    shifted onto [0, inf) (free variables split in two, upper bounds become
    rows with a slack), >= rows get a surplus column.
    """
    A0 = _dense(lp)
    m0, n0 = A0.shape
    cols = []        # (original j, sign, offset) : x_j = offset + sign * z
    Acols, cz = [], []
    ub_rows = []     # (z index, width)
    const_obj = 0.0
    bshift = lp.b.astype(float).copy()
    for j in range(n0):
        lj, uj = lp.l[j], lp.u[j]
        if np.isfinite(lj):
            bshift -= A0[:, j] * lj
            const_obj += lp.c[j] * lj
            Acols.append(A0[:, j])
            cz.append(lp.c[j])
            cols.append((j, 1.0, lj))
            if np.isfinite(uj):
                ub_rows.append((len(Acols) - 1, uj - lj))
        elif np.isfinite(uj):
            bshift -= A0[:, j] * uj
            const_obj += lp.c[j] * uj
            Acols.append(-A0[:, j])
            cz.append(-lp.c[j])
            cols.append((j, -1.0, uj))
        else:
            Acols.append(A0[:, j])
            cz.append(lp.c[j])
            cols.append((j, 1.0, 0.0))
            Acols.append(-A0[:, j])
            cz.append(-lp.c[j])
            cols.append((j, -1.0, 0.0))
    nz = len(Acols)
    ge = np.nonzero(lp.row_kind == 1)[0]
    nub = len(ub_rows)
    M = m0 + nub
    N = nz + len(ge) + nub
    T = np.zeros((M, N))
    T[:m0, :nz] = np.array(Acols).T if nz else 0.0
    for k, i in enumerate(ge):
        T[i, nz + k] = -1.0
    rhs = np.concatenate([bshift, np.array([w for _, w in ub_rows])])
    for k, (zi, _) in enumerate(ub_rows):
        T[m0 + k, zi] = 1.0
        T[m0 + k, nz + len(ge) + k] = 1.0
    cost = np.concatenate([np.array(cz), np.zeros(len(ge) + nub)])
    # rows with negative rhs are negated so the artificial basis is feasible
    sgn = np.where(rhs < 0, -1.0, 1.0)
    T = T * sgn[:, None]
    rhs = rhs * sgn
    # phase 1 tableau with artificials
    tab = np.zeros((M + 1, N + M + 1))
    tab[:M, :N] = T
    tab[:M, N:N + M] = np.eye(M)
    tab[:M, -1] = rhs
    basis = list(range(N, N + M))

    def pivot(r, q):
        tab[r] /= tab[r, q]
        f = tab[:, q].copy()
        f[r] = 0.0
        tab[:] -= np.outer(f, tab[r])
        basis[r] = q

    def run(obj_row_cost, allowed):
        # reduced-cost row for the current basis
        tab[M, :] = 0.0
        tab[M, :len(obj_row_cost)] = obj_row_cost
        for r, q in enumerate(basis):
            if q < len(obj_row_cost) and obj_row_cost[q] != 0.0:
                tab[M] -= obj_row_cost[q] * tab[r]
        for _ in range(max_pivots):
            red = tab[M, :allowed]
            cand = np.nonzero(red < -tol)[0]
            if len(cand) == 0:
                return OPTIMAL
            q = int(cand[0])
            col = tab[:M, q]
            pos = np.nonzero(col > tol)[0]
            if len(pos) == 0:
                return UNBOUNDED
            ratios = tab[pos, -1] / col[pos]
            rmin = ratios.min()
            ties = pos[np.abs(ratios - rmin) <= tol * (1 + abs(rmin))]
            r = int(min(ties, key=lambda i: basis[i]))
            pivot(r, q)
        raise RuntimeError("simplex pivot limit reached")

    c1 = np.concatenate([np.zeros(N), np.ones(M)])
    run(c1, N + M)
    if -tab[M, -1] > 1e-7 * (1 + np.abs(rhs).sum()):
        return INFEASIBLE, None, np.inf, None
    # drive artificials out of the basis
    keep = np.ones(M, bool)
    for r in range(M):
        if basis[r] >= N:
            nzc = np.nonzero(np.abs(tab[r, :N]) > 1e-9)[0]
            if len(nzc):
                pivot(r, int(nzc[0]))
            else:
                keep[r] = False
    tab = np.vstack([tab[:M][keep], tab[M:]])
    basis = [b for b, k in zip(basis, keep) if k]
    M = len(basis)
    tab = np.delete(tab, np.s_[N:N + tab.shape[1] - N - 1], axis=1)
    st = run(cost, N)
    if st == UNBOUNDED:
        return UNBOUNDED, None, -np.inf, None
    z = np.zeros(N)
    for r, q in enumerate(basis):
        z[q] = tab[r, -1]
    x = np.zeros(n0)
    for k, (j, s, off) in enumerate(cols):
        x[j] += s * z[k]
    for j in range(n0):
        if np.isfinite(lp.l[j]):
            x[j] += lp.l[j]
        elif np.isfinite(lp.u[j]):
            x[j] += lp.u[j]
    obj = float(lp.c @ x)
    # duals: B' w = c_B over the (sign-adjusted) rows that were kept
    Bm = T[np.nonzero(keep)[0]][:, basis]
    w, *_ = np.linalg.lstsq(Bm.T, cost[basis], rcond=None)
    yfull = np.zeros(len(keep))
    yfull[np.nonzero(keep)[0]] = w
    yfull *= sgn
    return OPTIMAL, x, obj, yfull[:m0]


def highs(lp, method="highs"):
    """scipy.optimize.linprog(method=...): (status, x, objective, y).

    method is one of scipy's HiGHS front ends: 'highs' (HiGHS picks),
    'highs-ds' (dual simplex) or 'highs-ipm' (interior point with crossover,
    the faster one on LPs of millions of columns)."""
    from scipy.optimize import linprog
    import scipy.sparse as sp
    A = sp.csr_matrix((lp.val, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))
    eq = lp.row_kind == 0
    kw = {}
    if (~eq).any():
        kw.update(A_ub=-A[~eq], b_ub=-lp.b[~eq])
    if eq.any():
        kw.update(A_eq=A[eq], b_eq=lp.b[eq])
    bounds = list(zip(np.where(np.isinf(lp.l), None, lp.l), np.where(np.isinf(lp.u), None, lp.u)))
    res = linprog(lp.c, bounds=bounds, method=method, **kw)
    if res.status == 2:
        return INFEASIBLE, None, np.inf, None
    if res.status == 3:
        return UNBOUNDED, None, -np.inf, None
    if res.status != 0:
        raise RuntimeError(res.message)
    y = np.zeros(lp.m)
    if eq.any():
        y[eq] = res.eqlin.marginals
    if (~eq).any():
        y[~eq] = -res.ineqlin.marginals
    return OPTIMAL, res.x, float(res.fun), y
