"""Seeded synthetic DC unit-commitment LP relaxations.

The paper solves the LP relaxation of a multi-period DC unit-commitment
model (Section II, Table I gives the sizes of the 4224/6049/6717-bus
systems).  The ARPA-E data it uses is not available, so this module draws
instances of the same shape from a seeded generator.  It is the one module
that both the HIP path and the CPU oracle consume: it builds the LP
(CSR A, b, c, l, u, row kinds) and holds none of the solver's arithmetic.

Formulation (one period t of length dt hours, generators g, buses i,
lines k):

    variables, t-major: [u_g v_g w_g p_g]*G, theta_i*N, f_k*L,
                        s+_i*N, s-_i*N, r
    p - Pmin u >= 0              Pmax u - p >= 0
    p_t - p_{t-1} <= RU          p_{t-1} - p_t <= RD          (t >= 1)
    u_t - u_{t-1} - v_t + w_t = 0   (u_{-1} = u0 = 0)
    sum_{g@i} p - sum_{out} f + sum_{in} f + s+_i - s-_i = D_{i,t}
    f_k - (100/x_k)(theta_from - theta_to) = 0
    sum_g (Pmax u - p) + r >= reserve_frac * sum_i D_{i,t}
    u,v,w in [0,1]; p in [0,Pmax]; theta free (reference bus fixed to 0);
    f in [-Fmax, Fmax]; s+, s-, r >= 0.
    cost: NL*dt*u + SU*v + cost*dt*p + 1000*dt*(s+ + s- + r)

The slacks make every instance feasible: the point with every generator
off, all flows zero and s+ = D, r = reserve is feasible for any bound
fixing of u.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

ROW_EQ = 0
ROW_GE = 1
BASE_MVA = 100.0
PENALTY = 1000.0


@dataclasses.dataclass
class Network:
    n_bus: int
    frm: np.ndarray     # int64[L]
    to: np.ndarray      # int64[L]
    x: np.ndarray       # reactance, pu
    fmax: np.ndarray    # MW


@dataclasses.dataclass
class Gens:
    bus: np.ndarray     # int64[G]
    pmax: np.ndarray
    pmin: np.ndarray
    ramp: np.ndarray    # MW per period, up and down
    cost: np.ndarray    # $/MWh
    noload: np.ndarray  # $/h
    startup: np.ndarray  # $ per start


@dataclasses.dataclass
class UCLP:
    """An LP  min c'x  s.t.  A x (= or >=) b,  l <= x <= u  in canonical CSR."""
    m: int
    n: int
    row_ptr: np.ndarray   # int32[m+1]
    col_idx: np.ndarray   # int32[nnz]
    val: np.ndarray       # float64[nnz]
    row_kind: np.ndarray  # uint8[m]
    b: np.ndarray
    c: np.ndarray
    l: np.ndarray
    u: np.ndarray
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def copy(self) -> "UCLP":
        return UCLP(self.m, self.n, self.row_ptr.copy(), self.col_idx.copy(),
                    self.val.copy(), self.row_kind.copy(), self.b.copy(),
                    self.c.copy(), self.l.copy(), self.u.copy(), dict(self.meta))


def size_formulas(N: int, G: int, L: int, T: int) -> dict:
    """Closed-form counts for the formulation above."""
    return dict(
        n=(4 * G + 3 * N + L + 1) * T,
        m=T * (3 * G + N + L + 1) + 2 * G * (T - 1),
        m_eq=T * (G + N + L),
        nnz=T * (11 * G + 5 * L + 2 * N + 1) - G + 4 * G * (T - 1),
    )


# ---------------------------------------------------------------------------
# random parameters


def random_network(rng: np.random.Generator, N: int, L: int) -> Network:
    """Random recursive tree over a random bus permutation plus extra edges."""
    if L < N - 1:
        raise ValueError("need at least N-1 lines for a spanning tree")
    perm = rng.permutation(N)
    frm, to = [], []
    seen = set()
    if N > 1:
        parents = np.floor(rng.random(N - 1) * np.arange(1, N)).astype(np.int64)
        for k in range(1, N):
            a, b_ = int(perm[k]), int(perm[parents[k - 1]])
            frm.append(a)
            to.append(b_)
            seen.add((min(a, b_), max(a, b_)))
    extra = L - (N - 1)
    max_edges = N * (N - 1) // 2
    if L > max_edges:
        raise ValueError("too many lines for a simple graph")
    while extra > 0:
        a, b_ = (int(v) for v in rng.integers(0, N, size=2))
        if a == b_:
            continue
        key = (min(a, b_), max(a, b_))
        if key in seen:
            continue
        seen.add(key)
        frm.append(a)
        to.append(b_)
        extra -= 1
    frm = np.array(frm, dtype=np.int64)
    to = np.array(to, dtype=np.int64)
    flip = rng.random(L) < 0.5
    frm2 = np.where(flip, to, frm)
    to2 = np.where(flip, frm, to)
    x = rng.uniform(0.01, 0.2, size=L)
    fmax = rng.uniform(50.0, 200.0, size=L)
    return Network(N, frm2, to2, x, fmax)


def random_gens(rng: np.random.Generator, N: int, G: int) -> Gens:
    bus = rng.integers(0, N, size=G)
    pmax = rng.uniform(50.0, 400.0, size=G)
    cost = rng.uniform(10.0, 60.0, size=G)
    noload = rng.uniform(100.0, 500.0, size=G)
    startup = rng.uniform(500.0, 5000.0, size=G)
    return Gens(bus, pmax, 0.3 * pmax, 0.5 * pmax, cost, noload, startup)


def daily_load(base: np.ndarray, T: int, dt: float) -> np.ndarray:
    """D[i, t] = base_i * (1 + 0.2 sin(2 pi (h_t - 12) / 24)), peak at 18:00."""
    h = np.arange(T) * dt
    shape = 1.0 + 0.2 * np.sin(2.0 * np.pi * (h - 12.0) / 24.0)
    return base[:, None] * shape[None, :]


# ---------------------------------------------------------------------------
# LP assembly


def build_uc_lp(net: Network, gens: Gens, load: np.ndarray, T: int, dt: float,
                reserve_frac: float = 0.05, u0: float = 0.0) -> UCLP:
    """Assemble the DC-UC LP relaxation in canonical CSR (see module doc)."""
    N, L, G = net.n_bus, len(net.frm), len(gens.bus)
    P = 4 * G + 3 * N + L + 1                      # columns per period
    n = P * T
    g = np.arange(G, dtype=np.int64)
    ib = np.arange(N, dtype=np.int64)
    kl = np.arange(L, dtype=np.int64)

    def cu(t): return t * P + 4 * g
    def cv(t): return t * P + 4 * g + 1
    def cw(t): return t * P + 4 * g + 2
    def cp(t): return t * P + 4 * g + 3
    def cth(t): return t * P + 4 * G + ib
    def cf(t): return t * P + 4 * G + N + kl
    def csp(t): return t * P + 4 * G + N + L + ib
    def csm(t): return t * P + 4 * G + 2 * N + L + ib
    def cr(t): return t * P + 4 * G + 3 * N + L

    rows, cols, vals = [], [], []
    b_parts, kind_parts = [], []
    bal_rows = np.zeros((T, N), dtype=np.int64)
    res_rows = np.zeros(T, dtype=np.int64)
    r0 = 0
    bsum = BASE_MVA / net.x
    for t in range(T):
        # generator limit rows
        rmin = r0 + g
        rows += [rmin, rmin]; cols += [cp(t), cu(t)]
        vals += [np.ones(G), -gens.pmin]
        rmax = r0 + G + g
        rows += [rmax, rmax]; cols += [cu(t), cp(t)]
        vals += [gens.pmax.copy(), -np.ones(G)]
        b_parts += [np.zeros(2 * G)]
        kind_parts += [np.full(2 * G, ROW_GE, np.uint8)]
        r = r0 + 2 * G
        if t >= 1:
            rup = r + g
            rows += [rup, rup]; cols += [cp(t), cp(t - 1)]
            vals += [-np.ones(G), np.ones(G)]
            rdn = r + G + g
            rows += [rdn, rdn]; cols += [cp(t), cp(t - 1)]
            vals += [np.ones(G), -np.ones(G)]
            b_parts += [-gens.ramp, -gens.ramp]
            kind_parts += [np.full(2 * G, ROW_GE, np.uint8)]
            r += 2 * G
        # commitment logic rows
        rlg = r + g
        rows += [rlg, rlg, rlg]; cols += [cu(t), cv(t), cw(t)]
        vals += [np.ones(G), -np.ones(G), np.ones(G)]
        if t >= 1:
            rows += [rlg]; cols += [cu(t - 1)]; vals += [-np.ones(G)]
            b_parts += [np.zeros(G)]
        else:
            b_parts += [np.full(G, float(u0))]
        kind_parts += [np.full(G, ROW_EQ, np.uint8)]
        r += G
        # nodal balance rows
        rbal = r + ib
        bal_rows[t] = rbal
        rows += [rbal[gens.bus], rbal[net.frm], rbal[net.to], rbal, rbal]
        cols += [cp(t), cf(t), cf(t), csp(t), csm(t)]
        vals += [np.ones(G), -np.ones(L), np.ones(L), np.ones(N), -np.ones(N)]
        b_parts += [load[:, t].copy()]
        kind_parts += [np.full(N, ROW_EQ, np.uint8)]
        r += N
        # DC flow rows
        rfl = r + kl
        rows += [rfl, rfl, rfl]; cols += [cf(t), cth(t)[net.frm], cth(t)[net.to]]
        vals += [np.ones(L), -bsum, bsum.copy()]
        b_parts += [np.zeros(L)]
        kind_parts += [np.full(L, ROW_EQ, np.uint8)]
        r += L
        # spinning reserve row
        res_rows[t] = r
        rows += [np.full(G, r), np.full(G, r), np.array([r])]
        cols += [cu(t), cp(t), np.array([cr(t)])]
        vals += [gens.pmax.copy(), -np.ones(G), np.ones(1)]
        b_parts += [np.array([reserve_frac * load[:, t].sum()])]
        kind_parts += [np.full(1, ROW_GE, np.uint8)]
        r += 1
        r0 = r
    m = r0
    rows = np.concatenate(rows).astype(np.int64)
    cols = np.concatenate(cols).astype(np.int64)
    vals = np.concatenate(vals).astype(np.float64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
    if dup.any():
        raise AssertionError("duplicate entries in generated matrix")
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])

    b = np.concatenate(b_parts)
    kind = np.concatenate(kind_parts)
    c = np.zeros(n)
    lo = np.zeros(n)
    hi = np.full(n, np.inf)
    for t in range(T):
        for cc in (cu(t), cv(t), cw(t)):
            hi[cc] = 1.0
        hi[cp(t)] = gens.pmax
        lo[cth(t)] = -np.inf
        hi[cth(t)] = np.inf
        lo[cth(t)[0]] = 0.0
        hi[cth(t)[0]] = 0.0
        lo[cf(t)] = -net.fmax
        hi[cf(t)] = net.fmax
        c[cu(t)] = gens.noload * dt
        c[cv(t)] = gens.startup
        c[cp(t)] = gens.cost * dt
        c[csp(t)] = PENALTY * dt
        c[csm(t)] = PENALTY * dt
        c[cr(t)] = PENALTY * dt
    u_cols = np.stack([cu(t) for t in range(T)])
    p_cols = np.stack([cp(t) for t in range(T)])
    meta = dict(N=N, G=G, L=L, T=T, dt=dt, reserve_frac=reserve_frac,
                load=load.copy(), bal_rows=bal_rows, res_rows=res_rows,
                u_cols=u_cols, p_cols=p_cols, gen_cost=gens.cost.copy(),
                period_cols=P)
    return UCLP(m, n, row_ptr.astype(np.int32), cols.astype(np.int32), vals,
                kind.astype(np.uint8), b, c, lo, hi, meta)


def random_uc(N: int, G: int, L: int, T: int, dt: float = 1.0, seed=0,
              reserve_frac: float = 0.05) -> UCLP:
    """Draw network, generators and loads (in that order) and build the LP."""
    rng = np.random.default_rng(seed)
    net = random_network(rng, N, L)
    gens = random_gens(rng, N, G)
    base = rng.lognormal(mean=3.0, sigma=0.5, size=N)
    load = daily_load(base, T, dt)
    lp = build_uc_lp(net, gens, load, T, dt, reserve_frac)
    lp.meta.update(seed=seed, net=net, gens=gens)
    return lp


def fix_commitments(lp: UCLP, seed, frac: Optional[float] = None) -> UCLP:
    """Branch-and-bound-node variant: fix a random share of the u_{g,t} to 0 or 1.

    The share is drawn U[0, 0.2] unless given; fixed values are Bernoulli(0.5).
    Returns a copy with l = u = value on the fixed columns and the list of
    fixings in meta['fix_idx'], meta['fix_val'].
    """
    rng = np.random.default_rng(seed)
    if frac is None:
        frac = rng.uniform(0.0, 0.2)
    ucols = lp.meta["u_cols"].ravel()
    k = int(round(frac * len(ucols)))
    pick = np.sort(rng.choice(len(ucols), size=k, replace=False))
    idx = ucols[pick].astype(np.int32)
    vals = (rng.random(k) < 0.5).astype(np.float64)
    out = lp.copy()
    out.l[idx] = vals
    out.u[idx] = vals
    out.meta["fix_idx"] = idx
    out.meta["fix_val"] = vals
    out.meta["fix_frac"] = frac
    return out


# ---------------------------------------------------------------------------
# the workloads


WORKLOADS = {
    # name: (N, G, L, T, dt, seed)
    "uc14_t24": (14, 5, 20, 24, 1.0, 0),
    "uc1000_t48": (1000, 200, 1400, 48, 1.0, 1),
    "uc6717_t96": (6717, 1100, 9000, 96, 0.25, 2),
    "uc4224_t48": (4224, 700, 5800, 48, 1.0, 3),
    "uc2000_t24": (2000, 300, 2700, 24, 1.0, 4),
}


def workload(name: str, seed=None) -> UCLP:
    N, G, L, T, dt, s = WORKLOADS[name]
    lp = random_uc(N, G, L, T, dt, s if seed is None else seed)
    lp.meta["workload"] = name
    return lp


def small_batch_instance(j: int) -> UCLP:
    """Small distinct instance j of the batched workload: N ~ U{500..2000}, T=24."""
    rng = np.random.default_rng(3100 + j)
    N = int(rng.integers(500, 2001))
    G = int(round(0.2 * N))
    L = int(round(1.4 * N))
    return random_uc(N, G, L, 24, 1.0, 3100 + j)


def all_slack_point(lp: UCLP) -> np.ndarray:
    """The feasibility certificate: units off, no flow, all load shed."""
    meta = lp.meta
    N, G, L, T = meta["N"], meta["G"], meta["L"], meta["T"]
    P = meta["period_cols"]
    x = np.zeros(lp.n)
    for t in range(T):
        x[t * P + 4 * G + N + L + np.arange(N)] = meta["load"][:, t]
        x[t * P + 4 * G + 3 * N + L] = meta["reserve_frac"] * meta["load"][:, t].sum()
    return x


def random_toy_lp(rng: np.random.Generator, m: int, n: int, density=0.7,
                  with_eq=True, bounded=True):
    """Small dense-ish random LP for enumeration pins (not a UC instance)."""
    A = np.where(rng.random((m, n)) < density, rng.integers(-4, 5, (m, n)), 0).astype(float)
    for i in range(m):
        if not A[i].any():
            A[i, rng.integers(n)] = 1.0
    kind = (rng.random(m) < 0.6).astype(np.uint8) if with_eq else np.ones(m, np.uint8)
    b = rng.integers(-5, 6, m).astype(float)
    c = rng.integers(-5, 6, n).astype(float)
    lo = np.where(rng.random(n) < 0.8, rng.integers(-3, 1, n).astype(float), -np.inf)
    hi = np.where(rng.random(n) < (0.9 if bounded else 0.3),
                  lo + rng.integers(0, 5, n), np.inf)
    hi = np.where(np.isfinite(lo), hi, np.where(rng.random(n) < 0.5, rng.integers(0, 4, n).astype(float), np.inf))
    return A, kind, b, c, lo, hi


def dense_to_lp(A, kind, b, c, lo, hi) -> UCLP:
    m, n = A.shape
    rp = [0]
    ci, vv = [], []
    for i in range(m):
        nz = np.nonzero(A[i])[0]
        ci += list(nz)
        vv += list(A[i, nz])
        rp.append(len(ci))
    return UCLP(m, n, np.array(rp, np.int32), np.array(ci, np.int32),
                np.array(vv, np.float64), np.asarray(kind, np.uint8),
                np.asarray(b, float), np.asarray(c, float),
                np.asarray(lo, float), np.asarray(hi, float), {})


def scipy_csr(lp: UCLP):
    import scipy.sparse as sp
    return sp.csr_matrix((lp.val, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))


def describe(lp: UCLP) -> str:
    return f"m={lp.m} n={lp.n} nnz={lp.nnz}"


if __name__ == "__main__":
    import sys
    import time
    for name in sys.argv[1:] or list(WORKLOADS):
        t0 = time.time()
        lp = workload(name)
        print(name, describe(lp), f"{time.time() - t0:.2f}s")
