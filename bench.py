"""Benchmark: restarted PDHG on the 6717-bus-shaped UC LP relaxation.

One step = one full pdhg_solve from a cold start to relative KKT 1e-4 on the
seeded synthetic 6717-bus, 96-period UC LP (3.22M variables, 2.03M rows,
7.19M nonzeros), with the problem already resident in HBM, in the mixed
precision of that workload (FP32 SpMVs and iterates, FP64 reductions,
restarts, step control and polish).  value = PDHG attempts per second over
the timed solves (one attempt = one A'y and one Ax product); ms_per_step =
time to 1e-4.

Also reported on the same line: the plain FP64 solve of the same LP (time to
1e-4 and the mixed-precision speedup), batched LPs/s against the same
instances solved one at a time, the unrolled solve and adjoint of the
2000-bus differentiable case, a live HIP-event timing of the dominant kernel
against its algorithmic bytes (roofline), and the FP64 CPU oracle timed on a
bounded sample of the workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PDHG iters/s + time-to-1e-4 KKT (6717-bus UC LP); batched LPs/s; % HBM peak"
HBM_PEAK_GBS = 8000.0


def kernel_bytes(kind: str, m: int, n: int, nnz: int, vb: int, compact: bool = True) -> int:
    """Algorithmic HBM bytes of one launch (each array element moved once).

    vb = bytes per matrix value and per iterate element (8 FP64, 4 FP32).
    Structure of the matrix the launch walks (rows r, tiles of 256 rows):
    32-bit CSR: pointers 4(r+1), indices 4 nnz; 16-bit tile-relative form
    (compact): row ends 2r, indices 2 nnz, per tile its smallest index and
    its nonzero range (8 bytes).
    dual:   structure of A, values vb nnz, gather x' vb n, read y, Ax, b
            (3 vb m) and the row kind (m), write y', Ax' (2 vb m), fold the
            accepted y into the running sum (read + write, 2 vb m).
    primal: structure of A', values vb nnz, gather y vb m, read x, c, l, u
            (4 vb n), write x' (vb n), fold x into the sum (2 vb n).
    """
    def structure(r):
        return 2 * r + 8 * ((r + 255) // 256) + 2 * nnz if compact else 4 * (r + 1) + 4 * nnz
    if kind == "dual":
        return structure(m) + vb * nnz + vb * n + 3 * vb * m + m + 2 * vb * m + 2 * vb * m
    if kind == "primal":
        return structure(n) + vb * nnz + vb * m + 4 * vb * n + vb * n + 2 * vb * n
    raise ValueError(kind)


def unit_bytes(kind: str, m: int, n: int, nnz: int, vb: int) -> int:
    """The method's algorithmic bytes per unit of work as the scope table
    states them (32-bit indices, each element moved once), vb = 8 or 4:
    primal: the fused primal step, A' CSR ((4 + vb) nnz + 4(n+1)), gather y
            (vb m), stream x, c, l, u (4 vb n), write x' and one more column
            vector (2 vb n);
    dual:   the fused dual step, A CSR ((4 + vb) nnz + 4(m+1)), gather x
            (vb n), stream y, b, Ax (3 vb m), write y', Ax' (2 vb m);
    attempt: both with the Ax cache and the averages, (8 + 2 vb) nnz
            + (4 + 9 vb) n + (4 + 8 vb) m."""
    if kind == "primal":
        return (4 + vb) * nnz + 4 * (n + 1) + vb * m + 6 * vb * n
    if kind == "dual":
        return (4 + vb) * nnz + 4 * (m + 1) + vb * n + 5 * vb * m
    if kind == "attempt":
        return (8 + 2 * vb) * nnz + (4 + 9 * vb) * n + (4 + 8 * vb) * m
    raise ValueError(kind)


def merge_spmv_bytes(rows: int, gathered: int, nnz: int, vb: int) -> int:
    """Algorithmic bytes of one unfused SpMV over a 32-bit CSR matrix of
    `rows` rows: pointers 4(rows+1), indices 4 nnz, values vb nnz, the
    gathered vector vb gathered, the result vb rows."""
    return 4 * (rows + 1) + 4 * nnz + vb * nnz + vb * gathered + vb * rows


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("attempt.hip", "device.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2512_06715_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str, precision: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if source_hash() != d.get("source_hash"):
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(lp, sample_lo: int, sample_hi: int):
    """Oracle attempts/s from two capped runs (difference removes setup)."""
    import oracle
    oracle.build()
    t0 = time.perf_counter()
    oracle.pdhg(lp, tol=1e-4, max_iter=sample_lo)
    t1 = time.perf_counter()
    oracle.pdhg(lp, tol=1e-4, max_iter=sample_hi)
    t2 = time.perf_counter()
    per_attempt = ((t2 - t1) - (t1 - t0)) / (sample_hi - sample_lo)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(value=1.0 / per_attempt, unit="attempts/s", cores=1, kind="oracle",
                cpu_model=model, host_threads=os.cpu_count(),
                sample=f"FP64 oracle PDHG, {sample_hi - sample_lo} attempts "
                       f"(runs capped at {sample_lo} and {sample_hi} attempts, difference), "
                       f"same LP, single thread; {t2 - t0:.1f}s of CPU work")


def reference_objective(workload: str):
    """The workload's exact optimum from tests/golden/lp_refs.json, if stored."""
    path = os.path.join(ROOT, "tests", "golden", "lp_refs.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        refs = json.load(f)
    r = refs.get(workload)
    return r["objective"] if r and r.get("status") == "optimal" else None


def oracle_run(workload: str, tol: float):
    """The FP64 oracle's own solve of the workload to the same tolerance, if
    stored (tests/golden/oracle_runs.json, written by make_oracle_runs.py)."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_runs.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        runs = json.load(f)
    return runs.get(f"{workload}@{tol:g}")


def fp64_compare(lp, args):
    """One cold FP64 solve of the same LP on the device (for the speedup)."""
    import torch
    from paper_2512_06715_amd.solver import Problem
    p = Problem(lp, tol=args.tol, max_iter=args.max_iter, precision="fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, info = p.solve()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    p.close()
    return dict(fp64_time_to_tol_s=round(dt, 3), fp64_attempts=info["attempts"],
                fp64_primal_obj=info["primal_obj"],
                fp64_attempts_per_s=round(info["attempts"] / dt, 1),
                fp64_rel_kkt=info["rel_kkt"], fp64_status=info["status_name"])


def config3_run(args):
    """The batched workload as stated: branch-and-bound variants of the
    4224-bus, 48-period LP (a random 0-20% of the commitments fixed, one
    shared matrix) and small distinct LPs (500-2000 buses, 24 periods), all in
    one batched solve, mixed precision, KKT 1e-4 each, autotuned SpMV
    partitions.  Sequential is the same library solving the instances one at a
    time (a batch of one for a variant, pdhg_solve for a small LP), measured
    on the first `seq_sample` of each kind and scaled to all of them."""
    import numpy as np
    import torch
    from paper_2512_06715_amd import ucgen
    from paper_2512_06715_amd.solver import Problem, solve_batch
    lp = ucgen.workload("uc4224_t48")
    opts = dict(tol=args.tol, precision="mixed", max_iter=args.max_iter, autotune=1)
    # verbose: the library prints a progress line every 64 evaluations of the batch
    base = Problem(lp, verbose=1, **opts)
    smalls = [ucgen.small_batch_instance(j) for j in range(args.batch_small)]
    sp = [Problem(s_, **opts) for s_ in smalls]
    variants = []
    for k in range(args.batch_big):
        v = ucgen.fix_commitments(lp, seed=100 + k)
        variants.append(dict(base=0, fix_idx=v.meta["fix_idx"], fix_val=v.meta["fix_val"]))
    insts = variants + [dict(base=1 + j) for j in range(len(smalls))]
    print(f"[bench] batch of {len(insts)} ({len(variants)} variants of uc4224_t48, "
          f"{len(smalls)} small LPs) ...", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = solve_batch([base] + sp, insts)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    base.close()
    att = [r[2]["attempts"] for r in res]
    ok = sum(1 for r in res if r[2]["status"] == 1)
    print(f"[bench] batch: {tb:.1f}s, {ok} of {len(insts)} solved; sequential sample ...",
          file=sys.stderr, flush=True)
    seq = Problem(lp, **opts)   # the same base without progress lines
    t_big, t_small = [], []
    for d in variants[:args.seq_sample]:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        solve_batch([seq], [d])
        torch.cuda.synchronize()
        t_big.append(time.perf_counter() - t1)
    for p in sp[:args.seq_sample]:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p.solve()
        torch.cuda.synchronize()
        t_small.append(time.perf_counter() - t1)
    seq.close()
    for p in sp:
        p.close()
    est = len(variants) * float(np.mean(t_big or [0.0])) + len(smalls) * float(np.mean(t_small or [0.0]))
    nv = len(variants)
    return dict(
        workload="%d branch-and-bound variants of uc4224_t48 (4224 buses, 700 units, 5800 "
                 "lines, 48 periods; 0-20%% of the commitments fixed) and %d distinct LPs of "
                 "500-2000 buses (24 periods), one batched solve, mixed, KKT %g, autotuned "
                 "partitions" % (nv, len(smalls), args.tol),
        instances=len(insts), solved=ok, batch_s=round(tb, 3), lps_per_s=round(len(insts) / tb, 4),
        sequential_s_estimate=round(est, 3),
        sequential_lps_per_s=round(len(insts) / est, 4) if est > 0 else None,
        speedup=round(est / tb, 3) if est > 0 else None,
        sequential_sample="%d variants (%.2f s mean) and %d small LPs (%.2f s mean) solved one at "
                          "a time, scaled to %d and %d" % (len(t_big), float(np.mean(t_big or [0])),
                                                           len(t_small), float(np.mean(t_small or [0])),
                                                           nv, len(smalls)),
        attempts_variants_mean=round(float(np.mean(att[:nv])), 1) if nv else None,
        attempts_small_mean=round(float(np.mean(att[nv:])), 1) if smalls else None,
        attempts_max=int(max(att)), us_per_instance_attempt=round(1e6 * tb / sum(att), 3))


def nodes_run(args):
    """Branch-and-bound nodes of the 4224-bus, 48-period LP: the root is
    solved, then the children of its K most fractional commitments (each
    fixed to 0 and to 1, 2K nodes) are solved as one batch, warm-started from
    the root's point, primal weight and step size (in mixed precision, and
    in FP64 on a second handle of the same LP); for comparison from the
    point alone, and cold.  Reports the time, attempts and the safe bound's
    distance below each child's objective."""
    import numpy as np
    import torch
    from paper_2512_06715_amd import nodes as N, ucgen
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc4224_t48")
    prob = Problem(lp, tol=args.tol, precision="mixed", max_iter=args.max_iter)
    ucols = lp.meta["u_cols"].ravel()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    root = N.solve_nodes(prob, [N.root()])[0]
    t_root = time.perf_counter() - t0
    picks = N.most_fractional(root, ucols, k=args.nodes)
    out = dict(workload="children of the %d most fractional commitments of the root of "
                        "uc4224_t48 (4224 buses, 700 units, 5800 lines, 48 periods), "
                        "mixed, KKT %g" % (len(picks), args.tol),
               root_s=round(t_root, 3), root_attempts=root.info["attempts"],
               root_gap=(root.objective - root.bound) / abs(root.objective))
    prob64 = Problem(lp, tol=args.tol, precision="fp64", max_iter=args.max_iter)
    for mode in ("warm", "warm_fp64", "warm_point_only", "cold"):
        kids = [k for j in picks for k in N.branch(root, int(j))]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        N.solve_nodes(prob64 if mode == "warm_fp64" else prob, kids, warm=mode != "cold",
                      weights=mode in ("warm", "warm_fp64"))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        gaps = np.array([(k.objective - k.bound) / abs(k.objective) for k in kids])
        att = [k.info["attempts"] for k in kids]
        out[mode] = dict(
            nodes=len(kids), solved=sum(k.info["status"] == 1 for k in kids),
            batch_s=round(dt, 3), nodes_per_s=round(len(kids) / dt, 3),
            attempts_mean=round(float(np.mean(att)), 1), attempts_max=int(max(att)),
            attempts_fp32_mean=round(float(np.mean([k.info["attempts_fp32"] for k in kids])), 1),
            bound_gap_median=float(np.median(gaps)), bound_gap_max=float(gaps.max()),
            bounds_finite=int(np.isfinite([k.bound for k in kids]).sum()))
    # an infeasible child: the penalty slacks and every unit of period 5
    # fixed to 0 (the load of that period cannot be met); fixings keep the
    # base's implied bounds, which the certificate needs for the bus angles
    n_unit, n_bus, n_line = 700, 4224, 5800
    pos = np.arange(lp.n) % (4 * n_unit + 3 * n_bus + n_line + 1)
    cols = np.concatenate([np.nonzero(pos >= 4 * n_unit + n_bus + n_line)[0],
                           lp.meta["u_cols"][5]])
    bad = N.Node(cols.astype(np.int32), np.zeros(len(cols)), 1, x0=root.x, y0=root.y,
                 omega0=float(root.info["omega"]), eta0=float(root.info["eta"]),
                 hold=int(root.info["attempts"]))
    for mode in ("warm", "cold"):
        nd = N.Node(bad.fix_idx, bad.fix_val)
        if mode == "warm":
            nd = bad
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        N.solve_nodes(prob, [nd], warm=mode == "warm")
        torch.cuda.synchronize()
        out["infeasible_child_" + mode] = dict(
            status=nd.info["status_name"], attempts=nd.info["attempts"],
            seconds=round(time.perf_counter() - t0, 3))
    prob.close()
    prob64.close()
    out["warm_speedup"] = round(out["cold"]["batch_s"] / out["warm"]["batch_s"], 3)
    out["warm_fp64_speedup"] = round(out["cold"]["batch_s"] / out["warm_fp64"]["batch_s"], 3)
    return out


def polish_run(args, p, x, y, info):
    """Feasibility polishing of the last timed solve's point (pdhg_polish to
    relative residuals 100 times below the solve's tolerance): its time and
    the residuals before and after."""
    import torch
    ptol = args.tol / 100
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, pi = p.polish(x, y, tol=ptol, omega=info["omega"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dict(workload="%s, the timed solve's point (KKT %g), polished to relative residuals "
                         "%g" % (args.workload, args.tol, ptol),
                seconds=round(dt, 3), attempts=pi["attempts"],
                before=dict(rel_primal=info["rel_primal"], rel_dual=info["rel_dual"],
                            rel_gap=info["rel_gap"], primal_obj=info["primal_obj"]),
                after=dict(rel_primal=pi["rel_primal"], rel_dual=pi["rel_dual"],
                           rel_gap=pi["rel_gap"], primal_obj=pi["primal_obj"],
                           dual_bound=pi["dual_bound"]))


def tol_sweep(args, dev_lp):
    """Attempts and time to relative KKT 1e-3 ... 1e-6 on the benched LP in both
    precisions (cold starts; each solve capped at args.sweep_max_iter
    attempts; the library prints one line per evaluation to stderr)."""
    import torch
    from paper_2512_06715_amd.solver import Problem
    out = []
    for prec in ("mixed", "fp64"):
        for tol in (1e-3, 1e-4, 1e-5, 1e-6):
            p = Problem(dev_lp, device=True, tol=tol, max_iter=args.sweep_max_iter, precision=prec,
                        verbose=1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info = p.solve()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            p.close()
            rec = dict(precision=prec, tol=tol, status=info["status_name"], seconds=round(dt, 3),
                       attempts=info["attempts"], attempts_fp32=info["attempts_fp32"],
                       rel_kkt=info["rel_kkt"], primal_obj=info["primal_obj"],
                       dual_bound=info["dual_bound"])
            print(f"[bench] sweep {json.dumps(rec)}", file=sys.stderr, flush=True)
            out.append(rec)
    return out


def adjoint_run():
    """Unrolled solve (1000 steps, checkpoints every 50) and its adjoint on the
    2000-bus, 24-period differentiable case."""
    import torch
    from paper_2512_06715_amd import ucgen
    from paper_2512_06715_amd.solver import Problem
    lp = ucgen.workload("uc2000_t24")
    p = Problem(lp, unroll_iters=1000, checkpoint_every=50)
    p.solve()
    p.backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, info = p.solve()
    t1 = time.perf_counter()
    p.backward()
    t2 = time.perf_counter()
    p.close()
    return dict(adjoint=dict(workload="uc2000_t24 (2000 buses, 300 units, 2700 lines, 24 periods)",
                             unroll_iters=1000, checkpoint_every=50,
                             forward_ms=round(1e3 * (t1 - t0), 2),
                             backward_ms=round(1e3 * (t2 - t1), 2)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uc6717_t96")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--no-compare-fp64", action="store_true")
    ap.add_argument("--batch-big", type=int, default=96,
                    help="branch-and-bound variants of the 4224-bus, 48-period LP in the "
                         "batched workload (one shared matrix)")
    ap.add_argument("--batch-small", type=int, default=32,
                    help="small distinct LPs in the batched workload (both 0 skip it)")
    ap.add_argument("--seq-sample", type=int, default=4,
                    help="instances of each kind solved one at a time for the sequential rate")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-polish", action="store_true")
    ap.add_argument("--tol-sweep", action="store_true",
                    help="also solve the benched LP to relative KKT 1e-3 ... 1e-6 in both precisions")
    ap.add_argument("--sweep-max-iter", type=int, default=1_500_000)
    ap.add_argument("--nodes", type=int, default=0,
                    help="K > 0: branch-and-bound children of the K most fractional "
                         "commitments of the 4224-bus LP's root, warm against cold")
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--max-iter", type=int, default=2_000_000)
    ap.add_argument("--kernel-attempts", type=int, default=200)
    ap.add_argument("--merge-attempts", type=int, default=100,
                    help="repetitions of the merge-path SpMV timing (0: skip)")
    ap.add_argument("--cold-attempts", type=int, default=50,
                    help="attempts timed with the caches flushed before each (0 skips)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", default="64,384")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: this solver has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2512_06715_amd import ucgen
    from paper_2512_06715_amd.solver import Problem

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {src.numel() * 8} bytes read and written per launch",
              file=sys.stderr, flush=True)
        del src, dst

    lp = ucgen.workload(args.workload)
    print(f"[bench] {args.workload}: {ucgen.describe(lp)}", file=sys.stderr, flush=True)
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).cuda()

    class DevLP:
        m, n = lp.m, lp.n
        row_ptr = dev(lp.row_ptr, torch.int32)
        col_idx = dev(lp.col_idx, torch.int32)
        val = dev(lp.val, torch.float64)
        row_kind = dev(lp.row_kind, torch.uint8)
        b = dev(lp.b, torch.float64)
        c = dev(lp.c, torch.float64)
        l = dev(lp.l, torch.float64)
        u = dev(lp.u, torch.float64)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob = Problem(DevLP, device=True, tol=args.tol, max_iter=args.max_iter,
                   precision=args.precision)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print(f"[bench] setup {setup_s:.3f}s", file=sys.stderr, flush=True)

    for w in range(args.warmup):
        _, _, info = prob.solve()
        print(f"[bench] warmup {w}: {info['attempts']} attempts, {info['solve_s']:.2f}s, "
              f"{info['status_name']}", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for s in range(args.steps):
        xs, ys, info = prob.solve()
        infos.append(info)
        print(f"[bench] step {s}: {info['attempts']} attempts, {info['solve_s']:.2f}s, "
              f"{info['status_name']} kkt={info['rel_kkt']:.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    attempts = sum(i["attempts"] for i in infos)

    # live per-kernel timing on the library stream (warm: the solve's own
    # operating point), then with L2 and the Infinity Cache flushed
    kt = prob.time_kernels(args.kernel_attempts)
    compact = bool(prob.partition()["compact"])
    vb = 8 if args.precision == "fp64" else 4
    dom = "dual" if kt["dual"] >= kt["primal"] else "primal"
    ubytes = unit_bytes(dom, lp.m, lp.n, lp.nnz, vb)
    nbytes = kernel_bytes(dom, lp.m, lp.n, lp.nnz, vb, compact)
    achieved = ubytes / (kt[dom] * 1e-3) / 1e9
    attempt_unit = unit_bytes("attempt", lp.m, lp.n, lp.nnz, vb)
    attempt_bytes = sum(kernel_bytes(k, lp.m, lp.n, lp.nnz, vb, compact) for k in ("primal", "dual"))
    kname = f"k_{dom}"

    def frac(b, ms):
        return round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=load_traffic(kname, args.workload, args.precision),
                    kernel=kname, ms_per_launch=round(kt[dom], 5),
                    algorithmic_bytes_per_launch=ubytes,
                    bytes_unit="fused step with 32-bit indices (bench.unit_bytes)",
                    moved=dict(bytes_per_launch=nbytes, frac=frac(nbytes, kt[dom]),
                               index_form="16-bit tile-relative" if compact else "32-bit CSR",
                               note="the bytes this kernel has to move in its own storage "
                                    "form (bench.kernel_bytes)"),
                    other_kernel=dict(
                        kernel="k_dual" if dom == "primal" else "k_primal",
                        frac=frac(unit_bytes("dual" if dom == "primal" else "primal",
                                             lp.m, lp.n, lp.nnz, vb),
                                  kt["dual" if dom == "primal" else "primal"])),
                    kernel_ms=dict((k, round(v, 5)) for k, v in kt.items()),
                    attempt=dict(algorithmic_bytes=attempt_unit, ms=round(kt["attempt"], 5),
                                 frac=frac(attempt_unit, kt["attempt"]),
                                 moved_bytes=attempt_bytes,
                                 moved_frac=frac(attempt_bytes, kt["attempt"]),
                                 note="a whole attempt with the Ax cache and averages over "
                                      "its duration (step control and launch gaps included)"))
    if args.merge_attempts > 0:
        # the merge-path SpMV on the same scaled (and reordered) matrices, in
        # the iteration precision: a load-balanced, unfused alternative
        km = prob.time_spmv_merge(args.merge_attempts)
        mb = dict(transpose=merge_spmv_bytes(lp.n, lp.m, lp.nnz, vb),
                  forward=merge_spmv_bytes(lp.m, lp.n, lp.nnz, vb))
        roofline["spmv_merge"] = dict(
            (k, dict(ms=round(km[k], 5), algorithmic_bytes=mb[k],
                     frac=round(mb[k] / (km[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)))
            for k in ("transpose", "forward"))
        roofline["spmv_merge"]["note"] = ("y = A x alone (no fused update), 32-bit CSR, plan "
                                          "made once; transpose = the primal kernel's A'y")
    if args.cold_attempts > 0:
        kc = prob.time_kernels_cold(args.cold_attempts)
        roofline["cold"] = dict(
            kernel_ms=dict((k, round(v, 5)) for k, v in kc.items()),
            frac=frac(ubytes, kc[dom]), moved_frac=frac(nbytes, kc[dom]),
            note="1 GiB read between attempts evicts L2 and the 256 MB Infinity Cache")
    extra = {}
    if args.tol_sweep:
        extra["tol_sweep"] = tol_sweep(args, DevLP)
    if not args.no_polish:
        print("[bench] feasibility polish ...", file=sys.stderr, flush=True)
        extra["polish"] = polish_run(args, prob, xs, ys, infos[-1])
    prob.close()
    del DevLP

    if not args.no_compare_fp64 and args.precision == "mixed":
        print("[bench] plain FP64 solve of the same LP ...", file=sys.stderr, flush=True)
        extra.update(fp64_compare(lp, args))
    if args.batch_big > 0 or args.batch_small > 0:
        extra["batch"] = config3_run(args)
    if args.nodes > 0:
        print("[bench] branch-and-bound nodes ...", file=sys.stderr, flush=True)
        extra["nodes"] = nodes_run(args)
    if not args.no_adjoint:
        print("[bench] unrolled solve + adjoint ...", file=sys.stderr, flush=True)
        extra.update(adjoint_run())

    cpu = None
    if not args.no_cpu_baseline:
        lo, hi = (int(v) for v in args.cpu_sample.split(","))
        print("[bench] cpu baseline ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(lp, lo, hi)

    if "fp64_time_to_tol_s" in extra:
        extra["mixed_speedup_vs_fp64"] = round(extra["fp64_time_to_tol_s"] / (elapsed / args.steps), 3)
    last = infos[-1]
    ref = reference_objective(args.workload)
    extra["objective_error"] = dict(
        reference=ref, source="tests/golden/lp_refs.json (HiGHS through the oracle package)",
        relative=(abs(last["primal_obj"] - ref) / abs(ref)) if ref is not None else None,
        fp64_relative=(abs(extra["fp64_primal_obj"] - ref) / abs(ref))
        if ref is not None and "fp64_primal_obj" in extra else None,
        dual_bound_gap=(last["primal_obj"] - last["dual_bound"]) / abs(last["primal_obj"]))
    orc = oracle_run(args.workload, args.tol)
    if orc is not None:
        o = orc["info"]["pobj"]
        extra["objective_error"]["oracle_same_tol"] = dict(
            objective=o, attempts=orc["info"]["attempts"], rel_kkt=orc["kkt"]["rel_kkt"],
            relative=abs(last["primal_obj"] - o) / abs(o),
            fp64_relative=(abs(extra["fp64_primal_obj"] - o) / abs(o))
            if "fp64_primal_obj" in extra else None,
            note="the oracle's own FP64 solve to the same tolerance (another trajectory: "
                 "both points are within the tolerance, not the same point)")
    out = dict(
        metric=METRIC,
        value=round(attempts / elapsed, 1),
        unit="attempts/s",
        n_gpus=1,
        steps=args.steps,
        warmup=args.warmup,
        ms_per_step=round(1e3 * elapsed / args.steps, 2),
        higher_is_better=True,
        scaling="weak",
        vs_baseline=None,
        dtype="f64" if args.precision == "fp64" else "f32+f64",
        data="synthetic",
        config=dict(workload=f"{args.workload} (seeded DC-UC LP relaxation, 6717 buses, "
                             f"1100 units, 9000 lines, 96 periods)",
                    m=lp.m, n=lp.n, nnz=lp.nnz, tol=args.tol, precision=args.precision),
        time_to_tol_s=round(elapsed / args.steps, 3),
        attempts_per_solve=last["attempts"],
        attempts_fp32=last.get("attempts_fp32"),
        status=last["status_name"],
        rel_kkt=last["rel_kkt"],
        primal_obj=last["primal_obj"],
        setup_s=round(setup_s, 3),
        **extra,
        roofline=roofline,
        cpu_baseline=cpu,
    )
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
