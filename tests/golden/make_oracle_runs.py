"""Write tests/golden/oracle_runs.json: the FP64 oracle's own restarted PDHG
solve of a seeded workload to a relative KKT tolerance (attempts, objectives,
KKT measures by the oracle's checker), the CPU counterpart of a GPU solve.

Runs only the oracle package on the seeded generator's instances; the
paper-scale LP takes about an hour on one core.
Usage: python tests/golden/make_oracle_runs.py [--tol 1e-4] [names]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2512_06715_amd import ucgen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_runs.json")


def main(args):
    tol = 1e-4
    if args[:1] == ["--tol"]:
        tol, args = float(args[1]), args[2:]
    for name in args or ["uc6717_t96"]:
        lp = ucgen.workload(name)
        t0 = time.time()
        x, y, info = oracle.pdhg(lp, tol=tol, max_iter=1000000)
        k = oracle.kkt(lp, x, y)
        runs = json.load(open(OUT)) if os.path.exists(OUT) else {}
        runs[f"{name}@{tol:g}"] = dict(
            workload=name, tol=tol, seconds=round(time.time() - t0, 1),
            info={key: (float(v) if hasattr(v, "__float__") else v) for key, v in info.items()},
            kkt={key: float(v) for key, v in k.items()},
            solver="oracle.pdhg (FP64, CPU), checked by oracle.kkt")
        print(name, runs[f"{name}@{tol:g}"], flush=True)
        json.dump(runs, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
