"""Write tests/golden/lp_refs.json: exact LP optima of the seeded workloads.

Runs only the oracle package (scipy's HiGHS through oracle.exact.highs) on the
seeded generator's instances.
Usage: python tests/golden/make_refs.py [--method highs|highs-ds|highs-ipm] [names]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402
from paper_2512_06715_amd import ucgen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lp_refs.json")


def main(args):
    method = "highs"
    if args[:1] == ["--method"]:
        method, args = args[1], args[2:]
    names = args or ["uc14_t24", "uc1000_t48", "uc2000_t24"]
    for name in names:
        lp = ucgen.workload(name)
        t0 = time.time()
        st, x, obj, y = exact.highs(lp, method=method)
        # re-read just before writing: several runs may fill the file in turn
        refs = json.load(open(OUT)) if os.path.exists(OUT) else {}
        refs[name] = dict(status=st, objective=obj, m=lp.m, n=lp.n, nnz=lp.nnz,
                          solver=f"HiGHS (scipy.optimize.linprog, method='{method}')",
                          seconds=round(time.time() - t0, 1))
        print(name, refs[name], flush=True)
        json.dump(refs, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
