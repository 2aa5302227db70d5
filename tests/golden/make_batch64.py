"""Writes batch64_oracle.json: the CPU oracle's Algorithm 2 (defaults, tol 1e-6, at most 60 outer iterations) on
the 64 problems of the uneven batch workload (seeds 0..63 of 'batch'): status, iterations, estimate, residual
and the residual history.  Calls only the oracle and the seeded input generator.

    python tests/golden/make_batch64.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import kot_oracle as ko  # noqa: E402
from paper_2310_14087_amd.inputs import make_problem  # noqa: E402

MAX_ITER = 60


def main():
    out = []
    t0 = time.time()
    for s in range(64):
        p = make_problem("batch", s)
        core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
        r = ko.solve(core, ko.Params(tol=p.tol, max_iter=MAX_ITER))
        out.append(dict(seed=s, l=p.l, n=p.n_src, d=p.d, status=r["status"], iters=r["iters"], ot=r["ot"],
                        residual=r["residual"], history=[h["res"] for h in r["history"]]))
        print(f"seed {s} l={p.l} d={p.d} {r['status']} it={r['iters']} res={r['residual']:.3e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch64_oracle.json"), "w") as f:
        json.dump(dict(max_iter=MAX_ITER, tol=1e-6, problems=out), f, indent=0)


if __name__ == "__main__":
    main()
