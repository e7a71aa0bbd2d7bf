"""Write tests/golden/oracle_optima.json: the oracle's optimum of each seeded host workload that
the GPU tests solve at full size, computed by the oracle alone (its direct-solver FP64 IPM,
Algorithm 3 with the exact normal-equations solve, run to the stop test at gap 1e-8).

Usage: python tests/golden/make_oracle_optima.py   (several minutes on 8 cores)

Each record holds the oracle's final objective c^T x and dual objective b^T y, its stop metrics
and iteration count, and a fingerprint of the generated LP (a few entries of b and c and sums of
A's first row) so that a test can confirm it regenerated the same LP before comparing. Both the
oracle's and a GPU solve's c^T x are upper bounds of the optimum within their own gap (x
feasible to rounding), so two solves that each reach relative gap <= 1e-8 have objectives within
1e-8 relative of each other.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lpgen  # noqa: E402
from oracle import ipm as oipm  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_optima.json")

CASES = ([("dense_500x100000", s) for s in range(5)] + [("dense_500x100000_bf16", 0)]
         + [("csr_1000x1000000", 0), ("csr_5000x2000000", 0)])


def fingerprint(lp) -> dict:
    row0 = lp.A[0].toarray().ravel() if hasattr(lp.A, "toarray") else np.asarray(lp.A[0])
    return {"b": [float(v) for v in lp.b[:4]], "c": [float(v) for v in lp.c[:4]],
            "row0_sum": float(row0.sum()), "row0_abs_sum": float(np.abs(row0).sum())}


def main() -> int:
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    only = set(sys.argv[1:])
    for name, seed in CASES:
        key = f"{name}/{seed}"
        if only and key not in only:
            continue
        t0 = time.perf_counter()
        lp = lpgen.workload(name, seed=seed)
        res = oipm.solve(lp.A, lp.b, lp.c, oipm.Params(), "exact")
        last = res.infos[-1]
        rec = {"converged": bool(res.converged), "iterations": len(res.infos) - 1,
               "objective": float(lp.c @ res.state.x), "dual_objective": float(lp.b @ res.state.y),
               "relgap": last.relgap, "rp_rel": last.rp_rel, "rd_rel": last.rd_rel,
               "fingerprint": fingerprint(lp), "seconds": time.perf_counter() - t0}
        out[key] = rec
        print(f"{key}: {rec['iterations']} iterations, objective {rec['objective']:.15e}, "
              f"relgap {rec['relgap']:.2e}, {rec['seconds']:.1f} s", flush=True)
        json.dump(out, open(OUT, "w"), indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
