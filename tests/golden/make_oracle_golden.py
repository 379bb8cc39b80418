"""Writes the oracle's results for the full-size workloads into JSON files
next to this script (tests/golden/oracle_c<N>.json).  Calls only the CPU
oracle and the seeded workload generators; the GPU tests read these files to
compare at sizes the oracle cannot run inside a test.

    python tests/golden/make_oracle_golden.py 1 2
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main(cfgs):
    for c in cfgs:
        p = W.config(int(c))
        t0 = time.perf_counter()
        r = O.run(p)
        dt = time.perf_counter() - t0
        out = dict(
            config=int(c), name=p.name, n=p.n, s=p.s, p=p.p, alpha=p.alpha, beta=p.beta,
            n_c=p.n_c, rule=p.rule, m=p.m, steps=p.steps, sigma=p.sigma, nev_b=p.nev_b,
            psi=p.psi, nev=p.nev, mu=int(r.mu), k=int(r.k), rank=int(r.rank),
            theta=[float(x) for x in r.theta], resid=[float(x) for x in r.resid],
            reference_eigs=[float(x) for x in p.exact[:p.nev + 1]],
            oracle_seconds=dt, oracle_phase_seconds=r.times,
            threads=os.environ.get("OMP_NUM_THREADS", "all"),
        )
        path = os.path.join(HERE, f"oracle_c{c}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        err = np.max(np.abs(r.theta - p.exact[:p.nev]) / p.exact[:p.nev])
        print(f"config {c}: {len(r.theta)} Ritz values, max rel err vs reference {err:.2e}, "
              f"max resid {r.resid.max():.2e}, {dt:.1f} s -> {path}")


if __name__ == "__main__":
    main(sys.argv[1:] or ["1", "2"])
