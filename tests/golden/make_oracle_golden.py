"""Writes the oracle's results for the full-size workloads into JSON files
next to this script (tests/golden/oracle_c<N>.json).  Calls only the CPU
oracle and the seeded workload generators; the GPU tests read these files to
compare at sizes the oracle cannot run inside a test.

    python tests/golden/make_oracle_golden.py 1 2 3

The 63^3 pencil (3) runs the oracle's pole-streamed path (one pole's dense
S(zeta), 18.5 GB, at a time) at one block step with nev_b = 20, psi = 4, the
largest setting whose Rayleigh-Ritz basis fits this host's memory beside the
oracle's own work; besides the Ritz values it stores the first 16 columns of
the filtered block F Y0 (eq. (3.5)) in oracle_c3_w1.npy.
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


C3_PARAMS = dict(steps=1, nev_b=20, psi=4)
W1_COLS = 16


def main(cfgs):
    for c in cfgs:
        streamed = int(c) == 3
        if streamed:
            ref = json.load(open(os.path.join(HERE, "reference_c3.json")))
            lam = np.array(ref["reference_eigs"])
            p = W.config(3, known=(ref["alpha"], ref["beta"], lam), **C3_PARAMS)
        else:
            p = W.config(int(c))
        t0 = time.perf_counter()
        r = O.run(p, streamed=streamed)
        dt = time.perf_counter() - t0
        if streamed:
            np.save(os.path.join(HERE, "oracle_c3_w1.npy"),
                    np.ascontiguousarray(r.W1[:, :W1_COLS]))
        out = dict(
            config=int(c), name=p.name, n=p.n, s=p.s, p=p.p, alpha=p.alpha, beta=p.beta,
            n_c=p.n_c, rule=p.rule, m=p.m, steps=p.steps, sigma=p.sigma, nev_b=p.nev_b,
            psi=p.psi, nev=p.nev, mu=int(r.mu), k=int(r.k), rank=int(r.rank),
            theta=[float(x) for x in r.theta], resid=[float(x) for x in r.resid],
            reference_eigs=[float(x) for x in p.exact[:p.nev + 1]],
            oracle_seconds=dt, oracle_phase_seconds=r.times,
            threads=os.environ.get("OMP_NUM_THREADS", "all"),
            streamed=streamed, w1_cols=W1_COLS if streamed else 0,
        )
        path = os.path.join(HERE, f"oracle_c{c}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        err = np.max(np.abs(r.theta - p.exact[:p.nev]) / p.exact[:p.nev])
        print(f"config {c}: {len(r.theta)} Ritz values, max rel err vs reference {err:.2e}, "
              f"max resid {r.resid.max():.2e}, {dt:.1f} s -> {path}")


if __name__ == "__main__":
    main(sys.argv[1:] or ["1", "2"])
