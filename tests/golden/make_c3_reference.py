"""Writes tests/golden/reference_c3.json: the interval of the 63^3 workload
and the lowest 501 eigenvalues of its pencil from the reference eigensolver
of the input recipe (ARPACK shift-invert; not RF-DDES), so that the workload
can be built without repeating that eigensolve.  Calls only the seeded
generators.

    python tests/golden/make_c3_reference.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402


def main():
    t0 = time.perf_counter()
    p = W.config(3)
    dt = time.perf_counter() - t0
    out = dict(config=3, name=p.name, n=p.n, s=p.s, p=p.p, alpha=p.alpha, beta=p.beta,
               nev=p.nev, reference_eigs=[float(x) for x in p.exact[:p.nev + 1]],
               seconds=dt)
    with open(os.path.join(HERE, "reference_c3.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"beta {p.beta} in {dt:.0f} s")


if __name__ == "__main__":
    main()
