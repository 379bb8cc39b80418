"""Benchmark of the RF-DDES path on one MI355X.

Headline (one JSON line on stdout): a step is one complete solve of the 3D
63^3 pencil with diagonal random M (n = 250047, 64 subdomains of 15^3,
interface s = 34047 split into 8 octant groups and the 11719-node central
separator, the lowest 500 eigenvalues, 8 Gauss-Legendre poles, block of 700,
4 block-Krylov steps, nev_b = 40, psi = 4): every factorization is
recomputed (caches invalidated), then filter_interface, solve_interior and
rayleigh_ritz with eigenvectors and residuals.  The pencil and the starting
block are resident on the device before the timed region.  A Ritz value
counts when it lies within 1e-10 (relative) of the reference eigenvalue of
the same rank (tests/golden/reference_c3.json); the count that also asks
for a residual ||Ax - theta Mx|| / (||A|| ||x||) <= 1e-9 is reported beside
it.  Three precision modes run: a precision per factor, FP32 with FP64
refinement to the 1e-10 target where that costs less than FP64
(RFD_FP32_AUTO; the value: at 63^3 every factor comes out FP64, the
interior blocks because their Schur solves then run on trailing blocks;
the batched 2D pencils take FP32 interior blocks), every factor in FP32
with FP64 refinement (RFD_FP32_REFINE, beside it) and plain FP64 (beside
it).

Beside the headline:
  spectral -- the same pencil with the spectral interior path (one
              eigendecomposition of every subdomain block, Sec. 4.1): a first
              solve that computes it and a solve on the stored decomposition,
              both modes;
  c2       -- the 2D 255x255 pencil (n = 65025, 64 subdomains, 200
              eigenvalues, 5 block steps, nev_b 40, psi 6), both modes,
              counted against the oracle's stored Ritz values
              (tests/golden/oracle_c2.json) and the residual target;
  batched  -- the 256 pencils of the batched workload (variable coefficient,
              random M, uneven sizes) run as one rfd_batch_run on several
              worker streams in FP32+refine (RFD_FP32_AUTO), against the
              same jobs on one worker, with every factor FP32, and in plain
              FP64;
  serving  -- a seeded Poisson stream of spectrum-slicing requests on the
              31x31, 255x255 and 63^3 pencils (weights 0.6 / 0.3 / 0.1),
              replayed at 0.5x and 0.8x the measured saturated rate: p50 /
              p99 latency, throughput, cache hits and evictions;
  roofline -- the hand-written kernel with the most summed time over the
              timed steps and, as roofline_mfma, the matrix-core GEMM with the
              most summed time beside it, each timed per launch with HIP
              events stamped by the launch;
  cpu_baseline -- the CPU oracle on a bounded sample of the 63^3 workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode fp32|fp64|fp32all|both|all]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_MFMA_PEAK = 157.3   # TFLOP/s, dense FP32 matrix
FP64_PEAK = 78.6         # TFLOP/s, dense FP64 (matrix and vector)
HBM_PEAK = 8000.0        # GB/s
TARGET_TOL = 1e-10       # refinement tolerance matching the accuracy target
ACCOUNT_EVERY = 8        # kernel timing samples every 8th launch of each kernel


def rule_of(R, prob):
    return R.RFD_RULE_GAUSS if prob.rule == "gauss" else R.RFD_RULE_MIDPOINT


def make_pencil(R, W, prob, mode, refine_tol=0.0, spectral=False):
    P = R.Pencil(prob.A, prob.M)
    P.set_partition(prob.part)
    groups = W.interface_groups(prob.grid, prob.meta["P"])
    if groups is not None:
        P.set_interface_groups(groups)
    if spectral:
        P.set_interior_solver(R.RFD_INTERIOR_SPECTRAL)
    P.set_interval_and_poles(prob.alpha, prob.beta, prob.n_c, rule_of(R, prob))
    P.set_precision({"fp32": R.RFD_FP32_AUTO, "fp32all": R.RFD_FP32_REFINE}.get(mode, R.RFD_FP64),
                    refine_tol)
    return P


def one_step(P, prob, Y0):
    P.reset_caches(False)
    # V_j and the B_sigma factors do not depend on Q: they run beside the filter
    P.prepare_interior(prob.sigma, prob.nev_b)
    P.filter_interface(Y0, prob.steps)
    k = P.solve_interior(prob.sigma, prob.nev_b, prob.psi)
    ev, X, r = P.rayleigh_ritz(prob.nev + 50)
    return ev, r, k


RESID_TARGET = 1e-9


def count_good(th, ref, resid=None, tol=1e-10):
    """Reference eigenvalues matched by a Ritz value within tol (relative),
    pairing the two ascending lists in order (a Ritz value serves one
    eigenvalue); the same count restricted to pairs whose residual is at most
    RESID_TARGET; and the largest relative error when the counts agree."""
    order = np.argsort(th)
    th, ref = th[order], np.sort(ref)
    rs = None if resid is None else np.asarray(resid)[order]
    i = j = good = strict = 0
    while i < ref.size and j < th.size:
        if abs(th[j] - ref[i]) <= tol * abs(ref[i]):
            good += 1
            if rs is not None and rs[j] <= RESID_TARGET:
                strict += 1
            i += 1
            j += 1
        elif th[j] < ref[i]:
            j += 1
        else:
            i += 1
    err = float(np.max(np.abs(th - ref) / np.abs(ref))) if th.size == ref.size and th.size else float("inf")
    return good, strict, err


def run_mode(R, W, prob, mode, steps, warmup, ref, torch, refine_tol, account):
    P = make_pencil(R, W, prob, mode, refine_tol)
    Y0 = torch.from_numpy(np.ascontiguousarray(prob.Y0.T)).cuda()
    for _ in range(warmup):
        one_step(P, prob, Y0)
    torch.cuda.synchronize()
    P.set_timing(True)
    P.phase_times()                        # clear
    if account:
        R.rfd_kernel_accounting(ACCOUNT_EVERY)
        R.rfd_kernel_stats()               # clear
    lat, outs, good, strict, errs, res = [], [], [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        ev, r, k = one_step(P, prob, Y0)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        outs.append((ev, r))               # checked after the timed region
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    for ev, r in outs:
        rr = r.cpu().numpy()
        g, gs, e = count_good(ev.cpu().numpy(), ref, rr)
        good.append(g)
        strict.append(gs)
        errs.append(e)
        res.append(float(rr.max()) if rr.size else 0.0)
    kstats = None
    if account:
        kstats = R.rfd_kernel_stats()
        R.rfd_kernel_accounting(0)
    ph = P.phase_times() / steps
    P.close()
    del Y0, outs
    torch.cuda.empty_cache()
    return dict(total=total, lat=lat, good=good, strict=strict, errs=errs, resid=res, phases=ph,
                k=k, kstats=kstats, steps=steps)


def summary(r, prob):
    sps = r["total"] / r["steps"]
    lat = np.array(r["lat"]) * 1e3
    return {"value": min(r["good"]) / sps, "eigenpairs": min(r["good"]),
            "value_resid_1e-9": min(r["strict"]) / sps, "eigenpairs_resid_1e-9": min(r["strict"]),
            "ms_per_step": 1e3 * sps, "steps": r["steps"],
            "latency_ms": {"p50": float(np.percentile(lat, 50)),
                           "p99": float(np.percentile(lat, 99))},
            "max_rel_err": max(r["errs"]), "max_resid": max(r["resid"]), "rr_columns": r["k"],
            "phases_ms": np.round(r["phases"][:12], 2).tolist(),
            "refinement_sweeps": r["phases"][12:14].tolist()}


# ---------------------------------------------------------------------------
# roofline entries
# ---------------------------------------------------------------------------
# HBM traffic per launch measured with rocprofv3 (FETCH_SIZE and WRITE_SIZE,
# scaled by a plain copy of known size) is kept in profiles/ together with
# the workload it was measured on and the hash of the source file the kernel
# lives in; it is reported only for that workload while that source is
# unchanged.
PROFILE_OF = {"k_tri_symv": ("tri_symv_63cube.md", "eig.hip"),
              "k_dgemm<false, true, false>": ("dgemm_tn_63cube.md", "gemm.hip"),
              "k_dgemm<false, false, false>": ("dgemm_nn_63cube.md", "gemm.hip"),
              "k_dgemm<true, false, false>": ("dgemm_c_nn_63cube.md", "gemm.hip")}


def measured_traffic(kname, workload):
    import hashlib
    import re
    if kname not in PROFILE_OF:
        return None
    prof, src = PROFILE_OF[kname]
    path = os.path.join(ROOT, "profiles", prof)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m1 = re.search(r"traffic_bytes_per_launch\s*=\s*([0-9.eE+]+)", txt)
    m2 = re.search(r"source_sha256\s*=\s*([0-9a-f]{64})", txt)
    m3 = re.search(r"workload\s*=\s*(.+)", txt)
    if not (m1 and m2 and m3) or m3.group(1).strip() != workload:
        return None
    cur = hashlib.sha256(open(os.path.join(ROOT, "paper_1711_09487_amd", "csrc", src),
                              "rb").read()).hexdigest()
    return float(m1.group(1)) if cur == m2.group(1) else None


def roofline_entry(kname, st, f32, steps, workload):
    # ms, flops and bytes: estimates over all launches of the timed steps
    launches, sampled, ms, flops, byts = st
    if kname == "k_tri_symv":
        achieved = byts / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        e = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK, "unit": "GB/s",
             "kernel": "k_tri_symv (trailing-block mat-vec of the Householder tridiagonalization)"}
    else:
        peak = FP32_MFMA_PEAK if "float" in kname else FP64_PEAK
        rate = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        e = {"bound": "mfma", "peak": peak, "unit": "TFLOP/s",
             "kernel": f"{kname} (LU updates, triangular solves, products)"}
        if "float, true" in kname or kname.startswith("k_dgemm<true"):
            # Gauss's three real products: 6 flops per complex multiply-add run
            # on the matrix cores; the 8-flop rate is the effective one
            e["achieved"] = 0.75 * rate
            e["achieved_effective_8_flops_per_complex_fma"] = rate
            e["flops_counted"] = ("executed: 6 per complex multiply-add (three real products); "
                                  "the effective rate counts 8")
        else:
            e["achieved"] = rate
    e["frac"] = e["achieved"] / e["peak"]
    e["traffic"] = measured_traffic(kname, workload)
    e["launches_per_step"] = launches / steps
    e["timed_launches"] = sampled
    e["avg_launch_us"] = 1e3 * ms / max(launches, 1)
    e["algorithmic_bytes_per_launch"] = byts / max(launches, 1)
    e["flops_per_launch"] = flops / max(launches, 1)
    return e


# ---------------------------------------------------------------------------
# spectral interior path
# ---------------------------------------------------------------------------
def spectral_leg(R, W, prob, ref, torch, refine_tol, modes):
    """The headline pencil with rfd_set_interior_solver(SPECTRAL), per mode:
    a first solve that computes the eigendecomposition of every subdomain
    block, then a solve on the stored decomposition (the pencil-level cache a
    served pencil keeps between requests; everything that depends on the
    interval or sigma is recomputed)."""
    out = {}
    Y0 = torch.from_numpy(np.ascontiguousarray(prob.Y0.T)).cuda()
    for mode in modes:
        P = make_pencil(R, W, prob, mode, refine_tol, spectral=True)
        P.set_timing(True)
        rows = []
        for first in (True, False):
            P.reset_caches(first)
            P.phase_times()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev, r, k = one_step(P, prob, Y0)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ph = P.phase_times()
            rr = r.cpu().numpy()
            g, gs, e = count_good(ev.cpu().numpy(), ref, rr)
            rows.append(dict(seconds=dt, eigenpairs=g, eigenpairs_resid_1e_9=gs, max_rel_err=e,
                             max_resid=float(rr.max()) if rr.size else 0.0,
                             decomposition_ms=float(ph[6]), phases_ms=np.round(ph[:12], 1).tolist()))
        P.close()
        torch.cuda.empty_cache()
        a, b = rows
        out[mode] = {"first_solve": a, "stored_decomposition": b,
                     "value_stored": b["eigenpairs"] / b["seconds"],
                     "value_first": a["eigenpairs"] / a["seconds"]}
        print(f"# spectral {mode}: first {a['seconds']:.2f} s (decomposition "
              f"{a['decomposition_ms']:.0f} ms), stored {b['seconds']:.2f} s, good "
              f"{b['eigenpairs']}/{prob.nev}, max rel err {b['max_rel_err']:.2e}",
              file=sys.stderr, flush=True)
    del Y0
    return out


# ---------------------------------------------------------------------------
# batched leg
# ---------------------------------------------------------------------------
# parameters of the batched pencils: with 4-8 poles and m = 1.5 nev the
# interface block needs 5 block steps (3 or 4 leave up to 1e-9 on pencils cut
# 3 x 3); nev_b 30, psi 4 then reach 1e-10 (checked on the oracle)
BATCH_NEV_B, BATCH_PSI, BATCH_STEPS = 30, 4, 5


def batch_leg(R, W, torch, count, workers):
    """The batched workload as rfd_batch_run calls: FP32+refine on `workers`
    streams (the value) and on one stream, and plain FP64 on `workers`
    streams beside it."""
    specs = W.batch_specs(count)
    probs = [W.batch_problem(b, sp, nev_b=BATCH_NEV_B, psi=BATCH_PSI, steps=BATCH_STEPS)
             for b, sp in enumerate(specs)]
    pens = []
    for prob in probs:
        P = R.Pencil(prob.A, prob.M)
        P.set_partition(prob.part)
        pens.append(P)
    y0 = [torch.from_numpy(np.ascontiguousarray(pr.Y0.T)).cuda() for pr in probs]

    def jobs(mode):
        return [R.Job(P, pr.alpha, pr.beta, pr.n_c, y, pr.steps, pr.sigma, pr.nev_b, pr.psi,
                      pr.nev + 30, mode=mode, rule=rule_of(R, pr),
                      refine_tol=TARGET_TOL if mode != R.RFD_FP64 else 0.0)
                for P, pr, y in zip(pens, probs, y0)]

    R.batch_run(jobs(R.RFD_FP32_AUTO), workers=workers)   # first use: maps, reordered matrices
    out = {}
    for key, mode, w in (("fp32", R.RFD_FP32_AUTO, workers), ("fp32_1", R.RFD_FP32_AUTO, 1),
                         ("fp32all", R.RFD_FP32_REFINE, workers), ("fp64", R.RFD_FP64, workers)):
        js = jobs(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R.batch_run(js, workers=w)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        good = found = 0
        for j, pr in zip(js, probs):
            ev = j.outputs()[0].cpu().numpy()
            found += ev.size
            g, _, _ = count_good(ev, pr.exact[:pr.nev])
            good += g
        out[key] = dict(wall=wall, good=good, found=found)
        del js
    for P in pens:
        P.close()
    b, s1, d, a32 = out["fp32"], out["fp32_1"], out["fp64"], out["fp32all"]
    return {"pencils": count, "workers": workers, "eigenpairs": b["good"],
            "eigenpairs_wanted": int(sum(pr.nev for pr in probs)),
            "eigenpairs_found": b["found"], "value": b["good"] / b["wall"],
            "unit": "eigenpairs/s", "wall_s": b["wall"], "one_worker_value": s1["good"] / s1["wall"],
            "one_worker_wall_s": s1["wall"], "speedup_vs_one_worker": s1["wall"] / b["wall"],
            "fp64": {"value": d["good"] / d["wall"], "eigenpairs": d["good"], "wall_s": d["wall"]},
            "fp32_over_fp64": (b["good"] / b["wall"]) / max(d["good"] / d["wall"], 1e-30),
            "fp32all": {"value": a32["good"] / a32["wall"], "eigenpairs": a32["good"],
                        "wall_s": a32["wall"], "precision": "RFD_FP32_REFINE: every factor FP32"},
            "fp32all_over_fp64": (a32["good"] / a32["wall"]) / max(d["good"] / d["wall"], 1e-30),
            "mode": "fp32+refine (RFD_FP32_AUTO)", "counted": "Ritz values within 1e-10 of a reference eigensolver",
            "nev_b": BATCH_NEV_B, "psi": BATCH_PSI, "block_steps": BATCH_STEPS,
            "sizes": {"N": [s["N"] for s in specs], "P": [s["P"] for s in specs],
                      "nev": [s["nev"] for s in specs], "n_c": [s["n_c"] for s in specs]}}


# ---------------------------------------------------------------------------
# serving leg
# ---------------------------------------------------------------------------
SERVE_STEPS = {"C1": 2, "C2": 3, "C3": 3}


def serve_leg(R, W, torch, prob2, gold2, prob3, lam3, nreq, workers):
    """Spectrum-slicing requests on the 31x31, 255x255 and 63^3 pencils
    (weights 0.6 / 0.3 / 0.1), Poisson arrivals replayed at 0.5x and 0.8x the
    saturated rate; the pencils keep their maps, two-level grouping and
    caches between requests (admission by device-memory footprint), the
    eigendecomposition of their subdomain blocks among them (spectral
    interior path)."""
    import scipy.linalg as sl
    c1 = W.config(1)
    pencils = {"C1": c1, "C2": prob2, "C3": prob3}
    spectra = {"C1": sl.eigh(c1.A.toarray(), c1.M.toarray(), eigvals_only=True),
               "C2": np.array(gold2["reference_eigs"]), "C3": np.asarray(lam3)}
    weights = {"C1": 0.6, "C2": 0.3, "C3": 0.1}
    reqs, gaps = W.serving_requests(nreq, spectra, weights)
    replicas = {nm: [] for nm in pencils}
    for nm, pr in pencils.items():
        groups = W.interface_groups(pr.grid, pr.meta["P"])
        for _ in range(1 if nm == "C3" else 2):
            P = R.Pencil(pr.A, pr.M)
            P.set_partition(pr.part)
            if groups is not None:
                P.set_interface_groups(groups)
            # one eigendecomposition per pencil serves every slice (Sec. 4.1)
            P.set_interior_solver(R.RFD_INTERIOR_SPECTRAL)
            replicas[nm].append(P)

    def build(i, rq):
        pr = pencils[rq["pencil"]]
        reps = replicas[rq["pencil"]]
        P = reps[i % len(reps)]
        k = rq["k"]
        m = min(pr.s, int(math.ceil(1.5 * k)))
        y = np.random.default_rng([5, 1, i]).standard_normal((m, pr.s))
        Y0 = torch.from_numpy(y).cuda()
        a, b = rq["alpha"], rq["beta"]
        # interior basis sized with the slice: 1.5 k over the subdomains
        nev_b = max(20, int(math.ceil(1.5 * k / pr.p)) + 10)
        return R.Job(P, a, b, 8, Y0, SERVE_STEPS[rq["pencil"]], 0.5 * (a + b), nev_b, 6, k + 40,
                     mode=R.RFD_FP32_AUTO, refine_tol=TARGET_TOL, vectors=True)

    def check(rq, job):
        lam = spectra[rq["pencil"]][rq["i0"] - 1: rq["i0"] - 1 + rq["k"]]
        ev = job.outputs()[0].cpu().numpy()
        g, _, _ = count_good(ev, lam)
        return g

    def replay(qps):
        srv = R.Server(workers=workers)
        jobs = [build(i, rq) for i, rq in enumerate(reqs)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        arrive = np.cumsum(gaps) / qps if qps else np.zeros(len(reqs))
        ids, lat, pending = {}, {}, set()
        i = 0
        while i < len(jobs) or pending:
            now = time.perf_counter() - t0
            while i < len(jobs) and arrive[i] <= now:
                ids[i] = srv.submit(jobs[i])
                pending.add(i)
                i += 1
            for q in list(pending):
                r = srv.poll(ids[q])
                if r is not None:
                    if r["status"] != 0:
                        raise RuntimeError(r["message"])
                    lat[q] = r["queued_s"] + r["run_s"]
                    pending.discard(q)
            time.sleep(0.0005)
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        per = {}
        good = 0
        for rq, j in zip(reqs, jobs):
            g = check(rq, j)
            good += g
            d = per.setdefault(rq["pencil"], dict(requests=0, eigenpairs=0, wanted=0))
            d["requests"] += 1
            d["eigenpairs"] += g
            d["wanted"] += rq["k"]
        want = sum(rq["k"] for rq in reqs)
        L = np.array([lat[q] for q in range(len(jobs))]) * 1e3
        for nm in per:
            Ln = np.array([lat[q] for q, rq in enumerate(reqs) if rq["pencil"] == nm]) * 1e3
            per[nm]["p50_ms"] = float(np.percentile(Ln, 50))
            per[nm]["p99_ms"] = float(np.percentile(Ln, 99))
        del jobs
        torch.cuda.empty_cache()
        return dict(wall_s=wall, eigenpairs=good, eigenpairs_wanted=want,
                    throughput=good / wall, p50_ms=float(np.percentile(L, 50)),
                    p99_ms=float(np.percentile(L, 99)), evictions=st["evictions"],
                    cache_hits=st["cache_hits"], cache_misses=st["cache_misses"], per_pencil=per)

    replay(None)                                   # first use of every pencil
    sat = replay(None)                             # all requests at once
    rate = nreq / sat["wall_s"]
    out = {"requests": nreq, "workers": workers, "interior_solver": "spectral",
           "replicas_per_pencil": {nm: len(v) for nm, v in replicas.items()},
           "interior": "nev_b = max(20, ceil(1.5 k / p) + 10), psi = 6, m = min(s, 1.5 k)",
           "block_steps": SERVE_STEPS, "mix": weights,
           "pencils": {nm: pr.name for nm, pr in pencils.items()},
           "mode": "fp32+refine", "unit_latency": "ms", "unit_throughput": "eigenpairs/s",
           "counted": "Ritz values within 1e-10 of the reference eigenvalues of the slice",
           "saturated": dict(sat, requests_per_s=rate)}
    for frac in (0.5, 0.8):
        out[f"qps_{frac}x"] = dict(replay(frac * rate), qps=frac * rate)
    for ps in replicas.values():
        for P in ps:
            P.close()
    return out


# ---------------------------------------------------------------------------
# CPU oracle on a bounded sample
# ---------------------------------------------------------------------------
def cpu_baseline(prob, k_rr):
    """The oracle (unchanged) on a bounded sample of the 63^3 workload, timed
    on this host's cores, and the full job extrapolated from it.

    Sample: the pencil restricted to the box x < 32, y < 16, z < 16 of the
    grid (two whole 15^3 subdomains and their separators, Dirichlet-cut
    beyond) runs the oracle's Schur assembly for one pole; one of the two
    subdomains runs the oracle's subdomain eigenpairs and resolvent levels
    for one block of m columns; the oracle's LU and block solve run on a 6144
    x 6144 complex S-sized sample; and the oracle's Rayleigh-Ritz runs on the
    full pencil with 1/12 of the columns.  Extrapolation: Schur assembly
    linearly in subdomains (64 / 2), interior work linearly in subdomains and
    columns, the S LU cubically and its solves quadratically in the interface
    size (34047 / 6144), poles x block steps factorizations (the oracle
    streams the poles: every block step factors again), and Rayleigh-Ritz
    quadratically in its columns (its n k^2 QR dominates)."""
    import oracle as O
    import scipy.linalg as sl
    coords = np.indices(prob.grid[::-1]).reshape(3, -1)[::-1]
    box = np.flatnonzero((coords[0] < 32) & (coords[1] < 16) & (coords[2] < 16))
    part = prob.part[box].copy()
    used = np.unique(part[part >= 0])
    remap = -np.ones(int(part.max()) + 1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    part[part >= 0] = remap[part[part >= 0]]
    t = {}
    t0 = time.perf_counter()
    dd = O.DD(prob.A[box][:, box], prob.M[box][:, box], part)
    t["setup"] = time.perf_counter() - t0
    z, w = O.quadrature(prob.alpha, prob.beta, prob.n_c, prob.rule)
    t0 = time.perf_counter()
    O.schur(dd, z[0])
    t["schur_2_subdomains"] = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    ns = 6144
    Ss = np.asfortranarray(rng.standard_normal((ns, ns)) + 1j * rng.standard_normal((ns, ns)))
    t0 = time.perf_counter()
    f = sl.lu_factor(Ss, overwrite_a=True, check_finite=False)
    t["slu_sample"] = time.perf_counter() - t0
    Y = rng.standard_normal((ns, prob.m))
    t0 = time.perf_counter()
    O.filter_apply([f], [w[0]], Y)
    t["fsolve_sample"] = time.perf_counter() - t0
    del Ss, f, Y
    for attr in ("interior", "adj", "B", "MB", "E", "ME"):
        setattr(dd, attr, getattr(dd, attr)[:1])
    dd.p = 1
    t0 = time.perf_counter()
    V, _ = O.interior_basis(dd, prob.sigma, prob.nev_b)
    t["vbasis_1_subdomain"] = time.perf_counter() - t0
    q = min(prob.m, dd.s)
    Qs, _ = np.linalg.qr(rng.standard_normal((dd.s, q)))
    t0 = time.perf_counter()
    O.interior_levels(dd, prob.sigma, prob.psi, Qs, V)
    t["levels_1_subdomain"] = time.perf_counter() - t0
    del dd
    ddf = O.DD.__new__(O.DD)           # the full pencil's reordering for Rayleigh-Ritz
    ddf.A, ddf.M, ddf.part = prob.A, prob.M, prob.part
    ddf.interior = [np.flatnonzero(prob.part == j) for j in range(prob.p)]
    ddf.iface = np.flatnonzero(prob.part < 0)
    kq = max(1, k_rr // 12)
    Zs = rng.standard_normal((prob.n, kq))
    t0 = time.perf_counter()
    O.rayleigh_ritz(ddf, Zs, prob.alpha, prob.beta)
    t["rr_sample"] = time.perf_counter() - t0
    del Zs
    sample = sum(t.values())
    mu = prob.steps * prob.m
    sr = prob.s / ns
    passes = prob.n_c * prob.steps
    est = (t["setup"] * prob.p / used.size
           + passes * (prob.p / used.size * t["schur_2_subdomains"] + sr ** 3 * t["slu_sample"]
                       + sr ** 2 * t["fsolve_sample"])
           + prob.p * (t["vbasis_1_subdomain"] + t["levels_1_subdomain"] * mu / q)
           + (k_rr / kq) ** 2 * t["rr_sample"])
    threads = os.environ.get("OMP_NUM_THREADS")
    cores = int(threads) if threads else os.cpu_count()
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    full = {}
    try:
        g3 = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_c3.json")))
        full = {"seconds": g3["oracle_seconds"], "threads": g3["threads"],
                "params": f"steps={g3['steps']}, nev_b={g3['nev_b']}, psi={g3['psi']}",
                "host": "the build container (8 cores), tests/golden/make_oracle_golden.py"}
    except (OSError, KeyError, ValueError):
        pass
    return dict(value=prob.nev / est, unit="eigenpairs/s", cores=cores, kind="oracle",
                full_oracle_run_smaller_setting=full,
                cpu_model=cpu,
                sample=(f"oracle on the 63^3 pencil: one pole's Schur assembly on 2 of {prob.p} "
                        f"subdomains, S LU and a {prob.m}-column solve at {ns} of {prob.s}, "
                        f"subdomain eigenpairs and levels on 1 subdomain, Rayleigh-Ritz on "
                        f"{kq} of {k_rr} columns; {sample:.1f} s sampled, full job extrapolated "
                        f"to {est:.0f} s"),
                seconds_sampled=sample, seconds_full_estimate=est, phases=t)


def load_c3(W):
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "reference_c3.json")))
    lam = np.array(ref["reference_eigs"])
    return W.config(3, known=(ref["alpha"], ref["beta"], lam)), lam


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2,
                    help="timed FP64 solves of the headline workload beside the FP32 ones")
    ap.add_argument("--mode", default="all", choices=["fp32", "fp64", "fp32all", "both", "all"],
                    help="fp32: FP32 factors + FP64 refinement where the cost model says they "
                         "pay (RFD_FP32_AUTO); fp32all: every factor FP32 (RFD_FP32_REFINE); "
                         "both: fp32 and fp64; all: the three")
    ap.add_argument("--c2-steps", type=int, default=3,
                    help="timed solves per mode of the 255x255 workload (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-spectral", action="store_true",
                    help="skip the spectral-interior leg of the headline pencil")
    ap.add_argument("--refine-tol", type=float, default=TARGET_TOL,
                    help="FP32 refinement tolerance (relative max-norm residual)")
    ap.add_argument("--batch-pencils", type=int, default=256,
                    help="pencils of the batched workload (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="requests per serving replay (0: skip)")
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (reference kernel for "
                         "the HBM byte counters of a profiler)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU: the library runs the whole path on a single "
              "MI355X (the path would shard by pole, with one all-reduce of the filtered "
              "block per step); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1711_09487_amd as R
    import workloads as W

    if a.calibrate_copy > 0:
        nel = a.calibrate_copy * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy kernel: {nel * 8} bytes read, {nel * 8} bytes written", file=sys.stderr)
        del src, dst
    prob, lam = load_c3(W)
    ref = lam[:prob.nev]
    print(f"# workload {prob.name}: n={prob.n} p={prob.p} s={prob.s} m={prob.m} "
          f"steps={prob.steps} nev_b={prob.nev_b} psi={prob.psi} n_c={prob.n_c}",
          file=sys.stderr, flush=True)
    modes = {"both": ["fp32", "fp64"], "all": ["fp32", "fp64", "fp32all"]}.get(a.mode, [a.mode])
    res = {}
    for mode in modes:
        k = a.steps if (mode == "fp32" or a.mode in ("fp64", "fp32all")) else a.fp64_steps
        res[mode] = run_mode(R, W, prob, mode, k, a.warmup, ref, torch, a.refine_tol,
                             account=True)
        r = res[mode]
        print(f"# {mode}: {1e3 * r['total'] / k:.1f} ms/step, max rel err "
              f"{max(r['errs']):.2e}, good {min(r['good'])}/{prob.nev}, with resid<=1e-9 "
              f"{min(r['strict'])}, max resid {max(r['resid']):.2e}, phases(ms) "
              f"{np.round(r['phases'][:12], 1).tolist()} sweeps {r['phases'][12:14].tolist()}",
              file=sys.stderr, flush=True)
    head = res["fp32"] if "fp32" in res else res[modes[0]]
    hs = summary(head, prob)
    # roofline of the dominant accounted kernel (largest summed time over the
    # timed steps), and of the complex GEMM on the matrix cores beside it
    f32 = "fp32" in res and head is res["fp32"]
    ks = head["kstats"]
    # (the accounting's estimate of the summed time of all launches)
    dom = max(ks, key=lambda k: ks[k][2])
    roof = roofline_entry(dom, ks[dom], f32, head["steps"], prob.name)
    # beside it: the matrix-core GEMM with the most summed time (the next one
    # when the dominant kernel is itself a GEMM)
    gemms = [k for k in ks if k.startswith("k_gemm") or k.startswith("k_dgemm")]
    gemms = [k for k in gemms if k != dom] or gemms
    gname = max(gemms, key=lambda k: ks[k][2]) if gemms else R.GEMM_KEYS[12]
    roof_mfma = roofline_entry(gname, ks.get(gname, (0, 0, 0.0, 0.0, 0.0)), f32, head["steps"],
                               prob.name)
    # FP32 factors always refine (a sweep or more); none ran when RFD_FP32_AUTO
    # found FP64 cheaper for every factor
    any32 = f32 and (head["phases"][12] > 0 or head["phases"][13] > 0)
    out = {
        "metric": "eigenpairs/sec at 1e-10 rel err, FP32+refine batched vs FP64; p50/p99",
        "value": hs["value"], "unit": "eigenpairs/s", "n_gpus": 1, "steps": head["steps"],
        "warmup": a.warmup, "ms_per_step": hs["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64" if any32 else "f64",
        "precision": (("RFD_FP32_AUTO: per factor, FP32 refined in FP64 where the refinement "
                       "costs less than the FP32 factorization saves, else FP64; ") +
                      ("some factors FP32 at this size" if any32 else
                       "every factor FP64 at this size (the shifted interior blocks: their "
                       "interface-coupled rows fit a trailing part of under half the block, "
                       "so the Schur solves need only the trailing blocks of the factors; "
                       "S: the column count)")) if f32 else "RFD_FP64",
        "data": "synthetic",
        "config": {"workload": prob.name, "n": prob.n, "p": prob.p, "s": prob.s,
                   "interface_groups": "8 octants + central separator (11719 nodes)",
                   "nev": prob.nev, "n_c": prob.n_c, "m": prob.m, "block_steps": prob.steps,
                   "nev_b": prob.nev_b, "psi": prob.psi, "rr_columns": head["k"],
                   "refine_tol": a.refine_tol},
        "counted": ("Ritz values within 1e-10 of the reference eigenvalue of the same rank "
                    "(ARPACK shift-invert, tol 1e-13, tests/golden/reference_c3.json)"),
        "latency_ms": hs["latency_ms"],
        "accuracy": {"max_rel_err_vs_reference": hs["max_rel_err"], "max_resid": hs["max_resid"],
                     "eigenpairs": hs["eigenpairs"],
                     "eigenpairs_with_resid_le_1e-9": hs["eigenpairs_resid_1e-9"],
                     "value_with_resid_le_1e-9": hs["value_resid_1e-9"]},
        "roofline": roof,
        "roofline_mfma": roof_mfma,
    }
    if "fp64" in res and "fp32" in res:
        out["fp64"] = summary(res["fp64"], prob)
        out["fp32_over_fp64"] = out["value"] / max(out["fp64"]["value"], 1e-30)
    if "fp32all" in res and head is not res["fp32all"]:
        out["fp32all"] = summary(res["fp32all"], prob)
        out["fp32all"]["precision"] = "RFD_FP32_REFINE: every factor FP32, refined in FP64"
    out["phases_ms"] = {m: np.round(res[m]["phases"][:12], 3).tolist() for m in res}
    out["kernels"] = {m: {k: dict(launches=v[0], timed=v[1],
                                  ms_per_step=v[2] / res[m]["steps"],
                                  tflops=v[3] / max(v[2], 1e-9) / 1e9,
                                  gbps=v[4] / max(v[2], 1e-9) / 1e6)
                          for k, v in res[m]["kstats"].items()} for m in res}
    if not a.no_spectral:
        out["spectral"] = spectral_leg(R, W, prob, ref, torch, a.refine_tol,
                                       [m for m in modes if m != "fp32all"])
        if "fp64" in out["spectral"] and "fp32" in out["spectral"]:
            out["spectral"]["fp32_over_fp64_stored"] = (
                out["spectral"]["fp32"]["value_stored"] /
                max(out["spectral"]["fp64"]["value_stored"], 1e-30))
    gold2 = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_c2.json")))
    prob2 = W.config(2)
    if a.c2_steps > 0:
        assert (prob2.steps, prob2.nev_b, prob2.psi) == (gold2["steps"], gold2["nev_b"], gold2["psi"])
        c2 = {}
        for mode in modes:
            if mode == "fp32all":
                continue
            r = run_mode(R, W, prob2, mode, a.c2_steps, a.warmup, np.array(gold2["theta"]),
                         torch, a.refine_tol, account=False)
            c2[mode] = summary(r, prob2)
        out["c2"] = {"workload": prob2.name, "block_steps": prob2.steps, "nev_b": prob2.nev_b,
                     "psi": prob2.psi, "interface_groups": "4 quadrants + central cross (509 nodes)",
                     "counted": "Ritz values within 1e-10 of the oracle's stored values",
                     **c2}
        if "fp64" in c2 and "fp32" in c2:
            out["c2"]["fp32_over_fp64"] = c2["fp32"]["value"] / max(c2["fp64"]["value"], 1e-30)
        print(f"# c2: {json.dumps(out['c2'])}", file=sys.stderr, flush=True)
    if a.batch_pencils > 0:
        out["batched"] = batch_leg(R, W, torch, a.batch_pencils, a.workers)
        print(f"# batched: {json.dumps({k: v for k, v in out['batched'].items() if k != 'sizes'})}",
              file=sys.stderr, flush=True)
    if a.serve_requests > 0:
        out["serving"] = serve_leg(R, W, torch, prob2, gold2, prob, lam, a.serve_requests,
                                   a.workers)
        print(f"# serving: {json.dumps(out['serving'])}", file=sys.stderr, flush=True)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, head["k"])
        print(f"# cpu_baseline: {json.dumps(out['cpu_baseline'])}", file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
