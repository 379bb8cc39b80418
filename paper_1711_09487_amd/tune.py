"""Autotuner of the matrix-core GEMM's tile choices.

    python -m paper_1711_09487_amd.tune [--out PATH] [--reps R]

For each product class of the solve (precision, complex, transposes, and
floor(log2) of M, N, K and the batch) it times, on one representative shape,
the library's built-in choice (rfd_test_gemm) and every kernel variant that
can run the class (rfd_test_gemm_variant: 1 = the 64 x 64 tile, 2 = the
128 x 128 tile for real FP32, 3 = the large-tile FP64 kernel), twice: alone
on the device, and beside a stream of large FP64 products (inside the solve
most products share the device with the subdomain eigensolver, the B_sigma
factorization or the Rayleigh-Ritz rows, and a kernel that wins alone can
lose there).  A class gets an entry only where a variant beats the built-in
choice by at least 5 % in both measurements.
The table goes to tuning/<arch>.json (arch of the current device), which
the binding hands to rfd_set_gemm_tuning when it loads the library; the
measurements are kept beside the entries.

The shapes are those of the 63^3, 255x255 and batched workloads: the
basis construction's level projections, long-K inner products and Gram
matrices, the deflation and back-transformation products of the
subdomains, the trailing updates and triangular-solve updates of the LU of
the shifted blocks and of S(zeta), and the Ritz vectors.
"""
import argparse
import json
import math
import os
import sys
import time


# (name, fp64, complex, transA, transB, M, N, K, batch)
SHAPES = [
    ("level projection X -= Zp T", 1, 0, 0, 0, 250047, 2800, 2800, 1),
    ("long-K projection Zp^T (M X)", 1, 0, 1, 0, 8400, 2800, 250047, 1),
    ("Gram matrix B^T M B", 1, 0, 1, 0, 2800, 2800, 250047, 1),
    ("Rayleigh-Ritz rows Z^T (A Z)", 1, 0, 1, 0, 2800, 11200, 250047, 1),
    ("Ritz vectors Z G", 1, 0, 0, 0, 250047, 500, 13760, 1),
    ("subdomain deflation X -= V T", 1, 0, 0, 0, 3392, 2816, 52, 64),
    ("subdomain V^T (M X)", 1, 0, 1, 0, 52, 2816, 3392, 64),
    ("subdomain back-transformation", 1, 0, 0, 0, 3375, 40, 3375, 64),
    ("B_sigma LU trailing update", 1, 0, 0, 0, 3328, 3328, 64, 64),
    ("B_sigma level solve update", 1, 0, 0, 0, 1696, 2816, 1696, 64),
    ("255x255 level projection", 1, 0, 0, 0, 65025, 1500, 1500, 1),
    ("255x255 long-K projection", 1, 0, 1, 0, 4500, 1500, 65025, 1),
    ("S top block LU update", 1, 1, 0, 0, 5888, 5888, 5888, 8),
    ("S top block LU short update", 1, 1, 0, 0, 11648, 11648, 64, 8),
    ("S group LU update", 1, 1, 0, 0, 1408, 1408, 1408, 64),
    ("S top block solve update", 1, 1, 0, 0, 5888, 2816, 5888, 8),
    ("S group solve update", 1, 1, 0, 0, 1408, 2816, 1408, 64),
    ("S_gT^T X_g (top complement)", 1, 1, 1, 0, 3456, 2816, 1408, 64),
    ("batched pencil level projection", 1, 0, 0, 0, 12000, 200, 200, 1),
    ("FP32 square real product", 0, 0, 0, 0, 4096, 4096, 1024, 1),
    ("FP32 real tall product", 0, 0, 0, 0, 65536, 512, 512, 1),
]


def _time(fn, reps, load=None):
    """Milliseconds per call of fn on the current stream; with load, while
    load() keeps another stream busy for longer than the timed calls."""
    import torch
    fn()
    torch.cuda.synchronize()
    if load is not None:
        load()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.current_stream().synchronize()
    t = (time.perf_counter() - t0) / reps * 1e3
    torch.cuda.synchronize()
    return t


class Load:
    """Large FP64 products queued on a stream of their own (default
    priority), enough to outlast the timed calls."""

    def __init__(self):
        import torch
        self.s = torch.cuda.Stream()
        self.a = torch.randn(8192, 8192, dtype=torch.float64, device="cuda")
        self.b = torch.randn(8192, 8192, dtype=torch.float64, device="cuda")
        self.c = torch.empty_like(self.a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        torch.mm(self.a, self.b, out=self.c)
        torch.cuda.synchronize()
        self.ms = (time.perf_counter() - t0) * 1e3

    def queue(self, ms):
        import torch
        with torch.cuda.stream(self.s):
            for _ in range(int(ms / max(self.ms, 1e-3)) + 2):
                torch.mm(self.a, self.b, out=self.c)


def measure(R, shape, reps, load):
    import torch
    name, f64, cplx, ta, tb, M, N, K, b = shape
    dt = torch.float64 if f64 else torch.float32
    ra, ca = (K, M) if ta else (M, K)
    rb, cb = (N, K) if tb else (K, N)
    planes = 2 if cplx else 1
    A = [torch.randn(b * ra * ca, dtype=dt, device="cuda") for _ in range(planes)]
    B = [torch.randn(b * rb * cb, dtype=dt, device="cuda") for _ in range(planes)]
    Cm = [torch.zeros(b * M * N, dtype=dt, device="cuda") for _ in range(planes)]
    args = lambda: (int(f64), ta, tb, M, N, K, 1.0, 0.0, A[0].data_ptr(),
                    A[-1].data_ptr() if cplx else None, ra, ra * ca, B[0].data_ptr(),
                    B[-1].data_ptr() if cplx else None, rb, rb * cb, Cm[0].data_ptr(),
                    Cm[-1].data_ptr() if cplx else None, M, M * N, b, None)
    L = R.lib()
    alone, loaded = {}, {}

    def run_default():
        if L.rfd_test_gemm(*args()) != 0:
            raise R.RfdError(1, L.rfd_last_error().decode())
    fns = {0: run_default}
    for v in ([1, 3] if f64 else ([1, 2] if not cplx else [])):
        def run(v=v):
            code = L.rfd_test_gemm_variant(v, *args())
            if code != 0:
                raise R.RfdError(code, L.rfd_last_error().decode())
        fns[v] = run
    for v, fn in fns.items():
        try:
            alone[v] = _time(fn, reps)
        except R.RfdError:
            continue
        loaded[v] = _time(fn, reps, lambda: load.queue(3.0 * reps * alone[v] + 20.0))
    del A, B, Cm
    torch.cuda.empty_cache()
    return alone, loaded


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="output file (default tuning/<arch>.json)")
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    os.environ["RFD_GEMM_TUNING"] = "off"      # time the built-in rules
    import torch
    import paper_1711_09487_amd as R
    arch = R.device_arch()
    if arch is None:
        sys.exit("no GPU device")
    entries, meas = [], []
    load = Load()
    for sh in SHAPES:
        name, f64, cplx, ta, tb, M, N, K, b = sh
        alone, loaded = measure(R, sh, a.reps, load)
        wins = [v for v in alone if v != 0 and alone[v] <= 0.95 * alone[0]
                and loaded[v] <= 0.95 * loaded[0]]
        pick = min(wins, key=lambda v: alone[v] + loaded[v]) if wins else 0
        key = [f64, cplx, ta, tb] + [int(math.floor(math.log2(x))) for x in (M, N, K, b)]
        if pick:
            entries.append(key + [pick])
        flops = (8.0 if cplx else 2.0) * M * N * K * b
        meas.append({"name": name, "shape": [f64, cplx, ta, tb, M, N, K, b],
                     "ms_alone": {str(v): round(t, 4) for v, t in alone.items()},
                     "ms_beside_load": {str(v): round(t, 4) for v, t in loaded.items()},
                     "pick": pick, "tflops_default": flops / alone[0] / 1e9})
        print(f"{name:36s} {'f64' if f64 else 'f32'}{' cplx' if cplx else '     '} "
              f"{M}x{N}x{K} b={b}: alone " +
              ", ".join(f"{v}: {t:.3f}" for v, t in alone.items()) + " | loaded " +
              ", ".join(f"{v}: {t:.3f}" for v, t in loaded.items()) +
              f" ms -> {pick or 'built-in'}", flush=True)
    out = a.out or os.path.join(R.TUNING_DIR, arch + ".json")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    json.dump({"arch": arch, "device": torch.cuda.get_device_name(0),
               "tool": "python -m paper_1711_09487_amd.tune",
               "entry_fields": ["fp64", "complex", "transA", "transB", "log2M", "log2N",
                                "log2K", "log2batch", "variant"],
               "entries": entries, "measurements": meas}, open(out, "w"), indent=1)
    print(f"wrote {out}: {len(entries)} entries", flush=True)


if __name__ == "__main__":
    main()
