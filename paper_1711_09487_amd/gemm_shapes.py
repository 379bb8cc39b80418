"""Per-shape throughput of the library's MFMA GEMM (rfd_test_gemm) on the
products that dominate a 63^3 solve, beside torch's matmul on the same shapes
(the vendor BLAS, as a yardstick only: the solve never calls it).

    python -m paper_1711_09487_amd.gemm_shapes [--reps R]

Prints one line per shape: TFLOP/s of the library kernel and of torch, with
flops counted as 2 M N K per real product and 8 M N K per complex one.
Operands are column-major and planar complex (real and imaginary planes) on
the library side; torch gets row-major views of the same real data, and
complex128 tensors for the complex shapes.
"""
import argparse
import sys

import paper_1711_09487_amd as R

# (label, dtype 0 = FP32 / 1 = FP64, complex, transA, M, N, K, batch)
SHAPES = [
    ("level projection X -= Zp T", 1, False, 0, 250047, 2800, 2800, 1),
    ("long-K projection Zp^T (M X)", 1, False, 1, 8400, 2800, 250047, 1),
    ("Rayleigh-Ritz block Z^T (A Z)", 1, False, 1, 2800, 11200, 250047, 1),
    ("refinement residual S_TT X (8 poles)", 1, True, 0, 11719, 700, 11719, 8),
    ("subdomain back-transformation", 1, False, 0, 3375, 40, 3375, 64),
    ("LU trailing update B_j(zeta), 128 items", 0, True, 0, 3328, 3328, 64, 128),
    ("S_TT solve block update (8 poles)", 0, True, 0, 11719, 700, 2048, 8),
]


def _flops(cplx, M, N, K, b):
    return (8.0 if cplx else 2.0) * M * N * K * b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=0, help="timed repetitions (0: about 2e13 flops)")
    a = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        print("no GPU", file=sys.stderr)
        sys.exit(1)
    L = R.lib()
    for label, dt, cplx, ta, M, N, K, b in SHAPES:
        tdt = torch.float32 if dt == 0 else torch.float64
        ra, ca = (K, M) if ta else (M, K)
        planes = 2 if cplx else 1
        A = [torch.randn(b, ca, ra, dtype=tdt, device="cuda") for _ in range(planes)]
        B = [torch.randn(b, N, K, dtype=tdt, device="cuda") for _ in range(planes)]
        C = [torch.zeros(b, N, M, dtype=tdt, device="cuda") for _ in range(planes)]

        def ours():
            rc = L.rfd_test_gemm(dt, ta, 0, M, N, K, 1.0, 0.0,
                                 A[0].data_ptr(), A[-1].data_ptr() if cplx else None, ra, ra * ca,
                                 B[0].data_ptr(), B[-1].data_ptr() if cplx else None, K, K * N,
                                 C[0].data_ptr(), C[-1].data_ptr() if cplx else None, M, M * N, b,
                                 None)
            if rc != 0:
                raise RuntimeError(R.rfd_last_error())

        # torch on the row-major views: the (ca, ra) tensor of A is op(A)^T
        # (ta = 0) or op(A) (ta = 1), the (N, K) tensor of B is B^T, and
        # C^T = B^T op(A)^T
        if cplx:
            Az = torch.complex(A[0], A[1])
            Bz = torch.complex(B[0], B[1])
        else:
            Az, Bz = A[0], B[0]
        At = Az.transpose(1, 2).contiguous() if ta else Az     # op(A)^T, (b, K, M)

        def theirs():
            torch.matmul(Bz, At)

        f = _flops(cplx, M, N, K, b)
        reps = a.reps or max(2, min(20, int(2e13 / f)))
        res = []
        for fn in (ours, theirs):
            fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            res.append((ms, f / (ms * 1e-3) / 1e12))
        print(f"{label:42s} {'f32' if dt == 0 else 'f64'}{' cplx' if cplx else '     '} "
              f"ta={ta} {M}x{N}x{K} b={b}: library {res[0][0]:9.3f} ms {res[0][1]:6.1f} TF/s | "
              f"torch {res[1][0]:9.3f} ms {res[1][1]:6.1f} TF/s", flush=True)
        del A, B, C, Az, Bz, At
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
