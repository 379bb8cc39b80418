"""The allocation-free product (rfd_test_gemm_static) against the allocating
one (rfd_test_gemm) through the C ABI: the same results on two calls in a
row, the second smaller (the fixed scratch array keeps the first call's
partial tiles, which must not leak into the second), split-K shapes that
use the scratch and shapes that do not, and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _call(fn, torch, dtype, ta, tb, M, N, K, batch, cplx, seed):
    """Column-major operands: an r x c matrix is a (c, r) torch block (leading
    dimension r); op(A) is M x K (A stored K x M when ta), op(B) is K x N."""
    rs = np.random.default_rng(seed)
    dt = torch.float32 if dtype == 0 else torch.float64
    ra, ca = (K, M) if ta else (M, K)
    rb, cb = (N, K) if tb else (K, N)
    def dev(r, c):
        return torch.from_numpy(rs.standard_normal((batch, c, r))).to(dt).cuda()
    Ar, Ai, Br, Bi = dev(ra, ca), dev(ra, ca), dev(rb, cb), dev(rb, cb)
    Cr, Ci = dev(M, N), dev(M, N)
    # every element the product touches lies inside the blocks
    assert (ra - 1) + (ca - 1) * ra < ra * ca and (rb - 1) + (cb - 1) * rb < rb * cb
    code = fn(dtype, ta, tb, M, N, K, -0.75, 0.5,
              Ar.data_ptr(), Ai.data_ptr() if cplx else None, ra, ra * ca,
              Br.data_ptr(), Bi.data_ptr() if cplx else None, rb, rb * cb,
              Cr.data_ptr(), Ci.data_ptr() if cplx else None, M, M * N, batch,
              torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    out = Cr.double().cpu().numpy() + (1j * Ci.double().cpu().numpy() if cplx else 0)
    return code, out


# (dtype, ta, tb, M, N, K, batch, complex): split-K products (few tiles, long
# K) in both precisions, real and complex, and a many-tile product without
# split K
CASES = [(1, 1, 0, 300, 200, 30000, 1, False), (0, 0, 0, 130, 70, 9000, 2, True),
         (1, 0, 1, 100, 90, 20000, 1, True), (1, 0, 0, 1100, 1030, 300, 2, False)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_static_gemm_equals_the_allocating_gemm(case):
    torch = _torch()
    import paper_1711_09487_amd as R
    L = R.lib()
    dtype, ta, tb, M, N, K, batch, cplx = CASES[case]
    # two calls in a row, the second with a smaller product
    for (m, n, k, b), seed in (((M, N, K, batch), 1), ((M // 2 + 1, N // 3 + 1, K // 2 + 3, 1), 2)):
        c0, ref = _call(L.rfd_test_gemm, torch, dtype, ta, tb, m, n, k, b, cplx, seed)
        c1, got = _call(L.rfd_test_gemm_static, torch, dtype, ta, tb, m, n, k, b, cplx, seed)
        assert c0 == 0 and c1 == 0, R.rfd_last_error()
        tol = 2e-5 if dtype == 0 else 1e-13
        assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)) * np.sqrt(k)


def test_static_gemm_rejects_outputs_beyond_its_scratch():
    """A complex FP64 2048 x 2048 output takes 64 MiB, above the 32 MiB limit:
    rejected before any launch (all operands are real buffers of the right
    size, so nothing could be read out of bounds either way)."""
    torch = _torch()
    import paper_1711_09487_amd as R
    L = R.lib()
    M = N = 2048
    K = 64
    a = [torch.zeros(K * M, dtype=torch.float64, device="cuda") for _ in range(2)]
    b = [torch.zeros(K * N, dtype=torch.float64, device="cuda") for _ in range(2)]
    c = [torch.zeros(M * N, dtype=torch.float64, device="cuda") for _ in range(2)]
    code = L.rfd_test_gemm_static(1, 0, 0, M, N, K, 1.0, 0.0, a[0].data_ptr(), a[1].data_ptr(), M,
                                  0, b[0].data_ptr(), b[1].data_ptr(), K, 0, c[0].data_ptr(),
                                  c[1].data_ptr(), M, 0, 1, None)
    torch.cuda.synchronize()
    assert code == 1 and "at most" in R.rfd_last_error()
    # null operand planes are rejected before anything is launched
    code = L.rfd_test_gemm_static(1, 0, 0, 64, 64, 64, 1.0, 0.0, None, None, 64, 0, None, None, 64,
                                  0, None, None, 64, 0, 1, None)
    assert code == 1 and "null" in R.rfd_last_error()
