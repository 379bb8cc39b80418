"""Kernel-level GPU checks of the dense building blocks (batched MFMA GEMM,
LU without and with pivoting, block triangular solves) against FP64 host
computations, through the library's test entry points."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a, dt):
    """numpy (batch, rows, cols) -> device tensor laid out column-major per item."""
    t = torch.from_numpy(np.ascontiguousarray(np.swapaxes(a, 1, 2))).to(dt).cuda()
    return t  # shape (batch, cols, rows): item stride rows*cols, ld = rows


def _host(t):
    return np.swapaxes(t.double().cpu().numpy(), 1, 2)


# (M, N, K, batch): ragged small tiles with unaligned leading dimensions;
# 128-wide FP32 tiles with aligned operands and ragged edges; a long K split
# over workgroups (partial sums reduced by a second kernel); a single long-K
# product; few tiles over a long K; FP64 products on the large-product
# kernel (64 x 128 real, 64 x 64 complex tiles) with ragged M, N and a K that
# ends in a partial slab, the first one with odd leading dimensions
GEMM_SHAPES = {"small_unaligned": (70, 130, 37, 3), "tile128_ragged": (1100, 1030, 72, 3),
               "tile128_k200": (300, 260, 200, 2), "split_k": (100, 70, 5000, 2),
               "split_k_single": (100, 70, 9000, 1), "tile128_split_k": (390, 250, 20000, 1),
               "dgemm_tall": (4099, 501, 293, 2), "dgemm_square": (4100, 4130, 261, 1)}


@pytest.mark.parametrize("shape", list(GEMM_SHAPES))
@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_batched(dtype, cplx, ta, tb, shape):
    torch = _torch()
    import paper_1711_09487_amd as R
    rs = np.random.default_rng(1)
    M, N, K, batch = GEMM_SHAPES[shape]
    dt = torch.float32 if dtype == 0 else torch.float64
    Ash = (batch, K, M) if ta else (batch, M, K)
    Bsh = (batch, N, K) if tb else (batch, K, N)
    Ar, Ai = rs.standard_normal(Ash), rs.standard_normal(Ash)
    Br, Bi = rs.standard_normal(Bsh), rs.standard_normal(Bsh)
    Cr, Ci = rs.standard_normal((batch, M, N)), rs.standard_normal((batch, M, N))
    alpha, beta = -0.75, 0.5
    A = Ar + 1j * Ai if cplx else Ar
    B = Br + 1j * Bi if cplx else Br
    Cref = Cr + 1j * Ci if cplx else Cr.copy()
    opA = np.swapaxes(A, 1, 2) if ta else A
    opB = np.swapaxes(B, 1, 2) if tb else B
    ref = alpha * (opA @ opB) + beta * Cref
    t = {k: _dev(torch, v, dt) for k, v in dict(ar=Ar, ai=Ai, br=Br, bi=Bi, cr=Cr, ci=Ci).items()}
    lda, ldb, ldc = Ash[1], Bsh[1], M
    code = R.lib().rfd_test_gemm(
        dtype, ta, tb, M, N, K, alpha, beta,
        t["ar"].data_ptr(), t["ai"].data_ptr() if cplx else None, lda, Ash[1] * Ash[2],
        t["br"].data_ptr(), t["bi"].data_ptr() if cplx else None, ldb, Bsh[1] * Bsh[2],
        t["cr"].data_ptr(), t["ci"].data_ptr() if cplx else None, ldc, M * N, batch,
        torch.cuda.current_stream().cuda_stream)
    assert code == 0, R.rfd_last_error()
    torch.cuda.synchronize()
    got = _host(t["cr"]) + (1j * _host(t["ci"]) if cplx else 0)
    tol = 2e-5 if dtype == 0 else 1e-13
    assert np.max(np.abs(got - ref)) < tol * np.max(np.abs(ref)) * np.sqrt(K)


@pytest.mark.parametrize("M,N,K,batch", [(8192, 512, 512, 1), (8191, 515, 515, 2),
                                         (4099, 640, 700, 2), (70, 130, 130, 3)])
def test_gemm_upper_triangular_b(M, N, K, batch):
    """C = alpha A B + beta C with B upper triangular (B[k, j] = 0 for
    k > j), the Cholesky-QR product of the basis construction: the large
    shapes take the large-tile FP64 kernel, which skips each tile column's
    zero K range (ragged tiles, K beyond N, batches); the small one the
    64 x 64 kernel over the whole K."""
    torch = _torch()
    import paper_1711_09487_amd as R
    rs = np.random.default_rng(7)
    A = rs.standard_normal((batch, M, K))
    B = np.triu(rs.standard_normal((batch, K, N)))
    Cm = rs.standard_normal((batch, M, N))
    alpha, beta = 0.625, -1.5
    ref = alpha * (A @ B) + beta * Cm
    a, b, c = (_dev(torch, v, torch.float64) for v in (A, B, Cm))
    code = R.lib().rfd_test_gemm_triu_b(M, N, K, alpha, beta, a.data_ptr(), M, M * K,
                                        b.data_ptr(), K, K * N, c.data_ptr(), M, M * N, batch,
                                        torch.cuda.current_stream().cuda_stream)
    assert code == 0, R.rfd_last_error()
    torch.cuda.synchronize()
    got = _host(c)
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref)) * np.sqrt(K)


def _shifted_blocks(rs, n, batch, cplx):
    """Shifted 1D/2D-Laplacian-like blocks B - z M, complex symmetric."""
    out = []
    for b in range(batch):
        T = np.diag(4.0 + rs.uniform(0, 0.1, n)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
        k = int(np.sqrt(n))
        T -= np.diag(np.ones(n - k), k) + np.diag(np.ones(n - k), -k)
        Md = np.diag(rs.uniform(0.5, 1.5, n))
        z = (0.3 + 0.05j * (b + 1)) if cplx else 0.0
        out.append(T - z * Md)
    return np.array(out)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("cplx", [False, True])
def test_lu_nopiv_solve(dtype, cplx):
    torch = _torch()
    import paper_1711_09487_amd as R
    rs = np.random.default_rng(2)
    n, batch, r = 192, 3, 70
    dt = torch.float32 if dtype == 0 else torch.float64
    A = _shifted_blocks(rs, n, batch, cplx)
    Rh = rs.standard_normal((batch, n, r)) + (1j * rs.standard_normal((batch, n, r)) if cplx else 0)
    X = np.linalg.solve(A, Rh)
    ar, ai = _dev(torch, A.real, dt), _dev(torch, A.imag, dt)
    rr, ri = _dev(torch, Rh.real, dt), _dev(torch, np.imag(Rh), dt)
    flags = C.c_uint32(7)
    code = R.lib().rfd_test_lu(dtype, 0, n, batch, ar.data_ptr(), ai.data_ptr() if cplx else None,
                               n, n * n, rr.data_ptr(), ri.data_ptr() if cplx else None, n, n * r,
                               r, C.byref(flags), torch.cuda.current_stream().cuda_stream)
    assert code == 0, R.rfd_last_error()
    assert flags.value == 0
    got = _host(rr) + (1j * _host(ri) if cplx else 0)
    tol = 2e-5 if dtype == 0 else 1e-12
    assert np.max(np.abs(got - X)) < tol * np.max(np.abs(X))
    # the factors themselves: L U = A
    F = _host(ar) + (1j * _host(ai) if cplx else 0)
    L = np.tril(F, -1) + np.eye(n)
    U = np.triu(F)
    assert np.max(np.abs(L @ U - A)) < (5e-6 if dtype == 0 else 1e-13) * np.max(np.abs(A))


@pytest.mark.parametrize("dtype", [0, 1])
def test_lu_partial_pivoting_solve(dtype):
    torch = _torch()
    import paper_1711_09487_amd as R
    rs = np.random.default_rng(3)
    n, batch, r = 192, 2, 65
    dt = torch.float32 if dtype == 0 else torch.float64
    A = rs.standard_normal((batch, n, n))          # needs pivoting
    A[:, 0, 0] = 0.0
    Rh = rs.standard_normal((batch, n, r))
    X = np.linalg.solve(A, Rh)
    ar, rr = _dev(torch, A, dt), _dev(torch, Rh, dt)
    flags = C.c_uint32(7)
    code = R.lib().rfd_test_lu(dtype, 1, n, batch, ar.data_ptr(), None, n, n * n, rr.data_ptr(),
                               None, n, n * r, r, C.byref(flags),
                               torch.cuda.current_stream().cuda_stream)
    assert code == 0, R.rfd_last_error()
    assert flags.value == 0
    got = _host(rr)
    cond = np.linalg.cond(A[0])
    tol = (1e-6 if dtype == 0 else 1e-14) * cond
    assert np.max(np.abs(got - X)) < tol * np.max(np.abs(X))


def test_lu_breakdown_flag():
    """A singular block (a zero leading pivot, no pivoting) raises the flag."""
    torch = _torch()
    import paper_1711_09487_amd as R
    n = 64
    A = np.eye(n)[None].copy()
    A[0, 0, 0] = 0.0
    ar = _dev(torch, A, torch.float64)
    flags = C.c_uint32(0)
    code = R.lib().rfd_test_lu(1, 0, n, 1, ar.data_ptr(), None, n, n * n, None, None, n, 0, 0,
                               C.byref(flags), torch.cuda.current_stream().cuda_stream)
    assert code == 0
    assert flags.value != 0


def test_symmetric_eigensolver_beyond_the_staged_tridiagonal():
    """n above 4096: the Sturm counts and the bisection read the tridiagonal
    from global memory (smaller ones stage it in shared memory).  A is built
    from known eigenvalues, A = Q diag(lam) Q^T, so no dense reference solve
    is needed; the tolerances allow for the rounding of that construction."""
    torch = _torch()
    import paper_1711_09487_amd as R
    n, num = 4100, 16
    rs = np.random.default_rng(11)
    Q, _ = np.linalg.qr(rs.standard_normal((n, n)))
    lam = np.sort(rs.uniform(-2, 3, n))
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    At = torch.from_numpy(A.reshape(1, n, n).copy()).cuda()
    lam_d = torch.zeros(num, dtype=torch.float64, device="cuda")
    Y_d = torch.zeros(num * n, dtype=torch.float64, device="cuda")
    code = R.lib().rfd_test_syevx(n, 1, At.data_ptr(), 0, num, lam_d.data_ptr(), Y_d.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)
    assert code == 0, R.rfd_last_error()
    torch.cuda.synchronize()
    got = lam_d.cpu().numpy()
    X = Y_d.cpu().numpy().reshape(num, n).T
    nrm = np.abs(lam).max()
    assert np.max(np.abs(got - lam[:num])) <= 1e-11 * nrm
    assert np.max(np.abs(A @ X - X * got)) <= 1e-11 * nrm
    assert np.max(np.abs(X.T @ X - np.eye(num))) <= 1e-11


@pytest.mark.parametrize("n,batch,lo,num", [(100, 3, 5, 20), (77, 2, 0, 30), (40, 1, 0, 40),
                                             (300, 2, 10, 40), (517, 1, 100, 30)])
def test_symmetric_eigensolver(n, batch, lo, num):
    """Blocked tridiagonalization + bisection + inverse iteration + back-
    transformation against LAPACK: ragged panels (n - 2 reflectors in panels
    of 32), several 64 x 64 tiles of the mat-vec with odd and even anchors,
    odd n (scalar loads), and a cluster of equal eigenvalues."""
    torch = _torch()
    import paper_1711_09487_amd as R
    rs = np.random.default_rng(7)
    mats = []
    for b in range(batch):
        Q, _ = np.linalg.qr(rs.standard_normal((n, n)))
        lam = np.sort(rs.uniform(-2, 3, n))
        lam[3:6] = lam[3]                      # a triple eigenvalue
        mats.append((Q * lam) @ Q.T)
    A = np.array([0.5 * (m + m.T) for m in mats])
    At = torch.from_numpy(A.copy()).cuda()   # symmetric: row- and column-major agree
    lam_d = torch.zeros(batch * num, dtype=torch.float64, device="cuda")
    Y_d = torch.zeros(batch * num * n, dtype=torch.float64, device="cuda")
    code = R.lib().rfd_test_syevx(n, batch, At.data_ptr(), lo, num, lam_d.data_ptr(),
                                  Y_d.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert code == 0, R.rfd_last_error()
    torch.cuda.synchronize()
    lam = lam_d.cpu().numpy().reshape(batch, num)
    Y = Y_d.cpu().numpy().reshape(batch, num, n)
    for b in range(batch):
        ref = np.linalg.eigvalsh(A[b])[lo:lo + num]
        nrm = np.abs(np.linalg.eigvalsh(A[b])).max()
        assert np.max(np.abs(lam[b] - ref)) <= 1e-13 * nrm
        X = Y[b].T
        res = A[b] @ X - X * lam[b]
        assert np.max(np.abs(res)) <= 1e-12 * nrm
        assert np.max(np.abs(X.T @ X - np.eye(num))) <= 1e-12


@pytest.mark.parametrize("dtype,cplx,ta,tb,M,N,K,batch", [
    (1, 0, 0, 0, 700, 520, 300, 2), (1, 0, 1, 0, 300, 260, 1200, 1),
    (1, 1, 0, 1, 513, 130, 290, 3), (0, 0, 0, 0, 640, 700, 300, 1), (0, 1, 1, 1, 130, 200, 77, 2)])
def test_gemm_variants_and_tuning_table(dtype, cplx, ta, tb, M, N, K, batch):
    """Every kernel variant the autotuner may pick (rfd_test_gemm_variant:
    the 64 x 64 tile, the 128 x 128 tile for real FP32, the large-tile FP64
    kernel) computes the product; a variant that cannot run the class says
    so.  A tuning table entry for the class makes the default entry point
    give the forced variant's result bit for bit."""
    torch = _torch()
    import paper_1711_09487_amd as R
    rs = np.random.default_rng(11)
    dt = torch.float32 if dtype == 0 else torch.float64
    Ash = (batch, K, M) if ta else (batch, M, K)
    Bsh = (batch, N, K) if tb else (batch, K, N)
    Ar, Ai, Br, Bi = (rs.standard_normal(s) for s in (Ash, Ash, Bsh, Bsh))
    Cr, Ci = rs.standard_normal((batch, M, N)), rs.standard_normal((batch, M, N))
    alpha, beta = 0.5, -1.25
    A = Ar + 1j * Ai if cplx else Ar
    B = Br + 1j * Bi if cplx else Br
    opA = np.swapaxes(A, 1, 2) if ta else A
    opB = np.swapaxes(B, 1, 2) if tb else B
    ref = alpha * (opA @ opB) + beta * (Cr + 1j * Ci if cplx else Cr)
    tol = (2e-5 if dtype == 0 else 1e-13) * np.max(np.abs(ref)) * np.sqrt(K)
    L = R.lib()

    def run(fn, *pre):
        t = {k: _dev(torch, v, dt) for k, v in dict(ar=Ar, ai=Ai, br=Br, bi=Bi, cr=Cr, ci=Ci).items()}
        code = fn(*pre, dtype, ta, tb, M, N, K, alpha, beta,
                  t["ar"].data_ptr(), t["ai"].data_ptr() if cplx else None, Ash[1], Ash[1] * Ash[2],
                  t["br"].data_ptr(), t["bi"].data_ptr() if cplx else None, Bsh[1], Bsh[1] * Bsh[2],
                  t["cr"].data_ptr(), t["ci"].data_ptr() if cplx else None, M, M * N, batch,
                  torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        return code, (_host(t["cr"]) + (1j * _host(t["ci"]) if cplx else 0)) if code == 0 else None

    runs = {}
    for v in (1, 2, 3):
        code, got = run(L.rfd_test_gemm_variant, v)
        runnable = v == 1 or (v == 2 and dtype == 0 and not cplx) or (v == 3 and dtype == 1)
        if not runnable:
            assert code == 1 and "variant" in R.rfd_last_error()
            continue
        assert code == 0, R.rfd_last_error()
        assert np.max(np.abs(got - ref)) < tol, v
        runs[v] = got
    pick = max(runs)
    key = [dtype, int(cplx), ta, tb] + [int(np.floor(np.log2(x))) for x in (M, N, K, batch)]
    try:
        R.rfd_set_gemm_tuning([key + [pick]])
        code, got = run(L.rfd_test_gemm)
        assert code == 0
        assert np.array_equal(got, runs[pick])
    finally:
        R.rfd_set_gemm_tuning(np.zeros((0, 9), dtype=np.int32))
        R._load_tuning(L)
