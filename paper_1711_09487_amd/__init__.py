"""Python binding of the RF-DDES gfx950 library (librfd.so, include/rfd.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors on ``cuda``) and the stream.
The functions keep the C names; ``Pencil`` is a thin convenience wrapper.
There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = [
    "RfdError", "lib", "Pencil", "Job", "Server", "batch_run", "RFD_FP64", "RFD_FP32_REFINE", "RFD_FP32_AUTO",
    "RFD_RULE_GAUSS", "RFD_RULE_MIDPOINT", "RFD_RULE_EXPLICIT", "LIB_PATH",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librfd.so")
RFD_FP64, RFD_FP32_REFINE, RFD_FP32_AUTO = 0, 1, 2
RFD_RULE_GAUSS, RFD_RULE_MIDPOINT, RFD_RULE_EXPLICIT = 0, 1, 2
RFD_INTERIOR_LU, RFD_INTERIOR_SPECTRAL = 0, 1
STATUS = {0: "RFD_OK", 1: "RFD_EINVAL", 2: "RFD_ENOMEM", 3: "RFD_EBREAKDOWN",
          4: "RFD_ENOCONV", 5: "RFD_EDEVICE", 6: "RFD_ESTATE", 7: "RFD_EPENDING"}
RFD_EPENDING = 7

EXPORTS = [
    "rfd_create_pencil", "rfd_set_partition", "rfd_set_interval_and_poles",
    "rfd_set_precision", "rfd_filter_interface", "rfd_filter_apply", "rfd_filter_lanczos",
    "rfd_prepare_interior",
    "rfd_solve_interior",
    "rfd_rayleigh_ritz",
    "rfd_destroy_pencil", "rfd_last_error", "rfd_pencil_info", "rfd_set_timing",
    "rfd_phase_times", "rfd_reset_caches", "rfd_set_pole_window", "rfd_set_interface_groups",
    "rfd_set_interior_solver",
    "rfd_inertia_count", "rfd_solve_slices",
    "rfd_batch_run", "rfd_server_create",
    "rfd_server_submit", "rfd_server_poll", "rfd_server_destroy", "rfd_server_stats",
    "rfd_server_cache_stats",
]


class rfd_job(C.Structure):
    """Mirror of struct rfd_job (include/rfd.h)."""
    _fields_ = [("alpha", C.c_double), ("beta", C.c_double), ("n_c", C.c_int32),
                ("rule", C.c_int32), ("mode", C.c_int32), ("max_sweeps", C.c_int32),
                ("refine_tol", C.c_double), ("m", C.c_int32), ("steps", C.c_int32),
                ("Y0", C.c_void_p), ("sigma", C.c_double), ("nev_b", C.c_int32),
                ("psi", C.c_int32), ("max_out", C.c_int32), ("evals", C.c_void_p),
                ("evecs", C.c_void_p), ("resid", C.c_void_p)]


class rfd_result(C.Structure):
    """Mirror of struct rfd_result (include/rfd.h)."""
    _fields_ = [("status", C.c_int32), ("nfound", C.c_int32), ("mu", C.c_int32),
                ("worker", C.c_int32), ("k", C.c_int64), ("bytes", C.c_int64),
                ("queued_s", C.c_double), ("run_s", C.c_double), ("message", C.c_char * 160)]


class RfdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None
P = C.c_void_p
I32, I64, F64 = C.c_int32, C.c_int64, C.c_double


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "paper_1711_09487_amd.build.build() (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        sig = {
            "rfd_create_pencil": [I64, P, P, P, P, P, P, C.POINTER(P)],
            "rfd_set_partition": [P, I32, P],
            "rfd_set_interval_and_poles": [P, F64, F64, I32, I32, P, P],
            "rfd_set_precision": [P, I32, F64, I32],
            "rfd_filter_interface": [P, I32, P, I32, P, I64, C.POINTER(I32), P],
            "rfd_filter_lanczos": [P, I32, P, F64, I32, I32, P, I64, C.POINTER(I32),
                                   C.POINTER(I32), P, C.POINTER(I32), P],
            "rfd_prepare_interior": [P, C.c_double, I32],
            "rfd_solve_interior": [P, F64, I32, I32, C.POINTER(I64), P],
            "rfd_filter_apply": [P, I32, P, P, P],
            "rfd_rayleigh_ritz": [P, I32, P, P, P, C.POINTER(I32), P],
            "rfd_destroy_pencil": [P],
            "rfd_pencil_info": [P, C.POINTER(I64), C.POINTER(I32), C.POINTER(I64),
                                C.POINTER(I64), C.POINTER(I64)],
            "rfd_set_timing": [P, I32],
            "rfd_set_pole_window": [P, I32],
            "rfd_set_interface_groups": [P, I32, P],
            "rfd_inertia_count": [P, F64, F64, C.POINTER(I64), P],
            "rfd_solve_slices": [P, I32, P, I32, I32, I32, P, I32, F64, I32, I32, I32, P, P, P,
                                 C.POINTER(I32), P, C.POINTER(I64), P],
            "rfd_reset_caches": [P, I32],
            "rfd_set_interior_solver": [P, I32],
            "rfd_test_spectral_orthogonality": [P, C.POINTER(F64)],
            "rfd_test_basis": [P, P, I64, C.POINTER(I64), P],
            "rfd_kernel_accounting": [I32],
            "rfd_kernel_stats": [P, P, P, P, P],
            "rfd_phase_times": [P, P],
            "rfd_test_gemm": [I32, I32, I32, I64, I64, I64, F64, F64, P, P, I64, I64, P, P, I64,
                              I64, P, P, I64, I64, I32, P],
            "rfd_test_gemm_static": [I32, I32, I32, I64, I64, I64, F64, F64, P, P, I64, I64, P, P,
                                     I64, I64, P, P, I64, I64, I32, P],
            "rfd_test_gemm_triu_b": [I64, I64, I64, F64, F64, P, I64, I64, P, I64, I64, P, I64,
                                     I64, I32, P],
            "rfd_test_gemm_variant": [I32, I32, I32, I32, I64, I64, I64, F64, F64, P, P, I64, I64,
                                      P, P, I64, I64, P, P, I64, I64, I32, P],
            "rfd_set_gemm_tuning": [P, I32],
            "rfd_device_arch": [P, I32],
            "rfd_test_lu": [I32, I32, I64, I32, P, P, I64, I64, P, P, I64, I64, I64,
                            C.POINTER(C.c_uint32), P],
            "rfd_test_syevx": [I64, I32, P, I32, I32, P, P, P],
            "rfd_test_schur_renumber": [I64, P, P, P, P, P, P, I32, P, C.POINTER(I64),
                                        C.POINTER(I64), C.POINTER(I64), P],
            "rfd_batch_run": [I32, P, C.POINTER(rfd_job), C.POINTER(rfd_result), I32, I64],
            "rfd_server_create": [I32, I64, C.POINTER(P)],
            "rfd_server_submit": [P, P, C.POINTER(rfd_job), C.POINTER(I64)],
            "rfd_server_poll": [P, I64, I32, C.POINTER(rfd_result)],
            "rfd_server_destroy": [P],
            "rfd_server_stats": [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I64),
                                 C.POINTER(I64), C.POINTER(I64)],
            "rfd_server_cache_stats": [P, C.POINTER(I64), C.POINTER(I64)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.rfd_last_error.argtypes = []
        L.rfd_last_error.restype = C.c_char_p
        _lib = L
        _load_tuning(L)
    return _lib


TUNING_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning")
tuning_loaded = None   # path of the GEMM tuning table in use, or None


def device_arch(L=None):
    """The current device's architecture name (e.g. 'gfx950'), or None
    without a device."""
    L = L or lib()
    buf = C.create_string_buffer(64)
    return buf.value.decode() if L.rfd_device_arch(buf, 64) == 0 else None


def _load_tuning(L):
    """Hands the autotuner's table for the device's architecture
    (tuning/<arch>.json, written by python -m paper_1711_09487_amd.tune) to
    rfd_set_gemm_tuning.  RFD_GEMM_TUNING=off keeps the built-in rules;
    RFD_GEMM_TUNING=<path> names another table (for the same architecture)."""
    global tuning_loaded
    env = os.environ.get("RFD_GEMM_TUNING", "")
    if env == "off":
        return
    arch = device_arch(L)
    if arch is None:
        return
    path = env or os.path.join(TUNING_DIR, arch + ".json")
    if not os.path.exists(path):
        return
    import json
    t = json.load(open(path))
    if t.get("arch") != arch:
        raise RuntimeError(f"{path} was tuned for {t.get('arch')}, the device is {arch}")
    ent = np.ascontiguousarray(np.array(t["entries"], dtype=np.int32).reshape(-1, 9))
    code = L.rfd_set_gemm_tuning(ent.ctypes.data, int(ent.shape[0]))
    if code != 0:
        raise RfdError(code, L.rfd_last_error().decode())
    tuning_loaded = path


def rfd_set_gemm_tuning(entries):
    """entries: (count, 9) int32 rows {fp64, complex, transA, transB, log2 M,
    log2 N, log2 K, log2 batch, variant}; an empty table restores the
    built-in rules."""
    ent = np.ascontiguousarray(np.asarray(entries, dtype=np.int32).reshape(-1, 9))
    _check(lib().rfd_set_gemm_tuning(ent.ctypes.data if ent.size else None, int(ent.shape[0])))


def _check(code):
    if code != 0:
        raise RfdError(code, lib().rfd_last_error().decode())


def _ptr(t):
    """Device (or host numpy) address of a contiguous array, None for None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        assert t.flags["C_CONTIGUOUS"] or t.flags["F_CONTIGUOUS"]
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


# ---------------------------------------------------------------------------
# the C entry points, same names
# ---------------------------------------------------------------------------
def rfd_create_pencil(A, M):
    """A, M: scipy.sparse matrices (full symmetric storage)."""
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    M = sp.csr_matrix(M)
    n = A.shape[0]
    arrs = []
    for X in (A, M):
        arrs += [np.ascontiguousarray(X.indptr, dtype=np.int64),
                 np.ascontiguousarray(X.indices, dtype=np.int32),
                 np.ascontiguousarray(X.data, dtype=np.float64)]
    h = P()
    _check(lib().rfd_create_pencil(n, *[a.ctypes.data for a in arrs], C.byref(h)))
    return h


def rfd_set_partition(h, p, part):
    part = np.ascontiguousarray(part, dtype=np.int32)
    _check(lib().rfd_set_partition(h, int(p), part.ctypes.data))


def rfd_set_interval_and_poles(h, alpha, beta, n_c, rule=RFD_RULE_GAUSS, zeta=None, omega=None):
    z = w = None
    if rule == RFD_RULE_EXPLICIT:
        z = np.ascontiguousarray(np.column_stack([np.real(zeta), np.imag(zeta)]).ravel())
        w = np.ascontiguousarray(np.column_stack([np.real(omega), np.imag(omega)]).ravel())
    _check(lib().rfd_set_interval_and_poles(h, float(alpha), float(beta), int(n_c), int(rule),
                                            None if z is None else z.ctypes.data,
                                            None if w is None else w.ctypes.data))


def rfd_set_precision(h, mode, refine_tol=0.0, max_sweeps=0):
    _check(lib().rfd_set_precision(h, int(mode), float(refine_tol), int(max_sweeps)))


def rfd_filter_interface(h, m, Y0, steps, Q, stream=None):
    """Y0: device tensor (s x m, column-major = torch tensor of shape (m, s)
    contiguous); Q: device tensor with room for ldq_cols columns of length s.
    Returns mu."""
    mu = I32()
    ldq_cols = Q.numel() // Y0.shape[-1]
    _check(lib().rfd_filter_interface(h, int(m), _ptr(Y0), int(steps), _ptr(Q), int(ldq_cols),
                                      C.byref(mu), _stream(stream)))
    return mu.value


def rfd_filter_apply(h, m, Y, W, stream=None):
    """W = 2 Re sum_l omega_l S(zeta_l)^{-1} Y; Y, W device tensors (s x m column-major)."""
    _check(lib().rfd_filter_apply(h, int(m), _ptr(Y), _ptr(W), _stream(stream)))


def rfd_filter_lanczos(h, m, Y0, tol, max_steps, Q, test_every=0, stream=None):
    """Alg. 3.1 with its stopping test.  Returns (mu, steps, traces, converged)."""
    mu, st, cv = I32(), I32(), I32()
    tr = np.zeros(max(int(max_steps), 1))
    ldq_cols = Q.numel() // Y0.shape[-1]
    _check(lib().rfd_filter_lanczos(h, int(m), _ptr(Y0), float(tol), int(max_steps),
                                    int(test_every), _ptr(Q), int(ldq_cols), C.byref(mu),
                                    C.byref(st), tr.ctypes.data, C.byref(cv), _stream(stream)))
    return mu.value, st.value, tr[:st.value].copy(), bool(cv.value)


def rfd_prepare_interior(h, sigma, nev_b):
    _check(lib().rfd_prepare_interior(h, float(sigma), int(nev_b)))


def rfd_solve_interior(h, sigma, nev_b, psi, stream=None):
    k = I64()
    _check(lib().rfd_solve_interior(h, float(sigma), int(nev_b), int(psi), C.byref(k),
                                    _stream(stream)))
    return k.value


def rfd_rayleigh_ritz(h, max_out, evals, evecs=None, resid=None, stream=None):
    nf = I32()
    code = lib().rfd_rayleigh_ritz(h, int(max_out), _ptr(evals), _ptr(evecs), _ptr(resid),
                                   C.byref(nf), _stream(stream))
    if code != 0:
        raise RfdError(code, lib().rfd_last_error().decode() + f" (nfound={nf.value})")
    return nf.value


def rfd_destroy_pencil(h):
    _check(lib().rfd_destroy_pencil(h))


def rfd_last_error():
    return lib().rfd_last_error().decode()


def rfd_pencil_info(h):
    n, s, d, b = I64(), I64(), I64(), I64()
    p = I32()
    _check(lib().rfd_pencil_info(h, C.byref(n), C.byref(p), C.byref(s), C.byref(d), C.byref(b)))
    return dict(n=n.value, p=p.value, s=s.value, d_max=d.value, device_bytes=b.value)


def rfd_reset_caches(h, release=False):
    _check(lib().rfd_reset_caches(h, int(bool(release))))


GEMM_KEYS = {8 * f + 4 * c + 2 * a + b: f"k_gemm<{'double' if f else 'float'}, "
             f"{'true' if c else 'false'}, {'true' if a else 'false'}, {'true' if b else 'false'}>"
             for f in (0, 1) for c in (0, 1) for a in (0, 1) for b in (0, 1)}
KERNEL_KEYS = dict(GEMM_KEYS)
KERNEL_KEYS[16] = "k_tri_symv"
KERNEL_KEYS.update({17 + 4 * c + 2 * a + b: f"k_dgemm<{'true' if c else 'false'}, "
                    f"{'true' if a else 'false'}, {'true' if b else 'false'}>"
                    for c in (0, 1) for a in (0, 1) for b in (0, 1)})


def rfd_kernel_accounting(every):
    """Sample every `every`-th launch of the accounted kernels (0: off)."""
    _check(lib().rfd_kernel_accounting(int(every)))


def rfd_kernel_stats():
    """{kernel name: (launches, timed, ms, flops, bytes)} since the last
    call; ms, flops and bytes are estimates over all launches (the launches
    timed for their size summed, a hashed sample of the rest scaled up)."""
    L, S, T, F, B = (np.zeros(32) for _ in range(5))
    _check(lib().rfd_kernel_stats(L.ctypes.data, S.ctypes.data, T.ctypes.data, F.ctypes.data,
                                  B.ctypes.data))
    return {KERNEL_KEYS[k]: (int(L[k]), int(S[k]), float(T[k]), float(F[k]), float(B[k]))
            for k in range(32) if L[k] > 0 and k in KERNEL_KEYS}


def rfd_set_pole_window(h, max_poles):
    _check(lib().rfd_set_pole_window(h, int(max_poles)))


def rfd_set_interior_solver(h, kind):
    _check(lib().rfd_set_interior_solver(h, int(kind)))


def rfd_test_spectral_orthogonality(h):
    v = C.c_double(0.0)
    _check(lib().rfd_test_spectral_orthogonality(h, C.byref(v)))
    return v.value


def rfd_test_schur_renumber(A, M, part):
    """Host-side renumbering behind the Schur solves on trailing blocks for
    scipy CSR matrices A, M (full symmetric storage) and a partition vector
    (subdomain index, -1 on the interface): returns (D, TS, SJ, pos) with pos
    the row of each interior node in its subdomain's renumbered block (-1 on
    the interface).  No device work."""
    A = A.tocsr()
    M = M.tocsr()
    n = A.shape[0]
    arrs = [np.ascontiguousarray(x, dtype=t) for x, t in
            ((A.indptr, np.int64), (A.indices, np.int32), (A.data, np.float64),
             (M.indptr, np.int64), (M.indices, np.int32), (M.data, np.float64))]
    part = np.ascontiguousarray(part, dtype=np.int32)
    pos = np.empty(n, dtype=np.int32)
    D, TS, SJ = I64(), I64(), I64()
    _check(lib().rfd_test_schur_renumber(n, *[a.ctypes.data for a in arrs], int(part.max()) + 1,
                                         part.ctypes.data, C.byref(D), C.byref(TS), C.byref(SJ),
                                         pos.ctypes.data))
    return D.value, TS.value, SJ.value, pos


def rfd_test_basis(h, dst, cap, stream=None):
    """Copies up to cap columns of the M-orthonormal basis of range(Z) (n
    rows, interiors then interface) into the device array dst; returns the
    number of columns the basis has."""
    k = I64()
    _check(lib().rfd_test_basis(h, _ptr(dst), int(cap), C.byref(k), _stream(stream)))
    return k.value


def rfd_set_interface_groups(h, group):
    """group: int32 per interface node (interface order), -1 for the top set,
    or None for the dense S."""
    if group is None:
        _check(lib().rfd_set_interface_groups(h, 0, None))
        return
    g = np.ascontiguousarray(group, dtype=np.int32)
    _check(lib().rfd_set_interface_groups(h, int(g.max()) + 1, g.ctypes.data))


def rfd_inertia_count(h, alpha, beta, stream=None):
    c = I64()
    _check(lib().rfd_inertia_count(h, float(alpha), float(beta), C.byref(c), _stream(stream)))
    return c.value


def rfd_solve_slices(h, cuts, n_c, rule, Y0, steps, sigma, nev_b, psi, evals, evecs=None,
                     resid=None, check_inertia=True, stream=None):
    cuts = np.ascontiguousarray(cuts, dtype=np.float64)
    ns = cuts.size - 1
    counts = np.zeros(ns, dtype=np.int32)
    nf, inert = I32(), I64()
    _check(lib().rfd_solve_slices(h, int(ns), cuts.ctypes.data, int(n_c), int(rule),
                                  int(Y0.shape[0]), _ptr(Y0), int(steps), float(sigma), int(nev_b),
                                  int(psi), int(evals.numel()), _ptr(evals),
                                  _ptr(evecs) if evecs is not None else None,
                                  _ptr(resid) if resid is not None else None, C.byref(nf),
                                  counts.ctypes.data, C.byref(inert) if check_inertia else None,
                                  _stream(stream)))
    return nf.value, counts, (inert.value if check_inertia else None)


def rfd_set_timing(h, on):
    _check(lib().rfd_set_timing(h, int(bool(on))))


def rfd_phase_times(h):
    out = np.zeros(16)
    _check(lib().rfd_phase_times(h, out.ctypes.data))
    return out


class Pencil:
    """Owning wrapper of a pencil handle (argument marshalling only)."""

    def __init__(self, A, M):
        self.h = rfd_create_pencil(A, M)
        self.n = A.shape[0]

    def close(self):
        if self.h is not None:
            rfd_destroy_pencil(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_partition(self, part):
        part = np.asarray(part, dtype=np.int32)
        rfd_set_partition(self.h, int(part.max()) + 1, part)
        self.s = int(np.count_nonzero(part < 0))

    def set_interval_and_poles(self, alpha, beta, n_c, rule=RFD_RULE_GAUSS, zeta=None, omega=None):
        rfd_set_interval_and_poles(self.h, alpha, beta, n_c, rule, zeta, omega)

    def set_precision(self, mode, refine_tol=0.0, max_sweeps=0):
        rfd_set_precision(self.h, mode, refine_tol, max_sweeps)

    def filter_interface(self, Y0, steps, stream=None):
        """Y0: torch float64 tensor on the GPU, shape (m, s) (i.e. s x m
        column-major).  Returns Q as a (mu, s) tensor (s x mu column-major)."""
        import torch
        m, s = Y0.shape
        cols = min(s, steps * m)
        Q = torch.empty((cols, s), dtype=torch.float64, device=Y0.device)
        mu = rfd_filter_interface(self.h, m, Y0, steps, Q, stream)
        return Q[:mu]

    def filter_lanczos(self, Y0, tol=1e-6, max_steps=64, test_every=0, stream=None):
        """Alg. 3.1 on the block Y0 ((m, s) tensor); returns (Q as (mu, s),
        info dict with steps, traces, converged)."""
        import torch
        m, s = Y0.shape
        Q = torch.empty((min(s, max_steps * m), s), dtype=torch.float64, device=Y0.device)
        mu, st, tr, cv = rfd_filter_lanczos(self.h, m, Y0, tol, max_steps, Q, test_every, stream)
        return Q[:mu], dict(steps=st, traces=tr, converged=cv)

    def filter_apply(self, Y, stream=None):
        import torch
        W = torch.empty_like(Y)
        rfd_filter_apply(self.h, Y.shape[0], Y, W, stream)
        return W

    def prepare_interior(self, sigma, nev_b):
        rfd_prepare_interior(self.h, sigma, nev_b)

    def solve_interior(self, sigma, nev_b, psi, stream=None):
        return rfd_solve_interior(self.h, sigma, nev_b, psi, stream)

    def rayleigh_ritz(self, max_out, vectors=True, residuals=True, device="cuda", stream=None):
        import torch
        ev = torch.empty(max_out, dtype=torch.float64, device=device)
        X = torch.empty((max_out, self.n), dtype=torch.float64, device=device) if vectors else None
        r = torch.empty(max_out, dtype=torch.float64, device=device) if residuals else None
        nf = rfd_rayleigh_ritz(self.h, max_out, ev, X, r, stream)
        return ev[:nf], (X[:nf] if X is not None else None), (r[:nf] if r is not None else None)

    def reset_caches(self, release=False):
        rfd_reset_caches(self.h, release)

    def set_timing(self, on=True):
        rfd_set_timing(self.h, on)

    def set_pole_window(self, max_poles):
        rfd_set_pole_window(self.h, max_poles)

    def set_interface_groups(self, group):
        rfd_set_interface_groups(self.h, group)

    def set_interior_solver(self, kind):
        rfd_set_interior_solver(self.h, kind)

    def spectral_orthogonality(self):
        return rfd_test_spectral_orthogonality(self.h)

    def basis(self, cap, stream=None):
        """The basis of range(Z) of the last solve_interior (device tensor
        of shape (k, n): column-major n x k, reordered numbering)."""
        import torch
        Z = torch.empty((max(int(cap), 1), self.n), dtype=torch.float64, device="cuda")
        k = rfd_test_basis(self.h, Z, cap, stream)
        return Z[:min(k, int(cap))]

    def inertia_count(self, alpha, beta, stream=None):
        return rfd_inertia_count(self.h, alpha, beta, stream)

    def solve_slices(self, cuts, n_c, Y0, steps, nev_b, psi, max_out, sigma=float("nan"),
                     rule=RFD_RULE_GAUSS, vectors=False, check_inertia=True, stream=None):
        """Spectrum slicing of [cuts[0], cuts[-1]]: returns (evals, evecs or
        None, resid, counts per slice, inertia count)."""
        import torch
        dev = Y0.device
        ev = torch.empty(max_out, dtype=torch.float64, device=dev)
        n = self.info()["n"]
        X = torch.empty((max_out, n), dtype=torch.float64, device=dev) if vectors else None
        r = torch.empty(max_out, dtype=torch.float64, device=dev)
        nf, counts, inert = rfd_solve_slices(self.h, cuts, n_c, rule, Y0, steps, sigma, nev_b, psi,
                                             ev, X, r, check_inertia, stream)
        return ev[:nf], (X[:nf] if vectors else None), r[:nf], counts, inert

    def phase_times(self):
        return rfd_phase_times(self.h)

    def info(self):
        return rfd_pencil_info(self.h)


# ---------------------------------------------------------------------------
# batching and serving
# ---------------------------------------------------------------------------
class Job:
    """One complete solve on a pencil (fields of struct rfd_job).  Y0 is a
    device tensor of shape (m, s) (s x m column-major); the outputs are
    allocated here on the device (evals, eigenvectors as (max_out, n),
    residuals) and stay referenced by the Job until it is collected."""

    def __init__(self, pencil, alpha, beta, n_c, Y0, steps, sigma, nev_b, psi, max_out,
                 mode=RFD_FP64, rule=RFD_RULE_GAUSS, refine_tol=0.0, max_sweeps=0,
                 vectors=True, residuals=True):
        import torch
        self.pencil = pencil
        self.Y0 = Y0
        m = Y0.shape[0]
        dev = Y0.device
        self.evals = torch.empty(max(max_out, 1), dtype=torch.float64, device=dev)
        self.evecs = (torch.empty((max(max_out, 1), pencil.n), dtype=torch.float64, device=dev)
                      if vectors else None)
        self.resid = torch.empty(max(max_out, 1), dtype=torch.float64, device=dev) if residuals else None
        self.c = rfd_job(float(alpha), float(beta), int(n_c), int(rule), int(mode),
                         int(max_sweeps), float(refine_tol), int(m), int(steps), _ptr(Y0),
                         float(sigma), int(nev_b), int(psi), int(max_out), _ptr(self.evals),
                         _ptr(self.evecs), _ptr(self.resid))
        self.result = None

    def outputs(self):
        """(evals, eigenvectors, residuals) of a finished job, trimmed to nfound."""
        nf = self.result.nfound if self.result is not None else 0
        return (self.evals[:nf], None if self.evecs is None else self.evecs[:nf],
                None if self.resid is None else self.resid[:nf])


def _result_dict(r):
    return dict(status=r.status, nfound=r.nfound, mu=r.mu, worker=r.worker, k=r.k,
                bytes=r.bytes, queued_s=r.queued_s, run_s=r.run_s, message=r.message.decode())


def rfd_batch_run(jobs, workers=0, hbm_budget=0):
    """Runs the Job objects concurrently (rfd_batch_run); sets job.result and
    returns the status code (0 when every job succeeded)."""
    nb = len(jobs)
    pens = (P * nb)(*[j.pencil.h for j in jobs])
    cj = (rfd_job * nb)(*[j.c for j in jobs])
    res = (rfd_result * nb)()
    code = lib().rfd_batch_run(nb, pens, cj, res, int(workers), int(hbm_budget))
    for j, r in zip(jobs, res):
        j.result = r
    return code


def batch_run(jobs, workers=0, hbm_budget=0):
    """As rfd_batch_run, raising if a job failed; returns the result dicts."""
    code = rfd_batch_run(jobs, workers, hbm_budget)
    out = [_result_dict(j.result) for j in jobs]
    if code != 0:
        bad = [o for o in out if o["status"] != 0]
        raise RfdError(code, f"{len(bad)} job(s) failed; first: {bad[0]['message'] if bad else ''}")
    return out


class Server:
    """Serving loop (rfd_server_*): submit Jobs, poll for results."""

    def __init__(self, workers=0, hbm_budget=0):
        self.h = P()
        _check(lib().rfd_server_create(int(workers), int(hbm_budget), C.byref(self.h)))
        self.jobs = {}

    def submit(self, job):
        rid = I64()
        _check(lib().rfd_server_submit(self.h, job.pencil.h, C.byref(job.c), C.byref(rid)))
        self.jobs[rid.value] = job
        return rid.value

    def poll(self, rid, wait=False):
        """The result dict when finished, None while pending."""
        r = rfd_result()
        code = lib().rfd_server_poll(self.h, int(rid), int(bool(wait)), C.byref(r))
        if code == RFD_EPENDING:
            return None
        _check(code)
        job = self.jobs.pop(rid)
        job.result = r
        return _result_dict(r)

    def stats(self):
        q, rn = I32(), I32()
        br, bc, ev = I64(), I64(), I64()
        _check(lib().rfd_server_stats(self.h, C.byref(q), C.byref(rn), C.byref(br), C.byref(bc),
                                      C.byref(ev)))
        hi, mi = I64(), I64()
        _check(lib().rfd_server_cache_stats(self.h, C.byref(hi), C.byref(mi)))
        return dict(queued=q.value, running=rn.value, bytes_running=br.value,
                    bytes_cached=bc.value, evictions=ev.value, cache_hits=hi.value,
                    cache_misses=mi.value)

    def close(self):
        if self.h is not None and self.h.value is not None:
            _check(lib().rfd_server_destroy(self.h))
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
