"""RF-DDES oracle (FP64, CPU, numpy/scipy LAPACK).  TEST INFRASTRUCTURE ONLY:
imported by the test-suite, the smoke check and the benchmark's CPU-baseline
leg, never by the GPU library.  See the package docstring for the map from
functions to the paper's sections and equations.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np
import scipy.linalg as sl
import scipy.sparse as sp

__all__ = [
    "quadrature", "rho", "DD", "schur", "factor_poles", "filter_apply", "filter_apply_streamed",
    "orth",
    "filter_interface", "filter_lanczos", "block_tridiagonal", "interior_basis",
    "interior_levels", "build_z",
    "rayleigh_ritz", "residuals", "norm_a", "inertia_count", "run", "OracleResult",
]

ORTH_TOL = 1e-13      # relative drop tolerance of the interface orthonormalisation
RR_TOL = 1e-12        # relative singular-value cut of the Rayleigh-Ritz basis
CLUSTER_RTOL = 1e-9   # V_j selection: keep whole clusters at the cut


# ---------------------------------------------------------------------------
# Sec. 2.1: the rational filter
# ---------------------------------------------------------------------------
def quadrature(alpha: float, beta: float, n_c: int, rule: str = "gauss"):
    """Poles zeta_l and weights omega_l (l = 1..n_c, upper half plane) of the
    discretised Cauchy integral of the indicator of [alpha, beta], eq. (2.1):
    I(z) = -1/(2 pi i) \\oint dnu / (z - nu) over the circle with centre
    c = (alpha+beta)/2 and radius r = (beta-alpha)/2, counter-clockwise.

    With nu(theta) = c + r e^{i theta}, dnu = i r e^{i theta} dtheta, so a rule
    with nodes theta_l and weights h_l on [0, 2 pi) gives
        rho(z) = sum_l omega_l / (z - zeta_l),  zeta_l = nu(theta_l),
        omega_l = -(1/(2 pi)) r e^{i theta_l} h_l.
    The nodes come in conjugate pairs; only the n_c with Im > 0 are returned
    and rho(x) = 2 Re sum_l omega_l / (x - zeta_l) for real x, eq. (2.3).

    rule = "midpoint": 2 n_c equispaced nodes theta_l = (l - 1/2) pi / n_c
    (the paper's rule, Sec. 6); rule = "gauss": n_c Gauss-Legendre nodes t_k
    mapped to the upper half circle, theta_k = (pi/2)(1 + t_k), h_k = (pi/2) w_k
    (the paper's Fig. 2.1, left).
    """
    if not (beta > alpha):
        raise ValueError("need alpha < beta")
    if n_c < 1:
        raise ValueError("need n_c >= 1")
    c = 0.5 * (alpha + beta)
    r = 0.5 * (beta - alpha)
    if rule == "midpoint":
        theta = (np.arange(1, n_c + 1) - 0.5) * np.pi / n_c
        h = np.full(n_c, np.pi / n_c)
    elif rule == "gauss":
        t, w = np.polynomial.legendre.leggauss(n_c)
        theta = 0.5 * np.pi * (1.0 + t)
        h = 0.5 * np.pi * w
    else:
        raise ValueError(rule)
    e = np.exp(1j * theta)
    zeta = c + r * e
    omega = -(1.0 / (2.0 * np.pi)) * r * e * h
    return zeta, omega


def rho(x, zeta, omega):
    """Filter value at real x, eq. (2.3)."""
    x = np.asarray(x, dtype=np.float64)
    return 2.0 * np.real(np.sum(omega[None, :] / (x.reshape(-1, 1) - zeta[None, :]), axis=1)
                         ).reshape(x.shape)


# ---------------------------------------------------------------------------
# Sec. 2.3: interior-first reordering, eqs. (2.5)-(2.6)
# ---------------------------------------------------------------------------
class DD:
    """Block structure of (A, M) under a partition.

    part[i] = j >= 0 puts node i in the interior of subdomain j, part[i] = -1
    makes it an interface node.  Interiors and the interface keep ascending
    global order.  Interface nodes belong to no subdomain (vertex separators),
    so E_j couples interior j to the interface nodes adjacent to it; these are
    the columns ``adj[j]`` (positions in the interface list) and the dense
    d_j x s_j matrix Ehat_j = E[interior_j, adj_j] plays the role of the
    nonzero part of E_j in eq. (2.5).
    """

    def __init__(self, A: sp.spmatrix, M: sp.spmatrix, part: np.ndarray,
                 dense_interface: bool = True):
        A = sp.csr_matrix(A)
        M = sp.csr_matrix(M)
        part = np.asarray(part)
        n = A.shape[0]
        self.n = n
        self.p = int(part.max()) + 1
        self.interior = [np.flatnonzero(part == j) for j in range(self.p)]
        self.iface = np.flatnonzero(part < 0)
        self.s = self.iface.size
        pos = -np.ones(n, dtype=np.int64)
        pos[self.iface] = np.arange(self.s)
        G = (abs(A) + abs(M)).tocsr()
        coo = G.tocoo()
        pi, pj = part[coo.row], part[coo.col]
        if np.any((pi >= 0) & (pj >= 0) & (pi != pj)):
            raise ValueError("two subdomains are coupled directly, not through the interface")
        self.adj = []
        self.B, self.MB, self.E, self.ME = [], [], [], []
        for j in range(self.p):
            I = self.interior[j]
            cols = np.unique(G[I].indices)
            cols = cols[part[cols] < 0]
            a = np.sort(pos[cols])
            self.adj.append(a)
            J = self.iface[a]
            self.B.append(A[I][:, I].toarray())
            self.MB.append(M[I][:, I].toarray())
            self.E.append(A[I][:, J].toarray())
            self.ME.append(M[I][:, J].toarray())
        # C and M_C dense, or sparse for large interfaces (dense_interface=False,
        # where an s x s real array per matrix would not fit beside S(z))
        self.C = A[self.iface][:, self.iface]
        self.MC = M[self.iface][:, self.iface]
        if dense_interface:
            self.C = self.C.toarray()
            self.MC = self.MC.toarray()
        self.A = A
        self.M = M
        self.part = part
        self.m_e_zero = all(np.count_nonzero(x) == 0 for x in self.ME)

    def order(self):
        """Global ids in the reordered sequence: interiors 0..p-1, then interface."""
        return np.concatenate(self.interior + [self.iface])


# ---------------------------------------------------------------------------
# Sec. 3.1: Schur complement and the interface filter
# ---------------------------------------------------------------------------
def schur(dd: DD, z: complex) -> np.ndarray:
    """S(z) = C_z - E_z^T B_z^{-1} E_z with B_z = B - z M_B, E_z = E - z M_E,
    C_z = C - z M_C (Sec. 3.1).  A - zM is complex *symmetric*, so the
    transpose is the plain transpose (the paper prints ^H; with real M_E the
    two differ only when M_E != 0).  B_z is block diagonal, so the sum runs
    over subdomains; each B_j(z) is factored with partial pivoting (zgetrf)."""
    if sp.issparse(dd.C):
        Cz = sp.coo_matrix(dd.C - z * dd.MC)
        S = np.zeros((dd.s, dd.s), dtype=np.complex128, order="F")
        S[Cz.row, Cz.col] = Cz.data
    else:
        S = np.asfortranarray((dd.C - z * dd.MC).astype(np.complex128))
    for j in range(dd.p):
        K = dd.B[j] - z * dd.MB[j]
        Ez = dd.E[j] - z * dd.ME[j]
        X = sl.lu_solve(sl.lu_factor(K, check_finite=False), Ez, check_finite=False)
        a = dd.adj[j]
        S[np.ix_(a, a)] -= Ez.T @ X
    return S


def factor_poles(dd: DD, zeta) -> list:
    return [sl.lu_factor(schur(dd, z), check_finite=False) for z in zeta]


def filter_apply(factors, omega, Y: np.ndarray) -> np.ndarray:
    """W = 2 Re sum_l omega_l S(zeta_l)^{-1} Y, the left side of eq. (3.5)."""
    W = np.zeros(Y.shape, dtype=np.float64)
    for f, w in zip(factors, omega):
        W += 2.0 * np.real(w * sl.lu_solve(f, Y.astype(np.complex128), check_finite=False))
    return W


def filter_apply_streamed(dd: DD, zeta, omega, Y: np.ndarray) -> np.ndarray:
    """The same W as filter_apply(factor_poles(dd, zeta), omega, Y), with one
    pole's S(zeta_l) and its LU in memory at a time: each pole is assembled,
    factored in place, applied and dropped, and the terms are added in the
    same (ascending pole) order.  For interfaces whose dense S(zeta) takes
    tens of GB per pole."""
    W = np.zeros(Y.shape, dtype=np.float64)
    Yc = Y.astype(np.complex128)
    for z, w in zip(zeta, omega):
        f = sl.lu_factor(schur(dd, z), overwrite_a=True, check_finite=False)
        W += 2.0 * np.real(w * sl.lu_solve(f, Yc, check_finite=False))
        del f
    return W


def orth(W: np.ndarray, K: Optional[np.ndarray] = None, tol: float = ORTH_TOL) -> np.ndarray:
    """Orthonormal basis of the part of range(W) outside range(K).

    W is first projected against K twice (full reorthogonalisation, Alg. 3.1
    lines 4-6).  Then Householder QR with column pivoting; directions whose
    pivot |R_ii| falls to tol times the largest column norm of the
    *unprojected* W are dropped (Alg. 3.1 lines 8-9 drop a vanishing w)."""
    scale = float(np.max(np.linalg.norm(W, axis=0))) if W.size else 0.0
    if scale == 0.0:
        return np.zeros((W.shape[0], 0))
    if K is not None and K.shape[1] > 0:
        for _ in range(2):
            W = W - K @ (K.T @ W)
    Qf, R, _ = sl.qr(W, mode="economic", pivoting=True, check_finite=False)
    d = np.abs(np.diag(R))
    keep = 0
    while keep < d.size and d[keep] > tol * scale:
        keep += 1
    return np.asfortranarray(Qf[:, :keep])


def filter_interface(dd: DD, zeta, omega, Y0: np.ndarray, steps: int, factors=None,
                     streamed: bool = False, keep: Optional[dict] = None):
    """Interface subspace Q (s x mu), Sec. 3.2.

    Alg. 3.1 is a Lanczos process on F = 2 Re sum omega_l S(zeta_l)^{-1} with
    full reorthogonalisation.  Here it is run on a block: Q_1 = orth(F Y0),
    Q_t = orth(F Q_{t-1}) against [Q_1..Q_{t-1}], t = 2..steps, and
    Q = [Q_1, .., Q_steps] spans the block Krylov space
    span{F Y0, F^2 Y0, .., F^steps Y0}.

    streamed=True applies F with filter_apply_streamed (every application
    factors the poles again, one at a time).  keep, when given, receives the
    first filtered block F Y0 under "W1"."""
    if streamed:
        F = lambda X: filter_apply_streamed(dd, zeta, omega, X)
    else:
        if factors is None:
            factors = factor_poles(dd, zeta)
        F = lambda X: filter_apply(factors, omega, X)
    W = F(Y0)
    if keep is not None:
        keep["W1"] = W
    Qt = orth(W)
    K = Qt
    for _ in range(2, steps + 1):
        if Qt.shape[1] == 0 or K.shape[1] >= dd.s:
            break
        W = F(Qt)
        Qt = orth(W, K)
        K = np.hstack([K, Qt])
    return np.asfortranarray(K), factors


LANCZOS_TOL = 1e-6    # Sec. 6: tolerance of the stopping test of Alg. 3.1
LANCZOS_EVERY = 10    # Sec. 6: the test is applied every ten iterations


def filter_lanczos(dd: DD, zeta, omega, Y0: np.ndarray, tol: float = LANCZOS_TOL,
                   max_steps: int = 64, factors=None, streamed: bool = False,
                   every: int = LANCZOS_EVERY, keep: Optional[dict] = None):
    """Alg. 3.1 (Sec. 3.2), Lanczos restricted to the interface, run on a
    block of m = Y0.shape[1] vectors with full reorthogonalisation, on
    F = 2 Re sum_l omega_l S(zeta_l)^{-1} (eq. (3.5)):

      Q_1 = orth(Y0)                               (the start block, line 0)
      for t = 1, 2, ...:
        W = F Q_t                                  (line 2)
        A_t = Q_t^T W                              (line 3, a_mu = w^T q)
        the sum of the eigenvalues of T_t is its trace, sum_i tr(A_i); the
        process stops when it changed by at most tol (relative) since the
        last test (line 13), the test running every `every` vectors
        Q_{t+1} = orth(W) against Q_1..Q_t, twice  (lines 4-12; a vanishing
        direction is dropped, line 8)
        B_{t+1} = Q_{t+1}^T W                      (b_{mu+1})
      Q = [Q_1 .. Q_t]                             (line 15)

    Returns (Q, info) with info: steps, traces (after every block), the
    blocks A_t and B_t (block tridiagonal T), converged."""
    if streamed:
        F = lambda X: filter_apply_streamed(dd, zeta, omega, X)
    else:
        if factors is None:
            factors = factor_poles(dd, zeta)
        F = lambda X: filter_apply(factors, omega, X)
    m = Y0.shape[1]
    test_blocks = max(1, -(-every // m))          # blocks per test of the stopping rule
    Qt = orth(Y0)
    K = Qt
    As, Bs, traces = [], [], []
    tr = 0.0
    tr_test = None
    converged = False
    t = 0
    while Qt.shape[1] > 0:
        t += 1
        W = F(Qt)
        A = Qt.T @ W
        As.append(A)
        tr += float(np.trace(A))
        traces.append(tr)
        if t % test_blocks == 0:
            if tr_test is not None and abs(tr - tr_test) <= tol * abs(tr):
                converged = True
                break
            tr_test = tr
        if t >= max_steps or K.shape[1] >= dd.s:
            break
        Qn = orth(W, K)
        if Qn.shape[1] == 0:
            break
        Bs.append(Qn.T @ W)
        K = np.hstack([K, Qn])
        Qt = Qn
    if keep is not None:
        keep["F"] = F
    return np.asfortranarray(K), dict(steps=t, traces=traces, A=As, B=Bs, converged=converged)


def block_tridiagonal(info) -> np.ndarray:
    """T_t of Alg. 3.1 in block form: diagonal blocks A_1..A_t, sub-diagonal
    blocks B_2..B_t (B_{i+1} sits below A_i) and their transposes above."""
    sizes = [a.shape[0] for a in info["A"]]
    off = np.concatenate([[0], np.cumsum(sizes)])
    T = np.zeros((off[-1], off[-1]))
    for i, a in enumerate(info["A"]):
        T[off[i]:off[i + 1], off[i]:off[i + 1]] = a
    for i, b in enumerate(info["B"][:len(sizes) - 1]):
        T[off[i + 1]:off[i + 2], off[i]:off[i + 1]] = b
        T[off[i]:off[i + 1], off[i + 1]:off[i + 2]] = b.T
    return T


# ---------------------------------------------------------------------------
# Sec. 4 / 5: interior part
# ---------------------------------------------------------------------------
def interior_basis(dd: DD, sigma: float, nev_b: int):
    """V_j: eigenvectors of (B_j, M_B^(j)) for the nev_b eigenvalues closest
    to sigma (Alg. 5.1 step 3 asks for the smallest in magnitude of
    (B_j - sigma M_B, M_B)), M_B-orthonormal (dsygvd).  A cluster straddling
    the cut is kept whole.  Columns in ascending eigenvalue order."""
    V, D = [], []
    for j in range(dd.p):
        d = dd.B[j].shape[0]
        if nev_b <= 0 or d == 0:
            V.append(np.zeros((d, 0)))
            D.append(np.zeros(0))
            continue
        w, X = sl.eigh(dd.B[j], dd.MB[j], check_finite=False)
        dist = np.abs(w - sigma)
        order = np.argsort(dist, kind="stable")
        k = min(nev_b, d)
        cut = dist[order[k - 1]]
        while k < d and dist[order[k]] <= cut * (1.0 + CLUSTER_RTOL) + 1e-300:
            k += 1
        sel = np.sort(order[:k])
        V.append(np.asfortranarray(X[:, sel]))
        D.append(w[sel])
    return V, D


def interior_levels(dd: DD, sigma: float, psi: int, Q: np.ndarray, V=None):
    """Sigma_j^(psi) and Gamma_j^(psi), eqs. (5.2)-(5.4):
    Phi_j = (E_j - sigma M_E^(j)) Q_j, Psi_j = M_E^(j) Q_j,
    level 1 = B_sigma^{-1} Phi, level k+1 = B_sigma^{-1} M_B (level k).
    B_sigma^(j) = B_j - sigma M_B^(j) is real symmetric indefinite in general:
    LU with partial pivoting (dgetrf).

    If V is given, each level is made M_B-orthogonal to V_j before it is
    used and before the next level is formed (deflated recurrence).  V_j is
    part of Z and B_sigma^{-1} M_B maps span(V_j) into itself, so this leaves
    span(Z) unchanged while removing the directions that the recurrence
    amplifies by 1/|delta - sigma|^k."""
    Sig, Gam = [], []
    for j in range(dd.p):
        a = dd.adj[j]
        Qj = Q[a, :]
        d = dd.B[j].shape[0]
        lu = sl.lu_factor(dd.B[j] - sigma * dd.MB[j], check_finite=False)
        Vj = None if V is None else V[j]

        def defl(X):
            if Vj is None or Vj.shape[1] == 0:
                return X
            return X - Vj @ (Vj.T @ (dd.MB[j] @ X))

        def levels(R):
            out = []
            X = defl(sl.lu_solve(lu, R, check_finite=False))
            out.append(X)
            for _ in range(1, psi):
                X = defl(sl.lu_solve(lu, dd.MB[j] @ X, check_finite=False))
                out.append(X)
            return np.hstack(out) if out else np.zeros((d, 0))

        Sig.append(levels((dd.E[j] - sigma * dd.ME[j]) @ Qj))
        Gam.append(None if dd.m_e_zero else levels(dd.ME[j] @ Qj))
    return Sig, Gam


def build_z(dd: DD, V, Sig, Gam, Q: np.ndarray, psi: int) -> np.ndarray:
    """Z of eq. (5.5) in the reordered numbering (interiors, then interface):
    block rows [V_j, -Sigma_j^(psi), Gamma_j^(psi)] and the interface row
    [0, [Q, 0_{s,(psi-1)mu}], 0]."""
    mu = Q.shape[1]
    kap = sum(v.shape[1] for v in V)
    ng = 0 if dd.m_e_zero else psi * mu
    k = kap + psi * mu + ng
    d_off = np.cumsum([0] + [b.shape[0] for b in dd.B])
    Z = np.zeros((dd.n, k))
    c = 0
    for j in range(dd.p):
        r0, r1 = d_off[j], d_off[j + 1]
        Z[r0:r1, c:c + V[j].shape[1]] = V[j]
        c += V[j].shape[1]
    for j in range(dd.p):
        r0, r1 = d_off[j], d_off[j + 1]
        Z[r0:r1, kap:kap + psi * mu] = -Sig[j]
        if ng:
            Z[r0:r1, kap + psi * mu:] = Gam[j]
    Z[d_off[-1]:, kap:kap + mu] = Q
    return Z


def _m_half(Mr: sp.spmatrix):
    """Returns (apply L^T, apply L^{-T}) with Mr = L L^T: sqrt for a diagonal
    M, dense Cholesky otherwise (small test pencils only)."""
    Mr = sp.csr_matrix(Mr)
    off = Mr - sp.diags(Mr.diagonal())
    if off.nnz == 0 or np.all(off.data == 0):
        h = np.sqrt(Mr.diagonal())
        return (lambda X: h[:, None] * X), (lambda X: X / h[:, None])
    L = np.linalg.cholesky(Mr.toarray())
    return (lambda X: L.T @ X), (lambda X: sl.solve_triangular(L.T, X, lower=False))


def rayleigh_ritz(dd: DD, Z: np.ndarray, alpha: float, beta: float, tol: float = RR_TOL):
    """Alg. 5.1 step 7: Z^T A Z G = Z^T M Z G Lambda, solved through an
    M-orthonormal basis of range(Z): columns scaled to unit M-norm, Householder
    QR of L^T Z (M = L L^T), SVD of R, singular values <= tol * max dropped.
    Returns the Ritz values in [alpha, beta] (ascending) and the Ritz vectors
    in the reordered numbering."""
    order = dd.order()
    Ar = dd.A[order][:, order]
    Mr = dd.M[order][:, order]
    lt, lti = _m_half(Mr)
    cn = np.sqrt(np.maximum(np.einsum("ij,ij->j", Z, Mr @ Z), 0.0))
    keep = cn > 0
    # (intermediates of n x k are dropped as soon as they are used, so that
    # the largest pencils hold about three of them at a time)
    LZ = np.asfortranarray(lt(Z[:, keep] / cn[keep]))
    Qh, R = sl.qr(LZ, mode="economic", overwrite_a=True, check_finite=False)
    del LZ
    U, sv, _ = np.linalg.svd(R)
    r = int(np.count_nonzero(sv > tol * sv[0]))
    Xb = Qh @ U[:, :r]
    del Qh
    Xb = lti(Xb)                          # M-orthonormal basis of range(Z)
    AX = Ar @ Xb
    H = Xb.T @ AX
    del AX
    H = 0.5 * (H + H.T)
    th, G = np.linalg.eigh(H)
    sel = (th >= alpha) & (th <= beta)
    return th[sel], Xb @ G[:, sel], r


def norm_a(A: sp.spmatrix) -> float:
    """||A|| in the residual: the largest absolute row sum (= ||A||_1 = ||A||_inf
    for symmetric A), an upper bound of ||A||_2 that needs no iteration."""
    return float(np.max(np.asarray(abs(A).sum(axis=1)).ravel()))


def residuals(A, M, theta, X) -> np.ndarray:
    """||A x - theta M x||_2 / (||A|| ||x||_2) per Ritz pair."""
    if X.shape[1] == 0:
        return np.zeros(0)
    R = A @ X - (M @ X) * theta[None, :]
    return np.linalg.norm(R, axis=0) / (norm_a(A) * np.linalg.norm(X, axis=0))


# ---------------------------------------------------------------------------
# Sylvester inertia: exact eigenvalue count in [alpha, beta]
# ---------------------------------------------------------------------------
def _neg_count_dense(Xs: np.ndarray) -> int:
    _, D, _ = sl.ldl(Xs, lower=True)
    # D is block diagonal with 1x1 and 2x2 blocks; its inertia is that of Xs
    return int(np.count_nonzero(np.linalg.eigvalsh(D) < 0))


def inertia_count(A, M, alpha: float, beta: float, dd: Optional[DD] = None) -> int:
    """Number of eigenvalues of (A, M) in [alpha, beta] = nu(A - beta M) -
    nu(A - alpha M), nu = number of negative eigenvalues (Sylvester).  For a
    large pencil, with a partition, Haynsworth additivity gives
    nu(A - tau M) = sum_j nu(B_j - tau M_Bj) + nu(S(tau)) at real tau."""
    def nu(tau):
        if dd is None:
            return _neg_count_dense((A - tau * M).toarray())
        tot = 0
        S = dd.C - tau * dd.MC
        for j in range(dd.p):
            K = dd.B[j] - tau * dd.MB[j]
            Et = dd.E[j] - tau * dd.ME[j]
            tot += _neg_count_dense(K)
            a = dd.adj[j]
            S[np.ix_(a, a)] -= Et.T @ np.linalg.solve(K, Et)
        return tot + _neg_count_dense(0.5 * (S + S.T))
    return nu(beta) - nu(alpha)


# ---------------------------------------------------------------------------
# end to end: Alg. 5.1
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class OracleResult:
    theta: np.ndarray
    X: np.ndarray           # Ritz vectors in the ORIGINAL numbering
    resid: np.ndarray
    mu: int
    k: int
    rank: int
    Q: np.ndarray
    times: dict
    W1: Optional[np.ndarray] = None   # first filtered block F Y0 (eq. (3.5))


def run(prob, want_vectors: bool = True, deflate_levels: bool = True,
        streamed: bool = False, lanczos: Optional[dict] = None) -> OracleResult:
    """Alg. 5.1 on a workloads.Problem.  streamed=True: sparse C, M_C and one
    pole's S(zeta) at a time (filter_apply_streamed), for the largest
    pencils; the arithmetic is that of the default path.  lanczos = dict(tol=,
    max_steps=) computes Q by filter_lanczos (Alg. 3.1 with its stopping test)
    instead of prob.steps fixed block-Krylov steps."""
    t = {}
    t0 = time.perf_counter()
    dd = DD(prob.A, prob.M, prob.part, dense_interface=not streamed)
    zeta, omega = quadrature(prob.alpha, prob.beta, prob.n_c, prob.rule)
    t["setup"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    V, _ = interior_basis(dd, prob.sigma, prob.nev_b)
    t["interior_basis"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    kept = {}
    if lanczos is not None:
        Q, info = filter_lanczos(dd, zeta, omega, prob.Y0, streamed=streamed, **lanczos)
        t["lanczos_steps"] = info["steps"]
    else:
        Q, _ = filter_interface(dd, zeta, omega, prob.Y0, prob.steps, streamed=streamed,
                                keep=kept)
    t["filter"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    Sig, Gam = interior_levels(dd, prob.sigma, prob.psi, Q, V if deflate_levels else None)
    Z = build_z(dd, V, Sig, Gam, Q, prob.psi)
    t["interior"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    th, Xr, rank = rayleigh_ritz(dd, Z, prob.alpha, prob.beta)
    order = dd.order()
    X = np.zeros_like(Xr)
    X[order, :] = Xr                       # Alg. 5.1 step 8: permute back
    res = residuals(prob.A, prob.M, th, X) if want_vectors else np.zeros(0)
    t["rr"] = time.perf_counter() - t0
    return OracleResult(theta=th, X=X if want_vectors else np.zeros((0, 0)), resid=res,
                        mu=Q.shape[1], k=Z.shape[1], rank=rank, Q=Q, times=t,
                        W1=kept.get("W1"))
