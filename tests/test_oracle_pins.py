"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test compares the oracle with something that is not the oracle:
printed values (tests/golden), closed forms, exact identities of the paper
checked with an independent route (sparse LU of the whole pencil, a dense
eigendecomposition), brute force on tiny pencils, and the paper's bounds.
Together they are chosen so that a dropped term, a wrong sign, a wrong index
or a transposed operand anywhere in the oracle fails at least one of them.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import oracle as O
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _legendre(n, t):
    """P_n(t) and P_n'(t) by the three-term recurrence (independent of numpy)."""
    p0, p1 = np.ones_like(t), t.copy()
    if n == 0:
        return p0, np.zeros_like(t)
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * t * p1 - (k - 1) * p0) / k
    dp = n * (t * p1 - p0) / (t * t - 1.0)
    return p1, dp


# ---------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n_c", [1, 2, 3, 4, 8, 16])
def test_midpoint_filter_closed_form(n_c):
    """Midpoint rule: the 2 n_c nodes are the roots of z^{2 n_c} = -1 on the
    scaled circle, so the discrete sum is the partial-fraction expansion of
    1 / (1 + ((x - c)/r)^{2 n_c})."""
    a, b = -0.7, 2.3
    z, w = O.quadrature(a, b, n_c, "midpoint")
    c, r = 0.5 * (a + b), 0.5 * (b - a)
    x = np.linspace(-5, 7, 1001)
    ref = 1.0 / (1.0 + ((x - c) / r) ** (2 * n_c))
    assert np.max(np.abs(O.rho(x, z, w) - ref)) < 1e-13


def test_gauss_legendre_textbook_nodes():
    g = json.load(open(os.path.join(GOLD, "gauss_legendre_4.json")))
    a, b = 0.0, 2.0  # c = 1, r = 1: theta = pi/2 (1 + t)
    z, w = O.quadrature(a, b, 4, "gauss")
    theta = np.angle(z - 1.0)
    t = 2.0 * theta / np.pi - 1.0
    assert np.allclose(np.sort(t), g["nodes"], atol=1e-15, rtol=0)
    h = -4.0 * w / (z - 1.0)            # omega = -(h/4) r e^{i theta}
    assert np.allclose(h.imag, 0, atol=1e-15)
    assert np.allclose(h.real[np.argsort(t)], g["weights"], atol=1e-15, rtol=0)


@pytest.mark.parametrize("n_c", [1, 2, 5, 8, 13])
def test_gauss_legendre_nodes_are_legendre_roots(n_c):
    z, w = O.quadrature(0.0, 2.0, n_c, "gauss")
    t = 2.0 * np.angle(z - 1.0) / np.pi - 1.0
    P, dP = _legendre(n_c, t)
    assert np.max(np.abs(P)) < 1e-13
    h = (-4.0 * w / (z - 1.0)).real
    assert np.allclose(h, 2.0 / ((1 - t * t) * dP * dP), rtol=1e-12)


@pytest.mark.parametrize("rule", ["gauss", "midpoint"])
@pytest.mark.parametrize("n_c", [1, 2, 4, 8, 16])
def test_filter_center_and_endpoints(rule, n_c):
    """rho(c) = 1 and rho(alpha) = rho(beta) = 1/2 (Fig. 2.1 scaling), poles in
    the upper half plane on the circle, and rho decays outside the interval."""
    a, b = 0.3, 1.1
    z, w = O.quadrature(a, b, n_c, rule)
    assert np.all(z.imag > 0)
    assert np.allclose(np.abs(z - 0.7), 0.4, atol=1e-15)
    v = O.rho(np.array([0.7, a, b]), z, w)
    assert np.allclose(v, [1.0, 0.5, 0.5], atol=4e-15)
    if n_c >= 4:
        assert abs(O.rho(np.array([3.0]), z, w)[0]) < 1e-2


def test_quadrature_rejects_bad_input():
    with pytest.raises(ValueError):
        O.quadrature(1.0, 1.0, 4)
    with pytest.raises(ValueError):
        O.quadrature(0.0, 1.0, 0)


# ---------------------------------------------------------------- generators
def test_grid_eigenvalues_against_paper_tables():
    g = json.load(open(os.path.join(GOLD, "paper_grid_eigs.json")))
    for case in g["cases"]:
        grid = tuple(case["grid"])
        lam = W.closed_form_eigs(grid)
        assert lam.size == case["n"]
        if grid[0] * grid[1] <= 250000:
            A = W.laplacian(grid)
            assert round(A.nnz / A.shape[0], 2) == case["nnz_per_row"]
        if "beta" in case:
            assert abs(lam[99] - case["beta"]) < 5e-5
        for k, v in case.get("lambda", {}).items():
            ndig = len(f"{v:.2e}".split("e")[0].replace(".", "").rstrip("0"))
            tol = 10.0 ** (np.floor(np.log10(v)) - ndig + 1)
            assert abs(lam[int(k) - 1] - v) <= tol, (case["name"], k, lam[int(k) - 1], v)


def test_closed_form_matches_dense_eigh():
    A = W.laplacian((9, 7))
    lam = np.linalg.eigvalsh(A.toarray())
    assert np.max(np.abs(lam - W.closed_form_eigs((9, 7)))) < 1e-13
    A3 = W.laplacian((5, 4, 3))
    assert np.max(np.abs(np.linalg.eigvalsh(A3.toarray()) - W.closed_form_eigs((5, 4, 3)))) < 1e-13


def test_config_shapes():
    p = W.config(1)
    dd = O.DD(p.A, p.M, p.part)
    assert (dd.p, dd.s, dd.n) == (4, 61, 961)
    assert [len(i) for i in dd.interior] == [225] * 4
    assert [len(a) for a in dd.adj] == [30] * 4
    assert abs(p.beta - 0.313379) < 1e-6


# ---------------------------------------------------------------- Schur complement
def _pencils():
    return [W.tiny(N=9, P=2, nev=4, mass_kind="identity"),
            W.tiny(N=9, P=3, nev=5, mass_kind="random", cfg_id=7),
            W.tiny(N=9, P=2, nev=4, mass_kind="coupled", cfg_id=8),
            W.tiny(N=5, dim=3, P=2, nev=4, mass_kind="coupled", cfg_id=9),
            W.tiny(N=10, P=2, nev=5, mass_kind="random", kfield=True, cfg_id=10)]


@pytest.mark.parametrize("k", range(5))
def test_schur_inverse_is_interface_block_of_full_inverse(k):
    """S(z)^{-1} y = [(A - zM)^{-1} (0; y)] on the interface (Sec. 3.1,
    block inverse), with the full pencil solved by sparse LU in the original
    numbering.  With a coupled M (M_E != 0) this also fixes the transpose
    reading: A - zM is complex symmetric."""
    prob = _pencils()[k]
    dd = O.DD(prob.A, prob.M, prob.part)
    rs = np.random.default_rng(5)
    for z in [0.3 + 0.2j, 1.7 + 0.01j, -0.5 + 2.0j]:
        S = O.schur(dd, z)
        y = rs.standard_normal(dd.s) + 1j * rs.standard_normal(dd.s)
        rhs = np.zeros(dd.n, dtype=complex)
        rhs[dd.iface] = y
        full = sla.spsolve((prob.A - z * prob.M).tocsc().astype(complex), rhs)
        x = np.linalg.solve(S, y)
        assert np.max(np.abs(x - full[dd.iface])) < 1e-12 * np.max(np.abs(full))
        assert np.allclose(S, S.T, atol=1e-12)      # complex symmetric


def test_dd_rejects_direct_coupling():
    A = W.laplacian((6, 6))
    part = np.zeros(36, dtype=np.int32)
    part[18:] = 1                                    # no separator between them
    with pytest.raises(ValueError):
        O.DD(A, sp.identity(36, format="csr"), part)


# ---------------------------------------------------------------- filter identity
@pytest.mark.parametrize("k", range(5))
@pytest.mark.parametrize("rule", ["gauss", "midpoint"])
def test_filter_identity_eq_3_5(k, rule):
    """2 Re sum omega_l S(zeta_l)^{-1} = sum_i rho(lambda_i) y_i y_i^T, eq. (3.5),
    with (lambda_i, x_i) from a dense generalized eigendecomposition
    (M-orthonormal x_i), y_i = interface part of x_i.  Exact for the discrete
    rule."""
    prob = _pencils()[k]
    dd = O.DD(prob.A, prob.M, prob.part)
    lam, X = sl.eigh(prob.A.toarray(), prob.M.toarray())
    z, w = O.quadrature(prob.alpha, prob.beta, 4, rule)
    F = O.filter_apply(O.factor_poles(dd, z), w, np.eye(dd.s))
    Y = X[dd.iface, :]
    ref = (Y * O.rho(lam, z, w)[None, :]) @ Y.T
    assert np.max(np.abs(F - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_prop_3_1_rank():
    """rank[y_1..y_nev] <= rank F <= s (Prop. 3.1)."""
    prob = W.config(1)
    dd = O.DD(prob.A, prob.M, prob.part)
    z, w = O.quadrature(prob.alpha, prob.beta, 8, "gauss")
    F = O.filter_apply(O.factor_poles(dd, z), w, np.eye(dd.s))
    lam, X = sl.eigh(prob.A.toarray())
    Yw = X[dd.iface][:, :prob.nev]
    r_y = np.linalg.matrix_rank(Yw, tol=1e-10)
    sv = np.linalg.svd(F, compute_uv=False)
    r_f = int(np.count_nonzero(sv > 1e-12 * sv[0]))
    assert r_y <= r_f <= dd.s
    assert r_y < prob.nev                  # C1: 20 wanted, rank well below 20


# ---------------------------------------------------------------- orthonormalisation
def test_orth_rank_and_span():
    rs = np.random.default_rng(3)
    B = rs.standard_normal((200, 7))
    W_ = np.hstack([B, B[:, :3] @ rs.standard_normal((3, 4)), 1e-9 * rs.standard_normal((200, 2))])
    Q = O.orth(W_)
    assert Q.shape[1] == 9                 # 7 + 2 small but independent
    assert np.max(np.abs(Q.T @ Q - np.eye(9))) < 1e-14
    P = W_ - Q @ (Q.T @ W_)
    assert np.max(np.abs(P)) < 1e-13 * np.max(np.abs(W_))
    K = Q[:, :4]
    Q2 = O.orth(W_, K)
    assert Q2.shape[1] == 5
    assert np.max(np.abs(K.T @ Q2)) < 1e-14
    assert O.orth(np.zeros((5, 3))).shape == (5, 0)


def test_filter_interface_saturates_at_s():
    prob = W.config(1)
    dd = O.DD(prob.A, prob.M, prob.part)
    z, w = O.quadrature(prob.alpha, prob.beta, prob.n_c, prob.rule)
    Q, _ = O.filter_interface(dd, z, w, prob.Y0, 4)   # 4 * 30 > s = 61
    assert Q.shape[1] <= dd.s
    assert np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1]))) < 1e-13


# ---------------------------------------------------------------- interior bounds
def _coupled():
    return W.tiny(N=11, P=2, nev=6, mass_kind="coupled", cfg_id=21)


def test_lemma_4_1_identity():
    """u - uhat = -[B_lam^{-1} - B_sig^{-1}] E_sig y + (lam - sig) B_lam^{-1} M_E y
    for an exact eigenpair, with uhat = -B_sig^{-1} E_sig y (eq. (4.1)) taken
    from the oracle's first resolvent level."""
    prob = _coupled()
    dd = O.DD(prob.A, prob.M, prob.part)
    order = dd.order()
    Ar, Mr = prob.A[order][:, order].toarray(), prob.M[order][:, order].toarray()
    lam, X = sl.eigh(Ar, Mr)
    d = sum(b.shape[0] for b in dd.B)
    Bfull = Ar[:d, :d]; MB = Mr[:d, :d]; E = Ar[:d, d:]; ME = Mr[:d, d:]
    sig = 0.13
    done = 0
    for i in range(6):
        u, y = X[:d, i], X[d:, i]
        if np.linalg.norm(y) < 1e-6:
            continue          # purely interior mode: B_lambda is singular there
        done += 1
        Sig, _ = O.interior_levels(dd, sig, 1, y.reshape(-1, 1))
        uhat = -np.concatenate([s[:, 0] for s in Sig])
        Bl = Bfull - lam[i] * MB
        Bs = Bfull - sig * MB
        Es = E - sig * ME
        rhs = -(np.linalg.solve(Bl, Es @ y) - np.linalg.solve(Bs, Es @ y)) \
            + (lam[i] - sig) * np.linalg.solve(Bl, ME @ y)
        assert np.max(np.abs((u - uhat) - rhs)) < 1e-11 * np.max(np.abs(u))
    assert done >= 3


def _mb_norm(v, MB):
    return float(np.sqrt(v @ (MB @ v)))


@pytest.mark.parametrize("psi,nev_b", [(1, 0), (2, 0), (3, 0), (2, 6), (3, 10)])
def test_theorems_4_2_to_4_4_bounds(psi, nev_b):
    """||u - uhat||_{M_B} <= the bound of Thm 4.2 (psi = 1), Thm 4.3 (psi > 1)
    and Thm 4.4 (with kappa deflated eigenvectors), uhat the M_B-orthogonal
    projection of u onto span{levels, V}."""
    prob = _coupled()
    dd = O.DD(prob.A, prob.M, prob.part)
    order = dd.order()
    Ar, Mr = prob.A[order][:, order].toarray(), prob.M[order][:, order].toarray()
    lam, X = sl.eigh(Ar, Mr)
    d = sum(b.shape[0] for b in dd.B)
    Bfull, MB, E, ME = Ar[:d, :d], Mr[:d, :d], Ar[:d, d:], Mr[:d, d:]
    delta, Vb = sl.eigh(Bfull, MB)
    sig = 0.5 * (lam[0] + lam[5])
    V, _ = O.interior_basis(dd, sig, nev_b)
    MBinv = np.linalg.inv(MB)
    for i in range(6):
        u, y = X[:d, i], X[d:, i]
        if np.linalg.norm(y) < 1e-6:
            continue          # purely interior mode: the bounds divide by zero
        Sig, Gam = O.interior_levels(dd, sig, psi, y.reshape(-1, 1))
        cols = [np.concatenate(S_) for S_ in zip(*[[S[:, c] for c in range(S.shape[1])] for S in Sig])]
        U = np.array(cols).T
        Gcols = [np.concatenate(G_) for G_ in zip(*[[G[:, c] for c in range(G.shape[1])] for G in Gam])]
        U = np.hstack([U, np.array(Gcols).T])
        if nev_b:
            Vd = sl.block_diag(*V)
            U = np.hstack([U, Vd])
        # M_B-orthogonal projection of u onto span(U)
        Gm = U.T @ MB @ U
        coef = np.linalg.lstsq(Gm, U.T @ MB @ u, rcond=1e-14)[0]
        err = _mb_norm(u - U @ coef, MB)
        Es_y = (E - sig * ME) @ y
        ME_y = ME @ y
        nE = float(np.sqrt(Es_y @ MBinv @ Es_y))
        nM = float(np.sqrt(ME_y @ MBinv @ ME_y))
        if nev_b:
            # the kappa eigenvalues of (B, M_B) closest to sigma (all blocks together)
            kap = sum(v.shape[1] for v in V)
            far = np.argsort(np.abs(delta - sig))[kap:]
        else:
            far = np.arange(delta.size)
        dl = delta[far]
        L = abs(lam[i] - sig)
        bound = np.max(L ** psi / np.abs((lam[i] - dl) * (sig - dl) ** psi)) * nE \
            + np.max(L ** (psi + 1) / np.abs((lam[i] - dl) * (sig - dl) ** psi)) * nM
        assert err <= bound * (1 + 1e-8) + 1e-13, (i, err, bound)


# ---------------------------------------------------------------- inertia
def test_inertia_count_matches_closed_form_and_haynsworth():
    p = W.config(1)
    assert O.inertia_count(p.A, p.M, p.alpha, p.beta) == 20
    dd = O.DD(p.A, p.M, p.part)
    assert O.inertia_count(p.A, p.M, p.alpha, p.beta, dd) == 20
    for prob in _pencils()[1:3]:
        lam = sl.eigh(prob.A.toarray(), prob.M.toarray(), eigvals_only=True)
        a, b = 0.2, 1.3
        exact = int(np.count_nonzero((lam >= a) & (lam <= b)))
        dd = O.DD(prob.A, prob.M, prob.part)
        assert O.inertia_count(prob.A, prob.M, a, b) == exact
        assert O.inertia_count(prob.A, prob.M, a, b, dd) == exact


# ---------------------------------------------------------------- end to end
def test_end_to_end_exact_interface_closed_form():
    """m = s: the filtered block spans the whole interface, so only the
    interior approximation remains; with psi = 6 and nev_b = 60 the Ritz
    values reach the closed form to ~1e-12."""
    prob = W.tiny(N=15, P=2, nev=11, n_c=4, steps=1, nev_b=60, psi=6)
    r = O.run(prob)
    ex = W.closed_form_eigs((15, 15))[:11]
    assert r.theta.size == 11
    assert np.max(np.abs(r.theta - ex) / ex) < 1e-11
    assert r.resid.max() < 1e-9


def test_end_to_end_random_mass_dense_reference():
    prob = W.tiny(N=13, P=2, nev=8, n_c=8, steps=1, nev_b=40, psi=6, mass_kind="random", cfg_id=31)
    r = O.run(prob)
    lam = sl.eigh(prob.A.toarray(), prob.M.toarray(), eigvals_only=True)
    ex = lam[(lam >= prob.alpha) & (lam <= prob.beta)]
    assert r.theta.size == ex.size == 8
    assert np.max(np.abs(r.theta - ex) / ex) < 1e-11


def test_end_to_end_coupled_mass_uses_gamma_blocks():
    prob = W.tiny(N=11, P=2, nev=6, n_c=8, steps=1, nev_b=30, psi=5, mass_kind="coupled", cfg_id=32)
    r = O.run(prob)
    lam = sl.eigh(prob.A.toarray(), prob.M.toarray(), eigvals_only=True)
    ex = lam[(lam >= prob.alpha) & (lam <= prob.beta)]
    assert r.theta.size == ex.size
    assert np.max(np.abs(r.theta - ex) / np.abs(ex)) < 1e-10
    dd = O.DD(prob.A, prob.M, prob.part)
    assert not dd.m_e_zero
    assert r.k == sum(min(30, b.shape[0]) for b in dd.B) + 2 * 5 * r.mu


def test_config1_end_to_end():
    """Config 1 at its stated parameters: all 20 eigenvalues, accurate to the
    method's floor at 2 block steps (~1e-10), inertia count 20."""
    p = W.config(1)
    r = O.run(p)
    ex = p.exact[:20]
    assert r.theta.size == 20
    assert np.max(np.abs(r.theta - ex) / ex) < 1e-9
    assert r.resid.max() < 1e-5
    assert r.mu == 60


def test_deflated_levels_keep_the_span():
    """The deflated resolvent recurrence spans the same Z as eq. (5.5)."""
    prob = W.tiny(N=11, P=2, nev=6, n_c=4, steps=1, nev_b=6, psi=3, mass_kind="random", cfg_id=33)
    dd = O.DD(prob.A, prob.M, prob.part)
    z, w = O.quadrature(prob.alpha, prob.beta, prob.n_c, prob.rule)
    Q, _ = O.filter_interface(dd, z, w, prob.Y0, 1)
    V, _ = O.interior_basis(dd, prob.sigma, prob.nev_b)
    Z1 = O.build_z(dd, V, *O.interior_levels(dd, prob.sigma, 3, Q, None), Q, 3)
    Z2 = O.build_z(dd, V, *O.interior_levels(dd, prob.sigma, 3, Q, V), Q, 3)
    def basis(Z):
        U, sv, _ = np.linalg.svd(Z / np.linalg.norm(Z, axis=0), full_matrices=False)
        r = int(np.count_nonzero(sv > 1e-10 * sv[0]))
        return U[:, :r], sv[r - 1] / sv[0]
    b1, c1 = basis(Z1)
    b2, c2 = basis(Z2)
    assert b1.shape == b2.shape
    sv = np.linalg.svd(b1.T @ b2, compute_uv=False)
    assert np.min(sv) > 1 - 1e-8
    assert c2 > 100 * c1          # the deflated basis is far better conditioned


# ---------------------------------------------------------------- residual and ||A||
def _norm_a_pin_errors(norm_a):
    """Deviations of a candidate ||A|| routine from closed-form largest
    absolute row sums: 8 for the 2D five-point stencil (4 + 4 x |-1|), 12
    for the 3D seven-point stencil, 7 for a hand-written 3 x 3 matrix."""
    hand = sp.csr_matrix(np.array([[2.0, -1.0, 0.0], [-1.0, 3.0, -2.0], [0.0, -2.0, 5.0]]))
    cases = [(W.laplacian((9, 9)), 8.0), (W.laplacian((6, 6, 6)), 12.0), (hand, 7.0)]
    return [abs(norm_a(A) - v) / v for A, v in cases]


def test_norm_a_closed_form_row_sums():
    assert max(_norm_a_pin_errors(O.norm_a)) < 1e-15
    # an upper bound of ||A||_2, which equals 8 sin^2(pi N / (2 (N + 1))) in 2D
    A = W.laplacian((9, 9))
    assert O.norm_a(A) >= 8.0 * np.sin(np.pi * 9 / 20.0) ** 2
    # a planted mistake (twice the norm, or the largest entry instead of the row sum) fails
    assert max(_norm_a_pin_errors(lambda A: 2.0 * O.norm_a(A))) > 0.5
    assert max(_norm_a_pin_errors(lambda A: float(abs(A).max()))) > 0.1


def _residual_pin_errors(residuals):
    """Exact eigenpairs (lam_i, x_i) of a random-diagonal-M pencil from a
    dense generalized eigensolver, perturbed to theta_i = lam_i (1 + delta_i):
    then A x_i - theta_i M x_i = -lam_i delta_i M x_i, whose 2-norm is known.
    With ||A|| = 8 (closed form of the 2D stencil) the relative residual is
    |lam_i delta_i| ||M x_i||_2 / (8 ||x_i||_2).  The columns carry arbitrary
    scales (the residual is scale-free).  Returns the largest deviation
    relative to the expected values (absolute where they vanish)."""
    prob = W.tiny(N=7, P=2, nev=4, mass_kind="random", cfg_id=61)
    mdiag = prob.M.diagonal()
    lam, X = sl.eigh(prob.A.toarray(), prob.M.toarray())
    pick = np.array([0, 3, 10, 25, 48])
    delta = np.array([0.0, 1e-3, -2e-2, 0.5, -1e-6])
    scale = np.array([1.0, 3.0, 0.25, -7.0, 1e3])
    Xs = X[:, pick] * scale[None, :]
    theta = lam[pick] * (1.0 + delta)
    mx = np.sqrt(np.sum((mdiag[:, None] * Xs) ** 2, axis=0))
    expect = np.abs(lam[pick] * delta) * mx / (8.0 * np.sqrt(np.sum(Xs ** 2, axis=0)))
    got = residuals(prob.A, prob.M, theta, Xs)
    err = np.abs(got - expect) / np.maximum(expect, 1e-300)
    err[delta == 0] = got[delta == 0]          # exact pair: rounding level only
    return err


def test_residuals_known_values():
    err = _residual_pin_errors(O.residuals)
    assert np.max(err[[1, 2, 3, 4]]) < 1e-8 and err[0] < 1e-14, err
    assert O.residuals(W.laplacian((3, 3)), sp.identity(9), np.zeros(0), np.zeros((9, 0))).size == 0
    # planted mistakes fail: M dropped from theta M x, ||A|| doubled, zeros returned
    drop_m = lambda A, M, th, X: O.residuals(A, sp.identity(A.shape[0], format="csr"), th, X)
    assert np.max(_residual_pin_errors(drop_m)[1:]) > 1e-2
    assert np.max(_residual_pin_errors(lambda A, M, th, X: 0.5 * O.residuals(A, M, th, X))[1:]) > 0.4
    assert np.max(_residual_pin_errors(lambda A, M, th, X: np.zeros(th.size))[1:]) > 0.9


# ---------------------------------------------------------------- pole-streamed path
@pytest.mark.parametrize("k", [1, 2, 3])
def test_streamed_filter_equals_the_stored_factor_path(k):
    """filter_apply_streamed (one pole's S(zeta) at a time, sparse C and M_C)
    computes the same eq. (3.5) as filter_apply over stored factors."""
    prob = _pencils()[k]
    z, w = O.quadrature(prob.alpha, prob.beta, 5, "gauss")
    dd = O.DD(prob.A, prob.M, prob.part)
    dds = O.DD(prob.A, prob.M, prob.part, dense_interface=False)
    Wa = O.filter_apply(O.factor_poles(dd, z), w, prob.Y0)
    Wb = O.filter_apply_streamed(dds, z, w, prob.Y0)
    assert np.max(np.abs(Wa - Wb)) <= 1e-14 * np.max(np.abs(Wa))


def test_streamed_run_equals_the_default_run():
    prob = W.tiny(N=13, P=3, nev=6, n_c=6, steps=2, nev_b=6, psi=3, mass_kind="random", cfg_id=62)
    a = O.run(prob)
    b = O.run(prob, streamed=True)
    assert a.theta.size == b.theta.size == 6
    assert np.max(np.abs(a.theta - b.theta) / a.theta) <= 1e-13
    assert np.max(np.abs(a.W1 - b.W1)) <= 1e-14 * np.max(np.abs(a.W1))


# ---------------------------------------------------------------- Alg. 3.1 (Lanczos)
def _lanczos_case(m=3, n_c=6, tol=0.0, max_steps=6, cfg=63):
    prob = W.tiny(N=13, P=3, nev=6, n_c=n_c, m=m, steps=1, nev_b=6, psi=3,
                  mass_kind="random", cfg_id=cfg)
    dd = O.DD(prob.A, prob.M, prob.part)
    z, w = O.quadrature(prob.alpha, prob.beta, prob.n_c, prob.rule)
    fac = O.factor_poles(dd, z)
    Q, info = O.filter_lanczos(dd, z, w, prob.Y0, tol=tol, max_steps=max_steps, factors=fac)
    return prob, dd, z, w, fac, Q, info


def test_lanczos_recurrence_is_the_projection_of_the_filter():
    """With full reorthogonalisation the block tridiagonal T_t built from the
    recurrence's A_t, B_t equals Q^T F Q for the filter of eq. (3.5) applied
    independently to the whole basis, including the zeros outside the band
    (the three-term structure of Lanczos)."""
    prob, dd, z, w, fac, Q, info = _lanczos_case()
    assert info["steps"] == 6 and Q.shape[1] == 18
    assert np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1]))) < 1e-13
    P = Q.T @ O.filter_apply(fac, w, Q)
    T = O.block_tridiagonal(info)
    assert np.max(np.abs(T - P)) <= 1e-12 * np.max(np.abs(P))
    # the sum of the eigenvalues of T_t is the traced quantity of the stopping test
    assert abs(np.sum(np.linalg.eigvalsh(T)) - info["traces"][-1]) <= 1e-12 * abs(info["traces"][-1])
    # a recurrence without the reorthogonalisation against older blocks would
    # leave T != Q^T F Q: a planted mistake (A and B swapped) fails
    bad = dict(info, A=[info["A"][0]] + info["B"][:5], B=info["A"][1:])
    assert np.max(np.abs(O.block_tridiagonal(bad) - P)) > 1e-3 * np.max(np.abs(P))


def test_lanczos_starts_from_the_start_block():
    prob, dd, z, w, fac, Q, info = _lanczos_case(max_steps=2)
    # Q_1 spans Y0 (line 0 of Alg. 3.1 normalises the start vector)
    Y = prob.Y0
    assert np.max(np.abs(Y - Q[:, :3] @ (Q[:, :3].T @ Y))) < 1e-13 * np.max(np.abs(Y))
    assert np.allclose(info["A"][0], Q[:, :3].T @ O.filter_apply(fac, w, Q[:, :3]), atol=1e-14)


def test_lanczos_terminates_early_and_captures_the_wanted_subspace():
    """Prop. 3.1 / Sec. 3.2: the trace of T_t stops growing once the range of
    F is captured, before the interface is exhausted; the resulting Q gives
    the eigenvalues of the pencil after the interior part and Rayleigh-Ritz."""
    prob = W.tiny(N=21, P=2, nev=8, n_c=8, m=4, steps=1, nev_b=30, psi=6, mass_kind="random",
                  cfg_id=64)
    dd = O.DD(prob.A, prob.M, prob.part)
    z, w = O.quadrature(prob.alpha, prob.beta, prob.n_c, prob.rule)
    Q, info = O.filter_lanczos(dd, z, w, prob.Y0, tol=1e-6, max_steps=200)
    assert info["converged"]
    assert Q.shape[1] < dd.s
    # successive traces settle: the last relative change is within the tolerance
    tr = info["traces"]
    assert abs(tr[-1] - tr[-4]) <= 1e-6 * abs(tr[-1])    # tested every 10 vectors = 3 blocks of 4
    r = O.run(prob, lanczos=dict(tol=1e-6, max_steps=200))
    lam = sl.eigh(prob.A.toarray(), prob.M.toarray(), eigvals_only=True)
    ex = lam[(lam >= prob.alpha) & (lam <= prob.beta)]
    assert r.theta.size == ex.size == 8
    assert np.max(np.abs(r.theta - ex) / ex) < 1e-9
    assert r.mu == Q.shape[1]
