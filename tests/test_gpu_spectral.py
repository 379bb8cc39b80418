"""The spectral interior path (rfd_set_interior_solver(RFD_INTERIOR_SPECTRAL):
one eigendecomposition of every (B_j, M_Bj) per pencil, (B_j - z M_Bj)^{-1} =
V_j (Lambda_j - z I)^{-1} V_j^T for every pole and sigma, Sec. 4.1) on the GPU
through the C ABI, against the oracle, which factors every shifted block.

Same seeded inputs on both sides; the checks:
  * the subdomain eigenvector blocks are orthonormal after the decomposition
    (|U^T U - I| <= 1e-14);
  * the filtered block F Y0 (eq. (3.5)) element by element (relative 1e-12 in
    FP64, 1e-11 with FP32 factors of S refined in FP64);
  * the Ritz values of whole solves (relative 1e-10) and their residuals
    (<= 10x the oracle's), both precision modes, dense and two-level S, 2D
    and 3D, uneven subdomains;
  * one decomposition serving several intervals and sigmas on one pencil
    gives each solve the results of a fresh LU-path pencil (relative 1e-12);
  * inertia counts and spectrum slices in the spectral mode;
  * the documented errors.
Cases include a non-diagonal M that couples the interiors to the interface
(dense and two-level S).
"""
import dataclasses

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
EIG_TOL = 1e-10


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


CASES = {
    # uneven subdomains (13 = 4 + 1 + 3 + 1 + 4): padding inside the eigensolver
    "p9_uneven": (lambda: W.tiny(N=13, P=3, nev=6, n_c=6, steps=2, nev_b=6, psi=3,
                                 mass_kind="random", cfg_id=61), False),
    "mid_7tiles": (lambda: W.tiny(N=41, P=2, nev=10, n_c=8, m=40, steps=2, nev_b=12, psi=4,
                                  mass_kind="random", cfg_id=62), False),
    "quad41_two_level": (lambda: W.tiny(N=41, P=4, nev=18, n_c=8, m=40, steps=2, nev_b=12,
                                        psi=5, mass_kind="random", cfg_id=63), True),
    "tiny3d_p8": (lambda: W.tiny(N=11, dim=3, P=2, nev=8, n_c=6, m=40, steps=2, nev_b=10,
                                 psi=4, mass_kind="random", cfg_id=64), False),
    "kfield_identity": (lambda: W.tiny(N=14, P=2, nev=5, n_c=4, m=12, steps=2, nev_b=8, psi=4,
                                       kfield=True, cfg_id=65), False),
    # non-diagonal M coupling the interiors to the interface (standard form of
    # (B_j, M_Bj), V^T Ehat_zeta = V^T Ehat - zeta V^T Mhat_E, Gamma levels)
    "coupled_p9": (lambda: W.tiny(N=27, P=3, nev=6, n_c=4, m=16, steps=1, nev_b=6, psi=2,
                                  mass_kind="coupled", cfg_id=49), False),
    "coupled_two_level": (lambda: W.tiny(N=41, P=4, nev=17, n_c=8, m=40, steps=2, nev_b=12,
                                         psi=5, mass_kind="coupled", cfg_id=51), True),
}
_cache = {}


def _case(name):
    if name not in _cache:
        make, groups = CASES[name]
        prob = make()
        dd = O.DD(prob.A, prob.M, prob.part)
        z, w = O.quadrature(prob.alpha, prob.beta, prob.n_c, prob.rule)
        W1 = O.filter_apply(O.factor_poles(dd, z), w, prob.Y0)
        _cache[name] = (prob, groups, W1, O.run(prob))
    return _cache[name]


def _pencil(prob, groups, mode, spectral=True):
    import paper_1711_09487_amd as R
    P = R.Pencil(prob.A, prob.M)
    P.set_partition(prob.part)
    if groups:
        P.set_interface_groups(W.interface_groups(prob.grid, prob.meta["P"]))
    if spectral:
        P.set_interior_solver(R.RFD_INTERIOR_SPECTRAL)
    P.set_interval_and_poles(prob.alpha, prob.beta, prob.n_c,
                             R.RFD_RULE_GAUSS if prob.rule == "gauss" else R.RFD_RULE_MIDPOINT)
    P.set_precision(mode)
    return P


def _dev(torch, Y):
    return torch.from_numpy(np.ascontiguousarray(Y.T)).cuda()


def _solve(torch, P, prob, Y0=None):
    Y0 = _dev(torch, prob.Y0) if Y0 is None else Y0
    P.filter_interface(Y0, prob.steps)
    P.solve_interior(prob.sigma, prob.nev_b, prob.psi)
    ev, _, res = P.rayleigh_ritz(prob.nev + 20, vectors=False)
    torch.cuda.synchronize()
    return ev.cpu().numpy(), res.cpu().numpy()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_spectral_path_matches_the_oracle(name, mode):
    torch = _torch()
    prob, groups, W1, ro = _case(name)
    P = _pencil(prob, groups, mode)
    try:
        Wg = P.filter_apply(_dev(torch, prob.Y0)).cpu().numpy().T
        orth = P.spectral_orthogonality()
        th, r = _solve(torch, P, prob)
    finally:
        P.close()
    assert 0.0 < orth <= 1e-14 or orth == 0.0
    err = np.max(np.abs(Wg - W1)) / np.max(np.abs(W1))
    assert err < (1e-12 if mode == 0 else 1e-11), err
    assert th.size == ro.theta.size
    assert np.max(np.abs(th - ro.theta) / np.abs(ro.theta)) <= EIG_TOL
    assert np.all(r <= 10 * ro.resid + 1e-12)


def test_one_decomposition_serves_many_intervals():
    """Three intervals and sigmas on one spectral pencil (the decomposition is
    made once) against a fresh LU-path pencil for each."""
    torch = _torch()
    import paper_1711_09487_amd as R
    prob, groups, _, _ = _case("mid_7tiles")
    lam = sl.eigh(prob.A.toarray(), prob.M.toarray(), eigvals_only=True)
    subs = []
    for lo, hi in [(0, 10), (4, 14), (10, 22)]:
        a = 0.0 if lo == 0 else 0.5 * (lam[lo - 1] + lam[lo])
        b = 0.5 * (lam[hi - 1] + lam[hi])
        subs.append(dataclasses.replace(prob, alpha=float(a), beta=float(b),
                                        sigma=0.5 * (a + b), nev=hi - lo))
    P = _pencil(prob, groups, 0)
    Y0 = _dev(torch, prob.Y0)
    try:
        got = []
        for q in subs:
            P.set_interval_and_poles(q.alpha, q.beta, q.n_c, R.RFD_RULE_GAUSS)
            got.append(_solve(torch, P, q, Y0))
            orth = P.spectral_orthogonality()
    finally:
        P.close()
    assert orth <= 1e-14
    for q, (th, r) in zip(subs, got):
        L = _pencil(q, groups, 0, spectral=False)
        try:
            th2, r2 = _solve(torch, L, q)
        finally:
            L.close()
        assert th.size == th2.size == q.nev
        assert np.max(np.abs(th - th2) / np.abs(th2)) <= 1e-12
        ex = lam[(lam >= q.alpha) & (lam <= q.beta)]
        assert np.max(np.abs(th - ex) / ex) <= EIG_TOL


@pytest.mark.parametrize("groups", [False, True])
def test_spectral_inertia_and_slices(groups):
    torch = _torch()
    import paper_1711_09487_amd as R
    prob = W.tiny(N=41, P=4, nev=18, n_c=8, m=40, steps=2, nev_b=12, psi=5,
                  mass_kind="random", cfg_id=81)
    lam = sl.eigh(prob.A.toarray(), prob.M.toarray(), eigvals_only=True)
    P = _pencil(prob, groups, 0)
    try:
        for a, b in [(prob.alpha, prob.beta), (0.5 * (lam[2] + lam[3]), 0.5 * (lam[9] + lam[10]))]:
            assert P.inertia_count(a, b) == int(np.count_nonzero((lam >= a) & (lam <= b)))
        inside = lam[(lam >= prob.alpha) & (lam <= prob.beta)]
        mids = [0.5 * (inside[i - 1] + inside[i]) for i in (6, 12)]
        cuts = np.array([prob.alpha] + mids + [prob.beta])
        ev, _, _, counts, inert = P.solve_slices(cuts, prob.n_c, _dev(torch, prob.Y0), prob.steps,
                                                 prob.nev_b, prob.psi, prob.nev + 20)
        torch.cuda.synchronize()
        th = ev.cpu().numpy()
    finally:
        P.close()
    assert inert == th.size == prob.nev
    off = 0
    for i in range(cuts.size - 1):
        sub = dataclasses.replace(prob, alpha=float(cuts[i]), beta=float(cuts[i + 1]),
                                  sigma=0.5 * (cuts[i] + cuts[i + 1]))
        ro = O.run(sub, want_vectors=False)
        assert counts[i] == ro.theta.size
        assert np.max(np.abs(th[off:off + counts[i]] - ro.theta) / np.abs(ro.theta)) <= EIG_TOL
        off += counts[i]


def test_interior_solver_errors():
    _torch()
    import paper_1711_09487_amd as R
    prob = W.tiny(N=11, P=2, nev=6, n_c=4, steps=2, nev_b=8, psi=3)
    P = R.Pencil(prob.A, prob.M)
    try:
        P.set_partition(prob.part)
        with pytest.raises(R.RfdError) as e:
            P.set_interior_solver(2)
        assert e.value.code == 1
    finally:
        P.close()
    # a block of M that is not positive definite: RFD_EBREAKDOWN from the
    # decomposition (two interior nodes coupled by 2 against unit diagonals)
    import scipy.sparse as sp
    cm = W.tiny(N=13, P=2, nev=6, n_c=4, m=8, steps=1, nev_b=4, psi=2, mass_kind="coupled",
                cfg_id=54)
    Mi = sp.lil_matrix(cm.M)
    i, k = (int(x) for x in np.flatnonzero(cm.part == 0)[[3, 17]])
    Mi[i, k] = Mi[k, i] = 2.0
    torch = _torch()
    P = R.Pencil(cm.A, sp.csr_matrix(Mi))
    try:
        P.set_partition(cm.part)
        P.set_interior_solver(R.RFD_INTERIOR_SPECTRAL)
        P.set_interval_and_poles(cm.alpha, cm.beta, cm.n_c, R.RFD_RULE_GAUSS)
        with pytest.raises(R.RfdError) as e:
            P.filter_interface(_dev(torch, cm.Y0), cm.steps)
        assert e.value.code == 3 and "positive definite" in str(e.value)
    finally:
        P.close()
