"""Spectrum slicing (Sec. 7) and the inertia count on the GPU, through the
C ABI, against the oracle.

  * rfd_inertia_count equals the oracle's Sylvester count (dense LDL^T of
    A - tau M) and the exact count from a dense eigensolve, with the dense and
    the two-level S(zeta);
  * rfd_solve_slices: every slice's Ritz values equal the oracle's whole
    solve on that slice (same poles, Y0, sigma, nev_b, psi, steps), relative
    1e-10, for a per-slice sigma and for one sigma shared by all slices; the
    merged count equals the inertia count and the exact count.
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


def _prob(kind):
    if kind == "quad41":
        return W.tiny(N=41, P=4, nev=18, n_c=8, m=40, steps=2, nev_b=12, psi=5,
                      mass_kind="random", cfg_id=81)
    return W.tiny(N=13, P=3, nev=12, n_c=8, m=30, steps=2, nev_b=10, psi=5, mass_kind="random",
                  cfg_id=82)


def _pencil(prob, groups):
    import paper_1711_09487_amd as R
    P = R.Pencil(prob.A, prob.M)
    P.set_partition(prob.part)
    if groups:
        P.set_interface_groups(W.interface_groups(prob.grid, prob.meta["P"]))
    P.set_interval_and_poles(prob.alpha, prob.beta, prob.n_c, R.RFD_RULE_GAUSS)
    return P


def _cuts(prob, lam, parts=3):
    """Cuts at midpoints of gaps: [alpha, ..., beta] with roughly equal counts."""
    inside = lam[(lam >= prob.alpha) & (lam <= prob.beta)]
    idx = [int(round(i * inside.size / parts)) for i in range(1, parts)]
    mids = [0.5 * (inside[i - 1] + inside[i]) for i in idx]
    return np.array([prob.alpha] + mids + [prob.beta])


@pytest.mark.parametrize("kind,groups", [("p9", False), ("quad41", False), ("quad41", True)])
def test_inertia_count_matches_the_oracle(kind, groups):
    _torch()
    prob = _prob(kind)
    lam = sl.eigh(prob.A.toarray(), prob.M.toarray(), eigvals_only=True)
    P = _pencil(prob, groups)
    try:
        for a, b in [(prob.alpha, prob.beta), (0.5 * (lam[2] + lam[3]), 0.5 * (lam[9] + lam[10]))]:
            exact = int(np.count_nonzero((lam >= a) & (lam <= b)))
            assert O.inertia_count(prob.A, prob.M, a, b) == exact
            assert P.inertia_count(a, b) == exact
    finally:
        P.close()


@pytest.mark.parametrize("shared_sigma", [False, True])
@pytest.mark.parametrize("kind,groups", [("p9", False), ("quad41", True)])
def test_slices_match_the_oracle_slice_by_slice(kind, groups, shared_sigma):
    torch = _torch()
    prob = _prob(kind)
    lam = sl.eigh(prob.A.toarray(), prob.M.toarray(), eigvals_only=True)
    cuts = _cuts(prob, lam)
    sigma = 0.5 * (prob.alpha + prob.beta) if shared_sigma else float("nan")
    P = _pencil(prob, groups)
    Y0 = torch.from_numpy(np.ascontiguousarray(prob.Y0.T)).cuda()
    try:
        ev, _, res, counts, inert = P.solve_slices(cuts, prob.n_c, Y0, prob.steps, prob.nev_b,
                                                   prob.psi, prob.nev + 20, sigma=sigma)
        torch.cuda.synchronize()
        th = ev.cpu().numpy()
    finally:
        P.close()
    exact = int(np.count_nonzero((lam >= cuts[0]) & (lam <= cuts[-1])))
    assert inert == exact == prob.nev
    off = 0
    for i in range(cuts.size - 1):
        sig = sigma if shared_sigma else 0.5 * (cuts[i] + cuts[i + 1])
        sub = dataclasses.replace(prob, alpha=float(cuts[i]), beta=float(cuts[i + 1]), sigma=sig)
        ro = O.run(sub, want_vectors=False)
        assert counts[i] == ro.theta.size, (i, counts, ro.theta)
        got = th[off:off + counts[i]]
        assert np.max(np.abs(got - ro.theta) / np.abs(ro.theta)) <= EIG_TOL
        off += counts[i]
    assert off == th.size == exact
