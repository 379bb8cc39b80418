"""The two-level (nested-dissection) S(zeta) on the GPU against the oracle.

With the interface split into groups and a top set (rfd_set_interface_groups),
the library factors S(zeta) as the block LU of its arrow form instead of one
dense LU.  The oracle keeps the dense S(zeta) of Sec. 3.1 (its definition),
so these tests check that the blocked path reproduces it:
  * the filtered block of eq. (3.5), element by element, both modes;
  * the Ritz values of the whole solve (relative error <= 1e-10), residuals;
  * the blocked and the dense GPU paths agree with each other;
  * groupings that would couple two groups are rejected (RFD_EINVAL).
Cases span one and several 64-wide tiles with ragged tails in both the group
blocks and the top block, 2D quadrants and 3D octants, random and coupled M,
a variable coefficient, and the wide diagonal leaves of the top solve.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
EIG_TOL = 1e-10


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


CASES = {
    # 4 groups of 39 (one tile), top 81 (two tiles, ragged)
    "quad41": lambda: W.tiny(N=41, P=4, nev=10, n_c=6, m=40, steps=2, nev_b=10, psi=4,
                             mass_kind="random", cfg_id=51),
    # groups of 79 (two tiles), top 161 (three tiles)
    "quad81_kfield": lambda: W.tiny(N=81, P=4, nev=12, n_c=4, m=40, steps=2, nev_b=10, psi=4,
                                    mass_kind="random", kfield=True, cfg_id=52),
    # 8 octant groups of 61, top 331 padded to 384: 128-wide leaves in the top solve
    "oct11": lambda: W.tiny(N=11, dim=3, P=4, nev=8, n_c=6, m=40, steps=2, nev_b=10, psi=4,
                            mass_kind="random", cfg_id=53),
    "quad41_identity_midpoint": lambda: W.tiny(N=41, P=4, nev=8, n_c=4, m=30, steps=2, nev_b=10,
                                               psi=4, rule="midpoint", cfg_id=54),
}
_cache = {}


def _prob(name):
    if name not in _cache:
        p = CASES[name]()
        _cache[name] = (p, O.run(p))
    return _cache[name]


def _groups(prob):
    g = W.interface_groups(prob.grid, prob.meta["P"])
    assert g is not None and g.size == prob.s
    return g


def _pencil(prob, mode, groups=True):
    import paper_1711_09487_amd as R
    P = R.Pencil(prob.A, prob.M)
    P.set_partition(prob.part)
    if groups:
        P.set_interface_groups(_groups(prob))
    rule = R.RFD_RULE_GAUSS if prob.rule == "gauss" else R.RFD_RULE_MIDPOINT
    P.set_interval_and_poles(prob.alpha, prob.beta, prob.n_c, rule)
    P.set_precision(mode)
    return P


def _dev(torch, Y):
    return torch.from_numpy(np.ascontiguousarray(Y.T)).cuda()


def _oracle_filter(prob, Y):
    dd = O.DD(prob.A, prob.M, prob.part)
    z, w = O.quadrature(prob.alpha, prob.beta, prob.n_c, prob.rule)
    return O.filter_apply(O.factor_poles(dd, z), w, Y)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_blocked_filter_elementwise(name, mode):
    torch = _torch()
    prob, _ = _prob(name)
    ref = _oracle_filter(prob, prob.Y0)
    P = _pencil(prob, mode)
    Wg = P.filter_apply(_dev(torch, prob.Y0)).cpu().numpy().T
    P.close()
    err = np.max(np.abs(Wg - ref)) / np.max(np.abs(ref))
    assert err < (1e-12 if mode == 0 else 1e-11), err


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_blocked_end_to_end(name, mode):
    torch = _torch()
    prob, ro = _prob(name)
    P = _pencil(prob, mode)
    Q = P.filter_interface(_dev(torch, prob.Y0), prob.steps)
    P.solve_interior(prob.sigma, prob.nev_b, prob.psi)
    ev, _, res = P.rayleigh_ritz(prob.nev + 20)
    torch.cuda.synchronize()
    th, r = ev.cpu().numpy(), res.cpu().numpy()
    mu = Q.shape[0]
    P.close()
    assert mu == ro.mu
    assert th.size == ro.theta.size == prob.nev
    assert np.max(np.abs(th - ro.theta) / np.abs(ro.theta)) <= EIG_TOL
    assert np.all(r <= 10 * ro.resid + 1e-12)


@pytest.mark.parametrize("mode", [0, 1])
def test_blocked_equals_dense_gpu_path(mode):
    torch = _torch()
    prob, _ = _prob("oct11")
    Y = _dev(torch, prob.Y0)
    out = []
    for groups in (True, False):
        P = _pencil(prob, mode, groups)
        out.append(P.filter_apply(Y).cpu().numpy())
        P.close()
    a, b = out
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("mode", [0, 1])
def test_blocked_filter_with_coupled_mass(mode):
    """A coupled M keeps the grouping valid (M_C has the stencil's pattern);
    the filter with M_E != 0 matches the oracle."""
    torch = _torch()
    prob = W.tiny(N=41, P=4, nev=6, n_c=4, m=16, steps=1, nev_b=6, psi=2,
                  mass_kind="coupled", cfg_id=55)
    ref = _oracle_filter(prob, prob.Y0)
    P = _pencil(prob, mode)
    Wg = P.filter_apply(_dev(torch, prob.Y0)).cpu().numpy().T
    P.close()
    err = np.max(np.abs(Wg - ref)) / np.max(np.abs(ref))
    assert err < (1e-12 if mode == 0 else 1e-11), err


def test_blocked_pole_windows_and_regrouping():
    """Pole windows of 2 on the blocked S, then switching back to the dense S
    on the same handle: both give the oracle's filter."""
    torch = _torch()
    prob, _ = _prob("quad41")
    ref = _oracle_filter(prob, prob.Y0)
    P = _pencil(prob, 1)
    P.set_pole_window(2)
    W1 = P.filter_apply(_dev(torch, prob.Y0)).cpu().numpy().T
    P.set_pole_window(0)
    P.set_interface_groups(None)
    W2 = P.filter_apply(_dev(torch, prob.Y0)).cpu().numpy().T
    P.close()
    for Wg in (W1, W2):
        assert np.max(np.abs(Wg - ref)) / np.max(np.abs(ref)) < 1e-11


def test_invalid_groupings_are_rejected():
    import paper_1711_09487_amd as R
    _torch()
    prob, _ = _prob("quad41")
    g = _groups(prob)
    dd = O.DD(prob.A, prob.M, prob.part)
    Cnz = abs(dd.C) > 0
    # a top node coupled in C to group 0, moved into group 1
    top = np.flatnonzero(g < 0)
    a = next(int(t) for t in top if np.any(g[np.flatnonzero(Cnz[t])] == 0))
    coupled = g.copy()
    coupled[a] = 1
    empty = np.where(g == 2, -1, g).astype(np.int32)      # groups 0, 1, 3: group 2 empty
    P = _pencil(prob, 0, groups=False)
    try:
        for bad in (coupled, empty):
            with pytest.raises(R.RfdError) as e:
                P.set_interface_groups(bad)
            assert e.value.code == 1
        # the handle still works with a valid grouping afterwards
        P.set_interface_groups(g)
        ref = _oracle_filter(prob, prob.Y0)
        Wg = P.filter_apply(_dev(_torch(), prob.Y0)).cpu().numpy().T
        assert np.max(np.abs(Wg - ref)) / np.max(np.abs(ref)) < 1e-12
    finally:
        P.close()


def test_config2_blocked_against_stored_oracle():
    """The 255 x 255 workload with the interface split into its four
    quadrants and the central cross: the Ritz values of both modes against
    the oracle's stored values."""
    torch = _torch()
    path = os.path.join(GOLD, "oracle_c2.json")
    if not os.path.exists(path):
        pytest.skip("stored oracle result missing")
    gold = json.load(open(path))
    prob = W.config(2, steps=gold["steps"], nev_b=gold["nev_b"], psi=gold["psi"])
    th_ref = np.array(gold["theta"])
    for mode in (0, 1):
        P = _pencil(prob, mode)
        P.filter_interface(_dev(torch, prob.Y0), gold["steps"])
        P.solve_interior(prob.sigma, gold["nev_b"], gold["psi"])
        ev, _, res = P.rayleigh_ritz(prob.nev + 50)
        torch.cuda.synchronize()
        th = ev.cpu().numpy()
        P.close()
        assert th.size == th_ref.size
        rel = np.max(np.abs(th - th_ref) / th_ref)
        print(f"mode {mode}: max rel err vs stored oracle {rel:.2e}")
        assert rel <= EIG_TOL
