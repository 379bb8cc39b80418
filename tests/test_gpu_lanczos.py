"""Alg. 3.1 (Lanczos restricted to the interface, with its stopping test) on
the GPU against the oracle's filter_lanczos, through the C ABI.

Same seeded inputs on both sides; the checks:
  * the same number of block steps, the same mu and the same stop decision;
  * the traces tr(T_t) after every block, element by element (relative
    1e-10): they are the quantity of the stopping test of line 13;
  * every block's filtered image lies in the GPU's span (the Krylov
    structure), with the oracle's filter;
  * the Ritz values of the whole solve with this Q (relative 1e-10) and the
    residuals;
both precision modes, the dense and the two-level S(zeta).
"""
import numpy as np
import pytest

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
    # small block: the stopping test runs every ceil(10 / 3) = 4 blocks
    "p9_m3": (lambda: W.tiny(N=13, P=3, nev=6, n_c=6, m=3, steps=1, nev_b=8, psi=4,
                             mass_kind="random", cfg_id=71), False, dict(tol=1e-6, max_steps=40)),
    # two-level S, block of 12 (tested every block)
    "quad41_m12": (lambda: W.tiny(N=41, P=4, nev=10, n_c=8, m=12, steps=1, nev_b=12, psi=5,
                                  mass_kind="random", cfg_id=72), True,
                   dict(tol=1e-6, max_steps=40)),
    # the 31 x 31 workload with 4 poles and a block of 4
    "config1_m4": (lambda: W.tiny(N=31, P=2, nev=20, n_c=4, m=4, steps=1, nev_b=20, psi=4),
                   False, dict(tol=1e-6, max_steps=60)),
}
_cache = {}


def _case(name):
    if name not in _cache:
        make, groups, lz = CASES[name]
        prob = make()
        dd = O.DD(prob.A, prob.M, prob.part)
        z, w = O.quadrature(prob.alpha, prob.beta, prob.n_c, prob.rule)
        fac = O.factor_poles(dd, z)
        Q, info = O.filter_lanczos(dd, z, w, prob.Y0, factors=fac, **lz)
        ro = O.run(prob, lanczos=lz)
        _cache[name] = (prob, groups, lz, fac, w, Q, info, ro)
    return _cache[name]


def _pencil(prob, mode, groups):
    import paper_1711_09487_amd as R
    P = R.Pencil(prob.A, prob.M)
    P.set_partition(prob.part)
    if groups:
        P.set_interface_groups(W.interface_groups(prob.grid, prob.meta["P"]))
    P.set_interval_and_poles(prob.alpha, prob.beta, prob.n_c, R.RFD_RULE_GAUSS)
    P.set_precision(mode)
    return P


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_lanczos_matches_the_oracle(name, mode):
    torch = _torch()
    prob, groups, lz, fac, w, Qo, info, ro = _case(name)
    P = _pencil(prob, mode, groups)
    Y0 = torch.from_numpy(np.ascontiguousarray(prob.Y0.T)).cuda()
    Qg, gi = P.filter_lanczos(Y0, **lz)
    P.solve_interior(prob.sigma, prob.nev_b, prob.psi)
    ev, _, res = P.rayleigh_ritz(prob.nev + 20)
    torch.cuda.synchronize()
    Qg = Qg.cpu().numpy().T
    th, r = ev.cpu().numpy(), res.cpu().numpy()
    P.close()
    # the same process: steps, stop decision, basis size
    assert gi["steps"] == info["steps"] and gi["converged"] == info["converged"]
    assert Qg.shape[1] == Qo.shape[1] == ro.mu
    tr_o = np.array(info["traces"])
    assert np.max(np.abs(gi["traces"] - tr_o) / np.abs(tr_o)) <= 1e-10
    assert np.max(np.abs(Qg.T @ Qg - np.eye(Qg.shape[1]))) < 1e-12
    # Krylov structure: the start block and F applied to every block but the
    # last lie in span(Q_gpu) (up to the dropped directions and the rounding
    # of F, both relative to the filter's scale on the start block: late
    # blocks, whose image under F has all but vanished, are held to the same
    # absolute level)
    Y = prob.Y0
    assert np.max(np.abs(Y - Qg @ (Qg.T @ Y))) < 1e-12 * np.max(np.abs(Y))
    sizes = [a.shape[0] for a in info["A"]]
    off = np.concatenate([[0], np.cumsum(sizes)])
    scale = np.max(np.abs(O.filter_apply(fac, w, Qg[:, :sizes[0]])))
    for t in range(len(sizes) - 1):
        B = Qg[:, off[t]:off[t + 1]]
        FB = O.filter_apply(fac, w, B)
        assert np.max(np.abs(FB - Qg @ (Qg.T @ FB))) < 1e-10 * scale, t
    # the whole solve with this interface basis
    assert th.size == ro.theta.size
    assert np.max(np.abs(th - ro.theta) / np.abs(ro.theta)) <= EIG_TOL
    assert np.all(r <= 10 * ro.resid + 1e-12)


def test_lanczos_single_step_and_no_test():
    """max_steps = 1 returns the orthonormalised start block (no stop test
    can fire with a single trace); tol = 0 runs to max_steps."""
    torch = _torch()
    prob, groups, lz, fac, w, Qo, info, ro = _case("p9_m3")
    P = _pencil(prob, 0, False)
    Y0 = torch.from_numpy(np.ascontiguousarray(prob.Y0.T)).cuda()
    Q1, g1 = P.filter_lanczos(Y0, tol=1e-6, max_steps=1)
    Q5, g5 = P.filter_lanczos(Y0, tol=0.0, max_steps=5)
    P.close()
    assert Q1.shape[0] == 3 and g1["steps"] == 1 and not g1["converged"]
    assert Q5.shape[0] == 15 and g5["steps"] == 5 and not g5["converged"]
    dd = O.DD(prob.A, prob.M, prob.part)
    z, w2 = O.quadrature(prob.alpha, prob.beta, prob.n_c, prob.rule)
    _, i5 = O.filter_lanczos(dd, z, w2, prob.Y0, tol=0.0, max_steps=5, factors=fac)
    assert np.max(np.abs(g5["traces"] - np.array(i5["traces"])) / np.abs(i5["traces"])) <= 1e-10
