"""Host-side renumbering behind the Schur solves on trailing blocks (no GPU).

S(zeta) = C_zeta - sum_j Ehat_j^T K_j^{-1} Ehat_j (Sec. 3.1, K_j = B_j -
zeta M_Bj) reads K_j^{-1} Ehat_j only on the rows Ehat_j touches.  The library
numbers those rows last in each padded block, so that, with the no-pivot
factors K = L U, the product needs only the trailing TS x TS blocks:
(K^{-1})_tt = U_tt^{-1} L_tt^{-1}.  These tests take the library's
renumbering (rfd_test_schur_renumber) and check

  * that it is a bijection of each subdomain's interior onto the last d_j
    rows of its D-row block, with the untouched rows first and the touched
    rows in the trailing TS rows, each group in ascending order;
  * D, TS and SJ against their definitions;
  * on the renumbered block, Ehat^T K^{-1} Ehat from a dense solve against
    Ehat_t^T U_tt^{-1} L_tt^{-1} Ehat_t from a no-pivot LU written out here.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W

CASES = {
    # two 20 x 20 interiors padded to 448 rows; M couples through the interface
    "2d_p2_coupled": lambda: W.tiny(N=41, P=2, nev=10, n_c=8, m=40, steps=2, nev_b=12, psi=4,
                                    mass_kind="coupled", cfg_id=50),
    # nine uneven interiors (different pads)
    "2d_p9_uneven": lambda: W.tiny(N=27, P=3, nev=6, n_c=4, m=16, steps=1, nev_b=6, psi=2,
                                   mass_kind="coupled", cfg_id=49),
    # 3D, eight subdomains, random coefficient field
    "3d_p8": lambda: W.tiny(N=11, dim=3, P=2, nev=8, n_c=6, m=40, steps=2, nev_b=10, psi=4,
                            mass_kind="coupled", kfield=True, cfg_id=52),
}


def _lib():
    R = pytest.importorskip("paper_1711_09487_amd")
    try:
        R.lib()
    except RuntimeError as e:
        pytest.skip(str(e))
    return R


def _lu_nopiv(K):
    """In-place LU without pivoting (unit lower L below the diagonal, U on
    and above it), one rank-1 update per column."""
    A = K.copy()
    for k in range(A.shape[0] - 1):
        A[k + 1:, k] /= A[k, k]
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    return A


@pytest.mark.parametrize("name", sorted(CASES))
def test_schur_renumbering(name):
    R = _lib()
    prob = CASES[name]()
    part = np.asarray(prob.part)
    A, M = prob.A.tocsr(), prob.M.tocsr()
    D, TS, SJ, pos = R.rfd_test_schur_renumber(A, M, part)
    iface = np.flatnonzero(part < 0)
    X = (abs(A) + abs(M)).tocsr()
    coupled = np.diff(X[:, iface].tocsr().indptr) > 0
    p = int(part.max()) + 1
    d = [int(np.count_nonzero(part == j)) for j in range(p)]
    assert D == -(-max(d) // 64) * 64
    assert np.all(pos[iface] == -1)
    touched_max, sj_max = 0, 0
    for j in range(p):
        rows = np.flatnonzero(part == j)               # ascending global ids
        pj = pos[rows]
        assert sorted(pj.tolist()) == list(range(D - rows.size, D))
        t = coupled[rows]
        touched_max = max(touched_max, int(t.sum()))
        sj_max = max(sj_max, int(np.unique(X[rows][:, iface].tocsr().indices).size))
        # untouched rows first, touched rows last, each in ascending order
        order = np.concatenate([rows[~t], rows[t]])
        assert np.array_equal(pos[order], np.arange(D - rows.size, D))
    assert TS == min(-(-max(touched_max, 1) // 64) * 64, D)
    assert SJ == sj_max
    assert np.all(pos[coupled & (part >= 0)] >= D - TS)

    # the trailing-block identity on the subdomain with the most touched rows
    j = max(range(p), key=lambda q: int(coupled[part == q].sum()))
    rows = np.flatnonzero(part == j)
    cols = np.unique(X[rows][:, iface].tocsr().indices)
    zeta = 0.37 + 0.21j
    Kz = (A - zeta * M).tocsr()
    K = np.eye(D, dtype=complex)
    idx = pos[rows]
    K[np.ix_(idx, idx)] = Kz[rows][:, rows].toarray()
    E = np.zeros((D, cols.size), dtype=complex)
    E[idx, :] = Kz[rows][:, iface[cols]].toarray()
    t0 = D - TS
    assert not np.any(E[:t0])
    G = E.T @ np.linalg.solve(K, E)
    LU = _lu_nopiv(K)
    Ltt = np.tril(LU[t0:, t0:], -1) + np.eye(TS)
    Utt = np.triu(LU[t0:, t0:])
    Y = sla.solve_triangular(Ltt, E[t0:], lower=True, unit_diagonal=True)
    Gt = E[t0:].T @ sla.solve_triangular(Utt, Y, lower=False)
    assert np.max(np.abs(Gt - G)) <= 1e-10 * np.max(np.abs(G))
