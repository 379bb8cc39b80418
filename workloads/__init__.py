"""Seeded synthetic inputs for the RF-DDES interface-filter path.

This module builds the *data* that both sides receive: sparse symmetric
pencils (A, M) from finite-difference grid stencils, geometric partitions
with one-line (one-plane) vertex separators, random starting blocks and
search intervals.  It holds none of the method's arithmetic (no poles, no
Schur complements, no filters, no projections); the oracle and the GPU
library each implement that on their own.

Recipe (all FP64, natural lexicographic node order, x fastest):

* 2D 5-point / 3D 7-point Laplacian, Dirichlet.  With a node coefficient
  field k the face coefficient is the harmonic mean 2 k_i k_j / (k_i + k_j)
  and a boundary face uses k_i; A_ii = sum of the node's face coefficients,
  A_ij = -k_face.  k == 1 gives the constant stencil (4, -1, -1, -1, -1).
  These are the paper's synthetic "FDmesh" family (Sec. 6, Tables 6.1/6.4:
  FD Laplacians with Dirichlet boundary conditions, M = I), generalised to a
  random diagonal M.
* Separators sit at 0-based grid lines floor(q (N+1) / P) - 1, q = 1..P-1,
  in every axis; a node on any separator line is an interface node
  (part = -1), the others belong to the box they fall in (subdomain ids in
  lexicographic box order, x fastest).  This is the paper's reordering
  (Sec. 2.3, eq. (2.5)) with vertex separators instead of METIS.
* Seeds: numpy default_rng([cfg_id, stream]) with streams
  0 = M diagonal, 1 = starting block Y0, 2 = coefficient field k,
  3 = shapes and intervals (batched / serving mixes), 4 = arrivals.
* Intervals "enclosing the lowest nev eigenvalues": alpha = 0 (all pencils
  here are SPD) and beta = (lam_nev + lam_{nev+1}) / 2 rounded to 10
  significant digits, so that no eigenvalue sits on the contour and the
  input is the same on every machine.  lam comes from the closed form when
  M = I with the constant stencil, else from a reference eigensolver
  (dense for small n, ARPACK shift-invert otherwise).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.sparse as sp

STREAM_M, STREAM_Y0, STREAM_K, STREAM_SHAPE, STREAM_ARRIVAL = 0, 1, 2, 3, 4


def rng(cfg_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(cfg_id), int(stream)])


# --------------------------------------------------------------------------
# pencils
# --------------------------------------------------------------------------
def laplacian(shape, kcoef: Optional[np.ndarray] = None) -> sp.csr_matrix:
    """Finite-difference Laplacian on a grid of the given shape (Dirichlet)."""
    shape = tuple(int(s) for s in shape)
    n = int(np.prod(shape))
    k = np.ones(n) if kcoef is None else np.asarray(kcoef, dtype=np.float64).ravel()
    assert k.shape == (n,)
    idx = np.arange(n).reshape(shape[::-1])  # idx[z, y, x]; x fastest
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    ndim = len(shape)
    for ax in range(ndim):
        a = ndim - 1 - ax  # numpy axis of grid axis `ax`
        lo = np.take(idx, np.arange(shape[ax] - 1), axis=a).ravel()
        hi = np.take(idx, np.arange(1, shape[ax]), axis=a).ravel()
        kf = 2.0 * k[lo] * k[hi] / (k[lo] + k[hi])
        diag[lo] += kf
        diag[hi] += kf
        rows += [lo, hi]
        cols += [hi, lo]
        vals += [-kf, -kf]
        # boundary faces (Dirichlet): the two ends of the axis
        first = np.take(idx, [0], axis=a).ravel()
        last = np.take(idx, [shape[ax] - 1], axis=a).ravel()
        diag[first] += k[first]
        diag[last] += k[last]
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    A.sum_duplicates()
    A.sort_indices()
    return A


def mass(n: int, kind: str, gen: Optional[np.random.Generator] = None,
         A: Optional[sp.csr_matrix] = None) -> sp.csr_matrix:
    """M = I, a random diagonal U[0.5, 1.5], or a non-diagonal SPD 'coupled'
    matrix (1 on the diagonal, 0.1 on every stencil neighbour: strictly
    diagonally dominant for 2D/3D stencils, so SPD)."""
    if kind == "identity":
        M = sp.identity(n, format="csr")
    elif kind == "random":
        M = sp.diags(gen.uniform(0.5, 1.5, n)).tocsr()
    elif kind == "coupled":
        assert A is not None
        P = A.copy().tocsr()
        P.data[:] = 0.1
        P.setdiag(1.0)
        M = P.tocsr()
    else:
        raise ValueError(kind)
    M = sp.csr_matrix(M)
    M.sort_indices()
    return M


def separators(N: int, P: int):
    return [int(math.floor(q * (N + 1) / P)) - 1 for q in range(1, P)]


def grid_partition(shape, P: int) -> np.ndarray:
    """part[i] = subdomain id of node i, or -1 for an interface node."""
    shape = tuple(int(s) for s in shape)
    ndim = len(shape)
    coords = np.indices(shape[::-1]).reshape(ndim, -1)[::-1]  # coords[ax] per node
    is_sep = np.zeros(coords.shape[1], dtype=bool)
    box = np.zeros(coords.shape[1], dtype=np.int64)
    stride = 1
    for ax in range(ndim):
        seps = np.array(separators(shape[ax], P), dtype=np.int64)
        c = coords[ax]
        is_sep |= np.isin(c, seps)
        b = np.searchsorted(seps, c, side="right")  # box index along the axis
        box += b * stride
        stride *= P
    part = np.where(is_sep, -1, box).astype(np.int32)
    # renumber subdomains densely in order of first appearance of the box id
    used = np.unique(part[part >= 0])
    remap = -np.ones(int(used.max()) + 1 if used.size else 1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    out = part.copy()
    out[part >= 0] = remap[part[part >= 0]]
    return out.astype(np.int32)


def interface_groups(shape, P: int) -> Optional[np.ndarray]:
    """Two-level grouping of the interface nodes of grid_partition(shape, P)
    (ascending global id): -1 for a node on the middle separator of any axis
    (the top set), else the index of the half-space box it lies in (one bit
    per axis, x lowest).  Defined for even P >= 4 (the middle separator
    exists and the halves hold separators of their own); None otherwise."""
    shape = tuple(int(s) for s in shape)
    if P < 4 or P % 2:
        return None
    ndim = len(shape)
    coords = np.indices(shape[::-1]).reshape(ndim, -1)[::-1]
    part = grid_partition(shape, P)
    iface = np.flatnonzero(part < 0)
    top = np.zeros(iface.size, dtype=bool)
    grp = np.zeros(iface.size, dtype=np.int64)
    for ax in range(ndim):
        mid = separators(shape[ax], P)[P // 2 - 1]
        c = coords[ax][iface]
        top |= c == mid
        grp += (c > mid).astype(np.int64) << ax
    return np.where(top, -1, grp).astype(np.int32)


def closed_form_eigs(shape) -> np.ndarray:
    """Eigenvalues of the constant-coefficient Dirichlet Laplacian with M = I:
    sum over axes of 4 sin^2(pi i / (2 (N+1))), i = 1..N (sorted)."""
    lam = np.zeros(1)
    for N in shape:
        e = 4.0 * np.sin(np.pi * np.arange(1, N + 1) / (2.0 * (N + 1))) ** 2
        lam = (lam[:, None] + e[None, :]).ravel()
    return np.sort(lam)


def lowest_eigs(A, M, k: int, closed_shape=None) -> np.ndarray:
    """The k smallest eigenvalues of (A, M) (reference eigensolver, not RF-DDES)."""
    n = A.shape[0]
    if closed_shape is not None:
        return closed_form_eigs(closed_shape)[:k]
    if n <= 1500:
        import scipy.linalg as sl
        return sl.eigh(A.toarray(), M.toarray(), eigvals_only=True)[:k]
    import scipy.sparse.linalg as sla
    w = sla.eigsh(A.tocsc(), k=k, M=M.tocsc(), sigma=0.0, which="LM",
                  return_eigenvectors=False, tol=1e-13)
    return np.sort(w)


def interval_lowest(A, M, nev: int, closed_shape=None):
    lam = lowest_eigs(A, M, nev + 1, closed_shape)
    if not lam[nev] - lam[nev - 1] > 1e-10 * abs(lam[nev]):
        raise ValueError("the interval would cut a multiple eigenvalue")
    # rounded to 10 significant digits so that the input does not depend on the
    # last bits of the reference eigensolver on a given machine
    beta = float(f"{0.5 * (lam[nev - 1] + lam[nev]):.10g}")
    return 0.0, beta, lam


def random_block(s: int, m: int, gen: np.random.Generator) -> np.ndarray:
    """Y0: s x m, N(0,1), FP64, column-major (Fortran order)."""
    return np.asfortranarray(gen.standard_normal((s, m)))


# --------------------------------------------------------------------------
# problems
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    name: str
    A: sp.csr_matrix
    M: sp.csr_matrix
    part: np.ndarray
    alpha: float
    beta: float
    n_c: int
    rule: str            # "gauss" | "midpoint"
    m: int               # block width
    steps: int           # block-Krylov steps
    sigma: float
    nev_b: int
    psi: int
    Y0: np.ndarray       # s x m, interface rows in ascending global id
    nev: int             # eigenvalues inside [alpha, beta]
    grid: tuple = ()
    exact: Optional[np.ndarray] = None   # closed-form or reference eigenvalues (lowest nev+1)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self):
        return self.A.shape[0]

    @property
    def s(self):
        return int(np.count_nonzero(self.part < 0))

    @property
    def p(self):
        return int(self.part.max()) + 1


def grid_problem(name, cfg_id, shape, P, nev, n_c, m, steps, nev_b, psi,
                 mass_kind="identity", kfield=False, rule="gauss", sigma="center", known=None):
    """known = (alpha, beta, lam) skips the reference eigensolve (values stored
    by a previous run of it, e.g. for the 63^3 pencil)."""
    shape = tuple(shape)
    n = int(np.prod(shape))
    kc = np.exp(rng(cfg_id, STREAM_K).standard_normal(n)) if kfield else None
    A = laplacian(shape, kc)
    M = mass(n, mass_kind, rng(cfg_id, STREAM_M), A)
    part = grid_partition(shape, P)
    closed = shape if (mass_kind == "identity" and not kfield) else None
    if known is not None:
        alpha, beta, lam = float(known[0]), float(known[1]), np.asarray(known[2])
    else:
        alpha, beta, lam = interval_lowest(A, M, nev, closed)
    s = int(np.count_nonzero(part < 0))
    m = min(m, s)
    Y0 = random_block(s, m, rng(cfg_id, STREAM_Y0))
    sig = 0.5 * (alpha + beta) if sigma == "center" else float(sigma)
    return Problem(name=name, A=A, M=M, part=part, alpha=alpha, beta=beta, n_c=n_c,
                   rule=rule, m=m, steps=steps, sigma=sig, nev_b=nev_b, psi=psi, Y0=Y0,
                   nev=nev, grid=shape, exact=lam,
                   meta=dict(cfg_id=cfg_id, P=P, mass=mass_kind, kfield=kfield))


def config(i: int, known=None, **override) -> Problem:
    """The measured workloads.

    1: 2D 31x31, M = I, 2x2 partition (4 interiors of 15x15, s = 61), lowest 20,
       4 Gauss-Legendre poles, m = 30.
    2: 2D 255x255, M = diag U[0.5,1.5], 8x8 partition (31x31 interiors,
       s = 3521), lowest 200, 8 poles, m = 300.
    3: 3D 63^3, M = diag U[0.5,1.5], 4x4x4 partition (15^3 interiors,
       s = 34047), lowest 500, 8 poles, m = 700.  Its interval needs the 501
       lowest eigenvalues of a 250047 x 250047 pencil; pass known = (alpha,
       beta, lam) from a stored run to skip that eigensolve.

    The method's free parameters (block-Krylov steps, nev_b, psi) are the
    smallest found to reach the accuracy targets against the exact or
    reference eigenvalues: 31x31 (2, 20, 4); 255x255 (5, 40, 6), where every
    residual also falls below 1e-9; 63^3 (4, 40, 4), where every eigenvalue
    is within 1e-10.  override = dict(steps=, nev_b=, psi=) replaces them.
    """
    def pick(d, key):
        return override.get(key, d)
    if i == 1:
        return grid_problem("C1 2D 31x31 M=I p=4", 1, (31, 31), 2, 20, 4, 30, pick(2, "steps"),
                            pick(20, "nev_b"), pick(4, "psi"))
    if i == 2:
        return grid_problem("C2 2D 255x255 Mdiag p=64", 2, (255, 255), 8, 200, 8, 300,
                            pick(5, "steps"), pick(40, "nev_b"), pick(6, "psi"),
                            mass_kind="random")
    if i == 3:
        return grid_problem("C3 3D 63^3 Mdiag p=64", 3, (63, 63, 63), 4, 500, 8, 700,
                            pick(4, "steps"), pick(40, "nev_b"), pick(4, "psi"),
                            mass_kind="random", known=known)
    raise ValueError(i)


def batch_specs(count: int = 256, cfg_id: int = 4):
    """Shapes of the batched workload: grid side N ~ U{31..127}, P ~ U{2,3,4},
    nev ~ U{10..60}, N_c ~ U{4..8} (stream 3)."""
    g = rng(cfg_id, STREAM_SHAPE)
    out = []
    for b in range(count):
        N = int(g.integers(31, 128))
        P = int(g.integers(2, 5))
        nev = int(g.integers(10, 61))
        n_c = int(g.integers(4, 9))
        out.append(dict(N=N, P=P, nev=nev, n_c=n_c))
    return out


def batch_problem(b: int, spec: dict, cfg_id: int = 4, nev_b: int = 20, psi: int = 4,
                  steps: int = 2) -> Problem:
    """One pencil of the batched workload: variable coefficient k ~ lognormal(0,1)
    per node, M = diag U[0.5,1.5], m = min(s, ceil(1.5 nev))."""
    sub_id = cfg_id * 100000 + b
    N, P, nev, n_c = spec["N"], spec["P"], spec["nev"], spec["n_c"]
    m = int(math.ceil(1.5 * nev))
    return grid_problem(f"B{b} 2D {N}x{N} P={P}", sub_id, (N, N), P, nev, n_c, m, steps,
                        nev_b, psi, mass_kind="random", kfield=True)


def tiny(N=11, dim=2, P=2, nev=6, n_c=4, m=None, steps=2, nev_b=8, psi=3,
         mass_kind="identity", kfield=False, rule="gauss", cfg_id=99, sigma="center"):
    """Small grid problems for pins and parity at a few tiles."""
    shape = (N,) * dim
    part = grid_partition(shape, P)
    s = int(np.count_nonzero(part < 0))
    return grid_problem(f"tiny {shape} P={P} {mass_kind}", cfg_id, shape, P, nev, n_c,
                        s if m is None else m, steps, nev_b, psi, mass_kind=mass_kind,
                        kfield=kfield, rule=rule, sigma=sigma)


def serving_requests(count: int, spectra: dict, weights: dict, cfg_id: int = 5,
                     kmin: int = 20, kmax: int = 300, i0max: int = 500):
    """A seeded stream of spectrum-slicing requests (stream 3 for shapes,
    stream 4 for arrivals).

    spectra: pencil name -> ascending known eigenvalues of that pencil (the
    lowest ones; a slice never reaches beyond them); weights: pencil name ->
    probability.  Each request picks a pencil, a count k ~ U{kmin..kmax} and a
    first index i0 ~ U{1..min(i0max, len - k - 1)} (1-based, clipped to what
    the known spectrum allows), and the interval alpha = (lam_{i0-1} +
    lam_{i0}) / 2 (0 for i0 = 1), beta = (lam_{i0+k-1} + lam_{i0+k}) / 2, both
    rounded to 10 significant digits; slices that would cut a multiple
    eigenvalue are moved by one.  Returns a list of dicts (pencil, alpha,
    beta, k, i0) and unit-rate exponential inter-arrival gaps (scale them by
    1 / QPS)."""
    g = rng(cfg_id, STREAM_SHAPE)
    names = sorted(weights)
    prob = np.array([weights[nm] for nm in names], dtype=float)
    prob /= prob.sum()
    out = []
    for _ in range(count):
        nm = names[int(g.choice(len(names), p=prob))]
        lam = np.asarray(spectra[nm])
        L = lam.size
        k = int(g.integers(kmin, min(kmax, L - 2) + 1))
        i0 = int(g.integers(1, max(1, min(i0max, L - k - 1)) + 1))
        gap = 1e-10 * max(1.0, abs(lam[-1]))
        while i0 > 1 and lam[i0 - 1] - lam[i0 - 2] <= gap:
            i0 -= 1
        while i0 + k < L and lam[i0 + k] - lam[i0 + k - 1] <= gap:
            k -= 1
        alpha = 0.0 if i0 == 1 else float(f"{0.5 * (lam[i0 - 2] + lam[i0 - 1]):.10g}")
        beta = float(f"{0.5 * (lam[i0 + k - 2] + lam[i0 + k - 1]):.10g}")
        out.append(dict(pencil=nm, alpha=alpha, beta=beta, k=k, i0=i0))
    gaps = rng(cfg_id, STREAM_ARRIVAL).exponential(1.0, count)
    return out, gaps
