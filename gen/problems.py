"""Input builders.  See the package docstring: inputs only, no method arithmetic.

Every builder returns an :class:`EminInput` whose arrays are plain numpy /
scipy objects in FP64 with int32 indices, CSR rows sorted by column.
Degrees of freedom are numbered with x fastest, then y, then z.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class EminInput:
    """What the RCG receives (Sec. 3: A, P0, V_f and V_c).

    ``A`` n x n SPD (CSR), ``P0`` n x nc tentative prolongation (CSR),
    ``B`` n x m fine near-kernel basis (row-major), ``Bc`` nc x m coarse basis.
    ``pattern_power`` is k in the pattern growth S^k P0 (with S = struct(A)).
    ``precond`` is "jacobi" or "bjacobi" (node block size ``block``).
    """

    name: str
    A: sp.csr_matrix
    P0: sp.csr_matrix
    B: np.ndarray
    Bc: np.ndarray
    pattern_power: int = 1
    maxit: int = 10
    precond: str = "jacobi"
    block: int = 1
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def nc(self) -> int:
        return self.P0.shape[1]

    @property
    def m(self) -> int:
        return self.B.shape[1]


def _csr(mat) -> sp.csr_matrix:
    """CSR with int32 indices, sorted columns, duplicates summed, explicit
    zeros kept (the stored structure is what counts)."""
    m = sp.csr_matrix(mat)
    m.sum_duplicates()
    m.sort_indices()
    m.indptr = m.indptr.astype(np.int32)
    m.indices = m.indices.astype(np.int32)
    m.data = np.ascontiguousarray(m.data, dtype=np.float64)
    return m


# --------------------------------------------------------------------------
# Finite-difference Poisson on a d-dimensional cell grid
# --------------------------------------------------------------------------

def fd_poisson(N: int, dim: int, kcell: Optional[np.ndarray] = None) -> sp.csr_matrix:
    """Cell-centred FD Laplacian -div(k grad u) on an N^dim grid, unscaled
    (no h^2 factor).  Interior faces carry the harmonic average
    2 k_a k_b / (k_a + k_b); Dirichlet boundary faces carry k of the cell
    and are eliminated.  With k = 1 this is the (2*dim, -1) stencil."""
    n = N ** dim
    if kcell is None:
        kcell = np.ones(n)
    kcell = np.asarray(kcell, dtype=np.float64).reshape(n)
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for _ in range(dim):
        coords.append(rem % N)
        rem //= N
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    stride = 1
    for d in range(dim):
        c = coords[d]
        a = idx[c < N - 1]
        b = a + stride
        ka, kb = kcell[a], kcell[b]
        face = 2.0 * ka * kb / (ka + kb)
        rows += [a, b]
        cols += [b, a]
        vals += [-face, -face]
        np.add.at(diag, a, face)
        np.add.at(diag, b, face)
        # Dirichlet faces on both ends of this axis
        lo = idx[c == 0]
        hi = idx[c == N - 1]
        np.add.at(diag, lo, kcell[lo])
        np.add.at(diag, hi, kcell[hi])
        stride *= N
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return _csr(A)


def _box_aggregation(N: int, dim: int, b: int) -> np.ndarray:
    """Aggregate id of each cell for b^dim box aggregates (x fastest)."""
    assert N % b == 0
    n = N ** dim
    idx = np.arange(n, dtype=np.int64)
    na = N // b
    agg = np.zeros(n, dtype=np.int64)
    rem = idx.copy()
    mul = 1
    for _ in range(dim):
        c = rem % N
        rem //= N
        agg += (c // b) * mul
        mul *= na
    return agg


def _piecewise_constant_P0(agg: np.ndarray, nc: int) -> sp.csr_matrix:
    """Piecewise-constant tentative prolongation, columns normalised."""
    n = agg.shape[0]
    sizes = np.bincount(agg, minlength=nc).astype(np.float64)
    vals = 1.0 / np.sqrt(sizes[agg])
    P0 = sp.csr_matrix((vals, (np.arange(n), agg)), shape=(n, nc))
    return _csr(P0)


def _scalar_constraint(P0: sp.csr_matrix):
    n = P0.shape[0]
    B = np.ones((n, 1))
    Bc = np.ascontiguousarray(P0.T @ B)  # B_c = P0^T B, as the workload defines it
    return B, Bc


def poisson2d_32() -> EminInput:
    """2D Poisson, 5-point FD on a 32x32 grid (n=1024), constant coefficient,
    2x2 aggregation (nc=256), B=ones, B_c=P0^T B, 10 iterations, Jacobi."""
    N, dim, b = 32, 2, 2
    A = fd_poisson(N, dim)
    agg = _box_aggregation(N, dim, b)
    P0 = _piecewise_constant_P0(agg, (N // b) ** dim)
    B, Bc = _scalar_constraint(P0)
    return EminInput("poisson2d_32", A, P0, B, Bc, pattern_power=1, maxit=10,
                     precond="jacobi")


def _lognormal_poisson(N: int, b: int, sigma: float, seed: int, name: str, maxit: int) -> EminInput:
    rng = np.random.default_rng(seed)
    g = rng.normal(0.0, sigma, size=N ** 3)  # one draw per cell, x fastest
    A = fd_poisson(N, 3, np.exp(g))
    agg = _box_aggregation(N, 3, b)
    P0 = _piecewise_constant_P0(agg, (N // b) ** 3)
    B, Bc = _scalar_constraint(P0)
    return EminInput(name, A, P0, B, Bc, pattern_power=1, maxit=maxit, precond="jacobi")


def poisson3d_het96(N: int = 96) -> EminInput:
    """3D Poisson, 7-point FD on 96^3 cells, k=exp(g), g~N(0,2^2) per cell
    (seed 2), harmonic face averages, 3x3x3 aggregation, B=ones, 20 it.
    ``N`` may be lowered (a multiple of 3) for small parity cases."""
    return _lognormal_poisson(N, 3, 2.0, 2, f"poisson3d_het{N}", 20)


def poisson3d_ln32(N: int = 32) -> EminInput:
    """3D Poisson, 7-point FD on 32^3 cells, k=exp(N(0,1)) (seed 5), 2x2x2
    aggregation, B=ones, 5 iterations; ``extra['e']`` is the fixed random
    vector of the two-grid loss term (seed 55)."""
    inp = _lognormal_poisson(N, 2, 1.0, 5, f"poisson3d_ln{N}", 5)
    inp.extra["e"] = np.random.default_rng(55).normal(size=inp.n)
    return inp


# --------------------------------------------------------------------------
# Trilinear (Q1) hexahedral linear elasticity
# --------------------------------------------------------------------------

def _q1_reference_stiffness(h: float, nu: float) -> np.ndarray:
    """24x24 stiffness of a cube element of side h for E=1, 2x2x2 Gauss.
    Local node a = (i, j, k) in {0,1}^3 with index i + 2j + 4k; local dof
    3a + c."""
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1.0 / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu  # engineering shear strains (xy, yz, zx)
    corners = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)], dtype=float)
    sgn = 2 * corners - 1  # reference coordinates of the nodes in [-1,1]^3
    gp = np.array([-1.0, 1.0]) / math.sqrt(3.0)
    Ke = np.zeros((24, 24))
    jac = h / 2.0
    for gx in gp:
        for gy in gp:
            for gz in gp:
                xi = np.array([gx, gy, gz])
                # dN/dxi for the 8 trilinear shape functions
                dN = np.zeros((8, 3))
                for a in range(8):
                    s = sgn[a]
                    f = 1 + s * xi
                    dN[a, 0] = s[0] * f[1] * f[2] / 8
                    dN[a, 1] = f[0] * s[1] * f[2] / 8
                    dN[a, 2] = f[0] * f[1] * s[2] / 8
                dNx = dN / jac
                Bm = np.zeros((6, 24))
                for a in range(8):
                    dx, dy, dz = dNx[a]
                    Bm[0, 3 * a + 0] = dx
                    Bm[1, 3 * a + 1] = dy
                    Bm[2, 3 * a + 2] = dz
                    Bm[3, 3 * a + 0] = dy
                    Bm[3, 3 * a + 1] = dx
                    Bm[4, 3 * a + 1] = dz
                    Bm[4, 3 * a + 2] = dy
                    Bm[5, 3 * a + 0] = dz
                    Bm[5, 3 * a + 2] = dx
                Ke += Bm.T @ D @ Bm * jac ** 3
    return Ke


def elasticity_q1_40(Ne: int = 40, seed: int = 3, sigma: float = 1.5, nu: float = 0.3,
                     maxit: int = 10, modes: int = 6) -> EminInput:
    """3D linear elasticity, Q1 hexahedra on Ne^3 elements of [0,1]^3
    ((Ne+1)^3 nodes), Young's modulus exp(N(0, sigma^2)) per element, Poisson
    ratio nu, the z=0 face clamped (its dofs eliminated).  Full 3x3 nodal
    blocks are stored.  B = six rigid-body modes from node coordinates.
    Aggregates: nodes grouped by (ix//3, iy//3, (iz-1)//3); each aggregate's
    block of B is factored B_a = Q_a R_a (thin QR), P0 = Q_a, B_c = R_a.
    Pattern growth k = 2, 3x3 block-Jacobi.  ``modes`` = 3 keeps only the
    three translations, ``modes`` = 1 uses the constant vector instead (both
    for tests of other near-kernel sizes on the same nodal structure)."""
    Nn = Ne + 1
    h = 1.0 / Ne
    rng = np.random.default_rng(seed)
    E = np.exp(rng.normal(0.0, sigma, size=Ne ** 3))  # one per element, x fastest
    Ke = _q1_reference_stiffness(h, nu)
    # global node of each element corner
    e = np.arange(Ne ** 3)
    ex, ey, ez = e % Ne, (e // Ne) % Ne, e // (Ne * Ne)
    corner_nodes = []
    for k in (0, 1):
        for j in (0, 1):
            for i in (0, 1):
                corner_nodes.append((ex + i) + Nn * (ey + j) + Nn * Nn * (ez + k))
    corner_nodes = np.stack(corner_nodes, axis=1)  # (nel, 8)
    # free numbering: nodes with iz >= 1 keep their order, shifted
    free_of = np.arange(Nn ** 3) - Nn * Nn
    free_of[: Nn * Nn] = -1
    fn = free_of[corner_nodes]  # (nel, 8)
    ldof = np.where(fn[:, :, None] >= 0, 3 * fn[:, :, None] + np.arange(3)[None, None, :], -1)
    ldof = ldof.reshape(-1, 24)
    n = 3 * Nn * Nn * (Nn - 1)
    R = np.repeat(ldof, 24, axis=1)
    C = np.tile(ldof, (1, 24))
    V = E[:, None] * Ke.reshape(1, -1)
    keep = (R >= 0) & (C >= 0)
    A = sp.coo_matrix((V[keep], (R[keep], C[keep])), shape=(n, n))
    A = _csr(A)
    A = _csr((A + A.T) * 0.5)  # exact symmetry (assembly order differs per triangle)
    # coordinates of free nodes
    fnode = np.arange(Nn * Nn, Nn ** 3)
    ix, iy, iz = fnode % Nn, (fnode // Nn) % Nn, fnode // (Nn * Nn)
    x, y, z = ix * h, iy * h, iz * h
    nf = fnode.shape[0]
    B = np.zeros((n, 6))
    B[0::3, 0] = 1.0
    B[1::3, 1] = 1.0
    B[2::3, 2] = 1.0
    B[0::3, 3] = -y
    B[1::3, 3] = x
    B[1::3, 4] = -z
    B[2::3, 4] = y
    B[0::3, 5] = z
    B[2::3, 5] = -x
    if modes == 3:
        B = B[:, :3].copy()
    elif modes == 1:
        B = np.ones((n, 1))
    elif modes != 6:
        raise ValueError("modes must be 6, 3 or 1")
    m = B.shape[1]
    na = (Nn + 2) // 3  # 14 for Nn = 41
    nz_a = (Nn - 1 + 2) // 3
    agg_node = (ix // 3) + na * (iy // 3) + na * na * ((iz - 1) // 3)
    nagg = na * na * nz_a
    rows_l, cols_l, vals_l = [], [], []
    Bc = np.zeros((m * nagg, m))
    order = np.argsort(agg_node, kind="stable")
    starts = np.searchsorted(agg_node[order], np.arange(nagg + 1))
    for a in range(nagg):
        nodes = order[starts[a]:starts[a + 1]]
        if nodes.size == 0:
            raise RuntimeError("empty aggregate")
        dofs = (3 * nodes[:, None] + np.arange(3)[None, :]).reshape(-1)
        Qa, Ra = np.linalg.qr(B[dofs, :])
        rows_l.append(np.repeat(dofs, m))
        cols_l.append(np.tile(m * a + np.arange(m), dofs.size))
        vals_l.append(Qa.reshape(-1))
        Bc[m * a:m * a + m, :] = Ra
    P0 = sp.coo_matrix((np.concatenate(vals_l), (np.concatenate(rows_l), np.concatenate(cols_l))),
                       shape=(n, m * nagg))
    P0 = _csr(P0)
    inp = EminInput(f"elasticity_q1_{Ne}", A, P0, B, Bc, pattern_power=2, maxit=maxit,
                    precond="bjacobi", block=3)
    inp.extra["n_nodes"] = nf
    return inp


def node_grid2d(N: int = 12, bs: int = 2, seed: int = 7, maxit: int = 5) -> EminInput:
    """A nodal system on an N x N grid of nodes with ``bs`` unknowns per node
    (for tests of the node kernels at other node sizes): A = kron(L, M) with
    L a 5-point graph Laplacian with random edge weights in [0.5, 2] plus a
    unit diagonal shift, and M a fixed SPD bs x bs coupling, so every stored
    node block is full.  B = the bs constant modes (m = bs); 2 x 2 node
    aggregates, P0 = Q_a and B_c = R_a from the thin QR of each aggregate's
    rows of B; pattern struct(A^2 P0); block-Jacobi."""
    rng = np.random.default_rng(seed)
    nn = N * N
    rows, cols, vals = [], [], []
    diag = np.ones(nn)
    for j in range(N):
        for i in range(N):
            a = i + N * j
            for di, dj in ((1, 0), (0, 1)):
                if i + di < N and j + dj < N:
                    b = (i + di) + N * (j + dj)
                    w = rng.uniform(0.5, 2.0)
                    rows += [a, b]
                    cols += [b, a]
                    vals += [-w, -w]
                    diag[a] += w
                    diag[b] += w
    L = sp.coo_matrix((vals + diag.tolist(), (rows + list(range(nn)), cols + list(range(nn)))),
                      shape=(nn, nn)).tocsr()
    M = np.eye(bs) * 2.0 + 0.5 * (np.ones((bs, bs)) - np.eye(bs))
    A = _csr(sp.kron(L, sp.csr_matrix(M)).tocsr())
    n = nn * bs
    B = np.tile(np.eye(bs), (nn, 1))
    node = np.arange(nn)
    agg = (node % N) // 2 + ((N + 1) // 2) * ((node // N) // 2)
    nagg = int(agg.max()) + 1
    rows_l, cols_l, vals_l = [], [], []
    Bc = np.zeros((bs * nagg, bs))
    for g in range(nagg):
        nodes = np.nonzero(agg == g)[0]
        dofs = (bs * nodes[:, None] + np.arange(bs)[None, :]).reshape(-1)
        Qa, Ra = np.linalg.qr(B[dofs, :])
        rows_l.append(np.repeat(dofs, bs))
        cols_l.append(np.tile(bs * g + np.arange(bs), dofs.size))
        vals_l.append(Qa.reshape(-1))
        Bc[bs * g:bs * g + bs, :] = Ra
    P0 = sp.coo_matrix((np.concatenate(vals_l), (np.concatenate(rows_l), np.concatenate(cols_l))),
                       shape=(n, bs * nagg))
    return EminInput(f"node_grid2d_{N}_bs{bs}", A, _csr(P0), B, Bc, pattern_power=2,
                     maxit=maxit, precond="bjacobi", block=bs)


# --------------------------------------------------------------------------
# Random geometric graph Laplacians with greedy aggregation
# --------------------------------------------------------------------------

def _rgg_laplacian(n: int, seed: int, degree: float = 14.0, shift: float = 1e-3):
    """Unit-weight graph Laplacian of a random geometric graph on n uniform
    points of the unit cube, radius chosen so the realised mean degree is
    exactly ``degree`` (the (degree*n/2)-th smallest pair distance), plus
    ``shift`` on the diagonal."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3))
    tree = cKDTree(pts)
    want = int(round(degree * n / 2))
    r = (degree / (n * 4.0 / 3.0 * math.pi)) ** (1.0 / 3.0) * 1.3
    while True:
        pairs = tree.query_pairs(r, output_type="ndarray")
        if pairs.shape[0] >= want + 1:
            break
        r *= 1.25
    d = np.linalg.norm(pts[pairs[:, 0]] - pts[pairs[:, 1]], axis=1)
    sel = np.argsort(d, kind="stable")[:want]
    pairs = pairs[sel]
    i, j = pairs[:, 0], pairs[:, 1]
    W = sp.coo_matrix((np.ones(2 * want), (np.concatenate([i, j]), np.concatenate([j, i]))),
                      shape=(n, n)).tocsr()
    deg = np.asarray(W.sum(axis=1)).ravel()
    L = sp.diags(deg + shift) - W
    return _csr(L)


def _greedy_aggregation(A: sp.csr_matrix) -> np.ndarray:
    """Greedy aggregation: (1) in index order, a node whose neighbours are all
    unaggregated becomes a root and takes them; (2) each leftover node joins
    the aggregate of its first aggregated neighbour (lowest index); (3) the
    rest become singletons."""
    n = A.shape[0]
    ip = A.indptr.tolist()
    ix = A.indices.tolist()
    agg = [-1] * n
    nagg = 0
    for i in range(n):
        if agg[i] >= 0:
            continue
        nb = ix[ip[i]:ip[i + 1]]
        ok = True
        for j in nb:
            if agg[j] >= 0:
                ok = False
                break
        if not ok:
            continue
        for j in nb:
            agg[j] = nagg
        agg[i] = nagg
        nagg += 1
    first = list(agg)
    for i in range(n):
        if first[i] >= 0:
            continue
        for j in ix[ip[i]:ip[i + 1]]:
            if first[j] >= 0:
                agg[i] = first[j]
                break
    for i in range(n):
        if agg[i] < 0:
            agg[i] = nagg
            nagg += 1
    return np.asarray(agg, dtype=np.int64), nagg


def rgg_sizes(count: int = 256, seed: int = 4, lo: float = 2e3, hi: float = 5e4) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)


def rgg_one(b: int, n: int) -> EminInput:
    A = _rgg_laplacian(int(n), 4000 + b)
    agg, nagg = _greedy_aggregation(A)
    P0 = _piecewise_constant_P0(agg, nagg)
    B, Bc = _scalar_constraint(P0)
    return EminInput(f"rgg_{b}", A, P0, B, Bc, pattern_power=1, maxit=15, precond="jacobi")


def rgg_batch(count: int = 256, first: int = 0) -> list:
    """Matrices ``first .. first+count-1`` of the 256-matrix batch (sizes
    log-uniform in [2e3, 5e4], seed 4; matrix b uses seed 4000+b)."""
    sizes = rgg_sizes()
    return [rgg_one(b, sizes[b]) for b in range(first, first + count)]


# --------------------------------------------------------------------------
# Small random problems for pinning tests
# --------------------------------------------------------------------------

def tiny_problem(seed: int, n: int = 14, nc: int = 5, m: int = 1, p0_per_row: int = 1,
                 extra_per_row: int = 2, satisfy: bool = False, dense_pattern: bool = False,
                 rational: bool = False) -> EminInput:
    """Random small SPD problem.  A = L + diag(shift) with L a random weighted
    graph Laplacian; P0 has ``p0_per_row`` random columns per row; B and B_c
    random (or, with ``satisfy``, B = P0 B_c).  ``extra['pattern']`` is a
    random CSR pattern containing P0's plus ``extra_per_row`` random columns
    per row (all columns when ``dense_pattern``).  With ``rational`` the
    values are small integers / simple fractions."""
    rng = np.random.default_rng(seed)
    # random symmetric sparse graph
    W = np.zeros((n, n))
    for i in range(n):
        for j in rng.choice(n, size=min(3, n - 1), replace=False):
            if j != i:
                w = float(rng.integers(1, 4)) if rational else rng.uniform(0.5, 2.0)
                W[i, j] = W[j, i] = w
    D = np.diag(W.sum(axis=1) + (1.0 if rational else rng.uniform(0.1, 1.0, size=n)))
    A = _csr(sp.csr_matrix(D - W))
    P0d = np.zeros((n, nc))
    for i in range(n):
        cols = rng.choice(nc, size=p0_per_row, replace=False)
        for c in cols:
            P0d[i, c] = float(rng.integers(1, 3)) if rational else rng.uniform(0.2, 1.0)
    P0 = _csr(sp.csr_matrix(P0d))
    if rational:
        Bc = rng.integers(1, 4, size=(nc, m)).astype(np.float64)
    else:
        Bc = rng.uniform(0.5, 1.5, size=(nc, m))
    if satisfy:
        B = P0d @ Bc
    else:
        B = (rng.integers(1, 4, size=(n, m)).astype(np.float64) if rational
             else rng.uniform(0.5, 1.5, size=(n, m)))
    patd = P0d != 0
    if dense_pattern:
        patd[:] = True
    else:
        for i in range(n):
            patd[i, rng.choice(nc, size=min(extra_per_row, nc), replace=False)] = True
    pat = sp.csr_matrix(patd.astype(np.float64))
    pat.sort_indices()
    inp = EminInput(f"tiny_{seed}", A, P0, np.ascontiguousarray(B), np.ascontiguousarray(Bc),
                    pattern_power=0, maxit=8, precond="jacobi")
    inp.extra["pattern"] = (pat.indptr.astype(np.int32), pat.indices.astype(np.int32))
    return inp


# --------------------------------------------------------------------------
# Classical C/F setting (P = [W; I]): inputs of the tentative set-up, Alg. 1
# --------------------------------------------------------------------------

@dataclasses.dataclass
class CFInput:
    """What Alg. 1 and the C/F form receive: A (SPD), the strength graph S
    (here A's structure), the near-kernel modes V (n x m), the C/F split
    ``cf`` (coarse index of every COARSE node, -1 for FINE nodes), the
    largest interpolation distance ``lmax``; B = V and B_c = V(C, :) in
    coarse order."""

    name: str
    A: sp.csr_matrix
    S: sp.csr_matrix
    V: np.ndarray
    cf: np.ndarray
    lmax: int
    pattern_power: int = 1
    maxit: int = 10
    precond: str = "jacobi"

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def nc(self) -> int:
        return int(self.cf.max()) + 1

    @property
    def m(self) -> int:
        return self.V.shape[1]

    @property
    def Bc(self) -> np.ndarray:
        order = np.flatnonzero(self.cf >= 0)
        order = order[np.argsort(self.cf[order])]
        return np.ascontiguousarray(self.V[order])


def _standard_coarsening(N: int, dim: int) -> np.ndarray:
    """Coarse index of every even-coordinate cell (x fastest), -1 elsewhere."""
    idx = np.arange(N ** dim)
    keep = np.ones(idx.size, dtype=bool)
    rem = idx.copy()
    for _ in range(dim):
        keep &= (rem % N) % 2 == 0
        rem //= N
    cf = np.full(idx.size, -1, dtype=np.int32)
    cf[keep] = np.arange(int(keep.sum()), dtype=np.int32)
    return cf


def cf_poisson2d(N: int = 32) -> CFInput:
    """2D 5-point Poisson on N x N cells, standard coarsening (even x and
    y), V = ones (m = 1), S = struct(A), l_max = 2 (FINE cells at odd x and
    odd y see their COARSE neighbours at distance 2), pattern A P0."""
    A = fd_poisson(N, 2)
    return CFInput(f"cf_poisson2d_{N}", A, A.copy(), np.ones((N * N, 1)),
                   _standard_coarsening(N, 2), lmax=2, pattern_power=1, maxit=10)


def cf_linear2d(N: int = 24, maxit: int = 8) -> CFInput:
    """2D 5-point Poisson on N x N cells, standard coarsening, V = (1, x, y)
    at the integer cell coordinates (m = 3): a FINE cell needs three COARSE
    cells off one line, which it reaches at distance 2 (odd x, odd y) or 3,
    so l_max = 3; pattern A P0."""
    A = fd_poisson(N, 2)
    idx = np.arange(N * N)
    V = np.stack([np.ones(N * N), (idx % N).astype(float), (idx // N).astype(float)], axis=1)
    return CFInput(f"cf_linear2d_{N}", A, A.copy(), V, _standard_coarsening(N, 2), lmax=3,
                   pattern_power=1, maxit=maxit)


def cf_random(seed: int, n: int = 60, m: int = 2, lmax: int = 3) -> CFInput:
    """A random SPD graph Laplacian (tiny_problem's), COARSE nodes a maximal
    independent set picked greedily in index order, V random (n x m)."""
    base = tiny_problem(seed, n=n, nc=5)
    A = base.A
    coarse = np.zeros(n, dtype=bool)
    blocked = np.zeros(n, dtype=bool)
    for i in range(n):
        if not blocked[i]:
            coarse[i] = True
            blocked[A.indices[A.indptr[i]:A.indptr[i + 1]]] = True
    cf = np.full(n, -1, dtype=np.int32)
    cf[coarse] = np.arange(int(coarse.sum()), dtype=np.int32)
    V = np.random.default_rng(1000 + seed).standard_normal((n, m))
    return CFInput(f"cf_random_{seed}", A, A.copy(), V, cf, lmax=lmax, pattern_power=1,
                   maxit=6)


def by_name(name: str) -> EminInput:
    table = {
        "poisson2d_32": poisson2d_32,
        "poisson3d_het96": poisson3d_het96,
        "poisson3d_ln32": poisson3d_ln32,
        "elasticity_q1_40": elasticity_q1_40,
    }
    return table[name]()
