"""Assembled sparse operators of the pressure path (test infrastructure only).

All matrices act on the TENSOR layout (see layout.py) and are built with scipy.sparse.kron
from 1D periodic matrices, following Section 2.1 of arXiv:1602.05806:

  D      1D weak gradient, block row i: -L~ on cell i, R~ on cell i+1           eq. (weakgradientop)
  H      1D pressure operator D^T M^-1 D (block tridiagonal L, C, R)           eq. (PerPrSyst)
  K      sum_d h_d^-2 (M on the other directions) (x) H_d                      eq. (pSyst)
  A_p    dt * K, acting on P^{n+theta}                                         eq. (LOpressure)
  A_v    M^{xyz} + nu dt K                                                     eqs. (uSDG12), (Ux), (implicitviscosity)
  B_d    h_d^-1 (M on the other directions) (x) D_d^T: RHS b = sum_d B_d U_d   eq. (LOpressure)
  G_d    dt h_d^-1 M_d^-1 D_d: velocity update U_d -= G_d q                    eq. (LOvelocityU)

Periodic boundaries in every direction: the block rows wrap (the paper's 1D periodic form,
eq. (pSyst1d), uses P_{Nx+1} = P_1).
"""
import numpy as np
import scipy.sparse as sp

from .basis import tables


class Grid:
    """Uniform Cartesian grid: cells=(nx,ny[,nz]), lengths=(Lx,Ly[,Lz]), degree N; periodic
    along every direction unless `periodic` (one flag per direction) says otherwise. A
    non-periodic direction carries a homogeneous Dirichlet pressure condition (see grad_1d)."""

    def __init__(self, cells, lengths, N, periodic=None):
        self.cells = tuple(int(c) for c in cells)
        self.lengths = tuple(float(x) for x in lengths)
        if len(self.cells) not in (2, 3) or len(self.lengths) != len(self.cells):
            raise ValueError("2D or 3D grids only")
        self.periodic = (tuple(bool(p) for p in periodic) if periodic is not None
                         else (True,) * len(self.cells))
        if len(self.periodic) != len(self.cells):
            raise ValueError("one periodic flag per direction")
        self.dim = len(self.cells)
        self.N = int(N)
        self.n = self.N + 1
        self.h = tuple(L / c for L, c in zip(self.lengths, self.cells))
        self.tab = tables(self.N)
        self.ndof = int(np.prod(self.cells)) * self.n ** self.dim

    def shape(self):
        """Tensor-layout shape, axes ordered (z,) y, x."""
        return tuple(c * self.n for c in reversed(self.cells))


# ---------------------------------------------------------------- 1D periodic matrices

def mass_1d(nc, N):
    """Global 1D mass matrix I_nc (x) diag(w) (GL basis: diagonal, text after eq. pDGpoly)."""
    return sp.kron(sp.identity(nc), sp.diags(tables(N).w), format="csr")


def grad_1d(nc, N):
    """Periodic weak gradient D of eq. (weakgradientop): (D P)_i = R~ P_{i+1} - L~ P_i.

    Row block i is dual cell i (between main cells i and i+1)."""
    t = tables(N)
    n = t.n
    D = sp.lil_matrix((nc * n, nc * n))
    for i in range(nc):
        ip = (i + 1) % nc
        D[i * n:(i + 1) * n, i * n:(i + 1) * n] = D[i * n:(i + 1) * n, i * n:(i + 1) * n].toarray() - t.Lt
        D[i * n:(i + 1) * n, ip * n:(ip + 1) * n] = D[i * n:(i + 1) * n, ip * n:(ip + 1) * n].toarray() + t.Rt
    return D.tocsr()


def pressure_1d(nc, N, periodic=True):
    """H = D^T M^-1 D (eq. PerPrSyst), exactly symmetrised against rounding.

    periodic=False: homogeneous Dirichlet pressure at both ends by odd reflection across the wall
    (method of images; reading of the paper's "appropriate pressure boundary conditions",
    Section 2.1): the pressure of the mirror cell beyond a wall is -J P of the adjacent cell, J
    reversing the node order, so the wall rows of eq. (pSyst1d) read (C - L J) P_0 + R P_1 and
    L P_{nc-2} + (C - R J) P_{nc-1}. This is the periodic operator of the doubled domain
    restricted to odd functions: symmetric, positive definite for even N; for odd N the odd
    cell-periodic mode of the periodic null space stays in the null space."""
    if not periodic:
        t = tables(N)
        n = t.n
        J = np.eye(n)[::-1]
        H = sp.lil_matrix((nc * n, nc * n))
        for i in range(nc):
            blk = t.Cblk.copy()
            if i == 0:
                blk = blk - t.Lblk @ J
            if i == nc - 1:
                blk = blk - t.Rblk @ J
            H[i * n:(i + 1) * n, i * n:(i + 1) * n] = blk
            if i > 0:
                H[i * n:(i + 1) * n, (i - 1) * n:i * n] = t.Lblk
            if i < nc - 1:
                H[i * n:(i + 1) * n, (i + 1) * n:(i + 2) * n] = t.Rblk
        H = H.tocsr()
        return ((H + H.T) * 0.5).tocsr()
    D = grad_1d(nc, N)
    Minv = sp.kron(sp.identity(nc), sp.diags(1.0 / tables(N).w))
    H = (D.T @ Minv @ D).tocsr()
    return ((H + H.T) * 0.5).tocsr()


def l2_dual_to_main_1d(nc, N):
    """pi_{*->#} along the staggered direction, eq. (l2forward):
    U#_i = M^-1 (M^L U*_{i-1} + M^R U*_i) (dual cell i-1 overlaps the left half of main cell i)."""
    t = tables(N)
    n = t.n
    P = sp.lil_matrix((nc * n, nc * n))
    Minv = np.diag(1.0 / t.w)
    for i in range(nc):
        im = (i - 1) % nc
        blk = P[i * n:(i + 1) * n, im * n:(im + 1) * n].toarray()
        P[i * n:(i + 1) * n, im * n:(im + 1) * n] = blk + Minv @ t.ML
        blk = P[i * n:(i + 1) * n, i * n:(i + 1) * n].toarray()
        P[i * n:(i + 1) * n, i * n:(i + 1) * n] = blk + Minv @ t.MR
    return P.tocsr()


def l2_main_to_dual_1d(nc, N):
    """pi_{#->*} along the staggered direction, eq. (l2backward):
    F*_i = M^-1 (M^L F#_i + M^R F#_{i+1})."""
    t = tables(N)
    n = t.n
    P = sp.lil_matrix((nc * n, nc * n))
    Minv = np.diag(1.0 / t.w)
    for i in range(nc):
        ip = (i + 1) % nc
        blk = P[i * n:(i + 1) * n, i * n:(i + 1) * n].toarray()
        P[i * n:(i + 1) * n, i * n:(i + 1) * n] = blk + Minv @ t.ML
        blk = P[i * n:(i + 1) * n, ip * n:(ip + 1) * n].toarray()
        P[i * n:(i + 1) * n, ip * n:(ip + 1) * n] = blk + Minv @ t.MR
    return P.tocsr()


# ---------------------------------------------------------------- d-dimensional assembly

def _kron_along(grid, d, mat_d, other):
    """kron over tensor axes (z,) y, x with mat_d on direction d and other(e) elsewhere."""
    mats = []
    for e in reversed(range(grid.dim)):          # tensor axis order: last direction first
        mats.append(mat_d if e == d else other(e))
    out = mats[0]
    for m in mats[1:]:
        out = sp.kron(out, m, format="csr")
    return out.tocsr()


def stiffness(grid):
    """K = sum_d h_d^-2 (W on the other directions) (x) H_d  (eq. pSyst without dt)."""
    K = None
    for d in range(grid.dim):
        H = pressure_1d(grid.cells[d], grid.N, grid.periodic[d])
        term = _kron_along(grid, d, H, lambda e: mass_1d(grid.cells[e], grid.N)) / grid.h[d] ** 2
        K = term if K is None else K + term
    return K.tocsr()


def full_mass(grid):
    """M^{xyz}: the d-fold tensor product of the 1D mass (diagonal)."""
    return _kron_along(grid, 0, mass_1d(grid.cells[0], grid.N),
                       lambda e: mass_1d(grid.cells[e], grid.N))


def pressure_operator(grid, dt):
    """A_p = dt K acting on q = P^{n+theta} (eq. LOpressure; eq. pSyst divided by theta)."""
    return (dt * stiffness(grid)).tocsr()


def viscous_operator(grid, dt, nu):
    """A_v = M^{xyz} + nu dt K (eq. implicitviscosity with the dt and h factors of eq. uSDG12)."""
    return (full_mass(grid) + nu * dt * stiffness(grid)).tocsr()


def null_basis_dirichlet(nc, N):
    """Orthonormal null basis of the Dirichlet (odd-reflection) 1D operator: the part of the
    cell-periodic kernel that is odd about the cell centre (J q = -q): the odd mode for odd N,
    nothing for even N (the constant is even and removed by the reflection)."""
    n = N + 1
    Z = null_basis_tiled(1, N)                       # per-cell kernel modes, orthonormal
    J = np.eye(n)[::-1]
    odd = 0.5 * (Z - J @ Z)
    u, sv, _ = np.linalg.svd(odd, full_matrices=False)
    modes = u[:, sv > 1e-8]
    return np.tile(modes, (nc, 1)) / np.sqrt(nc)


def null_bases(grid):
    """Per-direction orthonormal null bases: the cell-periodic kernel of D along periodic
    directions, its odd part along Dirichlet directions."""
    return [null_basis_tiled(grid.cells[d], grid.N) if grid.periodic[d]
            else null_basis_dirichlet(grid.cells[d], grid.N) for d in range(grid.dim)]


def div_rhs(grid, d):
    """B_d = h_d^-1 (W on the other directions) (x) D_d^T; b = sum_d B_d U_d (eq. LOpressure).

    The discrete divergence of eq. (pSDG1) is -sum_d B_d U_d."""
    Dt = grad_1d(grid.cells[d], grid.N).T.tocsr()
    return (_kron_along(grid, d, Dt, lambda e: mass_1d(grid.cells[e], grid.N)) / grid.h[d]).tocsr()


def grad_update(grid, d, dt):
    """G_d = dt h_d^-1 M_d^-1 D_d (identity on the other directions); eq. (LOvelocityU)."""
    nc = grid.cells[d]
    Minv = sp.kron(sp.identity(nc), sp.diags(1.0 / grid.tab.w))
    G1 = (Minv @ grad_1d(nc, grid.N)).tocsr() * (dt / grid.h[d])
    return _kron_along(grid, d, G1, lambda e: sp.identity(grid.cells[e] * grid.n))


# ---------------------------------------------------------------- null space (Section 2.1, end)

def null_basis_1d(nc, N, tol=1e-10):
    """Orthonormal basis of null(D) for the periodic 1D weak gradient, by dense SVD.

    The paper states that periodic pressures are defined up to weak solutions of dP = 0."""
    D = grad_1d(nc, N).toarray()
    _, s, vt = np.linalg.svd(D)
    keep = s <= tol * s.max() if s.max() > 0 else np.ones_like(s, dtype=bool)
    return vt[keep].T.copy()                      # columns


def apply_along(mat, X, axis):
    """Multiply tensor X by the (sparse or dense) matrix `mat` along `axis`."""
    Xm = np.moveaxis(X, axis, 0)
    shp = Xm.shape
    Y = mat @ Xm.reshape(shp[0], -1)
    Y = np.asarray(Y).reshape((mat.shape[0],) + shp[1:])
    return np.moveaxis(Y, 0, axis)


def null_basis_tiled(nc, N):
    """Orthonormal basis of null(D) for nc periodic cells without a size-nc SVD: the kernel of
    the periodic weak gradient is cell-periodic (the same polynomial in every cell; Section 2.1,
    end), so the per-cell modes are read off the kernel on 3 cells and tiled over nc cells."""
    n = N + 1
    Z3 = null_basis_1d(3, N)
    if Z3.shape[1] == 0:
        return np.zeros((nc * n, 0))
    modes, _ = np.linalg.qr(Z3[:n])                 # per-cell modes, orthonormal in R^n
    return np.tile(modes, (nc, 1)) / np.sqrt(nc)


def apply_operator(grid, X, alpha, beta, absolute=False):
    """(alpha M^{xyz} + beta K) X for a tensor-layout X without assembling the d-dimensional
    matrix: K = sum_d h_d^-2 (M on the other directions) (x) H_d applied one direction at a time
    with the 1D sparse H_d and the diagonal 1D masses (eq. pSyst).

    absolute=True gives |alpha M + beta K| |X| (entrywise absolute values of the operator and of
    X), the scale of the rounding error of any floating-point evaluation of the product."""
    X = np.asarray(X, dtype=np.float64).reshape(grid.shape())
    if absolute:
        X = np.abs(X)
        alpha, beta = abs(alpha), abs(beta)
    masses = [mass_1d(grid.cells[d], grid.N) for d in range(grid.dim)]
    out = np.zeros_like(X)
    if alpha != 0.0:
        MX = X
        for d in range(grid.dim):
            MX = apply_along(masses[d], MX, grid.dim - 1 - d)
        out = out + alpha * MX
    for d in range(grid.dim):
        H = pressure_1d(grid.cells[d], grid.N, grid.periodic[d])
        if absolute:
            H = abs(H)
        T = apply_along(H, X, grid.dim - 1 - d)
        for e in range(grid.dim):
            if e != d:
                T = apply_along(masses[e], T, grid.dim - 1 - e)
        out = out + beta / grid.h[d] ** 2 * T
    return out


def div_rhs_apply(grid, U):
    """b = sum_d B_d U_d (eq. LOpressure) without assembling the d-dimensional B_d: along
    direction d the 1D D_d^T / h_d, along every other direction the diagonal 1D mass. U: list of
    dual components in tensor layout."""
    b = np.zeros(grid.shape())
    for d in range(grid.dim):
        T = apply_along(grad_1d(grid.cells[d], grid.N).T.tocsr(), np.asarray(U[d], dtype=np.float64),
                        grid.dim - 1 - d) / grid.h[d]
        for e in range(grid.dim):
            if e != d:
                T = apply_along(mass_1d(grid.cells[e], grid.N), T, grid.dim - 1 - e)
        b = b + T
    return b


def project_null(grid, X, Zs):
    """v <- v - Z Z^T v with Z = kron of the per-direction orthonormal bases Zs[d].

    X is a tensor-layout array; returns the projected copy (range of A_p). A direction without
    null vectors (Dirichlet) makes Z empty: nothing is removed."""
    if any(z.shape[1] == 0 for z in Zs):
        return np.array(X, dtype=np.float64, copy=True)
    C = X
    for d in range(grid.dim):
        C = apply_along(Zs[d].T, C, grid.dim - 1 - d)
    back = C
    for d in range(grid.dim):
        back = apply_along(Zs[d], back, grid.dim - 1 - d)
    return X - back


def apply_at(grid, X, index, alpha, beta):
    """(alpha M^{xyz} + beta K) X evaluated at the tensor multi-indices `index` (array of shape
    (m, dim), axes ordered (z,) y, x), from the block form of eq. (pSyst): along direction d the
    output node l_d of cell i_d couples to the nodes of cells i_d-1, i_d, i_d+1 through the blocks
    L, C, R, weighted by the GL masses of the other directions and h_d^-2. Periodic wrap, or the
    odd reflection of pressure_1d beyond a Dirichlet wall.
    Used to check single outputs of full-size applications without assembling the matrix."""
    t = grid.tab
    n = grid.n
    X = np.asarray(X)
    index = np.atleast_2d(np.asarray(index, dtype=np.int64))
    out = np.zeros(index.shape[0])
    for r, idx in enumerate(index):
        g = [int(v) for v in idx]                       # tensor axes (z,) y, x
        ld = {d: g[grid.dim - 1 - d] % n for d in range(grid.dim)}
        wall = 1.0
        for d in range(grid.dim):
            wall *= t.w[ld[d]]
        val = alpha * wall * X[tuple(g)]
        for d in range(grid.dim):
            ax = grid.dim - 1 - d
            nc = grid.cells[d]
            i = g[ax] // n
            wperp = wall / t.w[ld[d]]
            acc = 0.0
            for off, blk in ((-1, t.Lblk), (0, t.Cblk), (1, t.Rblk)):
                mirror = not grid.periodic[d] and not 0 <= i + off < nc
                j = i if mirror else (i + off) % nc
                for m in range(n):
                    gg = list(g)
                    # beyond a Dirichlet wall: the odd reflection -J P of the adjacent cell
                    gg[ax] = j * n + (n - 1 - m if mirror else m)
                    acc += blk[ld[d], m] * (-X[tuple(gg)] if mirror else X[tuple(gg)])
            val += beta / grid.h[d] ** 2 * wperp * acc
        out[r] = val
    return out
