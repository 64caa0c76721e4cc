"""Solvers for the pressure and viscous systems (test infrastructure only).

On a periodic grid A_p is symmetric positive semi-definite (Section 2.1: H = D^T M^-1 D) and the
pressure is defined up to null(D). The result the GPU path must reproduce is therefore the
minimum-norm solution q = A_p^+ b for b in range(A_p): the unique solution orthogonal (in the
Euclidean DoF inner product) to the null space Z. Three independent ways to get it:

  cg              the paper's matrix-free conjugate gradient (Hestenes-Stiefel, no preconditioner,
                  x0 = 0, stop on ||r||_2 <= rtol ||b||_2), here on the assembled CSR matrix
  pcg             the same with a preconditioner (the paper's future work); block_jacobi gives
                  the cell-block Jacobi preconditioner of an assembled operator
  dense_min_norm  dense Cholesky of A + Z Z^T (SPD); for b orthogonal to Z its solution is the
                  minimum-norm solution (tiny grids only)
  FastDiag        tensor-product fast diagonalisation: each 1D operator M_d^-1/2 H_d M_d^-1/2 is
                  diagonalised once (dense symmetric eigensolver), and alpha M + beta K is then
                  diagonal in the tensor product of those eigenbases. Exact up to rounding.
"""
import numpy as np
import scipy.linalg as sla

from .operators import apply_along, pressure_1d, null_basis_1d, null_basis_dirichlet, project_null


def cg(A, b, rtol, maxit, x0=None):
    """Unpreconditioned conjugate gradient for SPD (or consistent SPSD) A.

    Returns (x, iters, rel_res_recurrence). Stops when ||r|| <= rtol ||b||."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    p = r.copy()
    rho = float(r @ r)
    bnorm = float(np.sqrt(b @ b))
    if bnorm == 0.0:
        return x, 0, 0.0
    it = 0
    while it < maxit and np.sqrt(rho) > rtol * bnorm:
        q = A @ p
        sigma = float(p @ q)
        alpha = rho / sigma
        x = x + alpha * p
        r = r - alpha * q
        rho_new = float(r @ r)
        p = r + (rho_new / rho) * p
        rho = rho_new
        it += 1
    return x, it, float(np.sqrt(rho) / bnorm)


def pcg(A, b, rtol, maxit, precond, x0=None):
    """Preconditioned conjugate gradient (Hestenes-Stiefel with the preconditioned inner product
    <r, z>, z = precond(r)); the preconditioners the paper names as future work for its
    matrix-free CG (Section 2.1, closing remark). Stops when ||r||_2 <= rtol ||b||_2 (the same
    stopping test as cg). Returns (x, iters, rel_res_recurrence)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    bnorm = float(np.sqrt(b @ b))
    if bnorm == 0.0:
        return x, 0, 0.0
    z = precond(r)
    p = z.copy()
    rho = float(r @ z)
    it = 0
    while it < maxit and np.sqrt(float(r @ r)) > rtol * bnorm:
        q = A @ p
        alpha = rho / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        z = precond(r)
        rho_new = float(r @ z)
        p = z + (rho_new / rho) * p
        rho = rho_new
        it += 1
    return x, it, float(np.sqrt(r @ r) / bnorm)


def block_jacobi(grid, A):
    """Cell-block Jacobi preconditioner of an operator assembled in the tensor layout: the
    inverse of the (N+1)^d x (N+1)^d diagonal block of every cell (the coupling of a cell's own
    nodes), applied cell by cell. Returns a function r -> z on flat tensor-layout vectors."""
    from .layout import tensor_to_blocked, blocked_to_tensor
    n = grid.n
    NC = n ** grid.dim
    idx = tensor_to_blocked(np.arange(grid.ndof).reshape(grid.shape()), grid.cells, n).astype(np.int64)
    ncells = grid.ndof // NC
    Ab = A.tocsr()[idx][:, idx]
    inv = np.stack([np.linalg.inv(Ab[c * NC:(c + 1) * NC, c * NC:(c + 1) * NC].toarray())
                    for c in range(ncells)])

    def apply(r):
        rb = np.asarray(r, dtype=np.float64).reshape(-1)[idx].reshape(ncells, NC)
        zb = np.einsum("cij,cj->ci", inv, rb).reshape(-1)
        z = np.empty(grid.ndof)
        z[idx] = zb
        return z
    return apply


def dense_min_norm(A, Z, b):
    """Minimum-norm solution of A x = b for b orthogonal to the columns of Z (orthonormal),
    via a dense Cholesky of the SPD matrix A + Z Z^T."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    S = Ad + Z @ Z.T
    c = sla.cho_factor(S)
    return sla.cho_solve(c, b)


class FastDiag:
    """Direct solver for alpha M^{xyz} + beta K on a uniform grid (tensor layout), periodic or
    with the Dirichlet directions of Grid.periodic (their 1D operators have no null space)."""

    def __init__(self, grid, zero_tol=1e-10):
        self.grid = grid
        self.V = []         # eigenvectors of M_d^-1/2 H_d M_d^-1/2 (orthogonal)
        self.lam = []       # eigenvalues
        self.zero = []      # per-direction boolean mask of zero eigenvalues
        self.sqw = []       # sqrt of the 1D global mass diagonal
        self.Z = []         # orthonormal null basis of D_d
        w = grid.tab.w
        for d in range(grid.dim):
            nc = grid.cells[d]
            per = grid.periodic[d]
            H = pressure_1d(nc, grid.N, per).toarray()
            sq = np.sqrt(np.tile(w, nc))
            Hh = H / sq[:, None] / sq[None, :]
            Hh = 0.5 * (Hh + Hh.T)
            lam, V = np.linalg.eigh(Hh)
            self.V.append(V)
            self.lam.append(lam)
            self.zero.append(np.abs(lam) <= zero_tol * np.abs(lam).max())
            self.sqw.append(sq)
            self.Z.append(null_basis_1d(nc, grid.N) if per else null_basis_dirichlet(nc, grid.N))

    def _weights(self):
        g = self.grid
        W = np.ones(g.shape())
        for d in range(g.dim):
            shp = [1] * g.dim
            shp[g.dim - 1 - d] = -1
            W = W * self.sqw[d].reshape(shp)
        return W           # sqrt of the diagonal of M^{xyz}

    def solve(self, b, alpha, beta, project=True):
        """Solve (alpha M + beta K) x = b, b in tensor layout. For alpha == 0 the minimum-norm
        solution is returned (b must be orthogonal to null(K); it is projected first)."""
        g = self.grid
        b = np.asarray(b, dtype=np.float64).reshape(g.shape())
        if alpha == 0.0:
            b = project_null(g, b, self.Z)
        sw = self._weights()
        y = b / sw
        for d in range(g.dim):
            y = apply_along(self.V[d].T, y, g.dim - 1 - d)
        # eigenvalues of alpha I + beta sum_d h_d^-2 Lambda_d, and the joint null mask
        lam = np.full(g.shape(), alpha, dtype=np.float64)
        allzero = np.ones(g.shape(), dtype=bool)
        for d in range(g.dim):
            shp = [1] * g.dim
            shp[g.dim - 1 - d] = -1
            lam = lam + beta / g.h[d] ** 2 * self.lam[d].reshape(shp)
            allzero = allzero & self.zero[d].reshape(shp)
        if alpha == 0.0:
            y = np.where(allzero, 0.0, y / np.where(allzero, 1.0, lam))
        else:
            y = y / lam
        for d in range(g.dim):
            y = apply_along(self.V[d], y, g.dim - 1 - d)
        x = y / sw
        if alpha == 0.0 and project:
            x = project_null(g, x, self.Z)
        return x
