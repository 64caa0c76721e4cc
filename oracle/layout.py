"""DoF layouts (test infrastructure only).

Element-blocked layout (the library boundary's layout): cells in C order (k, j, i) with i (x)
fastest, then the (N+1)^d nodal values of one cell in C order (l3, l2, l1) with l1 (x) fastest.
This is the DoF numbering hat{p}_{l,i,j,k} of eqs. (uDGpoly)-(pDGpoly) laid out cell by cell.

Tensor layout (used here for Kronecker assembly): one global index per direction,
g_x = i*(N+1) + l1, and the d-dimensional array indexed [g_z, g_y, g_x] (C order, x fastest),
so that kron(A_z, A_y, A_x) acts on its flattening.

For the staggered velocity components the same two layouts are used on the dual grid of that
component: dual cell i along the staggered direction is [x_i, x_{i+1}] between the centres of
main cells i and i+1 (periodic wrap).
"""
import numpy as np


def blocked_to_tensor(v, cells, n):
    """cells = (nx, ny) or (nx, ny, nz); v flat (element-blocked) -> tensor array."""
    v = np.asarray(v)
    if len(cells) == 2:
        nx, ny = cells
        a = v.reshape(ny, nx, n, n)              # [j, i, l2, l1]
        return a.transpose(0, 2, 1, 3).reshape(ny * n, nx * n)
    nx, ny, nz = cells
    a = v.reshape(nz, ny, nx, n, n, n)           # [k, j, i, l3, l2, l1]
    return a.transpose(0, 3, 1, 4, 2, 5).reshape(nz * n, ny * n, nx * n)


def tensor_to_blocked(t, cells, n):
    """Inverse of blocked_to_tensor; returns a flat array."""
    t = np.asarray(t)
    if len(cells) == 2:
        nx, ny = cells
        a = t.reshape(ny, n, nx, n).transpose(0, 2, 1, 3)
        return np.ascontiguousarray(a).reshape(-1)
    nx, ny, nz = cells
    a = t.reshape(nz, n, ny, n, nx, n).transpose(0, 2, 4, 1, 3, 5)
    return np.ascontiguousarray(a).reshape(-1)


def axis_of(d, dim):
    """Tensor axis that carries spatial direction d (0=x, 1=y, 2=z)."""
    return dim - 1 - d


def node_coords(cells, lengths, xi, d, staggered):
    """Coordinates along direction d of every tensor index of that axis.

    Main cell i covers [i h, (i+1) h]; its nodes sit at (i + xi_l) h. Dual cell i (staggered
    direction) covers [(i+1/2) h, (i+3/2) h]; its nodes sit at (i + 1/2 + xi_l) h.
    """
    nc = cells[d]
    h = lengths[d] / nc
    shift = 0.5 if staggered else 0.0
    i = np.arange(nc)[:, None]
    return ((i + shift + np.asarray(xi)[None, :]) * h).reshape(-1)
