"""Seeded synthetic inputs shared by the tests, bench.py and the oracle-side checks.

This module holds NO arithmetic of the numerical method: it only draws random numbers and
evaluates closed-form fields at coordinates the caller supplies (each side computes its own
node coordinates). It imports neither the oracle nor the HIP library.

Workloads (periodic boxes; each stands in for the periodic Taylor-Green / ABC-type flows on which
the paper validates its scheme):

  tgv2d     2D Taylor-Green velocity on the unit square, u = sin 2pi x cos 2pi y,
            v = -cos 2pi x sin 2pi y
  fourier   random low-pass velocity: every component is
            sum_{0<|k|_2<=kmax} a_k cos(2pi k.x / L) + b_k sin(2pi k.x / L), a, b ~ N(0,1),
            rescaled so that max |v| over a uniform sample lattice equals `vmax`
  rhs       a standard-normal vector per DoF (the batched random right-hand sides)
  batch     the list of (side, N, seed) of the batched workload
"""
import numpy as np

# Named workloads (sizes, degrees and physical parameters).
CONFIGS = {
    "tgv2d_16_N3": dict(dim=2, cells=(16, 16), lengths=(1.0, 1.0), N=3, dt=1e-3, theta=0.6,
                        nu=1e-2, field="tgv2d", rtol=1e-12),
    "rand2d_256_N6": dict(dim=2, cells=(256, 256), lengths=(1.0, 1.0), N=6, dt=5e-4, theta=0.6,
                          nu=1e-3, field="fourier", kmax=8, seed=2, vmax=0.1, steps=50,
                          rtol=1e-10),
    "rand3d_64_N4": dict(dim=3, cells=(64, 64, 64), lengths=(1.0, 1.0, 1.0), N=4, dt=1e-3,
                         theta=0.6, nu=1e-3, field="fourier", kmax=6, seed=3, vmax=0.1,
                         rtol=1e-10),
    "batch2d_64": dict(dim=2, count=64, side_range=(32, 256), N_range=(2, 8), seed=4,
                       dt=5e-4, rtol=1e-10, maxit=400000),
    "adjoint3d_48_N3": dict(dim=3, cells=(48, 48, 48), lengths=(1.0, 1.0, 1.0), N=3, dt=1e-3,
                            theta=0.6, nu=1e-2, field="fourier", kmax=6, seed=5, vmax=0.1,
                            steps=20, checkpoint=5, fd_dirs=16),
}


def tgv2d(coords):
    """2D Taylor-Green velocity. coords[d] = 1D coordinate arrays along x, y for the nodes of
    component d's own grid: coords = [(xu, yu), (xv, yv)]. Returns tensor arrays [y, x]."""
    (xu, yu), (xv, yv) = coords
    u = np.sin(2 * np.pi * xu)[None, :] * np.cos(2 * np.pi * yu)[:, None]
    v = -np.cos(2 * np.pi * xv)[None, :] * np.sin(2 * np.pi * yv)[:, None]
    return [u, v]


class FourierField:
    """Random periodic field with wavenumbers 0 < |k|_2 <= kmax (one per component)."""

    def __init__(self, seed, dim, kmax, lengths, ncomp=None):
        self.dim = dim
        self.kmax = int(kmax)
        self.lengths = tuple(float(x) for x in lengths)
        self.ncomp = dim if ncomp is None else ncomp
        rng = np.random.default_rng(seed)
        K = 2 * self.kmax + 1
        ks = np.arange(-self.kmax, self.kmax + 1)
        grids = np.meshgrid(*([ks] * dim), indexing="ij")      # [kz?, ky, kx] reversed below
        k2 = sum(g.astype(np.float64) ** 2 for g in grids)
        mask = (k2 > 0) & (k2 <= self.kmax ** 2)
        self.coef = []
        for _ in range(self.ncomp):
            a = rng.standard_normal((K,) * dim)
            b = rng.standard_normal((K,) * dim)
            # f = Re sum_k (a_k - i b_k) exp(i 2pi k.x/L)
            self.coef.append(np.where(mask, a - 1j * b, 0.0))
        self.ks = ks
        self.scale = 1.0

    def _eval(self, c, axes_coords):
        """axes_coords = list of 1D coordinate arrays ordered x, y(, z). Returns tensor [z,]y,x."""
        C = self.coef[c]
        # C is indexed [k_axis0, k_axis1, ...] with axis order matching tensor order (z,) y, x
        E = [np.exp(2j * np.pi * np.outer(self.ks, xc) / L)
             for xc, L in zip(axes_coords, self.lengths)]
        out = C
        for t, d in enumerate(reversed(range(self.dim))):      # tensor axis t carries direction d
            out = np.moveaxis(np.tensordot(out, E[d], axes=([t], [0])), -1, t)
        return self.scale * np.real(out)

    def eval(self, coords):
        """coords[c] = [x_c, y_c(, z_c)] node coordinates of component c's grid."""
        return [self._eval(c, coords[c]) for c in range(self.ncomp)]

    def normalise(self, vmax, samples=64):
        """Rescale so that max over components of max |f| on a uniform lattice equals vmax."""
        self.scale = 1.0
        lat = [np.arange(samples) * L / samples for L in self.lengths]
        m = max(np.abs(self._eval(c, lat)).max() for c in range(self.ncomp))
        self.scale = vmax / m
        return self


def random_rhs(seed, ndof):
    """Standard-normal right-hand side (one value per DoF)."""
    return np.random.default_rng(seed).standard_normal(ndof)


def batch_problems(seed=4, count=64, side_range=(32, 256), N_range=(2, 8)):
    """Batched workload: list of dicts (side, N, seed) with sides and degrees drawn uniformly
    (inclusive ranges) and per-problem RHS seed 1000*seed + j."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_range[0], side_range[1] + 1, size=count)
    Ns = rng.integers(N_range[0], N_range[1] + 1, size=count)
    return [dict(side=int(s), N=int(N), seed=1000 * seed + j) for j, (s, N) in enumerate(zip(sides, Ns))]


def tensor_to_blocked(t, cells, n):
    """Rearrange a tensor-layout array ([z,]y,x with x = i*n + l1) into the element-blocked
    layout (cells in C order (k,j,i), then nodes (l3,l2,l1)). Pure data movement."""
    t = np.asarray(t)
    if len(cells) == 2:
        nx, ny = cells
        return np.ascontiguousarray(t.reshape(ny, n, nx, n).transpose(0, 2, 1, 3)).reshape(-1)
    nx, ny, nz = cells
    return np.ascontiguousarray(
        t.reshape(nz, n, ny, n, nx, n).transpose(0, 2, 4, 1, 3, 5)).reshape(-1)


def blocked_to_tensor(v, cells, n):
    """Inverse of tensor_to_blocked."""
    v = np.asarray(v)
    if len(cells) == 2:
        nx, ny = cells
        return v.reshape(ny, nx, n, n).transpose(0, 2, 1, 3).reshape(ny * n, nx * n)
    nx, ny, nz = cells
    return v.reshape(nz, ny, nx, n, n, n).transpose(0, 3, 1, 4, 2, 5).reshape(nz * n, ny * n, nx * n)


def staggered_coords(cells, lengths, xi):
    """Node coordinates per component: component c is staggered (shifted by half a cell) along
    direction c. Main cell i covers [i h, (i+1) h]; nodes at (i + xi_l) h, dual nodes at
    (i + 1/2 + xi_l) h. Returns coords[c][d] (1D arrays)."""
    dim = len(cells)
    out = []
    for c in range(dim):
        per = []
        for d in range(dim):
            h = lengths[d] / cells[d]
            shift = 0.5 if d == c else 0.0
            per.append(((np.arange(cells[d])[:, None] + shift + np.asarray(xi)[None, :]) * h).reshape(-1))
        out.append(per)
    return out


def main_coords(cells, lengths, xi):
    """Node coordinates of the main grid along each direction."""
    return [((np.arange(c)[:, None] + np.asarray(xi)[None, :]) * (L / c)).reshape(-1)
            for c, L in zip(cells, lengths)]
