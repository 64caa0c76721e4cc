"""One semi-implicit fractional step (test infrastructure only).

Follows eqs. (LOdiffusionU)-(LOvelocityW) of arXiv:1602.05806, Section 2.1-2.3, in this order:
  1. pi_{*->#}: L2 projection of each dual velocity component to the main grid   eq. (l2forward)
  2. explicit convection on the main grid: DG residual with the Rusanov flux,
     advanced by the third-order TVD Runge-Kutta scheme (Shu-Osher form)       eqs. (Fu)-(Fw)
  3. implicit viscosity on the main grid: (M + nu dt K) U# = M Fu#              eq. (LOdiffusionU)
  4. pi_{#->*}: L2 projection back to the dual grids                            eq. (l2backward)
  5. pressure: A_p q = b, b = sum_d B_d U*_d, q = P^{n+theta}                    eq. (LOpressure)
  6. velocity update U_d^{n+1} = U*_d - dt h_d^-1 M_d^-1 D_d q                   eq. (LOvelocityU)
  7. P^{n+1} = (q - (1 - theta) P^n) / theta  (definition of P^{n+theta}, eq. uSDG1)

Readings where the paper leaves details open:
  * Rusanov speed: at a face normal to direction e, s = 2 max(|v_e^-|, |v_e^+|), the largest
    eigenvalue of the Jacobian of (v.n) v; the paper's additional viscous part of s belongs to
    its explicit-viscosity variant and is dropped because viscosity is implicit here.
  * Quadrature: collocation at the GL nodes (volume terms) and face values by extrapolation
    with phi_l(0), phi_l(1); transverse face integrals at the GL nodes.
  * Viscous operator: M + nu dt K (the dt and h factors of eq. uSDG12 made explicit).
  * All arrays are in TENSOR layout here; dual components use the tensor layout of their own
    dual grid.
"""
import numpy as np

from .operators import (Grid, apply_along, l2_dual_to_main_1d, l2_main_to_dual_1d,
                        div_rhs, grad_update, pressure_operator, viscous_operator)
from .solvers import FastDiag


def _ax(grid, d):
    return grid.dim - 1 - d


def dual_to_main(grid, Ud, d):
    """pi_{*->#} of component d (staggered along d)."""
    return apply_along(l2_dual_to_main_1d(grid.cells[d], grid.N), Ud, _ax(grid, d))


def main_to_dual(grid, Fm, d):
    """pi_{#->*} of component d."""
    return apply_along(l2_main_to_dual_1d(grid.cells[d], grid.N), Fm, _ax(grid, d))


def _split(X, axis, nc, n):
    """Move `axis` last and split it into (cell, node)."""
    Xm = np.moveaxis(X, axis, -1)
    return Xm.reshape(Xm.shape[:-1] + (nc, n))


def _merge(Xs, axis):
    Xm = Xs.reshape(Xs.shape[:-2] + (-1,))
    return np.moveaxis(Xm, -1, axis)


def convective_rate(grid, V, nu=0.0, convection=True):
    """L(V): time derivative of the main-grid velocity from the explicit DG convection term,
    -(1/|T|) M^-1 ( surface integral of omega F.n  -  volume integral of grad(omega).F ),
    eqs. (Fu)-(Fw), with F_q = q v and the Rusanov flux. V is a list of d tensor arrays.

    nu > 0 adds the explicit viscous flux of the same equations (the explicit-viscosity
    variant, Section 2.2): F_q = q v - nu grad q with the broken gradient of each cell's
    polynomial at the nodes, the face flux averages the two sides' normal derivatives, and the
    Rusanov speed gains the viscous part 2 nu (2N+1) / (h_e sqrt(pi/2)) (reading: h_e is the
    mesh size normal to the face, as for the convective part). convection=False keeps only the
    viscous flux (unsteady Stokes)."""
    t = grid.tab
    n = grid.n
    w = t.w
    # Kv[k, m] = w_m phi_k'(xi_m) / w_k  (collocated volume term)
    Kv = t.dphi * w[None, :] / w[:, None]
    out = [np.zeros_like(V[c]) for c in range(grid.dim)]
    for e in range(grid.dim):                      # face / derivative direction
        ax = _ax(grid, e)
        nc = grid.cells[e]
        he = grid.h[e]
        ve = _split(V[e], ax, nc, n)
        vm = ve @ t.phi1                           # value at the right face of each cell
        vp = np.roll(ve @ t.phi0, -1, axis=-1)     # value of cell i+1 at its left face
        s = 2.0 * np.maximum(np.abs(vm), np.abs(vp)) if convection else np.zeros_like(vm)
        if nu:
            s = s + 2.0 * nu * (2 * grid.N + 1) / (he * np.sqrt(np.pi / 2.0))
        for c in range(grid.dim):                  # momentum component q = V[c]
            qe = _split(V[c], ax, nc, n)
            F = qe * ve if convection else np.zeros_like(qe)   # flux along e at the nodes
            if nu:
                F = F - nu * (qe @ t.dphi) / he    # - nu dq/dx_e at the nodes
            vol = F @ Kv.T / he                    # sum_m Kv[k,m] F[m]
            qm = qe @ t.phi1
            qp = np.roll(qe @ t.phi0, -1, axis=-1)
            Fhat = 0.5 * (qm * vm + qp * vp) * convection - 0.5 * s * (qp - qm)   # face i+1/2
            if nu:
                dqm = qe @ t.dphi1 / he                               # left cell, right face
                dqp = np.roll(qe @ t.dphi0, -1, axis=-1) / he         # right cell, left face
                Fhat = Fhat - 0.5 * nu * (dqm + dqp)
            Fhat_left = np.roll(Fhat, 1, axis=-1)                       # at face i-1/2
            surf = (Fhat[..., None] * t.phi1[None, :] - Fhat_left[..., None] * t.phi0[None, :]) \
                / w[None, :] / he
            out[c] = out[c] - _merge(surf - vol, ax)
    return out


def rk3(grid, V, dt, nu=0.0, convection=True):
    """Third-order TVD Runge-Kutta (Shu-Osher) for dV/dt = L(V) (nu > 0: with the explicit
    viscous flux)."""
    L0 = convective_rate(grid, V, nu, convection)
    V1 = [V[c] + dt * L0[c] for c in range(grid.dim)]
    L1 = convective_rate(grid, V1, nu, convection)
    V2 = [0.75 * V[c] + 0.25 * (V1[c] + dt * L1[c]) for c in range(grid.dim)]
    L2 = convective_rate(grid, V2, nu, convection)
    return [V[c] / 3.0 + 2.0 / 3.0 * (V2[c] + dt * L2[c]) for c in range(grid.dim)]


class StepOracle:
    """The fractional step with exact (fast-diagonalisation) linear solves."""

    def __init__(self, grid, dt, theta, nu):
        self.grid, self.dt, self.theta, self.nu = grid, float(dt), float(theta), float(nu)
        self.fd = FastDiag(grid)
        self.B = [div_rhs(grid, d) for d in range(grid.dim)]
        self.G = [grad_update(grid, d, dt) for d in range(grid.dim)]
        self._Ap = None
        self._Av = None

    @property
    def Ap(self):
        if self._Ap is None:
            self._Ap = pressure_operator(self.grid, self.dt)
        return self._Ap

    @property
    def Av(self):
        if self._Av is None:
            self._Av = viscous_operator(self.grid, self.dt, self.nu)
        return self._Av

    def rhs(self, Ustar):
        """b = sum_d B_d U*_d."""
        g = self.grid
        b = np.zeros(g.shape())
        for d in range(g.dim):
            b = b + (self.B[d] @ Ustar[d].reshape(-1)).reshape(g.shape())
        return b

    def solve_pressure(self, b):
        return self.fd.solve(b, 0.0, self.dt)

    def solve_viscous(self, rhs):
        return self.fd.solve(rhs, 1.0, self.nu * self.dt)

    def project_velocity(self, q, Ustar):
        g = self.grid
        return [Ustar[d] - (self.G[d] @ q.reshape(-1)).reshape(g.shape())
                for d in range(g.dim)]

    def step(self, U, P, convection=True, explicit_viscosity=False):
        """One step. U: list of dual components (tensor layout), P: P^n (tensor layout).
        Returns dict with U_new, P_new, q, b, Ustar, Umain (after viscosity), Fmain.

        explicit_viscosity: the variant of Section 2.2 in which the viscous flux is part of the
        explicit TVD-RK3 advection-diffusion step (eqs. Fu-Fw with the viscous Rusanov speed)
        and the implicit viscous solve is skipped."""
        g = self.grid
        w = g.tab.w
        Um = [dual_to_main(g, U[d], d) for d in range(g.dim)]
        if explicit_viscosity:
            Fm = rk3(g, Um, self.dt, self.nu, convection) if (convection or self.nu) else Um
            Us = [main_to_dual(g, Fm[d], d) for d in range(g.dim)]
            b = self.rhs(Us)
            q = self.solve_pressure(b)
            Un = self.project_velocity(q, Us)
            Pn = (q - (1.0 - self.theta) * P) / self.theta
            return dict(U_new=Un, P_new=Pn, q=q, b=b, Ustar=Us, Umain=Fm, Fmain=Fm, Um0=Um)
        Fm = rk3(g, Um, self.dt) if convection else Um
        # M^{xyz} as a tensor of nodal weights
        Wt = np.ones(g.shape())
        for d in range(g.dim):
            shp = [1] * g.dim
            shp[g.dim - 1 - d] = -1
            Wt = Wt * np.tile(w, g.cells[d]).reshape(shp)
        Uv = [self.solve_viscous(Wt * Fm[d]) for d in range(g.dim)]
        Us = [main_to_dual(g, Uv[d], d) for d in range(g.dim)]
        b = self.rhs(Us)
        q = self.solve_pressure(b)
        Un = self.project_velocity(q, Us)
        Pn = (q - (1.0 - self.theta) * P) / self.theta
        return dict(U_new=Un, P_new=Pn, q=q, b=b, Ustar=Us, Umain=Uv, Fmain=Fm, Um0=Um)


def kinetic_energy(grid, U):
    """(1/|Omega|) integral of |v|^2 / 2 over the domain, with each dual component integrated by
    GL quadrature on its own dual grid (the K of the 3D Taylor-Green subsection)."""
    w = grid.tab.w
    vol = np.prod(grid.lengths)
    cellvol = np.prod(grid.h)
    Wt = np.ones(grid.shape())
    for d in range(grid.dim):
        shp = [1] * grid.dim
        shp[grid.dim - 1 - d] = -1
        Wt = Wt * np.tile(w, grid.cells[d]).reshape(shp)
    return 0.5 * sum(float(np.sum(Wt * U[d] ** 2)) for d in range(grid.dim)) * cellvol / vol


def kinetic_energy_grad(grid, U):
    """Gradient of kinetic_energy with respect to each dual component (Euclidean, per DoF):
    (cell volume / domain volume) W U_d, the quadrature weights times the field."""
    w = grid.tab.w
    scale = float(np.prod(grid.h)) / float(np.prod(grid.lengths))
    Wt = np.ones(grid.shape())
    for d in range(grid.dim):
        shp = [1] * grid.dim
        shp[grid.dim - 1 - d] = -1
        Wt = Wt * np.tile(w, grid.cells[d]).reshape(shp)
    return [scale * Wt * U[d] for d in range(grid.dim)]


__all__ = ["Grid", "StepOracle", "dual_to_main", "main_to_dual", "convective_rate", "rk3",
           "kinetic_energy", "kinetic_energy_grad"]
