"""Space-time pressure correction with Picard iterations (test infrastructure only).

Follows Section 3 of arXiv:1602.05806 ("Spectral space-time DG schemes on staggered Cartesian
grids"): the solution on the slab [t^n, t^n + dt] is a polynomial of degree M in time on the
nodal Gauss-Legendre basis psi_0..psi_M of [0, 1]; the time-derivative term integrated by parts
with upwinding from the previous slab gives the time matrices of eqs. (tmatrix1)-(tmatrix3),
and the pressure correction of Section 3.3 (eqs. LOdiffusionU_HO-LOvelocityW_HO) iterates
k = 0..M.

Readings (where the printed equations are ambiguous):
  * The time basis is the nodal GL basis of degree M, so M^t = diag(omega) (mass in time).
  * M^t_0 acts on the previous slab's coefficients: (M^t_0 U^n)_p = psi_p(0) u(t^n), with u(t^n)
    the end value of the previous slab; a step therefore carries only that end value.
  * The system the iteration solves is the momentum equations (eq. uSDG1_ST) with the divergence
    condition (eq. pSDG1_ST) at every time node. Writing R for the right-hand side of the
    momentum equations before the time solve (R_p = pi_{#->*}(psi_p(0) F^n + dt omega_p
    L(U_p)) - omega_p G P^(k)_p), the predictor is Uhat = (M^t_1 - M^t_V)^-1 R. The pressure term
    is applied on the dual grid, where G and the velocity live: the pi_{*->#} of the pressure
    term in eq. (LOdiffusionU_HO) serves the main-grid viscous solve, which the covered variants
    (nu = 0, explicit viscosity, or M = 0 where P^(0) = 0) do not have. Requiring the corrected
    velocity Uhat - (M^t_1 - M^t_V)^-1 M^t G dP to be divergence free at every node gives the
    decoupled pressure systems omega_s A_p dP_s = sum_d B_d pi_{#->*}(R)_{d,s} (eqs. pSyst_ST2 /
    LOpressure_HO with their right-hand side read as the divergence of R; the printed
    eq. LOvelocityU_HO multiplies the predictor by M^t_0, which would not keep the divergence
    condition and is read as this correction).
  * The advective terms of the first iteration are those of the semi-implicit scheme at t^n
    (Fu^{n+1,(0)} = Fu^n, end of Section 3.3): F^n is U^n advected by the TVD-RK3 step of
    Section 2.2 (with the explicit viscous flux in the explicit-viscosity variant) and enters
    every node as psi_p(0) F^n. Later iterations use the space-time advective term of
    eq. (Fu_ST): R_p = psi_p(0) U^n + dt omega_p L(U^(k)_p) with the DG rate L evaluated at the
    time nodes of the current iterate.
  * Implicit viscosity with M >= 1 needs the non-symmetric space-time viscous solve of
    eq. (implicitviscosity_ST) and is not covered: M >= 1 takes nu = 0 or the explicit viscous
    flux. M = 0 with implicit viscosity is the semi-implicit step (the reduction stated at the
    end of Section 3.3).
  * P^{(0)} = 0 at every node; the step returns the pressure at the time nodes and the velocity
    at the slab end, u(t^{n+1}) = sum_s psi_s(1) U_s.
"""
import numpy as np
from numpy.polynomial.legendre import leggauss

from .basis import lagrange, lagrange_deriv
from .step import StepOracle, dual_to_main, main_to_dual, rk3, convective_rate


class TimeTables:
    """Time matrices of degree M (eqs. tmatrix1-tmatrix3), nodal GL basis on [0, 1]:
      tau, omega   nodes and weights (M^t = diag(omega))
      M1[p, q] = psi_p(1) psi_q(1)
      M0[p, q] = psi_p(0) psi_q(1)
      MV[p, q] = int_0^1 psi_p'(tau) psi_q(tau) dtau
      psi0, psi1   psi_p(0), psi_p(1)"""

    def __init__(self, M):
        if M < 0:
            raise ValueError("M >= 0")
        self.M = M
        m = M + 1
        x, w = leggauss(m)
        self.tau, self.omega = 0.5 * (x + 1.0), 0.5 * w
        qx, qw = leggauss(M + 3)
        qx, qw = 0.5 * (qx + 1.0), 0.5 * qw
        self.psi0 = np.array([lagrange(self.tau, p, 0.0) for p in range(m)], dtype=np.float64)
        self.psi1 = np.array([lagrange(self.tau, p, 1.0) for p in range(m)], dtype=np.float64)
        self.Mt = np.array([[np.sum(qw * lagrange(self.tau, p, qx) * lagrange(self.tau, q, qx))
                             for q in range(m)] for p in range(m)])
        self.M1 = np.outer(self.psi1, self.psi1)
        self.M0 = np.outer(self.psi0, self.psi1)
        self.MV = np.array([[np.sum(qw * lagrange_deriv(self.tau, p, qx) * lagrange(self.tau, q, qx))
                             for q in range(m)] for p in range(m)])
        self.At = self.M1 - self.MV


class SpaceTimeStepOracle:
    """One space-time step with M + 1 Picard iterations (exact fast-diagonalisation solves)."""

    def __init__(self, grid, dt, nu, M, explicit_viscosity=False):
        if M >= 1 and nu > 0 and not explicit_viscosity:
            raise ValueError("M >= 1 with implicit viscosity is not covered")
        self.grid, self.dt, self.nu, self.M = grid, float(dt), float(nu), int(M)
        self.explicit = bool(explicit_viscosity)
        self.tt = TimeTables(M)
        self.semi = StepOracle(grid, dt, 1.0, nu)

    def step(self, U, convection=True, iterations=None):
        """U: list of dual components at t^n (tensor layout). Returns dict with U_new (slab end),
        U_nodes (per time node, per component), P_nodes (pressure per time node) and the
        per-iteration divergence residuals."""
        g, tt, dt = self.grid, self.tt, self.dt
        so = self.semi
        m = self.M + 1
        K = m if iterations is None else iterations
        dim = g.dim
        Ainv = np.linalg.inv(tt.At)
        # F^n: the semi-implicit predictor's advected (and, with implicit viscosity, diffused)
        # main-grid velocity at t^n + dt
        Um0 = [dual_to_main(g, U[d], d) for d in range(dim)]
        if self.explicit:
            Fm = rk3(g, Um0, dt, self.nu, convection) if (convection or self.nu) else Um0
        else:
            Fm = rk3(g, Um0, dt) if convection else Um0
            if self.nu > 0:
                Wt = np.ones(g.shape())
                for d in range(dim):
                    shp = [1] * dim
                    shp[dim - 1 - d] = -1
                    Wt = Wt * np.tile(g.tab.w, g.cells[d]).reshape(shp)
                Fm = [so.solve_viscous(Wt * Fm[d]) for d in range(dim)]
        P = [np.zeros(g.shape()) for _ in range(m)]
        Ust = None                 # U*_s^(k), dual grid, per node
        div = []
        for k in range(K):
            # right-hand side R_p of the momentum equations (main grid), per node p
            if k == 0:
                R = [[tt.psi0[p] * Fm[d] for d in range(dim)] for p in range(m)]
            else:
                R = []
                for p in range(m):
                    Um = [dual_to_main(g, Ust[p][d], d) for d in range(dim)]
                    L = convective_rate(g, Um, self.nu if self.explicit else 0.0, convection)
                    R.append([tt.psi0[p] * Um0[d] + dt * tt.omega[p] * L[d] for d in range(dim)])
            # advective part back to the dual grids, and the pressure term of the current
            # iterate, - omega_p G_d P_p, where the velocity lives
            Rst = [[main_to_dual(g, R[p][d], d)
                    - tt.omega[p] * (so.G[d] @ P[p].reshape(-1)).reshape(g.shape())
                    for d in range(dim)] for p in range(m)]
            # predictor Uhat = At^-1 R (time solve per DoF)
            Uhat = [[sum(Ainv[s, p] * Rst[p][d] for p in range(m)) for d in range(dim)]
                    for s in range(m)]
            # decoupled pressure corrections omega_s A_p dP_s = sum_d B_d R*_{d,s}
            dP = [so.solve_pressure(so.rhs(Rst[s])) / tt.omega[s] for s in range(m)]
            # corrected velocity U = Uhat - At^-1 M^t G dP
            GdP = [[(so.G[d] @ dP[p].reshape(-1)).reshape(g.shape()) for d in range(dim)]
                   for p in range(m)]
            Ust = [[Uhat[s][d] - sum(Ainv[s, p] * tt.omega[p] * GdP[p][d] for p in range(m))
                    for d in range(dim)] for s in range(m)]
            P = [P[s] + dP[s] for s in range(m)]
            div.append(max(np.linalg.norm(so.rhs(Ust[s])) for s in range(m)))
        Unew = [sum(tt.psi1[s] * Ust[s][d] for s in range(m)) for d in range(dim)]
        return dict(U_new=Unew, U_nodes=Ust, P_nodes=P, divergence=div)


def momentum_residual(grid, tt, dt, nu, U0, Ust, P, convection=True, explicit=True):
    """Residual of the space-time momentum equations (eq. uSDG1_ST, dual grid, divided by the
    spatial mass) for node values Ust and pressures P: (At U)_p - psi_p(0) U^n - pi_{#->*}(dt
    omega_p L(pi_{*->#} U_p)) + omega_p G P_p. Zero at the fixed point of the Picard iteration
    when the advective term is the space-time one of eq. (Fu_ST) at every node."""
    from .operators import grad_update
    dim = grid.dim
    m = tt.M + 1
    G = [grad_update(grid, d, dt) for d in range(dim)]
    out = []
    for p in range(m):
        Um = [dual_to_main(grid, Ust[p][d], d) for d in range(dim)]
        L = convective_rate(grid, Um, nu if explicit else 0.0, convection)
        Um0 = [dual_to_main(grid, U0[d], d) for d in range(dim)]
        res = []
        for d in range(dim):
            lhs = sum(tt.At[p, q] * Ust[q][d] for q in range(m))
            adv = main_to_dual(grid, tt.psi0[p] * Um0[d] + dt * tt.omega[p] * L[d], d)
            res.append(lhs - adv + tt.omega[p] * (G[d] @ P[p].reshape(-1)).reshape(grid.shape()))
        out.append(res)
    return out


__all__ = ["TimeTables", "SpaceTimeStepOracle", "momentum_residual"]
