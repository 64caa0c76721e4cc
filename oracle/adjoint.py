"""Adjoint of the fractional step (test infrastructure only).

The step of step.py maps the dual velocity U^n to U^{n+1} through
  pi_{*->#}  ->  TVD-RK3 convection  ->  viscous solve  ->  pi_{#->*}  ->  pressure projection.
Every stage but the convection is linear, and its transpose is the transpose of the oracle's own
matrices: the pressure and viscous operators are symmetric, so their inverses are their own
adjoints (the pressure pseudo-inverse included), and the L2 projections, B_d and G_d are
transposed as sparse matrices. The convective residual of eqs. (Fu)-(Fw) is nonlinear; its
linearisation is written out by hand below, with the Rusanov speed s = 2 max(|v^-|, |v^+|)
differentiated on the branch taken by the forward state (|v^-| >= |v^+| selects v^-), and its
transpose is written out operation by operation in reverse.

Loss convention for gradients: the kinetic energy of step.kinetic_energy, whose gradient with
respect to the dual component U_d is (cell volume / domain volume) W U_d (W: GL weights).
"""
import numpy as np

from .operators import apply_along, l2_dual_to_main_1d, l2_main_to_dual_1d
from .step import (StepOracle, dual_to_main, main_to_dual, convective_rate, kinetic_energy,
                   kinetic_energy_grad)


def _ax(grid, d):
    return grid.dim - 1 - d


def _split(X, axis, nc, n):
    Xm = np.moveaxis(X, axis, -1)
    return Xm.reshape(Xm.shape[:-1] + (nc, n))


def _merge(Xs, axis):
    Xm = Xs.reshape(Xs.shape[:-2] + (-1,))
    return np.moveaxis(Xm, -1, axis)


def _faces(t, ve):
    """Face values along the split axis: v^- (cell i at its right face), v^+ (cell i+1 at its
    left face), for the face i+1/2."""
    vm = ve @ t.phi1
    vp = np.roll(ve @ t.phi0, -1, axis=-1)
    return vm, vp


def convective_jvp(grid, V, dV):
    """Directional derivative dL(V)[dV] of step.convective_rate (lists of d tensor arrays)."""
    t = grid.tab
    n = grid.n
    w = t.w
    Kv = t.dphi * w[None, :] / w[:, None]
    out = [np.zeros_like(V[c]) for c in range(grid.dim)]
    for e in range(grid.dim):
        ax = _ax(grid, e)
        nc = grid.cells[e]
        he = grid.h[e]
        ve = _split(V[e], ax, nc, n)
        dve = _split(dV[e], ax, nc, n)
        vm, vp = _faces(t, ve)
        dvm, dvp = _faces(t, dve)
        s = 2.0 * np.maximum(np.abs(vm), np.abs(vp))
        use_m = np.abs(vm) >= np.abs(vp)
        a = np.where(use_m, vm, vp)
        ds = 2.0 * np.sign(a) * np.where(use_m, dvm, dvp)
        for c in range(grid.dim):
            qe = _split(V[c], ax, nc, n)
            dqe = _split(dV[c], ax, nc, n)
            dF = dqe * ve + qe * dve
            dvol = dF @ Kv.T / he
            qm, qp = _faces(t, qe)
            dqm, dqp = _faces(t, dqe)
            dFhat = 0.5 * (dqm * vm + qm * dvm + dqp * vp + qp * dvp) \
                - 0.5 * ds * (qp - qm) - 0.5 * s * (dqp - dqm)
            dFhat_left = np.roll(dFhat, 1, axis=-1)
            dsurf = (dFhat[..., None] * t.phi1[None, :] - dFhat_left[..., None] * t.phi0[None, :]) \
                / w[None, :] / he
            out[c] = out[c] - _merge(dsurf - dvol, ax)
    return out


def convective_vjp(grid, V, Ybar):
    """Transpose of convective_jvp at V applied to the cotangents Ybar (one per component)."""
    t = grid.tab
    n = grid.n
    w = t.w
    Kv = t.dphi * w[None, :] / w[:, None]
    Vbar = [np.zeros_like(V[c]) for c in range(grid.dim)]
    for e in range(grid.dim):
        ax = _ax(grid, e)
        nc = grid.cells[e]
        he = grid.h[e]
        ve = _split(V[e], ax, nc, n)
        vm, vp = _faces(t, ve)
        s = 2.0 * np.maximum(np.abs(vm), np.abs(vp))
        use_m = np.abs(vm) >= np.abs(vp)
        a = np.where(use_m, vm, vp)
        ve_bar = np.zeros_like(ve)
        for c in range(grid.dim):
            qe = _split(V[c], ax, nc, n)
            Y = _split(Ybar[c], ax, nc, n)
            # out[c] -= (surf - vol)
            surf_bar = -Y
            vol_bar = Y
            # vol[k] = sum_m Kv[k, m] F[m] / he
            F_bar = vol_bar @ Kv / he
            # surf[i, k] = (Fhat[i] phi1[k] - Fhat[i-1] phi0[k]) / (w[k] he)
            Fhat_bar = (surf_bar * (t.phi1 / w)[None, :]).sum(-1) / he
            Fleft_bar = -(surf_bar * (t.phi0 / w)[None, :]).sum(-1) / he
            Fhat_bar = Fhat_bar + np.roll(Fleft_bar, -1, axis=-1)
            # Fhat = 0.5 (qm vm + qp vp) - 0.5 s (qp - qm)
            qm, qp = _faces(t, qe)
            qm_bar = Fhat_bar * (0.5 * vm + 0.5 * s)
            qp_bar = Fhat_bar * (0.5 * vp - 0.5 * s)
            vm_bar = Fhat_bar * 0.5 * qm
            vp_bar = Fhat_bar * 0.5 * qp
            s_bar = -0.5 * Fhat_bar * (qp - qm)
            a_bar = 2.0 * np.sign(a) * s_bar
            vm_bar = vm_bar + np.where(use_m, a_bar, 0.0)
            vp_bar = vp_bar + np.where(use_m, 0.0, a_bar)
            # face values back to the nodes (qp, vp belong to cell i+1)
            qe_bar = qm_bar[..., None] * t.phi1[None, :] \
                + np.roll(qp_bar, 1, axis=-1)[..., None] * t.phi0[None, :]
            ve_bar = ve_bar + vm_bar[..., None] * t.phi1[None, :] \
                + np.roll(vp_bar, 1, axis=-1)[..., None] * t.phi0[None, :]
            # F = q v at the nodes
            qe_bar = qe_bar + F_bar * ve
            ve_bar = ve_bar + F_bar * qe
            Vbar[c] = Vbar[c] + _merge(qe_bar, ax)
        Vbar[e] = Vbar[e] + _merge(ve_bar, ax)
    return Vbar


def rk3_stages(grid, V, dt):
    """The stage inputs V0, V1, V2 of step.rk3 (Shu-Osher)."""
    L0 = convective_rate(grid, V)
    V1 = [V[c] + dt * L0[c] for c in range(grid.dim)]
    L1 = convective_rate(grid, V1)
    V2 = [0.75 * V[c] + 0.25 * (V1[c] + dt * L1[c]) for c in range(grid.dim)]
    return V, V1, V2


def rk3_jvp(grid, V, dt, dV):
    """Directional derivative of step.rk3 at V."""
    V0, V1, V2 = rk3_stages(grid, V, dt)
    J0 = convective_jvp(grid, V0, dV)
    dV1 = [dV[c] + dt * J0[c] for c in range(grid.dim)]
    J1 = convective_jvp(grid, V1, dV1)
    dV2 = [0.75 * dV[c] + 0.25 * (dV1[c] + dt * J1[c]) for c in range(grid.dim)]
    J2 = convective_jvp(grid, V2, dV2)
    return [dV[c] / 3.0 + 2.0 / 3.0 * (dV2[c] + dt * J2[c]) for c in range(grid.dim)]


def rk3_vjp(grid, V, dt, Ubar):
    """Transpose of rk3_jvp at V: the stages in reverse order."""
    V0, V1, V2 = rk3_stages(grid, V, dt)
    dim = grid.dim
    # U3 = V0/3 + 2/3 (V2 + dt L(V2))
    J2 = convective_vjp(grid, V2, Ubar)
    V2bar = [2.0 / 3.0 * (Ubar[c] + dt * J2[c]) for c in range(dim)]
    V0bar = [Ubar[c] / 3.0 for c in range(dim)]
    # V2 = 3/4 V0 + 1/4 (V1 + dt L(V1))
    J1 = convective_vjp(grid, V1, V2bar)
    V1bar = [0.25 * (V2bar[c] + dt * J1[c]) for c in range(dim)]
    V0bar = [V0bar[c] + 0.75 * V2bar[c] for c in range(dim)]
    # V1 = V0 + dt L(V0)
    J0 = convective_vjp(grid, V0, V1bar)
    return [V0bar[c] + V1bar[c] + dt * J0[c] for c in range(dim)]


def dual_to_main_T(grid, X, d):
    """Transpose of step.dual_to_main for component d (main -> dual)."""
    return apply_along(l2_dual_to_main_1d(grid.cells[d], grid.N).T.tocsr(), X, _ax(grid, d))


def main_to_dual_T(grid, X, d):
    """Transpose of step.main_to_dual for component d (dual -> main)."""
    return apply_along(l2_main_to_dual_1d(grid.cells[d], grid.N).T.tocsr(), X, _ax(grid, d))


def weights_tensor(grid):
    """Tensor of the products of GL weights (the diagonal of M^{xyz})."""
    w = grid.tab.w
    Wt = np.ones(grid.shape())
    for d in range(grid.dim):
        shp = [1] * grid.dim
        shp[grid.dim - 1 - d] = -1
        Wt = Wt * np.tile(w, grid.cells[d]).reshape(shp)
    return Wt


class StepAdjoint:
    """Transposed linearisation of StepOracle.step with respect to the velocity."""

    def __init__(self, grid, dt, theta, nu):
        self.fwd = StepOracle(grid, dt, theta, nu)
        self.grid = grid
        self.dt = float(dt)
        self.nu = float(nu)
        self.Wt = weights_tensor(grid)

    def vjp(self, U, Ubar, convection=True):
        """Given U^n (dual components) and the cotangent Ubar of U^{n+1}, return the cotangent
        of U^n. The pressure P^n does not enter U^{n+1}."""
        g = self.grid
        dim = g.dim
        f = self.fwd
        shp = g.shape()
        # U^{n+1}_d = U*_d - G_d q,  q = A_p^+ b,  b = sum_d B_d U*_d
        qbar = np.zeros(shp)
        for d in range(dim):
            qbar = qbar - (f.G[d].T @ Ubar[d].reshape(-1)).reshape(shp)
        bbar = f.fd.solve(qbar, 0.0, self.dt)
        Usbar = [Ubar[d] + (f.B[d].T @ bbar.reshape(-1)).reshape(shp) for d in range(dim)]
        # U*_d = pi_{#->*} U#_d;  U#_d = A_v^-1 W F_d
        Uvbar = [main_to_dual_T(g, Usbar[d], d) for d in range(dim)]
        Fbar = [self.Wt * f.fd.solve(Uvbar[d], 1.0, self.nu * self.dt) for d in range(dim)]
        # F = RK3(Um0), Um0_d = pi_{*->#} U_d
        if convection:
            Um0 = [dual_to_main(g, U[d], d) for d in range(dim)]
            Um0bar = rk3_vjp(g, Um0, self.dt, Fbar)
        else:
            Um0bar = Fbar
        return [dual_to_main_T(g, Um0bar[d], d) for d in range(dim)]


def rollout_gradient(grid, U0, steps, dt, theta, nu, convection=True):
    """Kinetic energy after `steps` fractional steps from U0 and its gradient with respect to
    U0 (all states kept: the oracle needs no checkpointing)."""
    adj = StepAdjoint(grid, dt, theta, nu)
    states = [U0]
    P = np.zeros(grid.shape())
    U = U0
    for _ in range(steps):
        r = adj.fwd.step(U, P, convection=convection)
        U, P = r["U_new"], r["P_new"]
        states.append(U)
    loss = kinetic_energy(grid, U)
    Ubar = kinetic_energy_grad(grid, U)
    for n in range(steps - 1, -1, -1):
        Ubar = adj.vjp(states[n], Ubar, convection=convection)
    return loss, Ubar
