"""Pins of the oracle's hand-written adjoint: each linearisation against central finite
differences of the oracle's forward map, each transpose against its linearisation through the
identity <J dV, Y> = <dV, J^T Y>, and the whole step and a short rollout against finite
differences of the kinetic energy."""
import numpy as np
import pytest

from oracle.operators import Grid
from oracle.step import convective_rate, rk3, StepOracle, kinetic_energy
from oracle.adjoint import (convective_jvp, convective_vjp, rk3_jvp, rk3_vjp, StepAdjoint,
                            rollout_gradient, dual_to_main_T, main_to_dual_T)
from oracle.step import dual_to_main, main_to_dual

CASES = [((5, 4), (1.0, 0.8), 3), ((6, 3), (1.0, 1.0), 2), ((3, 4, 3), (1.0, 1.0, 1.2), 2),
         ((4, 3, 3), (1.0, 1.0, 1.0), 1)]


def rand_fields(grid, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return [scale * rng.standard_normal(grid.shape()) for _ in range(grid.dim)]


def dot(A, B):
    return sum(float(np.sum(a * b)) for a, b in zip(A, B))


def axpy(a, X, Y):
    return [a * x + y for x, y in zip(X, Y)]


@pytest.mark.parametrize("cells,lengths,N", CASES)
def test_convective_jvp_matches_finite_differences(cells, lengths, N):
    g = Grid(cells, lengths, N)
    V = rand_fields(g, 1)
    dV = rand_fields(g, 2)
    eps = 1e-6
    Lp = convective_rate(g, axpy(eps, dV, V))
    Lm = convective_rate(g, axpy(-eps, dV, V))
    fd = [(p - m) / (2 * eps) for p, m in zip(Lp, Lm)]
    J = convective_jvp(g, V, dV)
    num = np.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(J, fd)))
    den = np.sqrt(sum(np.sum(a ** 2) for a in fd))
    assert num <= 1e-7 * den


@pytest.mark.parametrize("cells,lengths,N", CASES)
def test_convective_vjp_is_the_transpose(cells, lengths, N):
    g = Grid(cells, lengths, N)
    V = rand_fields(g, 3)
    dV = rand_fields(g, 4)
    Y = rand_fields(g, 5)
    lhs = dot(convective_jvp(g, V, dV), Y)
    rhs = dot(dV, convective_vjp(g, V, Y))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("cells,lengths,N", CASES[:3])
def test_rk3_jvp_and_vjp(cells, lengths, N):
    g = Grid(cells, lengths, N)
    V = rand_fields(g, 8, 0.3)
    dV = rand_fields(g, 9)
    Y = rand_fields(g, 10)
    dt = 1e-2
    eps = 1e-6
    fd = [(p - m) / (2 * eps) for p, m in zip(rk3(g, axpy(eps, dV, V), dt),
                                              rk3(g, axpy(-eps, dV, V), dt))]
    J = rk3_jvp(g, V, dt, dV)
    num = np.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(J, fd)))
    assert num <= 1e-7 * np.sqrt(sum(np.sum(a ** 2) for a in fd))
    lhs = dot(J, Y)
    rhs = dot(dV, rk3_vjp(g, V, dt, Y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("cells,lengths,N", [((4, 3), (1.0, 1.0), 2), ((5, 4), (1.0, 0.9), 3),
                                             ((3, 3, 2), (1.0, 1.0, 1.0), 1)])
def test_projection_transposes(cells, lengths, N):
    g = Grid(cells, lengths, N)
    X = rand_fields(g, 11)
    Y = rand_fields(g, 12)
    for d in range(g.dim):
        assert abs(np.sum(dual_to_main(g, X[d], d) * Y[d]) -
                   np.sum(X[d] * dual_to_main_T(g, Y[d], d))) <= 1e-12 * np.abs(X[d]).sum()
        assert abs(np.sum(main_to_dual(g, X[d], d) * Y[d]) -
                   np.sum(X[d] * main_to_dual_T(g, Y[d], d))) <= 1e-12 * np.abs(X[d]).sum()


@pytest.mark.parametrize("convection", [True, False])
@pytest.mark.parametrize("cells,lengths,N", [((4, 3), (1.0, 1.0), 2), ((5, 4), (1.0, 0.9), 3),
                                             ((3, 3, 2), (1.0, 1.0, 1.0), 1)])
def test_step_vjp_matches_finite_differences(cells, lengths, N, convection):
    g = Grid(cells, lengths, N)
    dt, theta, nu = 2e-3, 0.6, 1e-2
    adj = StepAdjoint(g, dt, theta, nu)
    U = rand_fields(g, 13, 0.5)
    dU = rand_fields(g, 14)
    Ubar = rand_fields(g, 15)
    P = np.zeros(g.shape())
    eps = 1e-6
    up = adj.fwd.step(axpy(eps, dU, U), P, convection=convection)["U_new"]
    um = adj.fwd.step(axpy(-eps, dU, U), P, convection=convection)["U_new"]
    fd = (dot(up, Ubar) - dot(um, Ubar)) / (2 * eps)
    got = dot(dU, adj.vjp(U, Ubar, convection=convection))
    assert abs(got - fd) <= 1e-7 * max(abs(fd), 1e-30)


def test_rollout_gradient_matches_finite_differences():
    g = Grid((4, 4), (1.0, 1.0), 2)
    dt, theta, nu = 2e-3, 0.6, 1e-2
    U0 = rand_fields(g, 16, 0.5)
    loss, grad = rollout_gradient(g, U0, 3, dt, theta, nu)
    step = StepOracle(g, dt, theta, nu)

    def rollout(U):
        P = np.zeros(g.shape())
        for _ in range(3):
            r = step.step(U, P)
            U, P = r["U_new"], r["P_new"]
        return kinetic_energy(g, U)

    assert abs(rollout(U0) - loss) <= 1e-15 * abs(loss) + 1e-300
    rng = np.random.default_rng(17)
    for _ in range(3):
        v = [rng.standard_normal(g.shape()) for _ in range(g.dim)]
        eps = 1e-6 * np.sqrt(dot(U0, U0)) / np.sqrt(dot(v, v))
        fd = (rollout(axpy(eps, v, U0)) - rollout(axpy(-eps, v, U0))) / (2 * eps)
        assert abs(dot(grad, v) - fd) <= 1e-6 * abs(fd)
