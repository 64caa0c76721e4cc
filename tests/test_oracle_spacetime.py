"""Pins of the space-time oracle (Section 3 of arXiv:1602.05806): the time matrices of
eqs. (tmatrix1)-(tmatrix3) against the paper's M = 0 statement, integration by parts and the
closed-form stability function of DG in time; the Picard pressure correction of Section 3.3
against the semi-implicit step (M = 0), the divergence condition at every time node, and the
space-time momentum equations at the fixed point of the iteration."""
from math import factorial

import numpy as np
import pytest

from oracle.operators import Grid
from oracle.spacetime import TimeTables, SpaceTimeStepOracle, momentum_residual
from oracle.step import StepOracle
import synthetic


def test_time_tables_degenerate_M0():
    """End of Section 3.3: for M = 0 the time matrices are M1 = 1, M0 = 1, MV = 0 (and M^t = 1)."""
    t = TimeTables(0)
    assert np.allclose(t.M1, [[1.0]], atol=1e-15) and np.allclose(t.M0, [[1.0]], atol=1e-15)
    assert np.allclose(t.MV, [[0.0]], atol=1e-15) and np.allclose(t.Mt, [[1.0]], atol=1e-15)


@pytest.mark.parametrize("M", range(0, 6))
def test_time_tables_identities(M):
    """eqs. (tmatrix1)-(tmatrix3): integration by parts in time gives MV + MV^T = psi(1) psi(1)^T
    - psi(0) psi(0)^T; the nodal GL basis makes M^t = diag(omega); M1 = psi(1) psi(1)^T and
    M0 = psi(0) psi(1)^T are rank one."""
    t = TimeTables(M)
    assert np.abs(t.MV + t.MV.T - (np.outer(t.psi1, t.psi1) - np.outer(t.psi0, t.psi0))).max() <= 1e-13
    assert np.abs(t.Mt - np.diag(t.omega)).max() <= 1e-14
    assert abs(t.omega.sum() - 1.0) <= 1e-15
    assert np.linalg.matrix_rank(t.M1) == 1 and np.linalg.matrix_rank(t.M0) == 1


def pade(M, z):
    """(M, M+1) Pade approximant of exp(z): the stability function of DG in time of degree M."""
    num = sum(factorial(2 * M + 1 - j) * factorial(M) /
              (factorial(2 * M + 1) * factorial(j) * factorial(M - j)) * z ** j for j in range(M + 1))
    den = sum(factorial(2 * M + 1 - j) * factorial(M + 1) /
              (factorial(2 * M + 1) * factorial(j) * factorial(M + 1 - j)) * (-z) ** j
              for j in range(M + 2))
    return num / den


@pytest.mark.parametrize("M", range(0, 5))
def test_dg_in_time_stability_function(M):
    """For u' = lambda u the slab equations ((M1 - MV) - z M^t) U = M0 U^n (z = lambda dt,
    upwinding from the previous slab) give u(t^{n+1}) = R(z) u(t^n) with R the (M, M+1) Pade
    approximant of exp(z), the classical result for DG in time (M = 0: backward Euler,
    1 / (1 - z))."""
    t = TimeTables(M)
    for z in (-0.3, -1.7, 0.4, -12.0):
        U = np.linalg.solve(t.At - z * t.Mt, t.M0 @ np.ones(M + 1))
        assert abs(t.psi1 @ U - pade(M, z)) <= 1e-12 * max(1.0, abs(pade(M, z)))


def _field(g, seed=3, kmax=3, vmax=0.5):
    co = synthetic.staggered_coords(g.cells, g.lengths, g.tab.xi)
    return synthetic.FourierField(seed, g.dim, kmax, g.lengths).normalise(vmax).eval(co)


@pytest.mark.parametrize("cells,N", [((8, 6), 3), ((4, 3, 4), 2)])
def test_spacetime_M0_is_the_semi_implicit_step(cells, N):
    """End of Section 3.3: with M = 0 the space-time scheme collapses to the semi-implicit scheme
    (here with implicit viscosity, convection on; the pressure is P^{n+1}, i.e. theta = 1)."""
    g = Grid(cells, (1.0,) * len(cells), N)
    U = _field(g)
    dt, nu = 2e-3, 1e-2
    r = SpaceTimeStepOracle(g, dt, nu, 0).step(U)
    ref = StepOracle(g, dt, 1.0, nu).step(U, np.zeros(g.shape()))
    for d in range(g.dim):
        assert np.abs(r["U_new"][d] - ref["U_new"][d]).max() <= 1e-13 * np.abs(ref["U_new"][d]).max()
    assert np.abs(r["P_nodes"][0] - ref["P_new"]).max() <= 1e-12 * np.abs(ref["P_new"]).max()


@pytest.mark.parametrize("M", [1, 2, 3])
def test_spacetime_picard_divergence_and_fixed_point(M):
    """Every Picard iterate is discretely divergence free at every time node (eq. pSDG1_ST), and
    the iteration converges to a solution of the space-time momentum equations (eq. uSDG1_ST with
    the advective term of eq. Fu_ST at every node): the momentum residual falls with each
    iteration and vanishes to rounding at the fixed point."""
    g = Grid((8, 6), (1.0, 1.0), 3)
    U = _field(g)
    dt, nu = 2e-3, 1e-2
    st = SpaceTimeStepOracle(g, dt, nu, M, explicit_viscosity=True)
    scale = max(np.abs(u).max() for u in U)
    res = []
    for K in (M + 1, 8, 30):
        r = st.step(U, iterations=K)
        assert max(r["divergence"]) <= 1e-12 * scale
        rr = momentum_residual(g, st.tt, dt, nu, U, r["U_nodes"], r["P_nodes"])
        res.append(max(np.abs(x).max() for p in rr for x in p))
    assert res[0] > res[1] > res[2]
    assert res[2] <= 1e-14 * scale


def test_spacetime_M_requires_explicit_viscosity():
    g = Grid((4, 4), (1.0, 1.0), 2)
    with pytest.raises(ValueError):
        SpaceTimeStepOracle(g, 1e-3, 1e-2, 1)
