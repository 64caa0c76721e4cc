"""GPU parity of the space-time step (Section 3: time matrices of eqs. tmatrix1-tmatrix3, Picard
pressure correction of Section 3.3) against the oracle's space-time step with exact solves, the
M = 0 reduction to the semi-implicit step, the divergence condition at the slab end, and the
rejected configurations.

Every case prints its parameters before touching the GPU so that a failure names its case."""
import numpy as np
import pytest

from oracle import layout
from oracle.operators import Grid
from oracle.spacetime import SpaceTimeStepOracle
import synthetic

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def mass_norm(g, T):
    W = np.ones(g.shape())
    for d in range(g.dim):
        shp = [1] * g.dim
        shp[g.dim - 1 - d] = -1
        W = W * np.tile(g.tab.w, g.cells[d]).reshape(shp)
    return np.sqrt(np.sum(W * T ** 2))


def field(g, seed=3, kmax=3, vmax=0.5):
    co = synthetic.staggered_coords(g.cells, g.lengths, g.tab.xi)
    return synthetic.FourierField(seed, g.dim, kmax, g.lengths).normalise(vmax).eval(co)


@pytest.mark.parametrize("dim,cells,N", [(2, (8, 6), 3), (3, (4, 3, 4), 2)])
def test_step_st_M0_equals_semi_implicit_step(pd, dim, cells, N):
    """M = 0 is the semi-implicit step (theta = 1) with implicit viscosity and convection."""
    import torch
    print(f"space-time M=0 vs pd_step dim={dim} cells={cells} N={N}", flush=True)
    L = (1.0,) * dim
    dt, nu = 2e-3, 1e-2
    g = Grid(cells, L, N)
    U = [layout.tensor_to_blocked(x, cells, g.n) for x in field(g)]
    ctx = pd.pd_setup(dim, cells, L, N, dt, 1.0, nu)
    pd.pd_configure(ctx, pd.PD_CFG_P_RTOL, 1e-12)
    a = [dev(x) for x in U]
    b = [dev(x) for x in U]
    p = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    pn = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    pd.pd_step(ctx, a, p)
    infos = pd.pd_step_st(ctx, 0, b, pn)
    assert infos[3]["status"] == pd.PD_OK and infos[3]["iters"] > 0
    for d in range(dim):
        assert np.abs(host(a[d]) - host(b[d])).max() <= 1e-14 * np.abs(host(a[d])).max()
    assert np.abs(host(p) - host(pn)).max() <= 1e-13 * np.abs(host(p)).max()
    ctx.close()


@pytest.mark.parametrize("dim,cells,N,M,conv", [(2, (8, 6), 3, 1, 1), (2, (7, 5), 2, 2, 1),
                                                (2, (6, 6), 4, 3, 0), (3, (4, 3, 4), 2, 1, 1),
                                                (3, (3, 4, 3), 3, 2, 1)])
def test_step_st_matches_oracle(pd, dim, cells, N, M, conv):
    """M + 1 Picard iterations with the explicit viscous flux: end velocity and the pressure at
    every time node against the oracle's space-time step with exact solves."""
    import torch
    print(f"space-time dim={dim} cells={cells} N={N} M={M} conv={conv}", flush=True)
    L = (1.0, 0.9, 1.1)[:dim]
    dt, nu = 1e-3, 5e-3
    g = Grid(cells, L, N)
    Ut = field(g)
    ref = SpaceTimeStepOracle(g, dt, nu, M, explicit_viscosity=True).step(Ut, convection=bool(conv))
    ctx = pd.pd_setup(dim, cells, L, N, dt, 1.0, nu)
    pd.pd_configure(ctx, pd.PD_CFG_EXPLICIT_VISC, 1)
    pd.pd_configure(ctx, pd.PD_CFG_CONVECTION, conv)
    pd.pd_configure(ctx, pd.PD_CFG_P_RTOL, 1e-13)
    u = [dev(layout.tensor_to_blocked(x, cells, g.n)) for x in Ut]
    pn = torch.zeros((M + 1) * g.ndof, dtype=torch.float64, device="cuda")
    infos = pd.pd_step_st(ctx, M, u, pn)
    assert all(i["status"] == pd.PD_OK for i in infos[3:])
    for d in range(dim):
        got = layout.blocked_to_tensor(host(u[d]), cells, g.n)
        assert mass_norm(g, got - ref["U_new"][d]) <= 1e-10 * mass_norm(g, ref["U_new"][d])
    ph = host(pn).reshape(M + 1, g.ndof)
    for s in range(M + 1):
        got = layout.blocked_to_tensor(ph[s], cells, g.n)
        assert mass_norm(g, got - ref["P_nodes"][s]) <= 1e-9 * mass_norm(g, ref["P_nodes"][s])
    # the end value is a combination of divergence-free node values
    b = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
    pd.pd_rhs_div(ctx, u, b)
    b0 = torch.empty_like(b)
    pd.pd_rhs_div(ctx, [dev(layout.tensor_to_blocked(x, cells, g.n)) for x in Ut], b0)
    assert float(b.norm()) <= 1e-11 * float(b0.norm())
    ctx.close()


def test_step_st_rejected_configurations(pd):
    import torch
    print("space-time rejected configurations", flush=True)
    cells, N = (6, 5), 2
    ctx = pd.pd_setup(2, cells, (1.0, 1.0), N, 1e-3, 1.0, 1e-2)
    u = [torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda") for _ in range(2)]
    pn = torch.zeros(2 * ctx.ndof, dtype=torch.float64, device="cuda")
    with pytest.raises(pd.PdError):          # M >= 1 with implicit viscosity
        pd.pd_step_st(ctx, 1, u, pn)
    with pytest.raises(pd.PdError):          # M beyond 4
        pd.pd_step_st(ctx, 5, u, torch.zeros(6 * ctx.ndof, dtype=torch.float64, device="cuda"))
    pd.pd_configure(ctx, pd.PD_CFG_EXPLICIT_VISC, 1)
    infos = pd.pd_step_st(ctx, 1, u, pn)     # zero velocity: zero right-hand sides
    assert all(i["status"] == pd.PD_OK for i in infos[3:])
    ctx.close()
