"""GPU parity of the explicit-viscosity variant (Section 2.2): the viscous flux -nu grad q with
the viscous Rusanov speed inside the explicit TVD-RK3 step (pd_convect with
PD_CFG_EXPLICIT_VISC), the step that skips the implicit viscous solve, and the viscous CFL check.

Every case prints its parameters before touching the GPU so that a failure names its case."""
import numpy as np
import pytest

from oracle import layout
from oracle.operators import Grid
from oracle.step import StepOracle, rk3
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


@pytest.mark.parametrize("dim,cells,N,conv", [(2, (6, 5), 3, 1), (2, (7, 4), 6, 0),
                                              (2, (5, 5), 0, 1), (3, (4, 3, 5), 2, 1),
                                              (3, (3, 4, 3), 4, 0)])
def test_convect_with_explicit_viscosity(pd, dim, cells, N, conv):
    """One RK3 step of the convective + explicit viscous rate against the oracle element by
    element (convection on and off)."""
    print(f"explicit viscosity convect dim={dim} cells={cells} N={N} conv={conv}", flush=True)
    L = (1.0, 0.8, 1.2)[:dim]
    dt, nu = 1e-4, 2e-3
    g = Grid(cells, L, N)
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, nu)
    pd.pd_configure(ctx, pd.PD_CFG_EXPLICIT_VISC, 1)
    pd.pd_configure(ctx, pd.PD_CFG_CONVECTION, conv)
    rng = np.random.default_rng(40 + N)
    V = [0.3 * rng.standard_normal(g.ndof) for _ in range(dim)]
    Vt = [layout.blocked_to_tensor(v, cells, g.n) for v in V]
    ref = rk3(g, Vt, dt, nu, bool(conv))
    vd = [dev(v) for v in V]
    pd.pd_convect(ctx, vd)
    for d in range(dim):
        r = layout.tensor_to_blocked(ref[d], cells, g.n)
        assert np.abs(host(vd[d]) - r).max() <= 1e-13 * np.abs(r).max()
    with pytest.raises(pd.PdError):
        pd.pd_convect_adjoint(ctx, vd, [v.clone() for v in vd])
    ctx.close()


@pytest.mark.parametrize("conv", [1, 0])
def test_step_explicit_viscosity_taylor_green(pd, conv):
    """Fractional steps of the explicit-viscosity variant on the 16^2 N = 3 Taylor-Green field
    against the oracle step with exact pressure solves (5 steps)."""
    import torch
    cells, N, dt, nu = (16, 16), 3, 2e-4, 5e-2
    print(f"explicit viscosity step tgv cells={cells} N={N} conv={conv}", flush=True)
    g = Grid(cells, (1.0, 1.0), N)
    so = StepOracle(g, dt, 0.6, nu)
    co = synthetic.staggered_coords(cells, g.lengths, g.tab.xi)
    Ut = synthetic.tgv2d([(co[0][0], co[0][1]), (co[1][0], co[1][1])])
    ctx = pd.pd_setup(2, cells, (1.0, 1.0), N, dt, 0.6, nu)
    pd.pd_configure(ctx, pd.PD_CFG_EXPLICIT_VISC, 1)
    pd.pd_configure(ctx, pd.PD_CFG_CONVECTION, conv)
    pd.pd_configure(ctx, pd.PD_CFG_P_RTOL, 1e-13)
    ud = [dev(layout.tensor_to_blocked(u, cells, g.n)) for u in Ut]
    p = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    P = np.zeros(g.shape())
    for _ in range(5):
        r = so.step(Ut, P, convection=bool(conv), explicit_viscosity=True)
        Ut, P = r["U_new"], r["P_new"]
        infos = pd.pd_step(ctx, ud, p)
        assert infos[3]["status"] == pd.PD_OK and infos[0]["iters"] == 0
    for d in range(2):
        got = layout.blocked_to_tensor(host(ud[d]), cells, g.n)
        assert mass_norm(g, got - Ut[d]) <= 1e-10 * mass_norm(g, Ut[d])
    got_p = layout.blocked_to_tensor(host(p), cells, g.n)
    assert mass_norm(g, got_p - P) <= 1e-8 * mass_norm(g, P)
    ctx.close()


def test_explicit_viscosity_cfl_and_adjoint_rejected(pd):
    import torch
    cells, N = (16, 16), 3
    print("explicit viscosity CFL check", flush=True)
    ctx = pd.pd_setup(2, cells, (1.0, 1.0), N, 1e-3, 0.6, 5e-2)   # dt above the viscous limit
    pd.pd_configure(ctx, pd.PD_CFG_EXPLICIT_VISC, 1)
    u = [torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda") for _ in range(2)]
    p = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    with pytest.raises(pd.PdError):
        pd.pd_step(ctx, u, p)
    with pytest.raises(pd.PdError):
        pd.pd_step_adjoint(ctx, u, [x.clone() for x in u])
    pd.pd_configure(ctx, pd.PD_CFG_EXPLICIT_VISC, 0)
    infos = pd.pd_step(ctx, u, p)                                    # implicit: any dt
    assert infos[3]["status"] == pd.PD_OK
    ctx.close()
