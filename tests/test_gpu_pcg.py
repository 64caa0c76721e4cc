"""GPU parity of the cell-block Jacobi preconditioned CG (PD_CFG_PRECOND; the preconditioning
the paper names as future work for its matrix-free CG, end of Section 2.1) against the oracle's
PCG with its own block-Jacobi preconditioner (dense per-cell inverses of the assembled
operator): the iterate after exactly m iterations, full solves against the direct minimum-norm
solution in both precisions, and the preconditioned fractional step.

Every case prints its parameters before touching the GPU so that a failure names its case."""
import numpy as np
import pytest

from oracle import layout
from oracle.operators import (Grid, pressure_operator, viscous_operator, null_basis_tiled,
                              project_null)
from oracle.solvers import FastDiag, pcg, block_jacobi
from oracle.step import StepOracle
import synthetic

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def mass_norm(g, T):
    W = np.ones(g.shape())
    for d in range(g.dim):
        shp = [1] * g.dim
        shp[g.dim - 1 - d] = -1
        W = W * np.tile(g.tab.w, g.cells[d]).reshape(shp)
    return np.sqrt(np.sum(W * T ** 2))


@pytest.mark.parametrize("dim,cells,N,m,op", [(2, (9, 7), 4, 3, 0), (2, (12, 10), 6, 17, 0),
                                              (2, (6, 5), 0, 9, 0), (2, (11, 7), 3, 25, 1),
                                              (3, (4, 5, 3), 3, 11, 0), (3, (3, 4, 3), 2, 6, 1),
                                              (2, (5, 4), 8, 12, 0)])
def test_pcg_iterates_match_oracle_pcg(pd, dim, cells, N, m, op):
    """After exactly m preconditioned iterations from x0 = 0 (maxit = m) the GPU iterate equals
    the oracle's PCG iterate x_m (pressure iterates compared after the null-space projection the
    solve applies at exit)."""
    import torch
    print(f"pcg iterates dim={dim} cells={cells} N={N} m={m} op={op}", flush=True)
    L = (1.0, 0.8, 1.2)[:dim]
    dt, nu = 5e-4, 0.3
    g = Grid(cells, L, N)
    A = pressure_operator(g, dt) if op == 0 else viscous_operator(g, dt, nu)
    Z = [null_basis_tiled(c, N) for c in cells]
    bt = layout.blocked_to_tensor(synthetic.random_rhs(31 + m, g.ndof), cells, g.n)
    if op == 0:
        bt = project_null(g, bt, Z)
    x_ref, it, _ = pcg(A, bt.reshape(-1), 1e-300, m, block_jacobi(g, A))
    assert it == m
    if op == 0:
        x_ref = project_null(g, x_ref.reshape(g.shape()), Z).reshape(-1)
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, nu)
    pd.pd_configure(ctx, pd.PD_CFG_PRECOND, 1)
    x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    info = pd.pd_cg_solve(ctx, op, pd.PD_FP64, dev(layout.tensor_to_blocked(bt, cells, g.n)), x,
                          1e-30, m)
    ctx.close()
    assert info["status"] == pd.PD_ENOCONV and info["iters"] == m
    got = layout.blocked_to_tensor(host(x), cells, g.n).reshape(-1)
    assert np.linalg.norm(got - x_ref) <= 1e-12 * np.linalg.norm(x_ref)


@pytest.mark.parametrize("dim,cells,N", [(2, (16, 16), 3), (2, (12, 9), 6), (2, (3, 2), 0),
                                         (2, (9, 7), 1), (2, (6, 5), 5), (2, (5, 6), 7),
                                         (2, (4, 5), 8), (3, (5, 4, 6), 3), (3, (4, 4, 4), 4),
                                         (3, (3, 4, 2), 0)])
@pytest.mark.parametrize("prec", [0, 2])
def test_pcg_solve_matches_min_norm(pd, dim, cells, N, prec):
    """Preconditioned pressure solves (FP64, and FP32 inner iterations with FP64 residual
    replacement) to rtol 1e-12 of an unprojected random right-hand side against the direct
    minimum-norm solution, in fewer iterations than the unpreconditioned solve."""
    import torch
    print(f"pcg solve dim={dim} cells={cells} N={N} prec={prec}", flush=True)
    L = (1.0,) * dim
    dt = 5e-4
    g = Grid(cells, L, N)
    b = synthetic.random_rhs(11, g.ndof)
    ref = FastDiag(g).solve(layout.blocked_to_tensor(b, cells, g.n), 0.0, dt)
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, 1e-2)
    x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    plain = pd.pd_cg_solve(ctx, 0, prec, dev(b), x, 1e-12, 400000)
    pd.pd_configure(ctx, pd.PD_CFG_PRECOND, 1)
    x.zero_()
    info = pd.pd_cg_solve(ctx, 0, prec, dev(b), x, 1e-12, 400000)
    ctx.close()
    err = mass_norm(g, layout.blocked_to_tensor(host(x), cells, g.n) - ref) / mass_norm(g, ref)
    print(f"  iters {info['iters']} (plain {plain['iters']}) true {info['rel_res_true']:.2e} "
          f"err {err:.2e}", flush=True)
    assert info["status"] == pd.PD_OK
    assert info["rel_res_true"] <= 2e-12
    assert err <= 1e-9
    if N >= 2:
        assert info["iters"] < plain["iters"]


def test_pcg_step_matches_oracle_step(pd):
    """The fractional step on the 16^2 N = 3 Taylor-Green field with preconditioned pressure and
    viscous solves against the oracle step with exact solves."""
    import torch
    cfg = synthetic.CONFIGS["tgv2d_16_N3"]
    cells, N = cfg["cells"], cfg["N"]
    print(f"pcg step tgv2d cells={cells} N={N}", flush=True)
    g = Grid(cells, cfg["lengths"], N)
    co = synthetic.staggered_coords(cells, g.lengths, g.tab.xi)
    Ut = synthetic.tgv2d([(co[0][0], co[0][1]), (co[1][0], co[1][1])])
    ref = StepOracle(g, cfg["dt"], cfg["theta"], cfg["nu"]).step(Ut, np.zeros(g.shape()))
    ctx = pd.pd_setup(2, cells, cfg["lengths"], N, cfg["dt"], cfg["theta"], cfg["nu"])
    pd.pd_configure(ctx, pd.PD_CFG_PRECOND, 1)
    pd.pd_configure(ctx, pd.PD_CFG_P_RTOL, 1e-12)
    pd.pd_configure(ctx, pd.PD_CFG_V_RTOL, 1e-13)
    u = [dev(layout.tensor_to_blocked(x, cells, g.n)) for x in Ut]
    p = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    infos = pd.pd_step(ctx, u, p)
    assert all(i["status"] == pd.PD_OK for i in infos[:2] + infos[3:])
    for d in range(2):
        got = layout.blocked_to_tensor(host(u[d]), cells, g.n)
        assert mass_norm(g, got - ref["U_new"][d]) <= 1e-10 * mass_norm(g, ref["U_new"][d])
    ctx.close()
