"""GPU parity of homogeneous Dirichlet pressure walls (odd reflection across the wall) against
the oracle: operator applies on every wall mask, tile shape and ragged tail, CG iterates, solves
against the fast-diagonalisation minimum-norm solution, the null-space projection, sampled
full-size applies, and the entry points that stay periodic-only.

Every case prints its parameters before touching the GPU so that a failure names its case."""
import numpy as np
import pytest

from oracle import layout
from oracle.operators import (Grid, apply_at, null_bases, pressure_operator, project_null,
                              viscous_operator)
from oracle.solvers import FastDiag, cg
import synthetic

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype or torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def periodic_flags(dim, mask):
    return tuple(bool((mask >> d) & 1) for d in range(dim))


def mass_norm(grid, v_tensor):
    W = np.ones(grid.shape())
    for d in range(grid.dim):
        shp = [1] * grid.dim
        shp[grid.dim - 1 - d] = -1
        W = W * np.tile(grid.tab.w, grid.cells[d]).reshape(shp)
    return np.sqrt(np.sum(W * v_tensor ** 2))


# (dim, cells, N, periodic_mask): walls across x, y, both (2D); z, x, y, all (3D); single-cell
# wall directions; ragged tile tails
APPLY_CASES = [
    (2, (9, 17), 3, 0b01), (2, (9, 17), 3, 0b10), (2, (9, 17), 3, 0b00), (2, (5, 3), 6, 0b00),
    (2, (16, 16), 2, 0b00), (2, (1, 4), 4, 0b10), (2, (3, 1), 5, 0b00), (2, (11, 7), 8, 0b01),
    (2, (13, 5), 0, 0b00), (2, (7, 6), 1, 0b10),
    (3, (5, 6, 9), 4, 0b011), (3, (5, 6, 9), 4, 0b110), (3, (5, 6, 9), 4, 0b101),
    (3, (5, 6, 9), 4, 0b000), (3, (3, 3, 3), 3, 0b000), (3, (2, 3, 9), 1, 0b010),
    (3, (3, 2, 2), 8, 0b000), (3, (9, 2, 3), 0, 0b100), (3, (1, 4, 1), 2, 0b010),
    (3, (3, 2, 6), 6, 0b001),
]


@pytest.mark.parametrize("dim,cells,N,mask", APPLY_CASES)
@pytest.mark.parametrize("op", [0, 1])
def test_apply_with_walls(pd, dim, cells, N, mask, op):
    """pd_apply (FP64 to 1e-13 of the largest output, FP32 to 3e-6 in norm) equals the assembled
    operator whose 1D blocks carry the reflected wall rows, for both operators."""
    import torch
    print(f"wall apply dim={dim} cells={cells} N={N} mask={mask:b} op={op}", flush=True)
    L = (1.0, 0.7, 1.3)[:dim]
    dt, nu = 1e-3, 0.37
    g = Grid(cells, L, N, periodic=periodic_flags(dim, mask))
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, nu, periodic_mask=mask)
    rng = np.random.default_rng(300 + N + mask)
    x = rng.standard_normal(g.ndof)
    A = pressure_operator(g, dt) if op == 0 else viscous_operator(g, dt, nu)
    ref = layout.tensor_to_blocked(A @ layout.blocked_to_tensor(x, cells, g.n).reshape(-1),
                                   cells, g.n)
    y = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
    pd.pd_apply(ctx, op, pd.PD_FP64, dev(x), y)
    got = host(y)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    y32 = torch.empty(g.ndof, dtype=torch.float32, device="cuda")
    pd.pd_apply(ctx, op, pd.PD_FP32, dev(x, torch.float32), y32)
    assert np.linalg.norm(host(y32) - ref) <= 3e-6 * np.linalg.norm(ref)
    ctx.close()


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("cells,N", [((23, 19), 3), ((17, 30), 6)])
def test_wall_apply_tile_shapes_agree(pd, cells, N, variant):
    """Several tiles per workgroup give the same wall apply bit for bit as one; a grid with walls
    runs the default tile shape, so a PD_CFG_TILE_VARIANT setting leaves the result unchanged."""
    import torch
    print(f"wall tile shapes cells={cells} N={N} variant={variant}", flush=True)
    g = Grid(cells, (1.0, 1.0), N, periodic=(False, False))
    ctx = pd.pd_setup(2, cells, (1.0, 1.0), N, 1e-3, 0.6, 1e-2, periodic_mask=0)
    x = dev(np.random.default_rng(41).standard_normal(g.ndof))
    y0 = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
    pd.pd_apply(ctx, 0, pd.PD_FP64, x, y0)
    pd.pd_configure(ctx, pd.PD_CFG_TILE_VARIANT, variant)
    pd.pd_configure(ctx, pd.PD_CFG_TILES_PER_WG, 3)
    y1 = torch.empty_like(y0)
    pd.pd_apply(ctx, 0, pd.PD_FP64, x, y1)
    ctx.close()
    assert torch.equal(y0, y1)


FORMS = {"one": (1, 1), "defer": (0, 1), "plain": (0, 0)}


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("dim,cells,N,mask,m", [(2, (9, 7), 4, 0b00, 23), (2, (12, 10), 5, 0b01, 37),
                                                (2, (17, 11), 3, 0b10, 9),
                                                (3, (4, 5, 3), 3, 0b000, 23),
                                                (3, (5, 3, 4), 2, 0b011, 15)])
def test_wall_cg_iterates_match_oracle_cg(pd, dim, cells, N, mask, m, form):
    """After exactly m FP64 iterations from x0 = 0 the GPU iterate equals the oracle's plain CG
    iterate on the assembled wall operator, in each form of the device loop (the one-kernel form
    is 2D only; 3D contexts run the two-kernel forms for it)."""
    import torch
    one, defer = FORMS[form]
    print(f"wall cg iterates dim={dim} cells={cells} N={N} mask={mask:b} m={m} form={form}",
          flush=True)
    L = (1.0,) * dim
    dt = 5e-4
    g = Grid(cells, L, N, periodic=periodic_flags(dim, mask))
    A = pressure_operator(g, dt)
    bt = layout.blocked_to_tensor(synthetic.random_rhs(61 + m, g.ndof), cells, g.n)
    bt = project_null(g, bt, null_bases(g))
    x_ref, it, _ = cg(A, bt.reshape(-1), 1e-30, m)
    assert it == m
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, 1e-2, periodic_mask=mask)
    pd.pd_configure(ctx, pd.PD_CFG_DEFER_X, defer)
    pd.pd_configure(ctx, pd.PD_CFG_ONE_KERNEL, one)
    x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    info = pd.pd_cg_solve(ctx, 0, pd.PD_FP64, dev(layout.tensor_to_blocked(bt, cells, g.n)), x,
                          1e-30, m)
    ctx.close()
    assert info["status"] == pd.PD_ENOCONV and info["iters"] == m
    got = layout.blocked_to_tensor(host(x), cells, g.n).reshape(-1)
    assert np.linalg.norm(got - x_ref) <= 1e-12 * np.linalg.norm(x_ref)


@pytest.mark.parametrize("dim,cells,N,mask", [(2, (16, 12), 3, 0b00), (2, (12, 9), 6, 0b01),
                                              (2, (9, 10), 5, 0b10), (2, (8, 8), 4, 0b00),
                                              (3, (5, 4, 6), 3, 0b000), (3, (4, 4, 4), 4, 0b110),
                                              (3, (4, 5, 3), 1, 0b011)])
@pytest.mark.parametrize("prec", [0, 2])
def test_wall_pressure_solve_matches_min_norm(pd, dim, cells, N, mask, prec):
    """FP64 and FP32+refinement pressure solves reach the minimum-norm solution of the oracle's
    fast diagonalisation on the wall operator (definite for even N; odd N keeps the odd
    cell-periodic mode, which the solve projects out)."""
    import torch
    print(f"wall solve dim={dim} cells={cells} N={N} mask={mask:b} prec={prec}", flush=True)
    L = (1.0,) * dim
    dt = 5e-4
    g = Grid(cells, L, N, periodic=periodic_flags(dim, mask))
    b = synthetic.random_rhs(17, g.ndof)
    ref_t = FastDiag(g).solve(layout.blocked_to_tensor(b, cells, g.n), 0.0, dt)
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, 1e-2, periodic_mask=mask)
    x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    info = pd.pd_cg_solve(ctx, 0, prec, dev(b), x, 1e-12, 200000)
    ctx.close()
    print(info, flush=True)
    got_t = layout.blocked_to_tensor(host(x), cells, g.n)
    err = mass_norm(g, got_t - ref_t) / mass_norm(g, ref_t)
    assert info["status"] == pd.PD_OK
    assert info["rel_res_true"] <= 2e-12
    assert err <= 1e-9


@pytest.mark.parametrize("dim,cells,N,mask", [(2, (7, 9), 3, 0b01), (2, (7, 9), 3, 0b00),
                                              (2, (7, 9), 4, 0b10), (3, (3, 4, 5), 5, 0b010),
                                              (3, (3, 4, 5), 2, 0b000)])
@pytest.mark.parametrize("noalloc", [0, 1])
def test_wall_project_null(pd, dim, cells, N, mask, noalloc):
    """pd_project_null and pd_project_null_noalloc remove exactly the oracle's wall null space:
    odd part of the cell-periodic kernel along Dirichlet directions (identity for even N)."""
    print(f"wall project dim={dim} cells={cells} N={N} mask={mask:b} noalloc={noalloc}",
          flush=True)
    L = (1.0,) * dim
    g = Grid(cells, L, N, periodic=periodic_flags(dim, mask))
    v = np.random.default_rng(5).standard_normal(g.ndof)
    ref = layout.tensor_to_blocked(project_null(g, layout.blocked_to_tensor(v, cells, g.n),
                                                null_bases(g)), cells, g.n)
    ctx = pd.pd_setup(dim, cells, L, N, 1e-3, 0.6, 1e-2, periodic_mask=mask)
    t = dev(v)
    (pd.pd_project_null_noalloc if noalloc else pd.pd_project_null)(ctx, pd.PD_FP64, t)
    ctx.close()
    assert np.abs(host(t) - ref).max() <= 1e-13 * np.abs(v).max()


def test_full_size_wall_apply_sampled(pd):
    """2D 256^2 N=6 and 3D 64^3 N=4 with walls on every side: sampled pd_apply outputs, the
    wall rows and corners included, against the block definition one output at a time."""
    import torch
    for dim, cells, N in [(2, (256, 256), 6), (3, (64, 64, 64), 4)]:
        print(f"full-size wall apply dim={dim} cells={cells} N={N}", flush=True)
        L = (1.0,) * dim
        g = Grid(cells, L, N, periodic=(False,) * dim)
        ctx = pd.pd_setup(dim, cells, L, N, 1e-3, 0.6, 1e-3, periodic_mask=0)
        rng = np.random.default_rng(78)
        x = rng.standard_normal(g.ndof)
        y = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
        pd.pd_apply(ctx, 0, pd.PD_FP64, dev(x), y)
        yt = layout.blocked_to_tensor(host(y), cells, g.n)
        xt = layout.blocked_to_tensor(x, cells, g.n)
        shp = np.array(g.shape())
        idx = np.stack([rng.integers(0, s, size=200) for s in shp], axis=1)
        idx[:4] = 0
        idx[4:8] = shp - 1
        for a in range(dim):                           # one wall face per axis, both ends
            idx[8 + 2 * a, a] = 0
            idx[9 + 2 * a, a] = shp[a] - 1
        ref = apply_at(g, xt, idx, 0.0, 1e-3)
        got = yt[tuple(idx.T)]
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        ctx.close()


def test_wall_contexts_reject_periodic_only_entry_points(pd):
    """Velocity, step, adjoint and loss entry points refuse a context with walls (PD_EINVAL);
    mask bits at or above dim are refused at setup."""
    import torch
    print("wall rejections", flush=True)
    cells, N = (6, 5), 3
    g = Grid(cells, (1.0, 1.0), N, periodic=(True, False))
    ctx = pd.pd_setup(2, cells, (1.0, 1.0), N, 1e-3, 0.6, 1e-2, periodic_mask=0b01)
    u = [torch.zeros(g.ndof, dtype=torch.float64, device="cuda") for _ in range(2)]
    q = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    calls = [lambda: pd.pd_rhs_div(ctx, u, q), lambda: pd.pd_project_velocity(ctx, q, u),
             lambda: pd.pd_convect(ctx, u), lambda: pd.pd_step(ctx, u, q),
             lambda: pd.pd_step_adjoint(ctx, u, [x.clone() for x in u]),
             lambda: pd.pd_kinetic_energy(ctx, u),
             lambda: pd.pd_l2_project(ctx, 0, 0, u[0], u[1])]
    for call in calls:
        with pytest.raises(pd.PdError) as e:
            call()
        assert e.value.code == pd.PD_EINVAL
    ctx.close()
    with pytest.raises(pd.PdError):
        pd.pd_setup(2, cells, (1.0, 1.0), N, 1e-3, 0.6, 1e-2, periodic_mask=0b101)


@pytest.mark.parametrize("dim,cells,N,mask", [(2, (16, 12), 3, 0b00), (2, (12, 9), 6, 0b01),
                                              (2, (10, 12), 5, 0b10), (3, (5, 4, 6), 4, 0b000),
                                              (3, (4, 5, 3), 3, 0b011)])
@pytest.mark.parametrize("prec", [0, 2])
def test_wall_preconditioned_solve(pd, dim, cells, N, mask, prec):
    """The cell-block Jacobi preconditioner (the interior block in every cell, exact away from
    the walls) with walls: FP64 and FP32+refinement solves reach the fast-diagonalisation
    minimum-norm solution and need fewer iterations than unpreconditioned CG."""
    import torch
    print(f"wall pcg dim={dim} cells={cells} N={N} mask={mask:b} prec={prec}", flush=True)
    L = (1.0,) * dim
    dt = 5e-4
    g = Grid(cells, L, N, periodic=periodic_flags(dim, mask))
    b = synthetic.random_rhs(23, g.ndof)
    ref_t = FastDiag(g).solve(layout.blocked_to_tensor(b, cells, g.n), 0.0, dt)
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, 1e-2, periodic_mask=mask)
    its = {}
    for pc in (0, 1):
        pd.pd_configure(ctx, pd.PD_CFG_PRECOND, pc)
        x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
        info = pd.pd_cg_solve(ctx, 0, prec, dev(b), x, 1e-12, 200000)
        print(f"  precond={pc}: {info}", flush=True)
        assert info["status"] == pd.PD_OK
        assert info["rel_res_true"] <= 2e-12
        got_t = layout.blocked_to_tensor(host(x), cells, g.n)
        assert mass_norm(g, got_t - ref_t) <= 1e-9 * mass_norm(g, ref_t)
        its[pc] = info["iters"]
    ctx.close()
    assert its[1] < its[0]
