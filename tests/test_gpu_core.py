"""GPU parity of the operator apply, the CG solves and the support operators against the oracle.

Every case prints its parameters before touching the GPU so that a failure names its case."""
import numpy as np
import pytest

from oracle import layout
from oracle.operators import (Grid, pressure_operator, viscous_operator, div_rhs, grad_update,
                              apply_at, apply_operator, null_basis_tiled, project_null)
from oracle.solvers import FastDiag, cg
from oracle.step import dual_to_main, main_to_dual, rk3, StepOracle
import synthetic

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype or torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def mass_norm(grid, v_tensor):
    W = np.ones(grid.shape())
    for d in range(grid.dim):
        shp = [1] * grid.dim
        shp[grid.dim - 1 - d] = -1
        W = W * np.tile(grid.tab.w, grid.cells[d]).reshape(shp)
    return np.sqrt(np.sum(W * v_tensor ** 2))


APPLY_CASES = [
    (2, (5, 3), 3), (2, (16, 16), 3), (2, (9, 17), 6), (2, (3, 2), 0), (2, (11, 7), 8),
    (2, (1, 4), 2), (2, (13, 5), 5),
    (3, (5, 6, 9), 4), (3, (3, 3, 3), 3), (3, (2, 3, 9), 1), (3, (3, 2, 2), 8), (3, (4, 4, 5), 2),
    (3, (9, 2, 3), 0), (3, (3, 2, 6), 6),
    # ragged and wrapped tiles of the coalesced 3D form (FP32 N = 1..4, FP64 N = 1)
    (3, (11, 5, 4), 1), (3, (10, 3, 5), 2), (3, (7, 9, 3), 3), (3, (6, 5, 4), 4), (3, (2, 7, 3), 4),
]


@pytest.mark.parametrize("dim,cells,N", APPLY_CASES)
@pytest.mark.parametrize("op", [0, 1])
def test_apply_fp64_fp32(pd, dim, cells, N, op):
    import torch
    print(f"apply dim={dim} cells={cells} N={N} op={op}", flush=True)
    L = (1.0, 0.7, 1.3)[:dim]
    dt, nu = 1e-3, 0.37
    g = Grid(cells, L, N)
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, nu)
    rng = np.random.default_rng(100 + N)
    x = rng.standard_normal(g.ndof)
    A = pressure_operator(g, dt) if op == 0 else viscous_operator(g, dt, nu)
    ref = layout.tensor_to_blocked(A @ layout.blocked_to_tensor(x, cells, g.n).reshape(-1), cells, g.n)
    y = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
    pd.pd_apply(ctx, op, pd.PD_FP64, dev(x), y)
    got = host(y)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-13 * scale
    y32 = torch.empty(g.ndof, dtype=torch.float32, device="cuda")
    pd.pd_apply(ctx, op, pd.PD_FP32, dev(x, torch.float32), y32)
    got32 = host(y32)
    assert np.linalg.norm(got32 - ref) <= 3e-6 * np.linalg.norm(ref)
    ctx.close()


def _solve_case(pd, dim, cells, N, op, prec, project_rhs, rtol, seed, one_kernel=None):
    import torch
    print(f"solve dim={dim} cells={cells} N={N} op={op} prec={prec} seed={seed}", flush=True)
    L = (1.0,) * dim
    dt, nu = 5e-4, 1e-2
    g = Grid(cells, L, N)
    fd = FastDiag(g)
    b = synthetic.random_rhs(seed, g.ndof)
    bt = layout.blocked_to_tensor(b, cells, g.n)
    if op == 0:
        ref_t = fd.solve(bt, 0.0, dt)
    else:
        ref_t = fd.solve(bt, 1.0, nu * dt)
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, nu)
    if one_kernel is not None:
        pd.pd_configure(ctx, pd.PD_CFG_ONE_KERNEL, one_kernel)
    x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    info = pd.pd_cg_solve(ctx, op, prec, dev(b), x, rtol, 200000)
    got_t = layout.blocked_to_tensor(host(x), cells, g.n)
    err = mass_norm(g, got_t - ref_t) / mass_norm(g, ref_t)
    ctx.close()
    return info, err


@pytest.mark.parametrize("dim,cells,N", [(2, (16, 16), 3), (2, (12, 9), 6), (2, (7, 8), 2),
                                         (2, (3, 2), 0), (2, (9, 7), 1), (2, (6, 5), 5),
                                         (2, (5, 6), 7), (2, (4, 5), 8),
                                         (3, (5, 4, 6), 3), (3, (4, 4, 4), 4), (3, (4, 3, 5), 1),
                                         (3, (3, 4, 2), 0)])
@pytest.mark.parametrize("prec", [0, 2])
def test_pressure_solve_matches_min_norm(pd, dim, cells, N, prec):
    info, err = _solve_case(pd, dim, cells, N, 0, prec, True, 1e-12, 11)
    print(info, err)
    assert info["status"] == pd.PD_OK
    assert info["rel_res_true"] <= 2e-12
    assert err <= 1e-9


# (PD_CFG_ONE_KERNEL, PD_CFG_DEFER_X): one kernel per iteration (2D, opt-in), operator kernel +
# update kernel with the deferred x update (default), and the plain two-kernel form
FORMS = {"one": (1, 1), "defer": (0, 1), "plain": (0, 0)}


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("dim,cells,N,m", [(2, (9, 7), 4, 1), (2, (9, 7), 4, 2), (2, (12, 10), 6, 37),
                                           (3, (4, 5, 3), 3, 23), (2, (6, 5), 0, 9),
                                           (2, (17, 11), 3, 3), (2, (17, 11), 3, 50)])
def test_cg_iterates_match_oracle_cg(pd, dim, cells, N, m, form):
    """After exactly m FP64 iterations from x0 = 0 (maxit = m) the GPU iterate equals the oracle's
    plain CG iterate x_m on the assembled matrix. Pins the iteration bookkeeping of the device
    loop in each form: the x update of the last iteration, which the apply kernel of the next
    iteration would have made and the stop leaves to the flush kernel (deferred forms), the
    residual update folded into the next operator kernel with rho_k from the expanded inner
    products (one-kernel form), and the plain form with x updated in the update kernel. (The
    oracle's own x_m moves by ~1e-15 relative under 1e-15 perturbations of b for these
    cases.)"""
    import torch
    one, defer = FORMS[form]
    print(f"cg iterates dim={dim} cells={cells} N={N} m={m} form={form}", flush=True)
    L = (1.0,) * dim
    dt = 5e-4
    g = Grid(cells, L, N)
    A = pressure_operator(g, dt)
    bt = layout.blocked_to_tensor(synthetic.random_rhs(21 + m, g.ndof), cells, g.n)
    bt = project_null(g, bt, [null_basis_tiled(c, N) for c in cells])   # b in range(A_p)
    x_ref, it, _ = cg(A, bt.reshape(-1), 1e-30, m)
    assert it == m
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, 1e-2)
    pd.pd_configure(ctx, pd.PD_CFG_DEFER_X, defer)
    pd.pd_configure(ctx, pd.PD_CFG_ONE_KERNEL, one)
    x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    info = pd.pd_cg_solve(ctx, 0, pd.PD_FP64, dev(layout.tensor_to_blocked(bt, cells, g.n)), x,
                          1e-30, m)
    ctx.close()
    assert info["status"] == pd.PD_ENOCONV and info["iters"] == m
    got = layout.blocked_to_tensor(host(x), cells, g.n).reshape(-1)
    assert np.linalg.norm(got - x_ref) <= 1e-12 * np.linalg.norm(x_ref)


@pytest.mark.parametrize("cells,N", [((6, 5, 7), 4), ((9, 7, 5), 2), ((11, 5, 6), 1), ((5, 4, 9), 3),
                                     ((4, 3, 6), 5), ((3, 2, 5), 6)])
def test_3d_launch_shapes_match_oracle_cg(pd, cells, N):
    """The 3D operator kernel's launch-shape settings cut the work differently, not what is
    computed: with the halo prefetch off (PD_CFG_PREFETCH 0) and with column segments of 1 and 3
    planes (PD_CFG_KZ) the FP64 iterate after m iterations equals the oracle's plain CG iterate
    (these shapes run both 3D kernel forms, ragged and wrapped tiles, and segments that end at the
    last plane). In FP32 (refined) the prefetch setting gives bit-identical iterates, the segment
    length changes only the grouping of the FP64 dot-product partials."""
    import torch
    m = 24
    print(f"3d launch shapes cells={cells} N={N}", flush=True)
    L = (1.0, 0.8, 1.2)
    dt = 5e-4
    g = Grid(cells, L, N)
    A = pressure_operator(g, dt)
    bt = layout.blocked_to_tensor(synthetic.random_rhs(300 + N, g.ndof), cells, g.n)
    bt = project_null(g, bt, [null_basis_tiled(c, N) for c in cells])
    x_ref, it, _ = cg(A, bt.reshape(-1), 1e-30, m)
    assert it == m
    ctx = pd.pd_setup(3, cells, L, N, dt, 0.6, 1e-2)
    b = dev(layout.tensor_to_blocked(bt, cells, g.n))

    def run(prec, pf, kz):
        pd.pd_configure(ctx, pd.PD_CFG_PREFETCH, pf)
        pd.pd_configure(ctx, pd.PD_CFG_KZ, kz)
        x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
        info = pd.pd_cg_solve(ctx, 0, prec, b, x, 1e-30, m)
        assert info["status"] == pd.PD_ENOCONV and info["iters"] == m
        return host(x)

    for pf, kz in [(1, 0), (0, 0), (1, 1), (1, 3), (0, 3)]:
        got = layout.blocked_to_tensor(run(pd.PD_FP64, pf, kz), cells, g.n).reshape(-1)
        err = np.linalg.norm(got - x_ref) / np.linalg.norm(x_ref)
        print(f"  fp64 prefetch={pf} kz={kz}: rel. diff vs oracle {err:.2e}", flush=True)
        assert err <= 1e-12
    r0 = run(pd.PD_FP32_REFINE64, 1, 0)
    assert np.array_equal(r0, run(pd.PD_FP32_REFINE64, 0, 0))
    for kz in (1, 3):
        d = np.linalg.norm(run(pd.PD_FP32_REFINE64, 1, kz) - r0) / np.linalg.norm(r0)
        print(f"  fp32 kz={kz}: rel. diff vs automatic segments {d:.2e}", flush=True)
        assert d <= 1e-5
    ctx.close()


@pytest.mark.parametrize("one", [1, 0])
def test_timing_samples_every_sth_launch(pd, one):
    """PD_CFG_TIMING = s times every s-th operator launch of a pressure solve (iterations
    0, s, 2s, ... below the final count) and reports the algorithmic bytes per launch: 8 words
    per DoF in the one-kernel form, 6 with the separate update kernel."""
    import torch
    cells, N, m, s = (10, 8), 3, 37, 4
    g = Grid(cells, (1.0, 1.0), N)
    ctx = pd.pd_setup(2, cells, (1.0, 1.0), N, 5e-4, 0.6, 1e-2)
    pd.pd_configure(ctx, pd.PD_CFG_ONE_KERNEL, one)
    pd.pd_configure(ctx, pd.PD_CFG_TIMING, s)
    pd.pd_timing(ctx, pd.PD_FP64, reset=True)
    x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    info = pd.pd_cg_solve(ctx, 0, pd.PD_FP64, dev(synthetic.random_rhs(5, g.ndof)), x, 1e-30, m)
    t = pd.pd_timing(ctx, pd.PD_FP64, reset=True)
    ctx.close()
    assert info["iters"] == m
    assert t["launches"] == (m + s - 1) // s and t["total_ms"] > 0.0
    assert t["bytes_per_launch"] == (8.0 if one else 6.0) * g.ndof * 8.0


@pytest.mark.parametrize("prec", [0, 2])
@pytest.mark.parametrize("cells,N,rtol", [((23, 19), 5, 1e-12), ((40, 33), 3, 1e-11)])
def test_one_kernel_form_matches_two_kernel_form(pd, cells, N, rtol, prec):
    """Full solves (FP64 with its true-residual continuation, FP32 with FP64 residual
    replacements, which restart the run at odd and even iterations and so exercise both
    residual buffers) in the one-kernel and the two-kernel form: both meet the tolerance on the
    true residual, reach the minimum-norm solution, and take iteration counts within 2 % of
    each other (the forms differ only in the rounding of rho_k)."""
    res = {}
    for one in (1, 0):
        print(f"one-kernel form cells={cells} N={N} prec={prec} one={one}", flush=True)
        info, err = _solve_case(pd, 2, cells, N, 0, prec, True, rtol, 31, one_kernel=one)
        assert info["status"] == pd.PD_OK
        assert info["rel_res_true"] <= 1.05 * rtol
        assert err <= 1e3 * rtol
        res[one] = info
    if prec == 2:
        assert res[1]["outer_iters"] >= 2
    assert abs(res[1]["iters"] - res[0]["iters"]) <= max(2, 0.02 * res[0]["iters"])


@pytest.mark.parametrize("prec", [0, 2])
def test_viscous_solve(pd, prec):
    info, err = _solve_case(pd, 2, (10, 12), 4, 1, prec, False, 1e-12, 12)
    assert info["status"] == pd.PD_OK
    assert err <= 1e-11


def test_status_codes(pd):
    import torch
    cells, N = (6, 6), 2
    ctx = pd.pd_setup(2, cells, (1.0, 1.0), N, 1e-3, 0.6, 0.0)
    g = Grid(cells, (1.0, 1.0), N)
    b = synthetic.random_rhs(3, g.ndof)
    x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    info = pd.pd_cg_solve(ctx, 0, pd.PD_FP64, dev(b), x, 1e-12, 2)
    assert info["status"] == pd.PD_ENOCONV and info["iters"] == 2
    bn = b.copy()
    bn[5] = np.nan
    x.zero_()
    info = pd.pd_cg_solve(ctx, 0, pd.PD_FP64, dev(bn), x, 1e-12, 100)
    assert info["status"] == pd.PD_EBREAKDOWN
    x.zero_()
    info = pd.pd_cg_solve(ctx, 0, pd.PD_FP64, dev(np.zeros(g.ndof)), x, 1e-12, 100)
    assert info["status"] == pd.PD_OK and float(x.abs().max()) == 0.0
    with pytest.raises(pd.PdError):
        pd.pd_cg_solve(ctx, 7, pd.PD_FP64, dev(b), x, 1e-12, 100)
    ctx.close()
    with pytest.raises(pd.PdError):
        pd.pd_setup(2, (4, 4), (1.0, 1.0), 9, 1e-3, 0.6, 0.0)


@pytest.mark.parametrize("dim,cells,N", [(2, (6, 5), 3), (2, (4, 7), 6), (3, (3, 4, 5), 2),
                                         (3, (4, 3, 3), 3)])
def test_line_operators(pd, dim, cells, N):
    import torch
    print(f"line ops dim={dim} cells={cells} N={N}", flush=True)
    L = (1.0, 0.8, 1.2)[:dim]
    dt = 2e-3
    g = Grid(cells, L, N)
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, 0.0)
    rng = np.random.default_rng(5)
    U = [rng.standard_normal(g.ndof) for _ in range(dim)]
    q = rng.standard_normal(g.ndof)
    Ut = [layout.blocked_to_tensor(u, cells, g.n) for u in U]
    # b = sum_d B_d U_d
    ref = sum(div_rhs(g, d) @ Ut[d].reshape(-1) for d in range(dim))
    b = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
    ud = [dev(u) for u in U]
    pd.pd_rhs_div(ctx, ud, b)
    ref_b = layout.tensor_to_blocked(ref.reshape(g.shape()), cells, g.n)
    assert np.abs(host(b) - ref_b).max() <= 1e-13 * np.abs(ref_b).max()
    # velocity update
    pd.pd_project_velocity(ctx, dev(q), ud)
    qt = layout.blocked_to_tensor(q, cells, g.n).reshape(-1)
    for d in range(dim):
        ref_u = Ut[d].reshape(-1) - grad_update(g, d, dt) @ qt
        ref_u = layout.tensor_to_blocked(ref_u.reshape(g.shape()), cells, g.n)
        assert np.abs(host(ud[d]) - ref_u).max() <= 1e-13 * np.abs(ref_u).max()
    # L2 projections
    for d in range(dim):
        out = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
        pd.pd_l2_project(ctx, d, 0, dev(U[d]), out)
        ref_m = layout.tensor_to_blocked(dual_to_main(g, Ut[d], d), cells, g.n)
        assert np.abs(host(out) - ref_m).max() <= 1e-13 * np.abs(ref_m).max()
        pd.pd_l2_project(ctx, d, 1, dev(U[d]), out)
        ref_s = layout.tensor_to_blocked(main_to_dual(g, Ut[d], d), cells, g.n)
        assert np.abs(host(out) - ref_s).max() <= 1e-13 * np.abs(ref_s).max()
    ctx.close()


@pytest.mark.parametrize("dim,cells,N", [(2, (6, 5), 3), (3, (3, 4, 3), 2)])
def test_convection_rk3(pd, dim, cells, N):
    print(f"convection dim={dim} cells={cells} N={N}", flush=True)
    L = (1.0,) * dim
    dt = 1e-3
    g = Grid(cells, L, N)
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, 0.0)
    rng = np.random.default_rng(9)
    V = [0.3 * rng.standard_normal(g.ndof) for _ in range(dim)]
    Vt = [layout.blocked_to_tensor(v, cells, g.n) for v in V]
    ref = rk3(g, Vt, dt)
    vd = [dev(v) for v in V]
    pd.pd_convect(ctx, vd)
    for d in range(dim):
        r = layout.tensor_to_blocked(ref[d], cells, g.n)
        assert np.abs(host(vd[d]) - r).max() <= 1e-13 * np.abs(r).max()
    ctx.close()


def _tgv_initial(g):
    coords = synthetic.staggered_coords(g.cells, g.lengths, g.tab.xi)
    U = synthetic.tgv2d([(coords[0][0], coords[0][1]), (coords[1][0], coords[1][1])])
    return U


@pytest.mark.parametrize("prec", [0, 2])
def test_step_tgv2d_16_N3(pd, prec):
    import torch
    cfg = synthetic.CONFIGS["tgv2d_16_N3"]
    cells, N = cfg["cells"], cfg["N"]
    print(f"step tgv2d cells={cells} N={N} prec={prec}", flush=True)
    g = Grid(cells, cfg["lengths"], N)
    so = StepOracle(g, cfg["dt"], cfg["theta"], cfg["nu"])
    Ut = _tgv_initial(g)
    P0 = np.zeros(g.shape())
    ref = so.step(Ut, P0)
    ctx = pd.pd_setup(2, cells, cfg["lengths"], N, cfg["dt"], cfg["theta"], cfg["nu"])
    pd.pd_configure(ctx, pd.PD_CFG_STEP_PREC, prec)
    pd.pd_configure(ctx, pd.PD_CFG_P_RTOL, 1e-12)
    pd.pd_configure(ctx, pd.PD_CFG_V_RTOL, 1e-13)
    ud = [dev(layout.tensor_to_blocked(u, cells, g.n)) for u in Ut]
    p = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    infos = pd.pd_step(ctx, ud, p)
    print(infos)
    assert all(i["status"] == pd.PD_OK for i in infos[:2] + infos[3:])
    for d in range(2):
        r = ref["U_new"][d]
        got = layout.blocked_to_tensor(host(ud[d]), cells, g.n)
        assert mass_norm(g, got - r) <= 1e-10 * mass_norm(g, r)
    got_p = layout.blocked_to_tensor(host(p), cells, g.n)
    assert mass_norm(g, got_p - ref["P_new"]) <= 1e-9 * mass_norm(g, ref["P_new"])
    ctx.close()


def test_full_size_apply_sampled(pd):
    """3D 64^3 N=4 (32.8M DoFs) and 2D 256^2 N=6: sampled outputs of pd_apply against the
    block definition evaluated one output at a time."""
    import torch
    for dim, cells, N in [(2, (256, 256), 6), (3, (64, 64, 64), 4)]:
        print(f"full-size apply dim={dim} cells={cells} N={N}", flush=True)
        L = (1.0,) * dim
        g = Grid(cells, L, N)
        ctx = pd.pd_setup(dim, cells, L, N, 1e-3, 0.6, 1e-3)
        rng = np.random.default_rng(77)
        x = rng.standard_normal(g.ndof)
        y = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
        pd.pd_apply(ctx, 0, pd.PD_FP64, dev(x), y)
        yt = layout.blocked_to_tensor(host(y), cells, g.n)
        xt = layout.blocked_to_tensor(x, cells, g.n)
        shp = g.shape()
        idx = np.stack([rng.integers(0, s, size=200) for s in shp], axis=1)
        # include the periodic seams
        idx[:4] = 0
        idx[4:8] = np.array(shp) - 1
        ref = apply_at(g, xt, idx, 0.0, 1e-3)
        got = yt[tuple(idx.T)]
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        ctx.close()


@pytest.mark.parametrize("cells,N", [((23, 19), 3), ((17, 30), 6), ((41, 9), 1)])
@pytest.mark.parametrize("one,prec", [(0, 0), (1, 0), (0, 2), (1, 2)])
def test_tiles_per_workgroup_shapes_agree(pd, cells, N, one, prec):
    """Workgroups taking several tiles strided over the grid (PD_CFG_TILES_PER_WG = 2, 3, 5 on
    ragged tile counts, so that some workgroups get one tile fewer) give the same operator apply
    bit for bit as one tile per workgroup (FP64 and FP32), and the same CG iterate after 9
    iterations up to the block order of the dot-product partial sums, in the two-kernel and the
    one-kernel form (whose per-slot partial tuples the next launch re-reads), in FP64 and in
    FP32+refine (9 FP32 iterations: the iterate agrees to FP32 rounding)."""
    import torch
    print(f"tiles per workgroup cells={cells} N={N} one={one} prec={prec}", flush=True)
    L = (1.0, 1.0)
    g = Grid(cells, L, N)
    ctx = pd.pd_setup(2, cells, L, N, 5e-4, 0.6, 1e-3)
    pd.pd_configure(ctx, pd.PD_CFG_ONE_KERNEL, one)
    rng = np.random.default_rng(17)
    xin = rng.standard_normal(g.ndof)
    b = dev(synthetic.random_rhs(18, g.ndof))
    fp32 = prec == pd.PD_FP32_REFINE64
    out = {}
    for per in (1, 2, 3, 5):
        pd.pd_configure(ctx, pd.PD_CFG_TILES_PER_WG, per)
        if fp32:
            y = torch.empty(g.ndof, dtype=torch.float32, device="cuda")
            pd.pd_apply(ctx, 0, pd.PD_FP32, dev(xin, torch.float32), y)
        else:
            y = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
            pd.pd_apply(ctx, 0, pd.PD_FP64, dev(xin), y)
        x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
        info = pd.pd_cg_solve(ctx, 0, prec, b, x, 1e-30, 9)
        assert info["iters"] == 9
        out[per] = (host(y), host(x))
    ctx.close()
    y1, x1 = out[1]
    for per in (2, 3, 5):
        y, x = out[per]
        assert np.array_equal(y, y1)
        assert np.linalg.norm(x - x1) <= (1e-5 if fp32 else 1e-12) * np.linalg.norm(x1)


def test_large_2d_grids(pd):
    """2D grids with more tiles than one launch holds workgroups (2050^2 N = 0: 66049 tiles of
    8x8 cells; 1460^2 N = 6: 66795 tiles of 8x4) run with several tiles per workgroup: sampled
    pd_apply outputs (periodic seams included) against the definition evaluated one output at
    a time; 3 FP64 CG iterations equal the oracle's CG iterate (N = 0) or keep the recurrence
    and the recomputed residual consistent (N = 6); 3 FP32+refine iterations run."""
    import torch
    from scipy.sparse.linalg import LinearOperator
    for cells, N in [((2050, 2050), 0), ((1460, 1460), 6)]:
        print(f"large 2D grid cells={cells} N={N}", flush=True)
        L, dt = (1.0, 1.0), 5e-4
        g = Grid(cells, L, N)
        ctx = pd.pd_setup(2, cells, L, N, dt, 0.6, 1e-3)
        rng = np.random.default_rng(91)
        x = rng.standard_normal(g.ndof)
        y = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
        pd.pd_apply(ctx, 0, pd.PD_FP64, dev(x), y)
        xt = layout.blocked_to_tensor(x, cells, g.n)
        del x
        yt = layout.blocked_to_tensor(host(y), cells, g.n)
        del y
        shp = g.shape()
        idx = np.stack([rng.integers(0, s, size=200) for s in shp], axis=1)
        idx[:4] = 0
        idx[4:8] = np.array(shp) - 1
        ref = apply_at(g, xt, idx, 0.0, dt)
        got = yt[tuple(idx.T)]
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        del xt, yt
        b = synthetic.random_rhs(92, g.ndof)
        xs = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
        info = pd.pd_cg_solve(ctx, 0, pd.PD_FP64, dev(b), xs, 1e-30, 3)
        print(f"  fp64 {info}", flush=True)
        assert info["status"] == pd.PD_ENOCONV and info["iters"] == 3
        if N == 0:
            bt = project_null(g, layout.blocked_to_tensor(b, cells, g.n),
                              [null_basis_tiled(c, N) for c in cells])
            A = LinearOperator((g.ndof, g.ndof), dtype=np.float64,
                               matvec=lambda v: apply_operator(g, v, 0.0, dt).reshape(-1))
            x_ref, it, _ = cg(A, bt.reshape(-1), 1e-30, 3)
            got = layout.blocked_to_tensor(host(xs), cells, g.n).reshape(-1)
            assert np.linalg.norm(got - x_ref) <= 1e-12 * np.linalg.norm(x_ref)
        else:
            assert abs(info["rel_res_true"] - info["rel_res_recur"]) <= 1e-10
        xs.zero_()
        info = pd.pd_cg_solve(ctx, 0, pd.PD_FP32_REFINE64, dev(b), xs, 1e-30, 3)
        print(f"  fp32 refine {info}", flush=True)
        assert info["iters"] == 3 and np.isfinite(info["rel_res_true"])
        assert info["rel_res_true"] < 1.0
        del xs
        ctx.close()


def test_setup_rejects_too_many_3d_columns(pd):
    """A 3D workgroup owns one column of cells: a grid with more columns (4112^2 x 4 cells at
    N = 0, 16x16-cell columns: 66049) than one launch holds workgroups is refused at setup with
    PD_EINVAL, before any allocation."""
    with pytest.raises(pd.PdError) as e:
        pd.pd_setup(3, (4112, 4112, 4), (1.0, 1.0, 1.0), 0, 1e-3, 0.6, 1e-3)
    assert e.value.code == pd.PD_EINVAL


@pytest.mark.parametrize("dim,cells,N,dt,m,one", [(2, (256, 256), 6, 5e-4, 4, 0),
                                                   (2, (256, 256), 6, 5e-4, 5, 1),
                                                   (3, (64, 64, 64), 4, 1e-3, 2, 0)])
def test_full_size_cg_iterates_in_bench_configuration(pd, dim, cells, N, dt, m, one):
    """The fused CG kernels at full size in the launch configuration the benchmark times (256^2
    N = 6: three tiles per workgroup with the next tile's loads in flight; 64^3 N = 4: whole-column
    z segments), with the deferred x update (and, at 256^2, also in the opt-in one-kernel form at
    its own shape, four tiles per workgroup): after m FP64 iterations from x0 = 0 the iterate
    equals the oracle's plain CG iterate computed with the matrix-free oracle operator."""
    import torch
    from scipy.sparse.linalg import LinearOperator
    print(f"full-size CG iterates dim={dim} cells={cells} N={N} m={m} one={one}", flush=True)
    L = (1.0,) * dim
    g = Grid(cells, L, N)
    rng = np.random.default_rng(81)
    bt = project_null(g, rng.standard_normal(g.shape()), [null_basis_tiled(c, N) for c in cells])
    A = LinearOperator((g.ndof, g.ndof), dtype=np.float64,
                       matvec=lambda v: apply_operator(g, v, 0.0, dt).reshape(-1))
    x_ref, it, _ = cg(A, bt.reshape(-1), 1e-30, m)
    assert it == m
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, 1e-3)
    pd.pd_configure(ctx, pd.PD_CFG_ONE_KERNEL, one)
    x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    info = pd.pd_cg_solve(ctx, 0, pd.PD_FP64, dev(layout.tensor_to_blocked(bt, cells, g.n)), x,
                          1e-30, m)
    ctx.close()
    assert info["status"] == pd.PD_ENOCONV and info["iters"] == m
    got = layout.blocked_to_tensor(host(x), cells, g.n).reshape(-1)
    rel = np.linalg.norm(got - x_ref) / np.linalg.norm(x_ref)
    print(f"  relative difference {rel:.2e}", flush=True)
    assert rel <= 1e-12


# tolerances at which each path reaches the 1e-10 error target on a white-noise right-hand side
# with a margin (measured errors 3.2e-11 / 1.8e-11 at 256^2 N = 6, 4.7e-11 / 2.0e-11 at 64^3
# N = 4; the refined path's FP32 iterations leave more error in the smallest eigenmodes per unit
# residual than FP64 CG does)
WHITE_RTOL = {(2, 0): 2e-11, (2, 2): 2e-12, (3, 0): 5e-12, (3, 2): 2e-12}


@pytest.mark.parametrize("dim,cells,N,dt", [(2, (256, 256), 6, 5e-4), (3, (64, 64, 64), 4, 1e-3)])
def test_full_size_solves_match_direct_solution(pd, dim, cells, N, dt):
    """Full-size pressure solves (FP64 and FP32 + FP64 refinement, the benchmark's launch
    configuration) against the exact minimum-norm solution by fast diagonalisation, both at the
    error target 1e-10 (mass-weighted relative L2):
      * the workload's own kind of right-hand side, b = sum_d B_d U0_d of its seeded smooth
        initial velocity, at the benchmark's rtol 1e-10 (measured errors 1.7e-11 / 9.2e-11 at
        256^2 N = 6, 1.2e-11 / 4.2e-11 at 64^3 N = 4);
      * a white-noise right-hand side (every mode present) at the tolerance each path needs for
        the target (a residual bounds the error only up to cond(A), ~8e5 at 256^2 N = 6): at
        rtol 1e-10 the errors are 1.4e-10 / 1.1e-9 (2D) and 9.3e-10 / 4.1e-9 (3D).
    At every tolerance the oracle recomputes b - A x with its own matrix-free operator (<= 1.05
    rtol plus the rounding scale of an FP64 evaluation of it)."""
    import torch
    from oracle.operators import div_rhs_apply
    print(f"full-size solves dim={dim} cells={cells} N={N}", flush=True)
    L = (1.0,) * dim
    g = Grid(cells, L, N)
    cfg = synthetic.CONFIGS["rand2d_256_N6" if dim == 2 else "rand3d_64_N4"]
    field = synthetic.FourierField(cfg["seed"], dim, cfg["kmax"], L).normalise(cfg["vmax"])
    smooth = div_rhs_apply(g, field.eval(synthetic.staggered_coords(cells, L, g.tab.xi)))
    white = project_null(g, layout.blocked_to_tensor(synthetic.random_rhs(91, g.ndof), cells, g.n),
                         [null_basis_tiled(c, N) for c in cells])
    fd = FastDiag(g)
    ctx = pd.pd_setup(dim, cells, L, N, dt, 0.6, 1e-3)
    for kind, bt in (("workload", smooth), ("white", white)):
        ref = fd.solve(bt, 0.0, dt)
        b = layout.tensor_to_blocked(bt, cells, g.n)
        for prec in (pd.PD_FP64, pd.PD_FP32_REFINE64):
            rtol = 1e-10 if kind == "workload" else WHITE_RTOL[(dim, prec)]
            x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
            info = pd.pd_cg_solve(ctx, 0, prec, dev(b), x, rtol, 200000)
            assert info["status"] == pd.PD_OK, info
            X = layout.blocked_to_tensor(host(x), cells, g.n)
            rel = np.linalg.norm(bt - apply_operator(g, X, 0.0, dt)) / np.linalg.norm(bt)
            roundoff = 3 * (N + 1) * np.finfo(float).eps * \
                np.linalg.norm(apply_operator(g, X, 0.0, dt, absolute=True)) / np.linalg.norm(bt)
            err = mass_norm(g, X - ref) / mass_norm(g, ref)
            print(f"  {kind} rtol {rtol:.0e} prec {prec}: iters {info['iters']} residual {rel:.3e} "
                  f"(rounding scale {roundoff:.1e}) error vs direct {err:.2e}", flush=True)
            assert rel <= 1.05 * rtol + roundoff
            assert err <= 1e-10
    ctx.close()
