"""GPU parity on seeded random shapes: the operator apply and fixed-count CG iterates against the
oracle on grid sizes, degrees, boundary masks, cell lengths and precisions drawn from a fixed
seed, so that tile tails, grids narrower than a tile, single-cell directions, walls on any subset
of directions and every kernel form (2D tiles, the 3D z-line and coalesced forms, the wall forms)
meet in combinations the hand-picked cases do not list.

Every case prints its parameters before touching the GPU so that a failure names its case."""
import numpy as np
import pytest

from oracle import layout
from oracle.operators import Grid, null_bases, pressure_operator, project_null, viscous_operator
from oracle.solvers import FastDiag, cg
import synthetic

pytestmark = pytest.mark.gpu

MAX_DOFS = 40000


def _draw(seed, count, min_dofs=1):
    """`count` cases (dim, cells, lengths, N, mask) from a fixed seed, min_dofs..MAX_DOFS DoFs."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        dim = int(rng.integers(2, 4))
        N = int(rng.integers(0, 9 if dim == 2 else 7))
        hi = 26 if dim == 2 else 9
        cells = tuple(int(rng.integers(1, hi)) for _ in range(dim))
        if not min_dofs <= int(np.prod(cells)) * (N + 1) ** dim <= MAX_DOFS:
            continue
        lengths = tuple(float(rng.uniform(0.5, 2.0)) for _ in range(dim))
        # fully periodic in 2 of 5 cases (the periodic kernel forms), else any wall subset
        mask = (1 << dim) - 1 if rng.random() < 0.4 else int(rng.integers(0, 1 << dim))
        out.append((dim, cells, lengths, N, mask))
    return out


APPLY = _draw(20261203, 40)
ITER = _draw(1203, 16, min_dofs=300)   # (no Krylov space exhausted within 12 iterations)
SOLVE = _draw(3012, 12, min_dofs=300)


def _dev(a, dtype=None):
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype or torch.float64, device="cuda")


def _host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _flags(dim, mask):
    return tuple(bool((mask >> d) & 1) for d in range(dim))


@pytest.mark.parametrize("case", range(len(APPLY)))
def test_apply_random_shapes(pd, case):
    """pd_apply of both operators against the assembled oracle matrix: FP64 within 1e-13 of the
    largest output, FP32 within 3e-6 in norm."""
    import torch
    dim, cells, lengths, N, mask = APPLY[case]
    print(f"random apply {case}: dim={dim} cells={cells} N={N} mask={mask:b} "
          f"lengths={tuple(round(v, 3) for v in lengths)}", flush=True)
    dt, nu = 1e-3, 0.21
    g = Grid(cells, lengths, N, periodic=_flags(dim, mask))
    ctx = pd.pd_setup(dim, cells, lengths, N, dt, 0.6, nu, periodic_mask=mask)
    rng = np.random.default_rng(500 + case)
    x = rng.standard_normal(g.ndof)
    xt = layout.blocked_to_tensor(x, cells, g.n).reshape(-1)
    for op in (0, 1):
        A = pressure_operator(g, dt) if op == 0 else viscous_operator(g, dt, nu)
        ref = layout.tensor_to_blocked(A @ xt, cells, g.n)
        y = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
        pd.pd_apply(ctx, op, pd.PD_FP64, _dev(x), y)
        assert np.abs(_host(y) - ref).max() <= 1e-13 * np.abs(ref).max(), f"op {op} FP64"
        y32 = torch.empty(g.ndof, dtype=torch.float32, device="cuda")
        pd.pd_apply(ctx, op, pd.PD_FP32, _dev(x, torch.float32), y32)
        assert np.linalg.norm(_host(y32) - ref) <= 3e-6 * np.linalg.norm(ref), f"op {op} FP32"
    ctx.close()


@pytest.mark.parametrize("case", range(len(ITER)))
def test_cg_iterates_random_shapes(pd, case):
    """After exactly 12 FP64 iterations from x0 = 0 (maxit = 12) on a right-hand side in the
    operator's range, the GPU iterate equals the oracle's plain CG iterate within 1e-12."""
    import torch
    dim, cells, lengths, N, mask = ITER[case]
    print(f"random cg {case}: dim={dim} cells={cells} N={N} mask={mask:b}", flush=True)
    m, dt = 12, 5e-4
    g = Grid(cells, lengths, N, periodic=_flags(dim, mask))
    A = pressure_operator(g, dt)
    bt = layout.blocked_to_tensor(synthetic.random_rhs(700 + case, g.ndof), cells, g.n)
    bt = project_null(g, bt, null_bases(g))
    x_ref, it, _ = cg(A, bt.reshape(-1), 1e-30, m)
    assert it == m
    ctx = pd.pd_setup(dim, cells, lengths, N, dt, 0.6, 1e-2, periodic_mask=mask)
    x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
    info = pd.pd_cg_solve(ctx, 0, pd.PD_FP64, _dev(layout.tensor_to_blocked(bt, cells, g.n)), x,
                          1e-30, m)
    ctx.close()
    assert info["status"] == pd.PD_ENOCONV and info["iters"] == m
    got = layout.blocked_to_tensor(_host(x), cells, g.n).reshape(-1)
    assert np.linalg.norm(got - x_ref) <= 1e-12 * np.linalg.norm(x_ref)


def _mass_norm(g, T):
    W = np.ones(g.shape())
    for d in range(g.dim):
        shp = [1] * g.dim
        shp[g.dim - 1 - d] = -1
        W = W * np.tile(g.tab.w, g.cells[d]).reshape(shp)
    return np.sqrt(np.sum(W * T ** 2))


@pytest.mark.parametrize("case", range(len(SOLVE)))
def test_solves_random_shapes(pd, case):
    """Pressure solves to rtol 1e-12 (FP64, FP32+refine, and FP64 with the cell-block Jacobi
    preconditioner) of an unprojected random right-hand side reach the oracle's
    fast-diagonalisation minimum-norm solution (mass-weighted error <= 1e-9)."""
    import torch
    dim, cells, lengths, N, mask = SOLVE[case]
    print(f"random solve {case}: dim={dim} cells={cells} N={N} mask={mask:b}", flush=True)
    dt = 5e-4
    g = Grid(cells, lengths, N, periodic=_flags(dim, mask))
    b = synthetic.random_rhs(900 + case, g.ndof)
    ref = FastDiag(g).solve(layout.blocked_to_tensor(b, cells, g.n), 0.0, dt)
    ctx = pd.pd_setup(dim, cells, lengths, N, dt, 0.6, 1e-2, periodic_mask=mask)
    for prec, pc in ((pd.PD_FP64, 0), (pd.PD_FP32_REFINE64, 0), (pd.PD_FP64, 1)):
        pd.pd_configure(ctx, pd.PD_CFG_PRECOND, pc)
        x = torch.zeros(g.ndof, dtype=torch.float64, device="cuda")
        info = pd.pd_cg_solve(ctx, 0, prec, _dev(b), x, 1e-12, 400000)
        got = layout.blocked_to_tensor(_host(x), cells, g.n)
        err = _mass_norm(g, got - ref) / _mass_norm(g, ref)
        print(f"  prec={prec} precond={pc}: {info['iters']} it, true {info['rel_res_true']:.1e}, "
              f"error {err:.1e}", flush=True)
        assert info["status"] == pd.PD_OK
        assert info["rel_res_true"] <= 2e-12
        assert err <= 1e-9
    ctx.close()


def _draw_batch(seed, count):
    """`count` periodic 2D problems (cells, lengths, N) from a fixed seed, 300..20000 DoFs each."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        N = int(rng.integers(0, 9))
        cells = (int(rng.integers(1, 40)), int(rng.integers(1, 40)))
        if not 300 <= cells[0] * cells[1] * (N + 1) ** 2 <= 20000:
            continue
        out.append((cells, (float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.5, 2.0))), N))
    return out


BATCH = _draw_batch(4251, 14)   # (degrees 0, 1, 2, 4, 5, 6, 7, 8)


@pytest.mark.parametrize("mode", ["fp64", "refine", "pcg"])
def test_batch_random_mix(pd, mode):
    """A batch of 14 periodic 2D problems of seeded random sizes, cell lengths and degrees (every
    problem its own tile shape and iteration count) solved to rtol 1e-12 in FP64, FP32+refine or
    preconditioned FP64: each problem reaches the oracle's minimum-norm solution (<= 1e-9)."""
    import torch
    print(f"batch random mix {mode}: {[(c, N) for c, _, N in BATCH]}", flush=True)
    dt = 5e-4
    B = pd.pd_batch_setup([c for c, _, _ in BATCH], [ln for _, ln, _ in BATCH],
                          [N for _, _, N in BATCH], dt)
    pd.pd_batch_configure(B, pd.PD_BCFG_PRECOND, 1 if mode == "pcg" else 0)
    parts = [synthetic.random_rhs(1500 + j, c[0] * c[1] * (N + 1) ** 2)
             for j, (c, _, N) in enumerate(BATCH)]
    x = torch.zeros(B.total, dtype=torch.float64, device="cuda")
    prec = pd.PD_FP32_REFINE64 if mode == "refine" else pd.PD_FP64
    rc, infos = pd.pd_batch_cg_solve(B, prec, _dev(np.concatenate(parts)), x, 1e-12, 400000)
    xh = _host(x)
    offs = list(B.offsets)
    B.close()
    assert rc == pd.PD_OK, infos
    for j, (cells, lengths, N) in enumerate(BATCH):
        g = Grid(cells, lengths, N)
        ref = FastDiag(g).solve(layout.blocked_to_tensor(parts[j], cells, N + 1), 0.0, dt)
        got = layout.blocked_to_tensor(xh[offs[j]:offs[j + 1]], cells, N + 1)
        err = _mass_norm(g, got - ref) / _mass_norm(g, ref)
        print(f"  problem {j}: cells={cells} N={N} {infos[j]['iters']} it, "
              f"true {infos[j]['rel_res_true']:.1e}, error {err:.1e}", flush=True)
        assert infos[j]["status"] == pd.PD_OK
        # (the FP64 evaluation of b - A x for the N = 7, 8 problems has a rounding floor near
        # 1e-12: the FP64 batch ends there, e.g. 1.9e-12 for 8 x 14 cells at N = 7)
        assert infos[j]["rel_res_true"] <= 1e-11
        assert err <= 1e-9
