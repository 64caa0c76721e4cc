"""GPU parity of the hand-written adjoint: the transposed single operators through
<K x, y> = <x, K^T y>, the adjoint convection and the adjoint step against the oracle's
transposes element by element, and gradients of the kinetic energy through a checkpointed
rollout against the oracle's gradient.

Every case prints its parameters before touching the GPU so that a failure names its case."""
import numpy as np
import pytest

from oracle.operators import Grid
from oracle.step import dual_to_main
from oracle.adjoint import rk3_vjp, StepAdjoint, rollout_gradient
import synthetic

pytestmark = pytest.mark.gpu

CASES = [(2, (6, 5), (1.0, 0.8), 3), (2, (7, 4), (1.0, 1.0), 6), (3, (4, 3, 5), (1.0, 1.0, 1.2), 2),
         (3, (3, 4, 3), (1.0, 1.0, 1.0), 1)]
DT, THETA, NU = 1e-3, 0.6, 1e-2


def dev(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def setup(pd, dim, cells, lengths, N, nu=NU):
    ctx = pd.pd_setup(dim, cells, lengths, N, DT, THETA, nu)
    pd.pd_configure(ctx, pd.PD_CFG_P_RTOL, 1e-13)
    pd.pd_configure(ctx, pd.PD_CFG_V_RTOL, 1e-13)
    return ctx, Grid(cells, lengths, N)


def blocked(g, T):
    return synthetic.tensor_to_blocked(T, g.cells, g.n)


def tensor(g, v):
    return synthetic.blocked_to_tensor(v, g.cells, g.n)


@pytest.mark.parametrize("dim,cells,lengths,N", CASES)
def test_single_operator_transposes(pd, dim, cells, lengths, N):
    import torch
    print(f"transposes dim={dim} cells={cells} N={N}", flush=True)
    ctx, g = setup(pd, dim, cells, lengths, N)
    rng = np.random.default_rng(30 + N)
    X = [dev(rng.standard_normal(g.ndof)) for _ in range(dim)]
    Y = [dev(rng.standard_normal(g.ndof)) for _ in range(dim)]

    def ip(a, b):
        return float((a * b).sum())

    out = torch.empty(g.ndof, dtype=torch.float64, device="cuda")
    out2 = torch.empty_like(out)
    for d in range(dim):
        for direction in (0, 1):
            pd.pd_l2_project(ctx, d, direction, X[d], out)
            pd.pd_l2_project_adjoint(ctx, d, direction, Y[d], out2)
            lhs, rhs = ip(out, Y[d]), ip(X[d], out2)
            assert abs(lhs - rhs) <= 1e-13 * float(out.norm()) * float(Y[d].norm())
    # B: u -> b = sum_d B_d u_d
    b = torch.empty_like(out)
    pd.pd_rhs_div(ctx, X, b)
    ub = [torch.empty_like(out) for _ in range(dim)]
    pd.pd_rhs_div_adjoint(ctx, Y[0], ub)
    lhs = ip(b, Y[0])
    rhs = sum(ip(X[d], ub[d]) for d in range(dim))
    assert abs(lhs - rhs) <= 1e-13 * float(b.norm()) * float(Y[0].norm())
    # G: q -> u_d -= G_d q, so starting from u = 0 the output is -G q
    u0 = [torch.zeros_like(out) for _ in range(dim)]
    pd.pd_project_velocity(ctx, Y[1 % dim], u0)
    qbar = torch.empty_like(out)
    pd.pd_project_velocity_adjoint(ctx, X, qbar)
    lhs = sum(ip(u0[d], X[d]) for d in range(dim))
    rhs = ip(Y[1 % dim], qbar)
    assert abs(lhs - rhs) <= 1e-13 * float(qbar.norm()) * float(Y[1 % dim].norm())
    ctx.close()


@pytest.mark.parametrize("dim,cells,lengths,N", CASES)
def test_convect_adjoint_matches_oracle(pd, dim, cells, lengths, N):
    print(f"convect adjoint dim={dim} cells={cells} N={N}", flush=True)
    ctx, g = setup(pd, dim, cells, lengths, N)
    rng = np.random.default_rng(40 + N)
    Um = [0.5 * rng.standard_normal(g.shape()) for _ in range(dim)]
    Yb = [rng.standard_normal(g.shape()) for _ in range(dim)]
    ref = rk3_vjp(g, Um, DT, Yb)
    um = [dev(blocked(g, x)) for x in Um]
    ub = [dev(blocked(g, y)) for y in Yb]
    pd.pd_convect_adjoint(ctx, um, ub)
    for d in range(dim):
        got = tensor(g, host(ub[d]))
        assert np.abs(got - ref[d]).max() <= 1e-12 * np.abs(ref[d]).max()
        assert np.array_equal(host(um[d]), blocked(g, Um[d]))     # the state is left unchanged
    ctx.close()


@pytest.mark.parametrize("convection", [1, 0])
@pytest.mark.parametrize("dim,cells,lengths,N", CASES)
def test_step_adjoint_matches_oracle(pd, dim, cells, lengths, N, convection):
    print(f"step adjoint dim={dim} cells={cells} N={N} convection={convection}", flush=True)
    ctx, g = setup(pd, dim, cells, lengths, N)
    pd.pd_configure(ctx, pd.PD_CFG_CONVECTION, convection)
    rng = np.random.default_rng(50 + N)
    U = [0.5 * rng.standard_normal(g.shape()) for _ in range(dim)]
    Ub = [rng.standard_normal(g.shape()) for _ in range(dim)]
    ref = StepAdjoint(g, DT, THETA, NU).vjp(U, Ub, convection=bool(convection))
    u = [dev(blocked(g, x)) for x in U]
    ub = [dev(blocked(g, y)) for y in Ub]
    infos = pd.pd_step_adjoint(ctx, u, ub)
    assert all(i["status"] == pd.PD_OK for i in infos[:dim] + [infos[3]])
    num = np.sqrt(sum(np.sum((tensor(g, host(ub[d])) - ref[d]) ** 2) for d in range(dim)))
    den = np.sqrt(sum(np.sum(r ** 2) for r in ref))
    print(f"  relative difference {num / den:.2e}", flush=True)
    assert num <= 1e-10 * den
    ctx.close()


@pytest.mark.parametrize("dim,cells,lengths,N,steps,every", [(2, (6, 5), (1.0, 0.8), 3, 4, 2),
                                                             (3, (3, 4, 3), (1.0, 1.0, 1.0), 2, 3, 2)])
def test_rollout_gradient_matches_oracle(pd, dim, cells, lengths, N, steps, every):
    import torch
    from paper_1602_05806_amd.autograd import Rollout, kinetic_energy
    print(f"rollout gradient dim={dim} cells={cells} N={N} steps={steps}", flush=True)
    ctx, g = setup(pd, dim, cells, lengths, N)
    rng = np.random.default_rng(60 + N)
    U0 = [0.5 * rng.standard_normal(g.shape()) for _ in range(dim)]
    loss_ref, grad_ref = rollout_gradient(g, U0, steps, DT, THETA, NU)
    u0 = [dev(blocked(g, x)).requires_grad_(True) for x in U0]
    uT = Rollout.apply(ctx, steps, every, *u0)
    loss = kinetic_energy(ctx, uT)
    loss.backward()
    assert abs(float(loss.detach()) - loss_ref) <= 1e-11 * abs(loss_ref)
    num = np.sqrt(sum(np.sum((tensor(g, host(u0[d].grad)) - grad_ref[d]) ** 2) for d in range(dim)))
    den = np.sqrt(sum(np.sum(r ** 2) for r in grad_ref))
    print(f"  gradient relative difference {num / den:.2e}", flush=True)
    assert num <= 1e-9 * den
    ctx.close()


def _c5_like(pd, cells, steps, every, dirs, tol, smooth):
    """Gradient of the final kinetic energy with respect to the initial velocity through the
    checkpointed rollout, against central finite differences of the forward rollout on seeded
    directions (seed 5000 + k), eps = 1e-6 ||U0|| / ||v||; solves to 1e-13. smooth: random
    Fourier fields of the initial velocity's family (wavenumbers <= 6); else N(0,1) per DoF."""
    import torch
    from paper_1602_05806_amd.autograd import Rollout, kinetic_energy
    cfg = synthetic.CONFIGS["adjoint3d_48_N3"]
    N = cfg["N"]
    ctx = pd.pd_setup(3, cells, cfg["lengths"], N, cfg["dt"], cfg["theta"], cfg["nu"])
    pd.pd_configure(ctx, pd.PD_CFG_P_RTOL, 1e-13)
    pd.pd_configure(ctx, pd.PD_CFG_V_RTOL, 1e-13)
    xi, _ = pd.pd_nodes(ctx)
    field = synthetic.FourierField(cfg["seed"], 3, cfg["kmax"], cfg["lengths"])
    field.normalise(cfg["vmax"])
    U = field.eval(synthetic.staggered_coords(cells, cfg["lengths"], xi))
    u0 = [torch.tensor(synthetic.tensor_to_blocked(x, cells, N + 1), device="cuda") for x in U]

    def loss_of(u):
        with torch.no_grad():
            return float(kinetic_energy(ctx, Rollout.apply(ctx, steps, every, *u)))

    ur = [x.clone().requires_grad_(True) for x in u0]
    loss = kinetic_energy(ctx, Rollout.apply(ctx, steps, every, *ur))
    loss.backward()
    grad = [x.grad for x in ur]
    unorm = float(torch.sqrt(sum((x * x).sum() for x in u0)))
    worst = 0.0
    coords = synthetic.staggered_coords(cells, cfg["lengths"], xi)
    for k in dirs:
        if smooth:
            fk = synthetic.FourierField(5000 + k, 3, cfg["kmax"], cfg["lengths"])
            fk.normalise(1.0)
            v = [torch.tensor(synthetic.tensor_to_blocked(x, cells, N + 1), device="cuda")
                 for x in fk.eval(coords)]
        else:
            g = torch.Generator(device="cpu").manual_seed(5000 + k)
            v = [torch.randn(x.numel(), generator=g, dtype=torch.float64).to("cuda") for x in u0]
        vnorm = float(torch.sqrt(sum((x * x).sum() for x in v)))
        eps = 1e-6 * unorm / vnorm
        fp = loss_of([a + eps * b for a, b in zip(u0, v)])
        fm = loss_of([a - eps * b for a, b in zip(u0, v)])
        fd = (fp - fm) / (2 * eps)
        gv = float(sum((a * b).sum() for a, b in zip(grad, v)))
        rel = abs(gv - fd) / abs(fd)
        worst = max(worst, rel)
        print(f"  direction {k}: grad.v {gv:.12e} fd {fd:.12e} rel {rel:.2e}", flush=True)
    ctx.close()
    assert worst <= tol


def test_gradient_fd_small_3d(pd):
    """16 white-noise directions, 20 steps with checkpoints every 5, on 12^3 cells of the 48^3
    N=3 setting."""
    print("adjoint FD 12^3 N=3, 20 steps, 16 white-noise directions", flush=True)
    _c5_like(pd, (12, 12, 12), 20, 5, range(16), 1e-6, smooth=False)


@pytest.mark.parametrize("first", [0, 4, 8, 12])
def test_gradient_fd_full_48(pd, first):
    """The full 48^3 N=3 workload (7.1M DoFs per component), 20 steps, checkpoints every 5, on the
    16 smooth random directions (seeds 5000..5015), four per test so that each test stays short.
    White-noise directions are not used at this size: their directional derivatives are ~1e-3
    smaller relative to |grad| |v|, and a perturbation of 1e-6 ||U0|| then crosses enough kinks of
    the Rusanov speed max(|v-|, |v+|) (face jumps of a smooth 48^3 flow are tiny) for central
    differences to miss by up to a few 1e-6 (measured), independently of the adjoint."""
    print(f"adjoint FD 48^3 N=3, 20 steps, smooth directions {first}..{first + 3}", flush=True)
    _c5_like(pd, (48, 48, 48), 20, 5, range(first, first + 4), 1e-6, smooth=True)


@pytest.mark.parametrize("dim,cells,lengths,N", CASES)
def test_kinetic_energy_and_cotangent(pd, dim, cells, lengths, N):
    """pd_kinetic_energy against the oracle's energy and its gradient (both pinned on the CPU by
    closed forms and differences), element by element for the cotangent gscale * W u / ncells."""
    import torch
    from oracle.step import kinetic_energy, kinetic_energy_grad
    print(f"kinetic energy dim={dim} cells={cells} N={N}", flush=True)
    ctx, g = setup(pd, dim, cells, lengths, N)
    rng = np.random.default_rng(70 + N)
    U = [rng.standard_normal(g.shape()) for _ in range(dim)]
    u = [dev(blocked(g, x)) for x in U]
    e = pd.pd_kinetic_energy(ctx, u)
    ref = kinetic_energy(g, U)
    assert abs(e - ref) <= 1e-13 * abs(ref)
    grads = [torch.full_like(x, float("nan")) for x in u]
    gscale = 0.7
    e2 = pd.pd_kinetic_energy(ctx, u, grads, gscale)
    assert e2 == e
    gref = kinetic_energy_grad(g, U)
    for d in range(dim):
        got = tensor(g, host(grads[d]))
        assert np.abs(got - gscale * gref[d]).max() <= 1e-14 * np.abs(gref[d]).max()
    with pytest.raises(pd.PdError):
        pd.pd_kinetic_energy(ctx, u, u, 1.0)
    ctx.close()
