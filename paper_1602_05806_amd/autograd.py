"""torch.autograd bindings of the fractional step and its hand-written adjoint.

Argument marshalling only: the forward runs pd_step and the backward pd_step_adjoint of libpd
(arXiv:1602.05806 Section 2.1-2.3 for the step; the adjoint is the transposed linearisation of
that step, see include/pd.h). The velocity is a tuple of dual components (FP64 CUDA tensors in
the element-blocked layout); the pressure does not influence the velocity and is not
differentiated.

  Step.apply(ctx, *u)                      one step, all intermediate data recomputed in backward
  Rollout.apply(ctx, steps, every, *u0)    `steps` steps; the forward keeps U every `every` steps
                                           (checkpoints), the backward recomputes each segment
                                           from its checkpoint and runs the adjoint in reverse
  kinetic_energy(ctx, u)                   the mean kinetic energy (1/|Omega|) int |v|^2 / 2 with
                                           each component integrated by GL quadrature on its grid
                                           (pd_kinetic_energy; its backward is the library's
                                           cotangent W u / ncells)
"""
import torch

from . import pd_kinetic_energy, pd_step, pd_step_adjoint, PD_OK, PdError


# solver work done through this module (forward steps, recomputed steps, adjoint steps)
stats = {"steps": 0, "adjoint_steps": 0, "pressure_iters": 0, "viscous_iters": 0}


def _check(infos, what, dim):
    for i in infos[:dim] + [infos[3]]:
        if i["status"] != PD_OK:
            raise PdError(i["status"], f"{what}: solve failed ({i})")
    stats["pressure_iters"] += infos[3]["iters"]
    stats["viscous_iters"] += sum(i["iters"] for i in infos[:dim])


def _step_inplace(ctx, u, p):
    _check(pd_step(ctx, u, p), "pd_step", ctx.dim)
    stats["steps"] += 1


def _adjoint_inplace(ctx, u, ubar):
    _check(pd_step_adjoint(ctx, u, ubar), "pd_step_adjoint", ctx.dim)
    stats["adjoint_steps"] += 1


class Step(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx, *u):
        out = [x.detach().clone() for x in u]
        p = torch.zeros_like(out[0])
        _step_inplace(ctx, out, p)
        fctx.pd = ctx
        fctx.save_for_backward(*u)
        return tuple(out)

    @staticmethod
    def backward(fctx, *gout):
        u = [x.detach().contiguous() for x in fctx.saved_tensors]
        ubar = [torch.zeros_like(u[0]) if g is None else g.detach().clone().contiguous()
                for g in gout]
        _adjoint_inplace(fctx.pd, u, ubar)
        return (None, *ubar)


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx, steps, every, *u0):
        if steps < 0 or every < 1:
            raise ValueError("steps >= 0 and every >= 1 required")
        u = [x.detach().clone() for x in u0]
        p = torch.zeros_like(u[0])
        ckpt = {0: [x.clone() for x in u]}
        for n in range(steps):
            _step_inplace(ctx, u, p)
            if (n + 1) % every == 0 and n + 1 < steps:
                ckpt[n + 1] = [x.clone() for x in u]
        fctx.pd = ctx
        fctx.steps = steps
        fctx.every = every
        fctx.ckpt = ckpt
        return tuple(u)

    @staticmethod
    def backward(fctx, *gout):
        ctx, steps, every, ckpt = fctx.pd, fctx.steps, fctx.every, fctx.ckpt
        ref = ckpt[0][0]
        ubar = [torch.zeros_like(ref) if g is None else g.detach().clone().contiguous()
                for g in gout]
        for start in sorted(ckpt, reverse=True):
            end = min(start + every, steps)
            # forward states U^start .. U^{end-1} of this segment, from its checkpoint
            u = [x.clone() for x in ckpt[start]]
            p = torch.zeros_like(ref)
            states = [[x.clone() for x in u]]
            for _ in range(start, end - 1):
                _step_inplace(ctx, u, p)
                states.append([x.clone() for x in u])
            for k in range(end - start - 1, -1, -1):
                _adjoint_inplace(ctx, states[k], ubar)
            del states
        return (None, None, None, *ubar)


class KineticEnergy(torch.autograd.Function):
    """Loss K(U) of pd_kinetic_energy; its backward asks the library for gscale * dK/dU."""

    @staticmethod
    def forward(fctx, ctx, *u):
        fctx.pd = ctx
        fctx.save_for_backward(*u)
        e = pd_kinetic_energy(ctx, [x.detach().contiguous() for x in u])
        return torch.tensor(e, dtype=torch.float64, device=u[0].device)

    @staticmethod
    def backward(fctx, g):
        u = [x.detach().contiguous() for x in fctx.saved_tensors]
        grads = [torch.empty_like(x) for x in u]
        pd_kinetic_energy(fctx.pd, u, grads, float(g))
        return (None, *grads)


def kinetic_energy(ctx, u):
    """(1/|Omega|) int |v|^2 / 2 of the dual velocity u, differentiable (pd_kinetic_energy)."""
    return KineticEnergy.apply(ctx, *u)
