"""torch.autograd wrappers over the HIP pair sum and the checkpointed RK4
adjoint.  Forward and backward both run in libptrom; these classes only pass
tensors through."""
from __future__ import annotations

import torch

from . import native


class _Velocity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xy, gamma, delta):
        xy_c, g_c = xy.detach().contiguous(), gamma.detach().contiguous()
        ctx.save_for_backward(xy_c, g_c)
        ctx.delta = float(delta)
        return native.velocity(xy_c, g_c, ctx.delta)

    @staticmethod
    def backward(ctx, gf):
        xy, g = ctx.saved_tensors
        if gf is None:
            return None, None, None
        gx, gg = native.vjp(xy, g, ctx.delta, gf.contiguous())
        return gx, gg, None


def velocity(xy, gamma, delta):
    """Differentiable f(x; Gamma): backward is the adjoint pair kernel."""
    return _Velocity.apply(xy, gamma, delta)


class _RK4Flow(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xy0, gamma, delta, dt, nsteps, every):
        x0, g = xy0.detach().contiguous(), gamma.detach().contiguous()
        ckpt, xT = native.rk4_fwd_ckpt(x0, g, float(delta), float(dt), int(nsteps), int(every))
        ctx.save_for_backward(ckpt, g)
        ctx.args = (float(delta), float(dt), int(nsteps), int(every))
        return xT

    @staticmethod
    def backward(ctx, gxT):
        ckpt, g = ctx.saved_tensors
        if gxT is None:
            return None, None, None, None, None, None
        delta, dt, nsteps, every = ctx.args
        lam0, gg = native.rk4_bwd(ckpt, g, delta, dt, nsteps, every, gxT.contiguous())
        return lam0, gg, None, None, None, None


def rk4_flow(xy0, gamma, delta, dt, nsteps, every=20):
    """x(T) after ``nsteps`` RK4 steps; gradients with respect to x(0) and
    Gamma come from the discrete adjoint with checkpoints every ``every`` steps."""
    return _RK4Flow.apply(xy0, gamma, delta, dt, nsteps, every)


def angular_kinetic_qoi(xT, gamma, delta):
    """Q = 1/2 sum_i Gamma_i |x_i|^2 |f_i(x)|^2 (angular-impulse-weighted kinetic
    energy of the final state)."""
    n = gamma.numel()
    f = velocity(xT, gamma, delta)
    r2 = xT[:n] ** 2 + xT[n:] ** 2
    v2 = f[:n] ** 2 + f[n:] ** 2
    return 0.5 * (gamma * r2 * v2).sum()
