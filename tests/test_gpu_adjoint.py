"""GPU parity of the checkpointed discrete RK4 adjoint and its autograd
wrapper against the FP64 oracle adjoint (gate 1e-4 relative L2 on gradients)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2103_01983_amd import native
from paper_2103_01983_amd import workloads as W
from paper_2103_01983_amd import autograd as AG

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.mark.parametrize("n,steps,every", [(300, 10, 3), (1031, 8, 8), (64, 5, 20)])
def test_rk4_adjoint_parity(dev, n, steps, every):
    c = W.shear_layer(n, seed=5 + n, delta=0.02)
    xy, g = f32(c.xy), f32(c.gamma * (1 + np.random.default_rng(1).random(n)))
    dt = float(np.float32(5e-3))
    lamT = f32(W.random_vectors(n, 1, 3)[0])
    ggd = f32(np.random.default_rng(2).standard_normal(n))
    x0 = torch.tensor(xy, dtype=torch.float32, device=dev)
    gd = torch.tensor(g, dtype=torch.float32, device=dev)
    ck, xT = native.rk4_fwd_ckpt(x0, gd, 0.02, dt, steps, every)
    lam0, gg = native.rk4_bwd(ck, gd, 0.02, dt, steps, every, torch.tensor(lamT, dtype=torch.float32, device=dev),
                              torch.tensor(ggd, dtype=torch.float32, device=dev))
    oT, olam, ogg = oracle.rk4_adjoint(xy, g, float(np.float32(0.02)), dt, steps, lamT, ggd)
    assert rel(xT.cpu().numpy() - xy, oT - xy) <= 1e-4
    assert rel(lam0.cpu().numpy(), olam) <= 1e-4
    assert rel(gg.cpu().numpy() - ggd, ogg - ggd) <= 1e-4


def test_linear_impulse_gradient_exact(dev):
    # P(T) = sum_i G_i x_i(T) is preserved by RK4: dP/dx(0) = (G, 0), dP/dG = x(0).
    n = 2048
    c = W.shear_layer(n, seed=8, delta=0.01)
    xy, g = f32(c.xy), f32(c.gamma)
    x0 = torch.tensor(xy, dtype=torch.float32, device=dev)
    gd = torch.tensor(g, dtype=torch.float32, device=dev)
    ck, xT = native.rk4_fwd_ckpt(x0, gd, 0.01, 5e-4, 40, 20)
    lamT = torch.cat([gd, torch.zeros_like(gd)])
    lam0, gg = native.rk4_bwd(ck, gd, 0.01, 5e-4, 40, 20, lamT, xT[:n].contiguous())
    assert rel(lam0.cpu().numpy(), lamT.cpu().numpy()) <= 1e-6
    assert rel(gg.cpu().numpy(), xy[:n]) <= 1e-6


def test_autograd_qoi_gradient(dev):
    # Q = 1/2 sum_i G_i |x_i(T)|^2 |f_i(x(T))|^2 through 20 RK4 steps with
    # checkpoints every 5 steps, versus the oracle's discrete adjoint.
    n, steps, every, dt, d = 512, 20, 5, float(np.float32(5e-4)), 0.02
    c = W.shear_layer(n, seed=21, delta=d)
    xy, g = f32(c.xy), f32(c.gamma)
    x0 = torch.tensor(xy, dtype=torch.float32, device=dev, requires_grad=True)
    gd = torch.tensor(g, dtype=torch.float32, device=dev, requires_grad=True)
    Q = AG.angular_kinetic_qoi(AG.rk4_flow(x0, gd, d, dt, steps, every), gd, d)
    Q.backward()
    # oracle: dQ/dx(T) and the direct Gamma partial, then the discrete adjoint
    dfl = float(np.float32(d))
    xT = oracle.rk4(xy, g, dfl, dt, steps)
    fT = oracle.velocity(xT, g, dfl)
    r2 = xT[:n] ** 2 + xT[n:] ** 2
    v2 = fT[:n] ** 2 + fT[n:] ** 2
    w = np.concatenate([g * r2 * fT[:n], g * r2 * fT[n:]])
    jw, gw = oracle.vjp(xT, g, dfl, w)
    lamT = np.concatenate([g * v2 * xT[:n], g * v2 * xT[n:]]) + jw
    ggd = 0.5 * r2 * v2 + gw
    _, olam, ogg = oracle.rk4_adjoint(xy, g, dfl, dt, steps, lamT, ggd)
    Qo = 0.5 * np.sum(g * r2 * v2)
    assert abs(Q.item() - Qo) <= 1e-5 * abs(Qo)
    assert rel(x0.grad.cpu().numpy(), olam) <= 1e-4
    assert rel(gd.grad.cpu().numpy(), ogg) <= 1e-4


def test_velocity_function_backward(dev):
    n = 700
    c = W.disk_cloud(n, seed=4, delta=0.02)
    xy, g = f32(c.xy), f32(c.gamma)
    x = torch.tensor(xy, dtype=torch.float32, device=dev, requires_grad=True)
    gd = torch.tensor(g, dtype=torch.float32, device=dev, requires_grad=True)
    w = f32(W.random_vectors(n, 1, 5)[0])
    f = AG.velocity(x, gd, 0.02)
    (f * torch.tensor(w, dtype=torch.float32, device=dev)).sum().backward()
    ox, og = oracle.vjp(xy, g, float(np.float32(0.02)), w)
    assert rel(x.grad.cpu().numpy(), ox) <= 1e-5
    assert rel(gd.grad.cpu().numpy(), og) <= 1e-5


def test_linear_impulse_gradient_c5_full_config(dev):
    # the adjoint configuration at full size: N = 131072 shear layer, 200 RK4
    # steps at dt 5e-4, checkpoints every 20.  P(T) = sum_i G_i x_i(T) is an
    # invariant of every RK step, so its exact gradient is dP/dx(0) = (G, 0)
    # and dP/dG = x(0); no oracle run is needed at this size.
    cfg = W.CONFIGS["c5_adjoint"]
    c = W.config_cloud("c5_adjoint")
    n = c.n
    xy, g = f32(c.xy), f32(c.gamma)
    x0 = torch.tensor(xy, dtype=torch.float32, device=dev)
    gd = torch.tensor(g, dtype=torch.float32, device=dev)
    ck, xT = native.rk4_fwd_ckpt(x0, gd, c.delta, cfg["dt"], cfg["steps"], cfg["every"])
    assert ck.numel() == cfg["steps"] // cfg["every"] * 2 * n
    lamT = torch.cat([gd, torch.zeros_like(gd)])
    lam0, gg = native.rk4_bwd(ck, gd, c.delta, cfg["dt"], cfg["steps"], cfg["every"], lamT, xT[:n].contiguous())
    assert rel(lam0.cpu().numpy(), lamT.cpu().numpy()) <= 1e-4
    assert rel(gg.cpu().numpy(), xy[:n]) <= 1e-4
    # and the y component: dP_y/dx(0) = (0, G), dP_y/dG = y(0)
    lamT = torch.cat([torch.zeros_like(gd), gd])
    lam0, gg = native.rk4_bwd(ck, gd, c.delta, cfg["dt"], cfg["steps"], cfg["every"], lamT, xT[n:].contiguous())
    assert rel(lam0.cpu().numpy(), lamT.cpu().numpy()) <= 1e-4
    assert rel(gg.cpu().numpy(), xy[n:]) <= 1e-4


def test_qoi_gradient_c5_steps_reduced_n(dev):
    # the adjoint configuration's QoI, step count, step and checkpoint spacing
    # (200 RK4 steps at dt 5e-4, every 20) on the shear layer at N = 4096,
    # through the autograd wrappers, against the oracle's FP64 discrete adjoint
    cfg = W.CONFIGS["c5_adjoint"]
    c = W.config_cloud("c5_adjoint", n=4096)
    n, d, dt = c.n, c.delta, float(np.float32(cfg["dt"]))
    xy, g = f32(c.xy), f32(c.gamma)
    x0 = torch.tensor(xy, dtype=torch.float32, device=dev, requires_grad=True)
    gd = torch.tensor(g, dtype=torch.float32, device=dev, requires_grad=True)
    Q = AG.angular_kinetic_qoi(AG.rk4_flow(x0, gd, d, dt, cfg["steps"], cfg["every"]), gd, d)
    Q.backward()
    dfl = float(np.float32(d))
    xT = oracle.rk4(xy, g, dfl, dt, cfg["steps"])
    fT = oracle.velocity(xT, g, dfl)
    r2 = xT[:n] ** 2 + xT[n:] ** 2
    v2 = fT[:n] ** 2 + fT[n:] ** 2
    w = np.concatenate([g * r2 * fT[:n], g * r2 * fT[n:]])
    jw, gw = oracle.vjp(xT, g, dfl, w)
    lamT = np.concatenate([g * v2 * xT[:n], g * v2 * xT[n:]]) + jw
    ggd = 0.5 * r2 * v2 + gw
    _, olam, ogg = oracle.rk4_adjoint(xy, g, dfl, dt, cfg["steps"], lamT, ggd)
    Qo = 0.5 * np.sum(g * r2 * v2)
    assert abs(Q.item() - Qo) <= 1e-5 * abs(Qo)
    assert rel(x0.grad.cpu().numpy(), olam) <= 1e-4
    assert rel(gd.grad.cpu().numpy(), ogg) <= 1e-4
