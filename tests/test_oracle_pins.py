"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(hand-worked values, closed-form vortex motions, invariants, equivariances,
finite differences, dot-product identities).  CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2103_01983_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------- velocity

def test_hand_worked_values():
    with open(os.path.join(GOLDEN, "hand_pairs.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        xy = np.array(c["x"] + c["y"])
        f = oracle.velocity(xy, np.array(c["gamma"]), c["delta"])
        n = len(c["x"])
        np.testing.assert_allclose(f[:n], c["f_x"], rtol=0, atol=1e-14, err_msg=c["name"])
        np.testing.assert_allclose(f[n:], c["f_y"], rtol=0, atol=1e-14, err_msg=c["name"])


@pytest.mark.parametrize("delta", [0.0, 0.3])
def test_two_vortex_rigid_rotation(delta):
    # Rigid counter-clockwise rotation about the circulation centroid at
    # omega = (G1 + G2) / (2 pi (d^2 + delta^2)).
    g = np.array([0.7, 1.9])
    p1, p2 = np.array([0.3, -0.2]), np.array([-0.5, 0.4])
    d2 = np.sum((p1 - p2) ** 2)
    xy = np.array([p1[0], p2[0], p1[1], p2[1]])
    f = oracle.velocity(xy, g, delta)
    omega = g.sum() / (2 * math.pi * (d2 + delta ** 2))
    c = (g[0] * p1 + g[1] * p2) / g.sum()
    for i, p in enumerate([p1, p2]):
        expect = omega * np.array([-(p - c)[1], (p - c)[0]])
        np.testing.assert_allclose([f[i], f[2 + i]], expect, rtol=1e-14, atol=1e-15)


def test_two_vortex_opposite_pair_translates():
    # G1 = -G2: both bodies translate perpendicular to the separation with
    # speed (G/2pi) d/(d^2 + delta^2).
    G, d, delta = 1.3, 0.8, 0.25
    xy = np.array([0.0, d, 0.0, 0.0])
    f = oracle.velocity(xy, np.array([G, -G]), delta)
    speed = G / (2 * math.pi) * d / (d * d + delta * delta)
    np.testing.assert_allclose(f, [0.0, 0.0, speed, speed], atol=1e-15)


@pytest.mark.parametrize("N,delta", [(3, 0.0), (5, 0.0), (6, 0.1), (9, 0.05)])
def test_polygon_rotation(N, delta):
    # N equal vortices on a circle of radius R rotate rigidly at
    # omega = (G/2pi) sum_m (1 - cos t_m) / (2R^2 (1 - cos t_m) + delta^2), t_m = 2 pi m / N,
    # which is G (N-1)/(4 pi R^2) at delta = 0.
    G, R = 0.9, 0.7
    t = 2 * math.pi * np.arange(N) / N + 0.3
    xy = np.concatenate([R * np.cos(t), R * np.sin(t)])
    f = oracle.velocity(xy, np.full(N, G), delta)
    tm = 2 * math.pi * np.arange(1, N) / N
    omega = G / (2 * math.pi) * np.sum((1 - np.cos(tm)) / (2 * R * R * (1 - np.cos(tm)) + delta ** 2))
    if delta == 0.0:
        assert omega == pytest.approx(G * (N - 1) / (4 * math.pi * R * R), rel=1e-14)
    np.testing.assert_allclose(f, omega * np.concatenate([-xy[N:], xy[:N]]), rtol=0, atol=1e-14)


def test_invariants_and_self_interaction():
    cl = W.disk_cloud(300, seed=5)
    xy, g = cl.xy, cl.gamma
    g = g + 0.1  # nonzero total circulation
    n = g.size
    f = oracle.velocity(xy, g, 0.02)
    scale = np.abs(g).sum() * np.abs(f).max()
    # linear impulse sum_i G_i f_i = 0 and angular impulse sum_i G_i x_i . f_i = 0
    assert abs(np.dot(g, f[:n])) < 1e-12 * scale
    assert abs(np.dot(g, f[n:])) < 1e-12 * scale
    assert abs(np.dot(g, xy[:n] * f[:n] + xy[n:] * f[n:])) < 1e-12 * scale
    # f_i does not depend on Gamma_i
    g2 = g.copy(); g2[17] += 3.0
    f2 = oracle.velocity(xy, g2, 0.02)
    assert f2[17] == f[17] and f2[n + 17] == f[n + 17]
    # a body of zero circulation changes nothing for the others
    xy3 = np.concatenate([xy[:n], [0.123], xy[n:], [-0.456]])
    f3 = oracle.velocity(xy3, np.concatenate([g, [0.0]]), 0.02)
    np.testing.assert_array_equal(np.concatenate([f3[:n], f3[n + 1:2 * n + 1]]), f)


def test_equivariance():
    cl = W.gaussian_patch(200, seed=7)
    xy, g, d = cl.xy, cl.gamma, 0.03
    n = g.size
    f = oracle.velocity(xy, g, d)
    a = 0.77
    R = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
    P = R @ np.stack([xy[:n], xy[n:]])
    fr = oracle.velocity(np.concatenate([P[0], P[1]]), g, d)
    np.testing.assert_allclose(np.stack([fr[:n], fr[n:]]), R @ np.stack([f[:n], f[n:]]), rtol=1e-12, atol=1e-12 * abs(f).max())
    ft = oracle.velocity(np.concatenate([xy[:n] + 0.5, xy[n:] - 0.25]), g, d)
    np.testing.assert_allclose(ft, f, rtol=1e-10, atol=1e-12 * abs(f).max())
    s = 2.5
    fs = oracle.velocity(s * xy, g, s * d)
    np.testing.assert_allclose(fs, f / s, rtol=1e-12, atol=1e-14 * abs(f).max())
    fl = oracle.velocity(xy, 3.0 * g - 0.0, d)
    np.testing.assert_allclose(fl, 3.0 * f, rtol=1e-13, atol=1e-15 * abs(f).max())


def test_velocity_at_matches_full():
    cl = W.disk_cloud(257, seed=3)
    f = oracle.velocity(cl.xy, cl.gamma, 0.02)
    idx = np.array([0, 5, 256, 100])
    fa = oracle.velocity_at(cl.xy, cl.gamma, 0.02, idx)
    np.testing.assert_array_equal(fa, np.concatenate([f[idx], f[257 + idx]]))


# ---------------------------------------------------------------- derivatives

def test_jvp_against_central_differences():
    cl = W.gaussian_patch(150, seed=11, delta=0.05)
    xy, g, d = cl.xy, cl.gamma, cl.delta
    rng = np.random.default_rng(0)
    for _ in range(3):
        v = rng.standard_normal(xy.size)
        h = 1e-6 * np.abs(xy).max()
        fd = (oracle.velocity(xy + h * v, g, d) - oracle.velocity(xy - h * v, g, d)) / (2 * h)
        assert rel(oracle.jvp(xy, g, d, v), fd) < 1e-8


def test_jvp_linearity_and_rigid_motions():
    cl = W.disk_cloud(120, seed=2)
    xy, g, d = cl.xy, cl.gamma, 0.02
    n = g.size
    rng = np.random.default_rng(1)
    v1, v2 = rng.standard_normal(2 * n), rng.standard_normal(2 * n)
    j1, j2 = oracle.jvp(xy, g, d, v1), oracle.jvp(xy, g, d, v2)
    np.testing.assert_allclose(oracle.jvp(xy, g, d, 2 * v1 - 3 * v2), 2 * j1 - 3 * j2, rtol=1e-12, atol=1e-12 * abs(j1).max())
    # uniform translation of every body leaves f unchanged: J (c, c, ..) = 0
    t = np.concatenate([np.full(n, 0.3), np.full(n, -1.1)])
    assert np.abs(oracle.jvp(xy, g, d, t)).max() < 1e-12 * abs(j1).max()
    # infinitesimal rotation v = e3 x x rotates f: J v = e3 x f
    f = oracle.velocity(xy, g, d)
    rot = np.concatenate([-xy[n:], xy[:n]])
    np.testing.assert_allclose(oracle.jvp(xy, g, d, rot), np.concatenate([-f[n:], f[:n]]), rtol=1e-10, atol=1e-11 * abs(f).max())


def test_block_jacobian_is_traceless_self_derivative():
    cl = W.gaussian_patch(80, seed=4, delta=0.04)
    xy, g, d = cl.xy, cl.gamma, cl.delta
    n = g.size
    B = oracle.block_jacobian(xy, g, d).reshape(4, n)
    assert np.abs(B[0] + B[3]).max() < 1e-12 * np.abs(B).max()
    # column q of the self block = d f_i / d x_i moving body i alone
    for i in [0, 33, 79]:
        for q in range(2):
            e = np.zeros(2 * n); e[i + q * n] = 1.0
            h = 1e-6
            fd = (oracle.velocity(xy + h * e, g, d) - oracle.velocity(xy - h * e, g, d)) / (2 * h)
            np.testing.assert_allclose([B[q, i], B[2 + q, i]], [fd[i], fd[n + i]], rtol=1e-7, atol=1e-9 * np.abs(B).max())


def test_vjp_dot_product_and_gamma_homogeneity():
    cl = W.disk_cloud(140, seed=9)
    xy, g, d = cl.xy, cl.gamma + 0.05, 0.02
    n = g.size
    rng = np.random.default_rng(3)
    for _ in range(3):
        v, w = rng.standard_normal(2 * n), rng.standard_normal(2 * n)
        gx, gg = oracle.vjp(xy, g, d, w)
        lhs, rhs = np.dot(w, oracle.jvp(xy, g, d, v)), np.dot(gx, v)
        assert abs(lhs - rhs) < 1e-13 * np.linalg.norm(w) * np.linalg.norm(oracle.jvp(xy, g, d, v)) * 10
        # f is linear in Gamma: sum_j Gamma_j d(w.f)/dGamma_j = w . f
        wf = np.dot(w, oracle.velocity(xy, g, d))
        assert abs(np.dot(g, gg) - wf) < 1e-12 * abs(wf) + 1e-14
        # and exact finite differences in Gamma
        e = np.zeros(n); e[7] = 1.0
        fd = np.dot(w, oracle.velocity(xy, g + e, d) - oracle.velocity(xy, g, d))
        assert gg[7] == pytest.approx(fd, rel=1e-9, abs=1e-13)


def test_sampled_entry_points_match_full():
    cl = W.gaussian_patch(190, seed=12, delta=0.03)
    xy, g, d = cl.xy, cl.gamma, cl.delta
    n = g.size
    rng = np.random.default_rng(4)
    v = rng.standard_normal(2 * n)
    idx = np.array([3, 0, 189, 77])
    jv = oracle.jvp(xy, g, d, v)
    np.testing.assert_array_equal(oracle.jvp_at(xy, g, d, v, idx), np.concatenate([jv[idx], jv[n + idx]]))
    gx, gg = oracle.vjp(xy, g, d, v)
    ax, ag = oracle.vjp_at(xy, g, d, v, idx)
    np.testing.assert_array_equal(ax, np.concatenate([gx[idx], gx[n + idx]]))
    np.testing.assert_array_equal(ag, gg[idx])
    B = oracle.block_jacobian(xy, g, d).reshape(4, n)
    np.testing.assert_array_equal(oracle.block_jacobian_at(xy, g, d, idx), B[:, idx].ravel())


# ---------------------------------------------------------------- steppers

def _two_vortex_state(G, p1, p2):
    return np.array([p1[0], p2[0], p1[1], p2[1]]), np.array(G, dtype=float)


def _omega(G, d2, delta):
    return sum(G) / (2 * math.pi * (d2 + delta * delta))


@pytest.mark.parametrize("delta", [0.0, 0.2])
def test_rk4_equals_scalar_rk4_on_relative_coordinate(delta):
    # For two vortices, z = x1 - x2 obeys dz/dt = i Omega(|z|) z, so vector RK4
    # on N=2 must equal RK4 applied to this scalar complex ODE, and the
    # circulation centroid is an exact linear invariant of every RK method.
    G = (0.8, 1.7)
    xy, g = _two_vortex_state(G, (0.2, 0.1), (-0.4, 0.5))
    dt, steps = 0.01, 50
    out = oracle.rk4(xy, g, delta, dt, steps)
    z = complex(xy[0] - xy[1], xy[2] - xy[3])
    F = lambda z: 1j * _omega(G, abs(z) ** 2, delta) * z
    for _ in range(steps):
        k1 = F(z); k2 = F(z + dt / 2 * k1); k3 = F(z + dt / 2 * k2); k4 = F(z + dt * k3)
        z = z + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    assert abs(complex(out[0] - out[1], out[2] - out[3]) - z) < 1e-13
    c0 = (g[0] * xy[[0, 2]] + g[1] * xy[[1, 3]]) / g.sum()
    c1 = (g[0] * out[[0, 2]] + g[1] * out[[1, 3]]) / g.sum()
    np.testing.assert_allclose(c1, c0, atol=1e-15)


def test_rk4_fourth_order():
    G, delta, T = (1.0, 1.0), 0.1, 0.5
    xy, g = _two_vortex_state(G, (0.25, 0.0), (-0.25, 0.0))
    z0 = complex(0.5, 0.0)
    om = _omega(G, 0.25, delta)
    exact = z0 * np.exp(1j * om * T)
    errs = []
    for steps in (10, 20, 40):
        out = oracle.rk4(xy, g, delta, T / steps, steps)
        errs.append(abs(complex(out[0] - out[1], out[2] - out[3]) - exact))
    assert 14 < errs[0] / errs[1] < 18 and 14 < errs[1] / errs[2] < 18


@pytest.mark.parametrize("delta", [0.0, 0.15])
def test_trapezoid_two_vortex_cayley_rotation(delta):
    # Trapezoid rule on dz/dt = i Omega(|z|) z keeps |z| and rotates by
    # 2 atan(dt Omega / 2) per step (Cayley map); the solution is unique for small dt.
    G = (0.9, 0.6)
    xy, g = _two_vortex_state(G, (0.3, 0.0), (-0.2, 0.1))
    dt, steps = 0.05, 20
    out, st = oracle.implicit(xy, g, delta, dt, steps, scheme=oracle.TRAPEZOID)
    assert st.nonconverged_steps == 0
    z0 = complex(xy[0] - xy[1], xy[2] - xy[3])
    om = _omega(G, abs(z0) ** 2, delta)
    z = z0 * np.exp(1j * steps * 2 * math.atan(dt * om / 2))
    assert abs(complex(out[0] - out[1], out[2] - out[3]) - z) < 1e-12


def test_backward_euler_two_vortex_fixed_point():
    # BE: z_{n+1} (1 - i dt Omega(|z_{n+1}|)) = z_n, i.e.
    # |z_{n+1}|^2 (1 + dt^2 Omega^2) = |z_n|^2 and the angle advances by atan(dt Omega).
    G, delta = (0.9, 0.6), 0.1
    xy, g = _two_vortex_state(G, (0.3, 0.0), (-0.2, 0.1))
    dt, steps = 0.05, 10
    out, st = oracle.implicit(xy, g, delta, dt, steps, scheme=oracle.BE)
    assert st.nonconverged_steps == 0
    z = complex(xy[0] - xy[1], xy[2] - xy[3])
    for _ in range(steps):
        rho = abs(z)
        for _ in range(200):  # scalar fixed point for the new radius
            rho = abs(z) / math.sqrt(1 + (dt * _omega(G, rho * rho, delta)) ** 2)
        z = z / abs(z) * rho * np.exp(1j * math.atan(dt * _omega(G, rho * rho, delta)))
    assert abs(complex(out[0] - out[1], out[2] - out[3]) - z) < 1e-12


@pytest.mark.parametrize("delta", [0.0, 0.15])
def test_block_newton_passive_tracer_is_exact_newton(delta):
    # A passive tracer (Gamma_2 = 0) around a vortex: the vortex feels no
    # velocity and the tracer's own 2x2 block is the only nonzero Jacobian
    # block, so the block-diagonal inexact Newton is exact Newton (same
    # iteration count: a transposed or sign-flipped block loses quadratic
    # convergence) and the trapezoid step is the Cayley rotation about the
    # vortex by 2 atan(dt Omega / 2).
    xy, g = _two_vortex_state((0.9, 0.0), (0.1, -0.05), (0.4, 0.2))
    dt, steps = 0.05, 20
    ob, sb = oracle.implicit_block(xy, g, delta, dt, steps, scheme=oracle.TRAPEZOID)
    oe, se = oracle.implicit(xy, g, delta, dt, steps, scheme=oracle.TRAPEZOID)
    assert sb.nonconverged_steps == 0 and sb.newton_iters == se.newton_iters
    assert ob[0] == xy[0] and ob[2] == xy[2]
    z0 = complex(xy[1] - xy[0], xy[3] - xy[2])
    om = _omega(g, abs(z0) ** 2, delta)
    z = z0 * np.exp(1j * steps * 2 * math.atan(dt * om / 2))
    assert abs(complex(ob[1] - ob[0], ob[3] - ob[2]) - z) < 1e-12


@pytest.mark.parametrize("scheme", [oracle.BE, oracle.TRAPEZOID])
def test_block_newton_same_root_as_exact_newton(scheme):
    # Both iterations drive the same residual to zero and differ only in the
    # linear model, so they reach the same states, the block version in more
    # (linearly convergent) iterations, for every Jacobian refresh period.
    cl = W.gaussian_patch(64, seed=21, delta=0.05)
    xy, g, d = cl.xy, cl.gamma * 64, cl.delta
    oe, se = oracle.implicit(xy, g, d, 2.5e-3, 3, scheme)
    for p in (0, 1, 2):
        ob, sb = oracle.implicit_block(xy, g, d, 2.5e-3, 3, scheme, jac_period=p)
        assert sb.nonconverged_steps == 0 and sb.newton_iters > se.newton_iters
        assert np.linalg.norm(ob - oe) <= 1e-10 * np.linalg.norm(oe - xy)


def test_block_newton_background_velocity_and_rest():
    # a uniform background velocity U shifts the trajectory by U t exactly;
    # with every Gamma = 0 the initial state is already the root
    cl = W.gaussian_patch(48, seed=22, delta=0.05)
    xy, g, d = cl.xy, cl.gamma * 48, cl.delta
    U = np.concatenate([np.full(48, 0.3), np.full(48, -0.2)])
    dt, k = 2e-3, 4
    o0, _ = oracle.implicit_block(xy, g, d, dt, k, oracle.TRAPEZOID, jac_period=1)
    o1, s1 = oracle.implicit_block(xy, g, d, dt, k, oracle.TRAPEZOID, jac_period=1, u=U)
    assert s1.nonconverged_steps == 0
    assert np.abs(o1 - (o0 + U * dt * k)).max() < 1e-12
    o2, s2 = oracle.implicit_block(xy, 0.0 * g, d, dt, k, oracle.BE)
    assert s2.newton_iters == 0 and np.array_equal(o2, xy)


def test_implicit_schemes_order_against_rk4():
    cl = W.gaussian_patch(64, seed=21, delta=0.05)
    xy, g, d = cl.xy, cl.gamma * 64, cl.delta
    T = 0.02
    ref = oracle.rk4(xy, g, d, T / 200, 200)
    e_be, e_tr = [], []
    for steps in (4, 8):
        e_be.append(np.linalg.norm(oracle.implicit(xy, g, d, T / steps, steps, oracle.BE)[0] - ref))
        e_tr.append(np.linalg.norm(oracle.implicit(xy, g, d, T / steps, steps, oracle.TRAPEZOID)[0] - ref))
    assert 1.7 < e_be[0] / e_be[1] < 2.3      # first order
    assert 3.5 < e_tr[0] / e_tr[1] < 4.5      # second order


# ---------------------------------------------------------------- adjoint

def test_adjoint_linear_impulse_exact():
    # P(T) = sum_i G_i x_i(T) equals sum_i G_i x_i(0) for every RK4 trajectory,
    # so dP/dx(0) = (G, 0) and dP/dGamma = x(0) exactly.
    cl = W.shear_layer(256, seed=31, delta=0.05)
    xy, g = cl.xy, cl.gamma * (1 + np.random.default_rng(0).random(256))
    n = g.size
    dt, steps = 5e-3, 12
    xT = oracle.rk4(xy, g, cl.delta, dt, steps)
    lamT = np.concatenate([g, np.zeros(n)])
    xT2, lam0, gg = oracle.rk4_adjoint(xy, g, cl.delta, dt, steps, lamT, gg_direct=xT[:n])
    np.testing.assert_array_equal(xT2, xT)
    np.testing.assert_allclose(lam0, lamT, rtol=0, atol=1e-10 * np.abs(g).max())
    np.testing.assert_allclose(gg, xy[:n], rtol=0, atol=1e-10)


def test_adjoint_against_finite_differences():
    cl = W.gaussian_patch(96, seed=41, delta=0.05)
    xy, g, d = cl.xy, cl.gamma * 96, cl.delta
    n = g.size
    dt, steps = 2e-3, 10
    rng = np.random.default_rng(5)
    c = rng.standard_normal(2 * n)
    Q = lambda x, gm: np.dot(c, oracle.rk4(x, gm, d, dt, steps)) + 0.5 * np.dot(gm, gm)
    _, lam0, gg = oracle.rk4_adjoint(xy, g, d, dt, steps, c, gg_direct=g)
    for _ in range(3):
        v = rng.standard_normal(2 * n); u = rng.standard_normal(n)
        h = 1e-6
        fdx = (Q(xy + h * v, g) - Q(xy - h * v, g)) / (2 * h)
        fdg = (Q(xy, g + h * u) - Q(xy, g - h * u)) / (2 * h)
        assert np.dot(lam0, v) == pytest.approx(fdx, rel=1e-6)
        assert np.dot(gg, u) == pytest.approx(fdg, rel=1e-6)


def test_hamiltonian_conserved_by_rk4():
    cl = W.disk_cloud(128, seed=8)
    H0 = oracle.hamiltonian(cl.xy, cl.gamma, 0.05)
    x = oracle.rk4(cl.xy, cl.gamma, 0.05, 1e-3, 20)
    assert abs(oracle.hamiltonian(x, cl.gamma, 0.05) - H0) < 1e-8 * abs(H0)


def test_hamiltonian_two_bodies():
    # H = -(1/4pi) * 2 * G1 G2 * (1/2) log(d^2 + delta^2)
    xy = np.array([0.0, 3.0, 0.0, 4.0])
    H = oracle.hamiltonian(xy, np.array([2.0, 0.5]), 0.0)
    assert H == pytest.approx(-(1 / (4 * math.pi)) * 2 * 1.0 * math.log(5.0), rel=1e-15)


# ---------------------------------------------------------------- least squares

def test_lstsq_matches_numpy():
    rng = np.random.default_rng(6)
    for m, n in [(16, 8), (32, 8), (8, 8), (50, 3)]:
        G = rng.standard_normal((m, n)); b = rng.standard_normal(m)
        x = oracle.lstsq(G, b)
        np.testing.assert_allclose(x, np.linalg.lstsq(G, b, rcond=None)[0], rtol=1e-11, atol=1e-12)


# ---------------------------------------------------------------- stream function, field points

def test_stream_function_gradient_is_velocity():
    # f_i = (d psi_i / d y_i, -d psi_i / d x_i) with the sources held fixed
    cl = W.gaussian_patch(90, seed=13, delta=0.03)
    xy, g, d = cl.xy, cl.gamma * 90, cl.delta
    n = g.size
    f = oracle.velocity(xy, g, d)
    h = 1e-6
    for i in [0, 41, 89]:
        e = np.zeros(2 * n)
        e[n + i] = h
        dpsi_dy = (oracle.stream_function(xy + e, g, d)[i] - oracle.stream_function(xy - e, g, d)[i]) / (2 * h)
        e[:] = 0.0
        e[i] = h
        dpsi_dx = (oracle.stream_function(xy + e, g, d)[i] - oracle.stream_function(xy - e, g, d)[i]) / (2 * h)
        assert dpsi_dy == pytest.approx(f[i], rel=1e-7, abs=1e-9)
        assert -dpsi_dx == pytest.approx(f[n + i], rel=1e-7, abs=1e-9)


def test_stream_function_two_bodies_and_hamiltonian():
    xy = np.array([0.0, 0.6, 0.0, 0.8])          # d = 1
    g = np.array([1.5, -0.7])
    psi = oracle.stream_function(xy, g, 0.5)
    np.testing.assert_allclose(psi, [0.7 / (4 * math.pi) * math.log(1.25), -1.5 / (4 * math.pi) * math.log(1.25)],
                               rtol=1e-15)
    cl = W.disk_cloud(150, seed=6)
    H = 0.5 * np.dot(cl.gamma, oracle.stream_function(cl.xy, cl.gamma, 0.02))
    assert H == pytest.approx(oracle.hamiltonian(cl.xy, cl.gamma, 0.02), rel=1e-12)


def test_stream_function_at_matches_full():
    cl = W.disk_cloud(257, seed=4)
    psi = oracle.stream_function(cl.xy, cl.gamma, 0.02)
    idx = np.array([256, 0, 17, 130])
    np.testing.assert_array_equal(oracle.stream_function_at(cl.xy, cl.gamma, 0.02, idx), psi[idx])


def test_velocity_at_points_matches_bodies_and_far_field():
    cl = W.gaussian_patch(120, seed=17, delta=0.02)
    n = cl.n
    # a point placed on a zero-strength body reproduces that body's velocity
    g = cl.gamma.copy()
    g[5] = 0.0
    p = np.array([cl.xy[5], cl.xy[n + 5]])
    fp = oracle.velocity_points(p, cl.xy, g, cl.delta)
    f = oracle.velocity(cl.xy, g, cl.delta)
    np.testing.assert_allclose(fp, [f[5], f[n + 5]], rtol=1e-13)
    # far away the field is that of a point vortex of the total circulation at the centroid
    R = 1e4
    fp = oracle.velocity_points(np.array([R, 0.0]), cl.xy, cl.gamma, cl.delta)
    assert fp[1] == pytest.approx(cl.gamma.sum() / (2 * math.pi * R), rel=1e-3)
