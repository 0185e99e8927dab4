"""Seeded synthetic vortex workloads.

This module only draws random inputs (positions, circulations, kernel cores,
unit vectors).  It holds none of the method's arithmetic and is shared by the
HIP path's tests/benchmark and the oracle's tests.  All draws are float64 from
``numpy.random.default_rng(seed)``; callers cast once to the dtype they need.

State vectors use the SoA layout ``xy = [x_0..x_{N-1}, y_0..y_{N-1}]``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Cloud:
    xy: np.ndarray          # [2N] float64
    gamma: np.ndarray       # [N] float64
    delta: float
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.gamma.size


def _soa(x, y):
    return np.concatenate([x, y])


def uniform_disk(n, seed, radius=1.0):
    """Points uniform in a disk: r = R sqrt(U), theta = 2 pi U'."""
    rng = np.random.default_rng(seed)
    r = radius * np.sqrt(rng.random(n))
    th = 2.0 * np.pi * rng.random(n)
    return rng, _soa(r * np.cos(th), r * np.sin(th))


def disk_cloud(n=1024, seed=1001, delta=0.02):
    """Uniform unit disk, Gamma ~ N(0,1) shifted to sum zero."""
    rng, xy = uniform_disk(n, seed)
    g = rng.standard_normal(n)
    g = g - g.mean()
    return Cloud(xy, g, delta, dict(kind="disk"))


def gaussian_patch(n=65536, seed=1002, sigma=0.25, delta=0.01, gamma0=1.0, width=0.1):
    """Gaussian vortex patch: x ~ N(0, sigma^2 I), Gamma_i = Gamma0 exp(-|x_i|^2/width)/N."""
    rng = np.random.default_rng(seed)
    x = sigma * rng.standard_normal(n)
    y = sigma * rng.standard_normal(n)
    g = gamma0 * np.exp(-(x * x + y * y) / width) / n
    return Cloud(_soa(x, y), g, delta, dict(kind="gaussian_patch", sigma=sigma))


def counter_rotating_patches(n=16384, seed=1003, sigma=0.15, delta=0.01, sep=0.5):
    """Two Gaussian patches at (-sep, 0) with Gamma = +1/(n/2) each and at
    (+sep, 0) with Gamma = -1/(n/2) each."""
    rng = np.random.default_rng(seed)
    h = n // 2
    x = np.concatenate([-sep + sigma * rng.standard_normal(h), sep + sigma * rng.standard_normal(n - h)])
    y = sigma * rng.standard_normal(n)
    g = np.concatenate([np.full(h, 1.0 / h), np.full(n - h, -1.0 / (n - h))])
    return Cloud(_soa(x, y), g, delta, dict(kind="counter_rotating", sigma=sigma))


def shear_layer(n=131072, seed=1005, delta=0.01, thickness=0.05, amp=1e-3):
    """Perturbed circular shear layer: theta ~ U[0,2pi), r = 1 + t(U - 1/2) + amp xi,
    Gamma = 1/N."""
    rng = np.random.default_rng(seed)
    th = 2.0 * np.pi * rng.random(n)
    r = 1.0 + thickness * (rng.random(n) - 0.5) + amp * rng.standard_normal(n)
    return Cloud(_soa(r * np.cos(th), r * np.sin(th)), np.full(n, 1.0 / n), delta, dict(kind="shear_layer"))


# single-vortex study: N -> (dt, Gamma of the centre body, t_f)
SINGLE_VORTEX = {
    100: (0.01, 500.0, 20.0), 500: (2.5e-3, 1e4, 5.0), 1000: (2.5e-4, 1e5, 0.5),
    2000: (1.25e-4, 2e5, 0.25), 3000: (1e-4, 3e5, 0.2), 4000: (7.5e-5, 4e5, 0.15),
    5000: (5e-5, 6.75e5, 0.1),
}


def single_vortex(n, gamma_center=None):
    """Deterministic initial state of the single-vortex study: N bodies evenly
    spaced on the diagonal from (-N, -N) to (N, N), Gamma = 0.01 except the
    centre body (index N // 2), delta = 0.  ``meta`` carries the study's dt
    and t_f for the listed N."""
    dt, gc, tf = SINGLE_VORTEX.get(n, (None, None, None))
    if gamma_center is not None:
        gc = gamma_center
    if gc is None:
        raise ValueError(f"no study conditions for N={n}; pass gamma_center")
    s = np.linspace(-n, n, n)
    g = np.full(n, 0.01)
    g[n // 2] = gc
    return Cloud(_soa(s, s.copy()), g, 0.0, dict(kind="single_vortex", dt=dt, tf=tf))


def vortex_pair(mu, n=500, half=52.93, delta=0.2121):
    """Vortex-pair parametric study: n bodies on the diagonal from (-half,
    -half) to (half, half), Gamma = 0.01 except the end bodies, which carry
    mu = (Gamma_1, Gamma_N); core delta (the initial spacing per coordinate)."""
    s = np.linspace(-half, half, n)
    g = np.full(n, 0.01)
    g[0], g[-1] = float(mu[0]), float(mu[1])
    return Cloud(_soa(s, s.copy()), g, float(delta), dict(kind="vortex_pair", mu=tuple(float(m) for m in mu)))


def mushroom_cloud(mu, n=500, half=37.43, y0=-10.0, delta=0.15):
    """Mushroom-cloud parametric study: n bodies on the line y = y0 from
    x = -half to x = half, Gamma = 0.01 except the end bodies, which carry
    mu = (Gamma_1, Gamma_N) of opposite signs; core delta (the initial
    spacing).  The inflow is ``mushroom_inflow(n)``."""
    g = np.full(n, 0.01)
    g[0], g[-1] = float(mu[0]), float(mu[1])
    return Cloud(_soa(np.linspace(-half, half, n), np.full(n, float(y0))), g, float(delta),
                 dict(kind="mushroom_cloud", mu=tuple(float(m) for m in mu)))


def mushroom_inflow(n, amp=5.0, radius=1.125, base=0.5):
    """Background velocity of the mushroom cloud, SoA [2n]: zero along x and
    a semicircle profile amp * sqrt(radius^2 - s^2) + base along y, with s
    running linearly from -1 to 1 over the bodies."""
    s = np.linspace(-1.0, 1.0, n)
    return np.concatenate([np.zeros(n), amp * np.sqrt(radius * radius - s * s) + base])


def latin_hypercube(k, lo, hi, seed):
    """k points of a Latin hypercube in the box [lo, hi]^2 (one per row and
    column stratum, uniform inside its cell); lo and hi may be
    per-dimension pairs."""
    rng = np.random.default_rng(seed)
    pts = np.empty((k, 2))
    for dim in range(2):
        pts[:, dim] = (rng.permutation(k) + rng.uniform(size=k)) / k
    return lo + (hi - lo) * pts


def parameter_grid(m, lo, hi):
    """m x m grid of parameter points spanning [lo, hi]^2 (row-major); lo and
    hi may be per-dimension pairs."""
    lo, hi = np.broadcast_to(lo, 2), np.broadcast_to(hi, 2)
    ga, gb = np.linspace(lo[0], hi[0], m), np.linspace(lo[1], hi[1], m)
    return np.array([(a, b) for a in ga for b in gb])


def unit_vectors(n, k, seed):
    """k random unit vectors of length 2n (Gaussian, normalized)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((k, 2 * n))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def random_vectors(n, k, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((k, 2 * n))


@dataclass
class Batch:
    offsets: np.ndarray     # [B+1] int64, instance b owns bodies offsets[b]..offsets[b+1]
    xy: np.ndarray          # [2 * total] float64: per-instance SoA blocks [x_b, y_b] back to back
    gamma: np.ndarray       # [total] float64
    delta: np.ndarray       # [B] float64
    scale: np.ndarray       # [B] float64


def batched_patches(B=256, seed=1004, nmin=2048, nmax=32768, dmin=0.005, dmax=0.05,
                    smin=0.5, smax=2.0, sigma=0.25, width=0.1):
    """Parametric batch: N_b = round(exp(U[ln nmin, ln nmax])), delta_b ~ U[dmin, dmax],
    scale s_b ~ U[smin, smax]; Gaussian patch positions, Gamma_i = s_b exp(-|x|^2/width)/N_b.

    Layout of ``xy``: instance b occupies [2*offsets[b], 2*offsets[b+1]) as
    its own SoA block [x_0..x_{Nb-1}, y_0..y_{Nb-1}]."""
    rng = np.random.default_rng(seed)
    nb = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), B))).astype(np.int64)
    dl = rng.uniform(dmin, dmax, B)
    sc = rng.uniform(smin, smax, B)
    off = np.zeros(B + 1, dtype=np.int64)
    off[1:] = np.cumsum(nb)
    xy = np.empty(2 * off[-1])
    g = np.empty(off[-1])
    for b in range(B):
        n = int(nb[b])
        x = sigma * rng.standard_normal(n)
        y = sigma * rng.standard_normal(n)
        xy[2 * off[b]: 2 * off[b] + n] = x
        xy[2 * off[b] + n: 2 * off[b + 1]] = y
        g[off[b]: off[b + 1]] = sc[b] * np.exp(-(x * x + y * y) / width) / n
    return Batch(off, xy, g, dl, sc)


# ---------------------------------------------------------------------------
# named workloads (sizes of the five benchmark configurations)
# ---------------------------------------------------------------------------

CONFIGS = {
    "c1_disk_fp64": dict(n=1024, seed=1001, delta=0.02, dt=1e-3, steps=100),
    "c2_gaussian_patch": dict(n=65536, seed=1002, delta=0.01, dt=5e-4, steps=50, njvp=8),
    "c3_ptrom_pipeline": dict(n=16384, seed=1003, delta=0.01, dt=1e-3, snapshots=400, M=8, Mr=16,
                              ns=16, depth=6, pc=1.0, tol=1e-4, max_iter=100, steps=400),
    "c4_batched": dict(B=256, seed=1004, dt=1e-3, steps=20),
    "c5_adjoint": dict(n=131072, seed=1005, delta=0.01, dt=5e-4, steps=200, every=20),
}


def config_cloud(name, n=None):
    c = CONFIGS[name]
    n = c["n"] if n is None else n
    if name == "c1_disk_fp64":
        return disk_cloud(n, c["seed"], c["delta"])
    if name == "c2_gaussian_patch":
        return gaussian_patch(n, c["seed"], delta=c["delta"])
    if name == "c3_ptrom_pipeline":
        return counter_rotating_patches(n, c["seed"], delta=c["delta"])
    if name == "c5_adjoint":
        return shear_layer(n, c["seed"], delta=c["delta"])
    raise KeyError(name)
