"""Every launch variant of the pair kernels (LDS or scalar-cache source
staging, 1/2/4 targets per lane, one-sided or each-pair-once tiles) against
the FP64 oracle, independent of which variant the autotuner selected.
Ragged sizes cover partial tiles, partial blocks and the self-pair masks."""
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
from paper_2103_01983_amd import native
from paper_2103_01983_amd import workloads as W

pytestmark = pytest.mark.gpu

# staging k waves sym
VARIANTS = [(0, 1, 16, 0), (1, 2, 8, 0), (0, 4, 4, 0), (1, 4, 16, 0), (0, 2, 4, 1), (0, 4, 2, 1), (0, 2, 8, 1),
            (0, 4, 4, 1)]
SIZES = [1, 2, 3, 513, 1024, 2500, 4099]


@pytest.fixture(scope="module", params=VARIANTS, ids=lambda v: "st%d_k%d_w%d_sym%d" % v)
def vctx(request, dev):
    st, k, w, sym = request.param
    fd, path = tempfile.mkstemp(suffix=".txt")
    with os.fdopen(fd, "w") as fh:
        for op in ("velocity", "jvp", "vjp", "block_jacobian", "velocity_block_jacobian", "stream_function"):
            fh.write("%s 16 %d %d %d %d\n" % (op, st, k, w, sym))
    h = native.make_context(0, path)
    os.unlink(path)
    yield h
    native.destroy_context(h)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("delta", [0.0, 0.01])
def test_variant_parity(dev, vctx, n, delta):
    c = W.disk_cloud(n, seed=900 + n, delta=delta)
    xy, g = f32(c.xy), f32(c.gamma)
    d = float(np.float32(delta))
    v = f32(W.random_vectors(n, 1, n)[0])
    t = lambda a: torch.tensor(a, dtype=torch.float32, device=dev)
    xd, gd, vd = t(xy), t(g), t(v)
    if n == 1:
        # a single body: no pair, every sum is exactly zero
        outs = [native.velocity(xd, gd, d, ctx=vctx), native.jvp(xd, gd, d, vd, ctx=vctx),
                *native.vjp(xd, gd, d, vd, ctx=vctx), native.block_jacobian(xd, gd, d, ctx=vctx),
                *native.velocity_block_jacobian(xd, gd, d, ctx=vctx), native.stream_function(xd, gd, d, ctx=vctx)]
        for o in outs:
            assert torch.count_nonzero(o).item() == 0
        return
    f = native.velocity(xd, gd, d, ctx=vctx).cpu().numpy()
    assert np.all(np.isfinite(f))
    assert rel(f, oracle.velocity(xy, g, d)) <= 1e-5
    jv = native.jvp(xd, gd, d, vd, ctx=vctx).cpu().numpy()
    assert rel(jv, oracle.jvp(xy, g, d, v)) <= 1e-5
    gx, gg = native.vjp(xd, gd, d, vd, ctx=vctx)
    ox, og = oracle.vjp(xy, g, d, v)
    assert rel(gx.cpu().numpy(), ox) <= 1e-5
    assert rel(gg.cpu().numpy(), og) <= 1e-5
    B = native.block_jacobian(xd, gd, d, ctx=vctx).cpu().numpy()
    ob = oracle.block_jacobian(xy, g, d)
    assert rel(B, ob) <= 1e-5
    f2, B2 = native.velocity_block_jacobian(xd, gd, d, ctx=vctx)
    assert rel(f2.cpu().numpy(), oracle.velocity(xy, g, d)) <= 1e-5
    assert rel(B2.cpu().numpy(), ob) <= 1e-5
    psi = native.stream_function(xd, gd, d, ctx=vctx).cpu().numpy()
    assert np.all(np.isfinite(psi))
    assert rel(psi, oracle.stream_function(xy, g, d)) <= 1e-5


def test_variant_coincident_bodies(dev, vctx):
    # distinct bodies at the same position (every third body repeats the one
    # before it): with delta > 0 each such pair adds nothing to the velocity
    # and the Jacobians and log(delta^2) to the stream function
    n = 1500
    c = W.disk_cloud(n, seed=77, delta=0.01)
    xy = f32(c.xy).copy()
    g = f32(c.gamma)
    for i in range(1, n, 3):
        xy[i] = xy[i - 1]
        xy[n + i] = xy[n + i - 1]
    d = float(np.float32(0.01))
    v = f32(W.random_vectors(n, 1, 77)[0])
    t = lambda a: torch.tensor(a, dtype=torch.float32, device=dev)
    xd, gd, vd = t(xy), t(g), t(v)
    f = native.velocity(xd, gd, d, ctx=vctx).cpu().numpy()
    assert rel(f, oracle.velocity(xy, g, d)) <= 1e-5
    jv = native.jvp(xd, gd, d, vd, ctx=vctx).cpu().numpy()
    assert rel(jv, oracle.jvp(xy, g, d, v)) <= 1e-5
    gx, gg = native.vjp(xd, gd, d, vd, ctx=vctx)
    ox, og = oracle.vjp(xy, g, d, v)
    assert rel(gx.cpu().numpy(), ox) <= 1e-5
    assert rel(gg.cpu().numpy(), og) <= 1e-5
    assert rel(native.block_jacobian(xd, gd, d, ctx=vctx).cpu().numpy(), oracle.block_jacobian(xy, g, d)) <= 1e-5
    psi = native.stream_function(xd, gd, d, ctx=vctx).cpu().numpy()
    assert rel(psi, oracle.stream_function(xy, g, d)) <= 1e-5


def test_variant_deterministic(dev, vctx):
    c = W.gaussian_patch(9000, seed=2)
    t = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
    xd, gd = t(c.xy), t(c.gamma)
    a = native.velocity(xd, gd, 0.01, ctx=vctx)
    b = native.velocity(xd, gd, 0.01, ctx=vctx)
    assert torch.equal(a, b)


def test_variant_full_size_sampled(dev, vctx):
    # the benchmark's Gaussian patch (N = 65536) on 128 sampled targets
    c = W.config_cloud("c2_gaussian_patch")
    xy, g, d = f32(c.xy), f32(c.gamma), float(np.float32(c.delta))
    n = c.n
    idx = np.random.default_rng(3).choice(n, 128, replace=False)
    sel = np.concatenate([idx, n + idx])
    v = f32(W.unit_vectors(n, 1, 1002)[0])
    t = lambda a: torch.tensor(a, dtype=torch.float32, device=dev)
    xd, gd, vd = t(xy), t(g), t(v)
    f = native.velocity(xd, gd, d, ctx=vctx).cpu().numpy()
    assert rel(f[sel], oracle.velocity_at(xy, g, d, idx)) <= 1e-5
    jv = native.jvp(xd, gd, d, vd, ctx=vctx).cpu().numpy()
    assert rel(jv[sel], oracle.jvp_at(xy, g, d, v, idx)) <= 1e-5
    gx, gg = native.vjp(xd, gd, d, vd, ctx=vctx)
    ox, og = oracle.vjp_at(xy, g, d, v, idx)
    assert rel(gx.cpu().numpy()[sel], ox) <= 1e-5
    assert rel(gg.cpu().numpy()[idx], og) <= 1e-5
    B = native.block_jacobian(xd, gd, d, ctx=vctx).cpu().numpy().reshape(4, n)
    ob = oracle.block_jacobian_at(xy, g, d, idx)
    assert rel(B[:, idx].ravel(), ob) <= 1e-5
    f2, B2 = native.velocity_block_jacobian(xd, gd, d, ctx=vctx)
    assert rel(f2.cpu().numpy()[sel], oracle.velocity_at(xy, g, d, idx)) <= 1e-5
    assert rel(B2.cpu().numpy().reshape(4, n)[:, idx].ravel(), ob) <= 1e-5
    psi = native.stream_function(xd, gd, d, ctx=vctx).cpu().numpy()
    assert rel(psi[idx], oracle.stream_function_at(xy, g, d, idx)) <= 1e-5
