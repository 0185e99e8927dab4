"""GPU parity of the batched persistent stepper (many instances with their own
N_b and delta_b) against the FP64 oracle run instance by instance, in every
launch the autotuner can choose (targets per lane, workgroups per CU)."""
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
from paper_2103_01983_amd import native
from paper_2103_01983_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def small_batch(sizes, seed):
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    xy, g = [], []
    for b, n in enumerate(sizes):
        c = W.gaussian_patch(int(n), seed=seed + b)
        xy.append(c.xy)
        g.append(c.gamma * rng.uniform(0.5, 2.0))
    delta = np.array([0.0 if b == 0 else 0.005 + 0.01 * b for b in range(len(sizes))])
    return off, f32(np.concatenate(xy)), f32(np.concatenate(g)), np.float32(delta)


def inst(off, xy, g, b):
    o0, o1 = off[b], off[b + 1]
    return xy[2 * o0:2 * o1], g[o0:o1]


SIZES = [1, 2, 300, 513, 2049, 257]

# targets per lane, workgroups per CU
LAUNCHES = [(1, 16), (2, 8), (4, 4)]


@pytest.fixture(scope="module", params=LAUNCHES, ids=lambda v: "k%d_bpc%d" % v)
def bctx(request, dev):
    k, bpc = request.param
    fd, path = tempfile.mkstemp(suffix=".txt")
    with os.fdopen(fd, "w") as fh:
        fh.write("batched_velocity 13 0 %d %d 1\n" % (k, bpc))
    h = native.make_context(0, path)
    os.unlink(path)
    cfg = native.pair_config("batched_velocity", 4096, ctx=h)
    assert (cfg["k"], cfg["waves_per_simd"]) == (k, bpc)
    yield h
    native.destroy_context(h)


def test_batched_velocity_launches(dev, bctx):
    off, xy, g, dl = small_batch(SIZES, 13)
    f = native.velocity_batched(off, torch.tensor(xy, dtype=torch.float32, device=dev),
                                torch.tensor(g, dtype=torch.float32, device=dev), dl, ctx=bctx).cpu().numpy()
    for b in range(len(SIZES)):
        x, gg = inst(off, xy, g, b)
        fb = f[2 * off[b]:2 * off[b + 1]]
        if SIZES[b] == 1:
            assert np.all(fb == 0)
            continue
        assert rel(fb, oracle.velocity(x, gg, float(dl[b]))) <= 1e-5, b
    # the graph-captured RK4 of the same launch
    x = torch.tensor(xy, dtype=torch.float32, device=dev)
    dl2 = dl.copy()
    dl2[0] = 0.01
    native.rk4_batched(off, x, torch.tensor(g, dtype=torch.float32, device=dev), dl2, 1e-3, 2, ctx=bctx)
    xs = x.cpu().numpy()
    for b in range(1, len(SIZES)):
        x0, gg = inst(off, xy, g, b)
        o = oracle.rk4(x0, gg, float(dl2[b]), float(np.float32(1e-3)), 2)
        xb = xs[2 * off[b]:2 * off[b + 1]]
        assert rel(xb - x0, o - x0) <= 1e-4, b


def test_batched_full_config_launches(dev, bctx):
    # the 256-instance set in each launch: sampled velocities of the largest
    # instances against the oracle
    bt = W.batched_patches()
    off = bt.offsets
    xy, g, dl = f32(bt.xy), f32(bt.gamma), np.float32(bt.delta)
    f = native.velocity_batched(off, torch.tensor(xy, dtype=torch.float32, device=dev),
                                torch.tensor(g, dtype=torch.float32, device=dev), dl, ctx=bctx).cpu().numpy()
    nb = np.diff(off)
    rng = np.random.default_rng(1)
    for b in list(np.argsort(nb)[-2:]) + [7]:
        x, gg = inst(off, xy, g, b)
        n = int(nb[b])
        idx = rng.choice(n, 32, replace=False)
        fb = f[2 * off[b]:2 * off[b + 1]]
        assert rel(np.concatenate([fb[idx], fb[n + idx]]), oracle.velocity_at(x, gg, float(dl[b]), idx)) <= 1e-5


def test_batched_velocity_parity(dev):
    off, xy, g, dl = small_batch(SIZES, 11)
    f = native.velocity_batched(off, torch.tensor(xy, dtype=torch.float32, device=dev),
                                torch.tensor(g, dtype=torch.float32, device=dev), dl).cpu().numpy()
    for b in range(len(SIZES)):
        x, gg = inst(off, xy, g, b)
        fb = f[2 * off[b]:2 * off[b + 1]]
        if SIZES[b] == 1:
            assert np.all(fb == 0)
            continue
        assert rel(fb, oracle.velocity(x, gg, float(dl[b]))) <= 1e-5, b


@pytest.mark.parametrize("use_graph", [True, False])
def test_batched_rk4_parity(dev, use_graph):
    off, xy, g, dl = small_batch(SIZES, 12)
    dl[0] = 0.01
    x = torch.tensor(xy, dtype=torch.float32, device=dev)
    native.rk4_batched(off, x, torch.tensor(g, dtype=torch.float32, device=dev), dl, 1e-3, 4, use_graph=use_graph)
    xs = x.cpu().numpy()
    for b in range(len(SIZES)):
        x0, gg = inst(off, xy, g, b)
        o = oracle.rk4(x0, gg, float(dl[b]), float(np.float32(1e-3)), 4)
        xb = xs[2 * off[b]:2 * off[b + 1]]
        if SIZES[b] == 1:
            assert np.array_equal(xb, x0)
            continue
        # displacement to 1e-4, plus the FP32 rounding of the stored state per step
        u = 2.0 ** -24
        assert rel(xb, o) <= 1e-6, b
        assert np.linalg.norm(xb - o) <= 1e-4 * np.linalg.norm(o - x0) + 4 * u * np.linalg.norm(o), b


def test_batched_full_config(dev):
    # 256 instances, N_b log-uniform in [2048, 32768], delta_b in [0.005, 0.05],
    # circulation scale in [0.5, 2]; sampled velocities of the largest
    # instances, and 20 RK4 steps of the three smallest against the oracle.
    bt = W.batched_patches()
    off = bt.offsets
    xy, g, dl = f32(bt.xy), f32(bt.gamma), np.float32(bt.delta)
    xd = torch.tensor(xy, dtype=torch.float32, device=dev)
    gd = torch.tensor(g, dtype=torch.float32, device=dev)
    f = native.velocity_batched(off, xd, gd, dl).cpu().numpy()
    nb = np.diff(off)
    rng = np.random.default_rng(0)
    for b in list(np.argsort(nb)[-3:]) + [0, 100]:
        x, gg = inst(off, xy, g, b)
        n = int(nb[b])
        idx = rng.choice(n, 32, replace=False)
        fb = f[2 * off[b]:2 * off[b + 1]]
        assert rel(np.concatenate([fb[idx], fb[n + idx]]), oracle.velocity_at(x, gg, float(dl[b]), idx)) <= 1e-5
    native.rk4_batched(off, xd, gd, dl, 1e-3, 20)
    xs = xd.cpu().numpy()
    for b in np.argsort(nb)[:3]:
        x0, gg = inst(off, xy, g, b)
        o = oracle.rk4(x0, gg, float(dl[b]), float(np.float32(1e-3)), 20)
        xb = xs[2 * off[b]:2 * off[b + 1]]
        assert rel(xb - x0, o - x0) <= 1e-4


def test_batched_rejects_bad_offsets(dev):
    x = torch.zeros(8, device=dev)
    g = torch.zeros(4, device=dev)
    with pytest.raises(native.PtromError):
        native.velocity_batched([0, 2, 2, 4], x, g, [0.1, 0.1, 0.1])


def test_batched_rejects_too_many_block_pairs(dev):
    # one instance of 3e6 bodies: 5860 blocks of 512, 17.2e6 block pairs > 2^24
    n = 3_000_000
    x = torch.zeros(2 * n, device=dev)
    g = torch.zeros(n, device=dev)
    with pytest.raises(native.PtromError):
        native.velocity_batched([0, n], x, g, [0.1])
