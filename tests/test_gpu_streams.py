"""The library's calls run on the stream they are given: the same calls on a
side stream of default priority (created by torch, which does not order it
against the null stream) give bitwise the results of the current stream,
with the inputs written and the outputs read through that side stream."""
import numpy as np
import pytest
import torch

from oracle import offline as off
from paper_2103_01983_amd import native
from paper_2103_01983_amd import workloads as W

pytestmark = pytest.mark.gpu


def _calls(dev, c, rom_art):
    n = c.n
    t = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
    xy, g = t(c.xy), t(c.gamma)
    v = t(W.unit_vectors(n, 1, 7)[0])
    out = {}
    out["velocity"] = native.velocity(xy, g, 0.01)
    out["jvp"] = native.jvp(xy, g, 0.01, v)
    out["vjp"] = torch.cat(native.vjp(xy, g, 0.01, v))
    out["psi"] = native.stream_function(xy, g, 0.01)
    x = xy.clone()
    native.implicit(x, g, 0.01, 1e-3, 3, scheme=native.TRAPEZOID, linear_solver=native.NEWTON_BLOCK)
    out["implicit_block"] = x
    x2 = xy.clone()
    native.implicit(x2, g, 0.01, 1e-3, 2)
    out["implicit_gmres"] = x2
    x3 = xy.clone()
    native.rk4(x3, g, 0.01, 1e-3, 3)
    out["rk4"] = x3
    M = int(rom_art["M"])
    rom = native.Rom(rom_art, tol=0.0, max_iter=3)
    xh = torch.zeros(M, dtype=torch.float64, device=dev)
    hist = torch.empty(4 * M, dtype=torch.float64, device=dev)
    rom.run(4, xh, hist, None)
    out["rom"] = hist
    # the outputs leave through the stream they were made on
    res = {k: o.cpu() for k, o in out.items()}
    rom.close()
    return res


def test_side_stream_matches_current_stream(dev):
    c = W.gaussian_patch(3000, seed=31, delta=0.01)
    cl = W.counter_rotating_patches(640, seed=41, delta=0.02)
    rng = np.random.default_rng(3)
    n = cl.n
    Phi = np.linalg.qr(rng.standard_normal((2 * n, 8)))[0]
    tree = off.QuadTree(off.weighted_points(Phi, np.sort(rng.uniform(1.0, 10.0, 8))[::-1]), 6)
    sample = np.sort(rng.choice(n, 16, replace=False))
    A = off.gappy_operator(np.linalg.qr(rng.standard_normal((2 * n, 16)))[0], sample)
    art = off.rom_artifacts(sample, tree, 1.0, cl.xy, Phi, cl.gamma, cl.delta, 1e-3, A=A)
    ref = _calls(dev, c, art)
    torch.cuda.synchronize()
    side = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(side):
        got = _calls(dev, c, art)
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(ref[k], got[k]), k
