"""GPU parity of the parametric online PTROM: clustered-circulation
reassignment for many parameters (device) and many queries in one launch,
one workgroup per query, against the oracle's online step with the
reassigned circulations."""
import numpy as np
import pytest
import torch

import oracle
from oracle import offline as off
from paper_2103_01983_amd import native
from paper_2103_01983_amd import workloads as W

pytestmark = pytest.mark.gpu


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def parametric():
    mus = [(40.0, 55.0), (60.0, 30.0)]
    clouds = [W.vortex_pair(m, n=64, half=6.0, delta=0.21) for m in mus]
    art, ex = off.train_parametric(clouds, 0.01, 40, M=16, Mr=32, ns=24, depth=6, pc=1.0, tol=1e-6)
    a = dict(art)
    for k in ("Phibar", "xbar0", "xqt0", "Phit", "Gt"):
        a[k] = f32(art[k])
    a["delta"] = float(np.float32(art["delta"]))
    a["dt"] = float(np.float32(art["dt"]))
    mem = art["members"]
    a["mem_off"] = np.concatenate([[0], np.cumsum([len(m) for m in mem])])
    a["mem_ids"] = np.concatenate([np.asarray(m) for m in mem])
    a["n"] = clouds[0].n
    queries = np.array([(40.0, 55.0), (25.0, 70.0), (64.0, 64.0), (50.0, 20.0), (33.0, 47.0)])
    return a, ex, queries


def test_reassign_matches_oracle(dev, parametric):
    a, ex, queries = parametric
    rom = native.Rom(a)
    G = np.stack([f32(W.vortex_pair(q, n=64, half=6.0).gamma) for q in queries])
    gt = rom.reassign(torch.tensor(G, dtype=torch.float32, device=dev)).cpu().numpy()
    mem = [a["mem_ids"][a["mem_off"][c]:a["mem_off"][c + 1]] for c in range(len(a["mem_off"]) - 1)]
    for q in range(len(queries)):
        ref = off.reassign_circulation(mem, G[q])
        np.testing.assert_allclose(gt[q], ref, rtol=1e-7, atol=1e-12)
    rom.close()


def test_batched_equals_single_runs(dev, parametric):
    # identical circulations in every slot reproduce the single-query run bitwise
    a, ex, _ = parametric
    M, steps, nq = a["M"], 25, 3
    rom = native.Rom(a, tol=1e-6, max_iter=50)
    xh = torch.zeros(M, dtype=torch.float64, device=dev)
    h1 = torch.empty(steps * M, dtype=torch.float64, device=dev)
    i1 = torch.empty(steps, dtype=torch.int32, device=dev)
    rom.run(steps, xh, h1, i1)
    gt = torch.tensor(np.tile(np.asarray(a["Gt"], np.float32), (nq, 1)), device=dev)
    xq = torch.zeros((nq, M), dtype=torch.float64, device=dev)
    hq = torch.empty((nq, steps, M), dtype=torch.float64, device=dev)
    iq = torch.empty((nq, steps), dtype=torch.int32, device=dev)
    rom.run_batched(gt, steps, xq, hq, iq)
    torch.cuda.synchronize()
    for q in range(nq):
        assert torch.equal(hq[q].reshape(-1), h1)
        assert torch.equal(iq[q], i1)
        assert torch.equal(xq[q], xh)
    rom.close()


@pytest.mark.parametrize("mode", [native.JAC_PAPER, native.JAC_EXACT])
def test_batched_queries_match_oracle(dev, parametric, mode):
    a, ex, queries = parametric
    M, steps, K = a["M"], 20, 3
    rom = native.Rom(a, tol=0.0, max_iter=K, jac_mode=mode)
    G = np.stack([f32(W.vortex_pair(q, n=64, half=6.0).gamma) for q in queries])
    gt = rom.reassign(torch.tensor(G, dtype=torch.float32, device=dev))
    nq = len(queries)
    xq = torch.zeros((nq, M), dtype=torch.float64, device=dev)
    hq = torch.empty((nq, steps, M), dtype=torch.float64, device=dev)
    rom.run_batched(gt, steps, xq, hq, None)
    torch.cuda.synchronize()
    gth = gt.cpu().numpy().astype(np.float64)
    for q in range(nq):
        aq = dict(a)
        aq["Gt"] = gth[q]
        o = oracle.Rom(aq, jac_mode=mode).run(steps, tol=0.0, max_iter=K)
        assert rel(hq[q].cpu().numpy(), o["hist"]) <= 1e-5, q
    rom.close()


def test_batched_rejects_oversized(dev):
    # a sample set whose run arrays do not fit in LDS cannot be batched
    cl = W.counter_rotating_patches(900, seed=5, delta=0.02)
    n = cl.n
    rng = np.random.default_rng(1)
    Phi = np.linalg.qr(rng.standard_normal((2 * n, 8)))[0]
    tree = off.QuadTree(off.weighted_points(Phi, np.linspace(8, 1, 8)), 6)
    sample = np.sort(rng.choice(n, 600, replace=False))
    Phi_r = np.linalg.qr(rng.standard_normal((2 * n, 16)))[0]
    art = off.rom_artifacts(sample, tree, 1.0, cl.xy, Phi, cl.gamma, cl.delta, 1e-3, A=off.gappy_operator(Phi_r, sample))
    rom = native.Rom(art)
    gt = torch.tensor(np.tile(np.asarray(art["Gt"], np.float32), (2, 1)), device=dev)
    xq = torch.zeros((2, 8), dtype=torch.float64, device=dev)
    with pytest.raises(native.PtromError):
        rom.run_batched(gt, 2, xq)
    rom.close()


@pytest.fixture(scope="module")
def mushroom():
    # a small mushroom cloud (opposite end circulations, inflow) trained by
    # the oracle pipeline at two parameters
    n = 64
    mus = [(-50.0, 40.0), (-30.0, 60.0)]
    clouds = [W.mushroom_cloud(m, n=n, half=4.8, delta=0.15) for m in mus]
    u = W.mushroom_inflow(n)
    art, ex = off.train_parametric(clouds, 0.005, 40, M=16, Mr=32, ns=24, depth=6, pc=1.0, tol=1e-6, u=u)
    a = dict(art)
    for k in ("Phibar", "xbar0", "xqt0", "Phit", "Gt"):
        a[k] = f32(art[k])
    a["delta"] = float(np.float32(art["delta"]))
    a["dt"] = float(np.float32(art["dt"]))
    mem = art["members"]
    a["mem_off"] = np.concatenate([[0], np.cumsum([len(m) for m in mem])])
    a["mem_ids"] = np.concatenate([np.asarray(m) for m in mem])
    a["n"] = n
    queries = np.array([(-50.0, 40.0), (-60.0, 30.0), (-35.0, 55.0)])
    return a, ex, queries


def test_batched_inflow_queries_match_oracle(dev, mushroom):
    a, ex, queries = mushroom
    assert "ubar" in a
    M, steps, K = a["M"], 20, 3
    rom = native.Rom(a, tol=0.0, max_iter=K)
    G = np.stack([f32(W.mushroom_cloud(q, n=64, half=4.8, delta=0.15).gamma) for q in queries])
    gt = rom.reassign(torch.tensor(G, dtype=torch.float32, device=dev))
    nq = len(queries)
    xq = torch.zeros((nq, M), dtype=torch.float64, device=dev)
    hq = torch.empty((nq, steps, M), dtype=torch.float64, device=dev)
    rom.run_batched(gt, steps, xq, hq, None)
    torch.cuda.synchronize()
    gth = gt.cpu().numpy().astype(np.float64)
    for q in range(nq):
        aq = dict(a)
        aq["Gt"] = gth[q]
        o = oracle.Rom(aq).run(steps, tol=0.0, max_iter=K)
        assert rel(hq[q].cpu().numpy(), o["hist"]) <= 1e-5, q
    rom.close()
