"""GPU parity of the split online runs (small basis, paper Jacobian): one
query's interaction lists spread over W workgroups that meet at a device-side
barrier per HyperPair evaluation, against the oracle's online step on the
same artifacts, and against the one-workgroup run."""
import numpy as np
import pytest
import torch

import oracle
from oracle import offline as off
from paper_2103_01983_amd import native
from paper_2103_01983_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def rounded(art):
    a = dict(art)
    for k in ("Phibar", "xbar0", "xqt0", "Phit", "Gt"):
        a[k] = f32(art[k])
    a["delta"] = float(np.float32(art["delta"]))
    a["dt"] = float(np.float32(art["dt"]))
    return a


def synth(cl, M, Mr, ns, depth, seed):
    """Artifacts built by the oracle's offline steps over random orthonormal
    bases (tree, sample, lists and gappy operator as in training)."""
    n = cl.n
    rng = np.random.default_rng(seed)
    Phi = np.linalg.qr(rng.standard_normal((2 * n, M)))[0]
    sig = np.sort(rng.uniform(1.0, 10.0, M))[::-1]
    tree = off.QuadTree(off.weighted_points(Phi, sig), depth)
    sample = np.sort(rng.choice(n, ns, replace=False))
    Phi_r = np.linalg.qr(rng.standard_normal((2 * n, Mr)))[0]
    A = off.gappy_operator(Phi_r, sample)
    return rounded(off.rom_artifacts(sample, tree, 1.0, cl.xy, Phi, cl.gamma, cl.delta, 1e-3, A=A))


@pytest.fixture(scope="module")
def c3():
    # the PTROM pipeline's sizes: N = 16384 in two counter-rotating patches,
    # depth 6, M = 8, M_r = 16, 16 sampled bodies (about 5700 list entries)
    return synth(W.config_cloud("c3_ptrom_pipeline"), 8, 16, 16, 6, 5)


@pytest.fixture(scope="module")
def small():
    # short lists: 40 sampled bodies of a 640-body cloud
    return synth(W.counter_rotating_patches(640, seed=41, delta=0.02), 8, 16, 40, 6, 7)


def run(art, W_, steps, K, tol=0.0, dev="cuda"):
    M = int(art["M"])
    rom = native.Rom(art, tol=tol, max_iter=K)
    rom.set_split(W_)
    xh = torch.zeros(M, dtype=torch.float64, device=dev)
    hist = torch.empty(steps * M, dtype=torch.float64, device=dev)
    it = torch.empty(steps, dtype=torch.int32, device=dev)
    plan = rom.split_plan(steps)
    rom.run(steps, xh, hist, it)
    torch.cuda.synchronize()
    rom.close()
    return plan, hist.cpu().numpy().reshape(steps, M), it.cpu().numpy(), xh.cpu().numpy()


def test_automatic_split_at_the_pipeline_size(dev, c3):
    rom = native.Rom(c3)
    nnz = np.asarray(c3["ids"]).size
    assert nnz > 4096
    assert rom.split_plan(400) == -(-nnz // 1024)
    rom.set_split(1)
    assert rom.split_plan(400) == 1
    rom.close()


@pytest.mark.parametrize("W_", [0, 2, 9, 16])
def test_split_run_matches_oracle(dev, c3, W_):
    # W = 2 leaves slices too long for LDS: the launch widens to the first W
    # whose slice fits
    steps, K = 8, 3
    o = oracle.Rom(c3).run(steps, tol=0.0, max_iter=K)
    plan, h, it, _ = run(c3, W_, steps, K)
    if W_ == 0:
        assert plan == -(-np.asarray(c3["ids"]).size // 1024)
    elif W_ == 2:
        assert 2 < plan <= 6
    else:
        assert plan == W_
    assert np.all(it == K)
    assert np.all(np.isfinite(h))
    assert rel(h, o["hist"]) <= 1e-5


def test_split_matches_one_workgroup(dev, c3):
    # the same terms, summed per slice and then over slices: FP32 rounding apart
    steps, K = 12, 3
    _, h1, i1, x1 = run(c3, 1, steps, K)
    p, h9, i9, x9 = run(c3, 0, steps, K)
    assert p > 1
    assert np.array_equal(i1, i9)
    assert rel(h9, h1) <= 1e-6
    assert rel(x9, x1) <= 1e-6


def test_split_run_is_deterministic(dev, c3):
    steps, K = 6, 3
    _, ha, ia, _ = run(c3, 7, steps, K)
    _, hb, ib, _ = run(c3, 7, steps, K)
    assert np.array_equal(ha, hb) and np.array_equal(ia, ib)


def test_split_run_with_tolerance(dev, c3):
    steps = 20
    o = oracle.Rom(c3).run(steps, tol=1e-4, max_iter=100)
    _, h, it, _ = run(c3, 0, steps, 100, tol=1e-4)
    assert np.all(np.abs(it - o["iters"]) <= 1)
    assert rel(h, o["hist"]) <= 1e-4


@pytest.mark.parametrize("W_", [3, 64])
def test_split_short_lists_and_empty_slices(dev, small, W_):
    # W = 64 over a few hundred entries: slices of a handful of entries, each
    # spanning parts of one or two lists; one sampled body's list emptied
    art = dict(small)
    off_ = np.asarray(art["off"]).copy()
    ids = np.asarray(art["ids"])
    t = 5
    keep = np.r_[0:off_[t], off_[t + 1]:ids.size]
    art["ids"] = ids[keep]
    art["off"] = np.r_[off_[:t + 1], off_[t + 1:] - (off_[t + 1] - off_[t])]
    assert art["off"][t] == art["off"][t + 1]
    steps, K = 6, 3
    o = oracle.Rom(art).run(steps, tol=0.0, max_iter=K)
    p, h, it, _ = run(art, W_, steps, K)
    assert p == W_
    assert np.all(it == K)
    assert rel(h, o["hist"]) <= 1e-5


def test_split_batched_queries(dev, c3):
    # three queries (scaled circulations), W workgroups each, against the
    # oracle per query and against the unsplit batched launch
    M, steps, K, nq = 8, 6, 3, 3
    scales = [1.0, 0.8, 1.25]
    gt = np.stack([np.asarray(c3["Gt"], np.float32) * np.float32(s) for s in scales])
    res = {}
    for W_ in (1, 6):
        rom = native.Rom(c3, tol=0.0, max_iter=K)
        rom.set_split(W_)
        assert rom.split_plan(steps, batched_nq=nq) == W_
        xq = torch.zeros((nq, M), dtype=torch.float64, device=dev)
        hq = torch.empty((nq, steps, M), dtype=torch.float64, device=dev)
        iq = torch.empty((nq, steps), dtype=torch.int32, device=dev)
        rom.run_batched(torch.tensor(gt, device=dev), steps, xq, hq, iq)
        torch.cuda.synchronize()
        res[W_] = (hq.cpu().numpy(), iq.cpu().numpy())
        rom.close()
    for q in range(nq):
        aq = dict(c3)
        aq["Gt"] = gt[q].astype(np.float64)
        o = oracle.Rom(aq).run(steps, tol=0.0, max_iter=K)
        assert np.all(res[6][1][q] == K)
        assert rel(res[6][0][q], o["hist"]) <= 1e-5
        assert rel(res[6][0][q], res[1][0][q]) <= 1e-6


def test_split_abort_path_exits_cleanly(dev, c3):
    # one failed barrier check aborts the launch (forced from the host); every
    # workgroup leaves at its next barrier.  Either the launch aborted (all
    # iters -1, NaN xhat) or, if every wait happened to find its barrier full,
    # it ran normally; a following default run on the same context is exact.
    steps, K = 4, 3
    M = 8
    rom = native.Rom(c3, tol=0.0, max_iter=K)
    rom.set_split(8, max_polls=1)
    xh = torch.zeros(M, dtype=torch.float64, device=dev)
    it = torch.empty(steps, dtype=torch.int32, device=dev)
    rom.run(steps, xh, None, it)
    torch.cuda.synchronize()
    its = it.cpu().numpy()
    o = oracle.Rom(c3).run(steps, tol=0.0, max_iter=K)
    if np.all(its == -1):
        assert np.all(np.isnan(xh.cpu().numpy()))
    else:
        assert np.all(its == K)
        assert rel(xh.cpu().numpy(), o["hist"][-1]) <= 1e-5
    rom.set_split(8)
    xh.zero_()
    hist = torch.empty(steps * M, dtype=torch.float64, device=dev)
    rom.run(steps, xh, hist, it)
    torch.cuda.synchronize()
    assert np.all(it.cpu().numpy() == K)
    assert rel(hist.cpu().numpy().reshape(steps, M), o["hist"]) <= 1e-5
    rom.close()


@pytest.mark.parametrize("shape,W_", [((13, 26, 26), 4), ((21, 42, 42), 3), ((32, 64, 32), 2)])
def test_split_at_larger_basis_bounds(dev, shape, W_):
    # forced splits of the single-vortex study's shapes, one per basis bound
    # (16, 24, 32) of the small kernel
    M, Mr, ns = shape
    art = synth(W.counter_rotating_patches(640, seed=41, delta=0.02), M, Mr, ns, 6, 50 + M)
    steps, K = 6, 3
    o = oracle.Rom(art).run(steps, tol=0.0, max_iter=K)
    p, h, it, _ = run(art, W_, steps, K)
    assert p >= W_
    assert np.all(it == K)
    assert rel(h, o["hist"]) <= 1e-5
    _, h1, i1, _ = run(art, 1, steps, K)
    assert np.array_equal(it, i1)
    assert rel(h, h1) <= 1e-6


def test_set_split_rejects_out_of_range(dev, small):
    rom = native.Rom(small)
    for bad in (-1, 65):
        with pytest.raises(RuntimeError):
            rom.set_split(bad)
    rom.close()
