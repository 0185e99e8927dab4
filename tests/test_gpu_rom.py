"""GPU parity of the online PTROM (HyperPair gather and the device-resident
Gauss-Newton loop) against the oracle's online step on identical offline
artifacts (trained by the oracle's offline pipeline, rounded to FP32 where the
GPU stores FP32)."""
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
    """The artifacts exactly as the GPU holds them (FP32 except A)."""
    a = dict(art)
    for k in ("Phibar", "xbar0", "xqt0", "Phit", "Gt"):
        a[k] = f32(art[k])
    a["delta"] = float(np.float32(art["delta"]))
    a["dt"] = float(np.float32(art["dt"]))
    return a


@pytest.fixture(scope="module")
def trained():
    cl = W.counter_rotating_patches(512, seed=31, delta=0.01)
    art, ex = off.train(cl, dt=1e-3, nsnap=40, M=8, Mr=16, ns=16, depth=6, pc=1.0)
    return cl, rounded(art), ex


@pytest.mark.parametrize("mode", [native.JAC_PAPER, native.JAC_EXACT])
def test_hyperpair_parity(dev, trained, mode):
    cl, art, ex = trained
    nd = 2 * len(art["sample"])
    rom_o = oracle.Rom(art, jac_mode=mode)
    rom_g = native.Rom(art, jac_mode=mode)
    rng = np.random.default_rng(0)
    xh = rng.standard_normal(8) * 0.05
    xp, fp = rng.standard_normal(nd) * 0.1 + art["xbar0"], rng.standard_normal(nd) * 0.1
    xb, fb, rb, C = rom_o.hyperpair(xh, xp, fp)
    t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    gx, gf, gr, gC = rom_g.hyperpair(t(xh), t(xp), t(fp))
    assert rel(gx.cpu().numpy(), xb) <= 1e-14
    assert rel(gf.cpu().numpy(), fb) <= 1e-5
    assert rel(gr.cpu().numpy(), rb) <= 1e-5
    assert rel(gC.cpu().numpy() - art["Phibar"], C - art["Phibar"]) <= 1e-5


def test_gnat_limit_matches_pair_sum(dev, trained):
    # with an infinitely wide neighbourhood nothing is clustered: the gather is
    # the exact pair sum at x0 + Phi xhat on the sampled rows
    cl, art, ex = trained
    n = cl.n
    Phi = f32(ex["Phi"])
    sample = art["sample"]
    a2 = rounded(off.rom_artifacts(sample, ex["tree"], np.inf, f32(cl.xy), Phi, f32(cl.gamma), cl.delta, 1e-3,
                                   A=art["A"]))
    rom = native.Rom(a2)
    xh = np.random.default_rng(1).standard_normal(8) * 0.05
    nd = 2 * sample.size
    t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    _, gf, _, _ = rom.hyperpair(t(xh), t(np.zeros(nd)), t(np.zeros(nd)))
    x = a2["xbar0"] * 0  # unused
    full = f32(cl.xy) + Phi @ xh
    assert rel(gf.cpu().numpy(), oracle.velocity_at(full, f32(cl.gamma), a2["delta"], sample)) <= 1e-5


def test_hook_lists_longer_than_the_lds_union(dev):
    # no clustering over 1600 bodies: every list holds 1599 surrogates, more
    # than a target group's union may hold in LDS, so each target forms a
    # group alone and reads the records from the global table
    cl = W.counter_rotating_patches(1600, seed=47, delta=0.02)
    n, M = cl.n, 8
    rng = np.random.default_rng(48)
    Phi = np.linalg.qr(rng.standard_normal((2 * n, M)))[0]
    sig = np.sort(rng.uniform(1.0, 10.0, M))[::-1]
    tree = off.QuadTree(off.weighted_points(Phi, sig), 6)
    sample = np.sort(rng.choice(n, 12, replace=False))
    A = off.gappy_operator(np.linalg.qr(rng.standard_normal((2 * n, 16)))[0], sample)
    art = rounded(off.rom_artifacts(sample, tree, np.inf, cl.xy, Phi, cl.gamma, cl.delta, 1e-3, A=A))
    assert np.min(np.diff(art["off"])) > 1024
    nd = 2 * sample.size
    xh = rng.standard_normal(M) * 0.05
    xp, fp = rng.standard_normal(nd) * 0.1 + art["xbar0"], rng.standard_normal(nd) * 0.1
    xb, fb, rb, C = oracle.Rom(art).hyperpair(xh, xp, fp)
    t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    gx, gf, gr, gC = native.Rom(art).hyperpair(t(xh), t(xp), t(fp))
    assert rel(gx.cpu().numpy(), xb) <= 1e-14
    assert rel(gf.cpu().numpy(), fb) <= 1e-5
    assert rel(gr.cpu().numpy(), rb) <= 1e-5
    assert rel(gC.cpu().numpy() - art["Phibar"], C - art["Phibar"]) <= 1e-5


@pytest.mark.parametrize("mode", [native.JAC_PAPER, native.JAC_EXACT])
def test_rom_run_fixed_iterations(dev, trained, mode):
    # tol = 0 forces exactly max_iter Gauss-Newton iterations per step on both
    # sides, so the xhat histories are compared without a tolerance crossing.
    cl, art, ex = trained
    steps, K = 30, 4
    o = oracle.Rom(art, jac_mode=mode).run(steps, tol=0.0, max_iter=K)
    rom = native.Rom(art, tol=0.0, max_iter=K, jac_mode=mode)
    xh = torch.zeros(8, dtype=torch.float64, device=dev)
    hist = torch.empty(steps * 8, dtype=torch.float64, device=dev)
    it = torch.empty(steps, dtype=torch.int32, device=dev)
    rom.run(steps, xh, hist, it)
    assert np.all(it.cpu().numpy() == K) and np.all(o["iters"] == K)
    assert rel(hist.cpu().numpy().reshape(steps, 8), o["hist"]) <= 1e-5


def test_rom_run_with_tolerance(dev, trained):
    cl, art, ex = trained
    steps = 40
    o = oracle.Rom(art).run(steps, tol=1e-4, max_iter=100)
    rom = native.Rom(art, tol=1e-4, max_iter=100)
    xh = torch.zeros(8, dtype=torch.float64, device=dev)
    hist = torch.empty(steps * 8, dtype=torch.float64, device=dev)
    it = torch.empty(steps, dtype=torch.int32, device=dev)
    rom.run(steps, xh, hist, it)
    its = it.cpu().numpy()
    assert np.all(np.abs(its - o["iters"]) <= 1)
    assert rel(hist.cpu().numpy().reshape(steps, 8), o["hist"]) <= 1e-4


def test_rom_rejects_bad_ids(dev, trained):
    cl, art, ex = trained
    bad = dict(art)
    bad["ids"] = np.array(art["ids"]).copy()
    bad["ids"][0] = len(art["Gt"]) + 5
    with pytest.raises(native.PtromError):
        native.Rom(bad)


@pytest.mark.parametrize("mode", [native.JAC_PAPER, native.JAC_EXACT])
def test_surrogate_on_its_target_at_zero_core(dev, trained, mode):
    # delta = 0 and one more source placed on sampled target 0 for every xhat
    # (its own x0 and mode rows): finite, and equal to the oracle, which
    # drops such a pair like the self pair.
    cl, art, ex = trained
    ns = len(art["sample"])
    a = dict(art)
    a["delta"] = 0.0
    Nc = art["Gt"].size
    M = art["Phibar"].shape[1]
    a["xqt0"] = np.vstack([art["xqt0"], [[art["xbar0"][0], art["xbar0"][ns]]]])
    a["Phit"] = np.concatenate([art["Phit"], np.stack([art["Phibar"][0], art["Phibar"][ns]])[None]])
    a["Gt"] = np.append(art["Gt"], f32(0.3))
    off_ = np.asarray(art["off"]).copy()
    ids = list(art["ids"])
    ids.insert(int(off_[1]), Nc)
    off_[1:] += 1
    a["off"], a["ids"] = off_, np.asarray(ids, dtype=np.int64)
    nd = 2 * ns
    rng = np.random.default_rng(3)
    xh = rng.standard_normal(M) * 0.05
    xp, fp = rng.standard_normal(nd) * 0.1 + art["xbar0"], rng.standard_normal(nd) * 0.1
    xb, fb, rb, C = oracle.Rom(a, jac_mode=mode).hyperpair(xh, xp, fp)
    t = lambda v: torch.tensor(v, dtype=torch.float64, device=dev)
    gx, gf, gr, gC = native.Rom(a, jac_mode=mode).hyperpair(t(xh), t(xp), t(fp))
    for g in (gx, gf, gr, gC):
        assert torch.isfinite(g).all()
    assert rel(gf.cpu().numpy(), fb) <= 1e-5
    assert rel(gr.cpu().numpy(), rb) <= 1e-5
    assert rel(gC.cpu().numpy() - a["Phibar"], C - a["Phibar"]) <= 1e-5


@pytest.fixture(scope="module")
def trained_shapes():
    """Well-conditioned artifacts at the paper's single-vortex sizes (M = 21,
    M_r = n_s = 42), at the largest supported basis (M = 32, M_r = 64) and
    with a sample set too large for the run kernel's LDS copies (n_s = 400).
    Phi and Phi_r are random orthonormal bases (a trained basis of this rank
    would need far richer snapshots); the clustering, sampling and gappy
    operator are built exactly as in training."""
    out = {}
    cl = W.counter_rotating_patches(640, seed=41, delta=0.02)
    n = cl.n
    rng = np.random.default_rng(42)
    for M, Mr, ns in [(21, 42, 42), (32, 64, 32), (8, 16, 400)]:
        Phi = np.linalg.qr(rng.standard_normal((2 * n, M)))[0]
        sig = np.sort(rng.uniform(1.0, 10.0, M))[::-1]
        tree = off.QuadTree(off.weighted_points(Phi, sig), 6)
        sample = np.sort(rng.choice(n, ns, replace=False))
        Phi_r = np.linalg.qr(rng.standard_normal((2 * n, Mr)))[0]
        A = off.gappy_operator(Phi_r, sample)
        out[(M, Mr, ns)] = rounded(off.rom_artifacts(sample, tree, 1.0, cl.xy, Phi, cl.gamma, cl.delta, 1e-3, A=A))
    return out


@pytest.mark.parametrize("shape", [(21, 42, 42), (32, 64, 32), (8, 16, 400)])
@pytest.mark.parametrize("mode", [native.JAC_PAPER, native.JAC_EXACT])
def test_rom_run_shapes(dev, trained_shapes, shape, mode):
    art = trained_shapes[shape]
    M = shape[0]
    steps, K = 12, 3
    o = oracle.Rom(art, jac_mode=mode).run(steps, tol=0.0, max_iter=K)
    rom = native.Rom(art, tol=0.0, max_iter=K, jac_mode=mode)
    xh = torch.zeros(M, dtype=torch.float64, device=dev)
    hist = torch.empty(steps * M, dtype=torch.float64, device=dev)
    it = torch.empty(steps, dtype=torch.int32, device=dev)
    rom.run(steps, xh, hist, it)
    torch.cuda.synchronize()
    assert np.all(it.cpu().numpy() == K)
    h = hist.cpu().numpy().reshape(steps, M)
    assert np.all(np.isfinite(h))
    assert rel(h, o["hist"]) <= 1e-5


LARGE = [(48, 96, 48), (85, 110, 60), (110, 185, 75)]


@pytest.fixture(scope="module")
def large_shapes():
    """Bases beyond 32 (the blocked path): M = 48 / M_r = 96 / n_s = 48, the
    paper's vortex-pair sizes M = 85 / M_r = 110 / n_s = 60 and its
    mushroom-cloud sizes M = 110 / M_r = 185 / n_s = 75 (with the inflow as a
    background velocity), with random orthonormal Phi and Phi_r and the
    training clustering and sampling."""
    out = {}
    cl = W.counter_rotating_patches(640, seed=43, delta=0.02)
    n = cl.n
    rng = np.random.default_rng(44)
    for M, Mr, ns in LARGE:
        Phi = np.linalg.qr(rng.standard_normal((2 * n, M)))[0]
        sig = np.sort(rng.uniform(1.0, 10.0, M))[::-1]
        tree = off.QuadTree(off.weighted_points(Phi, sig), 6)
        sample = np.sort(rng.choice(n, ns, replace=False))
        Phi_r = np.linalg.qr(rng.standard_normal((2 * n, Mr)))[0]
        A = off.gappy_operator(Phi_r, sample)
        u = 0.1 * W.mushroom_inflow(n) if M > 96 else None
        out[(M, Mr, ns)] = rounded(off.rom_artifacts(sample, tree, 1.0, cl.xy, Phi, cl.gamma, cl.delta, 1e-3, A=A,
                                                     u=u))
    return out


@pytest.mark.parametrize("shape", LARGE)
def test_large_hyperpair_parity(dev, large_shapes, shape):
    art = large_shapes[shape]
    M = shape[0]
    nd = 2 * shape[2]
    rng = np.random.default_rng(5)
    xh = rng.standard_normal(M) * 0.02
    xp, fp = rng.standard_normal(nd) * 0.1 + art["xbar0"], rng.standard_normal(nd) * 0.1
    xb, fb, rb, C = oracle.Rom(art).hyperpair(xh, xp, fp)
    t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    gx, gf, gr, gC = native.Rom(art).hyperpair(t(xh), t(xp), t(fp))
    assert rel(gx.cpu().numpy(), xb) <= 1e-14
    assert rel(gf.cpu().numpy(), fb) <= 1e-5
    assert rel(gr.cpu().numpy(), rb) <= 1e-5
    assert rel(gC.cpu().numpy() - art["Phibar"], C - art["Phibar"]) <= 1e-5


@pytest.mark.parametrize("shape", LARGE)
def test_large_run_fixed_iterations(dev, large_shapes, shape):
    art = large_shapes[shape]
    M = shape[0]
    steps, K = 10, 3
    o = oracle.Rom(art).run(steps, tol=0.0, max_iter=K)
    rom = native.Rom(art, tol=0.0, max_iter=K)
    xh = torch.zeros(M, dtype=torch.float64, device=dev)
    hist = torch.empty(steps * M, dtype=torch.float64, device=dev)
    it = torch.empty(steps, dtype=torch.int32, device=dev)
    rom.run(steps, xh, hist, it)
    torch.cuda.synchronize()
    assert np.all(it.cpu().numpy() == K)
    h = hist.cpu().numpy().reshape(steps, M)
    assert np.all(np.isfinite(h))
    assert rel(h, o["hist"]) <= 1e-5


def test_large_batched_queries(dev, large_shapes):
    art = large_shapes[(48, 96, 48)]
    M, steps, K, nq = 48, 8, 3, 3
    scales = [1.0, 0.7, 1.3]
    gt = np.stack([np.asarray(art["Gt"]) * s for s in scales]).astype(np.float32)
    rom = native.Rom(art, tol=0.0, max_iter=K)
    xq = torch.zeros((nq, M), dtype=torch.float64, device=dev)
    hq = torch.empty((nq, steps, M), dtype=torch.float64, device=dev)
    rom.run_batched(torch.tensor(gt, device=dev), steps, xq, hq, None)
    torch.cuda.synchronize()
    for q in range(nq):
        aq = dict(art)
        aq["Gt"] = gt[q].astype(np.float64)
        o = oracle.Rom(aq).run(steps, tol=0.0, max_iter=K)
        assert rel(hq[q].cpu().numpy(), o["hist"]) <= 1e-5, q


def test_large_exact_jacobian_rejected(dev, large_shapes):
    with pytest.raises(native.PtromError):
        native.Rom(large_shapes[(48, 96, 48)], jac_mode=native.JAC_EXACT)


def test_large_inflow_enters_the_residual(dev, large_shapes):
    # The same artifacts without their background velocity give a different
    # trajectory, which the GPU also follows.
    art = large_shapes[(110, 185, 75)]
    assert "ubar" in art
    art0 = dict(art)
    del art0["ubar"]
    steps, K, M = 4, 3, 110
    hs = []
    for a in (art, art0):
        rom = native.Rom(a, tol=0.0, max_iter=K)
        xh = torch.zeros(M, dtype=torch.float64, device=dev)
        hist = torch.empty(steps * M, dtype=torch.float64, device=dev)
        rom.run(steps, xh, hist, None)
        torch.cuda.synchronize()
        hs.append(hist.cpu().numpy().reshape(steps, M))
    o0 = oracle.Rom(art0).run(steps, tol=0.0, max_iter=K)
    assert rel(hs[1], o0["hist"]) <= 1e-5
    assert rel(hs[0], hs[1]) > 1e-3


@pytest.mark.parametrize("mode", [native.JAC_PAPER, native.JAC_EXACT])
def test_small_path_inflow_parity(dev, trained, mode):
    cl, art, ex = trained
    a = dict(art)
    nd = 2 * len(art["sample"])
    rng = np.random.default_rng(12)
    a["ubar"] = rng.uniform(0.5, 3.0, nd) * 1e-2
    xh = rng.standard_normal(8) * 0.05
    xp, fp = rng.standard_normal(nd) * 0.1 + a["xbar0"], rng.standard_normal(nd) * 0.1
    xb, fb, rb, C = oracle.Rom(a, jac_mode=mode).hyperpair(xh, xp, fp)
    t = lambda v: torch.tensor(v, dtype=torch.float64, device=dev)
    gx, gf, gr, gC = native.Rom(a, jac_mode=mode).hyperpair(t(xh), t(xp), t(fp))
    assert rel(gf.cpu().numpy(), fb) <= 1e-5
    assert rel(gr.cpu().numpy(), rb) <= 1e-5
    steps, K = 12, 3
    o = oracle.Rom(a, jac_mode=mode).run(steps, tol=0.0, max_iter=K)
    rom = native.Rom(a, tol=0.0, max_iter=K, jac_mode=mode)
    x = torch.zeros(8, dtype=torch.float64, device=dev)
    hist = torch.empty(steps * 8, dtype=torch.float64, device=dev)
    rom.run(steps, x, hist, None)
    torch.cuda.synchronize()
    assert rel(hist.cpu().numpy().reshape(steps, 8), o["hist"]) <= 1e-5


# ------------------------------------------------------------ edges of the blocked path

EDGE = [(33, 33, 17), (20, 65, 40), (112, 120, 61)]


@pytest.fixture(scope="module")
def edge_shapes():
    """Just past the small kernel (M = 33; M_r = 65 with M = 20), the largest
    basis (M = 112) and odd n_s (n_d not a multiple of 4), plus a shape whose
    arrays exceed one workgroup's LDS (M = 112, M_r = 256, n_s = 128)."""
    out = {}
    cl = W.counter_rotating_patches(640, seed=43, delta=0.02)
    n = cl.n
    rng = np.random.default_rng(45)
    for M, Mr, ns in EDGE + [(112, 256, 128)]:
        Phi = np.linalg.qr(rng.standard_normal((2 * n, M)))[0]
        sig = np.sort(rng.uniform(1.0, 10.0, M))[::-1]
        tree = off.QuadTree(off.weighted_points(Phi, sig), 6)
        sample = np.sort(rng.choice(n, ns, replace=False))
        Phi_r = np.linalg.qr(rng.standard_normal((2 * n, Mr)))[0]
        A = off.gappy_operator(Phi_r, sample)
        out[(M, Mr, ns)] = rounded(off.rom_artifacts(sample, tree, 1.0, cl.xy, Phi, cl.gamma, cl.delta, 1e-3, A=A))
    return out


def _hyperpair_check(dev, art, seed):
    M, nd = int(art["M"]), 2 * (len(art["off"]) - 1)
    rng = np.random.default_rng(seed)
    xh = rng.standard_normal(M) * 0.02
    xp, fp = rng.standard_normal(nd) * 0.1 + art["xbar0"], rng.standard_normal(nd) * 0.1
    xb, fb, rb, C = oracle.Rom(art).hyperpair(xh, xp, fp)
    t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    gx, gf, gr, gC = native.Rom(art).hyperpair(t(xh), t(xp), t(fp))
    assert rel(gx.cpu().numpy(), xb) <= 1e-14
    assert rel(gf.cpu().numpy(), fb) <= 1e-5
    assert rel(gr.cpu().numpy(), rb) <= 1e-5
    assert rel(gC.cpu().numpy() - art["Phibar"], C - art["Phibar"]) <= 1e-5


def _run_check(dev, art, steps=6, K=3):
    M = int(art["M"])
    o = oracle.Rom(art).run(steps, tol=0.0, max_iter=K)
    rom = native.Rom(art, tol=0.0, max_iter=K)
    xh = torch.zeros(M, dtype=torch.float64, device=dev)
    hist = torch.empty(steps * M, dtype=torch.float64, device=dev)
    it = torch.empty(steps, dtype=torch.int32, device=dev)
    rom.run(steps, xh, hist, it)
    torch.cuda.synchronize()
    assert np.all(it.cpu().numpy() == K)
    h = hist.cpu().numpy().reshape(steps, M)
    assert np.all(np.isfinite(h))
    assert rel(h, o["hist"]) <= 1e-5


@pytest.mark.parametrize("shape", EDGE)
def test_edge_shapes_parity(dev, edge_shapes, shape):
    _hyperpair_check(dev, edge_shapes[shape], 7)
    _run_check(dev, edge_shapes[shape])


BOUNDS = [(1, 2, 1), (9, 18, 9), (17, 34, 17), (25, 50, 25)]


@pytest.fixture(scope="module")
def bound_shapes():
    """The degenerate one-mode, one-body case (M = 1, M_r = 2, n_s = 1) and
    the first basis size of each of the small kernel's bounds 16, 24 and 32."""
    out = {}
    cl = W.counter_rotating_patches(640, seed=47, delta=0.02)
    n = cl.n
    rng = np.random.default_rng(48)
    for M, Mr, ns in BOUNDS:
        Phi = np.linalg.qr(rng.standard_normal((2 * n, M)))[0]
        sig = np.sort(rng.uniform(1.0, 10.0, M))[::-1]
        tree = off.QuadTree(off.weighted_points(Phi, sig), 6)
        sample = np.sort(rng.choice(n, ns, replace=False))
        Phi_r = np.linalg.qr(rng.standard_normal((2 * n, Mr)))[0]
        A = off.gappy_operator(Phi_r, sample)
        out[(M, Mr, ns)] = rounded(off.rom_artifacts(sample, tree, 1.0, cl.xy, Phi, cl.gamma, cl.delta, 1e-3, A=A))
    return out


@pytest.mark.parametrize("shape", BOUNDS)
def test_basis_bound_shapes_parity(dev, bound_shapes, shape):
    _hyperpair_check(dev, bound_shapes[shape], 11)
    _run_check(dev, bound_shapes[shape])


def test_largest_shape_beyond_lds_runs_from_global_memory(dev, edge_shapes):
    # arrays that do not fit one workgroup's LDS: [C | rbar] and the normal
    # matrix go to global memory and the run matches the oracle
    art = edge_shapes[(112, 256, 128)]
    _hyperpair_check(dev, art, 8)
    _run_check(dev, art)


def _drop_list(art, t):
    """The artifacts with target t's interaction list emptied."""
    a = dict(art)
    off_, ids = np.asarray(art["off"]), np.asarray(art["ids"])
    a["ids"] = np.concatenate([ids[:off_[t]], ids[off_[t + 1]:]])
    a["off"] = np.concatenate([off_[:t + 1], off_[t + 1:] - (off_[t + 1] - off_[t])])
    return a


def test_empty_list_parity(dev, trained, large_shapes):
    # a target whose list is empty feels no velocity and no 2 x 2 block; both
    # kernels and the gather entry point take it like the oracle
    cl, art_small, ex = trained
    for art in (art_small, large_shapes[(48, 96, 48)]):
        a = _drop_list(art, 1)
        assert a["off"][1] == a["off"][2]
        _hyperpair_check(dev, a, 9)
        _run_check(dev, a)


@pytest.fixture(scope="module")
def trained_large():
    """Artifacts trained by the oracle's offline pipeline at the paper's
    parametric sizes: the vortex pair (N = 500, M = 85, M_r = 110, n_s = 60)
    and the mushroom cloud with its inflow (N = 500, M = 110, M_r = 185,
    n_s = 75), four training parameters each, over the first 30 steps of the
    studies' time step (the full horizon takes minutes in the oracle)."""
    out = {}
    vp = [W.vortex_pair(m) for m in ((80.0, 200.0), (150.0, 100.0), (230.0, 240.0), (110.0, 70.0))]
    art, _ = off.train_parametric(vp, 0.01, 30, M=85, Mr=110, ns=60, depth=16, pc=1.0, tol=1e-4)
    out["vortex_pair"] = rounded(art)
    mc = [W.mushroom_cloud(m) for m in ((-200.0, 130.0), (-120.0, 210.0), (-170.0, 170.0), (-140.0, 120.0))]
    u = W.mushroom_inflow(500)
    art, ex = off.train_parametric(mc, 0.005, 30, M=110, Mr=185, ns=75, depth=16, pc=1.0, tol=1e-4, u=u)
    out["mushroom_cloud"] = rounded(art)
    # the same training with n_s = 120 sampled bodies (2 n_s >= M_r): the
    # query's arrays pass one workgroup's LDS, so [C | rbar] and the normal
    # matrix live in global memory
    sample = off.greedy_sample(ex["Phi_r"], 120)
    A = off.gappy_operator(ex["Phi_r"], sample)
    x0 = np.asarray(mc[0].xy, dtype=np.float64)
    a120 = off.rom_artifacts(sample, ex["tree"], 1.0, x0, ex["Phi"], ex["weights"], float(mc[0].delta), 0.005,
                             A=A, u=u)
    out["mushroom_cloud_ns120"] = rounded(a120)
    return out


@pytest.mark.parametrize("case", ["vortex_pair", "mushroom_cloud", "mushroom_cloud_ns120"])
def test_large_run_trained_artifacts(dev, trained_large, case):
    # the larger-basis path (normal equations of A C on the FP64 matrix cores,
    # blocked Gauss-Jordan, C held in FP32) on trained artifacts, fixed K
    # Gauss-Newton iterations per step, against the oracle's Householder QR
    art = trained_large[case]
    M = art["M"]
    xb, fb, rb, C = oracle.Rom(art).hyperpair(np.zeros(M), art["xbar0"], np.zeros(len(art["xbar0"])))
    cond = np.linalg.cond(art["A"] @ C)
    steps, K = 12, 3
    o = oracle.Rom(art).run(steps, tol=0.0, max_iter=K)
    rom = native.Rom(art, tol=0.0, max_iter=K)
    xh = torch.zeros(M, dtype=torch.float64, device=dev)
    hist = torch.empty(steps * M, dtype=torch.float64, device=dev)
    it = torch.empty(steps, dtype=torch.int32, device=dev)
    rom.run(steps, xh, hist, it)
    torch.cuda.synchronize()
    assert np.all(it.cpu().numpy() == K)
    h = hist.cpu().numpy().reshape(steps, M)
    assert np.all(np.isfinite(h))
    assert rel(h, o["hist"]) <= 1e-5, "cond(AC) = %.3g" % cond
    rom.close()
