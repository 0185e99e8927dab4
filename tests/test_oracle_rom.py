"""Pins of the oracle's PTROM pieces (offline training and the online
Gauss-Newton / HyperPair step) against special cases whose answer is known
without the ROM: no clustering reproduces the exact pair sum (GNAT limit of an
infinitely wide neighbourhood), cluster surrogates are linear in xhat, full-rank
LSPG reproduces the trapezoid FOM, the greedy sampler on hand-made bases."""
import numpy as np
import pytest

import oracle
from oracle import offline as off
from paper_2103_01983_amd import workloads as W


@pytest.fixture(scope="module")
def small_problem():
    cl = W.counter_rotating_patches(192, seed=77, delta=0.05)
    S = off.trapezoid_snapshots(cl.xy, cl.gamma, cl.delta, 2e-3, 24)
    Phi, sig = off.pod(S, 6)
    tree = off.QuadTree(off.weighted_points(Phi, sig), 6)
    return cl, S, Phi, sig, tree


def test_pod_basis_properties(small_problem):
    cl, S, Phi, sig, _ = small_problem
    np.testing.assert_allclose(Phi.T @ Phi, np.eye(Phi.shape[1]), atol=1e-12)
    # columns are eigenvectors of S S^T with eigenvalues sigma^2
    np.testing.assert_allclose(S @ (S.T @ Phi), Phi * sig ** 2, rtol=0, atol=1e-9 * sig[0] ** 2)
    assert np.all(np.diff(sig) <= 0)


def test_quadtree_partition(small_problem):
    cl, _, Phi, sig, tree = small_problem
    P = off.weighted_points(Phi, sig)
    n = cl.n
    seen = np.zeros(n, int)
    for nd in tree.nodes:
        if not nd.children:
            for j in nd.members:
                seen[j] += 1
                assert np.all(P[j] >= nd.lo - 1e-15) and np.all(P[j] <= nd.hi + 1e-15)
            assert len(nd.members) == 1 or nd.level == tree.max_level
        else:
            assert sorted(sum((c.members for c in nd.children), [])) == sorted(nd.members)
        assert nd.level <= tree.max_level
    assert np.all(seen == 1)


def test_surrogates_are_weighted_means_for_every_xhat(small_problem):
    # x0_c + Phit_c xhat equals the |Gamma|-weighted mean of the members'
    # x0 + Phi xhat, for any xhat; the root carries the total circulation.
    cl, _, Phi, sig, tree = small_problem
    n = cl.n
    rng = np.random.default_rng(0)
    xh = rng.standard_normal(Phi.shape[1])
    x = cl.xy + Phi @ xh
    for nd in tree.nodes[:40]:
        x0c, phc, gc = off.node_surrogates(nd, cl.xy, Phi, cl.gamma)
        w = np.abs(cl.gamma[nd.members])
        mean = np.array([np.sum(w * x[nd.members]), np.sum(w * x[n + np.array(nd.members)])]) / w.sum()
        np.testing.assert_allclose(x0c + phc @ xh, mean, atol=1e-13)
    assert off.node_surrogates(tree.root, cl.xy, Phi, cl.gamma)[2] == pytest.approx(cl.gamma.sum(), abs=1e-15)


def test_no_clustering_gives_exact_sampled_rows(small_problem):
    # An infinitely wide neighbourhood prunes nothing: every target sees every
    # other body, so HyperPair's velocity must equal the full pair sum at
    # x0 + Phi xhat on the sampled rows (the GNAT limit).
    cl, _, Phi, sig, tree = small_problem
    n = cl.n
    sample = np.array([0, 5, 90, 191])
    art = off.rom_artifacts(sample, tree, np.inf, cl.xy, Phi, cl.gamma, cl.delta, 1e-3)
    assert art["Gt"].size == n and np.all(np.diff(art["off"]) == n - 1)
    rom = oracle.Rom(art)
    xh = np.random.default_rng(1).standard_normal(Phi.shape[1]) * 0.1
    xbar, fbar, rbar, C = rom.hyperpair(xh, np.zeros(8), np.zeros(8))
    x = cl.xy + Phi @ xh
    np.testing.assert_allclose(xbar, x[off.sampled_rows(sample, n)], atol=1e-14)
    np.testing.assert_allclose(fbar, oracle.velocity_at(x, cl.gamma, cl.delta, sample), rtol=1e-12, atol=1e-14)
    # exact-mode C = (I - dt/2 J) Phi on the sampled rows
    rom1 = oracle.Rom(art, jac_mode=1)
    _, _, _, C1 = rom1.hyperpair(xh, np.zeros(8), np.zeros(8))
    JPhi = np.stack([oracle.jvp(x, cl.gamma, cl.delta, Phi[:, q]) for q in range(Phi.shape[1])], axis=1)
    expect = Phi - 0.5e-3 * JPhi
    np.testing.assert_allclose(C1, expect[off.sampled_rows(sample, n)], rtol=1e-11, atol=1e-13)


def test_pruned_lists_cover_every_body_once(small_problem):
    cl, _, Phi, sig, tree = small_problem
    keys_nodes = {nd.key: nd for nd in tree.nodes}
    for i in [0, 17, 100, 191]:
        members = []
        for k in off.find_clusters(tree, i, 1.0):
            members.extend([k[1]] if k[0] == 0 else keys_nodes[k].members)
        assert sorted(members) == [j for j in range(cl.n) if j != i]


def test_full_rank_lspg_reproduces_trapezoid_fom():
    # With Phi spanning the centred trapezoid snapshots, no clustering and no
    # hyper-reduction, the LSPG minimiser is the FOM state (zero residual).
    cl = W.gaussian_patch(64, seed=3, delta=0.05)
    g = cl.gamma * 64
    dt, T = 2e-3, 6
    S = off.trapezoid_snapshots(cl.xy, g, cl.delta, dt, T)
    Phi, sig = off.pod(S, T, x0=cl.xy)
    tree = off.QuadTree(off.weighted_points(Phi, sig), 6)
    art = off.rom_artifacts(np.arange(64), tree, np.inf, cl.xy, Phi, g, cl.delta, dt)
    out = oracle.Rom(art, jac_mode=1).run(T, tol=1e-13, max_iter=30)
    assert out["status"] == 0
    rec = cl.xy[:, None] + Phi @ out["hist"].T
    np.testing.assert_allclose(rec, S, rtol=0, atol=1e-9)


def test_gauss_newton_stops_on_relative_gradient():
    cl = W.gaussian_patch(48, seed=5, delta=0.05)
    g = cl.gamma * 48
    S = off.trapezoid_snapshots(cl.xy, g, cl.delta, 2e-3, 8)
    Phi, sig = off.pod(S, 3, x0=cl.xy)
    tree = off.QuadTree(off.weighted_points(Phi, sig), 6)
    art = off.rom_artifacts(np.arange(48), tree, 1.0, cl.xy, Phi, g, cl.delta, 2e-3)
    rom = oracle.Rom(art)
    out = rom.run(4, tol=1e-3, max_iter=100)
    assert out["status"] == 0 and np.all(out["iters"] >= 2)
    capped = rom.run(4, tol=0.0, max_iter=3)
    assert capped["status"] == 1 and np.all(capped["iters"] == 3)


def test_greedy_hand_made_basis():
    n = 10
    Phi_r = np.zeros((2 * n, 2))
    Phi_r[3, 0] = 1.0            # body 3, chi row
    Phi_r[n + 7, 1] = 1.0        # body 7, psi row
    assert list(off.greedy_sample(Phi_r, 2)) == [3, 7]
    # ties go to the lowest body index
    Phi_r2 = np.zeros((2 * n, 1)); Phi_r2[[2, 5, n + 8], 0] = 1.0
    assert list(off.greedy_sample(Phi_r2, 1)) == [2]


def test_greedy_full_sample_and_gappy_operator():
    rng = np.random.default_rng(2)
    n = 12
    Phi_r = np.linalg.qr(rng.standard_normal((2 * n, 6)))[0]
    assert list(off.greedy_sample(Phi_r, n)) == list(range(n))
    s = off.greedy_sample(Phi_r, 4)
    A = off.gappy_operator(Phi_r, s)
    # gappy reconstruction is exact for vectors in the span of Phi_r
    z = rng.standard_normal(6)
    r = Phi_r @ z
    np.testing.assert_allclose(A @ r[off.sampled_rows(s, n)], z, atol=1e-10)


def test_full_pipeline_small():
    cl = W.counter_rotating_patches(128, seed=9, delta=0.05)
    art, ex = off.train(cl, dt=2e-3, nsnap=12, M=4, Mr=8, ns=8, depth=6, pc=1.0)
    assert art["A"].shape == (8, 16) and art["Phibar"].shape == (16, 4)
    out = oracle.Rom(art).run(12, tol=1e-4)
    assert out["status"] == 0
    assert np.all(np.isfinite(out["hist"]))


def _with_extra_source(art, target, x0, phit, gt):
    """Copy of ``art`` with one more surrogate source appended to the list of
    sampled target ``target``."""
    a = dict(art)
    Nc = art["Gt"].size
    a["xqt0"] = np.vstack([art["xqt0"], np.asarray(x0, float)[None]])
    a["Phit"] = np.concatenate([art["Phit"], np.asarray(phit, float)[None]])
    a["Gt"] = np.append(art["Gt"], gt)
    off_ = np.asarray(art["off"]).copy()
    ids = list(art["ids"])
    ids.insert(int(off_[target + 1]), Nc)
    off_[target + 1:] += 1
    a["off"], a["ids"] = off_, np.asarray(ids, dtype=np.int64)
    return a


@pytest.mark.parametrize("mode", [0, 1])
def test_surrogate_on_its_target_adds_nothing(small_problem, mode):
    # At delta = 0 a surrogate that sits exactly on its sampled target has no
    # defined velocity; like the excluded self pair it contributes nothing,
    # so velocity, residual and Jacobian equal those of the list without it.
    cl, _, Phi, sig, tree = small_problem
    n = cl.n
    sample = np.array([3, 40, 150])
    art = off.rom_artifacts(sample, tree, 1.0, cl.xy, Phi, cl.gamma, 0.0, 1e-3)
    t = 1
    rows = off.sampled_rows(sample, n)
    # same initial position and same mode rows as body 40: coincident for all xhat
    extra = _with_extra_source(art, t, [cl.xy[40], cl.xy[n + 40]], [Phi[40], Phi[n + 40]], 0.7)
    xh = np.random.default_rng(4).standard_normal(Phi.shape[1]) * 0.01
    xp, fp = cl.xy[rows] + 0.01, np.zeros(rows.size)
    a = oracle.Rom(art, jac_mode=mode).hyperpair(xh, xp, fp)
    b = oracle.Rom(extra, jac_mode=mode).hyperpair(xh, xp, fp)
    for u, v in zip(a, b):
        assert np.all(np.isfinite(v))
        np.testing.assert_array_equal(u, v)


def _line_problem(n=100, steps=2000):
    """Bodies evenly spaced on the diagonal around one strong vortex, delta = 0
    (the single-vortex study's initial state): Gamma-weighted means of two
    bodies symmetric about a third fall exactly on it."""
    s = np.linspace(-n, n, n)
    g = np.full(n, 0.01)
    g[n // 2] = 500.0
    xy = np.concatenate([s, s])
    S = off.trapezoid_snapshots(xy, g, 0.0, 0.01, steps)
    return xy, g, S


def test_cells_on_their_target_are_opened():
    xy, g, S = _line_problem()
    n = g.size
    Phi, sig = off.pod(S, 13)
    rng = np.random.default_rng(11)
    by_key_fired = 0
    for trial in range(16):
        sg = np.ones(13) if trial == 0 else rng.choice([-1.0, 1.0], 13)
        tree = off.QuadTree(off.weighted_points(Phi * sg, sig), 16)
        nodes = {nd.key: nd for nd in tree.nodes}
        for i in range(n):
            plain = off.find_clusters(tree, i, 0.0, gamma=g)
            guarded = off.find_clusters(tree, i, 0.0, gamma=g, xy0=xy)
            # every other body is still represented exactly once
            members = []
            for k in guarded:
                members.extend([k[1]] if k[0] == 0 else nodes[k].members)
            assert sorted(members) == [j for j in range(n) if j != i]
            for k in guarded:
                if k[0] != 0:
                    x0c = off.node_surrogates(nodes[k], xy, Phi, g)[0]
                    assert np.hypot(*(x0c - [xy[i], xy[n + i]])) > 1e-9 * (1 + np.hypot(xy[i], xy[n + i]))
            if plain != guarded:
                by_key_fired += 1
                # only coincident cells were opened
                for k in set(plain) - set(guarded):
                    assert off.coincides(nodes[k], i, xy, g)
    assert by_key_fired > 0  # the configuration does produce coincident cells


def test_pod_sign_convention():
    rng = np.random.default_rng(8)
    S = rng.standard_normal((40, 15))
    Phi, sig = off.pod(S, 5)
    for m in range(5):
        j = np.argmax(np.abs(Phi[:, m]))
        assert Phi[j, m] > 0
    # the same basis for a column-permuted snapshot set
    Phi2, _ = off.pod(S[:, rng.permutation(15)], 5)
    np.testing.assert_allclose(Phi2, Phi, atol=1e-12)


def test_reassigned_circulation_pins(small_problem):
    cl, _, Phi, sig, tree = small_problem
    n = cl.n
    sample = np.array([0, 7, 100, 150, 191])
    art = off.rom_artifacts(sample, tree, 1.0, cl.xy, Phi, cl.gamma, cl.delta, 1e-3)
    mem = off.surrogate_members(tree, art["keys"])
    # at the training parameter the reassignment is the training Gamma~
    np.testing.assert_array_equal(off.reassign_circulation(mem, cl.gamma), art["Gt"])
    rng = np.random.default_rng(3)
    ga, gb = rng.standard_normal(n), rng.standard_normal(n)
    ra, rb = off.reassign_circulation(mem, ga), off.reassign_circulation(mem, gb)
    # linear in Gamma
    np.testing.assert_allclose(off.reassign_circulation(mem, 2.0 * ga - gb), 2.0 * ra - rb, rtol=0, atol=1e-12)
    # every target's list carries the total circulation of all other bodies
    for t, i in enumerate(sample):
        ids = art["ids"][art["off"][t]:art["off"][t + 1]]
        assert ra[ids].sum() == pytest.approx(ga.sum() - ga[i], abs=1e-11)


def test_parametric_training_small():
    # two training parameters of a small vortex pair; the online ROM with the
    # reassigned circulation follows the FOM at a training point and stays
    # finite at an untrained one
    mus = [(40.0, 55.0), (60.0, 30.0)]
    clouds = [W.vortex_pair(m, n=48, half=5.0, delta=0.21) for m in mus]
    dt, steps = 0.01, 40
    art, ex = off.train_parametric(clouds, dt, steps, M=16, Mr=32, ns=24, depth=6, pc=1.0, tol=1e-6)
    assert ex["S"].shape[1] == 2 * steps
    n = clouds[0].n
    x0 = clouds[0].xy
    for mu, trained in [(mus[0], True), ((50.0, 45.0), False)]:
        a = dict(art)
        a["Gt"] = off.reassign_circulation(art["members"], W.vortex_pair(mu, n=48, half=5.0).gamma)
        out = oracle.Rom(a).run(steps, tol=1e-6, max_iter=100)
        assert out["status"] == 0 and np.all(np.isfinite(out["hist"]))
        if trained:
            rec = x0[:, None] + ex["Phi"] @ out["hist"].T
            S = ex["S"][:, :steps]
            err = np.linalg.norm(rec - S) / np.linalg.norm(S - x0[:, None])
            assert err < 0.05, err


# ---------------------------------------------------------------- background velocity (inflow)

@pytest.mark.parametrize("scheme", [oracle.BE, oracle.TRAPEZOID])
def test_uniform_background_velocity_translates_the_fom(scheme):
    # The kernel sees only differences of positions, so a velocity U common
    # to every body carries the unforced solution along: x_U(t) = x(t) + U t.
    cl = W.gaussian_patch(40, seed=7, delta=0.05)
    g = cl.gamma * 40
    U = np.concatenate([np.full(40, 0.7), np.full(40, -0.3)])
    dt, k = 2e-3, 15
    x0, st0 = oracle.implicit(cl.xy, g, cl.delta, dt, k, scheme=scheme)
    assert st0.nonconverged_steps == 0
    xu, st = oracle.implicit(cl.xy, g, cl.delta, dt, k, scheme=scheme, u=U)
    assert st.nonconverged_steps == 0
    np.testing.assert_allclose(xu, x0 + U * dt * k, rtol=0, atol=1e-12)


def test_background_velocity_alone_moves_bodies_linearly():
    # Gamma = 0: dx/dt = u exactly, which both schemes integrate without error.
    n = 30
    xy = W.uniform_disk(n, seed=2)[1]
    u = W.mushroom_inflow(n)
    for scheme in (oracle.BE, oracle.TRAPEZOID):
        x, _ = oracle.implicit(xy, np.zeros(n), 0.1, 5e-3, 40, scheme=scheme, u=u)
        np.testing.assert_allclose(x, xy + u * 0.2, rtol=0, atol=1e-13)


def test_mushroom_inflow_profile():
    u = W.mushroom_inflow(5)
    np.testing.assert_array_equal(u[:5], 0.0)
    # s = -1, -0.5, 0, 0.5, 1: 5 sqrt(1.125^2 - s^2) + 0.5
    want = [5 * np.sqrt(1.265625 - s * s) + 0.5 for s in (-1.0, -0.5, 0.0, 0.5, 1.0)]
    np.testing.assert_allclose(u[5:], want, rtol=1e-15)
    np.testing.assert_allclose(u[7], 6.125, rtol=1e-15)


def test_full_rank_lspg_reproduces_forced_fom():
    # The full-rank reproduction pin with a non-uniform background velocity:
    # a dropped or mis-signed inflow term in HyperPair's residual rows breaks
    # the zero-residual reproduction of the forced trapezoid FOM.
    n = 48
    cl = W.gaussian_patch(n, seed=3, delta=0.05)
    g = cl.gamma * n
    u = 0.2 * W.mushroom_inflow(n)
    dt, T = 2e-3, 6
    S = off.trapezoid_snapshots(cl.xy, g, cl.delta, dt, T, u=u)
    Phi, sig = off.pod(S, T, x0=cl.xy)
    tree = off.QuadTree(off.weighted_points(Phi, sig), 6)
    art = off.rom_artifacts(np.arange(n), tree, np.inf, cl.xy, Phi, g, cl.delta, dt, u=u)
    out = oracle.Rom(art, jac_mode=1).run(T, tol=1e-13, max_iter=30)
    assert out["status"] == 0
    rec = cl.xy[:, None] + Phi @ out["hist"].T
    np.testing.assert_allclose(rec, S, rtol=0, atol=1e-9)
    # the same basis without the inflow in HyperPair misses the forced states
    art0 = dict(art)
    del art0["ubar"]
    out0 = oracle.Rom(art0, jac_mode=1).run(T, tol=1e-13, max_iter=30)
    rec0 = cl.xy[:, None] + Phi @ out0["hist"].T
    assert np.abs(rec0 - S).max() > 1e-4


def test_hyperpair_velocity_includes_the_background(small_problem):
    cl, S, Phi, sig, tree = small_problem
    g = cl.gamma
    n = g.size
    u = W.mushroom_inflow(n)
    sample = np.array([1, 5, 9])
    a0 = off.rom_artifacts(sample, tree, 1.0, cl.xy, Phi, g, cl.delta, 1e-3)
    a1 = off.rom_artifacts(sample, tree, 1.0, cl.xy, Phi, g, cl.delta, 1e-3, u=u)
    xh = np.linspace(-0.1, 0.2, Phi.shape[1])
    z = np.zeros(6)
    xb0, fb0, rb0, C0 = oracle.Rom(a0).hyperpair(xh, z, z)
    xb1, fb1, rb1, C1 = oracle.Rom(a1).hyperpair(xh, z, z)
    rows = np.concatenate([sample, n + sample])
    np.testing.assert_array_equal(xb1, xb0)
    np.testing.assert_allclose(fb1, fb0 + u[rows], rtol=0, atol=1e-15)
    np.testing.assert_allclose(rb1, rb0 - 0.5e-3 * u[rows], rtol=0, atol=1e-15)
    np.testing.assert_array_equal(C1, C0)


def test_one_gauss_newton_iteration_solves_a_linear_residual(small_problem):
    # With every surrogate strength zero and a background velocity u, the
    # sampled residual Phibar (xhat - xhat_prev) - dt ubar is linear in xhat:
    # the first Gauss-Newton step of every time step lands on the
    # least-squares minimiser of |A (Phibar d - dt ubar)| and the next one
    # finds a zero gradient.
    cl, _, Phi, sig, tree = small_problem
    n = cl.n
    sample = np.array([3, 40, 77, 120, 150, 190])
    u = np.random.default_rng(4).standard_normal(2 * n)
    A = np.random.default_rng(5).standard_normal((9, 12))
    art = off.rom_artifacts(sample, tree, 1.0, cl.xy, Phi, cl.gamma, cl.delta, 1e-3, A=A, u=u)
    art["Gt"] = np.zeros_like(art["Gt"])
    out = oracle.Rom(art).run(3, tol=1e-10, max_iter=10)
    rows = off.sampled_rows(sample, n)
    step = np.linalg.lstsq(A @ Phi[rows], A @ (1e-3 * u[rows]), rcond=None)[0]
    for t in range(3):
        np.testing.assert_allclose(out["hist"][t], (t + 1) * step, rtol=1e-10, atol=1e-15)
    assert out["status"] == 0 and np.all(out["iters"] <= 2)


def test_gnat_with_full_sample_and_full_residual_basis_is_lspg():
    # n_s = N sampled bodies and a residual basis spanning every residual the
    # LSPG iterations produce: A = Phi_r^T weighs those residuals exactly as
    # the unweighted norm does, so GNAT follows LSPG iterate by iterate.
    cl = W.gaussian_patch(40, seed=9, delta=0.05)
    g = cl.gamma * 40
    dt, T = 2e-3, 5
    S = off.trapezoid_snapshots(cl.xy, g, cl.delta, dt, T)
    Phi, sig = off.pod(S, 3, x0=cl.xy)
    tree = off.QuadTree(off.weighted_points(Phi, sig), 6)
    lspg = oracle.Rom(off.rom_artifacts(np.arange(40), tree, 1.0, cl.xy, Phi, g, cl.delta, dt)).run(
        T, tol=1e-12, max_iter=8, resid_cap=T * 8)
    R = lspg["resid"].T
    U, s, _ = np.linalg.svd(R, full_matrices=False)
    Phi_r = U[:, s > 1e-12 * s[0]]
    assert Phi_r.shape[1] < 80
    A = np.linalg.pinv(Phi_r[off.sampled_rows(np.arange(40), 40)])
    gnat = oracle.Rom(off.rom_artifacts(np.arange(40), tree, 1.0, cl.xy, Phi, g, cl.delta, dt, A=A)).run(
        T, tol=1e-12, max_iter=8)
    np.testing.assert_array_equal(gnat["iters"], lspg["iters"])
    np.testing.assert_allclose(gnat["hist"], lspg["hist"], rtol=1e-9, atol=1e-12)
    # a residual basis missing one of those directions weighs them
    # differently and moves the minimiser
    A2 = np.linalg.pinv(np.delete(Phi_r, 1, axis=1)[off.sampled_rows(np.arange(40), 40)])
    moved = oracle.Rom(off.rom_artifacts(np.arange(40), tree, 1.0, cl.xy, Phi, g, cl.delta, dt, A=A2)).run(
        T, tol=1e-12, max_iter=8)
    assert np.abs(moved["hist"] - lspg["hist"]).max() > 1e-4


def test_greedy_refit_on_sampled_rows_decides_the_second_pick():
    # Greedy sampling, later groups: the new residual-basis vector is replaced
    # by its gappy reconstruction error from the processed vectors, fitted on
    # the rows of the bodies sampled so far.  Worked by hand on n = 4 bodies
    # (rows chi_0..chi_3, psi_0..psi_3), two orthogonal columns, ns = 2, so
    # n_c = 2 and n_it = 2: one column and one body per group.
    #   a = ( 2, 0, -1,  0 |  0,  0, 1, 0) / sqrt(6)
    #   b = (-1, 0,  0, -2 | -2, -2, 2, 1) / sqrt(18)       a . b = 0
    # group 1 scores (a):  body 0: 4, body 1: 0, body 2: 2, body 3: 0  (x 1/6)  -> body 0
    # group 2, fit of b on a over body 0's rows (chi_0, psi_0): coefficient
    #   (2 (-1) + 0 (-2)) / (2^2 + 0^2) = -1/2 (in the unscaled entries), so
    #   R = b + a/2 = (0, 0, -1/2, -2 | -2, -2, 5/2, 1)
    #   scores: body 1: 4, body 2: 1/4 + 25/4 = 13/2, body 3: 5  -> body 2
    # Without the refit R = b: body 1: 4, body 2: 4, body 3: 5 -> body 3; a
    # fit over all rows has coefficient a . b = 0 and gives the same body 3.
    a = np.array([2, 0, -1, 0, 0, 0, 1, 0], float) / np.sqrt(6.0)
    b = np.array([-1, 0, 0, -2, -2, -2, 2, 1], float) / np.sqrt(18.0)
    Phi_r = np.column_stack([a, b])
    assert list(off.greedy_sample(Phi_r, 2)) == [0, 2]
    n = 4

    def second_pick(R):
        s = R[:n] ** 2 + R[n:] ** 2
        s[0] = -np.inf
        return int(np.argmax(s))

    # the two other readings pick body 3, so the pin tells them apart
    assert second_pick(b) == 3
    assert second_pick(b - a * (a @ b) / (a @ a)) == 3
    rows = [0, n]
    assert second_pick(b - a * (a[rows] @ b[rows]) / (a[rows] @ a[rows])) == 2
