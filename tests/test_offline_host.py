"""Host-side offline pieces of the product (native quadtree clustering,
greedy sampler) against the oracle's independent implementations: interaction
lists must agree exactly (index work), surrogate values to FP64 roundoff."""
import numpy as np
import pytest

from oracle import offline as oo
from paper_2103_01983_amd import native
from paper_2103_01983_amd import offline as po
from paper_2103_01983_amd import workloads as W


def setup(n, seed, M=6):
    cl = W.counter_rotating_patches(n, seed=seed, delta=0.02)
    rng = np.random.default_rng(seed)
    # any orthonormal basis with a position-like leading mode is a valid input
    Phi = np.linalg.qr(np.column_stack([cl.xy, rng.standard_normal((2 * n, M - 1))]))[0]
    sigma = np.sort(rng.uniform(0.5, 3.0, M))[::-1] * np.linspace(10, 1, M)
    return cl, Phi, sigma


@pytest.mark.parametrize("n,pc,depth", [(200, 1.0, 6), (513, 0.5, 4), (300, np.inf, 6), (64, 0.0, 6)])
def test_cluster_lists_match_oracle(n, pc, depth):
    cl, Phi, sigma = setup(n, 3 + n)
    P = oo.weighted_points(Phi, sigma)
    tree = oo.QuadTree(P, depth)
    targets = np.arange(0, n, 3)
    ox, oP, oG, ooff, oids, okeys = oo.cluster_artifacts(tree, targets, pc, cl.xy, Phi, cl.gamma)
    r = native.cluster_build(np.ascontiguousarray(P), cl.xy, Phi, cl.gamma, depth, pc, targets)
    assert np.array_equal(r["off"], ooff)
    assert np.array_equal(r["ids"], oids)
    # keys: bodies (j) then cells (2^60 | level<<40 | row<<20 | col)
    enc = [k[1] if k[0] == 0 else (1 << 60) | (k[1] << 40) | (k[2] << 20) | k[3] for k in okeys]
    assert np.array_equal(r["keys"], np.array(enc, dtype=np.int64))
    np.testing.assert_allclose(r["xqt0"], ox, rtol=0, atol=1e-13)
    np.testing.assert_allclose(r["Phit"], oP, rtol=0, atol=1e-13)
    # sums of up to n terms of size 1/n in different orders
    np.testing.assert_allclose(r["Gt"], oG, rtol=0, atol=1e-14)


def test_greedy_matches_oracle():
    rng = np.random.default_rng(5)
    for n, Mr, ns in [(100, 16, 16), (257, 8, 20), (64, 12, 5), (40, 6, 40)]:
        Phi_r = np.linalg.qr(rng.standard_normal((2 * n, Mr)))[0]
        assert np.array_equal(po.greedy_sample(Phi_r, ns), oo.greedy_sample(Phi_r, ns)), (n, Mr, ns)


def test_cluster_rejects_bad_input():
    cl, Phi, sigma = setup(50, 1)
    P = oo.weighted_points(Phi, sigma)
    with pytest.raises(native.PtromError):
        native.cluster_build(P, cl.xy, Phi, cl.gamma, 6, 1.0, np.array([0, 50]))


@pytest.mark.parametrize("n,theta,depth", [(200, 0.5, 6), (300, 1.0, 5), (128, 2.0, 6)])
def test_barnes_hut_lists_match_oracle(n, theta, depth):
    cl, Phi, sigma = setup(n, 50 + n)
    P = oo.weighted_points(Phi, sigma)
    tree = oo.QuadTree(P, depth)
    targets = np.arange(1, n, 4)
    ox, oP, oG, ooff, oids, okeys = oo.cluster_artifacts(tree, targets, 0.0, cl.xy, Phi, cl.gamma,
                                                          criterion="barnes-hut", theta=theta)
    r = native.cluster_build(np.ascontiguousarray(P), cl.xy, Phi, cl.gamma, depth, 0.0, targets,
                             native.BARNES_HUT, theta)
    assert np.array_equal(r["off"], ooff)
    assert np.array_equal(r["ids"], oids)
    np.testing.assert_allclose(r["Phit"], oP, rtol=0, atol=1e-13)


def test_barnes_hut_theta_zero_is_exact_and_lists_cover_all():
    cl, Phi, sigma = setup(150, 9)
    P = oo.weighted_points(Phi, sigma)
    tree = oo.QuadTree(P, 6)
    keys_nodes = {nd.key: nd for nd in tree.nodes}
    for i in [0, 70, 149]:
        assert sorted(k[1] for k in oo.find_clusters(tree, i, 0.0, "barnes-hut", 0.0, cl.gamma)) == \
            [j for j in range(150) if j != i]
        members = []
        for k in oo.find_clusters(tree, i, 0.0, "barnes-hut", 1.5, cl.gamma):
            members.extend([k[1]] if k[0] == 0 else keys_nodes[k].members)
        assert sorted(members) == [j for j in range(150) if j != i]


@pytest.mark.parametrize("criterion,theta", [("neighbor", 0.0), ("barnes-hut", 2.0)])
def test_lists_with_coincident_cells_match_oracle(criterion, theta):
    # Bodies evenly spaced on a line with equal Gamma: the weighted mean of
    # two bodies symmetric about a third sits exactly on it at x^0, and such
    # cells must be opened by both implementations.
    cl = W.single_vortex(100)
    n = cl.n
    S = oo.trapezoid_snapshots(cl.xy, cl.gamma, 0.0, 0.01, 2000)
    Phi, sig = oo.pod(S, 13)
    rng = np.random.default_rng(12)
    fired = 0
    for trial in range(8):
        sg = np.ones(13) if trial == 0 else rng.choice([-1.0, 1.0], 13)
        P = np.ascontiguousarray(oo.weighted_points(Phi * sg, sig))
        tree = oo.QuadTree(P, 16)
        targets = np.arange(n)
        ox, oP, oG, ooff, oids, okeys = oo.cluster_artifacts(tree, targets, 0.0, cl.xy, Phi, cl.gamma,
                                                             criterion, theta)
        kind = native.NEIGHBOR if criterion == "neighbor" else native.BARNES_HUT
        r = native.cluster_build(P, cl.xy, np.ascontiguousarray(Phi), cl.gamma, 16, 0.0, targets, kind, theta)
        assert np.array_equal(r["off"], ooff) and np.array_equal(r["ids"], oids)
        np.testing.assert_allclose(r["xqt0"], ox, rtol=0, atol=1e-12)
        fired += sum(oo.find_clusters(tree, i, 0.0, criterion, theta, cl.gamma)
                     != oo.find_clusters(tree, i, 0.0, criterion, theta, cl.gamma, cl.xy) for i in range(n))
    if criterion == "neighbor":
        assert fired > 0


@pytest.mark.parametrize("criterion,theta", [("neighbor", 1.0), ("barnes-hut", 1.0)])
def test_members_match_oracle(criterion, theta):
    cl, Phi, sigma = setup(300, 91)
    P = np.ascontiguousarray(oo.weighted_points(Phi, sigma))
    tree = oo.QuadTree(P, 6)
    targets = np.arange(0, 300, 5)
    *_, okeys = oo.cluster_artifacts(tree, targets, 1.0, cl.xy, Phi, cl.gamma, criterion, theta)
    kind = native.NEIGHBOR if criterion == "neighbor" else native.BARNES_HUT
    r = native.cluster_build(P, cl.xy, Phi, cl.gamma, 6, 1.0, targets, kind, theta)
    mem = oo.surrogate_members(tree, okeys)
    off = np.concatenate([[0], np.cumsum([len(m) for m in mem])])
    assert np.array_equal(r["mem_off"], off)
    assert np.array_equal(r["mem_ids"], np.concatenate([np.asarray(m) for m in mem]))
    # host reassignment of the package equals the oracle's
    g = np.random.default_rng(2).standard_normal(cl.n)
    art = dict(mem_off=r["mem_off"], mem_ids=r["mem_ids"])
    np.testing.assert_allclose(po.reassign_host(art, g), oo.reassign_circulation(mem, g), rtol=0, atol=1e-12)


def test_barnes_hut_distance_is_measured_from_the_weighted_mean():
    # checkPrune, Barnes-Hut branch: a cell is pruned when w / |s - s_i| <= theta,
    # s the cell's (|Gamma|-weighted) mean point.  Hand-built tree over five
    # points: root [0, 8]^2, level-1 cells of width 4.
    #   body 0 (target) (0, 0); bodies 1, 2 in cell [4, 8] x [0, 4):
    #   (4.2, 0.2) with Gamma 0.01 and (7.8, 0.2) with Gamma 1; bodies 3, 4
    #   alone in their cells at (0, 8) and (8, 8).
    # Cell of bodies 1, 2 at theta = 0.6:
    #   weighted mean (7.8427 / 1.01, 0.2) = (7.7644, 0.2), distance 7.7669,
    #   4 / 7.7669 = 0.515 <= 0.6 -> pruned, listed as one surrogate;
    #   the cell's geometric centre (6, 2) would give 4 / 6.325 = 0.632 and
    #   the plain member mean (6, 0.2) 4 / 6.003 = 0.666: both open the cell
    #   and list bodies 1 and 2 one by one.
    # Bodies 3 and 4: 4 / 8 and 4 / 11.3 -> pruned single bodies.
    P = np.array([[0.0, 0.0], [4.2, 0.2], [7.8, 0.2], [0.0, 8.0], [8.0, 8.0]])
    g = np.array([1.0, 0.01, 1.0, 1.0, 1.0])
    tree = oo.QuadTree(P, 6)
    want = [(0, 3, 0, 0), (0, 4, 0, 0), (1, 1, 0, 1)]
    assert sorted(oo.find_clusters(tree, 0, 0.0, "barnes-hut", 0.6, g)) == want
    # the same tree read with the other two centres opens the cell
    cell = [nd for nd in tree.nodes if nd.key == (1, 1, 0, 1)][0]
    for centre in ((cell.lo + cell.hi) / 2, P[[1, 2]].mean(axis=0)):
        assert cell.width / np.linalg.norm(centre - P[0]) > 0.6
    assert cell.width / np.linalg.norm(oo.weighted_point_mean(tree, cell, g) - P[0]) <= 0.6
    # the native clustering takes the same decision
    xy0 = np.concatenate([P[:, 0], P[:, 1]])
    phi = np.linalg.qr(np.random.default_rng(0).standard_normal((10, 2)))[0]
    r = native.cluster_build(P, xy0, phi, g, 6, 0.0, np.array([0]), native.BARNES_HUT, 0.6)
    assert list(r["keys"]) == [3, 4, (1 << 60) | (1 << 40) | (0 << 20) | 1]
    assert list(r["off"]) == [0, 3]
    # and lists bodies 1 and 2 separately once theta is below 0.515
    r = native.cluster_build(P, xy0, phi, g, 6, 0.0, np.array([0]), native.BARNES_HUT, 0.5)
    assert list(r["keys"]) == [1, 2, 3, 4]
    assert sorted(oo.find_clusters(tree, 0, 0.0, "barnes-hut", 0.5, g)) == [(0, j, 0, 0) for j in (1, 2, 3, 4)]
