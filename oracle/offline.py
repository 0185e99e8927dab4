"""Offline PTROM training in FP64 NumPy: the oracle's version (training
hierarchy, Stages 1-4).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Straightforward
loops and recursion, written for checking by eye against the paper:

* Stage 1  trapezoid FOM snapshots (``trapezoid_snapshots``);
* Stage 2  POD by the method of snapshots (``pod``), weighted POD space
           W_phi = Phi Sigma_hat (``weighted_points``), Barnes-Hut quadtree
           over it (``QuadTree``), weighted means per node and per-target
           neighbour-search clustering with UniqueSearch (Algorithms
           "ClusterPOD" and "checkPrune": ``node_surrogates``,
           ``find_clusters``, ``cluster_artifacts``);
* Stage 3  Tier-II LSPG with clustered sources over every body, residual
           snapshots and their POD basis Phi_r (``tier2_residual_basis``);
* Stage 4  greedy sample selection (Algorithm "greedy sampling",
           ``greedy_sample``) and the gappy operator A = [P Phi_r]^+;
* parametric: surrogate membership, the online reassignment of clustered
           circulations for a new parameter (``reassign_circulation``) and
           training over several parameters (``train_parametric``).

Readings of passages the paper leaves open (each also listed in the design
notes):
  - snapshots are used raw, S = [x^1 .. x^Nt] (POD construction), with the
    affine ansatz x ~ x^0 + Phi xhat; ``center=True`` uses S - x^0 instead;
  - a body's point in W_phi is ((Phi s)_i, (Phi s)_{i+N}), s = singular values;
  - root cell = tight bounding box of those points; cells split at the
    midpoint while they hold more than one body and are above the depth cap;
    membership is half-open [lo, mid), [mid, hi]; width = longer side;
  - weighted means use |Gamma| as weights (so mixed-sign cells stay
    defined); the surrogate strength is the plain sum of Gamma;
  - neighbour test as in the checkPrune listing (source cell bounds, strict
    inequalities); a cell that holds the target is never pruned; nor is a
    cell whose surrogate sits on the target at x^0 (rounding allowance
    1e-9 (1 + |x_i|)); an unpruned leaf is expanded into its bodies, the
    target itself excluded;
  - a POD mode's sign makes its largest-magnitude entry positive;
  - parametric training: one POD of all training snapshots; clustering
    weights = mean |Gamma| over the training points; only Gamma~ is
    reassigned per parameter (surrogate positions and rows stay fixed);
  - the greedy loop processes the residual basis in n_it groups and, after
    the first group, uses the gappy-POD reconstruction error of each group
    from the already-processed vectors on the current sample; ties go to the
    lowest body index.
"""
from __future__ import annotations

import numpy as np

import oracle


# ----------------------------------------------------------------- Stage 1

def trapezoid_snapshots(xy0, gamma, delta, dt, nsnap, u=None):
    """Columns x^1..x^nsnap of the trapezoid FOM (scheme of the online
    residual); ``u`` [2N] an optional background velocity (inflow)."""
    S = np.empty((xy0.size, nsnap))
    x = np.array(xy0, dtype=np.float64)
    for t in range(nsnap):
        x, st = oracle.implicit(x, gamma, delta, dt, 1, scheme=oracle.TRAPEZOID, u=u)
        assert st.nonconverged_steps == 0
        S[:, t] = x
    return S


# ----------------------------------------------------------------- Stage 2

def pod(S, M, x0=None):
    """Phi = first M left singular vectors of S (or of S - x0 1^T); returns
    (Phi [Nd, M], sigma [M]).  Each mode's sign makes its entry of largest
    magnitude positive (the lowest row on ties), so W_phi is reproducible."""
    A = S if x0 is None else S - np.asarray(x0)[:, None]
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    Phi = U[:, :M].copy()
    for m in range(M):
        if Phi[np.argmax(np.abs(Phi[:, m])), m] < 0.0:
            Phi[:, m] = -Phi[:, m]
    return Phi, s[:M].copy()


def weighted_points(Phi, sigma):
    """Each body's 2D point in the weighted POD space: (Phi sigma)_i, (Phi sigma)_{i+N}."""
    v = Phi @ sigma
    n = v.size // 2
    return np.stack([v[:n], v[n:]], axis=1)


class Node:
    __slots__ = ("lo", "hi", "level", "ix", "iy", "members", "children")

    def __init__(self, lo, hi, level, ix, iy, members):
        self.lo, self.hi = np.array(lo, float), np.array(hi, float)
        self.level, self.ix, self.iy = level, ix, iy
        self.members = members
        self.children = []

    @property
    def width(self):
        return float(max(self.hi[0] - self.lo[0], self.hi[1] - self.lo[1]))

    @property
    def key(self):
        return (1, self.level, self.iy, self.ix)


class QuadTree:
    """Barnes-Hut quadtree over the points P [N,2]; levels 0..max_level."""

    def __init__(self, P, max_level=6):
        self.P = np.asarray(P, dtype=np.float64)
        n = self.P.shape[0]
        self.max_level = max_level
        self.leaf_of = [None] * n
        self.nodes = []
        self.root = self._build(self.P.min(axis=0), self.P.max(axis=0), 0, 0, 0, list(range(n)))

    def _build(self, lo, hi, level, ix, iy, members):
        node = Node(lo, hi, level, ix, iy, members)
        self.nodes.append(node)
        if len(members) > 1 and level < self.max_level:
            mid = 0.5 * (node.lo + node.hi)
            quads = [[], [], [], []]
            for j in members:
                qx = 1 if self.P[j, 0] >= mid[0] else 0
                qy = 1 if self.P[j, 1] >= mid[1] else 0
                quads[qx + 2 * qy].append(j)
            for q in range(4):
                if not quads[q]:
                    continue
                qx, qy = q & 1, q >> 1
                clo = [node.lo[0] if qx == 0 else mid[0], node.lo[1] if qy == 0 else mid[1]]
                chi = [mid[0] if qx == 0 else node.hi[0], mid[1] if qy == 0 else node.hi[1]]
                node.children.append(self._build(clo, chi, level + 1, 2 * ix + qx, 2 * iy + qy, quads[q]))
        else:
            for j in members:
                self.leaf_of[j] = node
        return node


def node_surrogates(node, xy0, Phi, gamma):
    """Weighted mean of the member rows (WeightedMean): returns
    (x0 [2], Phi rows [2, M], Gamma sum).  Weights |Gamma|."""
    n = gamma.size
    idx = np.asarray(node.members)
    w = np.abs(gamma[idx])
    if w.sum() == 0.0:
        w = np.ones_like(w)
    w = w / w.sum()
    x0 = np.array([np.dot(w, xy0[idx]), np.dot(w, xy0[n + idx])])
    ph = np.stack([w @ Phi[idx], w @ Phi[n + idx]])
    return x0, ph, float(gamma[idx].sum())


def weighted_point_mean(tree, node, gamma):
    """|Gamma|-weighted mean of the members' points in the tree's space (the
    surrogate-source position s of Def. 1 in W_phi); plain mean if all
    weights vanish."""
    idx = np.asarray(node.members)
    w = np.abs(gamma[idx])
    if w.sum() == 0.0:
        w = np.ones_like(w)
    return (w[:, None] * tree.P[idx]).sum(axis=0) / w.sum()


def coincides(node, i, xy0, gamma):
    """True when the cell's surrogate (|Gamma|-weighted mean of its members'
    initial positions) lies on body i's initial position, to within 1e-9 of
    (1 + |x_i|).  At delta = 0 such a pair has no defined velocity."""
    n = gamma.size
    idx = np.asarray(node.members)
    w = np.abs(gamma[idx])
    if w.sum() == 0.0:
        w = np.ones_like(w)
    w = w / w.sum()
    sx, sy = float(np.dot(w, xy0[idx])), float(np.dot(w, xy0[n + idx]))
    xi, yi = float(xy0[i]), float(xy0[n + i])
    return np.hypot(sx - xi, sy - yi) <= 1e-9 * (1.0 + np.hypot(xi, yi))


def find_clusters(tree, i, pc, criterion="neighbor", theta=0.0, gamma=None, xy0=None):
    """Cluster keys seen by target body i (FindClusters / Traverse with
    checkPrune).  criterion "neighbor": prune a cell that does not overlap the
    target leaf grown by pc times its width; "barnes-hut": prune when
    w / |s - s_i| <= theta, s the cell's weighted mean point and s_i the
    target's point.  With ``xy0`` (initial positions) a cell whose surrogate
    coincides with the target there is opened instead of pruned.  Keys:
    (0, j, 0, 0) for a single body j, node.key for an agglomerated cell."""
    leaf = tree.leaf_of[i]
    w = leaf.width
    h_lo = leaf.lo - pc * w
    h_hi = leaf.hi + pc * w
    si = tree.P[i]
    out = []

    def visit(node):
        if criterion == "neighbor":
            ov = (h_hi[0] > node.lo[0] and h_lo[0] < node.hi[0] and
                  h_hi[1] > node.lo[1] and h_lo[1] < node.hi[1])
        else:
            dist = float(np.linalg.norm(weighted_point_mean(tree, node, gamma) - si))
            ov = not (dist > 0.0 and node.width / dist <= theta)
        if node.level <= leaf.level and (leaf.ix >> (leaf.level - node.level)) == node.ix \
                and (leaf.iy >> (leaf.level - node.level)) == node.iy:
            ov = True  # the cell holds the target
        if not ov and xy0 is not None and len(node.members) > 1 and coincides(node, i, xy0, gamma):
            ov = True
        if not ov:
            if len(node.members) == 1:
                out.append((0, node.members[0], 0, 0))
            else:
                out.append(node.key)
            return
        if not node.children:
            out.extend((0, j, 0, 0) for j in node.members if j != i)
            return
        for c in node.children:
            visit(c)

    visit(tree.root)
    return out


def cluster_artifacts(tree, targets, pc, xy0, Phi, gamma, criterion="neighbor", theta=0.0):
    """UniqueSearch over the cluster lists of ``targets``.  Returns
    (xqt0 [Nc,2], Phit [Nc,2,M], Gt [Nc], off [nt+1], ids [nnz], keys)."""
    n = gamma.size
    M = Phi.shape[1]
    lists = [find_clusters(tree, int(i), pc, criterion, theta, gamma, np.asarray(xy0, float)) for i in targets]
    keys = sorted(set(k for L in lists for k in L))
    index = {k: c for c, k in enumerate(keys)}
    by_key = {nd.key: nd for nd in tree.nodes}
    Nc = len(keys)
    xqt0 = np.empty((Nc, 2)); Phit = np.empty((Nc, 2, M)); Gt = np.empty(Nc)
    for c, k in enumerate(keys):
        if k[0] == 0:
            j = k[1]
            xqt0[c] = (xy0[j], xy0[n + j]); Phit[c, 0] = Phi[j]; Phit[c, 1] = Phi[n + j]; Gt[c] = gamma[j]
        else:
            xqt0[c], Phit[c], Gt[c] = node_surrogates(by_key[k], xy0, Phi, gamma)
    off = np.zeros(len(targets) + 1, dtype=np.int64)
    ids = []
    for t, L in enumerate(lists):
        cl = sorted(index[k] for k in L)
        ids.extend(cl)
        off[t + 1] = off[t] + len(cl)
    return xqt0, Phit, Gt, off, np.asarray(ids, dtype=np.int64), keys


def sampled_rows(sample, n):
    """Row indices of the sampled bodies in the order [chi of samples, psi of samples]."""
    s = np.asarray(sample, dtype=np.int64)
    return np.concatenate([s, n + s])


def rom_artifacts(sample, tree, pc, xy0, Phi, gamma, delta, dt, A=None, u=None):
    """Online artifacts; with a background velocity ``u`` [2N] its sampled
    rows become ``ubar``."""
    n = gamma.size
    rows = sampled_rows(sample, n)
    xqt0, Phit, Gt, off, ids, keys = cluster_artifacts(tree, sample, pc, xy0, Phi, gamma)
    art = dict(M=Phi.shape[1], Mr=(A.shape[0] if A is not None else rows.size), sample=np.asarray(sample),
               Phibar=Phi[rows].copy(), xbar0=np.asarray(xy0)[rows].copy(), xqt0=xqt0, Phit=Phit, Gt=Gt,
               off=off, ids=ids, A=A, delta=float(delta), dt=float(dt), keys=keys)
    if u is not None:
        art["ubar"] = np.asarray(u, dtype=np.float64)[rows].copy()
    return art


# ----------------------------------------------------------------- Stage 3

def tier2_residual_basis(tree, pc, xy0, Phi, gamma, delta, dt, nsteps, Mr, tol=1e-4, max_iter=100,
                         jac_mode=0, cap=None):
    """Tier-II LSPG with clustered sources over all N bodies (no
    hyper-reduction); residual snapshots of every Gauss-Newton iteration;
    Phi_r = their first Mr left singular vectors."""
    n = gamma.size
    art = rom_artifacts(np.arange(n), tree, pc, xy0, Phi, gamma, delta, dt, A=None)
    rom = oracle.Rom(art, jac_mode=jac_mode)
    cap = cap or nsteps * max_iter
    out = rom.run(nsteps, tol=tol, max_iter=max_iter, resid_cap=cap)
    R = out["resid"].T
    U, s, _ = np.linalg.svd(R, full_matrices=False)
    return U[:, :Mr].copy(), s[:Mr].copy(), out


# ----------------------------------------------------------------- Stage 4

def greedy_sample(Phi_r, ns, preseed=()):
    """Greedy selection of ns bodies from the residual basis Phi_r [2N, Mr]."""
    nd_full, Mr = Phi_r.shape
    n = nd_full // 2
    S = list(preseed)
    n_a = ns - len(S)
    n_c = min(Mr, 2 * ns)
    n_it = min(n_c, n_a)
    if n_it <= 0:
        return np.array(sorted(S), dtype=np.int64)
    nci_min, nai_min = n_c // n_it, n_a // n_it
    n_b = 0
    for i in range(1, n_it + 1):
        nci = nci_min + (1 if i <= n_c % n_it else 0)
        nai = nai_min + (1 if i <= n_a % n_it else 0)
        cols = Phi_r[:, n_b:n_b + nci]
        if n_b == 0:
            R = cols
        else:
            rows = sampled_rows(S, n)
            basis = Phi_r[:, :n_b]
            coef = np.linalg.lstsq(basis[rows], cols[rows], rcond=None)[0]
            R = cols - basis @ coef
        score = np.sum(R[:n] ** 2 + R[n:] ** 2, axis=1)
        for _ in range(nai):
            s = score.copy()
            s[S] = -np.inf
            S.append(int(np.argmax(s)))
        n_b += nci
    return np.array(sorted(S), dtype=np.int64)


def gappy_operator(Phi_r, sample):
    """A = [P Phi_r]^+ with P selecting the sampled rows; shape [Mr, nd]."""
    n = Phi_r.shape[0] // 2
    return np.linalg.pinv(Phi_r[sampled_rows(sample, n)])


# ----------------------------------------------------------------- pipeline

def train(cloud, dt, nsnap, M, Mr, ns, depth=6, pc=1.0, tol=1e-4, max_iter=100, jac_mode=0,
          center=False, S=None):
    """Stages 1-4; returns (artifacts, extras)."""
    xy0, g, d = np.asarray(cloud.xy, float), np.asarray(cloud.gamma, float), float(cloud.delta)
    if S is None:
        S = trapezoid_snapshots(xy0, g, d, dt, nsnap)
    Phi, sigma = pod(S, M, x0=(xy0 if center else None))
    tree = QuadTree(weighted_points(Phi, sigma), depth)
    Phi_r, sr, t2 = tier2_residual_basis(tree, pc, xy0, Phi, g, d, dt, nsnap, Mr, tol, max_iter, jac_mode)
    sample = greedy_sample(Phi_r, ns)
    A = gappy_operator(Phi_r, sample)
    art = rom_artifacts(sample, tree, pc, xy0, Phi, g, d, dt, A=A)
    return art, dict(S=S, Phi=Phi, sigma=sigma, tree=tree, Phi_r=Phi_r, sigma_r=sr, tier2=t2)


# ----------------------------------------------------------------- parametric

def surrogate_members(tree, keys):
    """The bodies each unique surrogate stands for: the body itself, or every
    body of the cell (the tree keeps the bodies of each cluster)."""
    by_key = {nd.key: nd for nd in tree.nodes}
    return [[k[1]] if k[0] == 0 else list(by_key[k].members) for k in keys]


def reassign_circulation(members, gamma_mu):
    """Gamma~ of every surrogate at parameter mu: the sum of its members'
    circulations (online computations: clustered circulations are reloaded
    for a new parameter without retraining)."""
    g = np.asarray(gamma_mu, dtype=np.float64)
    return np.array([float(np.sum(g[np.asarray(m, dtype=np.int64)])) for m in members])


def train_parametric(clouds, dt, nsnap, M, Mr, ns, depth=6, pc=1.0, tol=1e-4, max_iter=100, jac_mode=0, u=None):
    """Stages 1-4 over several training parameters.  ``clouds`` share x^0 and
    delta and differ in Gamma (the parameter).  Snapshots of every training
    point form one snapshot matrix (Stage 1 over the sampled parametric
    points); the clustering weights are the mean |Gamma| over the training
    points; Tier II runs at every training point with its reassigned Gamma~
    and its residual snapshots are pooled (Stage 3).  ``u`` [2N] is a
    background velocity shared by every parameter (the mushroom cloud's
    inflow), or None."""
    x0 = np.asarray(clouds[0].xy, dtype=np.float64)
    d = float(clouds[0].delta)
    n = x0.size // 2
    S = np.hstack([trapezoid_snapshots(x0, np.asarray(c.gamma, float), d, dt, nsnap, u=u) for c in clouds])
    Phi, sigma = pod(S, M)
    tree = QuadTree(weighted_points(Phi, sigma), depth)
    wgt = np.mean([np.abs(np.asarray(c.gamma, float)) for c in clouds], axis=0)
    full = rom_artifacts(np.arange(n), tree, pc, x0, Phi, wgt, d, dt, u=u)
    mem_full = surrogate_members(tree, full["keys"])
    R, t2 = [], []
    for c in clouds:
        a = dict(full)
        a["Gt"] = reassign_circulation(mem_full, c.gamma)
        out = oracle.Rom(a, jac_mode=jac_mode).run(nsnap, tol=tol, max_iter=max_iter, resid_cap=nsnap * max_iter)
        R.append(out["resid"])
        t2.append(out)
    U, sr, _ = np.linalg.svd(np.vstack(R).T, full_matrices=False)
    Phi_r = U[:, :Mr].copy()
    sample = greedy_sample(Phi_r, ns)
    A = gappy_operator(Phi_r, sample)
    art = rom_artifacts(sample, tree, pc, x0, Phi, wgt, d, dt, A=A, u=u)
    art["members"] = surrogate_members(tree, art["keys"])
    return art, dict(S=S, Phi=Phi, sigma=sigma, tree=tree, Phi_r=Phi_r, sigma_r=sr[:Mr].copy(), tier2=t2,
                     weights=wgt)
