"""Offline PTROM training (training hierarchy, Stages 1-4) on the GPU.

Stage 1  trapezoid FOM snapshots with the HIP implicit stepper;
Stage 2  POD by the method of snapshots: FP64 Gram matrix and basis
         combination in HIP kernels, the small symmetric eigenproblem on the
         host, CholeskyQR re-orthogonalisation on the GPU; weighted POD points
         W_phi = Phi Sigma_hat; native quadtree + neighbour-search clustering
         (Algorithms "ClusterPOD" and "checkPrune");
Stage 3  Tier-II LSPG over every body with clustered sources (HyperPair
         kernel on the GPU, Gauss-Newton least squares on the host), residual
         snapshots of every iteration and their POD basis Phi_r;
Stage 4  greedy sample selection (Algorithm "greedy sampling") and the gappy
         operator A = [P Phi_r]^+.
The result is the artifact dict consumed by ``native.Rom``.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import native


def trapezoid_snapshots(xy0, gamma, delta, dt, nsnap, newton_tol=1e-6, uinf=None):
    """Device FP64 [nsnap, 2N]: states x^1..x^nsnap of the trapezoid FOM;
    ``uinf`` (device FP32 [2N]) an optional background velocity."""
    x = xy0.clone()
    S = torch.empty((nsnap, xy0.numel()), dtype=torch.float64, device=xy0.device)
    for t in range(nsnap):
        st = native.implicit(x, gamma, delta, dt, 1, scheme=native.TRAPEZOID, newton_tol=newton_tol,
                             gmres_tol=1e-4, uinf=uinf)
        if st.nonconverged_steps:
            raise RuntimeError("trapezoid snapshot %d did not converge" % t)
        S[t].copy_(x)
    return S


def pod(S, M, center=None):
    """POD of the rows of S (device FP64 [k, nd]): with fewer snapshots than
    rows (k <= nd) by the method of snapshots (eigenvectors of the k x k Gram
    S S^T, modes = S^T v / sigma, re-orthonormalised by CholeskyQR2); with
    more, from the eigenvectors of the nd x nd Gram S^T S, which are the modes
    themselves.  Returns (Phi as device FP64 [M, nd] rows = modes, sigma [M]
    host); each mode's sign makes its largest-magnitude entry positive."""
    X = S if center is None else (S - center[None, :]).contiguous()
    k, nd = X.shape
    if k > nd:
        G = native.gram_f64(X.t().contiguous()).cpu().numpy()
        w, V = np.linalg.eigh(G)
        order = np.argsort(w)[::-1][:M]
        sig = np.sqrt(np.maximum(w[order], 0.0))
        if np.any(sig <= 0):
            raise RuntimeError("snapshot matrix has rank < M")
        Phi = torch.tensor(np.ascontiguousarray(V[:, order].T), dtype=torch.float64, device=S.device)
    else:
        G = native.gram_f64(X).cpu().numpy()
        w, V = np.linalg.eigh(G)
        order = np.argsort(w)[::-1][:M]
        sig = np.sqrt(np.maximum(w[order], 0.0))
        if np.any(sig <= 0):
            raise RuntimeError("snapshot matrix has rank < M")
        T = torch.tensor(np.ascontiguousarray(V[:, order] / sig[None, :]), dtype=torch.float64, device=S.device)
        Phi = native.combine_f64(X, T)
        for _ in range(2):  # CholeskyQR2
            G2 = native.gram_f64(Phi).cpu().numpy()
            R = np.linalg.cholesky(G2).T
            Rinv = torch.tensor(np.ascontiguousarray(np.linalg.inv(R)), dtype=torch.float64, device=S.device)
            Phi = native.combine_f64(Phi, Rinv)
    # sign convention: each mode's entry of largest magnitude is positive
    # (lowest row on ties), which fixes W_phi and so the clustering
    P = Phi.cpu().numpy()
    flip = P[np.arange(M), np.argmax(np.abs(P), axis=1)] < 0.0
    if flip.any():
        D = np.diag(np.where(flip, -1.0, 1.0))
        Phi = native.combine_f64(Phi, torch.tensor(D, dtype=torch.float64, device=S.device))
    return Phi, sig


def weighted_points(Phi_h, sigma):
    """[N, 2] points of the bodies in W_phi = Phi Sigma_hat (Phi_h: host [nd, M])."""
    v = Phi_h @ sigma
    n = v.size // 2
    return np.ascontiguousarray(np.stack([v[:n], v[n:]], axis=1))


def sample_rows(sample, n):
    s = np.asarray(sample, dtype=np.int64)
    return np.concatenate([s, n + s])


def artifacts(sample, wpts, xy0, Phi_h, gamma, depth, pc, delta, dt, A, criterion=native.NEIGHBOR, theta=0.0,
              u=None):
    """Online artifacts; a background velocity ``u`` [2N] contributes its
    sampled rows as ``ubar``."""
    n = gamma.size
    cl = native.cluster_build(wpts, xy0, Phi_h, gamma, depth, pc, sample, criterion, theta)
    rows = sample_rows(sample, n)
    art = dict(M=Phi_h.shape[1], Mr=A.shape[0], sample=np.asarray(sample), Phibar=Phi_h[rows].copy(),
               xbar0=np.asarray(xy0)[rows].copy(), xqt0=cl["xqt0"], Phit=cl["Phit"], Gt=cl["Gt"],
               off=cl["off"], ids=cl["ids"], keys=cl["keys"], A=A, delta=float(delta), dt=float(dt),
               mem_off=cl["mem_off"], mem_ids=cl["mem_ids"], n=int(n))
    if u is not None:
        art["ubar"] = np.asarray(u, dtype=np.float64)[rows].copy()
    return art


def reassign_host(art, gamma_mu):
    """Clustered circulations of the artifacts' surrogates at parameter
    gamma_mu (host, FP64): the sum of each surrogate's members."""
    g = np.asarray(gamma_mu, dtype=np.float64)
    off, ids = np.asarray(art["mem_off"]), np.asarray(art["mem_ids"])
    return np.array([g[ids[off[c]:off[c + 1]]].sum() for c in range(off.size - 1)])


def tier2(art, nsteps, tol, max_iter, alpha=1.0, jac_mode=native.JAC_PAPER, device=None, record=True, log=None):
    """Tier-II LSPG (no hyper-reduction) on the GPU gather: every body is a
    target, the weighting is the identity.  Same iteration as the online loop:
    HyperPair -> C, rbar -> d = argmin |C d - (-rbar)| -> xhat += alpha d, with the
    relative reduced gradient |C^T rbar| / (first value) against tol.
    Returns (residual snapshots device [count, nd], xhat history, iterations)."""
    rom = native.Rom(art, tol=tol, max_iter=max_iter, alpha=alpha, jac_mode=jac_mode, device=device)
    M, nd = art["M"], 2 * (len(art["off"]) - 1)
    dev = device
    Phibar = np.asarray(art["Phibar"])
    xbar0 = np.asarray(art["xbar0"])
    xh = np.zeros(M)
    tdev = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    zeros = tdev(np.zeros(nd))
    xb, fb, _, _ = rom.hyperpair(tdev(xh), zeros, zeros)
    xbar_prev, fbar_prev = xb.clone(), fb.clone()
    cap = nsteps * max_iter if record else 0
    R = torch.empty((max(min(cap, 4 * nsteps), 1), nd), dtype=torch.float64, device=dev) if record else None
    count = 0
    hist = np.empty((nsteps, M))
    iters = np.empty(nsteps, dtype=np.int32)
    for step in range(nsteps):
        k, g1 = 1, 0.0
        while True:
            xb, fb, rb, C = rom.hyperpair(tdev(xh), xbar_prev, fbar_prev)
            if record:
                if count == R.shape[0]:
                    R = torch.cat([R, torch.empty_like(R)])
                R[count].copy_(rb)
                count += 1
            Ch, rh = C.cpu().numpy(), rb.cpu().numpy()
            g = Ch.T @ rh
            gn = float(np.linalg.norm(g))
            if k == 1:
                g1 = gn
            eps = gn / g1 if g1 > 0 else 0.0
            d = np.linalg.lstsq(Ch, rh, rcond=None)[0]
            xh = xh - alpha * d
            k += 1
            if not (eps > tol) or k > max_iter:
                break
        hist[step] = xh
        iters[step] = k - 1
        if log and (step + 1) % 250 == 0:
            log("tier II: step %d of %d" % (step + 1, nsteps))
        xbar_prev = tdev(xbar0 + Phibar @ xh)
        fbar_prev = fb.clone()
    rom.close()
    return (R[:count] if record else None), hist, iters


def greedy_sample(Phi_r, ns):
    """Greedy body selection from the residual basis Phi_r (host [2N, Mr]):
    the basis is processed in groups; the first group scores bodies by the
    squared entries of its vectors, later groups by their gappy-POD
    reconstruction error from the vectors already processed, restricted to
    the current sample; each pick is the unsampled body with the largest
    summed squared error over its two rows (lowest index on ties)."""
    nd, Mr = Phi_r.shape
    n = nd // 2
    chosen = []
    n_c = min(Mr, 2 * ns)
    n_it = min(n_c, ns)
    if n_it <= 0:
        return np.zeros(0, dtype=np.int64)
    per_c, extra_c = divmod(n_c, n_it)
    per_a, extra_a = divmod(ns, n_it)
    done = 0
    taken = np.zeros(n, dtype=bool)
    for it in range(n_it):
        nc_i = per_c + (1 if it < extra_c else 0)
        na_i = per_a + (1 if it < extra_a else 0)
        block = Phi_r[:, done:done + nc_i]
        if done > 0:
            rows = sample_rows(chosen, n)
            coef, *_ = np.linalg.lstsq(Phi_r[rows, :done], block[rows], rcond=None)
            block = block - Phi_r[:, :done] @ coef
        err = (block[:n] ** 2).sum(axis=1) + (block[n:] ** 2).sum(axis=1)
        for _ in range(na_i):
            e = np.where(taken, -np.inf, err)
            j = int(np.argmax(e))
            taken[j] = True
            chosen.append(j)
        done += nc_i
    return np.array(sorted(chosen), dtype=np.int64)


def train(cloud, dt, nsnap, M, Mr, ns, depth=6, pc=1.0, tol=1e-4, max_iter=100, jac_mode=native.JAC_PAPER,
          center=False, device=None, criterion=native.NEIGHBOR, theta=0.0):
    """Stages 1-4 on one GPU.  Returns (artifacts, info)."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    t = {}
    n = cloud.n
    xy0_h = np.asarray(cloud.xy, np.float32).astype(np.float64)
    g_h = np.asarray(cloud.gamma, np.float32).astype(np.float64)
    x0 = torch.tensor(xy0_h, dtype=torch.float32, device=dev)
    g = torch.tensor(g_h, dtype=torch.float32, device=dev)
    d = float(cloud.delta)

    t0 = time.perf_counter()
    S = trapezoid_snapshots(x0, g, d, dt, nsnap)
    torch.cuda.synchronize()
    t["stage1_s"] = time.perf_counter() - t0

    t0 = time.perf_counter()
    Phi_d, sigma = pod(S, M, center=(x0.double() if center else None))
    Phi_h = np.ascontiguousarray(Phi_d.cpu().numpy().T)  # [nd, M]
    wpts = weighted_points(Phi_h, sigma)
    t["stage2_pod_s"] = time.perf_counter() - t0

    t0 = time.perf_counter()
    dummy_A = np.zeros((M, 2 * n))
    art2 = artifacts(np.arange(n), wpts, xy0_h, Phi_h, g_h, depth, pc, d, dt, dummy_A, criterion, theta)
    t["stage2_cluster_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    R, hist2, it2 = tier2(art2, nsnap, tol, max_iter, jac_mode=jac_mode, device=dev)
    t["stage3_tier2_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    Phir_d, sig_r = pod(R, Mr)
    Phi_r = np.ascontiguousarray(Phir_d.cpu().numpy().T)
    t["stage3_pod_s"] = time.perf_counter() - t0

    t0 = time.perf_counter()
    sample = greedy_sample(Phi_r, ns)
    A = np.linalg.pinv(Phi_r[sample_rows(sample, n)])
    art = artifacts(sample, wpts, xy0_h, Phi_h, g_h, depth, pc, d, dt, A, criterion, theta)
    t["stage4_s"] = time.perf_counter() - t0

    # reproduction quality of the Tier-II model (reported, not a gate)
    S_h = S.cpu().numpy()
    rec2 = xy0_h[None, :] + hist2 @ Phi_h.T
    report = dict(t, tier2_mean_iters=float(it2.mean()), nc=int(art["Gt"].size), nnz=int(art["ids"].size),
                  tier2_nc=int(art2["Gt"].size), tier2_nnz=int(art2["ids"].size),
                  residual_snapshots=int(R.shape[0]),
                  tier2_final_rel_state_err=float(np.linalg.norm(rec2[-1] - S_h[-1]) /
                                                  np.linalg.norm(S_h[-1] - xy0_h)))
    info = dict(Phi=Phi_h, sigma=sigma, sigma_r=sig_r, Phi_r=Phi_r, S=S_h, wpts=wpts, report=report,
                tier2_hist=hist2, tier2_iters=it2)
    return art, info


def mae_distance(xA, xB, n, length):
    """Mean distance between matching bodies of two SoA states, over a length scale."""
    dx = xA[:n] - xB[:n]
    dy = xA[n:] - xB[n:]
    return float(np.mean(np.sqrt(dx * dx + dy * dy)) / length)


def train_parametric(clouds, dt, nsnap, M, Mr, ns, depth=6, pc=1.0, tol=1e-4, max_iter=100,
                     jac_mode=native.JAC_PAPER, device=None, criterion=native.NEIGHBOR, theta=0.0, newton_tol=1e-6,
                     u=None, log=None):
    """Stages 1-4 over several training parameters on one GPU.  ``clouds``
    share x^0 and delta and differ in Gamma.  One POD of the snapshots of all
    training points; clustering weights = mean |Gamma| over the training
    points; Tier II at every training point with its reassigned Gamma~; the
    residual snapshots of all training points form Phi_r.  ``u`` [2N] is a
    background velocity common to all parameters (inflow), or None.  ``log``
    (a callable taking a string) receives a line after each stage.  Returns
    (artifacts with membership, info)."""
    log = log or (lambda msg: None)
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    t = {}
    n = clouds[0].n
    xy0_h = np.asarray(clouds[0].xy, np.float32).astype(np.float64)
    x0 = torch.tensor(xy0_h, dtype=torch.float32, device=dev)
    d = float(clouds[0].delta)

    t0 = time.perf_counter()
    u_h = None if u is None else np.asarray(u, np.float32).astype(np.float64)
    u_d = None if u is None else torch.tensor(u_h, dtype=torch.float32, device=dev)
    snaps = []
    for k, c in enumerate(clouds):
        snaps.append(trapezoid_snapshots(x0, torch.tensor(np.asarray(c.gamma, np.float32), device=dev), d, dt, nsnap,
                                         newton_tol=newton_tol, uinf=u_d))
        log("stage 1: snapshots of training point %d done" % k)
    S = torch.cat(snaps)
    torch.cuda.synchronize()
    t["stage1_s"] = time.perf_counter() - t0

    t0 = time.perf_counter()
    Phi_d, sigma = pod(S, M)
    Phi_h = np.ascontiguousarray(Phi_d.cpu().numpy().T)
    wpts = weighted_points(Phi_h, sigma)
    wgt = np.mean([np.abs(np.asarray(c.gamma, np.float32).astype(np.float64)) for c in clouds], axis=0)
    t["stage2_s"] = time.perf_counter() - t0

    t0 = time.perf_counter()
    full = artifacts(np.arange(n), wpts, xy0_h, Phi_h, wgt, depth, pc, d, dt, np.zeros((M, 2 * n)), criterion, theta,
                     u=u_h)
    R, hists, its = [], [], []
    for c in clouds:
        a = dict(full)
        a["Gt"] = reassign_host(full, np.asarray(c.gamma, np.float32).astype(np.float64))
        r, h, i = tier2(a, nsnap, tol, max_iter, jac_mode=jac_mode, device=dev, log=log)
        R.append(r)
        hists.append(h)
        its.append(i)
        log("stage 3: tier II of training point %d done" % len(R))
    t["stage3_tier2_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    log("stage 3: POD of %d residual snapshots" % sum(int(r.shape[0]) for r in R))
    Phir_d, sig_r = pod(torch.cat(R), Mr)
    Phi_r = np.ascontiguousarray(Phir_d.cpu().numpy().T)
    sample = greedy_sample(Phi_r, ns)
    A = np.linalg.pinv(Phi_r[sample_rows(sample, n)])
    art = artifacts(sample, wpts, xy0_h, Phi_h, wgt, depth, pc, d, dt, A, criterion, theta, u=u_h)
    t["stage34_s"] = time.perf_counter() - t0
    info = dict(Phi=Phi_h, sigma=sigma, sigma_r=sig_r, Phi_r=Phi_r, S=S.cpu().numpy(), wpts=wpts, weights=wgt,
                tier2_hist=hists, tier2_iters=its, report=dict(t, nc=int(art["Gt"].size), nnz=int(art["ids"].size),
                                                                  tier2_nc=int(full["Gt"].size)))
    return art, info
