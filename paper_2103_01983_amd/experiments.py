"""Reproductive single-vortex study of the paper's results section (table of
reproductive experiment conditions; narrow-width PTROM hyper-parameters):
N bodies on the diagonal (linspace(-N, N, N) in both coordinates), every
body with Gamma = 0.01 except the centre one, delta = 0, trapezoid FOM.

For one N it runs on one GPU:
  * the trapezoid FOM over [0, t_f] (timed: T_I),
  * the offline training (Stages 1-4) on those snapshots,
  * the online PTROM over the same steps (timed: T_III, device-resident loop),
and reports SF = T_I / T_III, the time-averaged MAE_D and AE_H (paper's
Hamiltonian, delta = 0) of the PTROM against the FOM.

    python -m paper_2103_01983_amd.experiments [--n 500] [--case 1]
    python -m paper_2103_01983_amd.experiments --study vortex_pair

The vortex-pair parametric study (results section, vortex pair parametric
experiment): mu = (Gamma_1, Gamma_N) in [0.25, 1]^2 Gamma_max, four
Latin-hypercube training points, a 6 x 6 grid of online queries run in one
launch (one workgroup per query) after reassigning the clustered
circulations of every query on the device.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import native
from . import offline
from . import workloads as W
from .workloads import single_vortex

# narrow-width Bases Cases: case -> (tol, {N: (M, p_c)}); M_r = 2M, n_s = M_r
BASES = {
    1: (1e-1, {100: (13, 0.0), 500: (21, 0.0), 1000: (21, 0.0), 2000: (21, 0.0), 3000: (23, 0.0),
               4000: (23, 0.0), 5000: (23, 0.0)}),
    2: (1e-2, {100: (14, 0.0), 500: (22, 0.0), 1000: (22, 0.0), 2000: (22, 0.0), 3000: (23, 0.0),
               4000: (23, 0.0), 5000: (24, 0.0)}),
    3: (1e-3, {100: (14, 0.0), 500: (23, 0.0), 1000: (23, 0.0), 2000: (23, 0.0), 3000: (25, 0.0),
               4000: (25, 0.0), 5000: (26, 0.0)}),
    4: (1e-4, {100: (16, 0.0), 500: (24, 0.0), 1000: (24, 0.0), 2000: (26, 0.0), 3000: (26, 0.5),
               4000: (26, 0.5), 5000: (26, 0.5)}),
}


def paper_hamiltonian(xy, gamma, dev):
    """The paper's Hamiltonian, (1/4pi) sum_j sum_{i != j} G_i G_j log|r| (the
    negative of the regularized form at delta = 0), from the stream-function kernel."""
    x = torch.tensor(np.asarray(xy, np.float32), device=dev)
    g = torch.tensor(np.asarray(gamma, np.float32), device=dev)
    return -float(native.hamiltonian(x, g, 0.0).item())


def run(n, case=1, depth=16, device=None):
    dev = torch.device("cuda", 0) if device is None else device
    cl = single_vortex(n)
    dt, tf = cl.meta["dt"], cl.meta["tf"]
    steps = int(round(tf / dt))
    tol, table = BASES[case]
    M, pc = table[n]
    Mr, ns = 2 * M, 2 * M
    x0 = torch.tensor(np.asarray(cl.xy, np.float32), device=dev)
    g = torch.tensor(np.asarray(cl.gamma, np.float32), device=dev)

    # FOM (Tier I) timing: trapezoid steps, Newton-GMRES on the GPU
    x = x0.clone()
    native.implicit(x, g, 0.0, dt, 2, scheme=native.TRAPEZOID)  # warm-up
    x = x0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = native.implicit(x, g, 0.0, dt, steps, scheme=native.TRAPEZOID, newton_tol=1e-6, gmres_tol=1e-4)
    torch.cuda.synchronize()
    t_fom = time.perf_counter() - t0
    # the same FOM with the paper's inexact Newton (block-diagonal Jacobian
    # at every iterate, at most 100 iterations), timed and compared
    xb = x0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stb = native.implicit(xb, g, 0.0, dt, steps, scheme=native.TRAPEZOID, newton_tol=1e-6, max_newton=100,
                          linear_solver=native.NEWTON_BLOCK)
    torch.cuda.synchronize()
    t_fom_block = time.perf_counter() - t0
    block_rel = float(torch.linalg.norm((xb - x).double()) / torch.linalg.norm((x - x0).double()))

    # offline training (snapshots recomputed inside, one per step)
    t0 = time.perf_counter()
    art, info = offline.train(cl, dt=dt, nsnap=steps, M=M, Mr=Mr, ns=ns, depth=depth, pc=pc, tol=tol,
                              max_iter=100, device=dev)
    t_off = time.perf_counter() - t0

    # online PTROM (Tier III)
    rom = native.Rom(art, tol=tol, max_iter=100)
    xh = torch.zeros(M, dtype=torch.float64, device=dev)
    hist = torch.empty(steps * M, dtype=torch.float64, device=dev)
    its = torch.empty(steps, dtype=torch.int32, device=dev)
    rom.run(1, xh, None, None)
    xh.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rom.run(steps, xh, hist, its)
    torch.cuda.synchronize()
    t_rom = time.perf_counter() - t0

    # accuracy against the FOM snapshots (every 10th step for the Hamiltonian)
    S = info["S"]
    Phi = info["Phi"]
    xy0 = np.asarray(cl.xy, np.float32).astype(np.float64)
    rec = xy0[None, :] + hist.cpu().numpy().reshape(steps, M) @ Phi.T
    length = float(np.hypot(xy0[n - 1] - xy0[0], xy0[2 * n - 1] - xy0[n]))
    mae = [offline.mae_distance(rec[t], S[t], n, length) for t in range(steps)]
    ae = []
    for t in range(0, steps, max(1, steps // 50)):
        hI = paper_hamiltonian(S[t], cl.gamma, dev)
        hIII = paper_hamiltonian(rec[t], cl.gamma, dev)
        ae.append(abs((hIII - hI) / hI))
    it = its.cpu().numpy()
    return dict(study="single_vortex_reproductive", N=n, bases_case=case, tol=tol, M=M, Mr=Mr, ns=ns, pc=pc,
                Nc=int(np.asarray(art["Gt"]).size), nnz=int(np.asarray(art["ids"]).size), steps=steps, dt=dt,
                fom_seconds=t_fom, fom_newton_iters=st.newton_iters, fom_krylov_iters=st.krylov_iters,
                fom_block_seconds=t_fom_block, fom_block_newton_iters=stb.newton_iters,
                fom_block_nonconverged_steps=stb.nonconverged_steps, fom_block_vs_gmres_final_rel=block_rel,
                ptrom_online_seconds=t_rom, speedup_SF=t_fom / t_rom, speedup_SF_block=t_fom_block / t_rom,
                offline_seconds=t_off,
                mean_gn_iterations=float(it.mean()), max_gn_iterations=int(it.max()),
                mae_d_time_avg=float(np.mean(mae)), ae_h_time_avg=float(np.mean(ae)),
                report=info["report"])


# The two parametric experiments of the paper's results (vortex pair and
# mushroom cloud): N = 500 bodies, mu = (Gamma_1, Gamma_N), 4 Latin-hypercube
# training points, a 6 x 6 query grid, and the paper's hyper-parameters.
PARAMETRIC = {
    "vortex_pair": dict(lo=(0.25 * 255.0, 0.25 * 255.0), hi=(255.0, 255.0), dt=0.01, t_f=5.0,
                        M=85, Mr=110, ns=60, inflow=False),
    "mushroom_cloud": dict(lo=(-220.0, 0.5 * 220.0), hi=(-0.5 * 220.0, 220.0), dt=0.005, t_f=5.0,
                           M=110, Mr=185, ns=75, inflow=True),
}


def parametric_study(case="vortex_pair", n=500, M=None, Mr=None, ns=None, pc=1.0, tol=1e-4, depth=16, ntrain=4,
                     grid=6, seed=2103, newton_tol=2e-5, device=None):
    """Parametric experiment: offline training at ntrain Latin-hypercube
    points, then grid x grid queries (Gamma~ reassigned on the device) in one
    batched launch; accuracy of every query against its trapezoid FOM.  The
    FP32 FOM's Newton tolerance sits just above the rounding floor of states
    of magnitude ~50."""
    cfg = PARAMETRIC[case]
    M = cfg["M"] if M is None else M
    Mr = cfg["Mr"] if Mr is None else Mr
    ns = cfg["ns"] if ns is None else ns
    dt, t_f = cfg["dt"], cfg["t_f"]
    make = W.vortex_pair if case == "vortex_pair" else W.mushroom_cloud
    dev = torch.device("cuda", 0) if device is None else device
    steps = int(round(t_f / dt))
    lo, hi = np.asarray(cfg["lo"]), np.asarray(cfg["hi"])
    mus_train = W.latin_hypercube(ntrain, lo, hi, seed)
    mus_q = W.parameter_grid(grid, lo, hi)
    clouds = [make(m, n=n) for m in mus_train]
    u = W.mushroom_inflow(n) if cfg["inflow"] else None
    t0 = time.perf_counter()
    log = lambda msg: print("[%s] %s" % (case, msg), file=sys.stderr, flush=True)
    art, info = offline.train_parametric(clouds, dt=dt, nsnap=steps, M=M, Mr=Mr, ns=ns, depth=depth, pc=pc, tol=tol,
                                         max_iter=100, device=dev, newton_tol=newton_tol, u=u, log=log)
    t_off = time.perf_counter() - t0
    log("offline done in %.1f s: Nc = %d, nnz = %d" % (t_off, np.asarray(art["Gt"]).size, np.asarray(art["ids"]).size))
    rom = native.Rom(art, tol=tol, max_iter=100)
    nq = len(mus_q)
    G = torch.tensor(np.stack([np.asarray(make(m, n=n).gamma, np.float32) for m in mus_q]), device=dev)
    gt = rom.reassign(G)
    xq = torch.zeros((nq, M), dtype=torch.float64, device=dev)
    hq = torch.empty((nq, steps, M), dtype=torch.float64, device=dev)
    iq = torch.empty((nq, steps), dtype=torch.int32, device=dev)
    rom.run_batched(gt[:1], 2, xq[:1].clone())  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gt = rom.reassign(G)
    rom.run_batched(gt, steps, xq, hq, iq)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    x1 = torch.zeros((1, M), dtype=torch.float64, device=dev)
    i1 = torch.empty((1, steps), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rom.run_batched(gt[:1], steps, x1, None, i1)
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    its_one = int(i1.sum().item())
    log("online: %d queries in %.3f s, one query %.3f s (%d GN iterations, %.1f us each)"
        % (nq, t_batch, t_one, its_one, 1e6 * t_one / max(its_one, 1)))

    # trapezoid FOM of every query (timed per query) and the QoIs
    Phi = info["Phi"]
    xy0 = np.asarray(clouds[0].xy, np.float32).astype(np.float64)
    length = float(np.hypot(xy0[n - 1] - xy0[0], xy0[2 * n - 1] - xy0[n]))
    delta = float(clouds[0].delta)
    ud = None if u is None else torch.tensor(np.asarray(u, np.float32), device=dev)
    maes, aes, t_fom = [], [], []
    t_fom_block, block_mae, block_nonconv = [], [], 0
    for q, m in enumerate(mus_q):
        cl = make(m, n=n)
        g = torch.tensor(np.asarray(cl.gamma, np.float32), device=dev)
        x = torch.tensor(xy0, dtype=torch.float32, device=dev)
        traj_d = torch.empty((steps, 2 * n), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(steps):
            native.implicit(x, g, delta, dt, 1, scheme=native.TRAPEZOID, newton_tol=newton_tol, gmres_tol=1e-4,
                            uinf=ud)
            traj_d[t].copy_(x)
        torch.cuda.synchronize()
        t_fom.append(time.perf_counter() - t0)
        # the paper's inexact Newton (block Jacobian at every iterate), same loop
        xb = torch.tensor(xy0, dtype=torch.float32, device=dev)
        trb_d = torch.empty((steps, 2 * n), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(steps):
            sb = native.implicit(xb, g, delta, dt, 1, scheme=native.TRAPEZOID, newton_tol=newton_tol, max_newton=100,
                                 uinf=ud, linear_solver=native.NEWTON_BLOCK)
            block_nonconv += sb.nonconverged_steps
            trb_d[t].copy_(xb)
        torch.cuda.synchronize()
        t_fom_block.append(time.perf_counter() - t0)
        traj = traj_d.double().cpu().numpy()
        trb = trb_d.double().cpu().numpy()
        block_mae.append(float(np.mean([offline.mae_distance(trb[t], traj[t], n, length) for t in range(steps)])))
        rec = xy0[None, :] + hq[q].cpu().numpy() @ Phi.T
        maes.append(float(np.mean([offline.mae_distance(rec[t], traj[t], n, length) for t in range(steps)])))
        hs = []
        for t in range(0, steps, max(1, steps // 25)):
            h1 = float(native.hamiltonian(torch.tensor(traj[t], dtype=torch.float32, device=dev), g, delta).item())
            h3 = float(native.hamiltonian(torch.tensor(rec[t], dtype=torch.float32, device=dev), g, delta).item())
            hs.append(abs((h3 - h1) / h1))
        aes.append(float(np.mean(hs)))
        log("query %d: FOM %.2f s (block Newton %.2f s), MAE_D %.3e" % (q, t_fom[-1], t_fom_block[-1], maes[-1]))
    it = iq.cpu().numpy()
    return dict(study=case + "_parametric", N=n, M=M, Mr=Mr, ns=ns, pc=pc, tol=tol, steps=steps, dt=dt,
                mu_lo=lo.tolist(), mu_hi=hi.tolist(), train_mu=mus_train.tolist(), queries=nq,
                Nc=int(np.asarray(art["Gt"]).size), nnz=int(np.asarray(art["ids"]).size), offline_seconds=t_off,
                online_batched_seconds=t_batch, online_one_query_seconds=t_one,
                online_one_query_gn_iterations=its_one, online_one_query_us_per_gn_iteration=1e6 * t_one / max(its_one, 1),
                batched_queries_per_one_query_time=nq * t_one / t_batch,
                fom_seconds_per_query=float(np.mean(t_fom)), speedup_SF_per_query=float(np.mean(t_fom)) / (t_batch / nq),
                fom_block_seconds_per_query=float(np.mean(t_fom_block)),
                speedup_SF_block_per_query=float(np.mean(t_fom_block)) / (t_batch / nq),
                fom_block_vs_gmres_mae_d_max=float(np.max(block_mae)), fom_block_nonconverged_steps=block_nonconv,
                mean_gn_iterations=float(it.mean()), max_gn_iterations=int(it.max()),
                mae_d_time_avg_mean=float(np.mean(maes)), mae_d_time_avg_max=float(np.max(maes)),
                ae_h_time_avg_mean=float(np.mean(aes)), ae_h_time_avg_max=float(np.max(aes)),
                mae_d_per_query=maes, report=info["report"])


def vortex_pair_study(**kw):
    """The vortex-pair parametric experiment (see ``parametric_study``)."""
    return parametric_study("vortex_pair", **kw)


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--study", default="single_vortex", choices=["single_vortex"] + sorted(PARAMETRIC))
    p.add_argument("--n", type=int, nargs="+", default=[500])
    p.add_argument("--case", type=int, default=1)
    p.add_argument("--basis", type=int, nargs=3, default=None, metavar=("M", "MR", "NS"),
                   help="parametric studies: M, M_r, n_s (default: the paper's)")
    a = p.parse_args(argv)
    if a.study in PARAMETRIC:
        M, Mr, ns = a.basis if a.basis else (None, None, None)
        print(json.dumps(parametric_study(a.study, M=M, Mr=Mr, ns=ns)), flush=True)
        return 0
    for n in a.n:
        print(json.dumps(run(n, a.case)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
