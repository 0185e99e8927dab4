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
                ptrom_online_seconds=t_rom, speedup_SF=t_fom / t_rom, offline_seconds=t_off,
                mean_gn_iterations=float(it.mean()), max_gn_iterations=int(it.max()),
                mae_d_time_avg=float(np.mean(mae)), ae_h_time_avg=float(np.mean(ae)),
                report=info["report"])


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--n", type=int, nargs="+", default=[500])
    p.add_argument("--case", type=int, default=1)
    a = p.parse_args(argv)
    for n in a.n:
        print(json.dumps(run(n, a.case)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
