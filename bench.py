#!/usr/bin/env python3
"""Benchmark of the regularized Biot-Savart hot path on one MI355X.

Timed step (Gaussian vortex patch, N = 65536, sigma 0.25,
Gamma_i = exp(-|x_i|^2/0.1)/N, delta = 0.01): one velocity evaluation, eight
Jacobian-vector products with random unit vectors, then 50 backward-Euler
steps (dt 5e-4) solved by Newton-GMRES over the Jacobian-product kernel.  The
state is reset at the start of every step so each step does the same work.

value = pair interactions evaluated in the timed steps (velocity and
Jacobian-product kernels, N(N-1) per evaluation) / timed wall time.

Also reported ("forms"): the batched persistent stepper (256 instances,
20 RK4 steps), the checkpointed adjoint (N = 131072, 200 RK4 steps, forward
+ backward) and the online PTROM step, each as pair interactions per second
on the same GPU; "roofline" for the dominant kernel (the Jacobian product);
"cpu_baseline" = the FP64 oracle timed on a bounded sample on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-forms] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3
# algorithmic FP32 work per ordered pair interaction (FMA = 2, reciprocal = 1),
# counted from the one-sided formulas the kernels evaluate
FLOP_PER_PAIR = {"velocity": 12, "jvp": 23, "vjp": 31, "block_jacobian": 22}
# FP32 work the each-unordered-pair-once kernels execute per UNORDERED pair:
# the shared distance/reciprocal terms once, the forward and reaction
# accumulations, and the per-step lane rotation of the reaction accumulators
SYM_FLOP_PER_UNORDERED_PAIR = {"velocity": 19, "jvp": 30, "vjp": 41}
PAIR_SOURCES = ("pair_core.h", "pair_sym_core.h", "pair.hip", "pair_sym.hip")
OP_ID = {"velocity": 0, "block_jacobian": 1, "jvp": 2, "vjp": 3, "stream_function": 4}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--no-forms", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--only", default="", help="comma list of forms to run (batched,adjoint,implicit,rom,next)")
    p.add_argument("--gather-ns", default="16,256,2048,16384",
                   help="sample-set sizes of the HyperPair gather sweep (rom form)")
    p.add_argument("--rom-workgroups", type=int, default=0,
                   help="workgroups per query of the small-basis online runs (0 automatic, 1 no split: "
                        "for profilers that do not follow cooperative launches)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain device copy of known size (HBM counter calibration)")
    return p.parse_args()


# workgroups per query of the small-basis online runs (--rom-workgroups)
ROM_WORKGROUPS = 0


def main():
    global ROM_WORKGROUPS
    args = parse()
    ROM_WORKGROUPS = args.rom_workgroups
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2
    if not args.no_cpu:
        import oracle
        oracle.lib()  # loaded (compiled if stale) before the GPU is touched
    import torch
    from paper_2103_01983_amd import native
    from paper_2103_01983_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = W.CONFIGS["c2_gaussian_patch"]
    cl = W.config_cloud("c2_gaussian_patch")
    n = cl.n
    x0 = torch.tensor(cl.xy, dtype=torch.float32, device=dev)
    g = torch.tensor(cl.gamma, dtype=torch.float32, device=dev)
    V = torch.tensor(W.unit_vectors(n, cfg["njvp"], 1002), dtype=torch.float32, device=dev)
    x = x0.clone()
    f = torch.empty_like(x0)
    jv = torch.empty_like(x0)
    d, dt = float(cl.delta), float(cfg["dt"])
    pairs = float(n) * (n - 1)
    stream = torch.cuda.current_stream(dev)

    timings = {"velocity": [], "jvp": []}
    counts = {"vel": 0, "jvp": 0, "newton": 0}

    def step(record):
        x.copy_(x0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        native.velocity(x, g, d, out=f)
        e1.record(stream)
        ev = []
        for k in range(cfg["njvp"]):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            native.jvp(x, g, d, V[k], out=jv)
            b.record(stream)
            ev.append((a, b))
        st = native.implicit(x, g, d, dt, cfg["steps"])
        if record:
            torch.cuda.synchronize()
            timings["velocity"].append(e0.elapsed_time(e1))
            timings["jvp"].extend(a.elapsed_time(b) for a, b in ev)
            counts["vel"] += 1 + cfg["steps"] + st.newton_iters
            counts["jvp"] += cfg["njvp"] + st.krylov_iters
            counts["newton"] += st.newton_iters
        return st

    log("warmup", args.warmup)
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log("timed steps", args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_pairs = pairs * (counts["vel"] + counts["jvp"])
    value = total_pairs / wall
    ms_step = 1e3 * wall / args.steps

    jvp_ms = float(np.mean(timings["jvp"]))
    vel_ms = float(np.mean(timings["velocity"]))
    roof = roofline_entry(native, "jvp", n, pairs, jvp_ms)
    roof_vel = roofline_entry(native, "velocity", n, pairs, vel_ms)
    roof_vel["pairs_per_s"] = pairs / (vel_ms * 1e-3)

    out = {
        "metric": "Biot-Savart pair-interactions/s at <=1e-5 rel err; batched & adjoint vs plain",
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "gaussian_patch_n65536: velocity + 8 JVP + 50 backward-Euler Newton-GMRES steps",
                   "N": n, "delta": d, "dt": dt, "be_steps": cfg["steps"], "jvp_vectors": cfg["njvp"],
                   "velocity_evals_per_step": counts["vel"] / args.steps,
                   "jvp_evals_per_step": counts["jvp"] / args.steps,
                   "newton_iters_per_step": counts["newton"] / args.steps},
        "roofline": roof,
        "roofline_velocity": roof_vel,
    }

    if not args.no_forms:
        only = set(s for s in args.only.split(",") if s)
        out["forms"] = run_forms(native, W, dev, only, pairs / (vel_ms * 1e-3),
                                 tuple(int(v) for v in args.gather_ns.split(",") if v))

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cl, f, native, x0, g, d)

    print(json.dumps(out), flush=True)
    return 0


def copy_calibration():
    """Five copies of a 256 MiB buffer: 256 MiB read + 256 MiB written each."""
    import torch
    a = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4, "copies": 5}))
    return 0


def kernel_names(op, cfg):
    """Kernels one launch of pair operation ``op`` runs under launch ``cfg``."""
    o = OP_ID[op]
    if cfg["sym"]:
        return ["sym_reset_kernel", f"pair_sym_kernel<{o}, {cfg['k']}>", f"sym_reduce_kernel<{o}>"]
    names = [f"pair_kernel<{o}, {cfg['k']}, {cfg['staging']}>"]
    if cfg["splits"] > 1:
        names.append(f"reduce_kernel<{o}>")
    return names


def roofline_entry(native, op, n, pairs, launch_ms):
    """Roofline record of one pair-operation launch timed with HIP events on
    its stream (all kernels of the launch)."""
    cfg = native.pair_config(op, n)
    ach = FLOP_PER_PAIR[op] * pairs / (launch_ms * 1e-3) / 1e12
    r = {
        "bound": "alu",
        "kernel": " + ".join(kernel_names(op, cfg)) + f" ({op}, N={n})",
        "launch": cfg,
        "achieved": ach,
        "peak": PEAK_FP32_TFLOPS,
        "unit": "TFLOP/s",
        "frac": ach / PEAK_FP32_TFLOPS,
        "frac_basis": "algorithmic FLOP (FLOP per ordered pair x N(N-1)) / launch time; executed_frac "
                      "counts the FP32 work the each-pair-once kernel issues",
        "avg_launch_ms": launch_ms,
        "flop_per_pair": FLOP_PER_PAIR[op],
        "traffic": traffic_for(op, cfg),
    }
    if cfg["sym"]:
        ex = SYM_FLOP_PER_UNORDERED_PAIR[op] * pairs / 2 / (launch_ms * 1e-3) / 1e12
        r["executed_flop_per_unordered_pair"] = SYM_FLOP_PER_UNORDERED_PAIR[op]
        r["executed_tflops"] = ex
        r["executed_frac"] = ex / PEAK_FP32_TFLOPS
    return r


def pair_source_sha():
    from hashlib import sha256
    h = sha256()
    for f in PAIR_SOURCES:
        with open(os.path.join(ROOT, "paper_2103_01983_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(op, cfg):
    """HBM bytes per launch (all kernels of the launch) from committed
    rocprofv3 counter runs, if they were taken on the current pair-kernel
    sources and the same launch configuration."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = t.get(op)
    if not ent or ent.get("source_sha") != pair_source_sha() or ent.get("launch") != cfg:
        return None
    return ent.get("bytes_per_launch")


def run_forms(native, W, dev, only, plain_pairs_per_s, gather_ns=(16, 256, 2048, 16384)):
    import torch
    forms = {"plain_velocity_pairs_per_s": plain_pairs_per_s}
    stream = torch.cuda.current_stream(dev)

    def timed(fn, reps=1):
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps * 1e-3

    if not only or "batched" in only:
        log("form: batched")
        bt = W.batched_patches()
        c4 = W.CONFIGS["c4_batched"]
        xb0 = torch.tensor(bt.xy, dtype=torch.float32, device=dev)
        gb = torch.tensor(bt.gamma, dtype=torch.float32, device=dev)
        xb = xb0.clone()
        nb = np.diff(bt.offsets).astype(np.float64)
        pairs_eval = float(np.sum(nb * (nb - 1)))
        native.rk4_batched(bt.offsets, xb, gb, bt.delta, c4["dt"], 1)  # plan + graph
        xb.copy_(xb0)
        sec = timed(lambda: native.rk4_batched(bt.offsets, xb, gb, bt.delta, c4["dt"], c4["steps"]))
        forms["batched"] = {"instances": int(nb.size), "bodies": int(nb.sum()), "rk4_steps": c4["steps"],
                            "seconds": sec, "pairs_per_s": 4 * c4["steps"] * pairs_eval / sec,
                            "ratio_to_plain": 4 * c4["steps"] * pairs_eval / sec / plain_pairs_per_s}
        xb.copy_(xb0)
        sec1 = timed(lambda: native.velocity_batched(bt.offsets, xb, gb, bt.delta), reps=3)
        forms["batched"]["velocity_eval_pairs_per_s"] = pairs_eval / sec1
        nbar = int(np.sum(nb * nb) / np.sum(nb))
        forms["batched"]["launch"] = dict(native.pair_config("batched_velocity", nbar), pair_weighted_mean_size=nbar,
                                          source="tuning table (ptrom_autotune)")
        del xb0, xb, gb

    if not only or "adjoint" in only:
        log("form: adjoint")
        c5 = W.CONFIGS["c5_adjoint"]
        cl = W.config_cloud("c5_adjoint")
        n = cl.n
        x0 = torch.tensor(cl.xy, dtype=torch.float32, device=dev)
        g = torch.tensor(cl.gamma, dtype=torch.float32, device=dev)
        steps, every, dt, d = c5["steps"], c5["every"], c5["dt"], cl.delta
        pairs = float(n) * (n - 1)
        holder = {}

        def fwd():
            holder["ck"], holder["xT"] = native.rk4_fwd_ckpt(x0, g, d, dt, steps, every)

        sec_f = timed(fwd)
        lamT = torch.ones_like(x0)

        def bwd():
            native.rk4_bwd(holder["ck"], g, d, dt, steps, every, lamT)

        sec_b = timed(bwd)
        forms["adjoint"] = {"N": n, "rk4_steps": steps, "checkpoint_every": every,
                            "forward_seconds": sec_f, "backward_seconds": sec_b,
                            "forward_pairs_per_s": 4 * steps * pairs / sec_f,
                            # recompute: 4 velocities per step but 3 on each segment's last step;
                            # then 4 vector-Jacobian products per step
                            "backward_pairs_per_s": (8 * steps - -(-steps // every)) * pairs / sec_b,
                            "backward_over_forward_time": sec_b / sec_f,
                            "note": "backward = recompute (velocity) + vector-Jacobian pair kernels"}
        del holder

    if not only or "implicit" in only:
        log("form: implicit")
        try:
            forms["implicit"] = implicit_form(native, W, dev)
        except Exception as e:
            forms["implicit"] = {"error": repr(e)}
    if not only or "rom" in only:
        log("form: rom")
        try:
            forms["rom"] = rom_form(native, W, dev, timed, gather_ns)
        except Exception as e:  # reported, not fatal to the headline line
            forms["rom"] = {"error": repr(e)}
    if not only or "next" in only:
        log("form: next")
        try:
            forms["next"] = next_rows(native, W, dev, timed)
        except Exception as e:
            forms["next"] = {"error": repr(e)}
    return forms


def implicit_form(native, W, dev):
    """The implicit FOM with both Newton linear models: the N = 65536 patch
    (50 backward-Euler steps, as in the timed step) and the vortex pair at the
    paper's size (N = 500, trapezoid, dt = 0.01, end circulations 255)."""
    import torch
    out = {}
    cases = []
    cfg = W.CONFIGS["c2_gaussian_patch"]
    cl = W.config_cloud("c2_gaussian_patch")
    cases.append(("gaussian_patch_n65536_be", cl, float(cl.delta), float(cfg["dt"]), cfg["steps"],
                  native.BACKWARD_EULER, 1e-6))
    vp = W.vortex_pair((255.0, 255.0), n=500)
    cases.append(("vortex_pair_n500_trapezoid", vp, float(vp.delta), 0.01, 100, native.TRAPEZOID, 2e-5))
    for name, c, d, dt, steps, scheme, tol in cases:
        n = c.n
        x0 = torch.tensor(np.asarray(c.xy, np.float32), device=dev)
        g = torch.tensor(np.asarray(c.gamma, np.float32), device=dev)
        pairs = float(n) * (n - 1)
        row, finals = {"N": n, "steps": steps, "dt": dt}, {}
        for label, kw in (("gmres", dict(linear_solver=native.NEWTON_GMRES, gmres_tol=1e-3)),
                          ("block", dict(linear_solver=native.NEWTON_BLOCK, max_newton=100))):
            x = x0.clone()
            native.implicit(x, g, d, dt, 2, scheme=scheme, newton_tol=tol, **kw)  # warm-up
            x = x0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = native.implicit(x, g, d, dt, steps, scheme=scheme, newton_tol=tol, **kw)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            # pair evaluations: a velocity per step and per Newton iterate, plus
            # a JVP per Krylov vector (GMRES) or a block Jacobian per iterate
            evals = steps + st.newton_iters + (st.krylov_iters if label == "gmres" else st.newton_iters)
            row[label] = {"seconds": sec, "ms_per_step": 1e3 * sec / steps,
                          "newton_iters_per_step": st.newton_iters / steps,
                          "krylov_iters_per_step": st.krylov_iters / steps,
                          "nonconverged_steps": st.nonconverged_steps,
                          "pairs_per_s": evals * pairs / sec}
            finals[label] = x
        disp = torch.linalg.norm((finals["gmres"] - x0).double())
        row["block_vs_gmres_final_rel"] = float(torch.linalg.norm((finals["block"] - finals["gmres"]).double()) / disp)
        out[name] = row
    return out


# FLOP per pair of the stream-function term: separation (2), |r|^2 + delta^2
# (2 FMA), log2 (1), Gamma log2 FMA (2)
PSI_FLOP_PER_PAIR = 9


def next_rows(native, W, dev, timed):
    """The widened rows on their own workloads: the log-kernel stream
    function over the C2 patch, the velocity at a 256 x 256 grid of field
    points from the same bodies, and the C3 pipeline clustered by the
    Barnes-Hut criterion instead of the neighbour overlap test."""
    import torch
    from paper_2103_01983_amd import offline
    out = {}
    c2 = W.CONFIGS["c2_gaussian_patch"]
    cl = W.config_cloud("c2_gaussian_patch")
    n = cl.n
    x = torch.tensor(cl.xy, dtype=torch.float32, device=dev)
    g = torch.tensor(cl.gamma, dtype=torch.float32, device=dev)
    psi = torch.empty_like(g)
    native.stream_function(x, g, c2["delta"], psi)
    sec = timed(lambda: native.stream_function(x, g, c2["delta"], psi), reps=10)
    pairs = float(n) * (n - 1)
    out["stream_function"] = {"N": n, "launch_ms": sec * 1e3, "pairs_per_s": pairs / sec,
                              "tflops": PSI_FLOP_PER_PAIR * pairs / sec / 1e12, "flop_per_pair": PSI_FLOP_PER_PAIR,
                              "frac_of_157_3": PSI_FLOP_PER_PAIR * pairs / sec / 157.3e12}
    side = 256
    gx = np.linspace(-1.0, 1.0, side)
    pts = np.concatenate([np.tile(gx, side), np.repeat(gx, side)])
    P = torch.tensor(pts, dtype=torch.float32, device=dev)
    fv = torch.empty_like(P)
    native.velocity_points(P, x, g, c2["delta"], fv)
    sec = timed(lambda: native.velocity_points(P, x, g, c2["delta"], fv), reps=10)
    pp = float(side * side) * n
    out["velocity_points"] = {"points": side * side, "N": n, "launch_ms": sec * 1e3, "pairs_per_s": pp / sec,
                              "tflops": 12 * pp / sec / 1e12}
    c3 = W.CONFIGS["c3_ptrom_pipeline"]
    cl3 = W.config_cloud("c3_ptrom_pipeline")
    for crit, theta in ((native.NEIGHBOR, 0.0), (native.BARNES_HUT, 0.5)):
        t0 = time.perf_counter()
        art, info = offline.train(cl3, dt=c3["dt"], nsnap=c3["snapshots"], M=c3["M"], Mr=c3["Mr"], ns=c3["ns"],
                                  depth=c3["depth"], pc=c3["pc"], tol=c3["tol"], max_iter=c3["max_iter"], device=dev,
                                  criterion=crit, theta=theta)
        t_off = time.perf_counter() - t0
        rom = native.Rom(art, tol=c3["tol"], max_iter=c3["max_iter"])
        rom.set_split(ROM_WORKGROUPS)
        steps = c3["steps"]
        xh = torch.zeros(art["M"], dtype=torch.float64, device=dev)
        hist = torch.empty(steps * art["M"], dtype=torch.float64, device=dev)
        it = torch.empty(steps, dtype=torch.int32, device=dev)
        rom.run(2, xh, None, None)
        xh.zero_()
        sec = timed(lambda: rom.run(steps, xh, hist, it))
        its = it.cpu().numpy()
        Phi, S = info["Phi"], info["S"]
        x0 = np.asarray(cl3.xy, np.float32).astype(np.float64)
        m = cl3.n
        length = float(np.hypot(x0[m - 1] - x0[0], x0[2 * m - 1] - x0[m]))
        xr = x0[None, :] + hist.cpu().numpy().reshape(steps, -1) @ Phi.T
        mae = [offline.mae_distance(xr[t], S[t], m, length) for t in range(min(steps, S.shape[0]))]
        key = "c3_neighbor" if crit == native.NEIGHBOR else "c3_barnes_hut_theta_0_5"
        out[key] = {"Nc": int(np.asarray(art["Gt"]).size), "nnz": int(np.asarray(art["ids"]).size),
                    "tier2_nnz": info["report"].get("tier2_nnz"), "offline_seconds": t_off,
                    "us_per_gn_iteration": 1e6 * sec / max(int(its.sum()), 1),
                    "mean_gn_iterations": float(its.mean()), "mae_d_time_avg": float(np.mean(mae))}
        rom.close()
    return out


def rom_form(native, W, dev, timed, gather_ns=(16, 256, 2048, 16384)):
    import torch
    from paper_2103_01983_amd import offline
    c3 = W.CONFIGS["c3_ptrom_pipeline"]
    cl = W.config_cloud("c3_ptrom_pipeline")
    t0 = time.perf_counter()
    art, info = offline.train(cl, dt=c3["dt"], nsnap=c3["snapshots"], M=c3["M"], Mr=c3["Mr"], ns=c3["ns"],
                              depth=c3["depth"], pc=c3["pc"], tol=c3["tol"], max_iter=c3["max_iter"], device=dev)
    t_off = time.perf_counter() - t0
    rom = native.Rom(art, tol=c3["tol"], max_iter=c3["max_iter"])
    rom.set_split(ROM_WORKGROUPS)
    steps = c3["steps"]
    xh = torch.zeros(art["M"], dtype=torch.float64, device=dev)
    hist = torch.empty(steps * art["M"], dtype=torch.float64, device=dev)
    it = torch.empty(steps, dtype=torch.int32, device=dev)
    rom.run(2, xh, None, None)
    xh.zero_()
    sec = timed(lambda: rom.run(steps, xh, hist, it))
    its = it.cpu().numpy()
    nnz = int(np.asarray(art["ids"]).size)
    res = {"N": cl.n, "M": art["M"], "Mr": art["Mr"], "ns": int(len(art["off"]) - 1), "Nc": int(np.asarray(art["Gt"]).size),
           "nnz": nnz, "steps": steps, "offline_seconds": t_off, "online_seconds": sec,
           "us_per_step": 1e6 * sec / steps, "us_per_gn_iteration": 1e6 * sec / max(int(its.sum()), 1),
           "mean_gn_iterations": float(its.mean()), "pairs_per_s": float(its.sum()) * nnz / sec,
           "workgroups_per_query": rom.split_plan(steps)}
    res.update(info.get("report", {}))
    # accuracy against the trapezoid FOM snapshots (reported, not a gate)
    Phi, S = info["Phi"], info["S"]
    x0 = np.asarray(cl.xy, np.float32).astype(np.float64)
    n = cl.n
    length = float(np.hypot(x0[n - 1] - x0[0], x0[2 * n - 1] - x0[n]))
    xr = x0[None, :] + hist.cpu().numpy().reshape(steps, -1) @ Phi.T
    mae = [offline.mae_distance(xr[t], S[t], n, length) for t in range(min(steps, S.shape[0]))]
    res["mae_d_time_avg"] = float(np.mean(mae))
    res["mae_d_final"] = float(mae[-1])
    res["final_rel_state_err"] = float(np.linalg.norm(xr[-1] - S[-1]) / np.linalg.norm(S[-1] - x0))
    res["gather_sweep"] = gather_sweep(native, offline, info, cl, art, dev, timed, gather_ns)
    return res


def gather_sweep(native, offline, info, cl, art, dev, timed, sizes=(16, 256, 2048, 16384)):
    """HyperPair gather (point form: surrogate positions once, then 4 bytes
    per list entry) over growing sample sets (random bodies; same tree, basis
    and clustering): algorithmic bytes per evaluation / time."""
    import torch
    n = cl.n
    rng = np.random.default_rng(11)
    xy0 = np.asarray(cl.xy, np.float32).astype(np.float64)
    g = np.asarray(cl.gamma, np.float32).astype(np.float64)
    out = []
    for ns in sizes:
        sample = np.arange(n) if ns >= n else np.sort(rng.choice(n, ns, replace=False))
        A = np.zeros((art["M"], 2 * sample.size))
        a = offline.artifacts(sample, info["wpts"], xy0, info["Phi"], g, 6, 1.0, cl.delta, art["dt"], A)
        rom = native.Rom(a)
        M, nd = a["M"], 2 * sample.size
        xh = torch.zeros(M, dtype=torch.float64, device=dev)
        prev = torch.zeros(nd, dtype=torch.float64, device=dev)
        rom.hyperpair(xh, prev, prev)
        reps = 20
        sec = timed(lambda: rom.hyperpair(xh, prev, prev), reps=reps)
        nnz = int(a["ids"].size)
        nc = int(np.asarray(a["Gt"]).size)
        # algorithmic bytes per evaluation: one 4-byte surrogate id per list
        # entry, the offsets, each unique surrogate's reference position,
        # basis rows and circulation (FP32), the sampled rows' basis and
        # reference positions (FP32), the previous-step rows read and xbar,
        # fbar, rbar, C written (FP64)
        byts = 4 * nnz + 4 * (sample.size + 1) + (8 + 8 * M + 4) * nc + 4 * nd * (M + 2) + 5 * nd * 8 + nd * M * 8
        # what the point form moves: the ids, the FP64 mode-major basis and
        # reference positions of all P = nd + 2 Nc coordinates, the positions
        # written (and the targets' read back), the circulations, the packed
        # 32-byte surrogate records written and read, Phibar (for C), the
        # inflow rows, the previous-step rows and the outputs
        P = nd + 2 * nc
        layout = (4 * nnz + 4 * (sample.size + 1) + 8 * P * (M + 1) + 8 * P + 8 * nd + 4 * nc + 64 * nc
                  + 4 * nd * M + 8 * nd + 5 * nd * 8 + nd * M * 8)
        out.append({"ns": int(sample.size), "nnz": nnz, "Nc": nc, "us": sec * 1e6, "bytes": byts,
                    "GB_per_s": byts / sec / 1e9, "layout_bytes": layout, "layout_GB_per_s": layout / sec / 1e9,
                    "pairs_per_s": nnz / sec})
        rom.close()
    return out


def cpu_baseline(cl, f_gpu, native, x0, g, d):
    """FP64 oracle on a bounded sample of targets of the same workload: pair
    interactions/s on the host cores.  Also the GPU result's relative error on
    that sample."""
    import oracle
    n = cl.n
    xy32 = np.asarray(cl.xy, np.float32).astype(np.float64)
    g32 = np.asarray(cl.gamma, np.float32).astype(np.float64)
    d32 = float(np.float32(d))
    rng = np.random.default_rng(7)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # repeat random target samples (each against all sources) until ~10 s of oracle work
    f = f_gpu.double().cpu().numpy()
    done, sec, errs = 0, 0.0, []
    while sec < 10.0:
        idx = rng.choice(n, 8192, replace=False)
        t = time.perf_counter()
        ref = oracle.velocity_at(xy32, g32, d32, idx)
        sec += time.perf_counter() - t
        done += idx.size
        got = np.concatenate([f[idx], f[n + idx]])
        errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
    # the same oracle on one core (the paper's setting), a smaller sample
    prev = oracle.set_threads(1)
    try:
        idx = rng.choice(n, 2048, replace=False)
        t = time.perf_counter()
        oracle.velocity_at(xy32, g32, d32, idx)
        one = idx.size * (n - 1) / (time.perf_counter() - t)
    finally:
        oracle.set_threads(prev)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": done * (n - 1) / sec, "unit": "pair-interactions/s", "cores": threads, "kind": "oracle",
            "build": "gcc -O2 -fopenmp, x86-64 baseline ISA (the oracle as the tests use it; built where the "
                     "library is built, so no -march=native)",
            "sample": "FP64 oracle velocity at %d random targets (batches of 8192) of the N=65536 Gaussian "
                      "patch, each against all sources" % done,
            "seconds": sec, "gpu_rel_err_on_sample_max": max(errs),
            "single_core_value": one, "single_core_sample": "2048 random targets, one thread",
            "nproc": os.cpu_count(), "cpu_model": model}


if __name__ == "__main__":
    sys.exit(main())
