"""Benchmark of the data-parallel hot path of sample-based in-hand pose
tracking on one MI355X.

A "step" is one world step of the whole population with the observation and
the cost (Alg. 1: step every simulation with the same command, observe, add
the step cost against the observed contact forces, update the argmin), plus
the population-based resampling every T steps.  The observed forces are the
tracker's input (the robot's contact sensors); here they come from a
separate batch holding the unperturbed ("real") simulation stepped with the
same commands, run before the timed region so that, like every other input,
they are resident in HBM when timing starts.  Inputs are seeded and synthetic (the paper's YCB objects
and teleoperation trajectories are not available): a 4-finger + palm capsule
hand on sinusoidal joint commands and a 64-sphere ellipsoid on a table.

Default workload: 256 simulations, 300 steps at 30 Hz, plain per-step
launches (the "plain256" scene).  The same run also times the batched path
(one persistent kernel per 10-step window, replayed from a HIP graph) and
the batched path with elite refinement (three gradient steps of the window
cost for the elites before every resampling) on the same workload, and both
batched variants on the 1024-simulation differentiation workload
("adjoint1024").  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)



def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300, help="timed world steps")
    ap.add_argument("--warmup", type=int, default=30, help="untimed world steps first")
    ap.add_argument("--config", default="plain256")
    ap.add_argument("--solve-precision", type=int, default=64, choices=[32, 64])
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the batched + elite-refinement legs")
    ap.add_argument("--realtime-windows", type=int, default=180,
                    help="timed windows of the 16384-simulation real-time workload: 180 x 10 steps is the "
                         "workload's 60 s at 30 Hz (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-optimizers", action="store_true",
                    help="skip the WRS / REPS / identity comparison on the real-time workload")
    ap.add_argument("--cpu-sample-steps", type=int, default=300)
    ap.add_argument("--profile", action="store_true", help="short run for the profiler (no CPU baseline)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB on the device three times (reference for the FETCH_SIZE / WRITE_SIZE "
                         "counters)")
    return ap.parse_args()


# HBM bytes per k_step launch of the 256-simulation workload (float64 solve),
# from FETCH_SIZE / WRITE_SIZE counters scaled by a plain device copy of known
# size (profiles/k_step_plain256.txt); None where the kernel changed since
# the counters were taken, and for any other configuration
MEASURED_TRAFFIC = {("plain256", 64): 1032426}

# VALU counters per k_step launch of the same workload (profiles/
# k_step_plain256.txt): SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU (quad-cycles) and
# SQ_THREAD_CYCLES_VALU summed over the chip; the same staleness rule
MEASURED_VALU = {("plain256", 64): (4030907, 4181518, 233401129)}
SIMDS, CLOCK_HZ = 1024, 2.4e9     # MI355X: 256 CUs x 4 SIMDs at 2.4 GHz; a VALU instruction issues in 4 cycles


def valu_figures(key, launch_s, waves):
    """VALU issue and busy fractions of the chip's peak over one launch of
    launch_s seconds, the active-lane fraction, from MEASURED_VALU; with one
    wavefront per simulation a launch of `waves` wavefronts occupies at most
    waves / SIMDS of the SIMDs (its ceiling)."""
    m = MEASURED_VALU.get(key)
    if m is None:
        return None
    insts, active_q, thread_cyc = m
    slots = SIMDS * CLOCK_HZ * launch_s
    return {"issue_frac": round(insts * 4 / slots, 4), "busy_frac": round(active_q * 4 / slots, 4),
            "lane_frac": round(thread_cyc / (active_q * 64), 3), "insts_per_launch": insts,
            "ceiling": round(min(1.0, waves / SIMDS), 4)}


# algorithmic floating-point operations (an FMA counts 2; a square root,
# division or reciprocal counts 1), counted from the arithmetic of one step
FLOP_SPHERE = 19            # sphere centre x + R s_k, and its table gap
FLOP_PAIR = 23              # sphere-capsule signed gap
FLOP_ENV = 360              # pose, inverse inertia, free velocity, integration, momentum remap
FLOP_ENV_PER_LINK = 25      # per sensor: force magnitude/direction and its cost terms
FLOP_CONTACT = 175          # contact setup (frame, Jacobian, free velocity), body sums, observation
FLOP_CONTACT_ITER = 860     # per Newton iteration: FB value + Jacobian, 3x3 solves, 6x6 contribution,
                            # dr, W dr, one merit trial, cross-contact sums
FLOP_ENV_ITER = 390         # per Newton iteration: 6x6 assembly, LU, velocity updates


def algorithmic_flops(S, L, N, env_steps, contacts):
    per_env = FLOP_ENV + FLOP_ENV_PER_LINK * L + S * FLOP_SPHERE + S * L * FLOP_PAIR + N * FLOP_ENV_ITER
    return env_steps * per_env + contacts * (FLOP_CONTACT + N * FLOP_CONTACT_ITER)


# algorithmic HBM bytes of the plain step kernel per environment-step: state
# (13 floats) and parameters (5) read, state and the consumed perturbation
# force written, the warm-start cache read and written and the contact buffer
# written (C_max x 16 B each); hand segments and sphere tables are shared by
# every simulation and stay in cache
def algorithmic_bytes(C_max):
    return 52 + 20 + 52 + 12 + 3 * 16 * C_max


def observed_forces(pt, sc, dev, solve_precision, n_steps, pose_every=None):
    """The observed ("real") simulation's sensor forces for steps
    0..n_steps-1, [n_steps][R][L][G] (R = 4, or 7 under the full cost of
    Eq. 3).  They are the tracker's input stream
    (the robot's contact sensors), so they are produced before any timed
    region and stay resident in HBM.  With pose_every = T also the observed
    object's state after every T steps ([n_steps / T][13][G], for the
    tracking error)."""
    import torch
    u_all = torch.as_tensor(sc.u.astype("float32"), device=dev)
    h = pt.Batch.from_scene(sc, hidden=True, solve_precision=solve_precision)
    out = torch.empty((n_steps, h.obs_rows, sc.L, sc.G), device=dev)
    poses = []
    for t in range(n_steps):
        h.step(u_all[max(t - 1, 0)], u_all[t])
        h.observe(out[t])
        if pose_every and (t + 1) % pose_every == 0:
            poses.append(h.state.clone())
    torch.cuda.synchronize()
    h.close()
    return (out, torch.stack(poses)) if pose_every else out


def batched_run(pt, S, sc, dev, solve_precision, n_win, n_warm, adjoint):
    """Windows of the batched path: each window's commands and observed
    forces are copied into the two buffers a captured HIP graph reads, the
    population's window is one persistent kernel replayed from that graph,
    then (adjoint) the elites are refined by three gradient steps of the
    window cost from their window start, then the resampler runs."""
    import torch
    cfg = sc.cfg
    K, G, L, T = sc.K, sc.G, sc.L, cfg.T
    n_total = n_warm + n_win + (1 if adjoint else 0)
    gts = observed_forces(pt, sc, dev, solve_precision, n_total * T)
    u_all = torch.as_tensor(sc.u.astype("float32"), device=dev)
    main_b = pt.Batch.from_scene(sc, solve_precision=solve_precision, window_checkpoints=adjoint)
    u_win = torch.empty((T + 1, sc.D), device=dev)
    gt_win = torch.empty((T, main_b.obs_rows, L, G), device=dev)
    cost = torch.zeros(K, device=dev)
    best = torch.zeros(G, dtype=torch.int32, device=dev)
    parent = torch.zeros(K, dtype=torch.int32, device=dev)
    snap = main_b.snapshot()
    improved = [0, 0]

    def window(w, count=False):
        t0_ = w * T
        u_win.copy_(u_all[t0_ - 1: t0_ + T] if t0_ > 0 else torch.cat([u_all[:1], u_all[:T]], 0))
        gt_win.copy_(gts[t0_: t0_ + T])
        if adjoint:
            snap[0].copy_(main_b.state)
            snap[1].copy_(main_b.params)
            snap[2].copy_(main_b.warm)
        main_b.run_window(u_win, gt_win, cost, best, None, graph=True)
        if adjoint:
            c0 = cost.clone() if count else None
            elites = main_b.refine_elites(u_win, gt_win, cost, snap, steps=3, step=0.5, best=best)
            if count:
                e = elites.long()
                improved[0] += int((cost[e] < c0[e]).sum())
                improved[1] += int(e.numel())
        main_b.resample(cost, w, parent)

    u_win.copy_(torch.cat([u_all[:1], u_all[:T]], 0))
    gt_win.copy_(gts[:T])
    tuned = main_b.autotune(u_win, gt_win)
    torch.cuda.synchronize()
    for w in range(n_warm):
        window(w)
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    for w in range(n_warm, n_warm + n_win):
        window(w)
    torch.cuda.synchronize()
    bwall = time.perf_counter() - tb0
    out = {"value": round(K * T * n_win / bwall, 1), "unit": "env-steps/s", "windows": n_win,
           "windows_per_s": round(n_win / bwall, 2), "ms_per_step": round(bwall / (n_win * T) * 1e3, 4),
           "waves_per_workgroup": tuned}
    if adjoint:
        # one more window, untimed, to count the elites the refinement improved
        window(n_warm + n_win, count=True)
        torch.cuda.synchronize()
        out.update({"elites": main_b.elite_count(), "refine_steps": 3,
                    "elites_improved_frac": round(improved[0] / max(improved[1], 1), 3)})
    main_b.close()
    return out


def add_distance(points, pa, pb):
    """Mean distance between the object's points placed at poses pa and pb
    (x(3), q(4)): the tracking error of a pose estimate."""
    import numpy as np

    def rot(q):
        w, x, y, z = q / np.linalg.norm(q)
        return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                         [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                         [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    a = points @ rot(pa[3:7]).T + pa[:3]
    b = points @ rot(pb[3:7]).T + pb[:3]
    return float(np.linalg.norm(a - b, axis=1).mean())


# optimiser hyperparameters of the comparison leg (the paper gives no values):
# WRS temperature per unit of window-mean cost, REPS KL bound
WRS_LAMBDA = 1.0
REPS_EPS = 1.0


def realtime_setup(pt, S, dev, solve_precision, n_total, cost_mode=0):
    """Scene, observed forces and observed poses of the real-time workload,
    shared by the optimisers compared on it (cost_mode 1: the full cost of
    Eq. 3 and its seven-row observation)."""
    import dataclasses
    import torch
    cfg = S.CONFIGS["realtime16384"]
    if cost_mode:
        cfg = cfg.with_(consts=dataclasses.replace(cfg.consts, cost_mode=cost_mode))
    T = cfg.T
    sc = S.make_scene(cfg, steps=(n_total + 1) * T + 1)
    gts, hposes = observed_forces(pt, sc, dev, solve_precision, n_total * T, pose_every=T)
    u_all = torch.as_tensor(sc.u.astype("float32"), device=dev)
    return {"cfg": cfg, "sc": sc, "gts": gts, "hposes": hposes, "u_all": u_all}


def eq3_weights(pt, setup, dev, solve_precision):
    """Weights w4..w10 of Eq. 3 such that every term's mean magnitude over
    the population's first window is 1 (Sec. III-C): one window without
    resampling, its observations against the observed ones, the mean of each
    gated term over simulations, sensors and steps."""
    import numpy as np
    import torch
    cfg, sc, gts, u_all = setup["cfg"], setup["sc"], setup["gts"], setup["u_all"]
    T, K, G, L = cfg.T, sc.K, sc.G, sc.L
    c = cfg.consts
    b = pt.Batch.from_scene(sc, solve_precision=solve_precision)
    obs_w = torch.zeros((T, 7, L, K), device=dev)
    b.run_window(torch.cat([u_all[:1], u_all[:T]], 0), gts[:T].contiguous(), torch.zeros(K, device=dev), None,
                 obs_w, graph=False)
    torch.cuda.synchronize()
    b.close()
    o = obs_w.cpu().numpy().astype(np.float64)
    group = np.repeat(np.arange(G), np.diff(np.asarray(sc.group_start)))
    g = gts[:T].cpu().numpy().astype(np.float64)[:, :, :, group]

    def angle(a, b):       # rows on axis 1
        if a.shape[1] == 2:
            cr = np.abs(a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0])
        else:
            cr = np.linalg.norm(np.cross(a, b, axis=1), axis=1)
        return np.arctan2(cr, (a * b).sum(axis=1))

    ina, inb = o[:, 0] > c.tau_contact, g[:, 0] > c.tau_contact
    sla, slb = (o[:, 4] != 0) | (o[:, 5] != 0), (g[:, 4] != 0) | (g[:, 5] != 0)
    roa, rob = o[:, 6] != 0, g[:, 6] != 0
    alpha, beta, gamma = ina == inb, sla == slb, roa == rob
    terms = [~alpha, alpha * np.abs(o[:, 0] - g[:, 0]), alpha * ina * angle(o[:, 1:4], g[:, 1:4]),
             ~beta, beta * sla * angle(o[:, 4:6], g[:, 4:6]),
             ~gamma, gamma * roa * np.abs((o[:, 6] > 0).astype(float) - (g[:, 6] > 0))]
    means = [float(np.mean(t)) for t in terms]
    return tuple(1.0 / m if m > 0 else 1.0 for m in means)


def realtime_run(pt, S, dev, solve_precision, n_win, n_warm=2, optimizer="pbo", setup=None, refine=True,
                 describe=False):
    """The real-time workload: 16384 simulations in 16 groups (one
    superquadric object each), batched windows; with optimizer "pbo", "wrs"
    or "reps" the elites are refined before every resampling by that
    optimiser, with "eye" the population is never refined nor resampled.
    Reports env-steps/s, the per-step latency (window time / T) against the
    33 ms budget of 30 Hz, the resampler's time per window and the tracking
    error: the mean distance between the object's points at the estimated
    pose and at the observed object's pose, after every window, over all
    groups -- the estimate being the lowest-cost simulation (for "eye" also
    the first simulation of each group alone, which is the open-loop
    baseline: without resampling each simulation evolves on its own)."""
    import numpy as np
    import torch
    n_total = n_warm + n_win
    if setup is None:
        setup = realtime_setup(pt, S, dev, solve_precision, n_total)
    cfg, sc, gts, hposes, u_all = setup["cfg"], setup["sc"], setup["gts"], setup["hposes"], setup["u_all"]
    T = cfg.T
    K, G, L = sc.K, sc.G, sc.L
    adapt = optimizer != "eye"
    refine = refine and adapt
    b = pt.Batch.from_scene(sc, solve_precision=solve_precision, window_checkpoints=refine)
    u_win = torch.empty((T + 1, sc.D), device=dev)
    gt_win = torch.empty((T, b.obs_rows, L, G), device=dev)
    cost = torch.zeros(K, device=dev)
    best = torch.zeros(G, dtype=torch.int32, device=dev)
    parent = torch.zeros(K, dtype=torch.int32, device=dev)
    first = torch.as_tensor(np.asarray(sc.group_start[:-1], dtype=np.int64), device=dev)
    snap = b.snapshot()
    est = torch.empty((n_total, 13, G), device=dev)
    est_olp = torch.empty((n_total, 13, G), device=dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_total)]
    ev_rs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_total)]
    ev_win = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_total)]

    def window(w):
        t0_ = w * T
        ev[w][0].record()
        u_win.copy_(u_all[t0_ - 1: t0_ + T] if t0_ > 0 else torch.cat([u_all[:1], u_all[:T]], 0))
        gt_win.copy_(gts[t0_: t0_ + T])
        if refine:
            snap[0].copy_(b.state)
            snap[1].copy_(b.params)
            snap[2].copy_(b.warm)
        ev_win[w][0].record()
        b.run_window(u_win, gt_win, cost, best, None, graph=True)
        ev_win[w][1].record()
        if refine:
            b.refine_elites(u_win, gt_win, cost, snap, steps=3, step=0.5, best=best)
        torch.index_select(b.state, 1, best, out=est[w])
        if not adapt:
            torch.index_select(b.state, 1, first, out=est_olp[w])
        ev_rs[w][0].record()
        if optimizer == "pbo":
            b.resample(cost, w, parent)
        elif optimizer == "wrs":
            b.resample_wrs(cost, T, w, WRS_LAMBDA, parent)
        elif optimizer == "reps":
            b.resample_reps(cost, T, w, REPS_EPS, parent)
        else:
            cost.zero_()
        ev_rs[w][1].record()
        ev[w][1].record()

    u_win.copy_(torch.cat([u_all[:1], u_all[:T]], 0))
    gt_win.copy_(gts[:T])
    tuned = b.autotune(u_win, gt_win)
    torch.cuda.synchronize()
    for w in range(n_warm):
        window(w)
    torch.cuda.synchronize()
    stats0 = b.read_stats()
    t0 = time.perf_counter()
    for w in range(n_warm, n_total):
        window(w)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats1 = b.read_stats()
    step_ms = np.array([ev[w][0].elapsed_time(ev[w][1]) / T for w in range(n_warm, n_total)])
    win_s = sum(ev_win[w][0].elapsed_time(ev_win[w][1]) for w in range(n_warm, n_total)) / 1e3
    # the population's window kernel alone (the graph replay of the
    # persistent k_window; the refinement's forward passes do not count
    # their steps): algorithmic flop of its steps / its HIP-event time
    d_env = stats1["env_steps"] - stats0["env_steps"]
    w_flops = algorithmic_flops(int(sc.n_spheres[0]), L, cfg.newton_iters, d_env,
                                stats1["contacts"] - stats0["contacts"])
    rs_ms = np.array([ev_rs[w][0].elapsed_time(ev_rs[w][1]) for w in range(n_warm, n_total)])
    hp = setup["hposes"].cpu().numpy()

    def tracking(e):
        errs = []
        for w in range(n_warm, n_total):
            for g in range(G):
                pts = sc.spheres[sc.hidden_type[g], :sc.n_spheres[sc.hidden_type[g]], :3]
                errs.append(add_distance(pts, e[w, :7, g], hp[w, :7, g]))
        return {"mean": round(1e3 * float(np.mean(errs)), 3), "p90": round(1e3 * float(np.quantile(errs, 0.9)), 3)}

    b.close()
    out = {"value": round(K * T * n_win / wall, 1), "unit": "env-steps/s",
           "per_step_ms": {"p50": round(float(np.median(step_ms)), 3),
                           "p99": round(float(np.quantile(step_ms, 0.99)), 3)},
           "budget_30hz_met": bool(np.quantile(step_ms, 0.99) < 1000.0 / 30.0),
           "resample_ms_per_window": round(float(np.median(rs_ms)), 4),
           "tracking_error_mm": tracking(est.cpu().numpy()),
           "waves_per_workgroup": tuned,
           "window_kernel": {"bound": "alu", "achieved": round(w_flops / win_s / 1e12, 4), "peak": 78.6,
                             "unit": "TFLOP/s", "frac": round(w_flops / win_s / 1e12 / 78.6, 5),
                             "avg_window_ms": round(win_s / n_win * 1e3, 3),
                             "flop_per_env_step": round(w_flops / max(d_env, 1), 1)}}
    if not adapt:
        out["open_loop_tracking_error_mm"] = tracking(est_olp.cpu().numpy())
    if describe:
        out = {"workload": f"{cfg.name}: {K} simulations in {G} groups (one {int(sc.n_spheres[0])}-sphere "
                           f"superquadric object each) + {G} observed, {L} capsule links, C_max={cfg.C_max}, "
                           f"{cfg.newton_iters} Newton iterations, {T}-step windows, elite refinement (3 steps) and "
                           f"resampling after every window, {n_win} timed windows", **out}
    return out


def plain_run(pt, sc, dev, solve_precision, steps, warmup):
    """The plain per-step path on a scene (step, observe, cost with the
    argmin, the resampler every T steps): env-steps/s over `steps` timed
    steps after `warmup`."""
    import torch
    K, G, T = sc.K, sc.G, sc.cfg.T
    gts = observed_forces(pt, sc, dev, solve_precision, warmup + steps)
    u_all = torch.as_tensor(sc.u.astype("float32"), device=dev)
    b = pt.Batch.from_scene(sc, solve_precision=solve_precision)
    cost = torch.zeros(K, device=dev)
    best = torch.zeros(G, dtype=torch.int32, device=dev)
    parent = torch.zeros(K, dtype=torch.int32, device=dev)
    obs = b.new_obs()

    def one(t):
        b.step(u_all[max(t - 1, 0)], u_all[t])
        b.observe(obs)
        b.cost(obs, gts[t], cost, best)
        if (t + 1) % T == 0:
            b.resample(cost, (t + 1) // T - 1, parent)

    for t in range(warmup):
        one(t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(warmup, warmup + steps):
        one(t)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.close()
    return {"value": round(K * steps / wall, 1), "unit": "env-steps/s", "ms_per_step": round(wall / steps * 1e3, 4)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (the population shards across GPUs by "
                                   "simulation; only the one-GPU part is implemented)"}))
        sys.exit(2)
    import numpy as np
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        a = torch.ones(64 * 1024 * 1024, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": a.numel() * 4, "copies": 3}), flush=True)
        return

    from paper_2002_12160_amd import pt
    from paper_2002_12160_amd import scene as S

    dev = torch.device("cuda:0")
    cfg = S.CONFIGS[args.config]
    total_steps = args.warmup + args.steps
    T = cfg.T
    sc = S.make_scene(cfg, steps=max(total_steps, cfg.steps) + 2 * cfg.T + 1)
    K, G, L = sc.K, sc.G, sc.L
    u_all = torch.as_tensor(sc.u.astype(np.float32), device=dev)

    # ---------------- plain per-step path ----------------------------------
    # step, observe, cost against the resident observed forces, argmin; the
    # resampler every T steps
    gts = observed_forces(pt, sc, dev, args.solve_precision, total_steps)
    main_b = pt.Batch.from_scene(sc, solve_precision=args.solve_precision)
    cost = torch.zeros(K, device=dev)
    best = torch.zeros(G, dtype=torch.int32, device=dev)
    parent = torch.zeros(K, dtype=torch.int32, device=dev)
    obs = main_b.new_obs()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    window = 0
    torch.cuda.synchronize()

    def plain_step(t, timed_idx=None):
        nonlocal window
        up, u = u_all[max(t - 1, 0)], u_all[t]
        if timed_idx is not None:
            ev[timed_idx][0].record(stream)
        main_b.step(up, u)
        if timed_idx is not None:
            ev[timed_idx][1].record(stream)
        main_b.observe(obs)
        main_b.cost(obs, gts[t], cost, best)
        if (t + 1) % T == 0:
            main_b.resample(cost, window, parent)
            window += 1

    for t in range(args.warmup):
        plain_step(t)
    torch.cuda.synchronize()
    stats0 = main_b.read_stats()
    t0 = time.perf_counter()
    for i in range(args.steps):
        plain_step(args.warmup + i, i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats1 = main_b.read_stats()
    step_ms = [a.elapsed_time(b) for a, b in ev]
    env_steps = K * args.steps
    plain_value = env_steps / wall
    d_env = stats1["env_steps"] - stats0["env_steps"]
    d_con = stats1["contacts"] - stats0["contacts"]
    d_cand = stats1["candidates"] - stats0["candidates"]
    S_sph = int(sc.n_spheres[0])
    flops = algorithmic_flops(S_sph, L, cfg.newton_iters, d_env, d_con)
    step_kernel_s = sum(step_ms) / 1e3
    achieved_tflops = flops / step_kernel_s / 1e12
    main_b.close()

    result = {
        "metric": "env-steps/sec (step+observe+cost) plain vs batched vs +adjoint, 30Hz budget met",
        "value": round(plain_value, 1),
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.solve_precision == 32 else "f32+f64solve",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {K} simulations + {G} observed, {args.steps} timed steps at "
                               f"{1 / cfg.consts.dt:.0f} Hz, {L} capsule links, {S_sph}-sphere object, "
                               f"C_max={cfg.C_max}, {cfg.newton_iters} Newton iterations, PBO every {T} steps",
                   "path": "plain per-step launches", "solve_precision": args.solve_precision,
                   "observed_forces": "precomputed by the observed simulation, resident in HBM"},
        "per_step_ms": {"p50": round(float(np.median(step_ms)), 4), "p99": round(float(np.quantile(step_ms, 0.99)), 4)},
        "budget_30hz_met": bool(wall / args.steps < 1.0 / 30.0),
        "contacts_per_env_step": round(d_con / max(d_env, 1), 2),
        "candidates_per_env_step": round(d_cand / max(d_env, 1), 2),
        "roofline": {"bound": "alu", "kernel": "k_step (hand kinematics evaluated inside it)",
                     "achieved": round(achieved_tflops, 4), "peak": 78.6,
                     "unit": "TFLOP/s", "frac": None,
                     "traffic": MEASURED_TRAFFIC.get((cfg.name, args.solve_precision)),
                     "flop_per_env_step": round(flops / max(d_env, 1), 1),
                     "hbm_bytes_per_env_step": algorithmic_bytes(cfg.C_max),
                     "hbm_gbps": round(algorithmic_bytes(cfg.C_max) * d_env / step_kernel_s / 1e9, 3),
                     "avg_launch_us": round(step_kernel_s / args.steps * 1e6, 2),
                     "valu": valu_figures((cfg.name, args.solve_precision), step_kernel_s / args.steps, K)},
    }
    result["roofline"]["frac"] = round(result["roofline"]["achieved"] / result["roofline"]["peak"], 6)

    # ---------------- batched path (persistent kernel + graph) -------------
    if not args.no_batched:
        n_win = max(1, args.steps // T)
        n_warm = max(1, args.warmup // T)
        bat = batched_run(pt, S, sc, dev, args.solve_precision, n_win, n_warm, adjoint=False)
        bat["speedup_vs_plain"] = round(bat["value"] / plain_value, 3)
        result["batched"] = bat
        if not args.no_adjoint:
            adj = batched_run(pt, S, sc, dev, args.solve_precision, n_win, n_warm, adjoint=True)
            adj["speedup_vs_plain"] = round(adj["value"] / plain_value, 3)
            result["batched_adjoint"] = adj
            # the differentiation workload: 1024 simulations, 64-sphere cuboid
            acfg = S.CONFIGS["adjoint1024"]
            asc = S.make_scene(acfg, steps=(n_win + n_warm + 2) * acfg.T + 1)
            a_b = batched_run(pt, S, asc, dev, args.solve_precision, n_win, n_warm, adjoint=False)
            a_a = batched_run(pt, S, asc, dev, args.solve_precision, n_win, n_warm, adjoint=True)
            result["adjoint1024"] = {
                "workload": f"{acfg.name}: {asc.K} simulations + {asc.G} observed, {asc.L} capsule links, "
                            f"{int(asc.n_spheres[0])}-sphere cuboid, C_max={acfg.C_max}, "
                            f"{acfg.newton_iters} Newton iterations, {acfg.T}-step windows",
                "batched": a_b, "batched_adjoint": a_a,
                "adjoint_cost_ratio": round(a_b["value"] / a_a["value"], 3)}
            # the batching workload: 4096 simulations of three object
            # types (32-, 64- and 128-sphere), 64-contact cap, plain
            # per-step launches against the persistent kernel + graph
            bcfg = S.CONFIGS["batched4096"]
            bsc = S.make_scene(bcfg, steps=max(total_steps, (n_win + n_warm + 2) * bcfg.T) + 1)
            b_p = plain_run(pt, bsc, dev, args.solve_precision, args.steps, args.warmup)
            b_b = batched_run(pt, S, bsc, dev, args.solve_precision, n_win, n_warm, adjoint=False)
            result["batched4096"] = {
                "workload": f"{bcfg.name}: {bsc.K} simulations + {bsc.G} observed, {bsc.L} capsule links, "
                            f"objects of {sorted(set(int(x) for x in bsc.n_spheres))} spheres, "
                            f"C_max={bcfg.C_max}, {bcfg.newton_iters} Newton iterations, {bcfg.T}-step windows",
                "plain": b_p, "batched": b_b, "speedup_vs_plain": round(b_b["value"] / b_p["value"], 3)}

    # ---------------- real-time workload (16384 simulations) -------------
    if not args.no_batched and not args.no_adjoint and args.realtime_windows > 0:
        n_rt = args.realtime_windows if not args.profile else 3
        rt_setup = realtime_setup(pt, S, dev, args.solve_precision, n_rt + 2)
        result["realtime16384"] = realtime_run(pt, S, dev, args.solve_precision, n_rt, setup=rt_setup,
                                               describe=True)
        if not args.no_optimizers:
            # the paper's other optimisers and its identity baseline on the
            # same workload (Sec. III-D, Sec. IV), same windows and refinement
            result["realtime16384"]["optimizers"] = {
                "wrs": {"lambda": WRS_LAMBDA,
                        **realtime_run(pt, S, dev, args.solve_precision, n_rt, optimizer="wrs", setup=rt_setup)},
                "reps": {"epsilon": REPS_EPS,
                         **realtime_run(pt, S, dev, args.solve_precision, n_rt, optimizer="reps", setup=rt_setup)},
                "eye": realtime_run(pt, S, dev, args.solve_precision, n_rt, optimizer="eye", setup=rt_setup),
                # the cost itself: PBO without refinement (the full cost has no
                # gradient) on the force terms and on the full Eq. 3
                "pbo_no_refinement": realtime_run(pt, S, dev, args.solve_precision, n_rt, setup=rt_setup,
                                                  refine=False)}
            eq3_setup = realtime_setup(pt, S, dev, args.solve_precision, n_rt + 2, cost_mode=1)
            w_eq3 = eq3_weights(pt, eq3_setup, dev, args.solve_precision)
            sc3 = eq3_setup["sc"]
            cfg3 = sc3.cfg.with_(consts=dataclasses.replace(sc3.cfg.consts, w_eq3=w_eq3))
            eq3_setup.update(cfg=cfg3, sc=dataclasses.replace(sc3, cfg=cfg3))
            result["realtime16384"]["optimizers"]["pbo_eq3_cost"] = {
                "w4_w10": [round(x, 4) for x in w_eq3],
                **realtime_run(pt, S, dev, args.solve_precision, n_rt, setup=eq3_setup, refine=False)}

    # ---------------- CPU baseline: the FP64 oracle ----------------------
    if not args.no_cpu_baseline and not args.profile:
        import oracle
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        osc = S.make_scene(cfg, steps=args.cpu_sample_steps + 1)
        tr = oracle.Tracker(osc)
        c0 = time.perf_counter()
        for _ in range(args.cpu_sample_steps):
            tr.step()
        csec = time.perf_counter() - c0
        result["cpu_baseline"] = {"value": round(osc.K * args.cpu_sample_steps / csec, 2), "unit": "env-steps/s",
                                  "cores": nthreads, "kind": "oracle",
                                  "sample": f"first {args.cpu_sample_steps} steps of the same workload, all {osc.K} "
                                            f"simulations + {osc.G} observed, FP64 dense-Newton oracle, "
                                            f"{csec:.1f} s"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
