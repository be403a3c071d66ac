"""Benchmark of the data-parallel hot path of sample-based in-hand pose
tracking on one MI355X.

A "step" is one world step of the whole population with its observation
and cost (Alg. 1: step every simulation with the same command, observe, add
the step cost against the observed contact forces, update the argmin); the
optimiser runs every T = 10 steps.  The observed forces are the tracker's
input (the robot's contact sensors); here they come from a separate batch
holding the unperturbed ("real") simulation of each group stepped with the
same commands, run before any timed region so that, like every other input,
they are resident in HBM when timing starts.  Inputs are seeded and
synthetic (the paper's YCB objects, teleoperation trajectories and hand are
not available).

Headline (`value`): the real-time workload -- 16384 simulations in 16
groups, each group tracking one seeded 128-sphere superquadric held by a
5-finger, 20-link capsule hand, 64-contact cap, 10 Newton iterations -- on
the batched path with adjoint elite refinement: every 10-step window is one
persistent kernel replayed from a captured HIP graph, then the elites of
each group take three gradient steps of their window cost, then the
population-based optimiser resamples.  Timed over the workload's 1800 steps
(60 s at 30 Hz) five times from the same start; `value` is the median.
The same workload also runs the plain per-step launch path and the batched
path without refinement; the other workloads (16, 256, 1024 and 4096
simulations) run the paths their definitions name.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import dataclasses
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "env-steps/sec (step+observe+cost) plain vs batched vs +adjoint, 30Hz budget met"
RUNS = 5
MIN_WINDOWS = 10


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1800,
                    help="timed world steps per run of the headline workload (at least 10 windows are timed)")
    ap.add_argument("--warmup", type=int, default=20, help="untimed world steps before each run")
    ap.add_argument("--runs", type=int, default=RUNS, help="timed runs per leg; the median is reported")
    ap.add_argument("--solve-precision", type=int, default=64, choices=[32, 64])
    ap.add_argument("--no-workloads", action="store_true", help="skip the 16/256/1024/4096-simulation workloads")
    ap.add_argument("--no-optimizers", action="store_true",
                    help="skip the WRS / REPS / identity / full-Eq. 3 comparison on the real-time workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=30)
    ap.add_argument("--profile", action="store_true",
                    help="run for the profiler: one run of the headline leg as timed (batched + refinement), "
                         "nothing else")
    ap.add_argument("--profile-leg", choices=["plain", "pd_hand", "distance_field"],
                    help="run for the profiler: one run of that leg on the real-time workload (the per-step path; "
                         "for the distance field also its batched windows), nothing else")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB on the device three times with the ceiling library's copy kernel "
                         "(reference for the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


# --------------------------------------------------------------------------
# counters from the profiler (profiles/k_window_realtime16384.txt): HBM bytes
# per launch of the headline workload's window kernel (FETCH_SIZE and
# WRITE_SIZE scaled by a plain device copy of known size) and its VALU
# counters.  Keyed by a hash of the kernel's sources: a figure taken before
# the kernel last changed is reported as null.
# --------------------------------------------------------------------------
KERNEL_SOURCES = ("pt_kernels.hip", "pt_step.hpp", "pt_device.hpp", "pt_io.hpp", "pt_internal.h")
MEASURED = {
    # "src": sha256 (first 16 hex digits) of KERNEL_SOURCES, in order;
    # traffic: (FETCH_SIZE x 1.9998 + WRITE_SIZE x 1.0000) KiB x 1024 per launch, the
    # factors from a 256 MiB device copy under the same counters; valu_*:
    # SQ_INSTS_VALU and SQ_ACTIVE_INST_VALU per launch, summed over the chip
    "k_window_realtime16384": {"src": "10211d1d59a9e1e3", "traffic": 404130685,
                               "fetch": 32036583, "write": 372094102,
                               "valu_insts": 2174533529, "valu_busy_quads": 2355665904},
}
SIMDS, CLOCK_HZ = 1024, 2.4e9     # MI355X: 256 CUs x 4 SIMDs at 2.4 GHz; a VALU instruction issues in 4 cycles
PEAK_F64_TFLOPS = 78.6            # MI355X published float64 vector peak (= non-packed float32)
PEAK_HBM_GBPS = 8000.0


def kernel_src_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2002_12160_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured(key):
    m = MEASURED.get(key)
    return m if m is not None and m.get("src") == kernel_src_sha() else None


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


# links against the objects' distance fields: per link sample its point, the
# point in the object frame and the trilinear value less the radius; per
# sphere its height over the table (the field's gradient at the kept
# contacts is not counted, so the figure is a lower bound)
FLOP_SAMPLE = 76
FLOP_TABLE = 7


def algorithmic_flops_sdf(S, L, M, N, env_steps, contacts):
    per_env = FLOP_ENV + FLOP_ENV_PER_LINK * L + S * FLOP_TABLE + L * M * FLOP_SAMPLE + N * FLOP_ENV_ITER
    return env_steps * per_env + contacts * (FLOP_CONTACT + N * FLOP_CONTACT_ITER)


def step_roofline(kernel, flops, env_steps, kernel_us, launches):
    """The ALU roofline of a per-step or window kernel: algorithmic flop per
    launch over its average launch time from HIP events on its stream."""
    per_launch = flops / launches
    achieved = per_launch / (kernel_us * 1e-6) / 1e12
    return {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 3), "peak": PEAK_F64_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_F64_TFLOPS, 4),
            "flop_per_env_step": round(flops / env_steps, 1), "env_steps_per_launch": round(env_steps / launches),
            "avg_launch_us": round(kernel_us, 2)}


def window_bytes(C_max, T, L, obs=False, checkpoints=False):
    """Algorithmic HBM bytes of the window kernel per environment-step: the
    state (13 floats), parameters (5) and warm-start cache (C_max x 16 B)
    read once and written once per window, the observed forces of the group
    (shared, cache resident) and the cost read and written once; with obs,
    the observation rows written every step; with checkpoints (the path with
    elite refinement), the per-step checkpoint the reverse sweep reads: the
    body (64 B) and every contact slot's key and float64 impulse (32 B)."""
    return ((2 * (13 + 5) * 4 + 2 * 16 * C_max + 8) / T + (16 * L if obs else 0)
            + (64 + 32 * C_max if checkpoints else 0))


def median_run(runs):
    """The run with the median value (odd counts) and the list of values."""
    vals = sorted(r["value"] for r in runs)
    mid = vals[len(vals) // 2]
    pick = next(r for r in runs if r["value"] == mid)
    return dict(pick, runs=[round(r["value"], 1) for r in runs])


# --------------------------------------------------------------------------
# inputs
# --------------------------------------------------------------------------

def observed_forces(pt, sc, dev, solve_precision, n_steps, pose_every=None):
    """The observed ("real") simulation's sensor forces for steps
    0..n_steps-1, [n_steps][R][L][G] (R = 4, or 7 under the full cost of
    Eq. 3): the tracker's input stream, produced before any timed region and
    resident in HBM.  With pose_every = T also the observed object's state
    after every T steps ([n_steps / T][13][G], for the tracking error)."""
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


def make_setup(pt, S, dev, solve_precision, cfg, n_windows):
    """Scene, observed forces, observed poses and commands for n_windows
    windows of a workload (plus one window of slack)."""
    import torch
    T = cfg.T
    sc = S.make_scene(cfg, steps=(n_windows + 1) * T + 1)
    gts, hposes = observed_forces(pt, sc, dev, solve_precision, n_windows * T, pose_every=T)
    u_all = torch.as_tensor(sc.u.astype("float32"), device=dev)
    return {"cfg": cfg, "sc": sc, "gts": gts, "hposes": hposes, "u_all": u_all}


def add_distance(points, pa, pb):
    """Mean distance between the object's points placed at poses pa and pb
    (x(3), q(4)): the tracking error of a pose estimate (ADD, Sec. IV)."""
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


# --------------------------------------------------------------------------
# the paths
# --------------------------------------------------------------------------

def windows_run(pt, setup, dev, solve_precision, n_win, n_warm, optimizer="pbo", refine=True):
    """Batched windows of a workload: each window's commands and observed
    forces are copied into the two buffers a captured HIP graph reads, the
    population's window is one persistent kernel replayed from that graph,
    then (refine) the elites are refined by three gradient steps of the
    window cost from their window start, then the optimiser resamples
    ("pbo", "wrs", "reps"; "eye" neither refines nor resamples).  Reports
    env-steps/s over the timed windows, the per-step latency (window time /
    T), the resampler's time, the window kernel's HIP-event time and
    algorithmic flop, and the tracking error after every window."""
    import numpy as np
    import torch
    cfg, sc, gts, u_all = setup["cfg"], setup["sc"], setup["gts"], setup["u_all"]
    T = cfg.T
    K, G, L = sc.K, sc.G, sc.L
    adapt = optimizer != "eye"
    refine = refine and adapt
    n_total = n_warm + n_win
    assert n_total * T <= gts.shape[0]
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
    mk = lambda: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))  # noqa: E731
    ev, ev_rs, ev_win = [mk() for _ in range(n_total)], [mk() for _ in range(n_total)], [mk() for _ in range(n_total)]
    improved = [0, 0]

    def window(w, count=False):
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
            c0 = cost.clone() if count else None
            elites = b.refine_elites(u_win, gt_win, cost, snap, steps=3, step=0.5, best=best)
            if count:
                e = elites.long()
                improved[0] += int((cost[e] < c0[e]).sum())
                improved[1] += int(e.numel())
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
        window(w, count=refine and w == n_warm - 1)
    torch.cuda.synchronize()
    stats0 = b.read_stats()
    t0 = time.perf_counter()
    for w in range(n_warm, n_total):
        window(w)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats1 = b.read_stats()
    step_ms = np.array([ev[w][0].elapsed_time(ev[w][1]) / T for w in range(n_warm, n_total)])
    win_ms = np.array([ev_win[w][0].elapsed_time(ev_win[w][1]) for w in range(n_warm, n_total)])
    rs_ms = np.array([ev_rs[w][0].elapsed_time(ev_rs[w][1]) for w in range(n_warm, n_total)])
    # the population's window (graph replay of the persistent k_window; the
    # refinement's own replays do not count their steps in the statistics)
    d_env = stats1["env_steps"] - stats0["env_steps"]
    d_con = stats1["contacts"] - stats0["contacts"]
    if cfg.consts.collision_mode == 1:
        flops = algorithmic_flops_sdf(int(sc.n_spheres.max()), L, cfg.consts.link_samples, cfg.newton_iters, d_env,
                                      d_con)
    else:
        flops = algorithmic_flops(int(sc.n_spheres.max()), L, cfg.newton_iters, d_env, d_con)
    hp = setup["hposes"].cpu().numpy()

    # windows in which the observed object touches a sensor at all (touch is
    # the tracker's only information: an object that left the hand cannot
    # be followed)
    fo = gts[:n_total * T, 0].sum(dim=1).reshape(n_total, T, G).amax(dim=1).cpu().numpy()
    touching = fo > 0.0

    def tracking(e):
        errs, errs_t = [], []
        for w in range(n_warm, n_total):
            for g in range(G):
                pts = sc.spheres[sc.hidden_type[g], :sc.n_spheres[sc.hidden_type[g]], :3]
                d = add_distance(pts, e[w, :7, g], hp[w, :7, g])
                errs.append(d)
                if touching[w, g]:
                    errs_t.append(d)
        out = {"mean": round(1e3 * float(np.mean(errs)), 3), "p90": round(1e3 * float(np.quantile(errs, 0.9)), 3)}
        if errs_t:
            out["touching"] = {"mean": round(1e3 * float(np.mean(errs_t)), 3),
                               "p90": round(1e3 * float(np.quantile(errs_t, 0.9)), 3),
                               "windows_frac": round(len(errs_t) / len(errs), 3)}
        return out

    n_elite = b.elite_count()
    b.close()
    out = {"value": K * T * n_win / wall, "unit": "env-steps/s", "windows": n_win,
           "ms_per_step": round(wall / (n_win * T) * 1e3, 4),
           "per_step_ms": {"p50": round(float(np.median(step_ms)), 4),
                           "p99": round(float(np.quantile(step_ms, 0.99)), 4)},
           "budget_30hz_met": bool(np.quantile(step_ms, 0.99) < 1000.0 / 30.0),
           "resample_ms_per_window": round(float(np.median(rs_ms)), 4),
           "tracking_error_mm": tracking(est.cpu().numpy()),
           "waves_per_workgroup": tuned,
           "window_kernel": {"avg_launch_us": round(float(win_ms.mean()) * 1e3, 2),
                             "flop_per_launch": flops / n_win, "env_steps_per_launch": d_env / n_win,
                             "contacts_per_env_step": round(d_con / max(d_env, 1), 2)}}
    if refine:
        out.update({"elites": n_elite, "refine_steps": 3,
                    "elites_improved_frac": round(improved[0] / max(improved[1], 1), 3)})
    if not adapt:
        out["open_loop_tracking_error_mm"] = tracking(est_olp.cpu().numpy())
    return out


def plain_run(pt, setup, dev, solve_precision, steps, warmup):
    """The plain per-step launch path: step, observe, cost with the argmin,
    the resampler every T steps; env-steps/s over `steps` timed steps after
    `warmup`, and the per-step latency of step + observe + cost (HIP events
    on the stream)."""
    import numpy as np
    import torch
    cfg, sc, gts, u_all = setup["cfg"], setup["sc"], setup["gts"], setup["u_all"]
    K, G, T = sc.K, sc.G, cfg.T
    assert warmup + steps <= gts.shape[0]
    b = pt.Batch.from_scene(sc, solve_precision=solve_precision)
    cost = torch.zeros(K, device=dev)
    best = torch.zeros(G, dtype=torch.int32, device=dev)
    parent = torch.zeros(K, dtype=torch.int32, device=dev)
    obs = b.new_obs()
    mk = lambda: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))  # noqa: E731
    ev, ev_k = [mk() for _ in range(steps)], [mk() for _ in range(steps)]

    def one(t, i=None):
        if i is not None:
            ev[i][0].record()
            ev_k[i][0].record()
        b.step(u_all[max(t - 1, 0)], u_all[t])
        if i is not None:
            ev_k[i][1].record()
        b.observe(obs)
        b.cost(obs, gts[t], cost, best)
        if i is not None:
            ev[i][1].record()
        if (t + 1) % T == 0:
            b.resample(cost, (t + 1) // T - 1, parent)

    for t in range(warmup):
        one(t)
    torch.cuda.synchronize()
    stats0 = b.read_stats()
    t0 = time.perf_counter()
    for i in range(steps):
        one(warmup + i, i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats1 = b.read_stats()
    b.close()
    step_ms = np.array([a.elapsed_time(c) for a, c in ev])
    kernel_us = 1e3 * float(np.mean([a.elapsed_time(c) for a, c in ev_k]))
    d_env = stats1["env_steps"] - stats0["env_steps"]
    d_con = stats1["contacts"] - stats0["contacts"]
    c = cfg.consts
    if c.collision_mode == 1:
        flops = algorithmic_flops_sdf(int(sc.n_spheres.max()), sc.L, c.link_samples, cfg.newton_iters, d_env, d_con)
    else:
        flops = algorithmic_flops(int(sc.n_spheres.max()), sc.L, cfg.newton_iters, d_env, d_con)
    return {"value": K * steps / wall, "unit": "env-steps/s", "steps": steps,
            "ms_per_step": round(wall / steps * 1e3, 4),
            "per_step_ms": {"p50": round(float(np.median(step_ms)), 4),
                            "p99": round(float(np.quantile(step_ms, 0.99)), 4)},
            "budget_30hz_met": bool(np.quantile(step_ms, 0.99) < 1000.0 / 30.0),
            "contacts_per_env_step": round(d_con / max(d_env, 1), 2),
            "step_kernel": {"avg_launch_us": round(kernel_us, 2), "flops": flops, "env_steps": d_env,
                            "launches": steps}}


def pd_run(pt, S, dev, cfg, steps, warmup, batched=False):
    """The PD-controlled hand: the observed simulations' forces and joint
    angles first (resident in HBM), then on the plain per-step path step,
    observe, cost with the argmin and the resampler every T steps, timed as
    plain_run; or (batched) one window call per T steps (the window kernel
    replayed from its graph, with the argmin) and the resampler, timed per
    window."""
    import numpy as np
    import torch
    cfg = cfg.with_(consts=dataclasses.replace(cfg.consts, hand_mode=1))
    sc = S.make_scene(cfg, steps=warmup + steps + 1)
    K, G, T, D = sc.K, sc.G, cfg.T, sc.D
    u_all = torch.as_tensor(sc.u.astype("float32"), device=dev)
    rest = np.concatenate([sc.u[0], np.zeros(D)])
    h = pt.Batch.from_scene(sc, hidden=True, hand_state=np.tile(rest, (G, 1)))
    gts = torch.empty((warmup + steps,) + h.obs_shape(G), device=dev)
    for t in range(warmup + steps):
        h.step(None, u_all[t])
        h.observe(gts[t])
    torch.cuda.synchronize()
    h.close()
    b = pt.Batch.from_scene(sc, hand_state=np.tile(rest, (K, 1)))
    cost = torch.zeros(K, device=dev)
    best = torch.zeros(G, dtype=torch.int32, device=dev)
    parent = torch.zeros(K, dtype=torch.int32, device=dev)
    obs = b.new_obs()
    if batched:
        assert steps % T == 0 and warmup % T == 0
        u_win = torch.empty((T + 1, D), device=dev)
        gt_win = torch.empty((T,) + h.obs_shape(G), device=dev)
        n_ev = steps // T
    else:
        n_ev = steps
    mk = lambda: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))  # noqa: E731
    ev, ev_k = [mk() for _ in range(n_ev)], [mk() for _ in range(n_ev)]

    def one(t, i=None):
        if i is not None:
            ev[i][0].record()
            ev_k[i][0].record()
        b.step(None, u_all[t])
        if i is not None:
            ev_k[i][1].record()
        b.observe(obs)
        b.cost(obs, gts[t], cost, best)
        if i is not None:
            ev[i][1].record()
        if (t + 1) % T == 0:
            b.resample(cost, (t + 1) // T - 1, parent)

    def window(w, i=None):
        t0_ = w * T
        u_win.copy_(u_all[t0_ - 1: t0_ + T] if t0_ > 0 else torch.cat([u_all[:1], u_all[:T]], 0))
        gt_win.copy_(gts[t0_: t0_ + T])
        if i is not None:
            ev[i][0].record()
        b.run_window(u_win, gt_win, cost, best, None, graph=True)
        if i is not None:
            ev[i][1].record()
        b.resample(cost, w, parent)

    if batched:
        for w in range(warmup // T):
            window(w)
    else:
        for t in range(warmup):
            one(t)
    torch.cuda.synchronize()
    stats0 = b.read_stats()
    t0 = time.perf_counter()
    if batched:
        for i in range(n_ev):
            window(warmup // T + i, i)
    else:
        for i in range(steps):
            one(warmup + i, i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats1 = b.read_stats()
    b.close()
    step_ms = np.array([a.elapsed_time(c) for a, c in ev]) / (T if batched else 1)
    d_env = stats1["env_steps"] - stats0["env_steps"]
    d_con = stats1["contacts"] - stats0["contacts"]
    out = {"value": K * steps / wall, "unit": "env-steps/s", "steps": steps,
           "ms_per_step": round(wall / steps * 1e3, 4),
           "per_step_ms": {"p50": round(float(np.median(step_ms)), 4),
                           "p99": round(float(np.quantile(step_ms, 0.99)), 4)},
           "contacts_per_env_step": round(d_con / max(d_env, 1), 2)}
    if not batched:
        # the kinematic step's arithmetic only (the PD step does all of it,
        # plus the hand's kinematics, mass matrix, hand blocks and group
        # eliminations, not counted): a lower bound
        c = cfg.consts
        flops = (algorithmic_flops_sdf(int(sc.n_spheres.max()), sc.L, c.link_samples, cfg.newton_iters, d_env, d_con)
                 if c.collision_mode == 1 else
                 algorithmic_flops(int(sc.n_spheres.max()), sc.L, cfg.newton_iters, d_env, d_con))
        out["step_kernel"] = {"avg_launch_us": round(1e3 * float(np.mean([a.elapsed_time(c_) for a, c_ in ev_k])), 2),
                              "flops": flops, "env_steps": d_env, "launches": steps}
    return out


def repeat(fn, runs):
    return median_run([fn() for _ in range(runs)])


def rounded(d):
    d = dict(d)
    d["value"] = round(d["value"], 1)
    return d


# --------------------------------------------------------------------------
# ceilings, CPU baseline
# --------------------------------------------------------------------------

def ceilings(dev):
    """Measured float64 FMA rate and HBM copy bandwidth of this device (the
    ceiling library's microbenchmarks), best of five."""
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2002_12160_amd", "libptceil.so"))
    lib.ptc_fma_f64.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    lib.ptc_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    blocks, iters = n_cu * 16, 8192
    out = torch.empty(blocks * 256, dtype=torch.float64, device=dev)
    flop = 2.0 * lib.ptc_fma_chains() * iters * blocks * 256
    best_fma = 0.0
    for _ in range(6):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        assert lib.ptc_fma_f64(ctypes.c_void_p(out.data_ptr()), blocks, iters, stream) == 0
        b.record()
        torch.cuda.synchronize()
        best_fma = max(best_fma, flop / (a.elapsed_time(b) * 1e-3) / 1e12)
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    best_copy = 0.0
    for _ in range(6):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        assert lib.ptc_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes, n_cu * 8,
                            stream) == 0
        b.record()
        torch.cuda.synchronize()
        best_copy = max(best_copy, 2.0 * nbytes / (a.elapsed_time(b) * 1e-3) / 1e9)
    del src, dst, out
    return {"fma_f64_tflops": round(best_fma, 2), "fma_f64_nominal_tflops": PEAK_F64_TFLOPS,
            "copy_gbps": round(best_copy, 1), "copy_gbps_nominal": PEAK_HBM_GBPS,
            "how": "float64 FMA loop (8 independent chains per thread, 16 workgroups of 256 threads per compute "
                   "unit) and a 1 GiB device-to-device copy (read + write bytes), best of 6"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(S, cfg, steps):
    """The FP64 oracle on a stratified sample of the headline workload:
    sims_per_group simulations of every group (every object) from the start,
    stepped with the observation and the cost against the observed
    simulations; env-steps/s counts the sampled simulations only.  The
    oracle's cost per simulation does not depend on the population size, so
    the rate applies to the full population (a linear extrapolation in K).
    Timed on all the host threads OpenMP uses, then on one thread."""
    import numpy as np
    import oracle
    sims_per_group = 16
    full = S.make_scene(cfg, steps=steps + 1)
    idx = np.concatenate([np.arange(full.group_start[g], full.group_start[g] + sims_per_group)
                          for g in range(full.G)])
    gs = np.arange(0, len(idx) + 1, sims_per_group, dtype=np.int32)
    sub = dataclasses.replace(full, env_type=np.ascontiguousarray(full.env_type[idx]), group_start=gs,
                              state=np.ascontiguousarray(full.state[idx]), params=np.ascontiguousarray(full.params[idx]))
    res = {}
    threads_all = oracle.max_threads()
    for label, threads, n_steps, n_sim in (("all", threads_all, steps, len(idx)), ("one", 1, max(steps // 5, 4), 32)):
        oracle.set_threads(threads)
        pick = np.arange(0, len(idx), len(idx) // n_sim)[:n_sim]
        s2 = sub if n_sim == len(idx) else dataclasses.replace(
            sub, env_type=np.ascontiguousarray(sub.env_type[pick]), state=np.ascontiguousarray(sub.state[pick]),
            params=np.ascontiguousarray(sub.params[pick]),
            group_start=np.arange(0, n_sim + 1, n_sim // full.G, dtype=np.int32))
        tr = oracle.Tracker(s2)
        c0 = time.perf_counter()
        for _ in range(n_steps):
            tr.step()
        sec = time.perf_counter() - c0
        res[label] = (s2.K * n_steps / sec, threads, s2.K, n_steps, sec)
    oracle.set_threads(threads_all)
    v, thr, k, n, sec = res["all"]
    v1, _, k1, n1, sec1 = res["one"]
    return {"value": round(v, 1), "unit": "env-steps/s", "cores": thr, "kind": "oracle",
            "sample": f"{k} simulations ({sims_per_group} of each of the {full.G} groups) of {cfg.name} for {n} steps "
                      f"from the start, with the {full.G} observed simulations, observation, cost and the resampler "
                      f"every {cfg.T} steps; FP64 dense-Newton oracle, {sec:.1f} s on {thr} threads; the rate per "
                      f"simulation does not depend on K (linear extrapolation to {full.K})",
            "cpu_model": cpu_model(), "one_thread": {"value": round(v1, 1), "simulations": k1, "steps": n1,
                                                     "seconds": round(sec1, 1)}}


# --------------------------------------------------------------------------
# Eq. 3 weights (full-cost comparison leg)
# --------------------------------------------------------------------------

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
    b.run_window(torch.cat([u_all[:1], u_all[:T]], 0).contiguous(), gts[:T].contiguous(), torch.zeros(K, device=dev),
                 None, obs_w, graph=False)
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


# --------------------------------------------------------------------------

def describe(cfg, sc):
    objs = sorted(set(int(x) for x in sc.n_spheres))
    kind = cfg.objects[0].kind
    return (f"{cfg.name}: {sc.K} simulations in {sc.G} group{'s' if sc.G > 1 else ''} + {sc.G} observed, "
            f"{sc.L} capsule links, {'/'.join(map(str, objs))}-sphere {kind} object{'s' if len(objs) > 1 else ''}, "
            f"C_max={cfg.C_max}, {cfg.newton_iters} Newton iterations, {cfg.T}-step windows")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (the population shards across GPUs by "
                                   "simulation; only the one-GPU part is implemented)"}))
        sys.exit(2)
    import numpy as np
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        lib = ctypes.CDLL(os.path.join(ROOT, "paper_2002_12160_amd", "libptceil.so"))
        lib.ptc_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
        nbytes = 256 << 20
        a = torch.ones(nbytes // 4, device=dev)
        b = torch.empty_like(a)
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        for _ in range(3):
            assert lib.ptc_copy(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), nbytes, 2048, s) == 0
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 3}), flush=True)
        return

    from paper_2002_12160_amd import pt
    from paper_2002_12160_amd import scene as S

    sp = args.solve_precision
    cfg = S.CONFIGS["realtime16384"]
    T = cfg.T
    n_win = max(MIN_WINDOWS, -(-args.steps // T))
    n_warm = max(1, -(-args.warmup // T))
    if args.profile_leg:
        steps = min(n_win * T, 300)
        if args.profile_leg == "plain":
            psetup = make_setup(pt, S, dev, sp, cfg, n_warm + -(-steps // T))
            r = plain_run(pt, psetup, dev, sp, steps, n_warm * T)
            sk = r.pop("step_kernel")
            r["roofline"] = step_roofline("k_hand_fk + k_step<double, false, false, true>", sk["flops"],
                                          sk["env_steps"], sk["avg_launch_us"], sk["launches"])
        elif args.profile_leg == "pd_hand":
            r = pd_run(pt, S, dev, cfg, steps, n_warm * T)
            sk = r.pop("step_kernel")
            r["roofline"] = step_roofline("k_step_pd", sk["flops"], sk["env_steps"], sk["avg_launch_us"],
                                          sk["launches"])
        else:
            scfg = cfg.with_(consts=dataclasses.replace(cfg.consts, collision_mode=1))
            nw = -(-steps // T)
            ssetup = make_setup(pt, S, dev, sp, scfg, n_warm + nw)
            r = plain_run(pt, ssetup, dev, sp, steps, n_warm * T)
            sk = r.pop("step_kernel")
            r["roofline"] = step_roofline("k_hand_fk + k_step<double, false, true, true>", sk["flops"], sk["env_steps"],
                                          sk["avg_launch_us"], sk["launches"])
            rb = windows_run(pt, ssetup, dev, sp, nw, n_warm, refine=False)
            wk = rb["window_kernel"]
            r["batched_roofline"] = step_roofline("k_window<double, false, false, true>", wk["flop_per_launch"] * nw,
                                                  wk["env_steps_per_launch"] * nw, wk["avg_launch_us"], nw)
        print(json.dumps({"leg": args.profile_leg, **rounded(r)}), flush=True)
        return
    runs = 1 if args.profile else args.runs
    print(f"bench: headline {cfg.name}, {runs} runs of {n_win} windows after {n_warm}", file=sys.stderr, flush=True)
    setup = make_setup(pt, S, dev, sp, cfg, n_warm + n_win)
    head = repeat(lambda: windows_run(pt, setup, dev, sp, n_win, n_warm), runs)
    print(f"bench: headline {head['value']:.4g} env-steps/s", file=sys.stderr, flush=True)
    sc = setup["sc"]
    K, G, L = sc.K, sc.G, sc.L
    wk = head["window_kernel"]
    achieved = wk["flop_per_launch"] / (wk["avg_launch_us"] * 1e-6) / 1e12
    m = measured("k_window_realtime16384")
    launch_s = wk["avg_launch_us"] * 1e-6
    roofline = {"bound": "alu", "kernel": "k_window (float64 solve; the 10-step window of all 16384 simulations)",
                "achieved": round(achieved, 3), "peak": PEAK_F64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_F64_TFLOPS, 4),
                "traffic": m["traffic"] if m else None,
                "flop_per_env_step": round(wk["flop_per_launch"] / wk["env_steps_per_launch"], 1),
                "env_steps_per_launch": int(wk["env_steps_per_launch"]),
                "avg_launch_us": wk["avg_launch_us"],
                "hbm_bytes_per_env_step": round(window_bytes(cfg.C_max, T, L, checkpoints=True), 1),
                "hbm_bytes_per_launch": round(window_bytes(cfg.C_max, T, L, checkpoints=True) *
                                              wk["env_steps_per_launch"]),
                "hbm_gbps": round(window_bytes(cfg.C_max, T, L, checkpoints=True) * wk["env_steps_per_launch"] /
                                  launch_s / 1e9, 2),
                "valu": ({"issue_frac": round(m["valu_insts"] * 4 / (SIMDS * CLOCK_HZ * launch_s), 4),
                          "busy_frac": round(m["valu_busy_quads"] * 4 / (SIMDS * CLOCK_HZ * launch_s), 4)}
                         if m else None)}
    result = {
        "metric": METRIC,
        "value": round(head["value"], 1),
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": n_win * T,
        "warmup": n_warm * T,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if sp == 32 else "f32+f64solve",
        "data": "synthetic",
        "config": {"workload": describe(cfg, sc) + f", {n_win * T} timed steps ({n_win * T / 30:.0f} s at 30 Hz)",
                   "path": "batched: persistent window kernel replayed from a HIP graph, then adjoint refinement of "
                           "the elites (3 gradient steps), then PBO resampling, every window",
                   "runs": runs, "steps_requested": args.steps,
                   "observed_forces": "precomputed by the observed simulations, resident in HBM"},
        "per_step_ms": head["per_step_ms"],
        "budget_30hz_met": head["budget_30hz_met"],
        "tracking_error_mm": head["tracking_error_mm"],
        "runs": head["runs"],
        "roofline": roofline,
    }
    if args.profile:
        print(json.dumps(result), flush=True)
        return

    # the other two paths on the same workload
    plain_steps = min(n_win * T, 300)
    plain = repeat(lambda: plain_run(pt, setup, dev, sp, plain_steps, n_warm * T), runs)
    print(f"bench: plain {plain['value']:.4g}", file=sys.stderr, flush=True)
    batched = repeat(lambda: windows_run(pt, setup, dev, sp, n_win, n_warm, refine=False), runs)
    print(f"bench: batched {batched['value']:.4g}", file=sys.stderr, flush=True)
    pv = plain["value"]
    sk, wk = plain.pop("step_kernel"), batched.pop("window_kernel")
    plain["roofline"] = step_roofline("k_hand_fk + k_step<double, false, false, true> (one step of every simulation)",
                                      sk["flops"], sk["env_steps"], sk["avg_launch_us"], sk["launches"])
    batched["roofline"] = step_roofline("k_window<double, false, false, false> (the window, no checkpoints)",
                                        wk["flop_per_launch"], wk["env_steps_per_launch"], wk["avg_launch_us"], 1)
    batched["contacts_per_env_step"] = wk["contacts_per_env_step"]
    result["paths"] = {
        "plain": rounded(plain),
        "batched": dict(rounded(batched), speedup_vs_plain=round(batched["value"] / pv, 3)),
        "batched_adjoint": {"value": result["value"], "speedup_vs_plain": round(head["value"] / pv, 3),
                            "vs_batched": round(head["value"] / batched["value"], 3),
                            "resample_ms_per_window": head["resample_ms_per_window"],
                            "elites_improved_frac": head.get("elites_improved_frac")},
    }
    result["ceilings"] = ceilings(dev)
    result["roofline"]["frac_of_measured_fma"] = round(achieved / result["ceilings"]["fma_f64_tflops"], 4)

    # the PD-controlled hand (joint state per simulation) on the plain path
    if not args.no_workloads:
        pd = {}
        for name in ("realtime16384", "small"):
            wcfg = S.CONFIGS[name]
            keys = ("value", "unit", "steps", "ms_per_step", "per_step_ms", "contacts_per_env_step", "runs")
            r = repeat(lambda: pd_run(pt, S, dev, wcfg, min(n_win * T, 300), n_warm * T), runs)
            pd[name] = rounded({k: r[k] for k in keys if k in r})
            sk = r["step_kernel"]
            pd[name]["roofline"] = step_roofline(
                "k_step_pd (one PD step of every simulation; flop of the kinematic step only, a lower bound)",
                sk["flops"], sk["env_steps"], sk["avg_launch_us"], sk["launches"])
            r = repeat(lambda: pd_run(pt, S, dev, wcfg, min(n_win * T, 300), n_warm * T, batched=True), runs)
            pd[name + "_batched"] = rounded({k: r[k] for k in keys if k in r})
            pd[name + "_batched_vs_plain"] = round(pd[name + "_batched"]["value"] / pd[name]["value"], 3)
        pd["path"] = ("the PD-controlled hand: plain per-step path (step: hand kinematics, mass matrix and the "
                      "(6 + D) contact solve per simulation; observe: forces and joint angles; cost with the "
                      "joint term) and batched windows (the T steps of a simulation, its observations and costs in "
                      "one wavefront, replayed from a HIP graph), PBO resampling every window")
        if not args.no_cpu_baseline:
            pd["cpu_baseline"] = cpu_baseline(S, cfg.with_(consts=dataclasses.replace(cfg.consts, hand_mode=1)), 10)
        result["pd_hand"] = pd
        print("bench: PD hand done", file=sys.stderr, flush=True)
        # links against the objects' signed distance fields (32^3 grids, 8 samples per link)
        scfg = cfg.with_(consts=dataclasses.replace(cfg.consts, collision_mode=1))
        n_sdf = min(n_win * T, 300)
        ssetup = make_setup(pt, S, dev, sp, scfg, n_warm + -(-n_sdf // T))
        r = repeat(lambda: plain_run(pt, ssetup, dev, sp, n_sdf, n_warm * T), runs)
        sw = -(-n_sdf // T)
        rb = repeat(lambda: windows_run(pt, ssetup, dev, sp, sw, n_warm, refine=False), runs)
        result["distance_field"] = {
            "path": "the links tested at 8 points each against the objects' signed distance fields (32^3 grids, "
                    "trilinear) instead of the sphere sets: the plain per-step path, and the batched windows "
                    "with PBO resampling",
            "realtime16384": rounded({k: r[k] for k in ("value", "unit", "steps", "ms_per_step", "per_step_ms",
                                                        "contacts_per_env_step", "runs") if k in r}),
            "realtime16384_batched": rounded({k: rb[k] for k in ("value", "unit", "windows", "ms_per_step",
                                                                 "per_step_ms", "tracking_error_mm",
                                                                 "waves_per_workgroup", "runs") if k in rb}),
            "roofline": {
                "plain": step_roofline("k_hand_fk + k_step<double, false, true, true> (one step of every simulation)",
                                       r["step_kernel"]["flops"], r["step_kernel"]["env_steps"],
                                       r["step_kernel"]["avg_launch_us"], r["step_kernel"]["launches"]),
                "batched": step_roofline("k_window<double, false, false, true> (the 10-step window)",
                                         rb["window_kernel"]["flop_per_launch"] * sw,
                                         rb["window_kernel"]["env_steps_per_launch"] * sw,
                                         rb["window_kernel"]["avg_launch_us"], sw)},
            "vs_sphere_set_plain": round(r["value"] / plain["value"], 3),
            "batched_vs_sphere_set_batched": round(rb["value"] / batched["value"], 3)}
        if not args.no_cpu_baseline:
            result["distance_field"]["cpu_baseline"] = cpu_baseline(S, scfg, 10)
        print("bench: distance field done", file=sys.stderr, flush=True)

    # the other workloads, the paths their definitions name
    if not args.no_workloads:
        wl = {}
        for name, paths in (("small", ("plain", "batched")), ("plain256", ("plain", "batched", "batched_adjoint")),
                            ("batched4096", ("plain", "batched")), ("adjoint1024", ("batched", "batched_adjoint"))):
            wcfg = S.CONFIGS[name]
            nw = MIN_WINDOWS * 3
            wsetup = make_setup(pt, S, dev, sp, wcfg, n_warm + nw)
            entry = {"workload": describe(wcfg, wsetup["sc"])}
            for p in paths:
                if p == "plain":
                    r = repeat(lambda: plain_run(pt, wsetup, dev, sp, nw * wcfg.T, n_warm * wcfg.T), runs)
                else:
                    r = repeat(lambda: windows_run(pt, wsetup, dev, sp, nw, n_warm, refine=p == "batched_adjoint"),
                               runs)
                keep = {k: r[k] for k in ("value", "unit", "ms_per_step", "per_step_ms", "runs", "waves_per_workgroup",
                                          "elites_improved_frac") if k in r}
                entry[p] = rounded(keep)
            if "plain" in entry:
                for p in ("batched", "batched_adjoint"):
                    if p in entry:
                        entry[p]["speedup_vs_plain"] = round(entry[p]["value"] / entry["plain"]["value"], 3)
            wl[name] = entry
            print(f"bench: {name} done", file=sys.stderr, flush=True)
        result["workloads"] = wl

    # the paper's other optimisers, its identity baseline and the full cost
    # on the real-time workload (same windows; tracking error is the point)
    if not args.no_optimizers:
        opt = {
            "wrs": {"lambda": WRS_LAMBDA, **windows_run(pt, setup, dev, sp, n_win, n_warm, optimizer="wrs")},
            "reps": {"epsilon": REPS_EPS, **windows_run(pt, setup, dev, sp, n_win, n_warm, optimizer="reps")},
            "eye": windows_run(pt, setup, dev, sp, n_win, n_warm, optimizer="eye"),
            "pbo_no_refinement": batched,
        }
        cfg3 = cfg.with_(consts=dataclasses.replace(cfg.consts, cost_mode=1))
        eq3_setup = make_setup(pt, S, dev, sp, cfg3, n_warm + n_win)
        w_eq3 = eq3_weights(pt, eq3_setup, dev, sp)
        cfg3 = cfg3.with_(consts=dataclasses.replace(cfg3.consts, w_eq3=w_eq3))
        eq3_setup.update(cfg=cfg3, sc=dataclasses.replace(eq3_setup["sc"], cfg=cfg3))
        opt["pbo_eq3_cost"] = {"w4_w10": [round(x, 4) for x in w_eq3],
                               **windows_run(pt, eq3_setup, dev, sp, n_win, n_warm, refine=False)}
        keep = ("lambda", "epsilon", "w4_w10", "value", "tracking_error_mm", "open_loop_tracking_error_mm",
                "resample_ms_per_window", "per_step_ms")
        result["optimizers"] = {k: rounded({x: v[x] for x in keep if x in v}) for k, v in opt.items()}
        print("bench: optimizers done", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(S, cfg, args.cpu_sample_steps)
    result["context"] = ("the paper's only throughput figure: about 30 Hz with 40 simulations on one GTX 1080 Ti "
                         "(about 1200 env-steps/s, Sec. IV-A), another machine and another simulator")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
