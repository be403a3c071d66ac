"""Helpers for GPU-vs-oracle parity (test infrastructure).

Tolerance (GPU vs the FP64 oracle run from the same float32-rounded inputs):
|a - b| <= 1e-4 * max(|b|, floor) per state component with floors 2 cm
(position), 1 (quaternion), 0.1 m/s (velocity), 1 rad/s (angular velocity);
a sensor's force to 1e-4 of max(|c_l|, m g) (m g: the object's weight), its
direction to the matching angle where the oracle's force is clear of the
contact threshold.

Where the rule applies.  The step map is piecewise smooth: the solve runs a
fixed number of Newton iterations whose Armijo decisions, the contact cap,
the candidate margin and the tangent-axis choice are discrete, and a fixed-N
solve far from convergence can also amplify rounding-level changes of its
inputs.  The GPU holds the geometry in float32, so its result is the
oracle's result for float32-rounded geometry; where that rounding moves the
result by more than rounding, no implementation can meet a 1e-4 bar.  A step
of one simulation is therefore *clear* -- and parity is asserted there with
no exceptions -- when all of these hold:
  1. the oracle from the double-precision state and from its float32-rounded
     copy agree to 1e-6 with identical contact sets (the reading's rule);
  2. two probes of float32 geometry -- every geometric value rounded to the
     nearest float32, and rounded then moved one float32 step by a hash of
     its bits -- move the state and the observation by at most a tenth of the
     tolerance, with identical contact sets;
  3. no decision is near its threshold: every Armijo trial whose outcome
     matters clears its bound by at least ARMIJO_BAND of the merit, no two
     gaps at the cap's boundary are closer than GAP_BAND, no gap is within
     GAP_BAND of the margin, and no sphere-link contact normal has its two
     smallest components within TANGENT_BAND.
At a cap tie alone (condition 3's cap clause) either choice is a correct
contact set: the sets must then agree up to the tied candidates.
"""
import numpy as np

import oracle

FLOORS = np.array([0.02] * 3 + [1.0] * 4 + [0.1] * 3 + [1.0] * 3)
TOL = 1e-4
CHAOS_TOL = 1e-6
PROBE_TOL = 1e-5
G = 9.81
ARMIJO_BAND = 1e-3
GAP_BAND = 1e-7
TANGENT_BAND = 1e-6
CAP_TIE = GAP_BAND


def rel_err(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), FLOORS)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def key_sets(wkey):
    return [frozenset(int(k) for k in row if k >= 0) for row in wkey]


def same_keys(ka, kb):
    return np.array([x == y for x, y in zip(key_sets(ka), key_sets(kb))])


def cap_tie(diag):
    return (diag["d_first_dropped"] - diag["d_last_kept"]) < CAP_TIE


def keys_match(gpu_keys, ora_keys, diag=None):
    """Per-env: contact sets equal, or differing by at most one swapped pair
    at a cap tie reported by the oracle."""
    out = []
    for i, (a, b) in enumerate(zip(key_sets(gpu_keys), key_sets(ora_keys))):
        if a == b:
            out.append(True)
            continue
        tie = diag is not None and bool(cap_tie(diag[i:i + 1])[0])
        out.append(bool(tie and len(a) == len(b) and len(a ^ b) <= 2))
    return np.array(out)


def obs_from_gpu(obs_t):
    """[R][L][K] tensor -> [K][L][R] numpy (float64)."""
    return obs_t.detach().cpu().numpy().transpose(2, 1, 0).astype(np.float64)


def force_scale(b_obs, mass):
    """Per-sensor force scale max(|c_l|, m g) [K][L]."""
    return np.maximum(np.abs(b_obs[..., 0]), np.asarray(mass)[:, None] * G)


def obs_err(a, b, mass, tau):
    """Per-env error of the force rows of observation a against b, in units
    of each sensor's force scale: magnitude |da| / S, direction
    |dc_hat| |c_b| / (2 S) where |c_b| is clear of tau by more than 1e-4 S
    (the direction of a force within rounding of the threshold is either
    zero or a unit vector)."""
    S = force_scale(b, mass)
    e_mag = np.abs(a[..., 0] - b[..., 0]) / S
    clear = np.abs(b[..., 0] - tau) > TOL * S
    e_dir = np.linalg.norm(a[..., 1:4] - b[..., 1:4], axis=-1) * np.abs(b[..., 0]) / (2.0 * S)
    e_dir = np.where(clear, e_dir, 0.0)
    return np.maximum(e_mag, e_dir).max(axis=-1)


def obs_close(a, b, mass, tau, tol=TOL):
    return obs_err(a, b, mass, tau) <= tol


class Probes:
    """The oracle reference of a step and its classification (module
    docstring).  `o` is the oracle the trajectory runs on."""

    def __init__(self, o):
        self.o = o
        m = o.m
        kw = dict(C_max=o.C_max, newton_iters=m.newton_iters, D=o.D, converged=bool(m.converged),
                  conv_tol=m.conv_tol, conv_max_iters=m.conv_max_iters, sdf=o.sdf, sdf_box=o.sdf_box)
        self.g = [oracle.Oracle(o.hand, o.spheres, o.n_spheres, o.inv_inertia, o.consts, geom_f32=mode, **kw)
                  for mode in (1, 2)]

    def step(self, env_type, u_prev, u, st64, pr64, wk, wr64, want_contacts=False):
        """Reference step from the float32-rounded inputs plus the probes.
        Returns a dict: st, pr, wkey, wr, obs, cont, diag (the reference),
        clear [n] bool, tie [n] bool (cap tie, sets compared up to it),
        reason [n] str ('' when clear)."""
        o = self.o
        n = st64.shape[0]
        B = [f32(st64), f32(pr64), wk.copy(), f32(wr64)]
        obs_b, cont_b, dg = o.batch_step(env_type, u_prev, u, *B, want_contacts=want_contacts, want_diag=True)
        A = [st64.copy(), pr64.copy(), wk.copy(), wr64.copy()]
        o.batch_step(env_type, u_prev, u, *A)
        mass = B[1][:, 0]
        reason = np.array([""] * n, dtype=object)

        def flag(mask, why):
            for i in np.nonzero(mask & (reason == ""))[0]:
                reason[i] = why

        flag(~((rel_err(A[0], B[0]).max(axis=1) < CHAOS_TOL) & same_keys(A[2], B[2])), "state-rounding")
        for k, og in enumerate(self.g):
            Cq = [f32(st64), f32(pr64), wk.copy(), f32(wr64)]
            obs_c, _, _ = og.batch_step(env_type, u_prev, u, *Cq)
            ok = (rel_err(Cq[0], B[0]).max(axis=1) <= PROBE_TOL) & same_keys(Cq[2], B[2]) & \
                obs_close(obs_c[..., :4], obs_b[..., :4], mass, o.consts.tau_contact, PROBE_TOL)
            flag(~ok, f"geometry-probe-{k + 1}")
        flag(dg["armijo_margin"] < ARMIJO_BAND, "armijo")
        flag(np.abs(dg["margin_gap"]) < GAP_BAND, "margin")
        flag(dg["tangent_tie"] < TANGENT_BAND, "tangent-axis")
        tie = cap_tie(dg)
        flag(tie, "cap-tie")
        return dict(st=B[0], pr=B[1], wkey=B[2], wr=B[3], obs=obs_b, cont=cont_b, diag=dg,
                    clear=reason == "", tie=tie & (reason == "cap-tie"), reason=reason)


    def step_pd(self, env_type, u, st64, pr64, hq64, wk, wr64):
        """The same for a step of the PD-controlled hand (hq64 [n][2D]: joint
        angles and rates, floors 1 rad and 1 rad/s).  Returns the dict of
        step() with hq (the reference joint state) added."""
        o = self.o
        n = st64.shape[0]
        B = [f32(st64), f32(pr64), f32(hq64), wk.copy(), f32(wr64)]
        obs_b, cont_b, dg = o.batch_step_pd(env_type, u, *B, want_contacts=True, want_diag=True)
        A = [st64.copy(), pr64.copy(), hq64.copy(), wk.copy(), wr64.copy()]
        o.batch_step_pd(env_type, u, *A)
        mass = B[1][:, 0]
        reason = np.array([""] * n, dtype=object)

        def flag(mask, why):
            for i in np.nonzero(mask & (reason == ""))[0]:
                reason[i] = why

        def err(X, Y):
            return np.maximum(rel_err(X[0], Y[0]).max(axis=1), hand_err(X[2], Y[2]).max(axis=1))

        flag(~((err(A, B) < CHAOS_TOL) & same_keys(A[3], B[3])), "state-rounding")
        for k, og in enumerate(self.g):
            Cq = [f32(st64), f32(pr64), f32(hq64), wk.copy(), f32(wr64)]
            obs_c, _, _ = og.batch_step_pd(env_type, u, *Cq)
            ok = (err(Cq, B) <= PROBE_TOL) & same_keys(Cq[3], B[3]) & \
                obs_close(obs_c, obs_b, mass, o.consts.tau_contact, PROBE_TOL)
            flag(~ok, f"geometry-probe-{k + 1}")
        flag(dg["armijo_margin"] < ARMIJO_BAND, "armijo")
        flag(np.abs(dg["margin_gap"]) < GAP_BAND, "margin")
        flag(dg["tangent_tie"] < TANGENT_BAND, "tangent-axis")
        tie = cap_tie(dg)
        flag(tie, "cap-tie")
        return dict(st=B[0], pr=B[1], hq=B[2], wkey=B[3], wr=B[4], obs=obs_b, cont=cont_b, diag=dg,
                    clear=reason == "", tie=tie & (reason == "cap-tie"), reason=reason)


def hand_err(a, b):
    """Relative error of joint states [n][2D] with floors 1 rad, 1 rad/s."""
    return np.abs(a - b) / np.maximum(np.abs(b), 1.0)


def describe(ref, j):
    """One line with the decision margins of env j of a reference step."""
    d = ref["diag"][j]
    return (f"armijo {d['armijo_margin']:.1e} cap {d['d_first_dropped'] - d['d_last_kept']:.1e} "
            f"margin {d['margin_gap']:.1e} tangent {d['tangent_tie']:.1e} fallback {d['n_fallback']} "
            f"C {d['n_contacts']}")


def segment_reference(probes, env_type, u_rows, st64, pr64, wk, wr64, obs_gt=None):
    """The oracle over a segment of T = len(u_rows) - 1 steps from the
    float32-rounded start (the reference), with the probes followed along
    it.  u_rows[0] is the command before the segment.  Returns a dict: st,
    pr, wkey, wr (end of the segment), obs [T][n][L][R], keys [T] (the
    contact keys after each step), cost [n] (sum of the step costs against
    obs_gt[T][n][L][R] when given), clear [n] (every step clear along the
    segment)."""
    o = probes.o
    n = st64.shape[0]
    A = [st64.copy(), pr64.copy(), wk.copy(), wr64.copy()]
    B = [f32(st64), f32(pr64), wk.copy(), f32(wr64)]
    Gq = [[f32(st64), f32(pr64), wk.copy(), f32(wr64)] for _ in probes.g]
    clear = np.ones(n, bool)
    obs_hist, keys_hist = [], []
    cost = np.zeros(n)
    tau = o.consts.tau_contact
    for t in range(len(u_rows) - 1):
        u_prev, u = u_rows[t], u_rows[t + 1]
        mass = B[1][:, 0].copy()
        o.batch_step(env_type, u_prev, u, *A)
        obs_b, _, dg = o.batch_step(env_type, u_prev, u, *B, want_diag=True)
        for og, q in zip(probes.g, Gq):
            obs_c, _, _ = og.batch_step(env_type, u_prev, u, *q)
            clear &= rel_err(q[0], B[0]).max(axis=1) <= PROBE_TOL
            clear &= same_keys(q[2], B[2])
            clear &= obs_close(obs_c[..., :4], obs_b[..., :4], mass, tau, PROBE_TOL)
        clear &= rel_err(A[0], B[0]).max(axis=1) < CHAOS_TOL
        clear &= same_keys(A[2], B[2])
        clear &= (dg["armijo_margin"] >= ARMIJO_BAND) & (np.abs(dg["margin_gap"]) >= GAP_BAND) & \
            (dg["tangent_tie"] >= TANGENT_BAND) & ~cap_tie(dg)
        obs_hist.append(obs_b)
        keys_hist.append(B[2].copy())
        if obs_gt is not None:
            cost += np.array([o.step_cost(obs_b[i], obs_gt[t][i]) for i in range(n)])
    return dict(st=B[0], pr=B[1], wkey=B[2], wr=B[3], obs=np.array(obs_hist), keys=keys_hist, cost=cost,
                clear=clear)
