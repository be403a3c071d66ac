"""GPU (libpt) against the FP64 oracle, element by element on the same seeded
inputs.  The tolerance and where it applies (the clear steps, with no
exceptions allowed there): tests/parity_util.py."""
import collections
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2002_12160_amd import scene as S
from tests import parity_util as PU
from tests import tiny

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_12160_amd import pt as _pt
    return _pt


def _u(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float32), device="cuda").contiguous()


def _say(*a):
    print(*a, flush=True)


def _scene(cfg, K, steps):
    """Scene tables (hand, commands, spheres, inertias) rounded to float32 for
    both sides; the population's initial state and parameters kept in double,
    so that the oracle's reference trajectory starts from the double values
    and the float32-rounded copy is a genuine perturbation from step 0 on."""
    sc = S.make_scene(cfg, K=K, steps=steps)
    return dataclasses.replace(S.round_to_f32(sc), state=sc.state, params=sc.params,
                               hidden_state=sc.hidden_state, hidden_params=sc.hidden_params)


def _put(b, idx, st, pr, wk, wr):
    """Write the sampled simulations' float32-rounded oracle state into the
    batch (the other simulations keep their own GPU trajectory)."""
    it = torch.as_tensor(np.asarray(idx, dtype=np.int64), device="cuda")
    b.state[:, it] = torch.as_tensor(PU.f32(st).T.astype(np.float32), device="cuda")
    b.params[:, it] = torch.as_tensor(PU.f32(pr).T.astype(np.float32), device="cuda")
    w = np.zeros((len(idx), b.C_max, 4), dtype=np.float32)
    w[:, :, 0] = np.asarray(wk, dtype=np.int32).view(np.float32)
    w[:, :, 1:] = wr
    b.warm[it] = torch.as_tensor(w, device="cuda")


def per_step_parity(pt, cfg_name, K, steps, sample=None, solve_precision=64, cfg=None):
    """The oracle follows the sampled simulations for `steps` steps (its
    double-precision trajectory); before every step the float32-rounded
    oracle state of those simulations goes to the GPU, both step, and the
    results are compared.  Returns (n_checked, n_clear, n_ties, failures,
    reasons, worst error on steps that are not clear)."""
    cfg = (cfg or S.CONFIGS[cfg_name]).with_(T=10 ** 6)
    sc = _scene(cfg, K, steps)
    o = oracle.Oracle.from_scene(sc)
    probes = PU.Probes(o)
    b = pt.Batch.from_scene(sc, solve_precision=solve_precision, T=10)   # windows unused here
    idx = np.arange(K) if sample is None else np.asarray(sample)
    st, pr = sc.state[idx].copy(), sc.params[idx].copy()
    wk, wr = o.new_warm(len(idx))
    n_chk = n_ok = n_tie = 0
    fails = []
    reasons = collections.Counter()
    worst_other = 0.0
    for t in range(steps):
        u_prev, u = sc.u[max(t - 1, 0)], sc.u[t]
        ref = probes.step(sc.env_type[idx], u_prev, u, st, pr, wk, wr)
        reasons.update(ref["reason"])
        _put(b, idx, st, pr, wk, wr)
        b.step(_u(u_prev), _u(u))
        g_obs = PU.obs_from_gpu(b.observe())[idx]
        g_st, _ = b.get_state()
        g_k, _ = b.get_warm()
        g_st, g_k = g_st[idx], g_k[idx]
        err = PU.rel_err(g_st, ref["st"]).max(axis=1)
        oerr = PU.obs_err(g_obs[..., :4], ref["obs"][..., :4], ref["pr"][:, 0], cfg.consts.tau_contact)
        keys_eq = PU.same_keys(g_k, ref["wkey"])
        for j in range(len(idx)):
            if ref["clear"][j]:
                n_ok += 1
                if not (err[j] <= PU.TOL and oerr[j] <= PU.TOL and keys_eq[j]):
                    fails.append((t, int(idx[j]), float(err[j]), float(oerr[j]), bool(keys_eq[j]),
                                  PU.describe(ref, j)))
            elif ref["tie"][j]:
                # either choice at a cap tie is correct: sets agree up to it
                n_tie += 1
                if not PU.keys_match(g_k[j:j + 1], ref["wkey"][j:j + 1], ref["diag"][j:j + 1])[0]:
                    fails.append((t, int(idx[j]), float(err[j]), float(oerr[j]), False, "cap tie: " +
                                  PU.describe(ref, j)))
            else:
                worst_other = max(worst_other, float(err[j]))
        n_chk += len(idx)
        # the oracle's own trajectory goes on from the double state
        o.batch_step(sc.env_type[idx], u_prev, u, st, pr, wk, wr)
    b.close()
    return n_chk, n_ok, n_tie, fails, reasons, worst_other


def _report(name, res):
    n_chk, n_ok, n_tie, fails, reasons, worst = res
    _say(f"{name}: {n_chk} env-steps, {n_ok} clear, {n_tie} at a cap tie, classification {dict(reasons)}; "
         f"worst state error where not clear {worst:.2e}; {len(fails)} outside tolerance")
    for f in fails[:20]:
        _say(f"  MISS t={f[0]} env={f[1]} state {f[2]:.2e} obs {f[3]:.2e} keys {f[4]} | {f[5]}")


def test_per_step_parity_small(pt):
    _say("per-step parity: small config, K=32, 60 steps")
    res = per_step_parity(pt, "small", 32, 60)
    _report("small", res)
    n_chk, n_ok, _, fails, _, _ = res
    assert n_ok >= 0.4 * n_chk
    assert not fails


@pytest.mark.xfail(reason="the float32 contact solve does not meet the 1e-4 bar: measured 231 of 1324 "
                          "non-chaotic steps outside it (worst 0.32) -- a fixed-N solve far from "
                          "convergence on a Schur system of condition ~1e3 -- so it is not a parity path; "
                          "the float64 solve is the default", strict=False)
def test_per_step_parity_small_fp32_solve(pt):
    _say("per-step parity, float32 contact solve: small config, K=32, 60 steps")
    res = per_step_parity(pt, "small", 32, 60, solve_precision=32)
    _report("small, float32 solve", res)
    assert not res[3]


def segment_parity(pt, cfg_name, K, n_seg, seg_len=10):
    """10-step segments from the oracle's trajectory: the GPU and the oracle
    both run seg_len steps from the float32-rounded state at the segment
    start (no resampling inside).  A simulation's segment is clear when every
    one of its steps is clear (tests/parity_util.py) along the reference run,
    the probes followed along the segment."""
    cfg = S.CONFIGS[cfg_name].with_(T=10 ** 6)
    steps = n_seg * seg_len
    sc = _scene(cfg, K, steps)
    tr = oracle.Tracker(sc)
    probes = PU.Probes(tr.o)
    b = pt.Batch.from_scene(sc, T=10)
    n_ok = 0
    fails = []
    for sgi in range(n_seg):
        t0 = sgi * seg_len
        u_rows = [sc.u[max(t0 - 1, 0)]] + [sc.u[t] for t in range(t0, t0 + seg_len)]
        ref = PU.segment_reference(probes, sc.env_type, u_rows, tr.state, tr.params, tr.wkey, tr.wr)
        b.set_state(PU.f32(tr.state), PU.f32(tr.params))
        b.set_warm(tr.wkey, PU.f32(tr.wr))
        keys_ok = np.ones(K, bool)
        for t in range(seg_len):
            b.step(_u(u_rows[t]), _u(u_rows[t + 1]))
            gk, _ = b.get_warm()
            keys_ok &= PU.same_keys(gk, ref["keys"][t])
        g_st, _ = b.get_state()
        err = PU.rel_err(g_st, ref["st"]).max(axis=1)
        for i in np.nonzero(ref["clear"])[0]:
            n_ok += 1
            if not (err[i] <= PU.TOL and keys_ok[i]):
                fails.append((t0, int(i), float(err[i]), bool(keys_ok[i])))
        for t in range(t0, t0 + seg_len):
            tr.step()
    b.close()
    return n_ok, fails


def test_segment_parity_small(pt):
    _say("10-step segment parity: small config, K=128, 6 segments")
    n_ok, fails = segment_parity(pt, "small", 128, 6)
    _say(f"{n_ok} clear segments, {len(fails)} outside tolerance: {fails[:10]}")
    assert n_ok >= 40
    assert not fails


def test_per_step_parity_plain256_sampled(pt):
    # the 256-simulation workload at full size, in the launch configuration the
    # benchmark times; the oracle follows a sample of 24 simulations
    _say("per-step parity: plain256 config, K=256, 30 steps, 24 sampled envs")
    sample = np.linspace(0, 255, 24).astype(int)
    res = per_step_parity(pt, "plain256", 256, 30, sample=sample)
    _report("plain256", res)
    assert res[1] >= 0.4 * res[0]
    assert not res[3]


@pytest.mark.parametrize("cfg_name,K", [("batched4096", 96), ("adjoint1024", 64), ("realtime16384", 64)])
def test_per_step_parity_other_workloads(pt, cfg_name, K):
    # the other scenes at reduced K: mixed object types, 64-contact caps (a
    # full wave of contact lanes), the 9-link hand and the 20-link hand with
    # superquadric objects in 16 groups
    _say(f"per-step parity: {cfg_name} config, K={K}, 30 steps")
    res = per_step_parity(pt, cfg_name, K, 30)
    _report(cfg_name, res)
    assert res[1] >= 0.3 * res[0]
    assert not res[3]


def test_per_step_parity_realtime16384_full_size(pt):
    # the 16384-simulation workload at full size (16 groups of 1024, one
    # superquadric each); the oracle follows 2 simulations of every group
    _say("per-step parity: realtime16384 config, K=16384, 12 steps, 32 sampled envs")
    sample = np.array([g * 1024 + o for g in range(16) for o in (5, 700)])
    res = per_step_parity(pt, "realtime16384", 16384, 12, sample=sample)
    _report("realtime16384 full size", res)
    assert res[1] >= 0.3 * res[0]
    assert not res[3]


def test_free_fall_and_resting_on_gpu(pt):
    # closed forms on the GPU: free fall is exact to float32 rounding; a
    # sphere resting on the table carries m g (r_n = m g dt)
    _say("closed forms on the GPU")
    rho, m = 0.01, 0.1
    sph, nsph, inv = tiny.single_sphere(rho)
    hand = np.array([tiny.far_link()])
    K = 2
    st = np.stack([tiny.state(x=(0, 0, 20.0), v=(0.3, 0.1, 0.5)), tiny.state(x=(0, 0, rho))])
    pr = np.stack([tiny.params(m, 0.5), tiny.params(m, 0.6)])
    b = pt.Batch(hand=hand, spheres=sph, n_spheres=nsph, inv_inertia=inv, env_type=np.zeros(K, np.int32),
                 group_start=np.array([0, K], np.int32), consts=tiny.consts(), C_max=4, newton_iters=10, T=10,
                 state=st, params=pr)
    u = _u(np.zeros(1))
    dt = 1.0 / 30.0
    for n in range(1, 41):
        b.step(u, u)
    g_st, _ = b.get_state()
    v0 = np.array([0.3, 0.1, 0.5])
    np.testing.assert_allclose(g_st[0, 7:10], v0 + 40 * np.array([0, 0, -9.81]) * dt, rtol=1e-5)
    for n in range(41, 301):
        b.step(u, u)
    k, r = b.get_warm()
    assert k[1, 0] == 1 and k[1, 1] == -1
    np.testing.assert_allclose(r[1, 0, 0], m * 9.81 * dt, rtol=1e-5)
    b.close()
