"""The PD-controlled hand on the GPU against the FP64 oracle: per-step parity
of object and joint state, contacts and observation (force rows and joint
angles) where the parity rule of tests/parity_util.py calls a step clear,
with no exceptions there; the joint-angle cost term; the resampler's copies
of the joint state; and the calls the PD hand does not support."""
import collections
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2002_12160_amd import scene as S
from tests import parity_util as PU

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


def _pd_cfg(name, **consts):
    cfg = S.CONFIGS[name]
    return cfg.with_(consts=dataclasses.replace(cfg.consts, hand_mode=1, **consts))


def _scene(cfg, K, steps):
    sc = S.make_scene(cfg, K=K, steps=steps)
    return dataclasses.replace(S.round_to_f32(sc), state=sc.state, params=sc.params,
                               hidden_state=sc.hidden_state, hidden_params=sc.hidden_params)


def _put(b, idx, st, pr, hq, wk, wr):
    """The sampled simulations' float32-rounded oracle state into the batch."""
    it = torch.as_tensor(np.asarray(idx, dtype=np.int64), device="cuda")
    b.state[:, it] = torch.as_tensor(PU.f32(st).T.astype(np.float32), device="cuda")
    b.params[:, it] = torch.as_tensor(PU.f32(pr).T.astype(np.float32), device="cuda")
    b.hand_state[:, it] = torch.as_tensor(PU.f32(hq).T.astype(np.float32), device="cuda")
    w = np.zeros((len(idx), b.C_max, 4), dtype=np.float32)
    w[:, :, 0] = np.asarray(wk, dtype=np.int32).view(np.float32)
    w[:, :, 1:] = wr
    b.warm[it] = torch.as_tensor(w, device="cuda")


def _obs_split(b, obs_t):
    """GPU observation [4L + D][K] -> (forces [K][L][4], joint angles [K][D])."""
    o = obs_t.detach().cpu().numpy().astype(np.float64)
    L = b.L
    force = o[:4 * L].reshape(4, L, -1).transpose(2, 1, 0)
    return force, o[4 * L:].T


def pd_parity(pt, cfg, K, steps, sample=None):
    """The oracle follows the sampled simulations for `steps` steps; before
    every step their float32-rounded oracle state goes to the GPU, both
    step, and the results are compared."""
    sc = _scene(cfg.with_(T=10 ** 6), K, steps)
    o = oracle.Oracle.from_scene(sc)
    assert o.hand_mode == 1
    probes = PU.Probes(o)
    D = o.D
    hq0 = o.new_hand(K, sc.u[0])
    b = pt.Batch.from_scene(sc, T=10, hand_state=hq0)
    idx = np.arange(K) if sample is None else np.asarray(sample)
    st, pr, hq = sc.state[idx].copy(), sc.params[idx].copy(), hq0[idx].copy()
    wk, wr = o.new_warm(len(idx))
    n_chk = n_ok = n_tie = n_contact = 0
    fails = []
    reasons = collections.Counter()
    worst_other = 0.0
    for t in range(steps):
        u = sc.u[t]
        ref = probes.step_pd(sc.env_type[idx], u, st, pr, hq, wk, wr)
        reasons.update(ref["reason"])
        _put(b, idx, st, pr, hq, wk, wr)
        b.step(None, _u(u))
        force, qo = _obs_split(b, b.observe())
        g_st, _ = b.get_state()
        g_hq = b.get_hand()
        g_k, _ = b.get_warm()
        g_st, g_hq, g_k, force, qo = g_st[idx], g_hq[idx], g_k[idx], force[idx], qo[idx]
        err = np.maximum(PU.rel_err(g_st, ref["st"]).max(axis=1), PU.hand_err(g_hq, ref["hq"]).max(axis=1))
        oerr = PU.obs_err(force, ref["obs"], ref["pr"][:, 0], cfg.consts.tau_contact)
        # the observed joint angles are the state's, bit for bit
        q_same = np.all(qo == PU.f32(g_hq[:, :D]), axis=1)
        keys_eq = PU.same_keys(g_k, ref["wkey"])
        cont, nc = ref["cont"], ref["diag"]["n_contacts"]
        n_contact += sum(bool(np.any((cont[i]["link"][:nc[i]] >= 0) & (cont[i]["link"][:nc[i]] < b.L)))
                         for i in range(len(idx)))
        for j in range(len(idx)):
            if not q_same[j]:
                fails.append((t, int(idx[j]), float(err[j]), float(oerr[j]), bool(keys_eq[j]), "joint rows"))
            elif ref["clear"][j]:
                n_ok += 1
                if not (err[j] <= PU.TOL and oerr[j] <= PU.TOL and keys_eq[j]):
                    fails.append((t, int(idx[j]), float(err[j]), float(oerr[j]), bool(keys_eq[j]),
                                  PU.describe(ref, j)))
            elif ref["tie"][j]:
                n_tie += 1
                if not PU.keys_match(g_k[j:j + 1], ref["wkey"][j:j + 1], ref["diag"][j:j + 1])[0]:
                    fails.append((t, int(idx[j]), float(err[j]), float(oerr[j]), False, "cap tie: " +
                                  PU.describe(ref, j)))
            else:
                worst_other = max(worst_other, float(err[j]))
        n_chk += len(idx)
        o.batch_step_pd(sc.env_type[idx], u, st, pr, hq, wk, wr)
    b.close()
    _say(f"PD per-step parity: {n_chk} env-steps ({n_contact} with a hand contact), {n_ok} clear, {n_tie} at a cap "
         f"tie, classification {dict(reasons)}; worst error where not clear {worst_other:.2e}; "
         f"{len(fails)} outside tolerance")
    for f in fails[:20]:
        _say(f"  MISS t={f[0]} env={f[1]} state {f[2]:.2e} obs {f[3]:.2e} keys {f[4]} | {f[5]}")
    return n_chk, n_ok, n_contact, fails


def test_pd_per_step_parity_small(pt):
    _say("PD hand per-step parity: small config (3 fingers x 3 joints), K=32, 60 steps")
    n_chk, n_ok, n_contact, fails = pd_parity(pt, _pd_cfg("small"), 32, 60)
    assert n_contact >= 0.25 * n_chk, "too few steps with hand contacts to test the coupled solve"
    assert n_ok >= 0.3 * n_chk
    assert not fails


def test_pd_per_step_parity_two_joint_fingers(pt):
    # 4 fingers with an abduction joint (two joints on the first link), a palm
    # of fixed links, 64-sphere ellipsoid: groups of 4 joints
    _say("PD hand per-step parity: plain256 hand, K=16 sampled of 64, 40 steps")
    n_chk, n_ok, n_contact, fails = pd_parity(pt, _pd_cfg("plain256"), 64, 40, sample=np.arange(0, 64, 4))
    assert n_contact >= 0.25 * n_chk
    assert n_ok >= 0.2 * n_chk
    assert not fails


def test_pd_per_step_parity_five_joint_fingers(pt):
    # the real-time hand with an abduction joint on every finger: groups of
    # 5 joints (the elimination sized for up to 6), D = 25, 16 object types
    _say("PD hand per-step parity: 5 fingers x 5 joints, real-time objects, K=32, 20 steps")
    cfg = _pd_cfg("realtime16384")
    cfg = cfg.with_(hand=dataclasses.replace(cfg.hand, abduction=True))
    n_chk, n_ok, n_contact, fails = pd_parity(pt, cfg, 32, 20)
    assert n_contact >= 0.25 * n_chk
    assert n_ok >= 0.15 * n_chk
    assert not fails


def test_pd_free_hand_tracks_the_oracle_without_contacts(pt):
    # the object far away: only the joints move (PD law and mass matrix)
    cfg = _pd_cfg("small")
    sc = _scene(cfg.with_(T=10 ** 6), 8, 30)
    sc.state[:, 0] += 1.0
    o = oracle.Oracle.from_scene(sc)
    hq = o.new_hand(8, sc.u[0] + 0.2)
    b = pt.Batch.from_scene(sc, T=10, hand_state=hq)
    st, pr = sc.state.copy(), sc.params.copy()
    wk, wr = o.new_warm(8)
    for t in range(30):
        u = sc.u[t]
        b.step(None, _u(u))
        o.batch_step_pd(sc.env_type, u, st, pr, hq, wk, wr)
    g_hq = b.get_hand()
    b.close()
    e = PU.hand_err(g_hq, hq).max()
    _say(f"free PD hand over 30 steps: worst joint-state error {e:.2e}")
    assert e <= 1e-4


def test_pd_cost_adds_the_joint_term(pt):
    cfg = _pd_cfg("small", w_q=50.0)
    sc = _scene(cfg.with_(T=10 ** 6), 16, 4)
    o = oracle.Oracle.from_scene(sc)
    hq = o.new_hand(16, sc.u[0])
    b = pt.Batch.from_scene(sc, T=10, hand_state=hq)
    for t in range(3):
        b.step(None, _u(sc.u[t]))
    obs = b.observe()
    rng = np.random.default_rng(5)
    gt = obs[:, :1].clone() + torch.as_tensor(rng.normal(scale=0.05, size=(obs.shape[0], 1)).astype(np.float32),
                                              device="cuda")
    cost = torch.zeros(16, device="cuda")
    best = torch.zeros(1, dtype=torch.int32, device="cuda")
    b.cost(obs, gt.contiguous(), cost, best)
    force, qo = _obs_split(b, obs)
    gforce, gq = _obs_split(b, gt)
    want = np.array([o.step_cost_pd(force[i], qo[i], gforce[0], gq[0]) for i in range(16)])
    got = cost.cpu().numpy().astype(np.float64)
    b.close()
    _say(f"PD step cost: worst relative error {np.max(np.abs(got - want) / np.maximum(want, 1e-6)):.2e}")
    np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-6)
    assert int(best.item()) == int(np.argmin(got))


def test_pd_resample_copies_the_joint_state(pt):
    cfg = _pd_cfg("small")
    sc = _scene(cfg.with_(T=10 ** 6), 64, 4)
    o = oracle.Oracle.from_scene(sc)
    rng = np.random.default_rng(9)
    hq = o.new_hand(64, sc.u[0]) + rng.normal(scale=0.01, size=(64, 2 * o.D))
    b = pt.Batch.from_scene(sc, T=10, hand_state=hq)
    before = b.get_hand()
    cost = torch.as_tensor(rng.uniform(size=64).astype(np.float32), device="cuda")
    parent = torch.empty(64, dtype=torch.int32, device="cuda")
    b.resample(cost, 0, parent)
    after = b.get_hand()
    par = parent.cpu().numpy()
    b.close()
    for j in range(64):
        src = j if par[j] < 0 else par[j]
        assert np.array_equal(after[j], before[src]), j
    assert (par >= 0).sum() == 64 - 16


def _pd_windows(pt, cfg, K, n_win, batched, graph=False, static=False, seed=3):
    """n_win windows of T steps, each followed by a resampling, on the plain
    path (T rounds of step/observe/cost) or the batched window; returns every
    output's raw bits after each window."""
    T = cfg.T
    sc = _scene(cfg.with_(T=10 ** 6), K, n_win * T + 1)
    o = oracle.Oracle.from_scene(sc)
    rng = np.random.default_rng(seed)
    hq = o.new_hand(K, sc.u[0]) + rng.normal(scale=0.02, size=(K, 2 * o.D))
    b = pt.Batch.from_scene(sc, T=T, hand_state=hq)
    G = b.G
    u_all = _u(sc.u)
    # observed rows: the plain path's own observation of a perturbed copy
    gts = torch.as_tensor(rng.normal(scale=0.3, size=(n_win * T, *b.obs_shape(G))).astype(np.float32),
                          device="cuda").abs().contiguous()
    cost = torch.zeros(K, device="cuda")
    best = torch.zeros(G, dtype=torch.int32, device="cuda")
    parent = torch.zeros(K, dtype=torch.int32, device="cuda")
    obs_win = b.new_obs(T)
    obs = b.new_obs()
    out = []
    for w in range(n_win):
        t0 = w * T
        gt_win = gts[t0:t0 + T].contiguous()
        if batched:
            u_win = u_all[max(t0 - 1, 0):t0 + T].contiguous() if t0 > 0 else torch.cat([u_all[:1], u_all[:T]], 0)
            if static:
                b.run_window_static(u_win.contiguous(), gt_win, cost, best, obs_win)
            else:
                b.run_window(u_win.contiguous(), gt_win, cost, best, obs_win, graph=graph)
        else:
            for t in range(T):
                b.step(None, u_all[t0 + t].contiguous())
                b.observe(obs)
                obs_win[t].copy_(obs)
                b.cost(obs, gt_win[t], cost, best if t == T - 1 else None)
        rec = [x.view(torch.int32).clone() for x in (b.state, b.params, b.warm, b.hand_state, cost, best, obs_win)]
        b.resample(cost, w, parent)
        rec.append(parent.clone())
        out.append(rec)
    torch.cuda.synchronize()
    b.close()
    return out


@pytest.mark.parametrize("cfg_name,K,abduction,sdf", [("small", 37, False, False), ("plain256", 40, False, False),
                                                       ("realtime16384", 48, True, False), ("small", 37, False, True),
                                                       ("small", 1100, False, False)])
def test_pd_window_equals_plain_bitwise(pt, cfg_name, K, abduction, sdf):
    # groups of 3 and 4 joints (the small elimination), of 5 (the large one),
    # and the distance-field collision; the window kernel against T rounds
    # of the per-step kernels, with and without the graph, and the
    # allocation-free entry point; two windows with a resampling between.
    # Past one simulation per SIMD (1100 > 4 x 256 compute units) the window
    # runs as per-step kernels inside the call: offsets of commands, rows and
    # observations
    cfg = _pd_cfg(cfg_name, collision_mode=1 if sdf else 0)
    if abduction:
        cfg = cfg.with_(hand=dataclasses.replace(cfg.hand, abduction=True))
    _say(f"PD window vs plain path: {cfg_name} K={K} abduction={abduction} distance field={sdf}")
    ref = _pd_windows(pt, cfg, K, 2, batched=False)
    for kw in ({"graph": False}, {"graph": True}, {"static": True}):
        got = _pd_windows(pt, cfg, K, 2, batched=True, **kw)
        names = ("state", "params", "warm", "hand_state", "cost", "best", "obs", "parent")
        for w in range(2):
            for n, x, y in zip(names, ref[w], got[w]):
                assert torch.equal(x, y), f"{kw} window {w}: {n} differs"


def test_pd_rejects_the_calls_it_does_not_support(pt):
    cfg = _pd_cfg("small")
    sc = _scene(cfg.with_(T=10 ** 6), 8, 12)
    o = oracle.Oracle.from_scene(sc)
    b = pt.Batch.from_scene(sc, T=10, hand_state=o.new_hand(8, sc.u[0]))
    u_win = _u(sc.u[:11])
    gt = torch.zeros((10, *b.obs_shape(1)), device="cuda")
    cost = torch.zeros(8, device="cuda")
    env = torch.arange(8, dtype=torch.int32, device="cuda")
    for call in (lambda: b.autotune(u_win, gt),
                 lambda: b.window_grad(u_win, gt, env, *b.start_of(env)),
                 lambda: b.resample_wrs(cost, 10, 0, 1.0, torch.zeros(8, dtype=torch.int32, device="cuda"))):
        with pytest.raises(pt.PtError) as ei:
            call()
        assert ei.value.code == 5
    b.close()
