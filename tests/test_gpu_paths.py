"""GPU paths against each other and the resampler / cost / argmin against the
oracle.  The batched window (persistent kernel, optionally replayed from a HIP
graph, any environments-per-workgroup) runs the same per-simulation
arithmetic as the plain per-step kernels, so the two must agree bit for bit."""
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


def _say(*a):
    print(*a, flush=True)


def _window_inputs(sc, w, T, dev="cuda"):
    t0 = w * T
    rows = [sc.u[max(t0 - 1, 0)]] + [sc.u[t0 + t] for t in range(T)]
    return torch.as_tensor(np.array(rows, dtype=np.float32), device=dev)


def run_plain(pt, sc, windows, T, resample=True, solve_precision=64):
    b = pt.Batch.from_scene(sc, solve_precision=solve_precision)
    h = pt.Batch.from_scene(sc, hidden=True, solve_precision=solve_precision)
    cost = torch.zeros(sc.K, device="cuda")
    best = torch.zeros(sc.G, dtype=torch.int32, device="cuda")
    parent = torch.zeros(sc.K, dtype=torch.int32, device="cuda")
    obs_hist, bests, parents, costs = [], [], [], []
    for w in range(windows):
        uw = _window_inputs(sc, w, T)
        for t in range(T):
            h.step(uw[t], uw[t + 1])
            gt = h.observe()
            b.step(uw[t], uw[t + 1])
            obs = b.observe()
            b.cost(obs, gt, cost, best)
            obs_hist.append(obs.clone())
        costs.append(cost.clone())
        bests.append(best.clone())
        if resample:
            b.resample(cost, w, parent)
            parents.append(parent.clone())
    torch.cuda.synchronize()
    stats = b.read_stats()
    out = dict(state=b.state.clone(), params=b.params.clone(), warm=b.warm.clone(), obs=torch.stack(obs_hist),
               best=torch.stack(bests), costs=torch.stack(costs),
               parent=torch.stack(parents) if parents else None, stats=stats)
    b.close()
    h.close()
    return out


def run_batched(pt, sc, windows, T, graph, wpb=None, resample=True, solve_precision=64):
    b = pt.Batch.from_scene(sc, solve_precision=solve_precision)
    h = pt.Batch.from_scene(sc, hidden=True, solve_precision=solve_precision)
    cost = torch.zeros(sc.K, device="cuda")
    costh = torch.zeros(sc.G, device="cuda")
    best = torch.zeros(sc.G, dtype=torch.int32, device="cuda")
    parent = torch.zeros(sc.K, dtype=torch.int32, device="cuda")
    R = b.obs_rows
    gtw = torch.zeros((T, R, sc.L, sc.G), device="cuda")
    dummy = torch.zeros((T, R, sc.L, sc.G), device="cuda")
    obs_w = torch.zeros((T, R, sc.L, sc.K), device="cuda")
    uw = torch.zeros((T + 1, sc.D), device="cuda")
    if wpb is not None:
        b.set_tuning(wpb)
    obs_hist, bests, parents, costs = [], [], [], []
    for w in range(windows):
        uw.copy_(_window_inputs(sc, w, T))
        h.run_window(uw, dummy, costh, None, gtw, graph=graph)
        b.run_window(uw, gtw, cost, best, obs_w, graph=graph)
        obs_hist.append(obs_w.clone())
        costs.append(cost.clone())
        bests.append(best.clone())
        if resample:
            b.resample(cost, w, parent)
            parents.append(parent.clone())
    torch.cuda.synchronize()
    stats = b.read_stats()
    out = dict(state=b.state.clone(), params=b.params.clone(), warm=b.warm.clone(), obs=torch.cat(obs_hist),
               best=torch.stack(bests), costs=torch.stack(costs),
               parent=torch.stack(parents) if parents else None, stats=stats)
    b.close()
    h.close()
    return out


def _assert_same(a, b, what):
    # compare raw bits (the warm cache holds integer keys; -1 is a NaN pattern)
    for k in ("state", "params", "warm", "obs", "best", "costs", "parent"):
        if a[k] is None:
            continue
        x, y = a[k].contiguous().view(torch.int32), b[k].contiguous().view(torch.int32)
        assert torch.equal(x, y), f"{what}: {k} differs in {(x != y).sum().item()} words"
    # the step statistics (summed over their atomic slots) count the same
    # steps, candidates, contacts and drops on both paths
    assert a["stats"] == b["stats"], f"{what}: {a['stats']} != {b['stats']}"


@pytest.mark.parametrize("cfg_name,K,prec", [("small", 37, 64), ("batched4096", 96, 64), ("small/C_max=64", 37, 64),
                                           ("small/C_max=64", 37, 32), ("small", 300, 64)])
def test_batched_equals_plain_bitwise(pt, cfg_name, K, prec):
    # K = 300: more simulations than statistics slots (they wrap around)
    # "small/C_max=64": a cap above 32 makes the window kernel try the line
    # search's step sizes one at a time while the per-step kernel still
    # pairs them on the two half-waves in every step with at most 32
    # contacts (16- and 32-lane sums): the two forms must give the same bits
    _say(f"plain vs batched: {cfg_name} K={K}, solve precision {prec}")
    name, _, cap = cfg_name.partition("/C_max=")
    cfg = S.CONFIGS[name]
    if cap:
        cfg = cfg.with_(C_max=int(cap))
    sc = S.make_scene(cfg, K=K, steps=40)
    ref = run_plain(pt, sc, 3, cfg.T, solve_precision=prec)
    for graph in (False, True):
        got = run_batched(pt, sc, 3, cfg.T, graph=graph, solve_precision=prec)
        _assert_same(ref, got, f"graph={graph}")


def test_deep_work_queue_bitwise_and_oracle(pt):
    # 65536 simulations (4 groups of 16384): far more than the chip holds at
    # once (at most 32 wavefronts per compute unit), so every wavefront of
    # the persistent kernel takes several simulations from the work queue
    # one after another, reusing its LDS and registers.  Bit for bit equal
    # to the plain path over two windows with resampling (graph and no
    # graph), and the first window of 256 sampled simulations against the
    # oracle on the clear ones.
    cfg = S.CONFIGS["small"].with_(group_types=(0, 0, 0, 0))
    K, T = 65536, cfg.T
    _say(f"deep work queue: small scene, K={K}, 2 windows")
    sc = S.round_to_f32(S.make_scene(cfg, K=K, steps=2 * T))
    ref = run_plain(pt, sc, 2, T)
    for graph in (False, True):
        got = run_batched(pt, sc, 2, T, graph=graph)
        _assert_same(ref, got, f"K={K} graph={graph}")
        del got
    # the sampled simulations' first window against the oracle
    idx = np.linspace(0, K - 1, 256).astype(int)
    o = oracle.Oracle.from_scene(sc)
    probes = PU.Probes(o)
    wk, wr = o.new_warm(len(idx))
    u_rows = [sc.u[0]] + [sc.u[t] for t in range(T)]
    seg = PU.segment_reference(probes, sc.env_type[idx], u_rows, sc.state[idx], sc.params[idx], wk, wr)
    g_obs = ref["obs"][:T].cpu().numpy()[:, :, :, idx].transpose(0, 3, 2, 1).astype(np.float64)  # [T][n][L][4]
    n_ok = 0
    for j in np.nonzero(seg["clear"])[0]:
        n_ok += 1
        for t in range(T):
            assert PU.obs_close(g_obs[t, j:j + 1], seg["obs"][t, j:j + 1], seg["pr"][j:j + 1, 0],
                                cfg.consts.tau_contact)[0], (t, idx[j])
    _say(f"{n_ok} of {len(idx)} sampled windows clear; their observations match the oracle at every step")
    assert n_ok >= 4
    del ref


@pytest.mark.parametrize("prec,choices", [(64, (1, 2, 4)), (32, (1, 2, 4, 8))])
def test_autotune_choices_agree_bitwise(pt, prec, choices):
    _say(f"every environments-per-workgroup choice gives the same bits (solve precision {prec})")
    cfg = S.CONFIGS["small"]
    sc = S.make_scene(cfg, K=40, steps=20)
    outs = []
    for wpb in choices:
        b = pt.Batch.from_scene(sc, solve_precision=prec)
        h = pt.Batch.from_scene(sc, hidden=True, solve_precision=prec)
        uw = _window_inputs(sc, 0, cfg.T)
        gtw = torch.zeros((cfg.T, 4, sc.L, sc.G), device="cuda")
        dummy = torch.zeros_like(gtw)
        cost = torch.zeros(sc.K, device="cuda")
        costh = torch.zeros(sc.G, device="cuda")
        h.run_window(uw, dummy, costh, None, gtw, graph=False)
        if wpb == 1:
            assert b.autotune(uw, gtw) in choices   # leaves the state untouched
        b.set_tuning(wpb)
        b.run_window(uw, gtw, cost, None, None, graph=(wpb % 2 == 0))
        torch.cuda.synchronize()
        outs.append((b.state.clone(), cost.clone()))
        b.close()
        h.close()
    for st, c in outs[1:]:
        assert torch.equal(st, outs[0][0]) and torch.equal(c, outs[0][1])


def test_resample_matches_oracle(pt):
    _say("resampler parity")
    cfg = S.CONFIGS["small"].with_(group_types=(0, 0, 0))
    K = 300
    sc = S.round_to_f32(S.make_scene(cfg, K=K, steps=2))
    rng = np.random.default_rng(3)
    st = PU.f32(sc.state.copy())
    st[:, 7:13] = PU.f32(rng.normal(size=(K, 6)))
    pr = sc.params.copy()
    keys = rng.integers(-1, 300, size=(K, cfg.C_max)).astype(np.int32)
    wr = PU.f32(rng.normal(size=(K, cfg.C_max, 3)))
    cost = PU.f32(rng.uniform(0, 5, size=K))
    cost[10] = cost[11]          # tie
    cost[12] = np.nan            # divergent simulation
    b = pt.Batch.from_scene(sc)
    b.set_state(st, pr)
    b.set_warm(keys, wr)
    c_dev = torch.as_tensor(cost.astype(np.float32), device="cuda")
    parent = torch.zeros(K, dtype=torch.int32, device="cuda")
    b.resample(c_dev, 7, parent)
    g_st, g_pr = b.get_state()
    g_k, g_r = b.get_warm()
    o = oracle.Oracle.from_scene(sc)
    o_st, o_pr, o_k, o_r, o_c = st.copy(), pr.copy(), keys.copy(), wr.copy(), cost.copy()
    o_par = o.resample(oracle.resample_cfg(cfg), sc.group_start, 7, o_c, o_st, o_pr, o_k, o_r)
    assert np.array_equal(parent.cpu().numpy(), o_par)
    assert np.array_equal(g_st, o_st)           # copies are bit-exact
    assert np.array_equal(g_k, o_k) and np.array_equal(g_r, o_r)
    np.testing.assert_allclose(g_pr, o_pr, rtol=1e-6, atol=1e-7)
    assert float(c_dev.abs().sum()) == 0.0
    b.close()


def test_cost_and_argmin_match_oracle(pt):
    _say("cost and argmin parity")
    cfg = S.CONFIGS["small"].with_(group_types=(0, 0))
    K = 50
    sc = S.round_to_f32(S.make_scene(cfg, K=K, steps=2))
    rng = np.random.default_rng(9)
    L = sc.L
    obs = np.zeros((K, L, 4))
    obs[..., 0] = rng.uniform(0, 3, size=(K, L)) * (rng.uniform(size=(K, L)) > 0.4)
    d = rng.normal(size=(K, L, 3))
    obs[..., 1:] = d / np.linalg.norm(d, axis=-1, keepdims=True) * (obs[..., :1] > 0)
    obs = PU.f32(obs)
    gt = PU.f32(obs[[3, 30]].copy())
    obs[20] = gt[0]              # an exact copy of group 0's observation
    obs[41] = obs[40]            # a tie in group 1
    b = pt.Batch.from_scene(sc)
    obs_t = torch.as_tensor(obs.transpose(2, 1, 0).astype(np.float32).copy(), device="cuda")
    gt_t = torch.as_tensor(gt.transpose(2, 1, 0).astype(np.float32).copy(), device="cuda")
    cost = torch.zeros(K, device="cuda")
    best = torch.zeros(2, dtype=torch.int32, device="cuda")
    b.cost(obs_t, gt_t, cost, best)
    torch.cuda.synchronize()
    o = oracle.Oracle.from_scene(sc)
    ref = np.zeros(K)
    o.batch_cost(sc.group_start, obs, gt, ref)
    np.testing.assert_allclose(cost.cpu().numpy(), ref, rtol=1e-6, atol=1e-7)
    g_best = best.cpu().numpy()
    for g in range(2):
        lo, hi = sc.group_start[g], sc.group_start[g + 1]
        assert g_best[g] == lo + oracle.argmin(cost.cpu().numpy()[lo:hi].astype(np.float64))
    assert cost[3].item() == 0.0 and cost[20].item() == 0.0 and g_best[0] == 3
    # NaN costs rank last
    c2 = torch.tensor([np.nan, 2.0, 1.0, 1.0] + [5.0] * (K - 4), device="cuda")
    b.cost(torch.zeros_like(obs_t), torch.zeros_like(gt_t), c2, best)
    torch.cuda.synchronize()
    assert best.cpu().numpy()[0] == 2
    b.close()


@pytest.mark.parametrize("K", [64, 256, 257, 4096, 4097, 9000])
def test_group_argmin_sizes(pt, K):
    # the cost kernel ranks the groups in its only workgroup up to 256
    # simulations, in its last workgroup up to 4096 and leaves it to a kernel
    # of its own beyond; all give the
    # lowest index of the minimum with NaN last, on repeated calls (the
    # last-workgroup counter is put back after each launch)
    _say(f"group argmin, K={K}")
    cfg = S.CONFIGS["small"].with_(group_types=(0, 0, 0))
    sc = S.make_scene(cfg, K=K, steps=2)
    b = pt.Batch.from_scene(sc)
    G, L = sc.G, sc.L
    zo = torch.zeros((4, L, K), device="cuda")
    zg = torch.zeros((4, L, G), device="cuda")
    best = torch.full((G,), -7, dtype=torch.int32, device="cuda")
    rng = np.random.default_rng(K)
    for rep in range(3):
        c = rng.integers(0, 40, size=K).astype(np.float32)   # many ties
        c[rng.uniform(size=K) < 0.1] = np.nan
        if rep == 2:
            lo, hi = sc.group_start[1], sc.group_start[2]
            c[lo:hi] = np.nan                                 # a group with no finite cost
        cost = torch.as_tensor(c, device="cuda")
        b.cost(zo, zg, cost, best)
        torch.cuda.synchronize()
        got = best.cpu().numpy()
        for g in range(G):
            lo, hi = sc.group_start[g], sc.group_start[g + 1]
            want = lo + oracle.argmin(c[lo:hi].astype(np.float64))
            assert got[g] == want, (rep, g, got[g], want)
    b.close()


def test_divergent_simulations(pt):
    # A simulation whose state is not finite (a divergent sample) gets a NaN
    # window cost, ranks last, is never the estimate nor an elite, and the
    # resampler overwrites it with a copy of an elite.  A group whose
    # simulations have all diverged keeps its lowest indices as elites (NaN
    # ranks as +inf, ties by index) and stays divergent: the caller has to
    # re-initialise it.
    _say("divergent simulations: NaN cost, never elite, replaced at resampling")
    cfg = S.CONFIGS["small"]
    K = 32
    sc = S.make_scene(cfg, K=K, steps=2 * cfg.T)
    b = pt.Batch.from_scene(sc)
    h = pt.Batch.from_scene(sc, hidden=True)
    T = cfg.T
    uw = _window_inputs(sc, 0, T)
    gtw = torch.zeros((T, 4, sc.L, sc.G), device="cuda")
    h.run_window(uw, torch.zeros_like(gtw), torch.zeros(sc.G, device="cuda"), None, gtw, graph=False)
    b.state[7:10, 5] = float("nan")
    b.state[7, 9] = 1e30
    cost = torch.zeros(K, device="cuda")
    best = torch.zeros(sc.G, dtype=torch.int32, device="cuda")
    parent = torch.zeros(K, dtype=torch.int32, device="cuda")
    b.run_window(uw, gtw, cost, best, None, graph=False)
    torch.cuda.synchronize()
    c = cost.cpu().numpy()
    assert np.isnan(c[5]) and not np.isfinite(c[9])
    assert best.item() not in (5, 9)
    b.resample(cost, 0, parent)
    torch.cuda.synchronize()
    par = parent.cpu().numpy()
    assert par[5] >= 0 and par[9] >= 0                      # replaced, not kept
    st = b.state.cpu().numpy()
    assert np.all(np.isfinite(st[:, 5])) and np.all(np.isfinite(st[:, 9]))
    assert np.array_equal(st[:, 5], st[:, par[5]])           # a copy of its elite
    # every simulation divergent
    b.state[7:10, :] = float("nan")
    cost.zero_()
    b.run_window(uw, gtw, cost, best, None, graph=False)
    b.resample(cost, 1, parent)
    torch.cuda.synchronize()
    kb = max(1, int(np.floor(np.float32(K) * np.float32(cfg.elite_frac))))
    assert best.item() == 0
    assert np.array_equal(np.nonzero(parent.cpu().numpy() == -1)[0], np.arange(kb))
    b.close()
    h.close()
