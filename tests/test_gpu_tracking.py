"""The tracking loop's own invariants on the GPU against the oracle: a copy
of the observed simulation inside the population has cost exactly 0 and is
the estimate (Eq. 2), on the plain and the batched path; and over a 10-step
window (Eq. 1) the window costs, and with them the elite sets the
resampler keeps (Sec. III-D.3), equal the oracle's on the simulations whose
window is clear (tests/parity_util.py)."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2002_12160_amd import scene as S
from tests import parity_util as PU
from tests.test_gpu_paths import _window_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_12160_amd import pt as _pt
    return _pt


def _say(*a):
    print(*a, flush=True)


def _with_copy(cfg, K, steps, slots):
    """Scene in float32 with the observed simulation of group 0 copied into
    the given slots (same pose, mass, friction)."""
    sc = S.round_to_f32(S.make_scene(cfg, K=K, steps=steps))
    for j in slots:
        sc.state[j] = sc.hidden_state[0]
        sc.params[j] = sc.hidden_params[0]
    return sc


@pytest.mark.parametrize("batched", [False, True])
def test_hidden_copy_has_zero_cost_and_is_best(pt, batched):
    # a simulation that is a copy of the observed one receives the same
    # inputs and runs the same code: its observation is the observed one bit
    # for bit, its cost exactly 0, it is the argmin of its group, and as an
    # elite it is never perturbed by the resampler
    _say(f"observed copy inside the population, {'batched' if batched else 'plain'} path")
    cfg = S.CONFIGS["small"]
    K, T, windows, j = 40, cfg.T, 3, 17
    sc = _with_copy(cfg, K, T * windows, [j])
    b = pt.Batch.from_scene(sc)
    h = pt.Batch.from_scene(sc, hidden=True)
    cost = torch.zeros(K, device="cuda")
    best = torch.zeros(sc.G, dtype=torch.int32, device="cuda")
    parent = torch.zeros(K, dtype=torch.int32, device="cuda")
    gtw = torch.zeros((T, 4, sc.L, sc.G), device="cuda")
    costh = torch.zeros(sc.G, device="cuda")
    for w in range(windows):
        uw = _window_inputs(sc, w, T)
        if batched:
            h.run_window(uw, torch.zeros_like(gtw), costh, None, gtw, graph=True)
            b.run_window(uw, gtw, cost, best, None, graph=True)
            torch.cuda.synchronize()
            assert cost[j].item() == 0.0 and best.item() == j, (w, cost[j].item(), best.item())
        else:
            for t in range(T):
                h.step(uw[t], uw[t + 1])
                gt = h.observe()
                b.step(uw[t], uw[t + 1])
                obs = b.observe()
                assert torch.equal(obs[:, :, j], gt[:, :, 0]), (w, t)
                b.cost(obs, gt, cost, best)
                torch.cuda.synchronize()
                # the estimate is the lowest index of cost 0 (j, once the
                # others have met a force that differs)
                assert cost[j].item() == 0.0 and cost[best.item()].item() == 0.0 and best.item() <= j, \
                    (w, t, cost[j].item(), best.item())
            assert best.item() == j
        assert torch.all(cost[torch.arange(K, device="cuda") != j] > 0)
        b.resample(cost, w, parent)
        torch.cuda.synchronize()
        assert parent[j].item() == -1
        assert torch.equal(b.state[:, j], h.state[:, 0]) and torch.equal(b.params[:, j], h.params[:, 0])
    b.close()
    h.close()


def _elites(ids, costs, kb):
    order = np.argsort(costs, kind="stable")
    return set(ids[order[:kb]].tolist())


@pytest.mark.parametrize("cfg_name,K", [("small", 256), ("adjoint1024", 512)])
def test_window_costs_and_elites_match_oracle(pt, cfg_name, K):
    # windows starting 10, 20 and 30 steps into the oracle's trajectory; the
    # observed forces come from the oracle's observed simulation (rounded to
    # float32) and are given to both sides.  On the clear simulations the
    # window costs agree to 1e-3 and the top quarter by cost -- the elites
    # the resampler keeps -- is the same set (up to a swap of two costs
    # within that tolerance at the boundary).
    cfg = S.CONFIGS[cfg_name].with_(T=10 ** 6)
    T = 10
    starts = (10, 20, 30)
    sc0 = S.make_scene(cfg, K=K, steps=max(starts) + T)
    sc = dataclasses.replace(S.round_to_f32(sc0), state=sc0.state, params=sc0.params,
                             hidden_state=sc0.hidden_state, hidden_params=sc0.hidden_params)
    tr = oracle.Tracker(sc)
    probes = PU.Probes(tr.o)
    b = pt.Batch.from_scene(sc, T=T)
    n_clear = 0
    for t0 in starts:
        while tr.t < t0:
            tr.step()
        u_rows = [sc.u[max(t0 - 1, 0)]] + [sc.u[t] for t in range(t0, t0 + T)]
        # the observed simulation's forces over the window
        hst, hpr, hk, hr = PU.f32(tr.hstate), PU.f32(tr.hparams), tr.hkey.copy(), PU.f32(tr.hr)
        gts = []
        for t in range(T):
            obs, _, _ = tr.o.batch_step(sc.hidden_type, u_rows[t], u_rows[t + 1], hst, hpr, hk, hr)
            gts.append(PU.f32(obs))
        gts = np.array(gts)                                           # [T][G][L][4]
        gt_per_env = gts[:, np.searchsorted(sc.group_start, np.arange(K), side="right") - 1]
        ref = PU.segment_reference(probes, sc.env_type, u_rows, tr.state, tr.params, tr.wkey, tr.wr,
                                   obs_gt=gt_per_env)
        b.set_state(PU.f32(tr.state), PU.f32(tr.params))
        b.set_warm(tr.wkey, PU.f32(tr.wr))
        uw = torch.as_tensor(np.array(u_rows, dtype=np.float32), device="cuda")
        gtw = torch.as_tensor(np.ascontiguousarray(gts.transpose(0, 3, 2, 1)).astype(np.float32), device="cuda")
        cost = torch.zeros(K, device="cuda")
        b.run_window(uw, gtw, cost, None, None, graph=True)
        g_cost = cost.cpu().numpy().astype(np.float64)
        ids = np.nonzero(ref["clear"])[0]
        n_clear += len(ids)
        _say(f"{cfg_name} window at step {t0}: {len(ids)} of {K} simulations clear")
        if len(ids) < 4:
            continue
        co, cg = ref["cost"][ids], g_cost[ids]
        np.testing.assert_allclose(cg, co, rtol=1e-3, atol=1e-7)
        kb = max(1, len(ids) // 4)
        eo, eg = _elites(ids, co, kb), _elites(ids, cg, kb)
        if eo != eg:
            srt = np.sort(co)
            assert srt[kb] - srt[kb - 1] <= 2e-3 * srt[kb], (t0, sorted(eo ^ eg))
            assert len(eo ^ eg) == 2
    b.close()
    assert n_clear >= 20
