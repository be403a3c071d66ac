"""WRS and REPS resamplers (Sec. III-D.1 / III-D.2) on the GPU against the
oracle: the per-group PMF and REPS temperature to float tolerance, every
draw a valid categorical draw under the oracle's own cumulative weights
(identical to the oracle's draw away from rounding ties), copies bit for
bit, exploration to float tolerance."""
import math

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


def _population(cfg, K, seed):
    sc = S.round_to_f32(S.make_scene(cfg, K=K, steps=2))
    rng = np.random.default_rng(seed)
    st = PU.f32(sc.state.copy())
    st[:, 7:13] = PU.f32(rng.normal(size=(K, 6)))
    pr = sc.params.copy()
    keys = rng.integers(-1, 300, size=(K, cfg.C_max)).astype(np.int32)
    wr = PU.f32(rng.normal(size=(K, cfg.C_max, 3)))
    # window sums over 10 steps, quantised so that ties occur, a few NaN
    cost = PU.f32(np.round(rng.gamma(2.0, 3.0, size=K), 1))
    cost[rng.uniform(size=K) < 0.03] = np.nan
    return sc, st, pr, keys, wr, cost


def _check(pt, sc, cfg, st, pr, keys, wr, cost, kind, hyper, window=5, n_steps=10):
    K = sc.K
    b = pt.Batch.from_scene(sc)
    b.set_state(st, pr)
    b.set_warm(keys, wr)
    c_dev = torch.as_tensor(cost.astype(np.float32), device="cuda")
    parent = torch.full((K,), -5, dtype=torch.int32, device="cuda")
    weights = torch.zeros(K, device="cuda")
    eta = torch.zeros(sc.G, device="cuda")
    if kind == "wrs":
        b.resample_wrs(c_dev, n_steps, window, hyper, parent, weights)
    else:
        b.resample_reps(c_dev, n_steps, window, hyper, parent, weights, eta)
    torch.cuda.synchronize()
    g_st, g_pr = b.get_state()
    g_k, g_r = b.get_warm()
    g_par = parent.cpu().numpy()
    g_w = weights.cpu().numpy()
    b.close()

    o = oracle.Oracle.from_scene(sc)
    o_st, o_pr, o_k, o_r, o_c = st.copy(), pr.copy(), keys.copy(), wr.copy(), cost.astype(np.float64)
    o_par, pmf, o_eta, cdf, target = o.resample_weighted(kind, hyper, oracle.resample_cfg(cfg), sc.group_start,
                                                         window, n_steps, o_c, o_st, o_pr, o_k, o_r)
    # PMF and temperature
    np.testing.assert_allclose(g_w, pmf, rtol=2e-5, atol=1e-9)
    if kind == "reps":
        g_eta = eta.cpu().numpy()
        for g in range(sc.G):
            lo, hi = sc.group_start[g], sc.group_start[g + 1]
            c = cost[lo:hi][np.isfinite(cost[lo:hi])]
            spread = (c.max() - c.min()) / n_steps if c.size else 0.0
            if math.isinf(o_eta[g]):
                assert math.isinf(g_eta[g])
            elif o_eta[g] < 1e-12 * max(spread, 1e-30):
                assert g_eta[g] == 0.0
            else:
                np.testing.assert_allclose(g_eta[g], o_eta[g], rtol=2e-5)
    # draws: each GPU parent is a valid draw under the oracle's cumulative
    # weights (a band of 1e-6 of the group total for rounding), and equals
    # the oracle's own draw except inside that band
    differ = 0
    for g in range(sc.G):
        lo, hi = sc.group_start[g], sc.group_start[g + 1]
        cw = cdf[lo:hi]
        band = 1e-6 * cw[-1]
        for j in range(lo, hi):
            i = g_par[j] - lo
            assert 0 <= i < hi - lo, (j, g_par[j])
            assert pmf[lo + i] > 0, (j, i)
            below = cw[i - 1] if i > 0 else 0.0
            assert below <= target[j] + band and target[j] < cw[i] + band, (j, i, target[j], below, cw[i])
            differ += int(g_par[j] != o_par[j])
    assert differ <= max(2, K // 1000), differ
    # copies bit for bit, exploration to float tolerance (same parents)
    same = g_par == o_par
    assert np.array_equal(g_st[same], o_st[same])
    assert np.array_equal(g_k[same], o_k[same]) and np.array_equal(g_r[same], o_r[same])
    np.testing.assert_allclose(g_pr[same], o_pr[same], rtol=1e-6, atol=1e-7)
    assert np.array_equal(g_st, st[g_par])
    assert float(c_dev.abs().sum()) == 0.0


@pytest.mark.parametrize("kind,hyper", [("wrs", 0.0), ("wrs", 0.7), ("wrs", 40.0),
                                        ("reps", 0.05), ("reps", 1.0), ("reps", 50.0)])
def test_weighted_resamplers_match_oracle(pt, kind, hyper):
    # three groups of 100: several draws per group, ties, NaN costs; REPS
    # with eps 50 is in the eta -> 0+ limit (uniform over the lowest costs)
    _say(f"weighted resampler parity: {kind} {hyper}")
    cfg = S.CONFIGS["small"].with_(group_types=(0, 0, 0))
    sc, st, pr, keys, wr, cost = _population(cfg, 300, 11)
    _check(pt, sc, cfg, st, pr, keys, wr, cost, kind, hyper)


@pytest.mark.parametrize("K", [16384, 5000])
def test_weighted_resamplers_full_group_sizes(pt, K):
    # one group of the largest size (16 simulations per thread of the draw
    # kernel) and a ragged one (5 per thread, the last thread short)
    _say(f"weighted resampler parity at K={K}")
    cfg = S.CONFIGS["small"]
    sc, st, pr, keys, wr, cost = _population(cfg, K, 12)
    _check(pt, sc, cfg, st, pr, keys, wr, cost, "reps", 0.3, window=9)
    _check(pt, sc, cfg, st, pr, keys, wr, cost, "wrs", 0.5, window=9)


def test_weighted_resamplers_degenerate_groups(pt):
    # a group without a finite cost (uniform draw), a group of equal costs
    # (uniform; REPS eta = +inf), a group of one simulation
    _say("weighted resamplers: degenerate groups")
    cfg = S.CONFIGS["small"].with_(group_types=(0, 0, 0))
    sc, st, pr, keys, wr, cost = _population(cfg, 41, 13)
    gs = sc.group_start
    assert gs[1] - gs[0] > 1
    cost[gs[0]:gs[1]] = np.nan
    cost[gs[1]:gs[2]] = 7.0
    for kind, hyper in (("wrs", 3.0), ("reps", 0.2)):
        _check(pt, sc, cfg, st, pr, keys, wr, cost.copy(), kind, hyper)
    cfg1 = S.CONFIGS["small"]
    sc1, st1, pr1, k1, r1, c1 = _population(cfg1, 1, 14)
    c1[:] = 3.0
    _check(pt, sc1, cfg1, st1, pr1, k1, r1, c1, "reps", 0.2)
