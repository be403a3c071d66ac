"""Pins of the oracle's weighted resamplers (WRS, Sec. III-D.1, Eq. 4; REPS,
Sec. III-D.2, Eqs. 5-6) against closed forms, optimality conditions,
limits and sampling statistics -- CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import resamplers as RS
from paper_2002_12160_amd import scene as S


def _kl_uniform(p):
    q = p[p > 0]
    return float(np.sum(q * np.log(q * p.shape[0])))


# ---------------------------------------------------------------- WRS ----
def test_wrs_zero_temperature_is_uniform():
    c = np.array([3.0, 1.0, 7.5, 2.0])
    np.testing.assert_allclose(RS.wrs_pmf(c, 0.0), np.full(4, 0.25), rtol=0, atol=1e-15)


def test_wrs_two_sims_closed_form():
    # P1 / P2 = exp(-lam (C1 - C2)) and P1 + P2 = 1
    lam, c1, c2 = 2.5, 0.3, 1.1
    p = RS.wrs_pmf(np.array([c1, c2]), lam)
    want1 = 1.0 / (1.0 + math.exp(-lam * (c2 - c1)))
    np.testing.assert_allclose(p, [want1, 1.0 - want1], rtol=1e-14)


def test_wrs_shift_invariance_and_order():
    rng = np.random.default_rng(3)
    c = rng.uniform(0, 5, size=50)
    p = RS.wrs_pmf(c, 1.7)
    np.testing.assert_allclose(RS.wrs_pmf(c + 1234.5, 1.7), p, rtol=1e-9)
    order = np.argsort(c, kind="stable")
    assert np.all(np.diff(p[order]) <= 1e-18)          # lower cost, higher probability
    assert abs(p.sum() - 1.0) < 1e-14


def test_wrs_sharp_limit_and_nan():
    c = np.array([2.0, 1.0, np.nan, 1.0, 5.0])
    p = RS.wrs_pmf(c, 1e6)
    np.testing.assert_allclose(p, [0, 0.5, 0, 0.5, 0], atol=1e-300)
    assert RS.wrs_pmf(np.array([np.nan, np.nan]), 3.0).tolist() == [0.5, 0.5]


# --------------------------------------------------------------- REPS ----
def _binary_entropy_root(target):
    """p in (1/2, 1) with -p log p - (1-p) log(1-p) = target, by bisection."""
    lo, hi = 0.5, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        h = -mid * math.log(mid) - (1 - mid) * math.log(1 - mid)
        if h > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("eps", [0.05, 0.2, 0.5])
def test_reps_two_sims_closed_form(eps):
    # two rewards a > b: P_a = sigma(delta / eta); the optimum sets
    # KL(P || uniform) = log 2 - H(P_a) = eps, so eta* = delta / logit(p*)
    c = np.array([1.0, 1.8])                 # rewards 1.8 and 1.0
    p, eta = RS.reps_pmf(c, eps)
    ps = _binary_entropy_root(math.log(2.0) - eps)
    delta = 0.8
    np.testing.assert_allclose(eta, delta / math.log(ps / (1 - ps)), rtol=1e-6)
    np.testing.assert_allclose(p, [ps, 1 - ps], rtol=1e-7)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_reps_first_order_condition(seed):
    # at eta* the dual's slope eps - KL(P_eta* || uniform) vanishes, and g is
    # no larger there than anywhere on a grid around it
    rng = np.random.default_rng(seed)
    c = rng.gamma(2.0, 0.5, size=200)
    eps = 0.3
    p, eta = RS.reps_pmf(c, eps)
    assert abs(_kl_uniform(p) - eps) < 1e-6
    r = RS.reps_rewards(c)
    g0 = RS.reps_dual(eta, r, eps)
    for f in np.geomspace(0.2, 5.0, 41):
        assert RS.reps_dual(eta * f, r, eps) >= g0 - 1e-12 * abs(g0)


def test_reps_rewards_and_order():
    c = np.array([0.5, 2.0, np.nan, 1.0])
    r = RS.reps_rewards(c)
    np.testing.assert_allclose(r[[0, 1, 3]], [2.0, 0.5, 1.5])
    assert np.isnan(r[2])
    p, _ = RS.reps_pmf(c, 0.1)
    assert p[2] == 0.0 and p[0] > p[3] > p[1] > 0


def test_reps_limits():
    # equal costs: uniform; eps >= log(K / #argmin): uniform over the minima
    p, eta = RS.reps_pmf(np.array([2.0, 2.0, 2.0]), 0.5)
    assert eta == math.inf and np.allclose(p, 1 / 3)
    c = np.array([1.0, 3.0, 1.0, 2.0])       # log(4 / 2) = 0.693
    p, eta = RS.reps_pmf(c, 1.0)
    assert eta < 1e-12
    np.testing.assert_allclose(p, [0.5, 0, 0.5, 0], atol=1e-300)
    p, eta = RS.reps_pmf(np.array([np.nan, np.nan]), 0.5)
    assert p.tolist() == [0.5, 0.5]


# ------------------------------------------------------------ drawing ----
def test_draw_frequencies_follow_pmf():
    # a categorical draw per simulation per window: the empirical frequency
    # over 400 windows x 64 draws matches the PMF within 5 standard errors
    pmf = np.array([0.5, 0.25, 0.125, 0.0625, 0.0625] + [0.0] * 59)
    K = pmf.shape[0]
    gs = np.array([0, K], dtype=np.int32)
    counts = np.zeros(K)
    for w in range(400):
        par, cdf, t = RS.draw_parents(pmf, gs, w, 0)
        np.add.at(counts, par, 1)
        i = par - 0
        below = np.where(i > 0, cdf[np.maximum(i - 1, 0)], 0.0)
        assert np.all(below <= t) and np.all(t < cdf[i])
    n = 400 * K
    freq = counts / n
    se = np.sqrt(pmf * (1 - pmf) / n)
    assert np.all(np.abs(freq - pmf) <= 5 * se + 1e-12)
    assert counts[5:].sum() == 0


def test_draw_u_in_open_unit_interval():
    us = [RS.draw_u(j, w, 0) for j in range(50) for w in range(4)]
    assert 0.0 < min(us) and max(us) < 1.0


# ------------------------------------------------- copy and explore ----
def test_apply_copies_from_the_snapshot_and_explores_everyone():
    cfg = S.CONFIGS["small"]
    sc = S.make_scene(cfg, K=6, steps=2)
    o = oracle.Oracle.from_scene(sc)
    st = sc.state.astype(np.float64).copy()
    pr = sc.params.astype(np.float64).copy()
    wk, wr = o.new_warm(6)
    wk[:] = np.arange(6)[:, None] * 100 + np.arange(cfg.C_max)[None, :]
    wr[:] = np.arange(6)[:, None, None]
    rc = oracle.resample_cfg(cfg)
    rc.sigma_mu = rc.sigma_m = rc.sigma_f = 0.0
    parent = np.array([1, 0, 0, 5, 4, 3], dtype=np.int32)   # swaps and a chain
    cost = np.ones(6)
    st0, pr0, wk0 = st.copy(), pr.copy(), wk.copy()
    oracle.lib().or_resample_apply(oracle.C.byref(o.m), oracle.C.byref(rc), 6, oracle._ip(parent), 0,
                                   oracle._dp(cost), oracle._dp(st), oracle._dp(pr), oracle._ip(wk),
                                   oracle._dp(wr))
    np.testing.assert_array_equal(st, st0[parent])
    np.testing.assert_array_equal(wk, wk0[parent])
    np.testing.assert_array_equal(pr[:, :2], pr0[parent, :2])
    assert np.all(pr[:, 2:] == 0) and np.all(cost == 0)


def test_apply_exploration_statistics():
    # with parents = identity every simulation still gets mu, m noise and a
    # fresh perturbation force: zero mean, the configured spread
    cfg = S.CONFIGS["small"]
    K = 4000
    sc = S.make_scene(cfg, K=K, steps=2)
    o = oracle.Oracle.from_scene(sc)
    st = sc.state.astype(np.float64).copy()
    pr = sc.params.astype(np.float64).copy()
    pr[:, 1] = 0.5 * (cfg.mu_range[0] + cfg.mu_range[1])
    pr[:, 0] = 0.5 * (cfg.m_range[0] + cfg.m_range[1])
    pr0 = pr.copy()
    wk, wr = o.new_warm(K)
    rc = oracle.resample_cfg(cfg)
    parent = np.arange(K, dtype=np.int32)
    oracle.lib().or_resample_apply(oracle.C.byref(o.m), oracle.C.byref(rc), K, oracle._ip(parent), 7,
                                   oracle._dp(np.ones(K)), oracle._dp(st), oracle._dp(pr), oracle._ip(wk),
                                   oracle._dp(wr))
    for col, sig in ((1, cfg.sigma_mu), (0, cfg.sigma_m)):
        d = pr[:, col] - pr0[:, col]
        assert abs(d.mean()) < 5 * sig / math.sqrt(K)
        assert abs(d.std() / sig - 1) < 0.08
    f = pr[:, 2:]
    assert np.all(np.abs(f.mean(axis=0)) < 5 * cfg.sigma_f / math.sqrt(K))
    assert np.all(np.abs(f.std(axis=0) / cfg.sigma_f - 1) < 0.08)


def test_resample_weighted_end_to_end():
    cfg = S.CONFIGS["small"].with_(group_types=(0, 0))
    sc = S.make_scene(cfg, K=40, steps=2)
    o = oracle.Oracle.from_scene(sc)
    rng = np.random.default_rng(5)
    cost = rng.uniform(0, 3, size=40) * 10
    cost[7] = np.nan
    st = sc.state.astype(np.float64).copy()
    pr = sc.params.astype(np.float64).copy()
    wk, wr = o.new_warm(40)
    rc = oracle.resample_cfg(cfg)
    st0 = st.copy()
    for kind, hyper in (("wrs", 2.0), ("reps", 0.4)):
        c = cost.copy()
        s1, p1 = st0.copy(), pr.copy()
        par, pmf, eta, cdf, t = o.resample_weighted(kind, hyper, rc, sc.group_start, 3, 10, c, s1, p1,
                                                    wk.copy(), wr.copy())
        assert np.all(c == 0)
        assert 7 not in par                                   # NaN cost is never drawn
        for g in range(2):
            lo, hi = sc.group_start[g], sc.group_start[g + 1]
            assert np.all((par[lo:hi] >= lo) & (par[lo:hi] < hi))
            assert abs(pmf[lo:hi].sum() - 1) < 1e-12
        np.testing.assert_array_equal(s1, st0[par])
        if kind == "reps":
            for g in range(2):
                lo, hi = sc.group_start[g], sc.group_start[g + 1]
                q = pmf[lo:hi][np.isfinite(cost[lo:hi])]
                assert abs(_kl_uniform(q) - hyper) < 1e-6
