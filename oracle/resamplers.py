"""Weighted resamplers of the oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product path never does.

Plain float64 definitions of the two sample-based optimisers that resample
with replacement (arXiv 2002.12160, Sec. III-D):

* WRS (Sec. III-D.1, Eq. 4): a softmax over the window's mean costs with a
  fixed temperature lambda, shifted by the minimum cost.
* REPS (Sec. III-D.2, Eqs. 5-6): costs turned into rewards
  R_i = max_j C_j + min_j C_j - C_i, a temperature eta* that minimises the
  dual g(eta) = eta eps + eta log((1/K) sum_i exp(R_i / eta)), and a softmax
  of R / eta*.

Readings (the paper leaves these open): the costs are the window means
(running sum / steps); a simulation whose cost is NaN (a divergent sample)
gets probability 0 and K counts the finite costs only; a group without a
finite cost resamples uniformly; when the dual has no interior minimum
(all finite costs equal, or eps >= log(K / #argmin)) the distribution is the
limit eta -> 0+: uniform over the lowest-cost simulations (uniform over all
of them when the costs are equal).

The draw (with replacement, one per simulation) takes u = (w + 1/2) 2^-32
from the first word w of Philox4x32-10 at counter (j, window, 3, 0) and
picks the first index whose cumulative weight exceeds u times the total.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import minimize_scalar
from scipy.special import logsumexp

from . import philox4x32_10

# the Philox counter word that distinguishes the categorical draw from the
# exploration draws (words 1 and 2) of the same simulation and window
DRAW_STREAM = 3


def _finite(cost_mean):
    c = np.asarray(cost_mean, dtype=np.float64)
    return c, np.isfinite(c)


def wrs_pmf(cost_mean, lam):
    """Eq. 4: P(i) proportional to exp(-lam (C_i - min_j C_j))."""
    c, ok = _finite(cost_mean)
    n = c.shape[0]
    if not ok.any():
        return np.full(n, 1.0 / n)
    cmin = c[ok].min()
    w = np.zeros(n)
    w[ok] = np.exp(-lam * (c[ok] - cmin))
    return w / w.sum()


def reps_dual(eta, rewards, eps):
    """Eq. 5's objective g(eta) = eta eps + eta log((1/K) sum_i exp(R_i / eta))."""
    r = np.asarray(rewards, dtype=np.float64)
    return eta * eps + eta * (logsumexp(r / eta) - math.log(r.shape[0]))


def reps_rewards(cost_mean):
    """R_i = max_j C_j + min_j C_j - C_i over the finite costs (NaN elsewhere)."""
    c, ok = _finite(cost_mean)
    r = np.full(c.shape[0], np.nan)
    if ok.any():
        r[ok] = c[ok].max() + c[ok].min() - c[ok]
    return r


def reps_pmf(cost_mean, eps):
    """Eqs. 5-6: (P, eta*).  eta* is found by a bounded scalar minimisation of
    g over log(eta); eta* is returned as 0 for the eta -> 0+ limit and +inf
    when every finite cost is equal or none is finite."""
    c, ok = _finite(cost_mean)
    n = c.shape[0]
    if not ok.any():
        return np.full(n, 1.0 / n), math.inf
    r = reps_rewards(c)[ok]
    spread = r.max() - r.min()
    p = np.zeros(n)
    if spread == 0.0:
        p[ok] = 1.0 / ok.sum()
        return p, math.inf
    # for eta >= spread / eps the dual's slope eps - KL(P_eta || uniform) is
    # already >= 0 (KL <= spread / eta), so the minimiser lies below it
    hi = math.log(spread / eps)
    res = minimize_scalar(lambda t: reps_dual(math.exp(t), r, eps), bounds=(hi - 60.0, hi),
                          method="bounded", options={"xatol": 1e-12, "maxiter": 2000})
    t = float(res.x)
    if t <= hi - 60.0 + 1e-6:
        # no interior minimum: the limit eta -> 0+
        best = r == r.max()
        q = np.zeros(ok.sum())
        q[best] = 1.0 / best.sum()
        p[ok] = q
        return p, 0.0
    eta = math.exp(t)
    z = (r - r.max()) / eta
    q = np.exp(z)
    p[ok] = q / q.sum()
    return p, eta


def draw_u(j, window_idx, seed):
    """Uniform in (0, 1) of simulation j's categorical draw in this window."""
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    w = philox4x32_10((j, window_idx, DRAW_STREAM, 0), key)
    return (w[0] + 0.5) / 4294967296.0


def draw_parents(pmf, group_start, window_idx, seed):
    """One draw with replacement per simulation from its group's PMF;
    returns (parent indices, cumulative weights, the draw targets u)."""
    K = pmf.shape[0]
    parent = np.zeros(K, dtype=np.int32)
    cdf = np.zeros(K)
    target = np.zeros(K)
    for g in range(len(group_start) - 1):
        lo, hi = int(group_start[g]), int(group_start[g + 1])
        if hi <= lo:
            continue
        cw = np.cumsum(pmf[lo:hi])
        cdf[lo:hi] = cw
        last = lo + int(np.nonzero(pmf[lo:hi] > 0)[0][-1])
        for j in range(lo, hi):
            t = draw_u(j, window_idx, seed) * cw[-1]
            target[j] = t
            i = int(np.searchsorted(cw, t, side="right"))
            parent[j] = min(lo + i, last)
    return parent, cdf, target


def group_pmf(kind, hyper, cost_sum, n_steps, group_start):
    """Per-group PMFs of WRS ('wrs', hyper = lambda) or REPS ('reps', hyper =
    eps) from the window's summed costs; returns (pmf [K], eta [G])."""
    mean = np.asarray(cost_sum, dtype=np.float64) / float(n_steps)
    G = len(group_start) - 1
    pmf = np.zeros(mean.shape[0])
    eta = np.full(G, np.nan)
    for g in range(G):
        lo, hi = int(group_start[g]), int(group_start[g + 1])
        if hi <= lo:
            continue
        if kind == "wrs":
            pmf[lo:hi] = wrs_pmf(mean[lo:hi], hyper)
        elif kind == "reps":
            pmf[lo:hi], eta[g] = reps_pmf(mean[lo:hi], hyper)
        else:
            raise ValueError(kind)
    return pmf, eta
