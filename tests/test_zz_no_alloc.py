"""pt_run_window_static (the window without allocation or graph capture, its
scratch in a static device array) against pt_run_window through the C ABI:
bit for bit on two calls in a row, the second with a smaller input (fewer
simulations, a shorter window and fewer links, so the static array holds the
larger first call's leftovers), and the size limit refused before any
launch."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2002_12160_amd import scene as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_12160_amd import pt as _pt
    return _pt


def _say(*a):
    print(*a, flush=True)


def _inputs(sc, T, dev="cuda"):
    u = torch.as_tensor(np.array([sc.u[0]] + [sc.u[t] for t in range(T)], dtype=np.float32), device=dev)
    gt = torch.zeros((T, 4, sc.L, sc.G), device=dev)
    return u, gt


def _pair(pt, sc, T):
    """The same window on two batches of the same scene: pt_run_window
    (graph == 0) on one, pt_run_window_static on the other; observed forces
    from the observed batch's own window."""
    h = pt.Batch.from_scene(sc, hidden=True, T=T)
    u, gt = _inputs(sc, T)
    h.run_window(u, torch.zeros_like(gt), torch.zeros(sc.G, device="cuda"), None, gt, graph=False)
    out = []
    for static in (False, True):
        b = pt.Batch.from_scene(sc, T=T)
        cost = torch.zeros(sc.K, device="cuda")
        best = torch.full((sc.G,), -1, dtype=torch.int32, device="cuda")
        obs = torch.zeros((T, 4, sc.L, sc.K), device="cuda")
        for _ in range(2):     # two windows: the counters are cleared on each call
            if static:
                b.run_window_static(u, gt, cost, best, obs)
            else:
                b.run_window(u, gt, cost, best, obs, graph=False)
        torch.cuda.synchronize()
        out.append({k: v.clone() for k, v in (("state", b.state), ("params", b.params), ("warm", b.warm),
                                                ("cost", cost), ("best", best), ("obs", obs))})
        b.close()
    h.close()
    return out


def _same(a, b, what):
    for k in a:
        x, y = a[k].contiguous().view(torch.int32), b[k].contiguous().view(torch.int32)
        assert torch.equal(x, y), f"{what}: {k} differs in {(x != y).sum().item()} words"


def test_static_window_equals_the_window_bitwise(pt):
    # first call: the batching scene's objects, 96 simulations in 3 groups,
    # 9 links, a 10-step window; second call: the small scene with 20
    # simulations, a 5-step window and one finger (3 links) fewer
    big = S.make_scene(S.CONFIGS["batched4096"], K=96, steps=12)
    _say("static-scratch window: batched4096 scene, K=96, T=10, then a smaller one")
    ref, got = _pair(pt, big, 10)
    _same(ref, got, "first call")
    cfg = S.CONFIGS["small"]
    cfg = cfg.with_(hand=dataclasses.replace(cfg.hand, n_fingers=2))
    small = S.make_scene(cfg, K=20, steps=8)
    assert small.L < big.L
    ref, got = _pair(pt, small, 5)
    _same(ref, got, "second, smaller call")


def test_static_window_refuses_sizes_beyond_its_scratch(pt):
    sc = S.make_scene(S.CONFIGS["small"], K=4, steps=2)
    T = 4096 // sc.L + 1                      # T x L above the 4096 segment records
    b = pt.Batch.from_scene(sc, T=T)
    u, gt = _inputs(S.make_scene(S.CONFIGS["small"], K=4, steps=T + 1), T)
    cost = torch.zeros(sc.K, device="cuda")
    with pytest.raises(pt.PtError) as e:
        b.run_window_static(u, gt, cost)
    assert e.value.code == 5
    b.close()
