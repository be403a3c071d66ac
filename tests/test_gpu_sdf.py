"""Links against the object's signed distance field (collision_mode 1) on the
GPU against the FP64 oracle: per-step parity of state, contacts and
observation where the parity rule of tests/parity_util.py calls a step
clear, with no exceptions there -- the exact box field of the small
workload's cuboid, the sampled fields of the real-time workload's sixteen
superquadrics, and the PD-controlled hand on the box field; the batched
window bit for bit equal to the per-step path; and the calls the
distance-field path does not support."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2002_12160_amd import scene as S
from tests import parity_util as PU
from tests.test_gpu_parity import _report, per_step_parity
from tests.test_gpu_pd import pd_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_12160_amd import pt as _pt
    return _pt


def _say(*a):
    print(*a, flush=True)


def _sdf_cfg(name, **consts):
    cfg = S.CONFIGS[name]
    return cfg.with_(consts=dataclasses.replace(cfg.consts, collision_mode=1, **consts))


def test_sdf_per_step_parity_box_field(pt):
    _say("distance-field per-step parity: small config (cuboid, exact box field), K=32, 60 steps")
    res = per_step_parity(pt, "small", 32, 60, cfg=_sdf_cfg("small"))
    _report("small, distance field", res)
    n_chk, n_ok, _, fails, _, _ = res
    assert n_ok >= 0.3 * n_chk
    assert not fails


def test_sdf_per_step_parity_superquadric_fields(pt):
    # 16 object types (4 simulations each), 20 links x 8 samples, C_max 64
    _say("distance-field per-step parity: real-time workload's hand and objects, K=64, 20 steps")
    res = per_step_parity(pt, "realtime16384", 64, 20, cfg=_sdf_cfg("realtime16384"))
    _report("realtime objects, distance field", res)
    n_chk, n_ok, _, fails, _, _ = res
    assert n_ok >= 0.2 * n_chk
    assert not fails


def test_sdf_pd_hand_per_step_parity(pt):
    _say("distance field with the PD-controlled hand: small config, K=32, 40 steps")
    cfg = _sdf_cfg("small", hand_mode=1)
    n_chk, n_ok, n_contact, fails = pd_parity(pt, cfg, 32, 40)
    assert n_contact >= 0.25 * n_chk
    assert n_ok >= 0.3 * n_chk
    assert not fails


@pytest.mark.parametrize("cfg_name,K", [("small", 37), ("realtime16384", 48), ("small/C_max=64", 37), ("small", 0)])
def test_sdf_batched_equals_plain_bitwise(pt, cfg_name, K):
    # the window kernel's distance-field instantiations against the per-step
    # kernel's, with and without the graph (C_max <= 32 pairs the line
    # search's trials in the window kernel); K = 0 stands for past eight
    # simulations per compute unit, where the per-step path takes the
    # step's hand segments from k_hand_fk
    if K == 0:
        K = 8 * torch.cuda.get_device_properties(0).multi_processor_count + 37
    from tests.test_gpu_paths import _assert_same, run_batched, run_plain
    name, _, cap = cfg_name.partition("/C_max=")
    cfg = _sdf_cfg(name)
    if cap:
        cfg = cfg.with_(C_max=int(cap))
    _say(f"distance field, plain vs batched: {cfg_name} K={K}")
    sc = S.make_scene(cfg, K=K, steps=40)
    ref = run_plain(pt, sc, 3, cfg.T)
    for graph in (False, True):
        got = run_batched(pt, sc, 3, cfg.T, graph=graph)
        _assert_same(ref, got, f"graph={graph}")


def test_sdf_rejects_the_calls_it_does_not_support(pt):
    cfg = _sdf_cfg("small")
    sc = S.make_scene(cfg.with_(T=10), K=8, steps=12)
    b = pt.Batch.from_scene(sc, T=10)
    u_win = torch.as_tensor(sc.u[:11].astype(np.float32), device="cuda")
    gt = torch.zeros((10, 4, b.L, 1), device="cuda")
    env = torch.arange(8, dtype=torch.int32, device="cuda")
    start, warm0 = b.start_of(env)
    with pytest.raises(pt.PtError) as ei:
        b.window_grad(u_win, gt, env, start, warm0)
    assert ei.value.code == 5
    b.close()
