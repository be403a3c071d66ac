"""The contact cap on the GPU at every candidate count the kernel ranks
differently (up to 64, 128, 192 and 256 candidates held in registers,
beyond that ranked through LDS) against the oracle: a row of spheres squeezed between the
table and one long capsule link, every sphere a candidate of both, with
well-separated seeded gaps, so the C_max kept keys are exact integers."""
import numpy as np
import pytest
import torch

import oracle
from tests import tiny

pytestmark = pytest.mark.gpu

R_SPH = 0.004
R_LINK = 0.006


@pytest.fixture(scope="module")
def pt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_12160_amd import pt as _pt
    return _pt


def _row(S, seed):
    """S spheres along x, 5 mm apart, resting on the table with height offsets
    that are a seeded permutation of a 20 um grid (so every gap to the table
    and to the link above differs by far more than float32 rounding)."""
    rng = np.random.default_rng(seed)
    dz = (rng.permutation(S) - S / 2) * 2e-5
    sph = np.zeros((1, S, 4))
    sph[0, :, 0] = (np.arange(S) - (S - 1) / 2) * 0.005
    sph[0, :, 2] = dz
    sph[0, :, 3] = R_SPH
    return sph.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("S,C_max", [(24, 1), (24, 16), (20, 64), (50, 32), (80, 32), (100, 32), (128, 64), (200, 16)])
def test_cap_keeps_the_oracles_keys(pt, S, C_max):
    ncand = 2 * S
    print(f"cap: {S} spheres, {ncand} candidates, C_max {C_max}", flush=True)
    sph = _row(S, seed=S)
    half = 0.005 * S / 2 + 0.01
    # link gaps 1.05e-4 - dz: a quarter grid step off every table gap
    z_link = 2 * R_SPH + R_LINK + 1.05e-4
    hand = np.array([tiny.link_row((-half, 0.0, z_link), (half, 0.0, z_link), R_LINK)])
    inv = np.array([[50.0, 50.0, 50.0]])
    st = tiny.state(x=(0.0, 0.0, R_SPH))[None]
    pr = tiny.params(0.1, 0.5)[None]
    c = tiny.consts()
    o = oracle.Oracle(hand, sph, np.array([S], np.int32), inv, c, C_max=C_max, newton_iters=10, D=0)
    ost, opr = st.copy(), pr.copy()
    wk, wr = o.new_warm(1)
    o.batch_step(np.zeros(1, np.int32), np.zeros(0), np.zeros(0), ost, opr, wk, wr)
    b = pt.Batch(hand=hand, spheres=sph, n_spheres=np.array([S], np.int32), inv_inertia=inv,
                 env_type=np.zeros(1, np.int32), group_start=np.array([0, 1], np.int32), consts=c,
                 C_max=C_max, newton_iters=10, T=10, state=st, params=pr)
    u = torch.zeros(1, device="cuda")
    b.step(u, u)
    gk, _ = b.get_warm()
    stats = b.read_stats()
    b.close()
    assert stats["candidates"] == ncand
    kept = min(ncand, C_max)
    assert stats["contacts"] == kept
    assert (gk[0] >= 0).sum() == kept and (wk[0] >= 0).sum() == kept
    # every candidate is both sphere-table and sphere-link: the kept keys are
    # the C_max smallest gaps (all of them below the cap), the same set on
    # both sides
    assert sorted(gk[0][gk[0] >= 0].tolist()) == sorted(wk[0][wk[0] >= 0].tolist())


@pytest.mark.parametrize("S,C_max", [(100, 32), (128, 64), (200, 16)])
def test_cap_ties_keep_the_lowest_keys(pt, S, C_max):
    """Every sphere of a flat row rests on the table: S sphere-table gaps of
    exactly 0 on both sides (all below the link's), more than C_max of them,
    so the cap's boundary lies inside a tie of gaps and the key decides: the
    C_max lowest keys, sphere-table contacts of spheres 0 .. C_max - 1."""
    ncand = 2 * S
    print(f"cap ties: {S} spheres at gap 0, {ncand} candidates, C_max {C_max}", flush=True)
    sph = np.zeros((1, S, 4))
    sph[0, :, 0] = (np.arange(S) - (S - 1) / 2) * 0.005
    sph[0, :, 3] = R_SPH
    sph = sph.astype(np.float32).astype(np.float64)
    half = 0.005 * S / 2 + 0.01
    z_link = 2 * R_SPH + R_LINK + 1.05e-4
    hand = np.array([tiny.link_row((-half, 0.0, z_link), (half, 0.0, z_link), R_LINK)])
    inv = np.array([[50.0, 50.0, 50.0]])
    st = tiny.state(x=(0.0, 0.0, R_SPH))[None]
    pr = tiny.params(0.1, 0.5)[None]
    c = tiny.consts()
    o = oracle.Oracle(hand, sph, np.array([S], np.int32), inv, c, C_max=C_max, newton_iters=10, D=0)
    ost, opr = st.copy(), pr.copy()
    wk, wr = o.new_warm(1)
    o.batch_step(np.zeros(1, np.int32), np.zeros(0), np.zeros(0), ost, opr, wk, wr)
    b = pt.Batch(hand=hand, spheres=sph, n_spheres=np.array([S], np.int32), inv_inertia=inv,
                 env_type=np.zeros(1, np.int32), group_start=np.array([0, 1], np.int32), consts=c,
                 C_max=C_max, newton_iters=10, T=10, state=st, params=pr)
    u = torch.zeros(1, device="cuda")
    b.step(u, u)
    gk, _ = b.get_warm()
    stats = b.read_stats()
    b.close()
    assert stats["candidates"] == ncand
    assert stats["contacts"] == C_max
    want = sorted(wk[0][wk[0] >= 0].tolist())
    assert want == [2 * k + 1 for k in range(C_max)]      # key k (L + 1) + L of the table pair, L = 1
    assert sorted(gk[0][gk[0] >= 0].tolist()) == want
