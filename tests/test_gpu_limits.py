"""The library at its largest declared sizes against the oracle: 62 capsule
links (PT_MAX_LINKS) with two joints each (124 commands), objects of 256
spheres (PT_MAX_SPHERES), a 64-contact cap, and every one of the
256 x 63 sphere-link and sphere-table pairs a candidate, i.e. the candidate
list filled to its capacity.  One step of two simulations (one of them
shifted); the kept keys are exact integers and the state follows the usual
parity rule."""
import numpy as np
import pytest
import torch

import oracle
from tests import parity_util as PU
from tests import tiny

pytestmark = pytest.mark.gpu

L_MAX = 62
S_MAX = 256
R_SPH = 0.004
R_LINK = 0.006


@pytest.fixture(scope="module")
def pt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_12160_amd import pt as _pt
    return _pt


def _scene():
    """256 spheres in a row resting on the table (heights a seeded
    permutation of a 20 um grid) under 62 parallel capsule links stacked
    3.7 um apart in height: every sphere is within the margin of every link."""
    rng = np.random.default_rng(62)
    S = S_MAX
    sph = np.zeros((1, S, 4))
    sph[0, :, 0] = (np.arange(S) - (S - 1) / 2) * 0.005
    sph[0, :, 2] = (rng.permutation(S) - S / 2) * 2e-5
    sph[0, :, 3] = R_SPH
    sph = sph.astype(np.float32).astype(np.float64)
    half = 0.005 * S / 2 + 0.01
    rows = []
    for l in range(L_MAX):
        # heights 3.7 um apart: with the 20 um grid of the sphere heights,
        # every gap differs from every other by at least 0.1 um
        z = 2 * R_SPH + R_LINK + 1.05e-4 + 3.7e-6 * l
        r = tiny.link_row((-half, 0.0, z), (half, 0.0, z), R_LINK)
        r[1] = l              # a joint about y and
        r[2] = L_MAX + l      # a second one about z, at zero angle
        r[6:9] = (0.0, 0.0, 1.0)
        rows.append(r)
    hand = np.array(rows).astype(np.float32).astype(np.float64)
    return hand, sph


def test_largest_sizes_match_the_oracle(pt):
    D = 2 * L_MAX
    C_max = 64
    hand, sph = _scene()
    ns = np.array([S_MAX], np.int32)
    inv = np.array([[40.0, 40.0, 40.0]])
    st = np.stack([tiny.state(x=(0.0, 0.0, R_SPH)), tiny.state(x=(0.0012, 0.0, R_SPH))])
    pr = np.stack([tiny.params(0.2, 0.5), tiny.params(0.2, 0.8)])
    c = tiny.consts()
    u = np.zeros(D)
    print(f"largest sizes: L={L_MAX}, D={D}, S={S_MAX}, C_max={C_max}, {S_MAX * (L_MAX + 1)} candidates", flush=True)
    o = oracle.Oracle(hand, sph, ns, inv, c, C_max=C_max, newton_iters=10, D=D)
    ost, opr = st.copy(), pr.copy()
    wk, wr = o.new_warm(2)
    _, _, dg = o.batch_step(np.zeros(2, np.int32), u, u, ost, opr, wk, wr, want_diag=True)
    b = pt.Batch(hand=hand, spheres=sph, n_spheres=ns, inv_inertia=inv, env_type=np.zeros(2, np.int32),
                 group_start=np.array([0, 2], np.int32), consts=c, C_max=C_max, newton_iters=10, T=10,
                 state=st, params=pr)
    ut = torch.zeros(D, device="cuda")
    b.step(ut, ut)
    g_st, _ = b.get_state()
    gk, _ = b.get_warm()
    stats = b.read_stats()
    b.close()
    assert stats["candidates"] == 2 * S_MAX * (L_MAX + 1)
    assert stats["contacts"] == 2 * C_max
    for i in range(2):
        assert sorted(gk[i].tolist()) == sorted(wk[i].tolist()), i
    err = PU.rel_err(g_st, ost).max(axis=1)
    assert np.all(err <= PU.TOL), err
