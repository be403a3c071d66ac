"""Pins of the oracle's full cost of Eq. 3 (contact-state, force, slip and
spin terms) and of its observation: hand-made observation pairs with known
angles and gates, and a sphere sliding and spinning on one capsule link
whose slip direction and spin sign follow from the set-up -- CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_2002_12160_amd.scene import ModelConsts
from tests import tiny

W = ModelConsts().w_eq3          # w4 .. w10


def _oracle(L=1, **kw):
    c = ModelConsts(cost_mode=1, **kw)
    hand = np.array([tiny.link_row((-0.1, 0, 0), (0.1, 0, 0), 0.01)] * L)
    # a solid sphere: principal inertia 2/5 m r^2
    sph, ns, inv = tiny.single_sphere(0.02, inv_inertia=(1 / (0.4 * 0.02 ** 2),) * 3)
    return oracle.Oracle(hand, sph, ns, inv, c, C_max=8, newton_iters=30, D=0)


def _obs(mag=0.0, chat=(0, 0, 0), d=(0, 0), rot=0.0):
    return np.array([mag, *chat, *d, rot], dtype=np.float64)


# ----------------------------------------------------------------- cost ----
def test_identical_observations_cost_nothing():
    o = _oracle(L=2)
    a = np.stack([_obs(1.2, (0, 0, 1), (0.6, 0.8), 1.0), _obs()])
    assert o.step_cost(a, a) == 0.0


def test_contact_state_gate():
    o = _oracle()
    # one side in contact, the other not: w4, whatever the magnitudes
    assert o.step_cost(_obs(1.0, (1, 0, 0))[None], _obs(0.005)[None]) == pytest.approx(W[0])
    # both out of contact: only the magnitude difference
    assert o.step_cost(_obs(0.004)[None], _obs(0.001)[None]) == pytest.approx(W[1] * 0.003)


def test_force_magnitude_and_angle():
    o = _oracle()
    a = _obs(2.0, (1, 0, 0))
    b = _obs(1.5, (0, 1, 0))
    assert o.step_cost(a[None], b[None]) == pytest.approx(W[1] * 0.5 + W[2] * math.pi / 2, rel=1e-12)
    c = _obs(1.5, (math.cos(0.3), math.sin(0.3), 0))
    assert o.step_cost(c[None], b[None]) == pytest.approx(W[2] * (math.pi / 2 - 0.3), rel=1e-9)


def test_slip_gate_and_angle():
    o = _oracle()
    base = dict(mag=1.0, chat=(0, 0, 1))
    a = _obs(**base, d=(1, 0))
    assert o.step_cost(a[None], _obs(**base, d=(-1, 0))[None]) == pytest.approx(W[4] * math.pi)
    assert o.step_cost(a[None], _obs(**base, d=(0, 1))[None]) == pytest.approx(W[4] * math.pi / 2)
    assert o.step_cost(a[None], _obs(**base)[None]) == pytest.approx(W[3])


def test_spin_gate_and_direction():
    o = _oracle()
    base = dict(mag=1.0, chat=(0, 0, 1))
    assert o.step_cost(_obs(**base, rot=1)[None], _obs(**base, rot=-1)[None]) == pytest.approx(W[6])
    assert o.step_cost(_obs(**base, rot=1)[None], _obs(**base, rot=1)[None]) == 0.0
    assert o.step_cost(_obs(**base, rot=-1)[None], _obs(**base)[None]) == pytest.approx(W[5])


def test_sensors_add_up():
    o = _oracle(L=3)
    a = np.stack([_obs(1.0, (1, 0, 0)), _obs(0.0), _obs(1.0, (0, 0, 1), (1, 0), 1)])
    b = np.stack([_obs(1.0, (1, 0, 0)), _obs(1.0, (0, 1, 0)), _obs(1.0, (0, 0, 1), (0, 1), -1)])
    want = W[0] + (W[4] * math.pi / 2 + W[6])
    assert o.step_cost(a, b) == pytest.approx(want, rel=1e-12)


# ---------------------------------------------------------- observation ----
def _slide(v, w, mu):
    """One step of a solid sphere (r 2 cm, 0.1 kg) resting on a capsule link
    along x, with velocity v and spin w (a point contact exerts no torque
    about its normal, so the spin about z stays)."""
    o = _oracle(gravity=(0.0, 0.0, -9.81))
    st = tiny.state(x=(0.0, 0.0, 0.03), v=v, w=w)[None].copy()
    pr = tiny.params(0.1, mu)[None].copy()
    wk, wr = o.new_warm(1)
    obs, cont, _ = o.batch_step(np.zeros(1, np.int32), np.zeros(0), np.zeros(0), st, pr, wk, wr,
                                want_contacts=True)
    return obs[0, 0], cont[0], st[0]


def test_sliding_along_the_link_axis():
    ob, cont, st = _slide((0.1, 0.0, 0.0), (0.0, 0.0, 1.0), 0.05)
    assert ob[0] == pytest.approx(0.1 * 9.81, rel=0.05)              # resting weight
    # force on the link: the weight down and, while sliding, Coulomb
    # friction mu N dragging it along the slip
    np.testing.assert_allclose(ob[1:4], np.array([0.05, 0, -1]) / math.hypot(1, 0.05), atol=1e-4)
    np.testing.assert_allclose(ob[4:6], [1, 0], atol=1e-9)            # slides along +axis
    assert ob[6] == 1.0                                               # spins + about the normal (+z)


def test_sliding_backwards_and_sideways():
    ob, _, _ = _slide((-0.1, 0.0, 0.0), (0.0, 0.0, -1.0), 0.05)
    np.testing.assert_allclose(ob[4:6], [-1, 0], atol=1e-9)
    assert ob[6] == -1.0
    # +y: e1 = x (the axis), e2 = n x e1 = z x x = +y
    ob, _, _ = _slide((0.0, 0.1, 0.0), (0.0, 0.0, 0.0), 0.05)
    np.testing.assert_allclose(ob[4:6], [0, 1], atol=1e-6)
    assert ob[6] == 0.0


def test_sticking_contact_does_not_slip():
    ob, cont, st = _slide((0.01, 0.0, 0.0), (0.0, 0.0, 0.0), 1.0)
    assert ob[0] > 0.5
    assert ob[4] == 0.0 and ob[5] == 0.0 and ob[6] == 0.0


def test_slip_velocity_is_the_kinematic_one():
    # the slip speed that decides the gate is the relative velocity of the
    # contact points (u - eps r): the sphere's velocity after the step plus
    # omega x rho at the contact point (the link is still)
    o = _oracle(gravity=(0.0, 0.0, -9.81))
    st = tiny.state(x=(0.0, 0.0, 0.03), v=(0.1, 0.0, 0.0))[None].copy()
    pr = tiny.params(0.1, 0.05)[None].copy()
    wk, wr = o.new_warm(1)
    _, cont, _ = o.batch_step(np.zeros(1, np.int32), np.zeros(0), np.zeros(0), st, pr, wk, wr,
                              want_contacts=True)
    c = cont[0][cont[0]["key"] >= 0][0]
    eps = ModelConsts().compliance
    vt = (c["u"][1] - eps * c["r"][1]) * c["t1"] + (c["u"][2] - eps * c["r"][2]) * c["t2"]
    rho = c["p"] - np.array([0.0, 0.0, 0.03])
    vp = st[0, 7:10] + np.cross(st[0, 10:13], rho)
    np.testing.assert_allclose(vt, [vp[0], vp[1], 0.0], atol=1e-6)
