"""Pins of the oracle's PD-controlled hand (joint angles and rates as state,
an implicit PD law toward the commands, contacts coupling the object and the
finger chains) against closed forms of rigid-body mechanics (no GPU)."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2002_12160_amd import scene as S
from tests import tiny

M_LINK = 0.03


def _pd_consts(**kw):
    kw.setdefault("hand_mode", 1)
    kw.setdefault("link_mass", M_LINK)
    return tiny.consts(**kw)


def _cyl(length, radius, m=M_LINK):
    """(axial, transverse) inertia of a solid cylinder about its centre."""
    return 0.5 * m * radius * radius, m * (3 * radius * radius + length * length) / 12.0


def test_mass_matrix_of_a_planar_two_link_chain():
    # two links along +x, both joints about y (a planar 2R arm in the x-z
    # plane): the textbook joint-space inertia with centres of mass at the
    # link midpoints, c_i = l_i / 2 and transverse inertias I_i
    l1, l2, R = 0.05, 0.04, 0.008
    r1 = tiny.link_row((0, 0, 0), (l1, 0, 0), R, joint=0, axis=(0, 1, 0))
    r2 = tiny.link_row((0, 0, 0), (l2, 0, 0), R, parent=0, joint=1, axis=(0, 1, 0))
    r2[9:12] = 0.0                    # the child starts at the parent's tip
    sph, nsph, inv = tiny.single_sphere(0.01)
    o = oracle.Oracle(np.array([r1, r2]), sph, nsph, inv, _pd_consts(), C_max=2, newton_iters=1, D=2)
    _, I1 = _cyl(l1, R)
    _, I2 = _cyl(l2, R)
    c1, c2, m = l1 / 2, l2 / 2, M_LINK
    for q1, q2 in ((0.0, 0.0), (0.3, -0.7), (-1.1, 1.4), (0.5, 2.5)):
        M = o.hand_mass(np.array([q1, q2]))
        M11 = I1 + I2 + m * c1 ** 2 + m * (l1 ** 2 + c2 ** 2 + 2 * l1 * c2 * math.cos(q2))
        M12 = I2 + m * (c2 ** 2 + l1 * c2 * math.cos(q2))
        M22 = I2 + m * c2 ** 2
        np.testing.assert_allclose(M, [[M11, M12], [M12, M22]], rtol=1e-12, atol=1e-18)


def test_mass_matrix_of_a_link_spinning_about_its_axis():
    # a joint along the link's own axis: its centre of mass does not move,
    # only the axial inertia m R^2 / 2 counts; with a second joint about y
    # at the same origin the two rotations are orthogonal, so M is diagonal
    l, R = 0.04, 0.01
    row = tiny.link_row((0, 0, 0), (l, 0, 0), R, joint=0, axis=(1, 0, 0))
    row[2] = 1
    row[6:9] = (0, 1, 0)
    sph, nsph, inv = tiny.single_sphere(0.01)
    o = oracle.Oracle(np.array([row]), sph, nsph, inv, _pd_consts(), C_max=2, newton_iters=1, D=2)
    Ia, It = _cyl(l, R)
    for q1 in (0.0, 0.7):
        M = o.hand_mass(np.array([q1, 0.0]))
        # joint 0 (about x) first, then joint 1 about the turned y axis: its
        # rotation is transverse, about the link's base
        np.testing.assert_allclose(M, [[Ia, 0.0], [0.0, It + M_LINK * (l / 2) ** 2]], rtol=1e-12, atol=1e-18)


@pytest.mark.parametrize("kp,kd", [(1.5, 0.05), (0.05, 0.001), (20.0, 0.0)])
def test_free_pd_joint_follows_the_discrete_closed_form(kp, kd):
    # one link turning about y at its base, nothing to touch: the implicit PD
    # step is the linear recurrence x_{n+1} = A x_n for x = (q - u, qdot)
    # with a = I + dt kd + dt^2 kp:
    #   qdot+ = (I qdot - dt kp (q - u)) / a,   q+ = q + dt qdot+,
    # solved in closed form by the eigen-decomposition of A: x_n = V L^n V^-1 x_0
    l, R = 0.045, 0.008
    row = tiny.link_row((0, 0, 0), (l, 0, 0), R, joint=0, axis=(0, 1, 0))
    sph, nsph, inv = tiny.single_sphere(0.01)
    c = _pd_consts(kp=kp, kd=kd, gravity=(0.0, 0.0, 0.0))
    o = oracle.Oracle(np.array([row]), sph, nsph, inv, c, C_max=2, newton_iters=4, D=1)
    _, It = _cyl(l, R)
    I = It + M_LINK * (l / 2) ** 2            # parallel axes: about the joint
    dt, u = c.dt, 0.4
    a = I + dt * kd + dt * dt * kp
    A = np.array([[1 - dt * dt * kp / a, dt * I / a], [-dt * kp / a, I / a]])
    lam, V = np.linalg.eig(A)
    x0 = np.array([0.1 - u, -0.3])
    coef = np.linalg.solve(V, x0)
    st = tiny.state(x=(5.0, 5.0, 5.0))
    pr = tiny.params(0.1, 0.5)
    hq = np.array([0.1, -0.3])
    wk, wr = o.new_warm(1)
    for n in range(1, 61):
        cont, _ = o.env_step_pd(np.array([u]), 0, st, pr, hq, wk[0], wr[0])
        assert len(cont) == 0
        xn = (V @ (lam ** n * coef)).real
        np.testing.assert_allclose(hq, [u + xn[0], xn[1]], rtol=0, atol=1e-12)
    assert abs(hq[0] - u) < 1e-2 * abs(0.1 - u) or kp < 0.1


def test_finger_pressing_a_fixed_object_balances_its_pd_torque():
    # a finger (one link, joint about y at its base) commanded to turn down
    # into a ball that cannot move (a huge mass, no rotation, no gravity):
    # at rest the PD torque kp (u - q) balances the moment about the joint
    # of the contact force on the link, and the sensor reads that force
    l, R, rho = 0.05, 0.008, 0.01
    z0 = 0.5                                            # far above the table
    row = tiny.link_row((0, 0, z0), (l, 0, z0), R, joint=0, axis=(0, 1, 0))
    sph, nsph, inv = tiny.single_sphere(rho)            # translation only (inv = 0)
    c = _pd_consts(gravity=(0.0, 0.0, 0.0))
    o = oracle.Oracle(np.array([row]), sph, nsph, inv, c, C_max=4, newton_iters=30, D=1, converged=True)
    # the ball under the link, 4 cm out along it: turning about +y by a
    # positive angle takes the tip down (-z)
    xb = np.array([0.04, 0.0, z0 - (R + rho) - 0.002])
    st = tiny.state(x=xb)
    pr = tiny.params(1e15, 0.5)
    u = 0.5
    hq = np.array([0.0, 0.0])
    wk, wr = o.new_warm(1)
    for _ in range(400):
        cont, dg = o.env_step_pd(np.array([u]), 0, st, pr, hq, wk[0], wr[0])
    assert len(cont) == 1 and dg["iters"] < 30
    q = hq[0]
    assert 0 < q < u and abs(hq[1]) < 1e-9
    ct = cont[0]
    f_obj = (ct["r"][0] * ct["n"] + ct["r"][1] * ct["t1"] + ct["r"][2] * ct["t2"]) / c.dt
    f_link = -f_obj
    axis = np.array([0.0, 1.0, 0.0])                    # the joint axis does not move (no parent)
    tau_c = axis @ np.cross(ct["p"] - np.array([0.0, 0.0, z0]), f_link)
    np.testing.assert_allclose(c.kp * (u - q) + tau_c, 0.0, atol=1e-9 * c.kp * (u - q))
    obs = o.observe(cont)
    np.testing.assert_allclose(obs[0, 0], np.linalg.norm(f_link), rtol=1e-12)
    np.testing.assert_allclose(obs[0, 1:], f_link / np.linalg.norm(f_link), atol=1e-12)
    np.testing.assert_allclose(st[:3], xb, atol=1e-12)   # the ball did not move


def test_pd_tracking_scene_steps_and_resamples():
    # the small tracking scene with PD fingers: the hands start at the first
    # command, contacts move them off it, a copy of the observed simulation
    # has cost 0 (its hand follows the observed hand), and resampling copies
    # a parent's hand state with its body
    cfg = S.CONFIGS["small"]
    cfg = cfg.with_(consts=dataclasses.replace(cfg.consts, hand_mode=1), T=10)
    sc = S.make_scene(cfg, K=12, steps=25)
    sc.state[4] = sc.hidden_state[0]
    sc.params[4] = sc.hidden_params[0]
    tr = oracle.Tracker(sc)
    moved = 0.0
    for t in range(25):
        out = tr.step()
        assert tr.cost_sum[4] == 0.0 or out["parent"] is not None
        if out["parent"] is not None:
            par = out["parent"]
            for j in np.nonzero(par >= 0)[0]:
                assert np.array_equal(tr.hand[j], tr.hand[par[j]])
        moved = max(moved, float(np.abs(tr.hand[:, :sc.D] - sc.u[t]).max()))
    assert moved > 1e-3          # contacts hold fingers off their commands
