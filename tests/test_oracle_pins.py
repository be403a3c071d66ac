"""Pins of the FP64 oracle against closed forms, invariants, brute force and
published known answers (no GPU).  Each check names the passage or the piece
of mechanics it follows; the discrete model is the one documented in
oracle/oracle.h."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2002_12160_amd import scene as S
from tests import tiny

HERE = os.path.dirname(os.path.abspath(__file__))
G = 9.81


def _oracle(hand_rows, sph, nsph, inv, C_max=4, N=10, converged=True, **ck):
    return oracle.Oracle(np.array(hand_rows), sph, nsph, inv, tiny.consts(**ck), C_max=C_max, newton_iters=N,
                         D=1, converged=converged)


def _run(o, st, pr, steps, u=None, want=False):
    """Step one env `steps` times with a static hand; returns the history."""
    seg = o.hand_fk(np.zeros(o.D) if u is None else u)
    wkey, wr = o.new_warm(1)
    hist = []
    for _ in range(steps):
        cont, dg = o.env_step(seg, seg, 0, st, pr, wkey[0], wr[0])
        hist.append((st.copy(), cont.copy(), dg))
    return hist


# -------------------------------------------------------------------------
# Philox4x32-10 (published known-answer vectors)
# -------------------------------------------------------------------------

def test_philox_known_answers():
    path = os.path.join(HERE, "golden", "philox4x32_10_kat.txt")
    n = 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        assert oracle.philox4x32_10(w[0:4], w[4:6]) == w[6:10]
        n += 1
    assert n == 3


# -------------------------------------------------------------------------
# hand kinematics
# -------------------------------------------------------------------------

def test_fk_single_joint_closed_form():
    # link along +x from the origin, joint about +y: rotating by th takes the
    # tip to len (cos th, 0, -sin th)
    row = tiny.link_row((0, 0, 0), (0.05, 0, 0), 0.01, joint=0)
    sph, nsph, inv = tiny.single_sphere(0.01)
    o = _oracle([row], sph, nsph, inv)
    for th in (-0.7, 0.0, 0.3, 1.2):
        seg = o.hand_fk(np.array([th]))
        np.testing.assert_allclose(seg[0, :3], 0.0, atol=1e-15)
        np.testing.assert_allclose(seg[0, 3:], [0.05 * math.cos(th), 0, -0.05 * math.sin(th)], atol=1e-15)


def test_fk_planar_chain_closed_form():
    # the generated claw hand: each finger is a planar chain, so its tip lies at
    # base + sum_k len (cos phi_k e_in - sin phi_k e_z) with cumulative angles
    cfg = S.CONFIGS["small"]
    hand, mean = S.build_hand(cfg.hand)
    sph, nsph, inv = tiny.single_sphere(0.01)
    o = oracle.Oracle(hand, sph, nsph, inv, cfg.consts, C_max=4, newton_iters=1, D=len(mean))
    rng = np.random.default_rng(3)
    u = mean + rng.uniform(-0.5, 0.5, size=mean.shape)
    seg = o.hand_fk(u)
    hs = cfg.hand
    for f in range(hs.n_fingers):
        psi = 2 * math.pi * f / hs.n_fingers
        base = np.array([hs.base_radius * math.cos(psi), hs.base_radius * math.sin(psi), hs.base_height])
        e_in = -np.array([math.cos(psi), math.sin(psi), 0.0])
        p = base.copy()
        phi = 0.0
        for k in range(hs.links_per_finger):
            phi += u[3 * f + k]
            np.testing.assert_allclose(seg[3 * f + k, :3], p, atol=1e-14)
            p = p + hs.link_len * (math.cos(phi) * e_in - math.sin(phi) * np.array([0, 0, 1.0]))
            np.testing.assert_allclose(seg[3 * f + k, 3:], p, atol=1e-14)


# -------------------------------------------------------------------------
# free flight (P1, P2)
# -------------------------------------------------------------------------

def test_free_fall_closed_form():
    # semi-implicit Euler: v_n = v0 + n g dt, x_n = x0 + n dt v0 + g dt^2 n(n+1)/2
    sph, nsph, inv = tiny.single_sphere(0.01, inv_inertia=(2500.0, 2500.0, 2500.0))
    o = _oracle([tiny.far_link()], sph, nsph, inv)
    dt = o.consts.dt
    x0 = np.array([0.1, -0.2, 20.0])
    v0 = np.array([0.3, 0.1, 0.5])
    st = tiny.state(x=x0, v=v0)
    pr = tiny.params(0.2, 0.5)
    hist = _run(o, st, pr, 40)
    g = np.array([0, 0, -G])
    for n, (s, cont, dg) in enumerate(hist, start=1):
        assert len(cont) == 0
        np.testing.assert_allclose(s[7:10], v0 + n * g * dt, rtol=0, atol=1e-12)
        np.testing.assert_allclose(s[0:3], x0 + n * dt * v0 + g * dt * dt * n * (n + 1) / 2, rtol=0, atol=1e-12)


def test_free_flight_momentum_and_perturbation_force():
    # no contact: m dv = (m g + f) dt on the first step (f acts once), world
    # angular momentum I_w(q) w is conserved by construction, |q| = 1
    inv = (1 / 3e-4, 1 / 7e-4, 1 / 9e-4)
    sph, nsph, invv = tiny.single_sphere(0.01, inv_inertia=inv)
    o = _oracle([tiny.far_link()], sph, nsph, invv)
    dt = o.consts.dt
    m = 0.15
    f = np.array([0.3, -0.2, 0.1])
    q0 = np.array([0.9, 0.1, -0.3, 0.2])
    q0 /= np.linalg.norm(q0)
    st = tiny.state(x=(0, 0, 20.0), q=q0, v=(0.1, 0.0, 0.0), w=(3.0, -2.0, 5.0))
    pr = tiny.params(m, 0.5, f)

    def ang_mom(s):
        w, x, y, z = s[3:7]
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        Iw = R @ np.diag(m / np.array(inv)) @ R.T
        return Iw @ s[10:13]

    h0 = ang_mom(st)
    v_prev = st[7:10].copy()
    hist = _run(o, st, pr, 30)
    for n, (s, cont, dg) in enumerate(hist):
        expect = m * np.array([0, 0, -G]) * dt + (f * dt if n == 0 else 0)
        np.testing.assert_allclose(m * (s[7:10] - v_prev), expect, atol=1e-13)
        v_prev = s[7:10].copy()
        np.testing.assert_allclose(ang_mom(s), h0, rtol=1e-12, atol=1e-15)
        assert abs(np.linalg.norm(s[3:7]) - 1) < 1e-14
    assert np.all(pr[2:] == 0)  # the perturbation force is consumed by the step


# -------------------------------------------------------------------------
# resting contact (P3)
# -------------------------------------------------------------------------

def test_resting_single_sphere_closed_form():
    # steady state on the plane: v+ = 0 so r_n = m g dt; the smoothed cone
    # complementarity x o y = delta^2 e with no tangential impulse gives
    # u_n = delta^2/(kappa mu r_n) - mu delta, and u_n = eps r_n + erp d/dt.
    rho, m, mu = 0.01, 0.1, 0.6
    sph, nsph, inv = tiny.single_sphere(rho)  # translation-only body
    o = _oracle([tiny.far_link()], sph, nsph, inv)
    c = o.consts
    st = tiny.state(x=(0, 0, rho))
    pr = tiny.params(m, mu)
    hist = _run(o, st, pr, 400)
    s, cont, dg = hist[-1]
    assert len(cont) == 1
    rn = m * G * c.dt
    np.testing.assert_allclose(cont[0]["r"][0], rn, rtol=1e-10)
    np.testing.assert_allclose(cont[0]["r"][1:], 0.0, atol=1e-15)
    un = c.fb_delta ** 2 / (c.kappa * mu * rn) - mu * c.fb_delta
    d_ss = (un - c.compliance * rn) * c.dt / c.erp
    np.testing.assert_allclose(s[2] - rho, d_ss, rtol=1e-8)
    np.testing.assert_allclose(s[7:10], 0.0, atol=1e-12)


def test_resting_cuboid_total_normal_force():
    # 26-sphere cuboid lying flat: the 9 bottom spheres share the load and the
    # total normal impulse per step balances gravity, sum r_n / dt = m g
    cfg = S.CONFIGS["small"]
    sph, inv, _, _ = S.build_object(cfg.objects[0])
    o = oracle.Oracle(np.array([tiny.far_link()]), sph[None], np.array([len(sph)], np.int32), inv[None],
                      cfg.consts, C_max=16, newton_iters=10, D=1, converged=True)
    rest = S.rest_pose_of(sph)
    st = tiny.state(x=rest[:3])
    pr = tiny.params(0.1, 0.6)
    hist = _run(o, st, pr, 200)
    s, cont, dg = hist[-1]
    assert len(cont) == 9
    np.testing.assert_allclose(cont["r"][:, 0].sum() / o.consts.dt, 0.1 * G, rtol=1e-10)
    np.testing.assert_allclose(s[7:13], 0.0, atol=1e-10)


# -------------------------------------------------------------------------
# friction cone (P4)
# -------------------------------------------------------------------------

@pytest.mark.parametrize("mu,alpha_deg", [(0.5, 20.0), (0.5, 35.0), (0.3, 10.0), (0.3, 25.0)])
def test_sliding_onset_translation_only(mu, alpha_deg):
    # block on an incline (gravity tilted by alpha): it sticks iff
    # tan(alpha) <= mu, else it accelerates by g (sin a - mu cos a).  A stuck
    # contact creeps: the compliance acts on every constraint row (eps |r_t|)
    # and the smoothed cone complementarity x o y = delta^2 e leaves a
    # tangential constraint velocity delta^2 |r_t| / (mu kappa (mu^2 r_n^2 - r_t^2)).
    a = math.radians(alpha_deg)
    rho, m = 0.01, 0.1
    sph, nsph, inv = tiny.single_sphere(rho)
    o = _oracle([tiny.far_link()], sph, nsph, inv, gravity=(G * math.sin(a), 0.0, -G * math.cos(a)))
    c = o.consts
    dt = c.dt
    st = tiny.state(x=(0, 0, rho))
    pr = tiny.params(m, mu)
    hist = _run(o, st, pr, 160)
    vx = np.array([h[0][7] for h in hist])
    if math.tan(a) <= mu:
        rn, rt = m * G * math.cos(a) * dt, m * G * math.sin(a) * dt
        creep = c.compliance * rt + c.fb_delta ** 2 * rt / (mu * c.kappa * (mu * mu * rn * rn - rt * rt))
        np.testing.assert_allclose(vx[-20:], creep, rtol=1e-6)
    else:
        acc = np.diff(vx[-21:]) / dt
        np.testing.assert_allclose(acc, G * (math.sin(a) - mu * math.cos(a)), rtol=1e-6)


@pytest.mark.parametrize("mu,alpha_deg", [(0.2, 20.0), (0.1, 30.0)])
def test_rolling_sphere_acceleration(mu, alpha_deg):
    # solid sphere (I = 2/5 m r^2) rolls without slipping iff tan a <= 3.5 mu,
    # with a = 5/7 g sin a and friction 2/7 m g sin a (the contact point then
    # creeps as a stuck contact does, see above); otherwise it slides with
    # g (sin a - mu cos a)
    a = math.radians(alpha_deg)
    rho, m = 0.02, 0.1
    ii = 1.0 / (0.4 * rho * rho)
    sph, nsph, inv = tiny.single_sphere(rho, inv_inertia=(ii, ii, ii))
    o = _oracle([tiny.far_link()], sph, nsph, inv, gravity=(G * math.sin(a), 0.0, -G * math.cos(a)))
    c = o.consts
    dt = c.dt
    st = tiny.state(x=(0, 0, rho))
    pr = tiny.params(m, mu)
    hist = _run(o, st, pr, 160)
    vx = np.array([h[0][7] for h in hist])
    acc = np.diff(vx[-21:]) / dt
    if math.tan(a) <= 3.5 * mu:
        np.testing.assert_allclose(acc, 5.0 / 7.0 * G * math.sin(a), rtol=1e-6)
        wy = np.array([h[0][11] for h in hist])
        slip = vx[-20:] - wy[-20:] * rho
        rn, rt = m * G * math.cos(a) * dt, 2.0 / 7.0 * m * G * math.sin(a) * dt
        creep = c.compliance * rt + c.fb_delta ** 2 * rt / (mu * c.kappa * (mu * mu * rn * rn - rt * rt))
        np.testing.assert_allclose(slip, creep, rtol=1e-5)
    else:
        np.testing.assert_allclose(acc, G * (math.sin(a) - mu * math.cos(a)), rtol=1e-6)


# -------------------------------------------------------------------------
# energy (P5)
# -------------------------------------------------------------------------

def _energy(s, m, inv):
    w, x, y, z = s[3:7]
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    Iw = R @ np.diag(m / np.asarray(inv)) @ R.T
    return 0.5 * m * s[7:10] @ s[7:10] + 0.5 * s[10:13] @ Iw @ s[10:13] + m * G * s[2]


def test_energy_non_increasing_drop_and_slide():
    cfg = S.CONFIGS["small"]
    sph, inv, _, _ = S.build_object(cfg.objects[0])
    o = oracle.Oracle(np.array([tiny.far_link()]), sph[None], np.array([len(sph)], np.int32), inv[None],
                      cfg.consts, C_max=16, newton_iters=10, D=1, converged=True)
    rest = S.rest_pose_of(sph)
    m = 0.1
    # dropped from 4 cm above with a lateral velocity (it lands and slides)
    st = tiny.state(x=rest[:3] + np.array([0, 0, 0.04]), v=(0.3, 0.1, 0.0))
    pr = tiny.params(m, 0.4)
    e_prev = _energy(st, m, inv)
    hist = _run(o, st, pr, 90)
    touched = False
    for s, cont, dg in hist:
        e = _energy(s, m, inv)
        assert e <= e_prev + 1e-12
        e_prev = e
        touched |= len(cont) > 0 and np.any(cont["r"][:, 0] > 0)
    assert touched


# -------------------------------------------------------------------------
# complementarity certificate on converged solves (P6)
# -------------------------------------------------------------------------

def test_ncp_certificate_on_tracking_trajectory():
    cfg = S.CONFIGS["small"].with_(T=10 ** 6)
    sc = S.make_scene(cfg, K=8, steps=30)
    tr = oracle.Tracker(sc, converged=True)
    c = cfg.consts
    n_checked = 0
    n_sliding = 0
    for t in range(30):
        out = tr.step(want=True)
        for i in range(sc.K):
            dg = out["diag"][i]
            if dg["iters"] >= 100:   # did not converge: no certificate
                continue
            assert dg["psi_final"] < 1e-20
            mu = tr.params[i, 1]
            for ct in out["contacts"][i]:
                if ct["key"] < 0:
                    continue
                r, u = ct["r"], ct["u"]
                rt = math.hypot(r[1], r[2])
                ut = math.hypot(u[1], u[2])
                scale = max(1e-3, r[0])
                assert r[0] >= -1e-12
                assert rt <= mu * r[0] + 1e-9 * scale
                assert u[0] >= -2 * mu * c.fb_delta
                # r . u_hat with the smoothed tangential norm is delta^2/kappa/mu
                uhat = np.array([u[0] + mu * math.sqrt(ut * ut + c.fb_delta ** 2), u[1], u[2]])
                assert abs(r @ uhat) <= 2 * c.fb_delta ** 2 / (c.kappa * mu) + 1e-12
                if ut > 1e-3 and r[0] > 1e-6:
                    n_sliding += 1
                    # maximal dissipation: friction opposes the sliding velocity
                    cosang = (r[1] * u[1] + r[2] * u[2]) / (rt * ut)
                    assert cosang < -1 + 1e-6
                    # on the cone up to the smoothing: kappa (mu r_n - |r_t|) <= delta^2 / y0
                    y0 = mu * ut
                    assert 0 <= mu * r[0] - rt <= 2 * c.fb_delta ** 2 / (c.kappa * y0)
                n_checked += 1
    assert n_checked > 200
    assert n_sliding > 5


# -------------------------------------------------------------------------
# single contact: brute-force mode enumeration (P7)
# -------------------------------------------------------------------------

def _coulomb_brute_force(W, uf, mu):
    """Exact solution of the 3-D Coulomb contact problem u = W r + uf by
    enumerating separation, sticking and sliding (dense angle scan plus
    bisection for the sliding direction)."""
    if uf[0] >= 0:
        return np.zeros(3), "separate"
    r = -np.linalg.solve(W, uf)
    if r[0] > 0 and math.hypot(r[1], r[2]) <= mu * r[0]:
        return r, "stick"

    def resid(th):
        a = np.array([1.0, -mu * math.cos(th), -mu * math.sin(th)])
        wa = W @ a
        rn = -uf[0] / wa[0]
        u = rn * wa + uf
        return u[1] * math.sin(th) - u[2] * math.cos(th), rn, u, a

    ths = np.linspace(0, 2 * math.pi, 20001)
    vals = [resid(t)[0] for t in ths]
    sols = []
    for k in range(len(ths) - 1):
        if vals[k] == 0 or vals[k] * vals[k + 1] < 0:
            lo, hi = ths[k], ths[k + 1]
            flo = vals[k]
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                fm = resid(mid)[0]
                if (fm < 0) == (flo < 0):
                    lo, flo = mid, fm
                else:
                    hi = mid
            th = 0.5 * (lo + hi)
            _, rn, u, a = resid(th)
            s = u[1] * math.cos(th) + u[2] * math.sin(th)
            if rn > 0 and s > 0:
                sols.append(rn * a)
    assert len(sols) >= 1
    return sols[0], "slide"


def test_single_contact_matches_brute_force():
    rng = np.random.default_rng(7)
    modes = set()
    n = 0
    for trial in range(60):
        rho = 0.01
        off = rng.uniform(-0.02, 0.02, size=3)
        inv = 1.0 / rng.uniform(2e-4, 9e-4, size=3)
        sph, nsph, invv = tiny.single_sphere(rho, inv_inertia=inv, offset=off)
        o = _oracle([tiny.far_link()], sph, nsph, invv, C_max=1, fb_delta=1e-7)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        # place the object so that the sphere just touches the table
        w_, x_, y_, z_ = q
        R = np.array([[1 - 2 * (y_ * y_ + z_ * z_), 2 * (x_ * y_ - w_ * z_), 2 * (x_ * z_ + w_ * y_)],
                      [2 * (x_ * y_ + w_ * z_), 1 - 2 * (x_ * x_ + z_ * z_), 2 * (y_ * z_ - w_ * x_)],
                      [2 * (x_ * z_ - w_ * y_), 2 * (y_ * z_ + w_ * x_), 1 - 2 * (x_ * x_ + y_ * y_)]])
        x = np.array([0, 0, rho + rng.uniform(-0.002, 0.001)]) - R @ off
        st = tiny.state(x=x, q=q, v=rng.normal(scale=0.3, size=3), w=rng.normal(scale=3.0, size=3))
        pr = tiny.params(rng.uniform(0.05, 0.3), rng.uniform(0.2, 1.2))
        seg = o.hand_fk(np.zeros(1))
        cont, W, uf = o.env_system(seg, seg, 0, st, pr)
        if len(cont) != 1:
            continue
        rb, mode = _coulomb_brute_force(W, uf, pr[1])
        wkey, wr = o.new_warm(1)
        st2 = st.copy()
        cont2, dg = o.env_step(seg, seg, 0, st2, pr.copy(), wkey[0], wr[0])
        assert dg["iters"] < 100
        np.testing.assert_allclose(cont2[0]["r"], rb, atol=1e-6 * max(1e-3, np.abs(rb).max()))
        modes.add(mode)
        n += 1
    assert n >= 40
    assert modes == {"separate", "stick", "slide"}


# -------------------------------------------------------------------------
# narrow phase (P8)
# -------------------------------------------------------------------------

def test_narrow_phase_brute_force():
    rng = np.random.default_rng(11)
    for trial in range(40):
        a = rng.uniform(-0.05, 0.05, size=3) + np.array([0, 0, 0.5])
        b = a + rng.normal(scale=0.03, size=3)
        R = rng.uniform(0.004, 0.012)
        rho = rng.uniform(0.003, 0.01)
        row = tiny.link_row(a, b, R)
        sph, nsph, inv = tiny.single_sphere(rho)
        o = _oracle([row], sph, nsph, inv, C_max=2, margin=10.0)
        c = 0.5 * (a + b) + rng.normal(scale=0.04, size=3)
        st = tiny.state(x=c)
        seg = o.hand_fk(np.zeros(1))
        cont, W, uf = o.env_system(seg, seg, 0, st, tiny.params(0.1, 0.5))
        cap = cont[cont["link"] == 0][0]
        pl = cont[cont["link"] == 1][0]
        # brute force over the segment
        s = np.linspace(0, 1, 200001)[:, None]
        pts = a + s * (b - a)
        dist = np.linalg.norm(pts - c, axis=1)
        k = int(np.argmin(dist))
        assert abs(cap["d"] - (dist[k] - rho - R)) < 1e-9
        np.testing.assert_allclose(cap["n"], (c - pts[k]) / dist[k], atol=1e-4)
        np.testing.assert_allclose(cap["p"], c - rho * cap["n"], atol=1e-15)
        # plane
        assert abs(pl["d"] - (c[2] - rho)) < 1e-15
        np.testing.assert_allclose(pl["n"], [0, 0, 1])
        # the tangent frame is right-handed and orthonormal
        for ct in cont:
            F = np.stack([ct["n"], ct["t1"], ct["t2"]])
            np.testing.assert_allclose(F @ F.T, np.eye(3), atol=1e-14)
            assert np.linalg.det(F) > 0


def test_contact_cap_keeps_deepest():
    # 26-sphere cuboid pushed 3 mm into the table with a wide margin: the cap
    # keeps the C_max candidates with the smallest (d, key), i.e. the 9 bottom
    # spheres first, then the middle layer by key
    cfg = S.CONFIGS["small"]
    sph, inv, _, _ = S.build_object(cfg.objects[0])
    o = oracle.Oracle(np.array([tiny.far_link()]), sph[None], np.array([len(sph)], np.int32), inv[None],
                      tiny.consts(margin=0.05), C_max=12, newton_iters=2, D=1)
    rest = S.rest_pose_of(sph)
    st = tiny.state(x=rest[:3] - np.array([0, 0, 0.003]))
    seg = o.hand_fk(np.zeros(1))
    cont, W, uf = o.env_system(seg, seg, 0, st, tiny.params(0.1, 0.5))
    d_all = rest[2] - 0.003 + sph[:, 2] - sph[:, 3]
    order = sorted(range(len(sph)), key=lambda k: (d_all[k], k * 2 + 1))
    assert list(cont["key"]) == [k * 2 + 1 for k in order[:12]]
    np.testing.assert_allclose(cont["d"], d_all[order[:12]], atol=1e-15)


# -------------------------------------------------------------------------
# observation, cost, argmin (P9), ADD (P11)
# -------------------------------------------------------------------------

def test_observation_of_object_resting_on_a_link():
    # a ball resting on top of a horizontal capsule, far above the table: in
    # steady state the link feels the object's weight, straight down
    rho, m, R = 0.01, 0.12, 0.008
    row = tiny.link_row((-0.05, 0, 1.0), (0.05, 0, 1.0), R)
    sph, nsph, inv = tiny.single_sphere(rho)
    o = _oracle([row], sph, nsph, inv)
    st = tiny.state(x=(0, 0, 1.0 + R + rho))
    pr = tiny.params(m, 0.5)
    hist = _run(o, st, pr, 300)
    s, cont, dg = hist[-1]
    obs = o.observe(cont)
    np.testing.assert_allclose(obs[0, 0], m * G, rtol=1e-9)
    np.testing.assert_allclose(obs[0, 1:], [0, 0, -1], atol=1e-12)


def test_cost_identities():
    cfg = S.CONFIGS["small"]
    hand, mean = S.build_hand(cfg.hand)
    sph, nsph, inv = tiny.single_sphere(0.01)
    o = oracle.Oracle(hand, sph, nsph, inv, cfg.consts, C_max=4, newton_iters=1, D=len(mean))
    rng = np.random.default_rng(5)
    L = hand.shape[0]
    for _ in range(20):
        a = np.zeros((L, 4))
        b = np.zeros((L, 4))
        for o_ in (a, b):
            o_[:, 0] = rng.uniform(0, 5, size=L) * (rng.uniform(size=L) > 0.3)
            d = rng.normal(size=(L, 3))
            o_[:, 1:] = d / np.linalg.norm(d, axis=1, keepdims=True) * (o_[:, :1] > 0)
        assert o.step_cost(a, a) == 0.0
        cab, cba = o.step_cost(a, b), o.step_cost(b, a)
        assert cab == cba and cab >= 0
        # the direction term alone is at most 4 w_dir per sensor
        a2 = a.copy()
        a2[:, 0] = b[:, 0]
        assert o.step_cost(a2, b) <= 4 * cfg.consts.w_dir * L + 1e-12
        # magnitude-only difference is w_mag (|c| - |c_gt|)^2 summed
        b2 = b.copy()
        b2[:, 1:] = a[:, 1:]
        np.testing.assert_allclose(o.step_cost(a, b2), cfg.consts.w_mag * np.sum((a[:, 0] - b[:, 0]) ** 2))


def test_argmin_ties_and_nan():
    assert oracle.argmin([3.0, 1.0, 1.0, 2.0]) == 1
    assert oracle.argmin([np.nan, 5.0, np.nan]) == 1
    assert oracle.argmin([np.nan, np.nan]) == 0
    assert oracle.argmin([np.inf, np.nan, np.inf]) == 0
    assert oracle.argmin([2.0, -np.inf, 0.0]) == 1


def test_add_identities():
    cfg = S.CONFIGS["small"]
    sph, inv, _, _ = S.build_object(cfg.objects[0])
    o = oracle.Oracle(np.array([tiny.far_link()]), sph[None], np.array([len(sph)], np.int32), inv[None],
                      cfg.consts, C_max=4, newton_iters=1, D=1)
    p = np.array([0.01, 0.02, 0.03, 1, 0, 0, 0], dtype=np.float64)
    assert o.add(0, p, p) == 0.0
    t = np.array([0.003, -0.004, 0.0])
    p2 = p.copy()
    p2[:3] += t
    np.testing.assert_allclose(o.add(0, p, p2), 0.005, rtol=1e-14)
    th = 0.3
    axis = np.array([0.0, 0.0, 1.0])
    p3 = p.copy()
    p3[3:7] = [math.cos(th / 2), *(math.sin(th / 2) * axis)]
    perp = np.linalg.norm(sph[:, :2], axis=1)
    np.testing.assert_allclose(o.add(0, p, p3), np.mean(2 * perp * math.sin(th / 2)), rtol=1e-12)


# -------------------------------------------------------------------------
# resampler (P10) and window bookkeeping
# -------------------------------------------------------------------------

def _resample_setup(K=64, G=2, seed=0):
    cfg = S.CONFIGS["small"]
    sc = S.make_scene(cfg.with_(group_types=(0,) * G), K=K, steps=2)
    o = oracle.Oracle.from_scene(sc)
    rng = np.random.default_rng(seed)
    state = sc.state.copy()
    state[:, 7:13] = rng.normal(size=(K, 6))
    params = sc.params.copy()
    wkey = rng.integers(-1, 200, size=(K, o.C_max)).astype(np.int32)
    wr = rng.normal(size=(K, o.C_max, 3))
    cost = rng.uniform(0, 10, size=K)
    cost[5] = cost[6] = 1.0          # a tie
    cost[7] = np.nan                 # a divergent simulation
    return sc, o, state, params, wkey, wr, cost


def test_resample_elites_parents_and_copies():
    sc, o, state, params, wkey, wr, cost = _resample_setup()
    rc = oracle.resample_cfg(sc.cfg)
    s0, p0, k0, r0, c0 = state.copy(), params.copy(), wkey.copy(), wr.copy(), cost.copy()
    parent = o.resample(rc, sc.group_start, 3, cost, state, params, wkey, wr)
    assert np.all(cost == 0)
    for g in range(sc.G):
        lo, hi = sc.group_start[g], sc.group_start[g + 1]
        cg = np.where(np.isnan(c0[lo:hi]), np.inf, c0[lo:hi])
        order = lo + np.argsort(cg, kind="stable")
        kb = max(1, int(math.floor((hi - lo) * sc.cfg.elite_frac)))
        elites = set(order[:kb].tolist())
        for j in range(lo, hi):
            if j in elites:
                assert parent[j] == -1
                assert np.array_equal(state[j], s0[j]) and np.array_equal(params[j], p0[j])
                assert np.array_equal(wkey[j], k0[j]) and np.array_equal(wr[j], r0[j])
            else:
                pj = parent[j]
                assert pj in elites
                assert np.array_equal(state[j], s0[pj])
                assert np.array_equal(wkey[j], k0[pj]) and np.array_equal(wr[j], r0[pj])
                assert sc.cfg.mu_range[0] <= params[j, 1] <= sc.cfg.mu_range[1]
                assert sc.cfg.m_range[0] <= params[j, 0] <= sc.cfg.m_range[1]
                assert np.linalg.norm(params[j, 2:]) > 0
                # parent rank draw from the first Philox word of counter (j, window, 0, 0)
                w = oracle.philox4x32_10([j, 3, 0, 0], [sc.cfg.seed & 0xFFFFFFFF, sc.cfg.seed >> 32])
                assert pj == order[(w[0] * kb) >> 32]
    assert parent[7] != -1  # the NaN-cost simulation is never kept


def test_resample_perturbation_statistics():
    K = 8192
    cfg = S.CONFIGS["small"]
    sc = S.make_scene(cfg, K=K, steps=2)
    o = oracle.Oracle.from_scene(sc)
    state, params = sc.state.copy(), sc.params.copy()
    params[:, 1] = 0.65   # far from the clamps
    params[:, 0] = 0.125
    wkey, wr = o.new_warm(K)
    cost = np.arange(K, dtype=np.float64)
    rc = oracle.resample_cfg(cfg)
    parent = o.resample(rc, sc.group_start, 0, cost, state, params, wkey, wr)
    nonel = parent >= 0
    dmu = params[nonel, 1] - 0.65
    dm = params[nonel, 0] - 0.125
    f = params[nonel, 2:]
    n = nonel.sum()
    for x, sig in ((dmu, cfg.sigma_mu), (dm, cfg.sigma_m), (f[:, 0], cfg.sigma_f), (f[:, 2], cfg.sigma_f)):
        assert abs(x.mean()) < 4 * sig / math.sqrt(n)
        assert abs(x.std() / sig - 1) < 0.05
    # parents spread over all elites
    # (6144 draws over 2048 elites cover 1 - e^-3 = 95% of them on average)
    assert len(np.unique(parent[nonel])) > 0.9 * (K // 4)


def test_hidden_env_copy_has_zero_cost_and_is_best():
    cfg = S.CONFIGS["small"].with_(T=10 ** 6)
    sc = S.make_scene(cfg, K=8, steps=20)
    sc.state[3] = sc.hidden_state[0]
    sc.params[3] = sc.hidden_params[0]
    tr = oracle.Tracker(sc)
    for t in range(20):
        out = tr.step()
        assert tr.cost_sum[3] == 0.0
        assert out["best"][0] == int(np.argmin(np.where(tr.cost_sum == 0.0, -1.0, tr.cost_sum)))
    assert np.any(tr.cost_sum > 0)


def test_window_cost_matches_stepping():
    cfg = S.CONFIGS["small"]
    sc = S.make_scene(cfg, K=4, steps=12)
    o = oracle.Oracle.from_scene(sc)
    hs, hp = sc.hidden_state.copy(), sc.hidden_params.copy()
    hk, hr = o.new_warm(1)
    gts = []
    for t in range(10):
        obs, _, _ = o.batch_step(sc.hidden_type, sc.u[max(t - 1, 0)], sc.u[t], hs, hp, hk, hr)
        gts.append(obs[0])
    gts = np.array(gts)
    u_seq = np.concatenate([sc.u[:1], sc.u[:10]])
    st, pr = sc.state.copy(), sc.params.copy()
    wk, wr = o.new_warm(4)
    tot = np.zeros(4)
    for t in range(10):
        obs, _, _ = o.batch_step(sc.env_type, sc.u[max(t - 1, 0)], sc.u[t], st, pr, wk, wr)
        for i in range(4):
            tot[i] += o.step_cost(obs[i], gts[t])
    for i in range(4):
        assert o.window_cost(0, sc.state[i], sc.params[i], u_seq, gts) == tot[i]


# -------------------------------------------------------------------------
# orientation update (world-frame exponential, applied on the left)
# -------------------------------------------------------------------------

def _rot(axis, th):
    """Rotation matrix about a coordinate axis (0, 1, 2) by th."""
    c, s = math.cos(th), math.sin(th)
    if axis == 0:
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    if axis == 1:
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def _quat_to_R(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _rodrigues(axis, th):
    k = np.asarray(axis, dtype=np.float64) / np.linalg.norm(axis)
    Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * Kx + (1 - math.cos(th)) * Kx @ Kx


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_torque_free_spin_about_a_principal_axis_of_a_rotated_body(axis):
    # A body with three distinct principal inertias, turned away from the
    # world axes by q0, spins about its principal axis R0 e_axis with no
    # contact: the spin is steady, omega stays the same world vector, and
    # after n steps R_n = Rot(R0 e_axis, n dt |omega|) R0 (a rotation about a
    # world axis composed on the left).  A body-frame update would turn about
    # R0^T applied to omega instead and leave this closed form.
    inv = (1 / 3e-4, 1 / 7e-4, 1 / 9e-4)
    sph, nsph, invv = tiny.single_sphere(0.01, inv_inertia=inv)
    o = _oracle([tiny.far_link()], sph, nsph, invv, gravity=(0.0, 0.0, 0.0))
    dt = o.consts.dt
    q0 = np.array([0.8, 0.3, -0.4, 0.33])
    q0 /= np.linalg.norm(q0)
    R0 = _quat_to_R(q0)
    spin = 4.0
    w = spin * R0[:, axis]
    st = tiny.state(x=(0, 0, 20.0), q=q0, w=w)
    pr = tiny.params(0.12, 0.5)
    hist = _run(o, st, pr, 25)
    for n, (s, cont, dg) in enumerate(hist, start=1):
        np.testing.assert_allclose(s[10:13], w, rtol=0, atol=1e-12)
        Rn = _rodrigues(R0[:, axis], n * dt * spin) @ R0
        np.testing.assert_allclose(_quat_to_R(s[3:7]), Rn, rtol=0, atol=1e-12)
    # the body-frame reading differs visibly here
    R_body = R0 @ _rodrigues(w, 25 * dt * spin)
    assert np.abs(R_body - _quat_to_R(hist[-1][0][3:7])).max() > 0.1


# -------------------------------------------------------------------------
# kinematics: two joints on one link, offset rotations, a child link
# -------------------------------------------------------------------------

def test_fk_two_joints_and_offsets_closed_form():
    # link 0: origin o0, offset rotation Rz(yaw0), joint 0 about its local z
    # by a, then joint 1 about its (once turned) local y by b -- the
    # abduction-then-flexion order of the generated hands; link 1 hangs off
    # link 0's tip, moved by p1 in link 0's tip frame and turned by Rx(roll1),
    # with one joint about its local y by c; link 2 is a fixed palm capsule
    # (offset rotation only).  Frames compose as parent tip frame x offset x
    # joint0 x joint1, so R0 = Rz(yaw0) Rz(a) Ry(b): swapping the joints
    # gives Rz(yaw0) Ry(b) Rz(a), which moves the tip.
    yaw0, roll1, yaw2 = 0.7, -0.4, 2.1
    o0, p1, o2 = np.array([0.01, -0.02, 0.1]), np.array([0.004, 0.003, -0.002]), np.array([-0.03, 0.02, 0.09])
    len0, len1, len2 = 0.04, 0.035, 0.05
    rows = []
    r0 = np.zeros(20)
    r0[0], r0[1], r0[2] = -1, 0, 1
    r0[3:6], r0[6:9] = (0, 0, 1), (0, 1, 0)
    r0[9:12] = o0
    r0[12:16] = (math.cos(yaw0 / 2), 0, 0, math.sin(yaw0 / 2))
    r0[16], r0[17] = len0, 0.008
    rows.append(r0)
    r1 = np.zeros(20)
    r1[0], r1[1], r1[2] = 0, 2, -1
    r1[3:6] = (0, 1, 0)
    r1[9:12] = p1
    r1[12:16] = (math.cos(roll1 / 2), math.sin(roll1 / 2), 0, 0)
    r1[16], r1[17] = len1, 0.008
    rows.append(r1)
    r2 = np.zeros(20)
    r2[0], r2[1], r2[2] = -1, -1, -1
    r2[9:12] = o2
    r2[12:16] = (math.cos(yaw2 / 2), 0, 0, math.sin(yaw2 / 2))
    r2[16], r2[17] = len2, 0.008
    rows.append(r2)
    sph, nsph, inv = tiny.single_sphere(0.01)
    o = oracle.Oracle(np.array(rows), sph, nsph, inv, tiny.consts(), C_max=2, newton_iters=1, D=3)
    ex = np.array([1.0, 0.0, 0.0])
    rng = np.random.default_rng(21)
    for _ in range(6):
        a, b, c = rng.uniform(-1.2, 1.2, size=3)
        seg = o.hand_fk(np.array([a, b, c]))
        Rl0 = _rot(2, yaw0) @ _rot(2, a) @ _rot(1, b)
        tip0 = o0 + len0 * Rl0 @ ex
        np.testing.assert_allclose(seg[0, :3], o0, atol=1e-15)
        np.testing.assert_allclose(seg[0, 3:], tip0, atol=1e-15)
        base1 = tip0 + Rl0 @ p1
        Rl1 = Rl0 @ _rot(0, roll1) @ _rot(1, c)
        np.testing.assert_allclose(seg[1, :3], base1, atol=1e-15)
        np.testing.assert_allclose(seg[1, 3:], base1 + len1 * Rl1 @ ex, atol=1e-15)
        np.testing.assert_allclose(seg[2, :3], o2, atol=1e-15)
        np.testing.assert_allclose(seg[2, 3:], o2 + len2 * _rot(2, yaw2) @ ex, atol=1e-15)
        swapped = o0 + len0 * _rot(2, yaw0) @ _rot(1, b) @ _rot(2, a) @ ex
        assert np.abs(swapped - seg[0, 3:]).max() > 1e-4


# -------------------------------------------------------------------------
# the fixed-N Newton iteration and its Armijo schedule
# -------------------------------------------------------------------------

def _fb_spectral(x, y, delta):
    """Smoothed Fischer-Burmeister function of the second-order cone in R^3,
    from the spectral decomposition of the Jordan algebra: with
    z = x o x + y o y + 2 delta^2 e (a o a = (|a|^2, 2 a0 abar)),
    z = l1 c1 + l2 c2, l = z0 -/+ |zbar|, c = (1, -/+ zbar/|zbar|)/2 and
    sqrt(z) = sqrt(l1) c1 + sqrt(l2) c2; Phi = x + y - sqrt(z).  Written
    with sums of squares and principal square roots only, so that it also
    evaluates at complex arguments (for complex-step derivatives)."""
    z0 = np.sum(x * x) + np.sum(y * y) + 2 * delta * delta
    zb = 2 * (x[0] * x[1:] + y[0] * y[1:])
    nz = np.sqrt(np.sum(zb * zb))
    d = zb / nz if nz.real > 0 else np.array([1.0, 0.0])
    c1 = 0.5 * np.concatenate([[1.0], -d])
    c2 = 0.5 * np.concatenate([[1.0], d])
    root = np.sqrt(z0 - nz) * c1 + np.sqrt(z0 + nz) * c2
    return x + y - root


def _phi_all(r, W, uf, mu, c):
    """Phi of every contact at impulses r (3C): x = kappa (mu r_n, r_t),
    y = (u_n + mu sqrt(|u_t|^2 + delta^2), mu u_t), u = W r + uf."""
    u = W @ r + uf
    out = []
    for k in range(len(r) // 3):
        rk, uk = r[3 * k:3 * k + 3], u[3 * k:3 * k + 3]
        x = c.kappa * np.array([mu * rk[0], rk[1], rk[2]])
        y = np.array([uk[0] + mu * np.sqrt(uk[1] * uk[1] + uk[2] * uk[2] + c.fb_delta ** 2), mu * uk[1], mu * uk[2]])
        out.append(_fb_spectral(x, y, c.fb_delta))
    return np.concatenate(out)


def _newton_replay(r, W, uf, mu, c, N):
    """N iterations of Newton on Phi(r) = 0 with the Jacobian by complex-step
    differentiation (Im Phi(r + i h e_j) / h), each followed by the Armijo
    rule: the first a of 1, 1/2, 1/4, 1/8 with Psi(r + a dr) <=
    (1 - 2 sigma a) Psi(r), Psi = |Phi|^2/2, else 1/8.  Returns the
    iterates, the chosen step sizes, the smallest relative distance of a
    trial from its bound and the smallest merit met (below ~1e-18 the trials
    compare round-off, not the rule)."""
    alphas, margin, psi_min = [], np.inf, np.inf
    for _ in range(N):
        phi = _phi_all(r, W, uf, mu, c)
        psi = 0.5 * phi @ phi
        psi_min = min(psi_min, psi)
        n = len(r)
        A = np.zeros((n, n))
        for j in range(n):
            rc = r.astype(np.complex128)
            rc[j] += 1e-30j
            A[:, j] = _phi_all(rc, W, uf, mu, c).imag / 1e-30
        dr = np.linalg.solve(A, -phi)
        chosen = 0.125
        for a in (1.0, 0.5, 0.25, 0.125):
            pt = 0.5 * np.sum(_phi_all(r + a * dr, W, uf, mu, c) ** 2)
            bound = (1 - 2 * c.armijo_sigma * a) * psi
            margin = min(margin, abs(pt - bound) / psi)
            if pt <= bound:
                chosen = a
                break
        alphas.append(chosen)
        r = r + chosen * dr
    return r, alphas, margin, psi_min


def _replay_case(o, seg0, seg1, typ, st, pr, wkey, wr, N):
    """Oracle step with N fixed iterations against the replay from the same
    contact system and warm start.  Returns the replay's step sizes, or None
    when a trial lies too close to its bound (or the merit at round-off) for
    the replay's finite differences to decide it."""
    cont, W, uf = o.env_system(seg0, seg1, typ, st, pr)
    C = len(cont)
    if C == 0:
        return None
    r0 = np.zeros((C, 3))
    for k, key in enumerate(cont["key"]):
        hit = np.nonzero(wkey == key)[0]
        if len(hit):
            r0[k] = wr[hit[0]]
    r_rep, alphas, margin, psi_min = _newton_replay(r0.reshape(-1).copy(), W, uf, pr[1], o.consts, N)
    if margin < 1e-9 or psi_min < 1e-24:
        return None
    got, dg = o.env_step(seg0, seg1, typ, st.copy(), pr.copy(), wkey.copy(), wr.copy())
    r_or = np.concatenate([g["r"] for g in got])
    np.testing.assert_allclose(r_or, r_rep, rtol=0, atol=1e-8 * max(np.abs(r_rep).max(), 1e-4))
    assert dg["iters"] == N
    assert dg["n_full_steps"] == sum(a == 1.0 for a in alphas)
    assert dg["n_fallback"] <= sum(a == 0.125 for a in alphas)
    return alphas


def test_fixed_n_newton_and_armijo_schedule():
    # The oracle's impulses after N fixed iterations equal an independent
    # replay (spectral FB function, finite-difference Newton matrix, the
    # Armijo rule written out), on (a) one or two spheres of a body touching
    # the table with random velocities and warm starts (Armijo parameter
    # 1e-4, and 0.3 where the bound's sign decides many trials), and (b) steps of the
    # small tracking scene (hand contacts squeezing the object), for N = 1 to
    # 4.  The cases cover a full step (a = 1), a rejected full step with
    # a = 1/2 or 1/4 accepted, and the fallback a = 1/8 when no trial passes.
    rng = np.random.default_rng(17)
    seen = []
    for trial in range(120):
        rho = 0.01
        two = trial % 2 == 1
        offs = np.array([[0.0, 0.0, 0.0], [0.03, 0.0, 0.0]]) if two else np.zeros((1, 3))
        sph = np.zeros((1, len(offs), 4))
        sph[0, :, :3] = offs - offs.mean(axis=0)
        sph[0, :, 3] = rho
        inv = 1.0 / rng.uniform(2e-4, 9e-4, size=3)
        N = 1 if trial % 4 < 2 else 3
        # sigma = 0.3 on every other pair of cases: the same rule with a
        # sufficient-decrease band wide enough that its sign decides trials
        sigma = 0.3 if trial % 8 >= 4 else 1e-4
        o = oracle.Oracle(np.array([tiny.far_link()]), sph, np.array([len(offs)], np.int32), inv[None],
                          tiny.consts(armijo_sigma=sigma), C_max=4, newton_iters=N, D=1)
        st = tiny.state(x=(0, 0, rho + rng.uniform(-0.001, 0.0005)), v=rng.normal(scale=0.3, size=3),
                        w=rng.normal(scale=2.0, size=3))
        pr = tiny.params(rng.uniform(0.05, 0.3), rng.uniform(0.2, 1.2))
        seg = o.hand_fk(np.zeros(1))
        cont, _, _ = o.env_system(seg, seg, 0, st, pr)
        wkey, wr = o.new_warm(1)
        C = len(cont)
        wkey[0, :C] = cont["key"]
        wr[0, :C] = rng.normal(scale=0.01, size=(C, 3)) * (rng.uniform() < 0.8)
        a = _replay_case(o, seg, seg, 0, st, pr, wkey[0], wr[0], N)
        if a is not None:
            seen.append(a)
    n_table = len(seen)
    cfg = S.CONFIGS["small"].with_(T=10 ** 6)
    sc = S.make_scene(cfg, K=4, steps=16)
    tr = oracle.Tracker(sc)
    for t in range(16):
        if t >= 4:
            seg0, seg1 = tr.o.hand_fk(sc.u[t - 1]), tr.o.hand_fk(sc.u[t])
            for i in range(sc.K):
                for N in (1, 2, 4):
                    o = oracle.Oracle.from_scene(sc, newton_iters=N)
                    a = _replay_case(o, seg0, seg1, sc.env_type[i], tr.state[i], tr.params[i], tr.wkey[i],
                                     tr.wr[i], N)
                    if a is not None:
                        seen.append(a)
        tr.step()
    flat = [x for a in seen for x in a]
    assert n_table >= 80 and len(seen) - n_table >= 60
    assert {1.0, 0.5, 0.125} <= set(flat), set(flat)


def test_bench_tracking_error_is_the_oracles_add():
    # the benchmark's tracking error (ADD of the estimate against the
    # observed pose, its own numpy code) equals the oracle's ADD
    import bench
    cfg = S.CONFIGS["realtime16384"]
    sc = S.make_scene(cfg, K=16, steps=2)
    o = oracle.Oracle.from_scene(sc)
    rng = np.random.default_rng(4)
    for t in range(sc.spheres.shape[0]):
        pts = sc.spheres[t, :sc.n_spheres[t], :3]
        for _ in range(5):
            pa = np.concatenate([rng.normal(scale=0.01, size=3), rng.normal(size=4)])
            pb = np.concatenate([rng.normal(scale=0.01, size=3), rng.normal(size=4)])
            np.testing.assert_allclose(bench.add_distance(pts, pa, pb), o.add(t, pa, pb), rtol=1e-12)
