"""Pins of the oracle's distance-field collision (collision_mode 1, the
simplified collision geometry of Sec. IV-A as a signed distance field): the
trilinear field against affine fields it must reproduce exactly, against
its own nodes and cell centres, and outside its box; a link over a flat
face against the closed-form gap, normal and contact point; an object
resting on a link against its weight (no GPU)."""
import math

import numpy as np
import pytest

import oracle
from tests import tiny

G = 9.81


def _grid(fn, n=12, half=0.06):
    """Node values of fn on a cubic grid [1][n][n][n] (z, y, x) and its box."""
    h = 2.0 * half / (n - 1)
    xs = -half + h * np.arange(n)
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    return fn(np.stack([X, Y, Z], axis=-1))[None], np.array([[-half, -half, -half, h]])


def _box_field(hx, hy, hz):
    a = np.array([hx, hy, hz])

    def f(P):
        q = np.abs(P) - a
        return np.linalg.norm(np.maximum(q, 0.0), axis=-1) + np.minimum(q.max(axis=-1), 0.0)
    return f


def _oracle(rows, sdf, box, C_max=16, N=10, converged=True, samples=8):
    sph, nsph, inv = tiny.single_sphere(0.005)
    c = tiny.consts(collision_mode=1, link_samples=samples)
    return oracle.Oracle(np.array(rows), sph, nsph, inv, c, C_max=C_max, newton_iters=N, D=1, converged=converged,
                         sdf=sdf, sdf_box=box)


def test_trilinear_field_reproduces_affine_fields():
    rng = np.random.default_rng(1)
    nrm = rng.normal(size=3)
    nrm /= np.linalg.norm(nrm)
    c0, half = 0.013, 0.06
    sdf, box = _grid(lambda P: P @ nrm - c0, half=half)
    o = _oracle([tiny.far_link()], sdf, box)
    for p in rng.uniform(-half, half, size=(200, 3)):
        v, g = o.sdf_eval(0, p)
        assert abs(v - (p @ nrm - c0)) < 1e-13
        np.testing.assert_allclose(g, nrm, atol=1e-12)
    # outside the box: the value at the nearest box point plus the distance to it
    for p in rng.uniform(-0.12, 0.12, size=(100, 3)):
        c = np.clip(p, -half, half)
        v, _ = o.sdf_eval(0, p)
        assert abs(v - (c @ nrm - c0 + np.linalg.norm(p - c))) < 1e-13


def test_trilinear_field_passes_through_its_nodes_and_averages_a_cell():
    rng = np.random.default_rng(2)
    n, half = 10, 0.05
    h = 2.0 * half / (n - 1)
    vals = rng.normal(size=(1, n, n, n))
    box = np.array([[-half, -half, -half, h]])
    o = _oracle([tiny.far_link()], vals, box)
    for _ in range(100):
        i, j, k = rng.integers(0, n, size=3)
        v, _ = o.sdf_eval(0, np.array([-half + i * h, -half + j * h, -half + k * h]))
        assert abs(v - vals[0, k, j, i]) < 1e-12
    for _ in range(50):
        i, j, k = rng.integers(0, n - 1, size=3)
        v, g = o.sdf_eval(0, np.array([-half + (i + 0.5) * h, -half + (j + 0.5) * h, -half + (k + 0.5) * h]))
        cell = vals[0, k:k + 2, j:j + 2, i:i + 2]
        assert abs(v - cell.mean()) < 1e-12
        # the gradient at the centre: mean difference across each axis / h
        np.testing.assert_allclose(g, [(cell[:, :, 1] - cell[:, :, 0]).mean() / h,
                                       (cell[:, 1, :] - cell[:, 0, :]).mean() / h,
                                       (cell[1] - cell[0]).mean() / h], rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("yaw", [0.0, 0.5])
def test_link_over_a_flat_face(yaw):
    # above the middle of a box's top face its field is z - hz, which the
    # grid reproduces exactly: every sample of a horizontal link there is a
    # contact with gap (height above the face - radius), normal straight
    # down and its contact point on the face below the sample
    hx, hy, hz = 0.03, 0.025, 0.01
    sdf, box = _grid(_box_field(hx, hy, hz), n=33, half=0.05)
    R, z0, gap, M = 0.006, 0.3, 0.003, 8
    zl = z0 + hz + R + gap
    a, b = np.array([-0.015, 0.004, zl]), np.array([0.015, 0.004, zl])
    o = _oracle([tiny.link_row(a, b, R)], sdf, box, C_max=32, samples=M)
    st = tiny.state(x=(0.0, 0.0, z0), q=(math.cos(yaw / 2), 0.0, 0.0, math.sin(yaw / 2)))
    seg = o.hand_fk(np.zeros(1))
    cont, _, _ = o.env_system(seg, seg, 0, st, tiny.params(0.1, 0.5))
    assert len(cont) == M
    assert sorted(int(c["key"]) for c in cont) == [2 * k for k in range(M)]
    for c in cont:
        s = a + (c["key"] // 2) / (M - 1) * (b - a)
        assert c["link"] == 0
        np.testing.assert_allclose(c["d"], gap, atol=1e-12)
        np.testing.assert_allclose(c["n"], [0.0, 0.0, -1.0], atol=1e-12)
        np.testing.assert_allclose(c["p"], [s[0], s[1], z0 + hz], atol=1e-12)


def test_object_resting_on_a_link_weighs_on_it():
    # a box that cannot turn, resting on a horizontal link far above the
    # table: in steady state the link feels the object's weight, straight down
    hx, hy, hz = 0.03, 0.025, 0.01
    sdf, box = _grid(_box_field(hx, hy, hz), n=33, half=0.05)
    R, m, zl = 0.006, 0.12, 1.0
    o = _oracle([tiny.link_row((-0.02, 0.0, zl), (0.02, 0.0, zl), R)], sdf, box, C_max=16)
    st = tiny.state(x=(0.0, 0.0, zl + R + hz))
    pr = tiny.params(m, 0.5)
    seg = o.hand_fk(np.zeros(1))
    wkey, wr = o.new_warm(1)
    for _ in range(300):
        cont, dg = o.env_step(seg, seg, 0, st, pr, wkey[0], wr[0])
    obs = o.observe(cont)
    np.testing.assert_allclose(obs[0, 0], m * G, rtol=1e-9)
    np.testing.assert_allclose(obs[0, 1:], [0.0, 0.0, -1.0], atol=1e-9)
    np.testing.assert_allclose(st[7:10], 0.0, atol=1e-9)
