"""Seeded synthetic scenes for sample-based in-hand pose tracking.

This module only *generates inputs*: the kinematic hand's link table, the
object sphere sets and their inertias, the seeded initial population (poses
perturbed around p0, parameters drawn from the prior -- Alg. 1, first line;
Sec. III-D) and the prescribed joint-command trajectory u_t.  It contains none
of the per-step arithmetic (kinematics, collision, contact solve, observation,
cost, resampling); both the GPU library and the CPU oracle consume its arrays
as plain data.

The paper's workloads (YCB objects, an Allegro hand on teleoperated
trajectories, Sec. IV) are not available; the scenes here stand in for them:
capsule-link hands on sinusoidal joint trajectories grasping sphere-set
objects resting on a table, with the population sizes of the five benchmark
workloads (16, 256, 4096, 1024 and 16384 simulations).

All arrays are float64 / int32 numpy arrays.  Link table rows have 20 entries:
parent, joint0, joint1, axis0(3), axis1(3), offset(3), offset quaternion
(w,x,y,z), length, radius, 2 reserved.  A link frame is the parent's tip frame
moved by the offset, turned about axis0 by u[joint0] then about axis1 by
u[joint1]; its capsule runs along local +x.  Joint index -1 means no joint.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

HAND_STRIDE = 20


# --------------------------------------------------------------------------
# configuration
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class ModelConsts:
    """Constants of the discrete contact model (shared reading, both sides)."""
    dt: float = 1.0 / 30.0
    gravity: tuple = (0.0, 0.0, -9.81)
    margin: float = 0.008        # speculative-contact margin [m]
    erp: float = 0.2             # Baumgarte depenetration factor
    compliance: float = 0.05     # epsilon added to the Delassus diagonal [1/kg]
    kappa: float = 10.0          # impulse -> velocity scale in the FB map [1/kg]
    fb_delta: float = 1e-4       # Fischer-Burmeister smoothing [m/s]
    armijo_sigma: float = 1e-4
    tau_contact: float = 0.01    # sensor contact threshold [N]
    w_mag: float = 1.0           # cost weight on the force magnitude
    w_dir: float = 0.1           # cost weight on the force direction
    # the full cost of Eq. 3 (cost_mode 1): contact-state, slip and spin terms
    cost_mode: int = 0           # 0: force magnitude / direction terms; 1: Eq. 3
    tau_slip: float = 0.005      # translational slip threshold [m/s]
    tau_spin: float = 0.1        # rotational slip threshold [rad/s]
    w_eq3: tuple = (1.0, 1.0, 0.6366197723675814, 1.0, 0.6366197723675814, 1.0, 1.0)  # w4..w10
    # the PD-controlled hand (hand_mode 1): its joints are state, driven
    # toward the commands by an implicit PD law
    hand_mode: int = 0           # 0: kinematic hand (joints follow u_t); 1: PD-controlled hand
    kp: float = 1.5              # joint stiffness [N m / rad]
    kd: float = 0.05             # joint damping [N m s / rad]
    link_mass: float = 0.03      # mass of every capsule link [kg]
    w_q: float = 100.0           # weight of the joint-angle term |q - q_gt|^2 [1 / rad^2]
    # link-object collision: 0 = the object's sphere set; 1 = the object's
    # signed distance field (a regular grid of sdf_res^3 nodes, interpolated
    # trilinearly) against link_samples points on each link's axis
    collision_mode: int = 0
    link_samples: int = 8
    sdf_res: int = 32
    sdf_pad: float = 0.02        # grid margin around the object's bounding box [m]


@dataclass(frozen=True)
class HandSpec:
    n_fingers: int = 3
    links_per_finger: int = 3
    abduction: bool = False      # one extra joint per finger at the base
    palm: bool = False           # fixed capsules joining the finger bases
    link_len: float = 0.040
    link_radius: float = 0.008
    base_radius: float = 0.065   # horizontal distance of finger bases from the object axis
    base_height: float = 0.13
    azimuth0: float = 0.0
    mean_angles: tuple = (1.25, 0.15, 0.1)  # per flexion joint, proximal first [rad]
    amplitude: float = 0.3       # sinusoid amplitude [rad]
    freq: float = 0.5            # sinusoid frequency [Hz]


@dataclass(frozen=True)
class ObjectSpec:
    kind: str = "cuboid"         # cuboid | ellipsoid | superquadric
    dims: tuple = (0.06, 0.04, 0.04)   # full extents (cuboid) or semi-axes (others)
    n_spheres: int = 26
    radius: float = 0.005
    lattice: tuple = (3, 3, 3)   # cuboid lattice counts
    drop_centre: bool = True     # cuboid 3x3x3 lattice without its centre
    exponents: tuple = (1.0, 1.0)  # superquadric e1, e2


@dataclass(frozen=True)
class TrackerConfig:
    name: str
    K: int
    steps: int
    C_max: int
    newton_iters: int
    hand: HandSpec
    objects: tuple               # ObjectSpec per object type
    group_types: tuple           # object type of each group (one hidden env each)
    T: int = 10
    m_range: tuple = (0.05, 0.2)
    mu_range: tuple = (0.3, 1.0)
    sigma_t: float = 0.005
    sigma_r_deg: float = 5.0
    hidden_mu: float = 0.6
    hidden_m: float = 0.1
    elite_frac: float = 0.25
    sigma_mu: float = 0.05
    sigma_m: float = 0.01
    sigma_f: float = 0.05
    seed: int = 0
    consts: ModelConsts = field(default_factory=ModelConsts)

    @property
    def G(self) -> int:
        return len(self.group_types)

    def with_(self, **kw) -> "TrackerConfig":
        return dataclasses.replace(self, **kw)


def _hand3():
    return HandSpec()


CONFIGS = {
    # 16 simulations, 3 fingers x 3 capsule links, 26-sphere cuboid
    "small": TrackerConfig(
        name="small", K=16, steps=60, C_max=16, newton_iters=10, hand=_hand3(),
        objects=(ObjectSpec(),), group_types=(0,)),
    # 256 simulations, 4 fingers + palm (16 links), 64-sphere ellipsoid
    "plain256": TrackerConfig(
        name="plain256", K=256, steps=300, C_max=32, newton_iters=15,
        hand=HandSpec(n_fingers=4, links_per_finger=3, abduction=True, palm=True,
                      base_radius=0.085, base_height=0.095, azimuth0=math.pi / 4,
                      mean_angles=(0.55, 0.55, 0.35)),
        objects=(ObjectSpec(kind="ellipsoid", dims=(0.04, 0.03, 0.025), n_spheres=64, radius=0.004),),
        group_types=(0,), m_range=(0.05, 0.3), mu_range=(0.2, 1.2), sigma_t=0.008, sigma_r_deg=8.0),
    # 4096 simulations, mixed 32/64/128-sphere cuboids, one group per object
    "batched4096": TrackerConfig(
        name="batched4096", K=4096, steps=300, C_max=64, newton_iters=10, hand=_hand3(),
        objects=(ObjectSpec(n_spheres=32, radius=0.005, lattice=(4, 4, 2), drop_centre=False),
                 ObjectSpec(n_spheres=64, radius=0.004, lattice=(4, 4, 4), drop_centre=False),
                 ObjectSpec(n_spheres=128, radius=0.003, lattice=(8, 4, 4), drop_centre=False)),
        group_types=(0, 1, 2)),
    # 1024 simulations, 64-sphere cuboid, adjoint-refined elites
    "adjoint1024": TrackerConfig(
        name="adjoint1024", K=1024, steps=60, C_max=32, newton_iters=10, hand=_hand3(),
        objects=(ObjectSpec(n_spheres=64, radius=0.004, lattice=(4, 4, 4), drop_centre=False),),
        group_types=(0,)),
    # 16384 simulations, 5 fingers x 4 links, 16 superquadric objects
    "realtime16384": TrackerConfig(
        name="realtime16384", K=16384, steps=1800, C_max=64, newton_iters=10,
        hand=HandSpec(n_fingers=5, links_per_finger=4, base_radius=0.09, base_height=0.10,
                      link_len=0.035, mean_angles=(0.5, 0.4, 0.35, 0.25)),
        objects=tuple(ObjectSpec(kind="superquadric", n_spheres=128, radius=0.004) for _ in range(16)),
        group_types=tuple(range(16)), m_range=(0.05, 0.5), mu_range=(0.2, 1.2)),
}


# --------------------------------------------------------------------------
# small quaternion utilities for input generation
# --------------------------------------------------------------------------

def _quat_axis_angle(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    s = math.sin(0.5 * angle)
    return np.array([math.cos(0.5 * angle), s * axis[0], s * axis[1], s * axis[2]])


def _quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _quat_from_rotvec(v):
    a = float(np.linalg.norm(v))
    if a < 1e-12:
        return np.array([1.0, 0.5 * v[0], 0.5 * v[1], 0.5 * v[2]]) / math.sqrt(1 + 0.25 * a * a)
    s = math.sin(0.5 * a) / a
    return np.array([math.cos(0.5 * a), s * v[0], s * v[1], s * v[2]])


def _quat_rotate(q, v):
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    return np.asarray(v) @ R.T


# --------------------------------------------------------------------------
# hand
# --------------------------------------------------------------------------

def build_hand(spec: HandSpec):
    """Link table [L][20] and mean joint angles [D] of a claw-like hand whose
    fingers hang from a ring above the object and flex towards its axis."""
    rows = []
    mean = []
    ey = (0.0, 1.0, 0.0)
    ez = (0.0, 0.0, 1.0)
    bases = []
    for f in range(spec.n_fingers):
        psi = spec.azimuth0 + 2.0 * math.pi * f / spec.n_fingers
        base = np.array([spec.base_radius * math.cos(psi), spec.base_radius * math.sin(psi), spec.base_height])
        bases.append(base)
        # local +x points horizontally at the object axis
        q_base = _quat_axis_angle(ez, psi + math.pi)
        first = len(rows)
        for k in range(spec.links_per_finger):
            row = np.zeros(HAND_STRIDE)
            row[0] = -1 if k == 0 else first + k - 1
            if k == 0 and spec.abduction:
                row[1] = len(mean)
                mean.append(0.0)
                row[3:6] = ez
                row[2] = len(mean)
                mean.append(spec.mean_angles[0])
                row[6:9] = ey
            else:
                row[1] = len(mean)
                mean.append(spec.mean_angles[k])
                row[3:6] = ey
                row[2] = -1
            if k == 0:
                row[9:12] = base
                row[12:16] = q_base
            else:
                row[12:16] = (1.0, 0.0, 0.0, 0.0)
            row[16] = spec.link_len
            row[17] = spec.link_radius
            rows.append(row)
    if spec.palm:
        for f in range(spec.n_fingers):
            a = bases[f]
            b = bases[(f + 1) % spec.n_fingers]
            d = b - a
            length = float(np.linalg.norm(d))
            yaw = math.atan2(d[1], d[0])
            row = np.zeros(HAND_STRIDE)
            row[0] = -1
            row[1] = -1
            row[2] = -1
            row[9:12] = a
            row[12:16] = _quat_axis_angle(ez, yaw)
            row[16] = length
            row[17] = spec.link_radius
            rows.append(row)
    return np.array(rows, dtype=np.float64), np.array(mean, dtype=np.float64)


def joint_trajectory(spec: HandSpec, mean: np.ndarray, steps: int, dt: float, rng: np.random.Generator):
    """u[t][j] = mean_j + A sin(2 pi f t dt + phi_j), phi_j ~ U[0, 2 pi)."""
    phases = rng.uniform(0.0, 2.0 * math.pi, size=mean.shape[0])
    t = np.arange(steps, dtype=np.float64)[:, None] * dt
    return mean[None, :] + spec.amplitude * np.sin(2.0 * math.pi * spec.freq * t + phases[None, :])


# --------------------------------------------------------------------------
# objects
# --------------------------------------------------------------------------

def _fibonacci_sphere(n):
    i = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def _superquadric_params(rng):
    a = rng.uniform(0.02, 0.04, size=3)
    e = rng.uniform(0.3, 1.0, size=2)
    return tuple(a), tuple(e)


def _sq_inside(p, a, e):
    e1, e2 = e
    x = np.abs(p[..., 0] / a[0])
    y = np.abs(p[..., 1] / a[1])
    z = np.abs(p[..., 2] / a[2])
    return (x ** (2.0 / e2) + y ** (2.0 / e2)) ** (e2 / e1) + z ** (2.0 / e1) <= 1.0


def build_object(spec: ObjectSpec, rng: np.random.Generator | None = None):
    """Body-frame sphere set [S][4] (centre, radius) and principal inverse
    inertia per unit mass [3].  The body origin is the centre of mass."""
    rho = spec.radius
    if spec.kind == "cuboid":
        h = np.asarray(spec.dims) / 2.0
        axes = [np.linspace(-(h[i] - rho), h[i] - rho, spec.lattice[i]) if spec.lattice[i] > 1
                else np.zeros(1) for i in range(3)]
        pts = np.array([[x, y, z] for x in axes[0] for y in axes[1] for z in axes[2]])
        if spec.drop_centre:
            keep = np.linalg.norm(pts, axis=1) > 1e-12
            pts = pts[keep]
        a, b, c = spec.dims
        inertia = np.array([(b * b + c * c), (a * a + c * c), (a * a + b * b)]) / 12.0
        dims = spec.dims
        exps = None
    elif spec.kind == "ellipsoid":
        a = np.asarray(spec.dims)
        u = _fibonacci_sphere(spec.n_spheres)
        surf = u * a
        nrm = u / a
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        pts = surf - rho * nrm
        inertia = np.array([a[1] ** 2 + a[2] ** 2, a[0] ** 2 + a[2] ** 2, a[0] ** 2 + a[1] ** 2]) / 5.0
        dims = spec.dims
        exps = None
    elif spec.kind == "superquadric":
        assert rng is not None
        dims, exps = _superquadric_params(rng)
        a = np.asarray(dims)
        e1, e2 = exps
        u = _fibonacci_sphere(spec.n_spheres)
        eta = np.arcsin(np.clip(u[:, 2], -1, 1))
        om = np.arctan2(u[:, 1], u[:, 0])

        def spow(x, p):
            return np.sign(x) * np.abs(x) ** p
        surf = np.stack([a[0] * spow(np.cos(eta), e1) * spow(np.cos(om), e2),
                         a[1] * spow(np.cos(eta), e1) * spow(np.sin(om), e2),
                         a[2] * spow(np.sin(eta), e1)], axis=1)
        # outward normal of the implicit surface
        def dpow(x, p):
            return np.sign(x) * np.abs(x) ** (p - 1.0) * p
        g = np.stack([dpow(surf[:, 0] / a[0], 2.0 / e2) / a[0],
                      dpow(surf[:, 1] / a[1], 2.0 / e2) / a[1],
                      dpow(surf[:, 2] / a[2], 2.0 / e1) / a[2]], axis=1)
        g /= np.maximum(np.linalg.norm(g, axis=1, keepdims=True), 1e-30)
        pts = surf - rho * g
        # inertia per unit mass by midpoint integration on a regular grid
        n = 48
        xs = [((np.arange(n) + 0.5) / n * 2.0 - 1.0) * a[i] for i in range(3)]
        X, Y, Z = np.meshgrid(*xs, indexing="ij")
        P = np.stack([X, Y, Z], axis=-1)
        ins = _sq_inside(P, a, exps)
        cnt = ins.sum()
        inertia = np.array([((Y ** 2 + Z ** 2) * ins).sum(), ((X ** 2 + Z ** 2) * ins).sum(),
                            ((X ** 2 + Y ** 2) * ins).sum()]) / cnt
    else:
        raise ValueError(spec.kind)
    spheres = np.concatenate([pts, np.full((pts.shape[0], 1), rho)], axis=1)
    return spheres.astype(np.float64), 1.0 / inertia, dims, exps


def build_sdf(spec: ObjectSpec, dims, exps, n: int, pad: float, n_surface: int = 40000):
    """Signed distance field of an object's shape (negative inside) on a
    cubic grid of n^3 nodes [n][n][n] (z, y, x), and its box: origin (object
    frame, 3) and node spacing.  The cuboid's field is the exact box
    distance; the ellipsoid's and the superquadric's are the distance to a
    dense sampling of the surface, signed by the shape's implicit function."""
    a = np.asarray(dims, dtype=np.float64) / (2.0 if spec.kind == "cuboid" else 1.0)
    half = float(a.max()) + pad
    h = 2.0 * half / (n - 1)
    xs = -half + h * np.arange(n)
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
    if spec.kind == "cuboid":
        q = np.abs(P) - a
        phi = np.linalg.norm(np.maximum(q, 0.0), axis=1) + np.minimum(q.max(axis=1), 0.0)
    else:
        from scipy.spatial import cKDTree
        u = _fibonacci_sphere(n_surface)
        if spec.kind == "ellipsoid":
            surf = u * a
            inside = ((P / a) ** 2).sum(axis=1) <= 1.0
        else:
            e1, e2 = exps
            eta = np.arcsin(np.clip(u[:, 2], -1, 1))
            om = np.arctan2(u[:, 1], u[:, 0])

            def spow(x, p):
                return np.sign(x) * np.abs(x) ** p
            surf = np.stack([a[0] * spow(np.cos(eta), e1) * spow(np.cos(om), e2),
                             a[1] * spow(np.cos(eta), e1) * spow(np.sin(om), e2),
                             a[2] * spow(np.sin(eta), e1)], axis=1)
            inside = _sq_inside(P, a, exps)
        dist, _ = cKDTree(surf).query(P)
        phi = np.where(inside, -dist, dist)
    box = np.array([-half, -half, -half, h])
    return phi.reshape(n, n, n), box


# --------------------------------------------------------------------------
# full scene
# --------------------------------------------------------------------------

@dataclass
class Scene:
    cfg: TrackerConfig
    hand: np.ndarray            # [L][20]
    mean_angles: np.ndarray     # [D]
    u: np.ndarray               # [steps][D] joint commands
    spheres: np.ndarray         # [n_types][S_max][4]
    n_spheres: np.ndarray       # [n_types] int32
    inv_inertia: np.ndarray     # [n_types][3]
    env_type: np.ndarray        # [K] int32
    group_start: np.ndarray     # [G+1] int32
    state: np.ndarray           # [K][13] x, q(w,x,y,z), v, w
    params: np.ndarray          # [K][5] m, mu, f_pert
    hidden_type: np.ndarray     # [G] int32
    hidden_state: np.ndarray    # [G][13]
    hidden_params: np.ndarray   # [G][5]
    rest_pose: np.ndarray       # [n_types][7] unperturbed pose p0 of each object
    sdf: np.ndarray | None = None      # [n_types][n][n][n] distance fields (collision_mode 1)
    sdf_box: np.ndarray | None = None  # [n_types][4] grid origin and spacing

    @property
    def L(self):
        return self.hand.shape[0]

    @property
    def D(self):
        return self.u.shape[1]

    @property
    def K(self):
        return self.env_type.shape[0]

    @property
    def G(self):
        return self.group_start.shape[0] - 1

    @property
    def S_max(self):
        return self.spheres.shape[1]


def rest_pose_of(spheres: np.ndarray, q=(1.0, 0.0, 0.0, 0.0)):
    """Pose with the given orientation whose lowest sphere touches z = 0."""
    c = _quat_rotate(np.asarray(q), spheres[:, :3])
    z = float(np.max(spheres[:, 3] - c[:, 2]))
    return np.array([0.0, 0.0, z, *q])


def split_groups(K: int, G: int):
    base, extra = divmod(K, G)
    sizes = [base + (1 if g < extra else 0) for g in range(G)]
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)


def make_scene(cfg: TrackerConfig, K: int | None = None, steps: int | None = None) -> Scene:
    """Build the seeded scene of a configuration (optionally with a different
    population size or trajectory length; the draws for the first K envs do
    not depend on K only through the group split)."""
    K = cfg.K if K is None else K
    steps = cfg.steps if steps is None else steps
    rng = np.random.Generator(np.random.PCG64(cfg.seed))
    hand, mean = build_hand(cfg.hand)
    u = joint_trajectory(cfg.hand, mean, steps, cfg.consts.dt, rng)

    sph_list, inv_list, shapes = [], [], []
    for ospec in cfg.objects:
        s, inv, dims, exps = build_object(ospec, rng)
        sph_list.append(s)
        inv_list.append(inv)
        shapes.append((ospec, dims, exps))
    n_types = len(sph_list)
    S_max = max(s.shape[0] for s in sph_list)
    spheres = np.zeros((n_types, S_max, 4))
    n_sph = np.zeros(n_types, dtype=np.int32)
    for t, s in enumerate(sph_list):
        spheres[t, :s.shape[0]] = s
        n_sph[t] = s.shape[0]
    inv_inertia = np.array(inv_list)
    rest = np.array([rest_pose_of(s) for s in sph_list])

    G = cfg.G
    gs = split_groups(K, G)
    env_type = np.zeros(K, dtype=np.int32)
    for g in range(G):
        env_type[gs[g]:gs[g + 1]] = cfg.group_types[g]

    # population: pose ~ N(p0, Sigma_p) with the rotation drawn in the tangent
    # space and applied on the left; parameters ~ the uniform prior.
    sig_r = math.radians(cfg.sigma_r_deg)
    dx = rng.normal(0.0, cfg.sigma_t, size=(K, 3))
    dr = rng.normal(0.0, sig_r, size=(K, 3))
    m = rng.uniform(cfg.m_range[0], cfg.m_range[1], size=K)
    mu = rng.uniform(cfg.mu_range[0], cfg.mu_range[1], size=K)
    state = np.zeros((K, 13))
    for i in range(K):
        p0 = rest[env_type[i]]
        state[i, 0:3] = p0[0:3] + dx[i]
        q = _quat_mul(_quat_from_rotvec(dr[i]), p0[3:7])
        state[i, 3:7] = q / np.linalg.norm(q)
    params = np.zeros((K, 5))
    params[:, 0] = m
    params[:, 1] = mu

    hidden_type = np.array(cfg.group_types, dtype=np.int32)
    hidden_state = np.zeros((G, 13))
    hidden_params = np.zeros((G, 5))
    for g in range(G):
        hidden_state[g, 0:7] = rest[hidden_type[g]]
        hidden_params[g, 0] = cfg.hidden_m
        hidden_params[g, 1] = cfg.hidden_mu
    sdf = sdf_box = None
    if cfg.consts.collision_mode == 1:
        c = cfg.consts
        grids = [build_sdf(o, d, e, c.sdf_res, c.sdf_pad) for o, d, e in shapes]
        sdf = np.array([g for g, _ in grids])
        sdf_box = np.array([b for _, b in grids])
    return Scene(cfg=cfg, hand=hand, mean_angles=mean, u=u, spheres=spheres, n_spheres=n_sph,
                 inv_inertia=inv_inertia, env_type=env_type, group_start=gs, state=state,
                 params=params, hidden_type=hidden_type, hidden_state=hidden_state,
                 hidden_params=hidden_params, rest_pose=rest, sdf=sdf, sdf_box=sdf_box)


def round_to_f32(scene: Scene) -> Scene:
    """Copy of the scene with every floating-point input rounded to float32
    (the GPU computes in float32; the oracle then starts from the same
    values)."""
    def r(a):
        return a.astype(np.float32).astype(np.float64)
    return dataclasses.replace(scene, hand=r(scene.hand), u=r(scene.u), spheres=r(scene.spheres),
                               inv_inertia=r(scene.inv_inertia), state=r(scene.state),
                               params=r(scene.params), hidden_state=r(scene.hidden_state),
                               hidden_params=r(scene.hidden_params),
                               sdf=None if scene.sdf is None else r(scene.sdf),
                               sdf_box=None if scene.sdf_box is None else r(scene.sdf_box))
