"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never imports it; the two share no code.

Thin ctypes wrapper around ``oracle.c`` (plain C, double precision), which
implements the discrete world model, observation, cost, argmin and the
population-based resampler of sample-based in-hand pose tracking
(arXiv 2002.12160, Sec. III, Alg. 1).  See ``oracle.h`` for the model.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

HAND_STRIDE = 20
MAX_CMAX = 64


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (IEEE double, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
               "-o", _LIB_PATH, os.path.join(_HERE, "oracle.c"), "-lm"]
        subprocess.check_call(cmd)
    return _LIB_PATH


class Model(C.Structure):
    _fields_ = [
        ("L", C.c_int32), ("D", C.c_int32), ("n_types", C.c_int32), ("S_max", C.c_int32), ("C_max", C.c_int32),
        ("newton_iters", C.c_int32), ("converged", C.c_int32), ("conv_max_iters", C.c_int32),
        ("conv_tol", C.c_double), ("dt", C.c_double), ("gravity", C.c_double * 3),
        ("margin", C.c_double), ("erp", C.c_double), ("compliance", C.c_double), ("kappa", C.c_double),
        ("fb_delta", C.c_double), ("armijo_sigma", C.c_double),
        ("tau_contact", C.c_double), ("w_mag", C.c_double), ("w_dir", C.c_double),
        ("hand", C.POINTER(C.c_double)), ("spheres", C.POINTER(C.c_double)),
        ("n_spheres", C.POINTER(C.c_int32)), ("inv_inertia", C.POINTER(C.c_double)),
        ("cost_mode", C.c_int32), ("tau_slip", C.c_double), ("tau_spin", C.c_double), ("w_eq3", C.c_double * 7),
        ("geom_f32", C.c_int32),
        ("kp", C.c_double), ("kd", C.c_double), ("link_mass", C.c_double), ("w_q", C.c_double),
        ("collision_mode", C.c_int32), ("link_samples", C.c_int32), ("sdf_n", C.c_int32),
        ("sdf", C.POINTER(C.c_double)), ("sdf_box", C.POINTER(C.c_double)),
    ]


class Contact(C.Structure):
    _fields_ = [("key", C.c_int32), ("link", C.c_int32), ("d", C.c_double),
                ("n", C.c_double * 3), ("t1", C.c_double * 3), ("t2", C.c_double * 3),
                ("p", C.c_double * 3), ("vlink", C.c_double * 3), ("r", C.c_double * 3),
                ("u", C.c_double * 3)]


class Diag(C.Structure):
    _fields_ = [("n_candidates", C.c_int32), ("n_contacts", C.c_int32), ("iters", C.c_int32),
                ("n_full_steps", C.c_int32), ("psi_first", C.c_double), ("psi_final", C.c_double),
                ("d_last_kept", C.c_double), ("d_first_dropped", C.c_double),
                ("armijo_margin", C.c_double), ("tangent_tie", C.c_double), ("margin_gap", C.c_double),
                ("n_fallback", C.c_int32), ("reserved", C.c_int32)]


class ResampleCfg(C.Structure):
    _fields_ = [("elite_frac", C.c_double), ("sigma_mu", C.c_double), ("sigma_m", C.c_double),
                ("sigma_f", C.c_double), ("mu_lo", C.c_double), ("mu_hi", C.c_double),
                ("m_lo", C.c_double), ("m_hi", C.c_double), ("seed", C.c_uint64)]


CONTACT_DTYPE = np.dtype([("key", np.int32), ("link", np.int32), ("d", np.float64),
                          ("n", np.float64, 3), ("t1", np.float64, 3), ("t2", np.float64, 3),
                          ("p", np.float64, 3), ("vlink", np.float64, 3), ("r", np.float64, 3),
                          ("u", np.float64, 3)])
DIAG_DTYPE = np.dtype([("n_candidates", np.int32), ("n_contacts", np.int32), ("iters", np.int32),
                       ("n_full_steps", np.int32), ("psi_first", np.float64), ("psi_final", np.float64),
                       ("d_last_kept", np.float64), ("d_first_dropped", np.float64),
                       ("armijo_margin", np.float64), ("tangent_tie", np.float64), ("margin_gap", np.float64),
                       ("n_fallback", np.int32), ("reserved", np.int32)])
assert CONTACT_DTYPE.itemsize == C.sizeof(Contact)
assert DIAG_DTYPE.itemsize == C.sizeof(Diag)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        mp = C.POINTER(Model)
        L.or_hand_fk.argtypes = [mp, dp, dp]
        L.or_env_step.argtypes = [mp, dp, dp, C.c_int, dp, dp, ip, dp, C.c_void_p, C.c_void_p]
        L.or_env_step.restype = C.c_int
        L.or_env_system.argtypes = [mp, dp, dp, C.c_int, dp, dp, C.c_void_p, dp, dp]
        L.or_env_system.restype = C.c_int
        L.or_observe.argtypes = [mp, C.c_int, C.c_void_p, dp]
        L.or_step_cost.argtypes = [mp, dp, dp]
        L.or_step_cost.restype = C.c_double
        L.or_observe_eq3.argtypes = [mp, C.c_int, C.c_void_p, dp, dp, dp, dp]
        L.or_step_cost_eq3.argtypes = [mp, dp, dp]
        L.or_step_cost_eq3.restype = C.c_double
        L.or_batch_step.argtypes = [mp, C.c_int, ip, dp, dp, dp, dp, ip, dp, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_batch_cost.argtypes = [mp, C.c_int, C.c_int, ip, dp, dp, dp]
        L.or_argmin.argtypes = [C.c_int, dp]
        L.or_argmin.restype = C.c_int
        L.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.or_resample_pbo.argtypes = [mp, C.POINTER(ResampleCfg), C.c_int, C.c_int, ip, C.c_uint32,
                                      dp, dp, dp, ip, dp, ip]
        L.or_resample_apply.argtypes = [mp, C.POINTER(ResampleCfg), C.c_int, ip, C.c_uint32, dp, dp, dp, ip, dp]
        L.or_add.argtypes = [mp, C.c_int, dp, dp]
        L.or_add.restype = C.c_double
        L.or_window_cost.argtypes = [mp, C.c_int, dp, dp, C.c_void_p, C.c_void_p, C.c_int, dp, dp]
        L.or_window_cost.restype = C.c_double
        L.or_env_step_pd.argtypes = [mp, dp, C.c_int, dp, dp, dp, ip, dp, C.c_void_p, C.c_void_p]
        L.or_env_step_pd.restype = C.c_int
        L.or_hand_mass.argtypes = [mp, dp, dp]
        L.or_batch_step_pd.argtypes = [mp, C.c_int, ip, dp, dp, dp, dp, ip, dp, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_step_cost_pd.argtypes = [mp, dp, dp, dp, dp]
        L.or_step_cost_pd.restype = C.c_double
        L.or_sdf_eval.argtypes = [mp, C.c_int, dp, dp]
        L.or_sdf_eval.restype = C.c_double
        L.or_max_threads.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _vp(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


class Oracle:
    """Holds one scene description (hand, objects, constants) for the C oracle."""

    def __init__(self, hand, spheres, n_spheres, inv_inertia, consts, C_max, newton_iters,
                 D=None, converged=False, conv_tol=1e-26, conv_max_iters=100, geom_f32=False, sdf=None,
                 sdf_box=None):
        self.hand = np.ascontiguousarray(hand, dtype=np.float64)
        self.spheres = np.ascontiguousarray(spheres, dtype=np.float64)
        self.n_spheres = np.ascontiguousarray(n_spheres, dtype=np.int32)
        self.inv_inertia = np.ascontiguousarray(inv_inertia, dtype=np.float64)
        assert self.hand.ndim == 2 and self.hand.shape[1] == HAND_STRIDE
        assert 1 <= C_max <= MAX_CMAX
        L = self.hand.shape[0]
        if D is None:
            D = int(max(self.hand[:, 1].max(), self.hand[:, 2].max())) + 1
        m = Model()
        m.L, m.D = L, D
        m.n_types, m.S_max = self.spheres.shape[0], self.spheres.shape[1]
        m.C_max = C_max
        m.newton_iters = newton_iters
        m.converged = 1 if converged else 0
        m.conv_max_iters = conv_max_iters
        m.conv_tol = conv_tol
        m.dt = consts.dt
        for i in range(3):
            m.gravity[i] = consts.gravity[i]
        m.margin, m.erp, m.compliance = consts.margin, consts.erp, consts.compliance
        m.kappa, m.fb_delta, m.armijo_sigma = consts.kappa, consts.fb_delta, consts.armijo_sigma
        m.tau_contact, m.w_mag, m.w_dir = consts.tau_contact, consts.w_mag, consts.w_dir
        m.cost_mode = int(getattr(consts, "cost_mode", 0))
        m.tau_slip, m.tau_spin = getattr(consts, "tau_slip", 0.005), getattr(consts, "tau_spin", 0.1)
        for i, wv in enumerate(getattr(consts, "w_eq3", (1.0,) * 7)):
            m.w_eq3[i] = wv
        # diagnostic: geometry rounded to float32 (see oracle.h)
        m.geom_f32 = int(geom_f32)
        m.kp, m.kd = getattr(consts, "kp", 1.5), getattr(consts, "kd", 0.05)
        m.link_mass, m.w_q = getattr(consts, "link_mass", 0.03), getattr(consts, "w_q", 100.0)
        self.hand_mode = int(getattr(consts, "hand_mode", 0))
        # links against the objects' distance fields (grids [n_types][n][n][n], z, y, x)
        m.collision_mode = int(getattr(consts, "collision_mode", 0))
        m.link_samples = int(getattr(consts, "link_samples", 8))
        self.sdf = self.sdf_box = None
        if m.collision_mode == 1:
            assert sdf is not None and sdf_box is not None, "collision_mode 1 needs the distance fields"
            self.sdf = np.ascontiguousarray(sdf, dtype=np.float64)
            self.sdf_box = np.ascontiguousarray(sdf_box, dtype=np.float64)
            assert self.sdf.ndim == 4 and self.sdf.shape[1] == self.sdf.shape[2] == self.sdf.shape[3]
            assert self.sdf_box.shape == (self.sdf.shape[0], 4)
            m.sdf_n = self.sdf.shape[1]
            m.sdf = _dp(self.sdf)
            m.sdf_box = _dp(self.sdf_box)
        m.hand = _dp(self.hand)
        m.spheres = _dp(self.spheres)
        m.n_spheres = _ip(self.n_spheres)
        m.inv_inertia = _dp(self.inv_inertia)
        self.m = m
        self.consts = consts
        self.L, self.D, self.C_max = L, D, C_max
        self.R = 7 if m.cost_mode == 1 else 4     # observation rows per sensor

    @classmethod
    def from_scene(cls, scene, **kw):
        cfg = scene.cfg
        kw.setdefault("C_max", cfg.C_max)
        kw.setdefault("newton_iters", cfg.newton_iters)
        kw.setdefault("sdf", getattr(scene, "sdf", None))
        kw.setdefault("sdf_box", getattr(scene, "sdf_box", None))
        return cls(scene.hand, scene.spheres, scene.n_spheres, scene.inv_inertia, cfg.consts, D=scene.D, **kw)

    # -- kinematics ------------------------------------------------------
    def hand_fk(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        seg = np.zeros((self.L, 6))
        lib().or_hand_fk(C.byref(self.m), _dp(u), _dp(seg))
        return seg

    # -- one env ---------------------------------------------------------
    def env_step(self, seg0, seg1, typ, st, pr, wkey, wr):
        """In-place step of one env; returns (contacts array, diag)."""
        cont = np.zeros(self.C_max, dtype=CONTACT_DTYPE)
        dg = np.zeros(1, dtype=DIAG_DTYPE)
        nc = lib().or_env_step(C.byref(self.m), _dp(seg0), _dp(seg1), int(typ), _dp(st), _dp(pr), _ip(wkey),
                               _dp(wr), _vp(cont), _vp(dg))
        return cont[:nc], dg[0]

    def env_system(self, seg0, seg1, typ, st, pr):
        """Contacts, W [3C][3C] and u_free [3C] at the current state (no step)."""
        cont = np.zeros(self.C_max, dtype=CONTACT_DTYPE)
        W = np.zeros((3 * self.C_max) ** 2)
        uf = np.zeros(3 * self.C_max)
        nc = lib().or_env_system(C.byref(self.m), _dp(np.ascontiguousarray(seg0, dtype=np.float64)),
                                 _dp(np.ascontiguousarray(seg1, dtype=np.float64)), int(typ),
                                 _dp(np.ascontiguousarray(st, dtype=np.float64)),
                                 _dp(np.ascontiguousarray(pr, dtype=np.float64)), _vp(cont), _dp(W), _dp(uf))
        n3 = 3 * nc
        return cont[:nc], W[:n3 * n3].reshape(n3, n3), uf[:n3]

    def observe(self, cont):
        cont = np.ascontiguousarray(cont, dtype=CONTACT_DTYPE)
        obs = np.zeros((self.L, 4))
        lib().or_observe(C.byref(self.m), len(cont), _vp(cont), _dp(obs))
        return obs

    def observe_eq3(self, cont, seg0, seg1, omega_obj):
        """Eq. 3's observation [L][7] of one env's contacts (see oracle.h)."""
        cont = np.ascontiguousarray(cont, dtype=CONTACT_DTYPE)
        obs = np.zeros((self.L, 7))
        lib().or_observe_eq3(C.byref(self.m), len(cont), _vp(cont),
                             _dp(np.ascontiguousarray(seg0, dtype=np.float64)),
                             _dp(np.ascontiguousarray(seg1, dtype=np.float64)),
                             _dp(np.ascontiguousarray(omega_obj, dtype=np.float64)), _dp(obs))
        return obs

    def step_cost(self, obs, obs_gt):
        f = lib().or_step_cost_eq3 if self.R == 7 else lib().or_step_cost
        return f(C.byref(self.m), _dp(np.ascontiguousarray(obs, dtype=np.float64)),
                 _dp(np.ascontiguousarray(obs_gt, dtype=np.float64)))

    # -- batch -----------------------------------------------------------
    # -- PD-controlled hand ------------------------------------------------
    def sdf_eval(self, typ, p):
        """(phi, gradient) of object type typ's distance field at object-frame point p."""
        g = np.zeros(3)
        v = lib().or_sdf_eval(C.byref(self.m), int(typ), _dp(np.ascontiguousarray(p, dtype=np.float64)), _dp(g))
        return v, g

    def hand_mass(self, q):
        M = np.zeros((self.D, self.D))
        lib().or_hand_mass(C.byref(self.m), _dp(np.ascontiguousarray(q, dtype=np.float64)), _dp(M))
        return M

    def env_step_pd(self, u, typ, st, pr, hq, wkey, wr):
        """In-place PD-hand step of one env (hq = [q, qdot]); returns
        (contacts, diag)."""
        cont = np.zeros(self.C_max, dtype=CONTACT_DTYPE)
        dg = np.zeros(1, dtype=DIAG_DTYPE)
        nc = lib().or_env_step_pd(C.byref(self.m), _dp(np.ascontiguousarray(u, dtype=np.float64)), int(typ), _dp(st),
                                  _dp(pr), _dp(hq), _ip(wkey), _dp(wr), _vp(cont), _vp(dg))
        return cont[:nc], dg[0]

    def batch_step_pd(self, env_type, u, state, params, hstate, wkey, wr, want_contacts=False, want_diag=False):
        """In-place PD-hand step of K envs; returns (obs [K][L][4], contacts,
        diag); the joint angles are hstate[:, :D]."""
        K = state.shape[0]
        obs = np.zeros((K, self.L, 4))
        cont = np.zeros((K, self.C_max), dtype=CONTACT_DTYPE) if want_contacts else None
        dg = np.zeros(K, dtype=DIAG_DTYPE) if want_diag else None
        lib().or_batch_step_pd(C.byref(self.m), K, _ip(env_type), _dp(np.ascontiguousarray(u, dtype=np.float64)),
                               _dp(state), _dp(params), _dp(hstate), _ip(wkey), _dp(wr), _vp(cont), _vp(dg), _vp(obs))
        return obs, cont, dg

    def step_cost_pd(self, obs, q, obs_gt, q_gt):
        return lib().or_step_cost_pd(C.byref(self.m), _dp(np.ascontiguousarray(obs, dtype=np.float64)),
                                     _dp(np.ascontiguousarray(q, dtype=np.float64)),
                                     _dp(np.ascontiguousarray(obs_gt, dtype=np.float64)),
                                     _dp(np.ascontiguousarray(q_gt, dtype=np.float64)))

    def new_hand(self, K, u0):
        """Hand state [K][2D] at rest at the command u0."""
        h = np.zeros((K, 2 * self.D))
        h[:, :self.D] = np.asarray(u0, dtype=np.float64)
        return h

    def new_warm(self, K):
        return np.full((K, self.C_max), -1, dtype=np.int32), np.zeros((K, self.C_max, 3))

    def batch_step(self, env_type, u_prev, u, state, params, wkey, wr, want_contacts=False, want_diag=False):
        """In-place step of K envs; returns (obs [K][L][4], contacts, diag)."""
        K = state.shape[0]
        obs = np.zeros((K, self.L, self.R))
        cont = np.zeros((K, self.C_max), dtype=CONTACT_DTYPE) if want_contacts else None
        dg = np.zeros(K, dtype=DIAG_DTYPE) if want_diag else None
        lib().or_batch_step(C.byref(self.m), K, _ip(env_type), _dp(np.ascontiguousarray(u_prev, dtype=np.float64)),
                            _dp(np.ascontiguousarray(u, dtype=np.float64)), _dp(state), _dp(params), _ip(wkey),
                            _dp(wr), _vp(cont), _vp(dg), _vp(obs))
        return obs, cont, dg

    def batch_cost(self, group_start, obs, obs_gt, cost_sum):
        K = obs.shape[0]
        G = group_start.shape[0] - 1
        lib().or_batch_cost(C.byref(self.m), K, G, _ip(group_start), _dp(obs), _dp(obs_gt), _dp(cost_sum))

    def resample(self, rcfg, group_start, window_idx, cost_sum, state, params, wkey, wr):
        K = state.shape[0]
        G = group_start.shape[0] - 1
        parent = np.zeros(K, dtype=np.int32)
        lib().or_resample_pbo(C.byref(self.m), C.byref(rcfg), K, G, _ip(group_start), window_idx, _dp(cost_sum),
                              _dp(state), _dp(params), _ip(wkey), _dp(wr), _ip(parent))
        return parent

    def resample_weighted(self, kind, hyper, rcfg, group_start, window_idx, n_steps, cost_sum, state, params,
                          wkey, wr):
        """WRS or REPS resampling (Sec. III-D.1/2) in place; returns
        (parent, pmf, eta, cdf, target) -- see oracle.resamplers."""
        from . import resamplers as RS
        pmf, eta = RS.group_pmf(kind, hyper, cost_sum, n_steps, group_start)
        parent, cdf, target = RS.draw_parents(pmf, group_start, window_idx, int(rcfg.seed))
        K = state.shape[0]
        lib().or_resample_apply(C.byref(self.m), C.byref(rcfg), K, _ip(parent), window_idx, _dp(cost_sum),
                                _dp(state), _dp(params), _ip(wkey), _dp(wr))
        return parent, pmf, eta, cdf, target

    def add(self, typ, pose_a, pose_b):
        return lib().or_add(C.byref(self.m), int(typ), _dp(np.ascontiguousarray(pose_a[:7], dtype=np.float64)),
                            _dp(np.ascontiguousarray(pose_b[:7], dtype=np.float64)))

    def window_cost(self, typ, st0, pr0, u_seq, obs_gt, wkey0=None, wr0=None):
        T = obs_gt.shape[0]
        return lib().or_window_cost(C.byref(self.m), int(typ), _dp(np.ascontiguousarray(st0, dtype=np.float64)),
                                    _dp(np.ascontiguousarray(pr0, dtype=np.float64)),
                                    _vp(None if wkey0 is None else np.ascontiguousarray(wkey0, dtype=np.int32)),
                                    _vp(None if wr0 is None else np.ascontiguousarray(wr0, dtype=np.float64)),
                                    T, _dp(np.ascontiguousarray(u_seq, dtype=np.float64)),
                                    _dp(np.ascontiguousarray(obs_gt, dtype=np.float64)))


def max_threads():
    """OpenMP threads the batched oracle calls use."""
    return int(lib().or_max_threads())


def set_threads(n):
    lib().or_set_threads(int(n))


def argmin(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().or_argmin(v.shape[0], _dp(v))


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def resample_cfg(cfg) -> ResampleCfg:
    rc = ResampleCfg()
    rc.elite_frac, rc.sigma_mu, rc.sigma_m, rc.sigma_f = cfg.elite_frac, cfg.sigma_mu, cfg.sigma_m, cfg.sigma_f
    rc.mu_lo, rc.mu_hi = cfg.mu_range
    rc.m_lo, rc.m_hi = cfg.m_range
    rc.seed = cfg.seed
    return rc


class Tracker:
    """The tracking loop of Alg. 1 on the oracle: a hidden batch (one env per
    group) supplies the observed contact forces; the population is stepped
    with the same commands, its step costs accumulate over the window, the
    argmin is the pose estimate and every T steps the resampler runs."""

    def __init__(self, scene, **okw):
        self.scene = scene
        self.o = Oracle.from_scene(scene, **okw)
        self.state = scene.state.copy()
        self.params = scene.params.copy()
        self.wkey, self.wr = self.o.new_warm(scene.K)
        self.hstate = scene.hidden_state.copy()
        self.hparams = scene.hidden_params.copy()
        self.hkey, self.hr = self.o.new_warm(scene.G)
        self.cost_sum = np.zeros(scene.K)
        self.rcfg = resample_cfg(scene.cfg)
        self.t = 0
        self.window = 0
        self.pd = self.o.hand_mode == 1
        if self.pd:
            # the hands start at rest at the first command
            self.hand = self.o.new_hand(scene.K, scene.u[0])
            self.hhand = self.o.new_hand(scene.G, scene.u[0])

    def step(self, want=False):
        s = self.scene
        u_prev = s.u[max(self.t - 1, 0)]
        u = s.u[self.t]
        if self.pd:
            obs_gt, _, _ = self.o.batch_step_pd(s.hidden_type, u, self.hstate, self.hparams, self.hhand, self.hkey,
                                                self.hr)
            obs, cont, dg = self.o.batch_step_pd(s.env_type, u, self.state, self.params, self.hand, self.wkey,
                                                 self.wr, want_contacts=want, want_diag=want)
            D = self.o.D
            for g in range(s.G):
                for i in range(s.group_start[g], s.group_start[g + 1]):
                    self.cost_sum[i] += self.o.step_cost_pd(obs[i], self.hand[i, :D], obs_gt[g], self.hhand[g, :D])
        else:
            obs_gt, _, _ = self.o.batch_step(s.hidden_type, u_prev, u, self.hstate, self.hparams, self.hkey,
                                             self.hr)
            obs, cont, dg = self.o.batch_step(s.env_type, u_prev, u, self.state, self.params, self.wkey, self.wr,
                                              want_contacts=want, want_diag=want)
            self.o.batch_cost(s.group_start, obs, obs_gt, self.cost_sum)
        best = [s.group_start[g] + argmin(self.cost_sum[s.group_start[g]:s.group_start[g + 1]])
                for g in range(s.G)]
        self.t += 1
        parent = None
        if self.t % s.cfg.T == 0:
            parent = self.o.resample(self.rcfg, s.group_start, self.window, self.cost_sum, self.state, self.params,
                                     self.wkey, self.wr)
            if self.pd:
                # a copy takes its parent's hand with its body (parents are
                # elites, which the resampler leaves unchanged)
                for j in np.nonzero(parent >= 0)[0]:
                    self.hand[j] = self.hand[parent[j]]
            self.window += 1
        return dict(obs=obs, obs_gt=obs_gt, best=best, contacts=cont, diag=dg, parent=parent)
