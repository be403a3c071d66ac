"""Python binding of libpt (include/pt.h): argument marshalling only.

Every computation runs in the HIP kernels of libpt.so; PyTorch supplies the
device memory (tensors) and the streams.  Importing this module fails loudly
when the library has not been built -- there is no fallback.

Names follow the C ABI: ``pt_create_batch``, ``pt_step``, ``pt_observe``,
``pt_cost``, ``pt_resample`` (and its weighted variants ``pt_resample_wrs``,
``pt_resample_reps``), ``pt_run_window``, ``pt_autotune``,
``pt_window_grad``, ``pt_refine_elites``, ``pt_read_stats``; :class:`Batch`
bundles a handle with its tensors and :class:`WindowFn` exposes the window
cost and its adjoint to ``torch.autograd``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libpt.so is not built ({LIB_PATH}); run paper_2002_12160_amd/build.py "
                      "or __graft_entry__.build() first")

_lib = C.CDLL(LIB_PATH)

HAND_STRIDE = 20
MAX_CMAX = 64
PT_OK = 0
ERROR_NAMES = {1: "PT_E_ARG", 2: "PT_E_HIP", 3: "PT_E_STATE", 4: "PT_E_CAPTURE", 5: "PT_E_UNSUPPORTED"}


class PtError(RuntimeError):
    def __init__(self, code, where, msg=None):
        if msg is None:
            msg = _lib.pt_last_error().decode(errors="replace")
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class BatchDesc(C.Structure):
    _fields_ = [
        ("K", C.c_int32), ("G", C.c_int32), ("L", C.c_int32), ("D", C.c_int32), ("n_types", C.c_int32),
        ("S_max", C.c_int32), ("C_max", C.c_int32), ("newton_iters", C.c_int32), ("T", C.c_int32),
        ("solve_precision", C.c_int32),
        ("dt", C.c_float), ("gravity", C.c_float * 3), ("margin", C.c_float), ("erp", C.c_float),
        ("compliance", C.c_float), ("kappa", C.c_float), ("fb_delta", C.c_float), ("armijo_sigma", C.c_float),
        ("tau_contact", C.c_float), ("w_mag", C.c_float), ("w_dir", C.c_float),
        ("elite_frac", C.c_float), ("sigma_mu", C.c_float), ("sigma_m", C.c_float), ("sigma_f", C.c_float),
        ("mu_lo", C.c_float), ("mu_hi", C.c_float), ("m_lo", C.c_float), ("m_hi", C.c_float),
        ("seed", C.c_uint64),
        ("hand", C.c_void_p), ("spheres", C.c_void_p), ("n_spheres", C.c_void_p), ("inv_inertia", C.c_void_p),
        ("env_type", C.c_void_p), ("group_start", C.c_void_p),
        ("state", C.c_void_p), ("params", C.c_void_p), ("warm", C.c_void_p),
        ("window_checkpoints", C.c_int32),
        ("cost_mode", C.c_int32), ("tau_slip", C.c_float), ("tau_spin", C.c_float), ("w_eq3", C.c_float * 7),
        ("hand_mode", C.c_int32), ("kp", C.c_float), ("kd", C.c_float), ("link_mass", C.c_float),
        ("w_q", C.c_float), ("hand_state", C.c_void_p),
        ("collision_mode", C.c_int32), ("link_samples", C.c_int32), ("sdf_n", C.c_int32),
        ("sdf", C.c_void_p), ("sdf_box", C.c_void_p),
    ]


_vp = C.c_void_p
_lib.pt_last_error.restype = C.c_char_p
_lib.pt_last_error.argtypes = []
_lib.pt_create_batch.argtypes = [C.POINTER(BatchDesc), C.POINTER(_vp)]
_lib.pt_destroy_batch.argtypes = [_vp]
_lib.pt_step.argtypes = [_vp, _vp, _vp, _vp]
_lib.pt_observe.argtypes = [_vp, _vp, _vp]
_lib.pt_cost.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
_lib.pt_resample.argtypes = [_vp, _vp, C.c_uint32, _vp, _vp]
_lib.pt_resample_wrs.argtypes = [_vp, _vp, C.c_int32, C.c_uint32, C.c_float, _vp, _vp, _vp]
_lib.pt_resample_reps.argtypes = [_vp, _vp, C.c_int32, C.c_uint32, C.c_float, _vp, _vp, _vp, _vp]
_lib.pt_run_window.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, C.c_int32, _vp]
_lib.pt_run_window_static.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.pt_autotune.argtypes = [_vp, _vp, _vp, C.POINTER(C.c_int32), _vp]
_lib.pt_read_stats.argtypes = [_vp, C.POINTER(C.c_int64), _vp]
_lib.pt_set_tuning.argtypes = [_vp, C.c_int32]
_lib.pt_window_grad.argtypes = [_vp, _vp, _vp, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.pt_refine_elites.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int32, C.c_float, _vp, _vp, _vp, _vp]
_lib.pt_elite_count.argtypes = [_vp]
_lib.pt_elite_count.restype = C.c_int32
for _f in ("pt_create_batch", "pt_destroy_batch", "pt_step", "pt_observe", "pt_cost", "pt_resample",
           "pt_resample_wrs", "pt_resample_reps", "pt_run_window", "pt_run_window_static", "pt_autotune",
           "pt_read_stats", "pt_set_tuning", "pt_window_grad",
           "pt_refine_elites"):
    getattr(_lib, _f).restype = C.c_int


def _check(code, where):
    if code != PT_OK:
        raise PtError(code, where)


def _ptr(t):
    if t is None:
        return None
    assert t.is_contiguous(), "tensor must be contiguous"
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------
# C-ABI mirrors
# ---------------------------------------------------------------------------

def pt_create_batch(desc: BatchDesc) -> C.c_void_p:
    h = C.c_void_p()
    _check(_lib.pt_create_batch(C.byref(desc), C.byref(h)), "pt_create_batch")
    return h


def pt_destroy_batch(h):
    _check(_lib.pt_destroy_batch(h), "pt_destroy_batch")


def pt_step(h, u_prev, u, stream=None):
    _check(_lib.pt_step(h, _ptr(u_prev), _ptr(u), _stream(stream)), "pt_step")


def pt_observe(h, obs, stream=None):
    _check(_lib.pt_observe(h, _ptr(obs), _stream(stream)), "pt_observe")


def pt_cost(h, obs, obs_gt, cost_sum, best=None, stream=None):
    _check(_lib.pt_cost(h, _ptr(obs), _ptr(obs_gt), _ptr(cost_sum), _ptr(best), _stream(stream)), "pt_cost")


def pt_resample(h, cost_sum, window_idx, parent=None, stream=None):
    _check(_lib.pt_resample(h, _ptr(cost_sum), int(window_idx), _ptr(parent), _stream(stream)), "pt_resample")


def pt_resample_wrs(h, cost_sum, n_steps, window_idx, lam, parent, weights=None, stream=None):
    _check(_lib.pt_resample_wrs(h, _ptr(cost_sum), int(n_steps), int(window_idx), float(lam), _ptr(parent),
                                _ptr(weights), _stream(stream)), "pt_resample_wrs")


def pt_resample_reps(h, cost_sum, n_steps, window_idx, eps, parent, weights=None, eta=None, stream=None):
    _check(_lib.pt_resample_reps(h, _ptr(cost_sum), int(n_steps), int(window_idx), float(eps), _ptr(parent),
                                 _ptr(weights), _ptr(eta), _stream(stream)), "pt_resample_reps")


def pt_run_window(h, u_win, obs_gt_win, cost_sum, best=None, obs_out=None, graph=True, stream=None):
    _check(_lib.pt_run_window(h, _ptr(u_win), _ptr(obs_gt_win), _ptr(cost_sum), _ptr(best), _ptr(obs_out),
                              1 if graph else 0, _stream(stream)), "pt_run_window")


def pt_run_window_static(h, u_win, obs_gt_win, cost_sum, best=None, obs_out=None, stream=None):
    _check(_lib.pt_run_window_static(h, _ptr(u_win), _ptr(obs_gt_win), _ptr(cost_sum), _ptr(best), _ptr(obs_out),
                                     _stream(stream)), "pt_run_window_static")


def pt_autotune(h, u_win, obs_gt_win, stream=None):
    r = C.c_int32(0)
    _check(_lib.pt_autotune(h, _ptr(u_win), _ptr(obs_gt_win), C.byref(r), _stream(stream)), "pt_autotune")
    return int(r.value)


def pt_set_tuning(h, waves_per_workgroup):
    _check(_lib.pt_set_tuning(h, int(waves_per_workgroup)), "pt_set_tuning")


def pt_window_grad(h, u_win, obs_gt_win, env, start, warm0, cost, grad=None, end_state=None, end_warm=None,
                   resid=None, stream=None):
    n = int(env.shape[0])
    _check(_lib.pt_window_grad(h, _ptr(u_win), _ptr(obs_gt_win), n, _ptr(env), _ptr(start), _ptr(warm0), _ptr(cost),
                               _ptr(grad), _ptr(end_state), _ptr(end_warm), _ptr(resid), _stream(stream)),
           "pt_window_grad")


def pt_refine_elites(h, u_win, obs_gt_win, cost_sum, start_state, start_params, start_warm, steps=3, step=0.5,
                     scale=None, best=None, elite_out=None, stream=None):
    sc = None
    if scale is not None:
        arr = np.ascontiguousarray(scale, dtype=np.float32)
        assert arr.shape == (15,)
        sc = C.c_void_p(arr.ctypes.data)
    _check(_lib.pt_refine_elites(h, _ptr(u_win), _ptr(obs_gt_win), _ptr(cost_sum), _ptr(start_state),
                                 _ptr(start_params), _ptr(start_warm), int(steps), float(step), sc, _ptr(best),
                                 _ptr(elite_out), _stream(stream)), "pt_refine_elites")


def pt_elite_count(h):
    return int(_lib.pt_elite_count(h))


def pt_read_stats(h, stream=None):
    out = (C.c_int64 * 4)()
    _check(_lib.pt_read_stats(h, out, _stream(stream)), "pt_read_stats")
    return {"env_steps": out[0], "candidates": out[1], "contacts": out[2], "dropped": out[3]}


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------

class Batch:
    """A population of simulations on one device: the handle plus the state
    tensors it is bound to (state [13][K], params [5][K], warm [K][C_max][4],
    and with the PD-controlled hand (consts.hand_mode 1) hand_state [2D][K]:
    joint angles, then joint rates)."""

    def __init__(self, *, hand, spheres, n_spheres, inv_inertia, env_type, group_start, consts, C_max,
                 newton_iters, T, state, params, resample=None, solve_precision=64, window_checkpoints=False,
                 hand_state=None, sdf=None, sdf_box=None, device="cuda"):
        self.device = torch.device(device)
        K = int(np.asarray(env_type).shape[0])
        self.K, self.C_max, self.T = K, int(C_max), int(T)
        self.hand = np.ascontiguousarray(hand, dtype=np.float32)
        self.spheres = np.ascontiguousarray(spheres, dtype=np.float32)
        self.n_spheres = np.ascontiguousarray(n_spheres, dtype=np.int32)
        self.inv_inertia = np.ascontiguousarray(inv_inertia, dtype=np.float32)
        self.env_type = np.ascontiguousarray(env_type, dtype=np.int32)
        self.group_start = np.ascontiguousarray(group_start, dtype=np.int32)
        self.L = self.hand.shape[0]
        self.G = self.group_start.shape[0] - 1
        self.D = int(max(self.hand[:, 1].max(), self.hand[:, 2].max())) + 1
        self.state = torch.empty((13, K), dtype=torch.float32, device=self.device)
        self.params = torch.empty((5, K), dtype=torch.float32, device=self.device)
        self.warm = torch.empty((K, self.C_max, 4), dtype=torch.float32, device=self.device)
        self.set_state(state, params)
        self.clear_warm()
        self.hand_mode = int(getattr(consts, "hand_mode", 0))
        self.hand_state = None
        if self.hand_mode == 1:
            self.hand_state = torch.zeros((2 * self.D, K), dtype=torch.float32, device=self.device)
            if hand_state is not None:
                self.set_hand(hand_state)
        d = BatchDesc()
        d.K, d.G, d.L, d.D = K, self.G, self.L, self.D
        d.n_types, d.S_max = self.spheres.shape[0], self.spheres.shape[1]
        d.C_max, d.newton_iters, d.T = self.C_max, int(newton_iters), self.T
        d.solve_precision = int(solve_precision)
        d.dt = consts.dt
        for i in range(3):
            d.gravity[i] = consts.gravity[i]
        d.margin, d.erp, d.compliance, d.kappa = consts.margin, consts.erp, consts.compliance, consts.kappa
        d.fb_delta, d.armijo_sigma = consts.fb_delta, consts.armijo_sigma
        d.tau_contact, d.w_mag, d.w_dir = consts.tau_contact, consts.w_mag, consts.w_dir
        r = resample or {}
        d.elite_frac = r.get("elite_frac", 0.25)
        d.sigma_mu, d.sigma_m, d.sigma_f = r.get("sigma_mu", 0.0), r.get("sigma_m", 0.0), r.get("sigma_f", 0.0)
        d.mu_lo, d.mu_hi = r.get("mu_range", (0.0, 10.0))
        d.m_lo, d.m_hi = r.get("m_range", (1e-6, 1e6))
        d.seed = int(r.get("seed", 0))
        d.hand = self.hand.ctypes.data
        d.spheres = self.spheres.ctypes.data
        d.n_spheres = self.n_spheres.ctypes.data
        d.inv_inertia = self.inv_inertia.ctypes.data
        d.env_type = self.env_type.ctypes.data
        d.group_start = self.group_start.ctypes.data
        d.state = self.state.data_ptr()
        d.params = self.params.data_ptr()
        d.warm = self.warm.data_ptr()
        d.window_checkpoints = 1 if window_checkpoints else 0
        d.cost_mode = int(getattr(consts, "cost_mode", 0))
        d.tau_slip, d.tau_spin = getattr(consts, "tau_slip", 0.005), getattr(consts, "tau_spin", 0.1)
        for i, wv in enumerate(getattr(consts, "w_eq3", (1.0,) * 7)):
            d.w_eq3[i] = wv
        self.obs_rows = 7 if d.cost_mode == 1 else 4
        d.hand_mode = self.hand_mode
        d.kp, d.kd = getattr(consts, "kp", 0.0), getattr(consts, "kd", 0.0)
        d.link_mass, d.w_q = getattr(consts, "link_mass", 0.0), getattr(consts, "w_q", 0.0)
        d.hand_state = self.hand_state.data_ptr() if self.hand_state is not None else None
        # links against the objects' distance fields: grids [n_types][n][n][n] (z, y, x), boxes [n_types][4]
        d.collision_mode = int(getattr(consts, "collision_mode", 0))
        d.link_samples = int(getattr(consts, "link_samples", 8))
        self.sdf = self.sdf_box = None
        if d.collision_mode == 1:
            if sdf is None or sdf_box is None:
                raise PtError(1, "Batch", "collision_mode 1 needs sdf and sdf_box")
            self.sdf = np.ascontiguousarray(sdf, dtype=np.float32)
            self.sdf_box = np.ascontiguousarray(sdf_box, dtype=np.float32)
            d.sdf_n = self.sdf.shape[1]
            d.sdf = self.sdf.ctypes.data
            d.sdf_box = self.sdf_box.ctypes.data
        self.desc = d
        self.handle = pt_create_batch(d)

    @classmethod
    def from_scene(cls, scene, hidden=False, device="cuda", **kw):
        cfg = scene.cfg
        common = dict(hand=scene.hand, spheres=scene.spheres, n_spheres=scene.n_spheres,
                      inv_inertia=scene.inv_inertia, consts=cfg.consts, C_max=kw.pop("C_max", cfg.C_max),
                      newton_iters=kw.pop("newton_iters", cfg.newton_iters), T=kw.pop("T", cfg.T),
                      resample=dict(elite_frac=cfg.elite_frac, sigma_mu=cfg.sigma_mu, sigma_m=cfg.sigma_m,
                                    sigma_f=cfg.sigma_f, mu_range=cfg.mu_range, m_range=cfg.m_range,
                                    seed=cfg.seed), sdf=getattr(scene, "sdf", None),
                      sdf_box=getattr(scene, "sdf_box", None), device=device)
        if hidden:
            G = scene.G
            return cls(env_type=scene.hidden_type, group_start=np.arange(G + 1, dtype=np.int32),
                       state=scene.hidden_state, params=scene.hidden_params, **common, **kw)
        return cls(env_type=scene.env_type, group_start=scene.group_start, state=scene.state,
                   params=scene.params, **common, **kw)

    # -- state transfer (host arrays are env-major [K][13] / [K][5]) -------
    def set_state(self, state, params=None):
        self.state.copy_(torch.as_tensor(np.ascontiguousarray(np.asarray(state, dtype=np.float32).T)))
        if params is not None:
            self.params.copy_(torch.as_tensor(np.ascontiguousarray(np.asarray(params, dtype=np.float32).T)))

    def get_state(self):
        torch.cuda.synchronize(self.device)
        return self.state.cpu().numpy().T.astype(np.float64), self.params.cpu().numpy().T.astype(np.float64)

    def set_warm(self, keys, r):
        w = np.zeros((self.K, self.C_max, 4), dtype=np.float32)
        w[:, :, 0] = np.asarray(keys, dtype=np.int32).view(np.float32)
        w[:, :, 1:] = np.asarray(r, dtype=np.float32)
        self.warm.copy_(torch.as_tensor(w))

    def get_warm(self):
        torch.cuda.synchronize(self.device)
        w = self.warm.cpu().numpy()
        return np.ascontiguousarray(w[:, :, 0]).view(np.int32).copy(), w[:, :, 1:].astype(np.float64)

    def set_hand(self, hand_state):
        """Joint state from a host array [K][2D] (angles, then rates)."""
        self.hand_state.copy_(torch.as_tensor(np.ascontiguousarray(np.asarray(hand_state, dtype=np.float32).T)))

    def get_hand(self):
        torch.cuda.synchronize(self.device)
        return self.hand_state.cpu().numpy().T.astype(np.float64)

    def clear_warm(self):
        self.set_warm(np.full((self.K, self.C_max), -1, dtype=np.int32), np.zeros((self.K, self.C_max, 3)))

    # -- argument checks (the C ABI takes raw device pointers and cannot see
    #    a buffer's extent: a buffer shorter than the batch's sizes would be
    #    read or written past its end) -----------------------------------
    def _need(self, t, shape, name, dtype=torch.float32):
        if t is None:
            return
        if not isinstance(t, torch.Tensor):
            raise PtError(1, name, "expected a torch tensor")
        if t.device != self.device and not (t.device.type == self.device.type and self.device.index is None):
            raise PtError(1, name, f"on {t.device}, the batch is on {self.device}")
        if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise PtError(1, name, f"expected a contiguous {dtype} tensor of shape {tuple(shape)}, "
                                   f"got {t.dtype} {tuple(t.shape)}{'' if t.is_contiguous() else ' (not contiguous)'}")

    def _need_cmd(self, t, shape, name):
        # a hand without joints (D = 0) reads no commands
        if self.D > 0:
            self._need(t, shape, name)

    def _need_window(self, u_win, obs_gt_win):
        self._need_cmd(u_win, (self.T + 1, self.D), "u_win")
        self._need(obs_gt_win, (self.T, *self.obs_shape(self.G)), "obs_gt_win")

    # -- the hot path ------------------------------------------------------
    def obs_shape(self, n):
        """Shape of an observation of n simulations: [R][L][n], or with the
        PD hand [4L + D][n] (force rows, then the joint angles)."""
        if self.hand_mode == 1:
            return (4 * self.L + self.D, n)
        return (self.obs_rows, self.L, n)

    def new_obs(self, T=None):
        shape = self.obs_shape(self.K) if T is None else (T, *self.obs_shape(self.K))
        return torch.zeros(shape, dtype=torch.float32, device=self.device)

    def step(self, u_prev, u, stream=None):
        if self.hand_mode != 1:
            self._need_cmd(u_prev, (self.D,), "u_prev")
        self._need_cmd(u, (self.D,), "u")
        pt_step(self.handle, u_prev, u, stream)

    def observe(self, obs=None, stream=None):
        if obs is None:
            obs = self.new_obs()
        self._need(obs, self.obs_shape(self.K), "obs")
        pt_observe(self.handle, obs, stream)
        return obs

    def cost(self, obs, obs_gt, cost_sum, best=None, stream=None):
        self._need(obs, self.obs_shape(self.K), "obs")
        self._need(obs_gt, self.obs_shape(self.G), "obs_gt")
        self._need(cost_sum, (self.K,), "cost_sum")
        self._need(best, (self.G,), "best", torch.int32)
        pt_cost(self.handle, obs, obs_gt, cost_sum, best, stream)

    def resample(self, cost_sum, window_idx, parent=None, stream=None):
        self._need(cost_sum, (self.K,), "cost_sum")
        self._need(parent, (self.K,), "parent", torch.int32)
        pt_resample(self.handle, cost_sum, window_idx, parent, stream)

    def resample_wrs(self, cost_sum, n_steps, window_idx, lam, parent, weights=None, stream=None):
        self._need(cost_sum, (self.K,), "cost_sum")
        self._need(parent, (self.K,), "parent", torch.int32)
        self._need(weights, (self.K,), "weights")
        pt_resample_wrs(self.handle, cost_sum, n_steps, window_idx, lam, parent, weights, stream)

    def resample_reps(self, cost_sum, n_steps, window_idx, eps, parent, weights=None, eta=None, stream=None):
        self._need(cost_sum, (self.K,), "cost_sum")
        self._need(parent, (self.K,), "parent", torch.int32)
        self._need(weights, (self.K,), "weights")
        self._need(eta, (self.G,), "eta")
        pt_resample_reps(self.handle, cost_sum, n_steps, window_idx, eps, parent, weights, eta, stream)

    def run_window(self, u_win, obs_gt_win, cost_sum, best=None, obs_out=None, graph=True, stream=None):
        self._need_window(u_win, obs_gt_win)
        self._need(cost_sum, (self.K,), "cost_sum")
        self._need(best, (self.G,), "best", torch.int32)
        self._need(obs_out, (self.T, *self.obs_shape(self.K)), "obs_out")
        pt_run_window(self.handle, u_win, obs_gt_win, cost_sum, best, obs_out, graph, stream)

    def run_window_static(self, u_win, obs_gt_win, cost_sum, best=None, obs_out=None, stream=None):
        """pt_run_window without allocation or graph capture (scratch in a
        static device array; see include/pt.h)."""
        self._need_window(u_win, obs_gt_win)
        self._need(cost_sum, (self.K,), "cost_sum")
        self._need(best, (self.G,), "best", torch.int32)
        self._need(obs_out, (self.T, *self.obs_shape(self.K)), "obs_out")
        pt_run_window_static(self.handle, u_win, obs_gt_win, cost_sum, best, obs_out, stream)

    def autotune(self, u_win, obs_gt_win, stream=None):
        self._need_window(u_win, obs_gt_win)
        return pt_autotune(self.handle, u_win, obs_gt_win, stream)

    def set_tuning(self, waves_per_workgroup):
        pt_set_tuning(self.handle, waves_per_workgroup)

    # -- gradients and elite refinement -------------------------------------
    def start_of(self, env, state=None, params=None, warm=None):
        """Window start [18][n] and warm cache [n][C_max][4] of the listed
        simulations, gathered from the batch's buffers (or the given copies)."""
        state = self.state if state is None else state
        params = self.params if params is None else params
        warm = self.warm if warm is None else warm
        idx = env.long()
        return torch.cat([state[:, idx], params[:, idx]]).contiguous(), warm[idx].contiguous()

    def window_grad(self, u_win, obs_gt_win, env, start, warm0, want_grad=True, want_end=False, resid=None,
                    stream=None):
        """(cost, grad, end_state, end_warm) of the listed simulations'
        windows; resid (a [n] float32 tensor, optional) receives the
        largest final merit of each window's contact solves."""
        n = int(env.shape[0])
        self._need(resid, (n,), "resid")
        self._need_window(u_win, obs_gt_win)
        self._need(env, (n,), "env", torch.int32)
        self._need(start, (18, n), "start")
        self._need(warm0, (n, self.C_max, 4), "warm0")
        dev = self.device
        cost = torch.empty(n, dtype=torch.float32, device=dev)
        grad = torch.empty((18, n), dtype=torch.float32, device=dev) if want_grad else None
        end_state = torch.empty((13, n), dtype=torch.float32, device=dev) if want_end else None
        end_warm = torch.empty((n, self.C_max, 4), dtype=torch.float32, device=dev) if want_end else None
        pt_window_grad(self.handle, u_win, obs_gt_win, env, start, warm0, cost, grad, end_state, end_warm, resid,
                       stream)
        return cost, grad, end_state, end_warm

    def snapshot(self):
        """Copies of (state, params, warm) to pass as a window start."""
        return self.state.clone(), self.params.clone(), self.warm.clone()

    def elite_count(self):
        return pt_elite_count(self.handle)

    def refine_elites(self, u_win, obs_gt_win, cost_sum, start, steps=3, step=0.5, scale=None, best=None,
                      stream=None):
        self._need_window(u_win, obs_gt_win)
        self._need(cost_sum, (self.K,), "cost_sum")
        self._need(start[0], (13, self.K), "start state")
        self._need(start[1], (5, self.K), "start params")
        self._need(start[2], (self.K, self.C_max, 4), "start warm")
        self._need(best, (self.G,), "best", torch.int32)
        elites = torch.empty(self.elite_count(), dtype=torch.int32, device=self.device)
        pt_refine_elites(self.handle, u_win, obs_gt_win, cost_sum, start[0], start[1], start[2], steps, step, scale,
                         best, elites, stream)
        return elites

    def read_stats(self, stream=None):
        return pt_read_stats(self.handle, stream)

    def close(self):
        if getattr(self, "handle", None) is not None:
            pt_destroy_batch(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class WindowFn(torch.autograd.Function):
    """Window cost of listed simulations as a differentiable function of their
    window start: ``cost = WindowFn.apply(start, batch, env, warm0, u_win,
    obs_gt_win)`` with start [18][n] (x, q, v, omega, mass, mu, f_pert).  The
    forward pass runs pt_window_grad (forward sweep with checkpoints and the
    reverse sweep) and keeps d cost / d start; backward scales it by the
    incoming gradient of each simulation's cost."""

    @staticmethod
    def forward(ctx, start, batch, env, warm0, u_win, obs_gt_win):
        cost, grad, _, _ = batch.window_grad(u_win, obs_gt_win, env, start.detach().contiguous(), warm0,
                                             want_grad=ctx.needs_input_grad[0])
        ctx.save_for_backward(grad if grad is not None else cost.new_empty(0))
        return cost

    @staticmethod
    def backward(ctx, grad_cost):
        (g,) = ctx.saved_tensors
        if g.numel() == 0:
            return (None,) * 6
        return g * grad_cost.unsqueeze(0), None, None, None, None, None
