"""The C-ABI library loads and exports every entry point include/pt.h
declares; descriptor validation errors are reported before any device call
(CPU only, no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2002_12160_amd", "libpt.so")
HEADER = os.path.join(ROOT, "include", "pt.h")


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^PT_API [^()]*?\b(pt_\w+)\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libpt.so is not built; run __graft_entry__.build()")
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("pt_create_batch", "pt_destroy_batch", "pt_step", "pt_observe", "pt_cost", "pt_resample",
                 "pt_run_window", "pt_autotune", "pt_read_stats", "pt_set_tuning", "pt_last_error",
                 "pt_window_grad", "pt_refine_elites", "pt_elite_count", "pt_resample_wrs", "pt_resample_reps"):
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_no_oracle_symbols_in_the_library(lib):
    # the product library shares no code with the test oracle
    for name in ("or_env_step", "or_hand_fk", "or_philox4x32_10", "or_resample_pbo", "or_resample_apply"):
        assert not hasattr(lib, name)


def _desc_module():
    from paper_2002_12160_amd import pt
    return pt


def _valid_desc(pt, keep):
    from paper_2002_12160_amd import scene as S
    sc = S.make_scene(S.CONFIGS["small"], K=8, steps=2)
    arrs = dict(hand=np.ascontiguousarray(sc.hand, np.float32), spheres=np.ascontiguousarray(sc.spheres, np.float32),
                nsph=np.ascontiguousarray(sc.n_spheres, np.int32),
                inv=np.ascontiguousarray(sc.inv_inertia, np.float32),
                typ=np.ascontiguousarray(sc.env_type, np.int32), gs=np.ascontiguousarray(sc.group_start, np.int32),
                st=np.zeros((13, 8), np.float32), pr=np.zeros((5, 8), np.float32), w=np.zeros((8, 16, 4), np.float32))
    keep.update(arrs)
    d = pt.BatchDesc()
    d.K, d.G, d.L, d.D, d.n_types, d.S_max, d.C_max, d.newton_iters, d.T = 8, 1, sc.L, sc.D, 1, sc.S_max, 16, 10, 10
    c = sc.cfg.consts
    d.dt, d.margin, d.erp, d.compliance, d.kappa, d.fb_delta = c.dt, c.margin, c.erp, c.compliance, c.kappa, c.fb_delta
    d.armijo_sigma, d.tau_contact, d.w_mag, d.w_dir = c.armijo_sigma, c.tau_contact, c.w_mag, c.w_dir
    d.gravity[2] = -9.81
    d.elite_frac, d.mu_lo, d.mu_hi, d.m_lo, d.m_hi = 0.25, 0.3, 1.0, 0.05, 0.2
    d.hand, d.spheres, d.n_spheres = arrs["hand"].ctypes.data, arrs["spheres"].ctypes.data, arrs["nsph"].ctypes.data
    d.inv_inertia, d.env_type, d.group_start = arrs["inv"].ctypes.data, arrs["typ"].ctypes.data, arrs["gs"].ctypes.data
    d.state, d.params, d.warm = arrs["st"].ctypes.data, arrs["pr"].ctypes.data, arrs["w"].ctypes.data
    return d


@pytest.mark.parametrize("field,value,code", [
    ("K", 0, 1), ("C_max", 65, 5), ("C_max", 0, 5), ("L", 0, 5), ("L", 63, 5), ("S_max", 257, 5),
    ("S_max", 300, 5), ("newton_iters", -1, 1),
    ("dt", 0.0, 1), ("T", 0, 1), ("G", 9, 1), ("elite_frac", 0.0, 1), ("fb_delta", 0.0, 1),
])
def test_descriptor_validation(lib, field, value, code):
    pt = _desc_module()
    keep = {}
    d = _valid_desc(pt, keep)
    setattr(d, field, value)
    h = C.c_void_p()
    rc = pt._lib.pt_create_batch(C.byref(d), C.byref(h))
    assert rc == code
    assert h.value is None
    assert len(pt._lib.pt_last_error()) > 0


def test_validation_of_tables(lib):
    pt = _desc_module()
    keep = {}
    d = _valid_desc(pt, keep)
    keep["typ"][3] = 7          # object type out of range
    h = C.c_void_p()
    assert pt._lib.pt_create_batch(C.byref(d), C.byref(h)) == 1
    assert b"env_type" in pt._lib.pt_last_error()
    keep["typ"][3] = 0
    keep["hand"][2, 0] = 5.0    # parent after child
    assert pt._lib.pt_create_batch(C.byref(d), C.byref(h)) == 1
    assert b"parent" in pt._lib.pt_last_error()
    keep["hand"][2, 0] = 1.0
    gs = np.array([0, 0, 8], np.int32)   # an empty group
    keep["gs2"] = gs
    d.G, d.group_start = 2, gs.ctypes.data
    assert pt._lib.pt_create_batch(C.byref(d), C.byref(h)) == 1
    assert b"non-empty" in pt._lib.pt_last_error()
    d.G, d.group_start = 1, keep["gs"].ctypes.data
    d.state = None
    assert pt._lib.pt_create_batch(C.byref(d), C.byref(h)) == 1


def test_null_handles_are_rejected(lib):
    pt = _desc_module()
    assert pt._lib.pt_step(None, None, None, None) == 1
    assert pt._lib.pt_observe(None, None, None) == 1
    assert pt._lib.pt_destroy_batch(None) == 0


def test_gradient_calls_reject_a_null_batch(lib):
    # argument errors come back before any device call
    lib.pt_window_grad.restype = C.c_int
    lib.pt_refine_elites.restype = C.c_int
    lib.pt_elite_count.restype = C.c_int32
    lib.pt_elite_count.argtypes = [C.c_void_p]
    assert lib.pt_window_grad(None, None, None, 0, None, None, None, None, None, None, None, None, None) == 1
    assert lib.pt_refine_elites(None, None, None, None, None, None, None, 3, C.c_float(0.5), None, None, None,
                                None) == 1
    assert lib.pt_elite_count(None) == -1


def test_weighted_resamplers_reject_bad_arguments(lib):
    # a NULL batch is rejected before any device call
    pt = _desc_module()
    f, g = pt._lib.pt_resample_wrs, pt._lib.pt_resample_reps
    assert f(None, None, 10, 0, C.c_float(1.0), None, None, None) == 1
    assert g(None, None, 10, 0, C.c_float(0.5), None, None, None, None) == 1


def test_binding_checks_buffer_shapes_before_the_call():
    # the binding rejects a buffer whose shape, type or layout does not match
    # the batch (the C ABI receives only its address) before anything runs
    import torch
    from paper_2002_12160_amd import pt

    b = pt.Batch.__new__(pt.Batch)
    b.device = torch.device("cpu")
    b.K, b.G, b.L, b.D, b.T, b.C_max, b.obs_rows, b.hand_mode = 8, 2, 3, 4, 10, 16, 4, 0
    ok_u = torch.zeros((11, 4))
    ok_gt = torch.zeros((10, 4, 3, 2))
    b._need_window(ok_u, ok_gt)
    for bad_u, bad_gt in ((torch.zeros((2, 4)), ok_gt),                 # fewer command rows than T + 1
                          (ok_u, torch.zeros((10, 4, 3, 1))),            # observed forces of too few groups
                          (ok_u.double(), ok_gt),                        # wrong type
                          (torch.zeros((4, 11)).t(), ok_gt)):           # not contiguous
        with pytest.raises(pt.PtError):
            b._need_window(bad_u, bad_gt)
    with pytest.raises(pt.PtError):
        b._need(torch.zeros(8, dtype=torch.float32), (8,), "best", torch.int32)
    with pytest.raises(pt.PtError):
        b._need(np.zeros(8, np.float32), (8,), "cost_sum")
    b._need(None, (8,), "optional")
    # the PD hand's window rows: 4 L force rows, then the D joint angles
    b.hand_mode = 1
    b._need_window(ok_u, torch.zeros((10, 4 * 3 + 4, 2)))
    with pytest.raises(pt.PtError):
        b._need_window(ok_u, ok_gt)


def _pd_desc(pt, keep):
    d = _valid_desc(pt, keep)
    d.hand_mode, d.kp, d.kd, d.link_mass, d.w_q = 1, 1.5, 0.05, 0.03, 100.0
    keep["hs"] = np.zeros((2 * d.D, 8), np.float32)
    d.hand_state = keep["hs"].ctypes.data
    return d


def _create_rc(pt, d):
    h = C.c_void_p()
    rc = pt._lib.pt_create_batch(C.byref(d), C.byref(h))
    if rc == 0:
        pt._lib.pt_destroy_batch(h)
    return rc


def test_pd_hand_descriptor_passes_validation(lib):
    # without a GPU the call gets as far as the first device call (PT_E_HIP)
    pt = _desc_module()
    keep = {}
    assert _create_rc(pt, _pd_desc(pt, keep)) in (0, 2)


@pytest.mark.parametrize("field,value,code", [
    ("hand_mode", 2, 1), ("kp", -1.0, 1), ("kd", float("nan"), 1), ("link_mass", 0.0, 1), ("w_q", -1.0, 1),
    ("solve_precision", 32, 5), ("cost_mode", 1, 5), ("hand_state", None, 1), ("window_checkpoints", 1, 5),
])
def test_pd_hand_descriptor_validation(lib, field, value, code):
    pt = _desc_module()
    keep = {}
    d = _pd_desc(pt, keep)
    setattr(d, field, value)
    assert _create_rc(pt, d) == code
    assert len(pt._lib.pt_last_error()) > 0


def test_pd_hand_needs_stiffness_or_damping(lib):
    pt = _desc_module()
    keep = {}
    d = _pd_desc(pt, keep)
    d.kp, d.kd = 0.0, 0.0
    assert _create_rc(pt, d) == 1


def test_pd_hand_structure_limits(lib):
    pt = _desc_module()
    keep = {}
    d = _pd_desc(pt, keep)
    # a joint driving two links
    keep["hand"][1, 1] = keep["hand"][0, 1]
    assert _create_rc(pt, d) == 5
    assert b"drives links" in pt._lib.pt_last_error()
    # a chain of seven links with one joint each: one group of seven joints
    chain = np.zeros((7, 20), np.float32)
    for l in range(7):
        chain[l, 0] = l - 1
        chain[l, 1], chain[l, 2] = l, -1
        chain[l, 4] = 1.0
        chain[l, 12] = 1.0
        chain[l, 16], chain[l, 17] = 0.02, 0.005
    keep["chain"] = chain
    keep["hs7"] = np.zeros((14, 8), np.float32)
    d.hand, d.L, d.D, d.hand_state = chain.ctypes.data, 7, 7, keep["hs7"].ctypes.data
    assert _create_rc(pt, d) == 5
    assert b"group" in pt._lib.pt_last_error()
    chain[6, 1] = -1            # six joints in the chain: within the limit
    d.D = 6
    assert _create_rc(pt, d) in (0, 2)


def _sdf_desc(pt, keep, n=8):
    d = _valid_desc(pt, keep)
    d.collision_mode, d.link_samples, d.sdf_n = 1, 8, n
    keep["sdf"] = np.zeros((1, n, n, n), np.float32)
    keep["sdf_box"] = np.array([[-0.05, -0.05, -0.05, 0.1 / (n - 1)]], np.float32)
    d.sdf, d.sdf_box = keep["sdf"].ctypes.data, keep["sdf_box"].ctypes.data
    return d


def test_sdf_descriptor_passes_validation(lib):
    pt = _desc_module()
    keep = {}
    assert _create_rc(pt, _sdf_desc(pt, keep)) in (0, 2)


@pytest.mark.parametrize("field,value,code", [
    ("collision_mode", 2, 1), ("link_samples", 0, 1), ("link_samples", 65, 1), ("sdf_n", 1, 5),
    ("sdf_n", 129, 5), ("sdf", None, 1), ("sdf_box", None, 1), ("solve_precision", 32, 5), ("cost_mode", 1, 5),
])
def test_sdf_descriptor_validation(lib, field, value, code):
    pt = _desc_module()
    keep = {}
    d = _sdf_desc(pt, keep)
    setattr(d, field, value)
    assert _create_rc(pt, d) == code
    assert len(pt._lib.pt_last_error()) > 0


def test_sdf_tables_are_checked(lib):
    pt = _desc_module()
    keep = {}
    d = _sdf_desc(pt, keep)
    keep["sdf_box"][0, 3] = 0.0             # zero spacing
    assert _create_rc(pt, d) == 1
    keep["sdf_box"][0, 3] = 0.01
    keep["sdf"][0, 3, 4, 5] = np.nan        # a node value that is not finite
    assert _create_rc(pt, d) == 1
    keep["sdf"][0, 3, 4, 5] = 0.0
    d.link_samples = 64                     # 9 links x 64 samples + 26 spheres: 602 candidates
    d.L = 9
    assert _create_rc(pt, d) in (0, 2)
    keep["hand25"] = np.tile(keep["hand"][:1], (25, 1))
    d.hand, d.L = keep["hand25"].ctypes.data, 25   # 25 x 64 + 26 > 1536
    assert _create_rc(pt, d) == 5
