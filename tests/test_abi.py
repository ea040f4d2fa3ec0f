"""The C ABI: exports and host-side validation (CPU only, no kernel launches)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1802_05839_amd import wx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(wx_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(wx.LIB_PATH):
        pytest.skip("libwx.so is not built (run __graft_entry__.build())")
    return wx.load_library()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert {"wx_create", "wx_step", "wx_physics", "wx_destroy"} <= declared
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(wx.EXPORTS) <= declared


def _dz(nz):
    return (ctypes.c_double * nz)(*np.geomspace(50.0, 1000.0, nz))


def test_create_validates_and_reports_layout(lib):
    p = lib.wx_create(5, 4, 3, 2.0, 100.0, _dz(3))
    assert p
    s = p.contents
    assert (s.nx, s.ny, s.nz, s.halo) == (5, 4, 3, 2)
    assert s.stride_j % 64 == 0 and s.stride_j >= 9
    assert s.stride_k == s.stride_j * 8
    assert s.origin == 2 + 2 * s.stride_j
    assert s.field_elems == 3 * s.stride_k and s.wfield_elems == 4 * s.stride_k
    assert lib.wx_workspace_bytes(p, wx.WX_F32) < lib.wx_workspace_bytes(p, wx.WX_F64)
    assert lib.wx_workspace_bytes(p, 7) == 0
    lib.wx_destroy(p)
    for bad in ((3, 4, 3), (4, 3, 3), (4, 4, 2)):
        assert not lib.wx_create(*bad, 2.0, 100.0, _dz(3))
        assert b"outside" in lib.wx_last_error()
    assert not lib.wx_create(8, 8, 3, -1.0, 100.0, _dz(3))
    dz = _dz(3)
    dz[1] = 0.0
    assert not lib.wx_create(8, 8, 3, 1.0, 100.0, dz)
    assert b"dz[1]" in lib.wx_last_error()


def test_params_defaults_match_oracle(lib):
    from oracle.params import DEFAULT
    p = lib.wx_create(8, 8, 4, 2.0, 100.0, _dz(4))
    v = ctypes.c_double()
    expect = {"gamma4": DEFAULT.gamma4, "k_min": DEFAULT.k_min, "mix_len": DEFAULT.mix_len,
              "kappa_q": DEFAULT.kappa_q, "cp": DEFAULT.cp, "t_dd": DEFAULT.t_dd,
              "theta_offset": 0.0, "mass_every": 1.0}
    for name, val in expect.items():
        assert lib.wx_get_param(p, wx.PARAMS[name], ctypes.byref(v)) == wx.WX_OK
        assert v.value == val, name
    assert lib.wx_set_param(p, wx.PARAMS["cp"], 0.0) == wx.WX_E_INVAL
    assert lib.wx_set_param(p, wx.PARAMS["k_min"], -1.0) == wx.WX_E_INVAL
    assert lib.wx_set_param(p, wx.PARAMS["mass_every"], 1.5) == wx.WX_E_INVAL
    assert lib.wx_set_param(p, 99, 1.0) == wx.WX_E_INVAL
    assert lib.wx_set_param(p, wx.PARAMS["theta_offset"], -300.0) == wx.WX_OK
    lib.wx_destroy(p)


def test_step_rejects_incomplete_state_before_any_launch(lib):
    p = lib.wx_create(8, 8, 4, 2.0, 100.0, _dz(4))
    assert lib.wx_step(p, 1, None) == wx.WX_E_STATE
    assert b"rho" in lib.wx_last_error()
    s = p.contents
    for name in ("rho", "theta", "q", "u", "v", "w", "workspace", "mass_out", "flags_out",
                 "theta_s", "q_s", "f0", "ch"):
        setattr(s, name, 4096)          # never dereferenced: validation fails first
    s.rho = 4100                        # misaligned
    assert lib.wx_step(p, 1, None) == wx.WX_E_INVAL
    assert b"aligned" in lib.wx_last_error()
    s.rho = 4096
    s.phys_mode = 9
    assert lib.wx_step(p, 1, None) == wx.WX_E_UNSUPPORTED
    s.phys_mode = wx.WX_PHYS_PLAIN
    s.dtype = 5
    assert lib.wx_step(p, 1, None) == wx.WX_E_INVAL
    s.dtype = wx.WX_F32
    assert lib.wx_step(p, -1, None) == wx.WX_E_INVAL
    assert lib.wx_physics(p, None, wx.WX_PHYS_PLAIN) == wx.WX_E_INVAL
    assert lib.wx_physics(p, None, 7) == wx.WX_E_UNSUPPORTED
    assert lib.wx_copy_probe(None, None, 16, None) == wx.WX_E_INVAL
    lib.wx_destroy(p)


def test_surrogate_modes_validate_before_any_launch(lib):
    """Surrogate modes need an FP32 state with nz = 58, a blob, a workspace
    and (judged) judge_out; wx_surrogate_rows checks its arguments likewise."""
    def filled(nz, dtype):
        p = lib.wx_create(8, 8, nz, 2.0, 100.0, _dz(nz))
        s = p.contents
        for name in ("rho", "theta", "q", "u", "v", "w", "workspace", "mass_out", "flags_out",
                     "theta_s", "q_s", "f0", "ch"):
            setattr(s, name, 4096)      # never dereferenced: validation fails first
        s.dtype = dtype
        return p
    p = filled(4, wx.WX_F32)
    p.contents.phys_mode = wx.WX_PHYS_SURROGATE
    assert lib.wx_step(p, 1, None) == wx.WX_E_UNSUPPORTED and b"nz" in lib.wx_last_error()
    assert lib.wx_surrogate_rows(p, 4096, None, 1, 4096) == wx.WX_E_UNSUPPORTED
    lib.wx_destroy(p)
    p = filled(58, wx.WX_F64)
    p.contents.phys_mode = wx.WX_PHYS_JUDGED
    assert lib.wx_step(p, 1, None) == wx.WX_E_UNSUPPORTED and b"FP32" in lib.wx_last_error()
    assert lib.wx_surrogate_rows(p, 4096, None, 1, 4096) == wx.WX_E_UNSUPPORTED
    lib.wx_destroy(p)
    p = filled(58, wx.WX_F32)
    s = p.contents
    s.phys_mode = wx.WX_PHYS_SURROGATE
    assert lib.wx_step(p, 1, None) == wx.WX_E_STATE               # no blob, no workspace
    s.mlp, s.surrogate_work = 4096, 4096
    s.phys_mode = wx.WX_PHYS_JUDGED
    assert lib.wx_step(p, 1, None) == wx.WX_E_STATE and b"judge_out" in lib.wx_last_error()
    assert lib.wx_surrogate_rows(p, None, None, 1, 4096) == wx.WX_E_INVAL
    assert lib.wx_surrogate_rows(p, 4096, None, -1, 4096) == wx.WX_E_INVAL
    assert lib.wx_surrogate_rows(p, 4096, None, 8 * 8 + 1, 4096) == wx.WX_E_INVAL
    assert lib.wx_surrogate_rows(p, 4100, None, 1, 4096) == wx.WX_E_INVAL   # misaligned blob
    lib.wx_destroy(p)


def test_mlp_entry_points_validate(lib):
    assert lib.wx_mlp_work_bytes(0) == 0 and lib.wx_mlp_work_bytes(65537) == 0
    assert lib.wx_mlp_forward_backward(4096, 4096, 4096, 4096, 4096, 0, 4096, None) == wx.WX_E_INVAL
    assert lib.wx_mlp_forward_backward(None, 4096, 4096, 4096, 4096, 16, 4096, None) == wx.WX_E_INVAL
    assert lib.wx_mlp_adam(4096, 1e-3, 0, None) == wx.WX_E_INVAL
    assert lib.wx_mlp_adam(4100, 1e-3, 1, None) == wx.WX_E_INVAL
    assert lib.wx_mlp_infer(4096, 4096, 4096, 0, 4096, None) == wx.WX_E_INVAL
    assert lib.wx_mlp_offset(-1) == -1 and lib.wx_mlp_offset(36) == -1


def test_judge_rate_range(lib):
    p = lib.wx_create(8, 8, 4, 2.0, 100.0, _dz(4))
    assert lib.wx_set_param(p, 10, 0.0) == wx.WX_E_INVAL
    assert lib.wx_set_param(p, 10, 1e12) == wx.WX_E_INVAL          # the kernels take a 32-bit rate
    assert lib.wx_set_param(p, 10, 2.5) == wx.WX_E_INVAL
    assert lib.wx_set_param(p, 10, 4294967295.0) == wx.WX_OK
    lib.wx_destroy(p)



def test_reduced_app_validates_before_any_launch(lib):
    inval = wx.WX_E_INVAL
    a, b, s, p = 4096, 8192, 12288, 16384       # fake aligned addresses, never dereferenced
    assert lib.wx_rw_step(a, a, s, p, 4, 4, 4, 0.1, None) == inval           # same array twice
    assert lib.wx_rw_step(a, b, s, p, 4, 4, 1, 0.1, None) == inval           # nz < 2
    assert lib.wx_rw_step(a, b, s, p, 0, 4, 4, 0.1, None) == inval           # nx < 1
    assert lib.wx_rw_step(a, b, s, p, 4, 0, 4, 0.1, None) == inval           # ny < 1
    assert lib.wx_rw_step(a + 4, b, s, p, 4, 4, 4, 0.1, None) == inval       # misaligned
    assert lib.wx_rw_step(None, b, s, p, 4, 4, 4, 0.1, None) == inval
    assert lib.wx_rw_step(a, b, s, None, 4, 4, 4, 0.1, None) == inval
    assert lib.wx_rw_step(a, b, s, p, 4, 4, 4, float("nan"), None) == inval
    assert lib.wx_rw_step(a, b, s, p, 30000, 30000, 2, 0.1, None) == inval   # more than 2^29 cells
    which = ctypes.c_int(7)
    assert lib.wx_rw_run(a, b, s, p, 4, 4, 4, 0.1, -1, ctypes.byref(which), None) == inval
    assert lib.wx_rw_run(a, b, s, p, 4, 4, 4, 0.1, 1, None, None) == inval
    assert lib.wx_rw_run(a, b, s, p, 4, 4, 1, 0.1, 1, ctypes.byref(which), None) == inval
    # zero steps launch nothing and leave the result in the first array
    assert lib.wx_rw_run(a, b, s, p, 4, 4, 4, 0.1, 0, ctypes.byref(which), None) == wx.WX_OK
    assert which.value == 0
    # the KIJ-order entry point validates the same way
    assert lib.wx_rw_run_kij(a, a, s, p, 4, 4, 4, 0.1, 1, ctypes.byref(which), None) == inval
    assert lib.wx_rw_run_kij(a, b, s, p, 4, 4, 1, 0.1, 1, ctypes.byref(which), None) == inval
    assert lib.wx_rw_run_kij(a, b, s, p, 4, 4, 4, 0.1, -1, ctypes.byref(which), None) == inval
    which.value = 7
    assert lib.wx_rw_run_kij(a, b, s, p, 4, 4, 4, 0.1, 0, ctypes.byref(which), None) == wx.WX_OK
    assert which.value == 0


def test_mass_noalloc_rejects_grids_beyond_its_static_array(lib):
    # ceil(64/64) * 40961 partial blocks > WX_MASS_NOALLOC_MAX_PARTS: rejected on
    # the host before any pointer is looked at or any device call is made
    p = lib.wx_create(64, 40961, 3, 2.0, 100.0, _dz(3))
    assert p
    assert lib.wx_mass_noalloc(p) == wx.WX_E_INVAL
    assert b"at most 40960" in lib.wx_last_error()
    lib.wx_destroy(p)
    assert lib.wx_mass_noalloc(None) == wx.WX_E_INVAL
