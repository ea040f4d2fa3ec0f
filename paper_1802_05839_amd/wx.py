"""Python binding of ``libwx.so`` (include/wx.h): argument marshalling only.

Every step of the weather step runs in the HIP library; this module allocates
device buffers with torch (PyTorch is used for device memory and streams
only), copies host arrays into the library's padded i-fastest layout, calls
the C entry points and copies results back.  There is no fallback: if the
library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libwx.so")

WX_OK, WX_E_INVAL, WX_E_HIP, WX_E_STATE, WX_E_UNSUPPORTED = 0, -1, -2, -3, -4
WX_F32, WX_F64 = 0, 1
WX_PHYS_OFF, WX_PHYS_PLAIN, WX_PHYS_SURROGATE, WX_PHYS_JUDGED, WX_PHYS_DATASET = 0, 1, 2, 3, 4
PROFILE_CLASSES = ("halo", "stage1", "stage2", "stage3", "physics", "mass_final", "judge",
                   "surrogate", "sampled_apply")
PARAMS = {"gamma4": 0, "k_min": 1, "mix_len": 2, "kappa_q": 3, "cp": 4, "t_dd": 5,
          "theta_offset": 6, "mass_every": 7, "judge_seed": 8, "judge_rel": 9, "judge_rate": 10,
          "step": 11, "phys_kernel": 12, "stage_tile": 13}
FLAG_NAMES = ("nonfinite", "rho_le0", "fp64_columns", "fallback_steps")
HALO = 2

EXPORTS = ("wx_create", "wx_destroy", "wx_last_error", "wx_workspace_bytes", "wx_set_param",
           "wx_get_param", "wx_halo", "wx_step", "wx_physics", "wx_mass", "wx_profile_step",
           "wx_copy_probe", "wx_features", "wx_dataset", "wx_surrogate_rows", "wx_mlp_bytes", "wx_mlp_offset",
           "wx_mlp_init", "wx_mlp_refresh", "wx_mlp_norm_scratch_bytes", "wx_mlp_fit_norm",
           "wx_mlp_normalize", "wx_mlp_work_bytes", "wx_mlp_forward_backward", "wx_mlp_adam",
           "wx_mlp_train_step", "wx_mlp_shuffle", "wx_mlp_infer_work_bytes", "wx_mlp_infer",
           "wx_surrogate_work_bytes", "wx_rw_step", "wx_rw_run", "wx_rw_run_kij", "wx_mass_noalloc",
           "wx_rw_run_block", "wx_hevi_grid_init", "wx_hevi_workspace_bytes", "wx_hevi_run")

# surrogate network shapes and blob sections (include/wx.h)
MLP_NZ, MLP_NIN, MLP_KIN, MLP_NHID, MLP_NOUT, MLP_NOUTP = 58, 294, 320, 512, 116, 128
MLP_SECTIONS = {"W1": 0, "b1": 1, "W2": 2, "b2": 3, "W3": 4, "b3": 5, "grad": 6, "adam_m": 12,
                "adam_v": 18, "W1_bf16": 24, "W2_bf16": 25, "W3_bf16": 26, "W2T_bf16": 27,
                "W3T_bf16": 28, "x_mean": 29, "x_invstd": 30, "y_mean": 31, "y_std": 32,
                "sigma": 33, "sigma64": 34, "wpack_bf16": 35}
MLP_PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")
MLP_PARAM_SHAPES = {"W1": (MLP_NHID, MLP_KIN), "b1": (MLP_NHID,), "W2": (MLP_NHID, MLP_NHID),
                    "b2": (MLP_NHID,), "W3": (MLP_NOUTP, MLP_NHID), "b3": (MLP_NOUTP,)}


class WxError(RuntimeError):
    pass


class _State(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("halo", ctypes.c_int32),
        ("stride_j", ctypes.c_int64), ("stride_k", ctypes.c_int64), ("origin", ctypes.c_int64),
        ("field_elems", ctypes.c_int64), ("wfield_elems", ctypes.c_int64),
        ("dt", ctypes.c_double), ("dx", ctypes.c_double),
        ("dtype", ctypes.c_int32), ("phys_mode", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("rho", ctypes.c_void_p), ("theta", ctypes.c_void_p), ("q", ctypes.c_void_p),
        ("u", ctypes.c_void_p), ("v", ctypes.c_void_p), ("w", ctypes.c_void_p),
        ("theta_s", ctypes.c_void_p), ("q_s", ctypes.c_void_p), ("f0", ctypes.c_void_p),
        ("ch", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("mass_out", ctypes.c_void_p), ("flags_out", ctypes.c_void_p),
        ("mlp", ctypes.c_void_p), ("surrogate_work", ctypes.c_void_p), ("judge_out", ctypes.c_void_p),
        ("impl", ctypes.c_void_p),
    ]


class _Tend(ctypes.Structure):
    _fields_ = [("dtheta", ctypes.c_void_p), ("dq", ctypes.c_void_p), ("features", ctypes.c_void_p),
                ("labels", ctypes.c_void_p)]


class _HeviGrid(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("stride_j", ctypes.c_int64), ("stride_k", ctypes.c_int64), ("origin", ctypes.c_int64),
        ("cell_elems", ctypes.c_int64), ("face_elems", ctypes.c_int64),
        ("dx", ctypes.c_double), ("tau", ctypes.c_double), ("c_sound", ctypes.c_double),
        ("n_bv", ctypes.c_double), ("kernel", ctypes.c_int32), ("pad", ctypes.c_int32),
    ]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libwx.so and declare the C signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise WxError(f"{path} is missing: build it with `python -m paper_1802_05839_amd._build`")
    lib = ctypes.CDLL(path)
    sp = ctypes.POINTER(_State)
    lib.wx_create.restype = sp
    lib.wx_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    lib.wx_destroy.restype = None
    lib.wx_destroy.argtypes = [sp]
    lib.wx_last_error.restype = ctypes.c_char_p
    lib.wx_last_error.argtypes = []
    lib.wx_workspace_bytes.restype = ctypes.c_size_t
    lib.wx_workspace_bytes.argtypes = [sp, ctypes.c_int]
    lib.wx_set_param.argtypes = [sp, ctypes.c_int, ctypes.c_double]
    lib.wx_get_param.argtypes = [sp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.wx_halo.argtypes = [sp, ctypes.c_void_p]
    lib.wx_step.argtypes = [sp, ctypes.c_int, ctypes.c_void_p]
    lib.wx_physics.argtypes = [sp, ctypes.POINTER(_Tend), ctypes.c_int]
    lib.wx_mass.argtypes = [sp]
    lib.wx_mass_noalloc.argtypes = [sp]
    lib.wx_profile_step.argtypes = [sp, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    lib.wx_copy_probe.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.wx_features.argtypes = [sp, ctypes.c_int, vp, vp]
    lib.wx_dataset.argtypes = [sp, vp, vp]
    lib.wx_surrogate_rows.argtypes = [sp, vp, vp, ctypes.c_int, vp]
    lib.wx_mlp_bytes.argtypes = []
    lib.wx_mlp_offset.argtypes = [ctypes.c_int]
    lib.wx_mlp_init.argtypes = [vp, ctypes.c_uint64, vp]
    lib.wx_mlp_refresh.argtypes = [vp, vp]
    lib.wx_mlp_norm_scratch_bytes.argtypes = [sz]
    lib.wx_mlp_fit_norm.argtypes = [vp, vp, vp, sz, vp, vp]
    lib.wx_mlp_normalize.argtypes = [vp, vp, vp, sz, vp, vp, vp]
    lib.wx_mlp_work_bytes.argtypes = [ctypes.c_int]
    lib.wx_mlp_forward_backward.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, vp, vp]
    lib.wx_mlp_adam.argtypes = [vp, ctypes.c_float, ctypes.c_int, vp]
    lib.wx_mlp_train_step.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_float, ctypes.c_int,
                                      vp, vp]
    lib.wx_mlp_shuffle.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, vp, vp]
    lib.wx_mlp_infer_work_bytes.argtypes = [ctypes.c_int]
    lib.wx_mlp_infer.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp]
    lib.wx_surrogate_work_bytes.argtypes = [sp]
    dbl, i32 = ctypes.c_double, ctypes.c_int
    lib.wx_rw_step.argtypes = [vp, vp, vp, vp, i32, i32, i32, dbl, vp]
    lib.wx_rw_run.argtypes = [vp, vp, vp, vp, i32, i32, i32, dbl, i32, ctypes.POINTER(i32), vp]
    lib.wx_rw_run_kij.argtypes = [vp, vp, vp, vp, i32, i32, i32, dbl, i32, ctypes.POINTER(i32), vp]
    lib.wx_rw_run_block.argtypes = [vp, vp, vp, vp, i32, i32, i32, dbl, i32, ctypes.POINTER(i32), i32, i32, vp]
    hg = ctypes.POINTER(_HeviGrid)
    lib.wx_hevi_grid_init.argtypes = [hg, i32, i32, i32, i32, dbl, dbl, dbl, dbl]
    lib.wx_hevi_workspace_bytes.argtypes = [hg]
    lib.wx_hevi_run.argtypes = [hg, ctypes.POINTER(dbl), vp, vp, vp, vp, vp, vp, i32, vp]
    size_returning = {"wx_workspace_bytes", "wx_mlp_bytes", "wx_mlp_norm_scratch_bytes",
                      "wx_mlp_work_bytes", "wx_mlp_infer_work_bytes", "wx_surrogate_work_bytes",
                      "wx_hevi_workspace_bytes"}
    for name in EXPORTS[4:]:
        if name in size_returning:
            getattr(lib, name).restype = ctypes.c_size_t
        elif name == "wx_mlp_offset":
            getattr(lib, name).restype = ctypes.c_int64
        else:
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str) -> None:
    if rc != WX_OK:
        msg = _lib.wx_last_error().decode() if _lib is not None else ""
        raise WxError(f"{what} failed ({rc}): {msg}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise WxError("no GPU visible: the wx library runs on an MI355X only")
    return torch


def _stream_ptr(stream=None) -> int:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class State:
    """A device-resident weather state borrowed by libwx (buffers owned here)."""

    def __init__(self, nx: int, ny: int, nz: int, dt: float, dx: float, dz, dtype: str = "f32",
                 phys_mode: int = WX_PHYS_PLAIN, device: str = "cuda:0"):
        torch = _torch()
        lib = load_library()
        self.lib = lib
        dz = np.ascontiguousarray(dz, dtype=np.float64)
        if dz.shape != (nz,):
            raise WxError("dz must have nz entries")
        p = lib.wx_create(nx, ny, nz, float(dt), float(dx),
                          dz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if not p:
            raise WxError("wx_create failed: " + lib.wx_last_error().decode())
        self._p = p
        s = p.contents
        self.nx, self.ny, self.nz = nx, ny, nz
        self.dt, self.dx, self.dz = float(dt), float(dx), dz.copy()
        self.sj, self.sk = int(s.stride_j), int(s.stride_k)
        self.field_elems, self.wfield_elems = int(s.field_elems), int(s.wfield_elems)
        self.dtype = dtype
        self.tdt = torch.float32 if dtype == "f32" else torch.float64
        self.np_dtype = np.float32 if dtype == "f32" else np.float64
        self.device = torch.device(device)
        s.dtype = WX_F32 if dtype == "f32" else WX_F64
        s.phys_mode = phys_mode
        dev = self.device

        def alloc(n):
            return torch.zeros(n, dtype=self.tdt, device=dev)

        self.t = {name: alloc(self.field_elems) for name in ("rho", "theta", "q", "u", "v")}
        self.t["w"] = alloc(self.wfield_elems)
        for name in ("theta_s", "q_s", "f0", "ch"):
            self.t[name] = alloc(nx * ny)
        wsb = int(lib.wx_workspace_bytes(p, s.dtype))
        self.t["workspace"] = torch.zeros(wsb, dtype=torch.uint8, device=dev)
        self.t["mass_out"] = torch.zeros(6, dtype=torch.float64, device=dev)
        self.t["flags_out"] = torch.zeros(4, dtype=torch.int32, device=dev)
        for name, ten in self.t.items():
            setattr(s, name, ten.data_ptr())
        self.theta_offset = 0.0

    # ---- layout helpers -------------------------------------------------
    def _padded(self, t, planes):
        return t.view(planes, self.ny + 2 * HALO, self.sj)

    def interior(self, name: str):
        planes = self.nz + 1 if name == "w" else self.nz
        return self._padded(self.t[name], planes)[:, HALO:HALO + self.ny, HALO:HALO + self.nx]

    # ---- parameters ------------------------------------------------------
    def set_param(self, name: str, value: float) -> None:
        _check(self.lib.wx_set_param(self._p, PARAMS[name], float(value)), f"wx_set_param({name})")
        if name == "theta_offset":
            self.theta_offset = float(value)

    def get_param(self, name: str) -> float:
        out = ctypes.c_double()
        _check(self.lib.wx_get_param(self._p, PARAMS[name], ctypes.byref(out)), "wx_get_param")
        return out.value

    # ---- data movement ---------------------------------------------------
    def upload(self, inp, theta_offset: Optional[float] = None) -> None:
        """Copy a host problem into the device buffers (halo filled by the library).

        theta (and theta_s) are stored as theta - theta_offset; the default is
        300 K for FP32 state and 0 for FP64.
        """
        torch = _torch()
        if theta_offset is None:
            theta_offset = 300.0 if self.dtype == "f32" else 0.0
        self.set_param("theta_offset", theta_offset)
        src = {"rho": inp.rho, "theta": inp.theta - theta_offset, "q": inp.q, "u": inp.u,
               "v": inp.v, "w": inp.w}
        for name, arr in src.items():
            self.interior(name).copy_(torch.from_numpy(np.ascontiguousarray(arr, dtype=self.np_dtype)))
        two = {"theta_s": inp.theta_s - theta_offset, "q_s": inp.q_s, "f0": inp.f0, "ch": inp.ch}
        for name, arr in two.items():
            self.t[name].copy_(torch.from_numpy(np.ascontiguousarray(arr, dtype=self.np_dtype).ravel()))
        self.halo()

    def download(self, names=("rho", "theta", "q")) -> Dict[str, np.ndarray]:
        """Interior of the state as float64 arrays (theta with the offset added back)."""
        torch = _torch()
        torch.cuda.synchronize(self.device)
        out = {}
        for name in names:
            a = self.interior(name).cpu().numpy().astype(np.float64)
            if name == "theta":
                a = a + self.theta_offset
            out[name] = a
        return out

    def download_raw(self, name: str) -> np.ndarray:
        """Whole padded buffer (halo included) in storage precision."""
        torch = _torch()
        torch.cuda.synchronize(self.device)
        planes = self.nz + 1 if name == "w" else self.nz
        return self._padded(self.t[name], planes).cpu().numpy()

    # ---- entry points ----------------------------------------------------
    def halo(self, stream=None) -> None:
        _check(self.lib.wx_halo(self._p, _stream_ptr(stream)), "wx_halo")

    def step(self, nsteps: int, stream=None) -> None:
        _check(self.lib.wx_step(self._p, int(nsteps), _stream_ptr(stream)), "wx_step")

    def set_phys_mode(self, mode: int) -> None:
        self._p.contents.phys_mode = int(mode)

    def attach_mlp(self, mlp: "Mlp") -> None:
        """Use a trained surrogate: sets the blob and allocates the surrogate workspace."""
        torch = _torch()
        s = self._p.contents
        self.mlp = mlp
        s.mlp = mlp.blob.data_ptr()
        self.t["surrogate_work"] = torch.zeros(int(self.lib.wx_surrogate_work_bytes(self._p)),
                                               dtype=torch.uint8, device=self.device)
        self.t["judge_out"] = torch.zeros(6, dtype=torch.float64, device=self.device)
        s.surrogate_work = self.t["surrogate_work"].data_ptr()
        s.judge_out = self.t["judge_out"].data_ptr()

    def judge(self):
        """(RMSE theta, RMSE q, fallback, sampled columns, fraction of sampled
        columns over the bound in theta, in q) of the last judged step."""
        torch = _torch()
        torch.cuda.synchronize(self.device)
        j = self.t["judge_out"].cpu().numpy()
        return float(j[0]), float(j[1]), bool(j[2]), int(j[3]), float(j[4]), float(j[5])

    def tendencies(self, stream=None, mode: int = WX_PHYS_PLAIN):
        """Tendencies (dtheta/dt, dq/dt) of the current state from wx_physics in
        ``mode`` (plain, surrogate or judged), (nz, ny, nx) float64."""
        torch = _torch()
        s = self._p.contents
        s.stream = _stream_ptr(stream)
        tt = torch.zeros(self.nx * self.ny * self.nz, dtype=self.tdt, device=self.device)
        tq = torch.zeros_like(tt)
        tend = _Tend(tt.data_ptr(), tq.data_ptr(), None, None)
        _check(self.lib.wx_physics(self._p, ctypes.byref(tend), int(mode)), "wx_physics")
        torch.cuda.synchronize(self.device)
        shp = (self.nz, self.ny, self.nx)
        return (tt.cpu().numpy().astype(np.float64).reshape(shp),
                tq.cpu().numpy().astype(np.float64).reshape(shp))

    def mass(self, compute: bool = False, stream=None) -> np.ndarray:
        """(M_rho, M_theta, M_q) as sum + compensation; ``compute`` runs wx_mass first."""
        torch = _torch()
        if compute:
            self._p.contents.stream = _stream_ptr(stream)
            _check(self.lib.wx_mass(self._p), "wx_mass")
        torch.cuda.synchronize(self.device)
        m = self.t["mass_out"].cpu().numpy()
        return np.array([m[0] + m[1], m[2] + m[3], m[4] + m[5]])

    def mass_noalloc(self, stream=None) -> None:
        """Run wx_mass_noalloc (the same sums into mass_out, partials in the
        library's static device array; the workspace is not used)."""
        self._p.contents.stream = _stream_ptr(stream)
        _check(self.lib.wx_mass_noalloc(self._p), "wx_mass_noalloc")

    def mass_raw(self) -> np.ndarray:
        torch = _torch()
        torch.cuda.synchronize(self.device)
        return self.t["mass_out"].cpu().numpy().copy()

    def flags(self) -> Dict[str, int]:
        torch = _torch()
        torch.cuda.synchronize(self.device)
        f = self.t["flags_out"].cpu().numpy()
        return {n: int(v) for n, v in zip(FLAG_NAMES, f)}

    def profile(self, nsteps: int, stream=None) -> np.ndarray:
        """Average ms per launch of each class (PROFILE_CLASSES order)."""
        n = len(PROFILE_CLASSES)
        out = (ctypes.c_double * n)()
        _check(self.lib.wx_profile_step(self._p, int(nsteps), _stream_ptr(stream), out, n),
               "wx_profile_step")
        return np.array(out[:])

    def features(self, mlp=None, stream=None):
        """Feature rows of the current state: raw FP32 (mlp None) or normalised BF16."""
        torch = _torch()
        self._p.contents.stream = _stream_ptr(stream)
        n = self.nx * self.ny
        if mlp is None:
            out = torch.zeros(n, MLP_KIN, dtype=torch.float32, device=self.device)
            _check(self.lib.wx_features(self._p, 0, out.data_ptr(), None), "wx_features")
        else:
            out = torch.zeros(n, MLP_KIN, dtype=torch.int16, device=self.device)
            _check(self.lib.wx_features(self._p, 1, out.data_ptr(), mlp.blob.data_ptr()), "wx_features")
        return out

    def surrogate_rows(self, mlp, cols=None, n=None, stream=None):
        """Normalised network outputs [n][128] of the fused kernel for columns
        cols (device int32 tensor) or columns 0..n-1."""
        torch = _torch()
        self._p.contents.stream = _stream_ptr(stream)
        if cols is not None:
            n = int(cols.shape[0])
        elif n is None:
            n = self.nx * self.ny
        out = torch.zeros(max(n, 1), MLP_NOUTP, dtype=torch.float32, device=self.device)
        _check(self.lib.wx_surrogate_rows(self._p, mlp.blob.data_ptr(),
                                          None if cols is None else cols.data_ptr(), int(n),
                                          out.data_ptr()), "wx_surrogate_rows")
        return out[:n]

    def dataset(self, x_raw=None, y_raw=None, stream=None):
        """(raw features [ncol, 320], plain-physics targets [ncol, 128]) as device tensors."""
        torch = _torch()
        self._p.contents.stream = _stream_ptr(stream)
        n = self.nx * self.ny
        if x_raw is None:
            x_raw = torch.zeros(n, MLP_KIN, dtype=torch.float32, device=self.device)
        if y_raw is None:
            y_raw = torch.zeros(n, MLP_NOUTP, dtype=torch.float32, device=self.device)
        _check(self.lib.wx_dataset(self._p, x_raw.data_ptr(), y_raw.data_ptr()), "wx_dataset")
        return x_raw, y_raw

    def dataset_via_physics(self, stream=None):
        """The same rows through wx_physics(WX_PHYS_DATASET)."""
        torch = _torch()
        self._p.contents.stream = _stream_ptr(stream)
        n = self.nx * self.ny
        x_raw = torch.zeros(n, MLP_KIN, dtype=torch.float32, device=self.device)
        y_raw = torch.zeros(n, MLP_NOUTP, dtype=torch.float32, device=self.device)
        tend = _Tend(None, None, x_raw.data_ptr(), y_raw.data_ptr())
        _check(self.lib.wx_physics(self._p, ctypes.byref(tend), WX_PHYS_DATASET), "wx_physics(DATASET)")
        return x_raw, y_raw

    def close(self) -> None:
        if getattr(self, "_p", None):
            _torch().cuda.synchronize(self.device)
            self.lib.wx_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            if getattr(self, "_p", None):
                self.lib.wx_destroy(self._p)
                self._p = None
        except Exception:
            pass


def copy_probe(dst, src, stream=None) -> None:
    """Run the library's plain copy kernel from one torch tensor to another."""
    lib = load_library()
    nbytes = src.numel() * src.element_size()
    _check(lib.wx_copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, _stream_ptr(stream)),
           "wx_copy_probe")


def state_from_inputs(inp, dtype: str = "f32", phys_mode: int = WX_PHYS_PLAIN,
                      theta_offset: Optional[float] = None, device: str = "cuda:0") -> State:
    st = State(inp.nx, inp.ny, inp.nz, inp.dt, inp.dx, inp.dz, dtype=dtype, phys_mode=phys_mode,
               device=device)
    st.upload(inp, theta_offset=theta_offset)
    return st


def bf16_bits_to_float(t):
    """Device int16 tensor of BF16 bit patterns -> float32 tensor (exact)."""
    torch = _torch()
    return (t.to(torch.int32) << 16).view(torch.float32)


def shuffle(seed: int, epoch: int, n: int, out, stream=None) -> None:
    """Training row order of one epoch, drawn on the device (wx_mlp_shuffle):
    out[i] = P(i) for the first out.numel() elements of a permutation P of
    0..n-1 fixed by (seed, epoch).  out: int32 CUDA tensor."""
    lib = load_library()
    _check(lib.wx_mlp_shuffle(int(seed), int(epoch), int(n), int(out.numel()), out.data_ptr(),
                              _stream_ptr(stream)), "wx_mlp_shuffle")


class Mlp:
    """The surrogate's parameter blob (device memory owned here)."""

    def __init__(self, device: str = "cuda:0"):
        torch = _torch()
        self.lib = load_library()
        self.device = torch.device(device)
        self.blob = torch.zeros(int(self.lib.wx_mlp_bytes()), dtype=torch.uint8, device=self.device)
        self._work = None
        self._work_batch = 0
        self._infer_work = None
        self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    def _sec(self, name: str, dtype, shape):
        torch = _torch()
        off = int(self.lib.wx_mlp_offset(MLP_SECTIONS[name] if isinstance(name, str) else name))
        n = int(np.prod(shape))
        esize = torch.empty(0, dtype=dtype).element_size()
        return self.blob[off:off + n * esize].view(dtype).view(*shape)

    def param(self, name: str, kind: str = "param"):
        """FP32 view of a parameter ("param"), its gradient ("grad") or Adam moment ("adam_m", "adam_v")."""
        torch = _torch()
        base = {"param": 0, "grad": 6, "adam_m": 12, "adam_v": 18}[kind]
        return self._sec(base + MLP_PARAM_NAMES.index(name), torch.float32, MLP_PARAM_SHAPES[name])

    def sigma(self):
        torch = _torch()
        return self._sec("sigma64", torch.float64, (2,))

    def init(self, seed: int, stream=None) -> None:
        _check(self.lib.wx_mlp_init(self.blob.data_ptr(), int(seed), _stream_ptr(stream)), "wx_mlp_init")

    def set_params(self, params: Dict[str, np.ndarray], stream=None) -> None:
        """Write FP32 weights (unpadded shapes are zero-padded) and refresh the BF16 copies."""
        torch = _torch()
        for name, arr in params.items():
            full = np.zeros(MLP_PARAM_SHAPES[name], dtype=np.float32)
            full[tuple(slice(0, n) for n in arr.shape)] = arr
            self.param(name).copy_(torch.from_numpy(full))
        _check(self.lib.wx_mlp_refresh(self.blob.data_ptr(), _stream_ptr(stream)), "wx_mlp_refresh")

    def fit_norm(self, x_raw, y_raw, stream=None) -> None:
        torch = _torch()
        n = x_raw.shape[0]
        scratch = torch.zeros(int(self.lib.wx_mlp_norm_scratch_bytes(n)), dtype=torch.uint8,
                              device=self.device)
        _check(self.lib.wx_mlp_fit_norm(self.blob.data_ptr(), x_raw.data_ptr(), y_raw.data_ptr(), n,
                                        scratch.data_ptr(), _stream_ptr(stream)), "wx_mlp_fit_norm")
        torch.cuda.synchronize(self.device)

    def normalize(self, x_raw, y_raw=None, stream=None):
        torch = _torch()
        n = x_raw.shape[0]
        xo = torch.zeros(n, MLP_KIN, dtype=torch.int16, device=self.device)
        yo = torch.zeros(n, MLP_NOUTP, dtype=torch.float32, device=self.device) if y_raw is not None else None
        _check(self.lib.wx_mlp_normalize(self.blob.data_ptr(), x_raw.data_ptr(),
                                         None if y_raw is None else y_raw.data_ptr(), n, xo.data_ptr(),
                                         None if yo is None else yo.data_ptr(), _stream_ptr(stream)),
               "wx_mlp_normalize")
        return xo, yo

    def _ensure_work(self, batch: int):
        torch = _torch()
        if self._work is None or self._work_batch < batch:
            self._work = torch.zeros(int(self.lib.wx_mlp_work_bytes(batch)), dtype=torch.uint8,
                                     device=self.device)
            self._work_batch = batch

    def forward_backward(self, x, y, rows, stream=None) -> None:
        batch = int(rows.shape[0])
        self._ensure_work(batch)
        _check(self.lib.wx_mlp_forward_backward(self.blob.data_ptr(), self._work.data_ptr(), x.data_ptr(),
                                                y.data_ptr(), rows.data_ptr(), batch, self._loss.data_ptr(),
                                                _stream_ptr(stream)), "wx_mlp_forward_backward")

    def adam(self, lr: float, t: int, stream=None) -> None:
        _check(self.lib.wx_mlp_adam(self.blob.data_ptr(), float(lr), int(t), _stream_ptr(stream)), "wx_mlp_adam")

    def train_step(self, x, y, rows, lr: float, t: int, stream=None) -> None:
        batch = int(rows.shape[0])
        self._ensure_work(batch)
        _check(self.lib.wx_mlp_train_step(self.blob.data_ptr(), self._work.data_ptr(), x.data_ptr(),
                                          y.data_ptr(), rows.data_ptr(), batch, float(lr), int(t),
                                          self._loss.data_ptr(), _stream_ptr(stream)), "wx_mlp_train_step")

    def last_loss_sum(self) -> float:
        torch = _torch()
        torch.cuda.synchronize(self.device)
        return float(self._loss.item())

    def infer(self, x, stream=None):
        """Normalised outputs [n, 128] FP32 for normalised BF16 inputs x [n, 320]."""
        torch = _torch()
        n = int(x.shape[0])
        need = int(self.lib.wx_mlp_infer_work_bytes(n))
        if self._infer_work is None or self._infer_work.numel() < need:
            self._infer_work = torch.zeros(need, dtype=torch.uint8, device=self.device)
        y = torch.zeros(n, MLP_NOUTP, dtype=torch.float32, device=self.device)
        _check(self.lib.wx_mlp_infer(self.blob.data_ptr(), self._infer_work.data_ptr(), x.data_ptr(), n,
                                     y.data_ptr(), _stream_ptr(stream)), "wx_mlp_infer")
        return y


class ReducedApp:
    """The paper's reduced weather application on the GPU (FP64, device buffers owned here).

    ``e`` is the field [nz][ny+2][nx+2] (i fastest, one-cell ring), ``surf``
    and ``pbl`` the [ny+2][nx+2] surface and boundary-layer values; ``run``
    advances it with the printed physics-then-diffusion step and pointer swap.
    ``order="kij"`` keeps the field on the device in KIJ order ([ny+2][nx+2][nz])
    and runs wx_rw_run_kij; upload and download reorder it.
    """

    def __init__(self, e, surf, pbl, nu: float, device: str = "cuda:0", order: str = "ijk",
                 block=None):
        torch = _torch()
        if order not in ("ijk", "kij"):
            raise WxError(f"unknown storage order {order!r}")
        if block is not None and order != "ijk":
            raise WxError("the thread-block shape applies to the IJK order")
        self.lib = load_library()
        self.order = order
        self.block = None if block is None else (int(block[0]), int(block[1]))
        self.nz, nyp, nxp = e.shape
        self.ny, self.nx = nyp - 2, nxp - 2
        self.nu = float(nu)
        dev = torch.device(device)
        host = np.ascontiguousarray(e if order == "ijk" else np.transpose(e, (1, 2, 0)), dtype=np.float64)
        self.buf = [torch.as_tensor(host).to(dev), torch.empty(host.shape, dtype=torch.float64, device=dev)]
        self.surf = torch.as_tensor(np.ascontiguousarray(surf, dtype=np.float64)).to(dev)
        self.pbl = torch.as_tensor(np.ascontiguousarray(pbl, dtype=np.float64)).to(dev)
        self.cur = 0

    def run(self, nsteps: int, stream=None) -> None:
        which = ctypes.c_int(0)
        args = (self.buf[self.cur].data_ptr(), self.buf[1 - self.cur].data_ptr(),
                self.surf.data_ptr(), self.pbl.data_ptr(), self.nx, self.ny, self.nz,
                self.nu, int(nsteps), ctypes.byref(which))
        if self.block is not None:
            _check(self.lib.wx_rw_run_block(*args, self.block[0], self.block[1], _stream_ptr(stream)),
                   "wx_rw_run_block")
        else:
            fn = self.lib.wx_rw_run if self.order == "ijk" else self.lib.wx_rw_run_kij
            _check(fn(*args, _stream_ptr(stream)), "wx_rw_run")
        self.cur = self.cur if which.value == 0 else 1 - self.cur

    def step_into(self, stream=None) -> None:
        """One step through wx_rw_step (the single-step entry point, IJK order)."""
        if self.order != "ijk":
            raise WxError("wx_rw_step takes the IJK order")
        _check(self.lib.wx_rw_step(self.buf[self.cur].data_ptr(), self.buf[1 - self.cur].data_ptr(),
                                   self.surf.data_ptr(), self.pbl.data_ptr(), self.nx, self.ny, self.nz,
                                   self.nu, _stream_ptr(stream)), "wx_rw_step")
        self.cur = 1 - self.cur

    @property
    def field(self):
        return self.buf[self.cur]

    def download(self) -> np.ndarray:
        """The field in the oracle's [nz][ny+2][nx+2] order."""
        torch = _torch()
        torch.cuda.synchronize(self.buf[0].device)
        f = self.field.cpu().numpy()
        return f if self.order == "ijk" else np.ascontiguousarray(np.transpose(f, (2, 0, 1)))



class Hevi:
    """Fast-mode (HEVI) fields on the GPU, advanced by wx_hevi_run (buffers owned here).

    ``f`` is an ``inputs.FastFields`` (u, v, pi of shape (nz, ny, nx); w, b of
    shape (nz + 1, ny, nx)); ``run`` advances it by short steps of ``tau``.
    """

    CELL = ("u", "v", "pi")
    FACE = ("w", "b")

    def __init__(self, f, tau: float, dtype: str = "f64", c_sound: float = 340.0, n_bv: float = 0.01,
                 device: str = "cuda:0", kernel: int = 2):
        torch = _torch()
        self.lib = load_library()
        nz, ny, nx = f.pi.shape
        self.nx, self.ny, self.nz = nx, ny, nz
        self.g = _HeviGrid()
        _check(self.lib.wx_hevi_grid_init(ctypes.byref(self.g), nx, ny, nz, WX_F32 if dtype == "f32" else WX_F64,
                                          float(f.dx), float(tau), float(c_sound), float(n_bv)),
               "wx_hevi_grid_init")
        self.g.kernel = int(kernel)
        self.dz = np.ascontiguousarray(f.dz, dtype=np.float64)
        self.sj = int(self.g.stride_j)
        self.tdt = torch.float32 if dtype == "f32" else torch.float64
        self.np_dtype = np.float32 if dtype == "f32" else np.float64
        self.device = torch.device(device)
        self.t = {}
        for name in self.CELL:
            self.t[name] = torch.zeros(int(self.g.cell_elems), dtype=self.tdt, device=self.device)
        for name in self.FACE:
            self.t[name] = torch.zeros(int(self.g.face_elems), dtype=self.tdt, device=self.device)
        self.ws = torch.zeros(int(self.lib.wx_hevi_workspace_bytes(ctypes.byref(self.g))), dtype=torch.uint8,
                              device=self.device)
        for name in self.CELL + self.FACE:
            self.interior(name).copy_(torch.from_numpy(np.ascontiguousarray(getattr(f, name),
                                                                            dtype=self.np_dtype)))

    def interior(self, name: str):
        planes = self.nz + 1 if name in self.FACE else self.nz
        return self.t[name].view(planes, self.ny + 2 * HALO, self.sj)[:, HALO:HALO + self.ny, HALO:HALO + self.nx]

    def run(self, nsteps: int, stream=None) -> None:
        t = self.t
        _check(self.lib.wx_hevi_run(ctypes.byref(self.g), self.dz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    t["u"].data_ptr(), t["v"].data_ptr(), t["w"].data_ptr(), t["b"].data_ptr(),
                                    t["pi"].data_ptr(), self.ws.data_ptr(), int(nsteps), _stream_ptr(stream)),
               "wx_hevi_run")

    def download(self) -> Dict[str, np.ndarray]:
        torch = _torch()
        torch.cuda.synchronize(self.device)
        return {name: self.interior(name).cpu().numpy().astype(np.float64) for name in self.CELL + self.FACE}

    def download_raw(self, name: str) -> np.ndarray:
        torch = _torch()
        torch.cuda.synchronize(self.device)
        planes = self.nz + 1 if name in self.FACE else self.nz
        return self.t[name].view(planes, self.ny + 2 * HALO, self.sj).cpu().numpy()
