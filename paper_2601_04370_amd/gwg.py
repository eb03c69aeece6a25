"""ctypes binding of libgwg.so (include/gwg.h) with PyTorch device tensors.

Argument marshalling only: every step of the trace, thin-film solve, adjoint
and loss runs in the HIP library.  There is no CPU fallback: if the library
or a gfx950 device is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgwg.so")

GWG_OK, GWG_E_INVAL, GWG_E_NOMEM, GWG_E_HIP, GWG_E_STATE, GWG_E_OVERFLOW, GWG_E_NODEVICE = range(7)
FP64, FP32_MIXED, FP32 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "mixed": FP32_MIXED, "fp32": FP32}
CAT_NAMES = ["eyebox", "miss", "leak", "end", "trunc", "lost", "face_r", "unused"]

_dp = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)
_i32p = C.POINTER(C.c_int32)


class GwgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gwg error {code}: {msg}")
        self.code = code


class Materials(C.Structure):
    _fields_ = [("n_lambda", C.c_int32), ("n_mat", C.c_int32), ("lambda_nm", _dp),
                ("n_re", _dp), ("n_im", _dp)]


class Stack(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("thk_nm", C.c_void_p), ("mat", _u8p),
                ("mat_in", C.c_int32), ("mat_out", C.c_int32)]


class Slab(C.Structure):
    _fields_ = [("T_mm", C.c_double), ("L_mm", C.c_double), ("eye_relief_mm", C.c_double),
                ("mat_glass", C.c_int32), ("mat_air", C.c_int32),
                ("pupil_x0_mm", C.c_double), ("pupil_w_mm", C.c_double), ("pupil_h_mm", C.c_double),
                ("eye_x0_mm", C.c_double), ("eye_y0_mm", C.c_double), ("eye_w_mm", C.c_double),
                ("eye_h_mm", C.c_double), ("bins_x", C.c_int32), ("bins_y", C.c_int32),
                ("n_eye_pupils", C.c_int32), ("eye_pupil_radius_mm", C.c_double), ("eye_pupil_xy_mm", _dp)]


class Prma(C.Structure):
    _fields_ = [("n_mirrors", C.c_int32), ("tilt_deg", C.c_double), ("pitch_mm", C.c_double),
                ("center_x_mm", C.c_double), ("omega", _dp)]


class Stacks(C.Structure):
    _fields_ = [("n_designs", C.c_int32), ("n_mirrors", C.c_int32), ("max_layers", C.c_int32),
                ("thk_nm", C.c_void_p), ("mat", _u8p), ("n_layers", _i32p)]


class Rays(C.Structure):
    _fields_ = [("n_lambda_sel", C.c_int32), ("lambda_sel", _i32p), ("fov_mode", C.c_int32),
                ("n_fov", C.c_int32), ("fov_deg", _dp), ("rays_per_point", C.c_int64),
                ("max_events", C.c_int32), ("first_design", C.c_int32)]


class Eyebox(C.Structure):
    _fields_ = [("q_bins", C.c_void_p), ("counts", C.c_void_p), ("irradiance", C.c_void_p),
                ("fp_shift", C.c_int32)]


class RayRecord(C.Structure):
    _fields_ = [("bin", C.c_int32), ("category", C.c_int32), ("n_events", C.c_int32),
                ("n_prma", C.c_int32), ("w", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("rays", C.c_int64), ("interactions", C.c_int64), ("prma_hits", C.c_int64),
                ("layer_steps", C.c_int64), ("fp64_hits", C.c_int64), ("saturated", C.c_int64),
                ("adjoint_rays", C.c_int64), ("adjoint_hits", C.c_int64),
                ("adjoint_layer_steps", C.c_int64), ("n_cat", C.c_int64 * 8),
                ("power", C.c_double * 8), ("adjoint_stored_layer_steps", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("n_cat", "power")}
        d["n_cat"] = {CAT_NAMES[k]: self.n_cat[k] for k in range(7)}
        d["power"] = {CAT_NAMES[k]: self.power[k] for k in range(7)}
        return d


class Tuning(C.Structure):
    _fields_ = [("block_threads", C.c_int32), ("rays_per_block", C.c_int64),
                ("bwd_block_threads", C.c_int32), ("bwd_rays_per_block", C.c_int64),
                ("adj_entries_per_ray", C.c_int32), ("memo_keys", C.c_int32), ("table_nodes", C.c_int32),
                ("ck_entries_per_ray", C.c_int32)]


#: every function declared in include/gwg.h
EXPORTS = ["gwg_abi_version", "gwg_create", "gwg_destroy", "gwg_last_error", "gwg_tmm_rt",
           "gwg_trace_forward", "gwg_trace_backward", "gwg_loss", "gwg_set_tuning", "gwg_get_tuning",
           "gwg_set_timing", "gwg_kernel_times", "gwg_set_step_source", "gwg_autotune", "gwg_forward_kept_entries",
           "gwg_omega_gradient", "gwg_source_hash", "gwg_loss_noalloc"]

KERNEL_FORWARD, KERNEL_ADJOINT, TIMING_RING = 0, 1, 64
GWG_FWD_GRAD = 1
GWG_FWD_MEMO = 2
GWG_FWD_TABLE = 4

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgwg.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(path)
    L.gwg_source_hash.restype = C.c_char_p
    built = L.gwg_source_hash().decode()
    if path == LIB_PATH:
        from . import build as _build
        want = _build.source_hash()
        if built != want:
            raise ImportError(f"{path} was built from other sources (library {built}, sources {want}): "
                              "rebuild it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L.gwg_abi_version.restype = C.c_int32
    L.gwg_create.argtypes = [C.POINTER(C.c_void_p), C.c_int32]
    L.gwg_destroy.argtypes = [C.c_void_p]
    L.gwg_last_error.argtypes = [C.c_void_p]
    L.gwg_last_error.restype = C.c_char_p
    L.gwg_tmm_rt.argtypes = [C.c_void_p, C.POINTER(Stack), C.POINTER(Materials), C.c_int64,
                             C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
    L.gwg_trace_forward.argtypes = [C.c_void_p, C.POINTER(Slab), C.POINTER(Prma), C.POINTER(Materials),
                                    C.POINTER(Stacks), C.POINTER(Rays), C.c_uint64, C.c_uint64, C.c_int32,
                                    C.c_uint32, C.POINTER(Eyebox), C.c_void_p, C.c_int64, C.POINTER(Stats), C.c_void_p]
    L.gwg_trace_backward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(Stats),
                                     C.c_void_p]
    L.gwg_loss.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                           C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
    L.gwg_loss_noalloc.argtypes = L.gwg_loss.argtypes
    L.gwg_set_tuning.argtypes = [C.c_void_p, C.POINTER(Tuning)]
    L.gwg_get_tuning.argtypes = [C.c_void_p, C.POINTER(Tuning)]
    L.gwg_set_timing.argtypes = [C.c_void_p, C.c_int32]
    L.gwg_set_step_source.argtypes = [C.c_void_p, C.c_void_p]
    L.gwg_forward_kept_entries.argtypes = [C.c_void_p, C.POINTER(C.c_int32)]
    L.gwg_omega_gradient.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.gwg_autotune.argtypes = [C.c_void_p, C.POINTER(Slab), C.POINTER(Prma), C.POINTER(Materials),
                               C.POINTER(Stacks), C.POINTER(Rays), C.c_uint64, C.c_int32, C.c_uint32,
                               C.c_char_p, C.POINTER(Tuning), C.c_void_p]
    L.gwg_kernel_times.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double)]
    _lib = L
    return L


def source_hash() -> str:
    """Source hash compiled into the loaded library (equal to the sources' own)."""
    return load_library().gwg_source_hash().decode()


def _np_ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _stream(torch, device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


@dataclass
class SceneSpec:
    """Host description of a waveguide scene (everything but the thicknesses).

    Arrays are numpy; they are kept alive by this object while ctypes structs
    point into them.
    """
    lambda_nm: np.ndarray
    n_re: np.ndarray
    n_im: np.ndarray
    T_mm: float
    L_mm: float
    eye_relief_mm: float
    mat_glass: int
    mat_air: int
    pupil: tuple
    eyebox: tuple
    bins: tuple
    n_mirrors: int
    tilt_deg: float
    pitch_mm: float
    center_x_mm: float
    omega: np.ndarray
    n_designs: int
    max_layers: int
    mat: np.ndarray
    n_layers: np.ndarray
    lambda_sel: np.ndarray
    fov_mode: int
    fov_deg: np.ndarray
    rays_per_point: int
    max_events: int
    fp_shift: int = 24
    # eye pupils: centres [P][2] (mm) and radius; None for the eyebox grid
    eye_pupils: Optional[np.ndarray] = None
    eye_pupil_r: float = 0.0
    # the designs are these designs of a larger batch (its random streams)
    first_design: int = 0
    _keep: dict = field(default_factory=dict, repr=False)

    @classmethod
    def from_workload(cls, w, inp: dict, rays_per_point: Optional[int] = None,
                      omega: Optional[np.ndarray] = None) -> "SceneSpec":
        """From a workload object (attributes as in the ``inputs`` module) and its tables."""
        glass, air = 1, 0
        return cls(
            lambda_nm=np.ascontiguousarray(inp["lambda_nm"], np.float64),
            n_re=np.ascontiguousarray(inp["n_re"], np.float64),
            n_im=np.ascontiguousarray(inp["n_im"], np.float64),
            T_mm=w.T_mm, L_mm=w.L_mm, eye_relief_mm=w.eye_relief_mm, mat_glass=glass, mat_air=air,
            pupil=tuple(inp["pupil"]), eyebox=tuple(inp["eyebox"]), bins=tuple(w.bins),
            n_mirrors=w.n_mirrors, tilt_deg=w.tilt_deg, pitch_mm=w.pitch_mm, center_x_mm=w.center_x_mm,
            omega=np.ascontiguousarray(inp["omega"] if omega is None else omega, np.float64),
            n_designs=inp["thk"].shape[0], max_layers=inp["thk"].shape[2],
            mat=np.ascontiguousarray(inp["mat"], np.uint8),
            n_layers=np.ascontiguousarray(inp["n_layers"], np.int32),
            lambda_sel=np.ascontiguousarray(inp["lambda_sel"], np.int32),
            fov_mode=w.fov_mode, fov_deg=np.ascontiguousarray(inp["fov"], np.float64),
            rays_per_point=int(w.rays_per_point if rays_per_point is None else rays_per_point),
            max_events=w.max_events, fp_shift=w.fp_shift,
            eye_pupils=(np.ascontiguousarray(inp["eye_pupils"], np.float64)
                        if inp.get("eye_pupils") is not None and len(inp["eye_pupils"]) else None),
            eye_pupil_r=float(inp.get("eye_pupil_r", 0.0)))

    @property
    def n_fov(self) -> int:
        return 1 if self.fov_mode == 1 else self.fov_deg.shape[0]

    @property
    def shape(self):
        return (self.n_designs, len(self.lambda_sel), self.n_fov, self.bins[1], self.bins[0])

    @property
    def thk_shape(self):
        return (self.n_designs, self.n_mirrors, self.max_layers)

    @property
    def n_rays(self) -> int:
        return self.n_designs * len(self.lambda_sel) * self.n_fov * self.rays_per_point

    def structs(self):
        k = self._keep
        m = Materials(self.n_re.shape[0], self.n_re.shape[1],
                      _np_ptr(self.lambda_nm, _dp), _np_ptr(self.n_re, _dp), _np_ptr(self.n_im, _dp))
        s = Slab(self.T_mm, self.L_mm, self.eye_relief_mm, self.mat_glass, self.mat_air,
                 self.pupil[0], self.pupil[1], self.pupil[2],
                 self.eyebox[0], self.eyebox[1], self.eyebox[2], self.eyebox[3], self.bins[0], self.bins[1])
        if self.eye_pupils is not None:
            s.n_eye_pupils = self.eye_pupils.shape[0]
            s.eye_pupil_radius_mm = self.eye_pupil_r
            s.eye_pupil_xy_mm = _np_ptr(self.eye_pupils, _dp)
        p = Prma(self.n_mirrors, self.tilt_deg, self.pitch_mm, self.center_x_mm, _np_ptr(self.omega, _dp))
        st = Stacks(self.n_designs, self.n_mirrors, self.max_layers, None, _np_ptr(self.mat, _u8p),
                    _np_ptr(self.n_layers, _i32p))
        r = Rays(len(self.lambda_sel), _np_ptr(self.lambda_sel, _i32p), self.fov_mode, self.n_fov,
                 _np_ptr(self.fov_deg, _dp), self.rays_per_point, self.max_events, self.first_design)
        k["structs"] = (m, s, p, st, r)
        return m, s, p, st, r


class Context:
    """One library context on one GPU (owns scratch memory and scene tables)."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise GwgError(GWG_E_NODEVICE, "no GPU visible to torch")
        self.device = device
        self.forward_id = 0
        h = C.c_void_p()
        rc = self.lib.gwg_create(C.byref(h), device)
        if rc != GWG_OK:
            raise GwgError(rc, self.lib.gwg_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.gwg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != GWG_OK:
            raise GwgError(rc, self.lib.gwg_last_error(self.h).decode())

    def set_tuning(self, block_threads=0, rays_per_block=0, bwd_block_threads=0, bwd_rays_per_block=0,
                   adj_entries_per_ray=0, memo_keys=0, table_nodes=0, ck_entries_per_ray=0):
        t = Tuning(block_threads, rays_per_block, bwd_block_threads, bwd_rays_per_block, adj_entries_per_ray,
                   memo_keys, table_nodes, ck_entries_per_ray)
        self._check(self.lib.gwg_set_tuning(self.h, C.byref(t)))

    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(self.lib.gwg_get_tuning(self.h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def omega_gradient(self, W, counts, scene: "SceneSpec"):
        """d/domega [M] of sum W * counts / N in the scalar-reflectance model,
        score-function estimate on the paths of the last forward (whose
        counts tensor is passed; its thk must still be alive)."""
        torch = self.torch
        dev = torch.device("cuda", self.device)
        W = W.to(dev, torch.float64).contiguous()
        counts = counts.to(dev).contiguous()
        assert W.numel() == int(np.prod(scene.shape)) and counts.numel() == W.numel() and counts.element_size() == 4
        g = torch.empty(scene.n_mirrors, dtype=torch.float64, device=dev)
        self._check(self.lib.gwg_omega_gradient(self.h, W.data_ptr(), counts.data_ptr(), g.data_ptr(),
                                                _stream(torch, dev)))
        return g

    def forward_kept_entries(self) -> bool:
        """True if the last forward stored adjoint entries for the backward."""
        v = C.c_int32(0)
        self._check(self.lib.gwg_forward_kept_entries(self.h, C.byref(v)))
        return bool(v.value)

    def set_step_source(self, d_step=None):
        """Device int32/uint32 tensor [1] whose value is added to `step` by the
        trace kernels (for captured graphs), or None."""
        if d_step is not None:
            assert d_step.is_cuda and d_step.numel() >= 1 and d_step.element_size() == 4
        self._step_src = d_step
        self._check(self.lib.gwg_set_step_source(self.h, d_step.data_ptr() if d_step is not None else None))

    def autotune(self, scene: "SceneSpec", thk, seed: int, precision: int = FP64, grad: bool = False,
                 cache_path: Optional[str] = None) -> dict:
        """Time launch configurations for this scene; the fastest becomes the tuning."""
        torch = self.torch
        dev = torch.device("cuda", self.device)
        assert tuple(thk.shape) == scene.thk_shape and thk.dtype == torch.float64 and thk.is_contiguous()
        m, s, p, st, r = scene.structs()
        st.thk_nm = thk.data_ptr()
        t = Tuning()
        self._check(self.lib.gwg_autotune(self.h, C.byref(s), C.byref(p), C.byref(m), C.byref(st), C.byref(r),
                                          seed & 0xFFFFFFFFFFFFFFFF, precision, GWG_FWD_GRAD if grad else 0,
                                          cache_path.encode() if cache_path else None, C.byref(t),
                                          _stream(torch, dev)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def set_timing(self, enable: bool = True):
        """Record HIP events around each forward / adjoint trace kernel launch."""
        self._check(self.lib.gwg_set_timing(self.h, 1 if enable else 0))

    def kernel_times(self, kernel: int, n: int):
        """Durations (ms) of the last n launches of KERNEL_FORWARD or KERNEL_ADJOINT."""
        out = (C.c_double * max(n, 1))()
        self._check(self.lib.gwg_kernel_times(self.h, kernel, n, out))
        return [out[i] for i in range(n)]

    # ------------------------------------------------------------ thin film
    def tmm_rt(self, thk, mat: np.ndarray, mat_in: int, mat_out: int, lambda_nm, n_re, n_im,
               lambda_idx, theta, precision: int = FP64):
        """Coefficients [n_q, 4] complex128 (r_s, r_p, t_s, t_p) on the GPU."""
        torch = self.torch
        dev = torch.device("cuda", self.device)
        thk = thk.to(dev, torch.float64).contiguous()
        mat = np.ascontiguousarray(mat, np.uint8)
        lam = np.ascontiguousarray(lambda_nm, np.float64)
        nre = np.ascontiguousarray(n_re, np.float64)
        nim = np.ascontiguousarray(n_im, np.float64)
        li = lambda_idx.to(dev, torch.int32).contiguous()
        th = theta.to(dev, torch.float64).contiguous()
        n = th.numel()
        out = torch.empty((n, 8), dtype=torch.float64, device=dev)
        st = Stack(len(mat), thk.data_ptr() if len(mat) else None, _np_ptr(mat, _u8p), mat_in, mat_out)
        mt = Materials(nre.shape[0], nre.shape[1], _np_ptr(lam, _dp), _np_ptr(nre, _dp), _np_ptr(nim, _dp))
        self._check(self.lib.gwg_tmm_rt(self.h, C.byref(st), C.byref(mt), n, li.data_ptr(), th.data_ptr(),
                                        precision, out.data_ptr(), _stream(torch, dev)))
        return torch.view_as_complex(out.view(n, 4, 2))

    # ---------------------------------------------------------------- trace
    def trace_forward(self, scene: SceneSpec, thk, seed: int, step: int = 0, precision: int = FP64,
                      record_stride: int = 0, stats: bool = False, want_irradiance: bool = True,
                      grad: bool = False, memo: bool = False, table: bool = False):
        """Returns (q_bins u64-as-int64, counts int32, irradiance f64 or None,
        records or None, stats dict or None); tensors on the context's GPU.
        grad=True prepares the adjoint entries for a following trace_backward;
        memo=True solves each distinct hit key of a work item once (results
        identical to the per-hit solves) and, with grad, makes that backward
        solve one thin-film adjoint per distinct key.  table=True interpolates
        the thin film from the angle table (tuning table_nodes angles)."""
        torch = self.torch
        dev = torch.device("cuda", self.device)
        assert tuple(thk.shape) == scene.thk_shape and thk.dtype == torch.float64 and thk.is_contiguous()
        assert thk.device == dev
        m, s, p, st, r = scene.structs()
        st.thk_nm = thk.data_ptr()
        shape = scene.shape
        q = torch.empty(shape, dtype=torch.int64, device=dev)
        c = torch.empty(shape, dtype=torch.int32, device=dev)
        irr = torch.empty(shape, dtype=torch.float64, device=dev) if want_irradiance else None
        eb = Eyebox(q.data_ptr(), c.data_ptr(), irr.data_ptr() if irr is not None else None, scene.fp_shift)
        rec = None
        if record_stride:
            n_rec = (scene.n_rays + record_stride - 1) // record_stride
            rec = torch.zeros((n_rec, 3), dtype=torch.float64, device=dev)  # 24-byte records
        sts = Stats() if stats else None
        self.forward_id += 1
        rc = self.lib.gwg_trace_forward(self.h, C.byref(s), C.byref(p), C.byref(m), C.byref(st), C.byref(r),
                                        seed & 0xFFFFFFFFFFFFFFFF, step, precision,
                                        (GWG_FWD_GRAD if grad else 0) | (GWG_FWD_MEMO if memo else 0)
                                        | (GWG_FWD_TABLE if table else 0), C.byref(eb),
                                        rec.data_ptr() if rec is not None else None, int(record_stride or 1),
                                        C.byref(sts) if sts is not None else None, _stream(torch, dev))
        if rc == GWG_E_OVERFLOW:
            pass  # saturation is reported in stats; outputs are complete
        else:
            self._check(rc)
        return q, c, irr, rec, (sts.as_dict() if sts is not None else None)

    def trace_backward(self, dLdI, scene: SceneSpec, sample_stride: int = 1, stats: bool = False):
        """dL/dthk [D][M][Lmax] for dL/dI of the last forward (and a stats dict if asked)."""
        torch = self.torch
        dev = torch.device("cuda", self.device)
        dLdI = dLdI.to(dev, torch.float64).contiguous()
        if dLdI.numel() != int(np.prod(scene.shape)):
            raise GwgError(GWG_E_INVAL, f"dL/dI has {dLdI.numel()} elements, the eyebox has {int(np.prod(scene.shape))}")
        grad = torch.empty(scene.thk_shape, dtype=torch.float64, device=dev)
        sts = Stats() if stats else None
        self._check(self.lib.gwg_trace_backward(self.h, dLdI.data_ptr(), grad.data_ptr(), int(sample_stride),
                                                C.byref(sts) if sts is not None else None, _stream(torch, dev)))
        if stats:
            return grad, sts.as_dict()
        return grad

    def loss(self, irr, kind: int = 0, w_f: float = 1.0, w_e: float = 1.0, want_grad: bool = True):
        torch = self.torch
        dev = torch.device("cuda", self.device)
        irr = irr.to(dev, torch.float64).contiguous()
        D, nl, F = irr.shape[:3]
        B = int(np.prod(irr.shape[3:]))
        out = torch.empty(1, dtype=torch.float64, device=dev)
        g = torch.empty_like(irr) if want_grad else None
        self._check(self.lib.gwg_loss(self.h, irr.data_ptr(), D, nl, F, B, kind, w_f, w_e, out.data_ptr(),
                                      g.data_ptr() if g is not None else None, _stream(torch, dev)))
        return out, g


def records_view(rec_tensor):
    """Decode a records tensor (n, 3 f64 words) into numpy fields."""
    raw = rec_tensor.cpu().numpy().view(np.uint8).reshape(-1, 24)
    ints = raw[:, :16].copy().view(np.int32).reshape(-1, 4)
    w = raw[:, 16:].copy().view(np.float64).reshape(-1)
    return dict(bin=ints[:, 0], category=ints[:, 1], n_events=ints[:, 2], n_prma=ints[:, 3], w=w)


def make_trace_function():
    """torch.autograd.Function: irradiance = trace(thk); grad via the adjoint kernel."""
    import torch

    class GWGTrace(torch.autograd.Function):
        @staticmethod
        def forward(fctx, thk, context: Context, scene: SceneSpec, seed: int, step: int, precision: int):
            # the library keeps this pointer and reads the thicknesses again in
            # the backward, so the contiguous copy must outlive this call
            thk_c = thk.detach().contiguous()
            q, c, irr, _, _ = context.trace_forward(scene, thk_c, seed, step, precision,
                                                    grad=thk.requires_grad)
            fctx.thk_c = thk_c
            fctx.context = context
            fctx.scene = scene
            fctx.forward_id = context.forward_id
            fctx.save_for_backward(thk)
            return irr

        @staticmethod
        def backward(fctx, grad_irr):
            (thk,) = fctx.saved_tensors
            if fctx.context.forward_id != fctx.forward_id:
                raise GwgError(GWG_E_STATE, "another forward ran on this context before this backward")
            g = fctx.context.trace_backward(grad_irr, fctx.scene)
            fctx.thk_c = None
            return g, None, None, None, None, None

    return GWGTrace
