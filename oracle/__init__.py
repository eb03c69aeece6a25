"""ctypes wrapper of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()``
and by ``bench.py``'s CPU-baseline leg, never by the product package.  The
oracle shares no code with the HIP path; both consume the seeded tables of
the ``inputs`` module.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

ORC_EYEBOX, ORC_MISS, ORC_LEAK, ORC_END, ORC_TRUNC, ORC_LOST, ORC_FACE_R = range(7)
ORC_NCAT = 8

_dp = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u64p = C.POINTER(C.c_uint64)
_u32p = C.POINTER(C.c_uint32)


class Scene(C.Structure):
    _fields_ = [
        ("n_lambda", C.c_int32), ("n_mat", C.c_int32),
        ("lambda_nm", _dp), ("n_re", _dp), ("n_im", _dp),
        ("T", C.c_double), ("Lx", C.c_double), ("eye_relief", C.c_double),
        ("mat_glass", C.c_int32), ("mat_air", C.c_int32),
        ("pupil_x0", C.c_double), ("pupil_w", C.c_double), ("pupil_h", C.c_double),
        ("eye_x0", C.c_double), ("eye_y0", C.c_double), ("eye_w", C.c_double), ("eye_h", C.c_double),
        ("bins_x", C.c_int32), ("bins_y", C.c_int32),
        ("n_mirrors", C.c_int32),
        ("tilt_deg", C.c_double), ("pitch", C.c_double), ("center_x", C.c_double),
        ("omega", _dp),
        ("n_designs", C.c_int32), ("max_layers", C.c_int32),
        ("thk", _dp), ("mat", _u8p), ("n_layers", _i32p),
        ("n_lsel", C.c_int32), ("lambda_sel", _i32p),
        ("fov_mode", C.c_int32), ("n_fov", C.c_int32), ("fov_deg", _dp),
        ("rays_per_point", C.c_int64), ("max_events", C.c_int32), ("fp_shift", C.c_int32),
        ("seed", C.c_uint64), ("step", C.c_uint64),
        ("table_nodes", C.c_int32),
        ("n_eye_pupils", C.c_int32), ("eye_pupil_r", C.c_double), ("eye_pupil_xy", _dp),
        ("first_design", C.c_int32),
    ]


class RayRecord(C.Structure):
    _fields_ = [
        ("ray_id", C.c_int64), ("bin", C.c_int32), ("category", C.c_int32),
        ("n_events", C.c_int32), ("n_prma", C.c_int32), ("w", C.c_double),
        ("exit_dir", C.c_double * 3), ("exit_pos", C.c_double * 3),
    ]


class Stats(C.Structure):
    _fields_ = [("counters", C.c_int64 * 16), ("power", C.c_double * ORC_NCAT)]


def lib():
    """Load (building if needed) liboracle.so."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.path.join(_HERE, "liboracle.so")
    srcs = [os.path.join(_HERE, s) for s in _build.SOURCES + ["oracle.h"]]
    if not os.path.exists(path) or any(os.path.getmtime(s) > os.path.getmtime(path) for s in srcs):
        _build.build()
    L = C.CDLL(path)
    L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.orc_tmm_rt.argtypes = [C.c_int, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                             C.c_double, C.c_double, _dp]
    L.orc_tmm_dthk.argtypes = L.orc_tmm_rt.argtypes
    L.orc_tmm_rt_batch.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, C.c_int64, _i32p, _dp, _dp]
    L.orc_trace_forward.argtypes = [C.POINTER(Scene), _u64p, _u32p, _dp, C.POINTER(Stats)]
    L.orc_trace_rays.argtypes = [C.POINTER(Scene), C.c_int64, _i64p, C.POINTER(RayRecord)]
    L.orc_ray_events.argtypes = [C.POINTER(Scene), C.c_int64, C.c_int, _dp]
    L.orc_trace_backward.argtypes = [C.POINTER(Scene), _dp, C.c_int64, _dp]
    L.orc_trace_forward_sampled.argtypes = [C.POINTER(Scene), C.c_int64, _dp]
    L.orc_split_bruteforce.argtypes = [C.POINTER(Scene), C.c_int32, C.c_int32, C.c_int32,
                                       C.c_int64, C.c_int64, _dp, _i64p]
    L.orc_trace_forced.argtypes = [C.POINTER(Scene), C.c_int64, C.c_uint64, C.c_int,
                                   _dp, _dp, C.POINTER(C.c_int)]
    L.orc_loss.argtypes = [_dp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                           C.c_double, C.c_double, _dp]
    L.orc_loss.restype = C.c_double
    L.orc_table_weights.argtypes = [C.c_double, C.c_int, _i32p, _dp]
    L.orc_event_probe.argtypes = [C.POINTER(Scene), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  _dp, _dp, _dp, _dp]
    _lib = L
    return L


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


# ------------------------------------------------------------------ Philox
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(out, _u32p))
    return out


# --------------------------------------------------------------- thin film
def tmm_rt(thk, n_layers_complex, n_in: float, n_out: complex, lambda_nm: float,
           theta: float = None, kappa: float = None) -> np.ndarray:
    """r_s, r_p, t_s, t_p (complex) of one stack (Eq. 3 amplitude convention)."""
    thk = np.ascontiguousarray(thk, dtype=np.float64)
    N = np.asarray(n_layers_complex, dtype=np.complex128)
    nre = np.ascontiguousarray(N.real)
    nim = np.ascontiguousarray(N.imag)
    if kappa is None:
        kappa = n_in * np.sin(theta)
    out = np.zeros(8)
    n_out = complex(n_out)
    lib().orc_tmm_rt(len(thk), _ptr(thk, _dp), _ptr(nre, _dp), _ptr(nim, _dp), float(n_in),
                     n_out.real, n_out.imag, float(lambda_nm), float(kappa), _ptr(out, _dp))
    return out[0::2] + 1j * out[1::2]


def tmm_rt_batch(thk, N_by_lambda, n_in, n_out, lambda_nm, lambda_idx, theta, threads: int = 1) -> np.ndarray:
    """[n_q, 4] complex coefficients of one stack for queries (lambda_idx[q],
    theta[q]); N_by_lambda [n_lambda][L] complex layer indices, n_in / n_out /
    lambda_nm per wavelength.  `threads` host threads split the queries (the
    C loop releases the interpreter lock)."""
    import threading
    thk = np.ascontiguousarray(thk, dtype=np.float64)
    N = np.asarray(N_by_lambda, dtype=np.complex128)
    nre, nim = np.ascontiguousarray(N.real), np.ascontiguousarray(N.imag)
    nin = np.ascontiguousarray(n_in, dtype=np.float64)
    no = np.asarray(n_out, dtype=np.complex128)
    nout = np.ascontiguousarray(np.stack([no.real, no.imag], -1).reshape(-1))
    lam = np.ascontiguousarray(lambda_nm, dtype=np.float64)
    li = np.ascontiguousarray(lambda_idx, dtype=np.int32)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    n = len(th)
    out = np.zeros((n, 8))
    L = lib()
    bounds = np.linspace(0, n, max(1, threads) + 1).astype(np.int64)

    def run(a, b):
        if b > a:
            L.orc_tmm_rt_batch(len(thk), _ptr(thk, _dp), _ptr(nre, _dp), _ptr(nim, _dp), _ptr(nin, _dp),
                               _ptr(nout, _dp), _ptr(lam, _dp), int(b - a),
                               li[a:b].ctypes.data_as(_i32p), th[a:b].ctypes.data_as(_dp),
                               out[a:b].ctypes.data_as(_dp))
    ts = [threading.Thread(target=run, args=(int(bounds[k]), int(bounds[k + 1]))) for k in range(len(bounds) - 1)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    return out[:, 0::2] + 1j * out[:, 1::2]


def tmm_dthk(thk, n_layers_complex, n_in: float, n_out: complex, lambda_nm: float,
             theta: float = None, kappa: float = None) -> np.ndarray:
    """[L][4] complex dc/dthk for c = r_s, r_p, t_s, t_p (per nm)."""
    thk = np.ascontiguousarray(thk, dtype=np.float64)
    N = np.asarray(n_layers_complex, dtype=np.complex128)
    nre = np.ascontiguousarray(N.real)
    nim = np.ascontiguousarray(N.imag)
    if kappa is None:
        kappa = n_in * np.sin(theta)
    L = len(thk)
    out = np.zeros(max(L, 1) * 16)
    n_out = complex(n_out)
    lib().orc_tmm_dthk(L, _ptr(thk, _dp), _ptr(nre, _dp), _ptr(nim, _dp), float(n_in),
                       n_out.real, n_out.imag, float(lambda_nm), float(kappa), _ptr(out, _dp))
    o = out[: L * 16].reshape(L, 4, 4)
    return o[:, :, 0] + 1j * o[:, :, 1]


def table_weights(theta: float, n: int):
    """Node indices and weights of the n-angle table at incidence angle theta."""
    idx = np.zeros(4, dtype=np.int32)
    w = np.zeros(4)
    lib().orc_table_weights(C.c_double(theta), C.c_int(n), _ptr(idx, _i32p), _ptr(w, _dp))
    return idx, w


# ------------------------------------------------------------------- scene
class OracleScene:
    """Holds the numpy arrays referenced by a Scene struct."""

    def __init__(self, w, inp: dict, seed: Optional[int] = None, step: int = 0,
                 thk: Optional[np.ndarray] = None, rays_per_point: Optional[int] = None,
                 omega: Optional[np.ndarray] = None, table_nodes: int = 0, first_design: int = 0):
        from inputs import MAT_AIR, MAT_GLASS
        self.w = w
        self.arrays = {}

        def keep(name, a, dtype):
            a = np.ascontiguousarray(a, dtype=dtype)
            self.arrays[name] = a
            return a

        lam = keep("lambda_nm", inp["lambda_nm"], np.float64)
        nre = keep("n_re", inp["n_re"], np.float64)
        nim = keep("n_im", inp["n_im"], np.float64)
        om = keep("omega", inp["omega"] if omega is None else omega, np.float64)
        th = keep("thk", inp["thk"] if thk is None else thk, np.float64)
        mt = keep("mat", inp["mat"], np.uint8)
        nl = keep("n_layers", inp["n_layers"], np.int32)
        ls = keep("lambda_sel", inp["lambda_sel"], np.int32)
        fov = keep("fov", inp["fov"], np.float64)
        px0, pw, ph = inp["pupil"]
        ex0, ey0, ew, eh = inp["eyebox"]
        s = Scene()
        s.n_lambda, s.n_mat = nre.shape
        s.lambda_nm, s.n_re, s.n_im = _ptr(lam, _dp), _ptr(nre, _dp), _ptr(nim, _dp)
        s.T, s.Lx, s.eye_relief = w.T_mm, w.L_mm, w.eye_relief_mm
        s.mat_glass, s.mat_air = MAT_GLASS, MAT_AIR
        s.pupil_x0, s.pupil_w, s.pupil_h = px0, pw, ph
        s.eye_x0, s.eye_y0, s.eye_w, s.eye_h = ex0, ey0, ew, eh
        s.bins_x, s.bins_y = w.bins
        s.n_mirrors = w.n_mirrors
        s.tilt_deg, s.pitch, s.center_x = w.tilt_deg, w.pitch_mm, w.center_x_mm
        s.omega = _ptr(om, _dp)
        s.n_designs, s.max_layers = th.shape[0], th.shape[2]
        s.thk, s.mat, s.n_layers = _ptr(th, _dp), _ptr(mt, _u8p), _ptr(nl, _i32p)
        s.n_lsel, s.lambda_sel = len(ls), _ptr(ls, _i32p)
        s.fov_mode = w.fov_mode
        s.n_fov = 1 if w.fov_mode == 1 else fov.shape[0]
        s.fov_deg = _ptr(fov, _dp)
        s.rays_per_point = w.rays_per_point if rays_per_point is None else rays_per_point
        s.max_events, s.fp_shift = w.max_events, w.fp_shift
        s.seed = w.seed if seed is None else seed
        s.step = step
        s.table_nodes = table_nodes
        s.first_design = first_design
        ep = inp.get("eye_pupils")
        if ep is not None and len(ep):
            xy = keep("eye_pupils", ep, np.float64)
            s.n_eye_pupils = xy.shape[0]
            s.eye_pupil_r = float(inp["eye_pupil_r"])
            s.eye_pupil_xy = _ptr(xy, _dp)
            assert (s.bins_x, s.bins_y) == (xy.shape[0], 1)
        self.s = s

    @property
    def shape(self):
        s = self.s
        F = 1 if s.fov_mode == 1 else s.n_fov
        return (s.n_designs, s.n_lsel, F, s.bins_y, s.bins_x)

    def forward(self):
        n = int(np.prod(self.shape))
        q = np.zeros(n, dtype=np.uint64)
        c = np.zeros(n, dtype=np.uint32)
        ws = np.zeros(n, dtype=np.float64)
        st = Stats()
        rc = lib().orc_trace_forward(C.byref(self.s), _ptr(q, _u64p), _ptr(c, _u32p), _ptr(ws, _dp),
                                     C.byref(st))
        assert rc == 0
        sh = self.shape
        return q.reshape(sh), c.reshape(sh), ws.reshape(sh), st

    def irradiance(self):
        q, c, ws, st = self.forward()
        return q.astype(np.float64) * 2.0 ** (-self.s.fp_shift) / self.s.rays_per_point

    def trace_rays(self, ray_ids):
        ids = np.ascontiguousarray(ray_ids, dtype=np.int64)
        rec = (RayRecord * len(ids))()
        rc = lib().orc_trace_rays(C.byref(self.s), len(ids), _ptr(ids, _i64p), rec)
        assert rc == 0
        return rec

    def events(self, ray_id, cap=64):
        ev = np.zeros(cap * 10)
        n = lib().orc_ray_events(C.byref(self.s), int(ray_id), cap, _ptr(ev, _dp))
        return ev.reshape(cap, 10)[:n]

    def backward(self, dL_dI, stride: int = 1):
        g = np.zeros(self.arrays["thk"].shape)
        d = np.ascontiguousarray(dL_dI, dtype=np.float64)
        assert d.size == int(np.prod(self.shape))
        rc = lib().orc_trace_backward(C.byref(self.s), _ptr(d, _dp), int(stride), _ptr(g, _dp))
        assert rc == 0
        return g

    def forward_sampled(self, stride: int = 1):
        irr = np.zeros(int(np.prod(self.shape)))
        rc = lib().orc_trace_forward_sampled(C.byref(self.s), int(stride), _ptr(irr, _dp))
        assert rc == 0
        return irr.reshape(self.shape)

    def split(self, d, li, f, n_rays, first=0):
        B = self.s.bins_x * self.s.bins_y
        bp = np.zeros(B)
        npaths = C.c_int64(0)
        rc = lib().orc_split_bruteforce(C.byref(self.s), d, li, f, int(first), int(n_rays),
                                        _ptr(bp, _dp), C.byref(npaths))
        assert rc == 0
        return bp, npaths.value

    def event(self, surface, dir_in, E_in, reflect=0, d=0, li=0):
        """One field-changing event in isolation (no Monte Carlo rescaling):
        returns (event type, outgoing direction, outgoing complex field)."""
        di = np.ascontiguousarray(dir_in, dtype=np.float64)
        Ec = np.asarray(E_in, dtype=np.complex128)
        ei = np.ascontiguousarray(np.stack([Ec.real, Ec.imag], -1).reshape(6))
        do = np.zeros(3)
        eo = np.zeros(6)
        ev = lib().orc_event_probe(C.byref(self.s), int(d), int(li), int(surface), int(reflect),
                                   _ptr(di, _dp), _ptr(ei, _dp), _ptr(do, _dp), _ptr(eo, _dp))
        assert ev > 0, ev
        return ev, do, eo[0::2] + 1j * eo[1::2]

    def forced(self, ray_id, bits, n_bits):
        w = C.c_double(0)
        p = C.c_double(0)
        nu = C.c_int(0)
        b = lib().orc_trace_forced(C.byref(self.s), int(ray_id), int(bits), int(n_bits),
                                   C.byref(w), C.byref(p), C.byref(nu))
        return b, w.value, p.value, nu.value


# ------------------------------------------- learned reflection probabilities
# (Methods, learned reflection probabilities) Each coating is idealised as a
# scalar reflectance equal to the mirror's reflection probability omega, so a
# sampled path carries weight one and a ray adds 1 / N to the bin it reaches.
_EV_MIRROR = 5
SURF_TOP, SURF_BOTTOM = 1000, 1001


def p_eff(omega) -> np.ndarray:
    """Sampling probability floor(omega 2^32) / 2^32 of each mirror."""
    t = np.floor(np.asarray(omega, dtype=np.float64) * 4294967296.0)
    return np.clip(t, 0.0, 4294967295.0) / 4294967296.0


def omega_score_gradient(osc: "OracleScene", W: np.ndarray, counts: np.ndarray, ray_ids=None):
    """Score-function estimate of dJ/domega for J = sum_points sum_b W I,
    I = counts / N: per ray, (W_bin - beta) S_m with S_m = sum over its hits
    on mirror m of 1/omega_m (reflected) or -1/(1 - omega_m) (transmitted),
    beta = the point's J; summed per point with 1/N.  Returns (gradient,
    per-ray contributions [n, M]).  ray_ids: all rays by default."""
    s = osc.s
    D, nl, F, by, bx = osc.shape
    B, N, M = by * bx, s.rays_per_point, s.n_mirrors
    p = p_eff(osc.arrays["omega"])
    Wf = np.asarray(W, dtype=np.float64).reshape(-1, B)
    cf = np.asarray(counts, dtype=np.float64).reshape(-1, B)
    ids = np.arange(D * nl * F * N) if ray_ids is None else np.asarray(ray_ids, dtype=np.int64)
    recs = osc.trace_rays(ids)
    contrib = np.zeros((len(ids), M))
    for k, (i, r) in enumerate(zip(ids, recs)):
        pt = int(i) // N
        beta = float(np.dot(Wf[pt], cf[pt])) / N
        S = np.zeros(M)
        for e in osc.events(int(i)):
            if int(e[0]) == _EV_MIRROR:
                m = int(e[1])
                S[m] += 1.0 / p[m] if e[9] != 0.0 else -1.0 / (1.0 - p[m])
        f = (Wf[pt][r.bin] if r.category == ORC_EYEBOX else 0.0) - beta
        contrib[k] = f * S / N
    return contrib.sum(axis=0), contrib


def scalar_expectation(osc: "OracleScene", W: np.ndarray, ray_ids) -> float:
    """Exact expectation over the reflect/transmit decisions of
    sum_rays W_bin / N for fixed births (scalar reflectance): every decision
    sequence of every ray is traced with forced decisions and weighted by its
    probability.  A sequence is enumerated from its first unset decision on."""
    s = osc.s
    D, nl, F, by, bx = osc.shape
    B, N = by * bx, s.rays_per_point
    Wf = np.asarray(W, dtype=np.float64).reshape(-1, B)
    total = 0.0
    for i in np.asarray(ray_ids, dtype=np.int64):
        pt = int(i) // N
        stack = [(0, 0)]
        while stack:
            bits, k = stack.pop()
            b, _, prob, used = osc.forced(int(i), bits, 64)
            total += prob * (Wf[pt][b] if b >= 0 else 0.0)
            for j in range(k, min(used, 64)):
                stack.append((bits | (1 << j), j + 1))
    return total / N


def loss(irr: np.ndarray, kind: int = 0, w_f: float = 1.0, w_e: float = 1.0):
    """Loss and dL/dI for irradiance [D][n_l][F][By][Bx]."""
    I = np.ascontiguousarray(irr, dtype=np.float64)
    D, nl, F = I.shape[:3]
    B = int(np.prod(I.shape[3:]))
    g = np.zeros_like(I)
    L = lib().orc_loss(_ptr(I, _dp), D, nl, F, B, kind, w_f, w_e, _ptr(g, _dp))
    return L, g
