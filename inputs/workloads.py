"""Synthetic geometric-waveguide workloads and their seeded input tables.

The paper (Results, "System Architecture"; Methods, "Multilayer thin-film
solver") describes a glass slab guiding light by total internal reflection to
an array of partially reflective mirrors, each coated with a multilayer
thin-film stack whose layer thicknesses are the design parameters.  The paper
does not give a complete geometry, so the workloads below are synthetic
stand-ins with the same structure:

* a slab of thickness ``T`` and length ``L`` (mm), glass index ``n_g``;
* ``M`` parallel mirrors tilted by ``tilt`` degrees about the y axis with
  constant ``pitch``, centred on ``center_x``;
* per mirror a stack of layers cycling SiO2 / TiO2 (/ Al2O3), layer 0 = SiO2;
* a rectangular injection window (pupil) on the top face and a binned eyebox
  plane at ``eye_relief`` above the top face.

Refractive indices follow a two-term Cauchy law n(lambda) = A + B / lambda^2
(lambda in micrometres) with A chosen so that n(0.55 um) equals the nominal
index; this is an input recipe, not part of the method.

Everything here is a seeded input generator: thickness draws use numpy's PCG64
generator, so both the oracle and the GPU path consume identical arrays.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# Material slots of the refractive-index table.
MAT_AIR, MAT_GLASS, MAT_SIO2, MAT_TIO2, MAT_AL2O3, MAT_AG, MAT_TA2O5 = range(7)
N_MAT = 7

# Nominal indices at 550 nm and Cauchy B coefficients (um^2).
_NOMINAL = {
    MAT_AIR: (1.0, 0.0),
    MAT_GLASS: (1.52, 0.00420),
    MAT_SIO2: (1.46, 0.00354),
    MAT_TIO2: (2.35, 0.0500),
    MAT_AL2O3: (1.63, 0.00700),
    MAT_TA2O5: (2.13, 0.0),
}
_AG = complex(0.12, 3.3)  # non-dispersive absorbing layer


@dataclasses.dataclass
class Workload:
    """One synthetic waveguide workload (geometry, stacks, rays)."""

    name: str
    seed: int
    # slab
    n_glass: float = 1.52
    T_mm: float = 2.0
    L_mm: float = 30.0
    eye_relief_mm: float = 15.0
    # mirrors
    n_mirrors: int = 6
    tilt_deg: float = 25.0
    pitch_mm: float = 3.0
    center_x_mm: float = 15.0
    # stacks
    n_designs: int = 1
    n_layers: int = 40               # layers per mirror (max layers when variable)
    variable_layers: Optional[Tuple[int, int]] = None   # (lo, hi) layer-count draw
    thk_range: Tuple[float, float] = (0.0, 250.0)
    cycle: Tuple[int, ...] = (MAT_SIO2, MAT_TIO2, MAT_AL2O3)
    ag_layer_at: Optional[int] = None  # insert one Ag layer at this index
    ag_thk_range: Tuple[float, float] = (10.0, 40.0)
    dispersion: bool = True
    # rays
    lambdas_nm: Tuple[float, ...] = (460.0, 530.0, 620.0)
    fov_mode: int = 0                # 0: grid, 1: uniform random per ray
    fov_n: int = 21                  # grid points per axis
    fov_half_deg: float = 15.0
    rays_per_point: int = 4096
    max_events: int = 64
    bins: Tuple[int, int] = (32, 32)  # (x, y)
    fp_shift: int = 24
    # eye pupils: a grid x grid array of circular pupils of this diameter
    # centred on the cells of an equal grid over the eyebox (0: eyebox bins)
    eye_pupil_grid: int = 0
    eye_pupil_diam_mm: float = 4.0
    # the loss of a training step (Eq. 1): kind 0 variances, 1 coefficients
    # of variation, 2 coefficients of variation on pupil images; weights
    loss_kind: int = 0
    loss_wf: float = 1.0
    loss_we: float = 1.0

    # ---- derived workload geometry (input recipe, not the method) ----
    @property
    def pupil(self) -> Tuple[float, float, float]:
        """Injection window (x0, width_x, width_y) on the top face, mm.

        The x width 2*T*tan(2*tilt) is the distance a guided centre-field ray
        advances between two top-face bounces, so the replicated pupils tile
        the slab without gaps; the y width spans the mirror array's eyebox.
        """
        px = 2.0 * self.T_mm * math.tan(math.radians(2.0 * self.tilt_deg))
        return 0.5, px, self.n_mirrors * self.pitch_mm

    @property
    def eyebox(self) -> Tuple[float, float, float, float]:
        """Eyebox rectangle (x0, y0, width, height), mm, centred on the array."""
        side = self.n_mirrors * self.pitch_mm
        return self.center_x_mm - side / 2, -side / 2, side, side

    @property
    def eye_pupils(self) -> np.ndarray:
        """Centres (x, y) of the eye pupils, mm, row by row (empty without
        pupils): the centres of a grid x grid partition of the eyebox."""
        g = self.eye_pupil_grid
        if g <= 0:
            return np.zeros((0, 2))
        ex0, ey0, ew, eh = self.eyebox
        return np.array([[ex0 + (i + 0.5) * ew / g, ey0 + (j + 0.5) * eh / g]
                         for j in range(g) for i in range(g)], dtype=np.float64)

    @property
    def n_bins(self) -> int:
        """Cells of one point's eyebox image: pupils, or bins."""
        return self.eye_pupil_grid ** 2 if self.eye_pupil_grid > 0 else self.bins[0] * self.bins[1]

    @property
    def n_fov(self) -> int:
        return 1 if self.fov_mode == 1 else self.fov_n * self.fov_n

    @property
    def n_points(self) -> int:
        return self.n_designs * len(self.lambdas_nm) * self.n_fov

    @property
    def n_rays(self) -> int:
        return self.n_points * self.rays_per_point

    @property
    def max_layers(self) -> int:
        return self.n_layers + (1 if self.ag_layer_at is not None else 0)

    @property
    def n_params(self) -> int:
        return self.n_designs * self.n_mirrors * self.max_layers


def _cauchy(mat: int, lam_nm: float, dispersion: bool) -> complex:
    if mat == MAT_AG:
        return _AG
    n0, b = _NOMINAL[mat]
    if not dispersion or b == 0.0:
        return complex(n0, 0.0)
    a = n0 - b / 0.55 ** 2
    lam_um = lam_nm * 1e-3
    return complex(a + b / lam_um ** 2, 0.0)


def _fov_grid(n: int, half: float) -> np.ndarray:
    ang = np.array([-half + (2.0 * half) * i / (n - 1) for i in range(n)]) if n > 1 else np.zeros(1)
    grid = np.empty((n * n, 2))
    k = 0
    for iy in range(n):
        for ix in range(n):
            grid[k, 0] = ang[ix]
            grid[k, 1] = ang[iy]
            k += 1
    return grid


def default_omega(m_count: int) -> np.ndarray:
    """Uniform-extraction reflection probabilities p_m = clamp(1/(M-m), .05, .95)."""
    return np.array([min(max(1.0 / (m_count - m), 0.05), 0.95) for m in range(m_count)])


def make_inputs(w: Workload) -> dict:
    """Build every input table for workload ``w`` (numpy, host memory)."""
    lam = np.array(w.lambdas_nm, dtype=np.float64)
    nre = np.zeros((len(lam), N_MAT))
    nim = np.zeros((len(lam), N_MAT))
    for li, l in enumerate(lam):
        for m in range(N_MAT):
            n = _cauchy(m, l, w.dispersion)
            if m == MAT_GLASS and not w.dispersion:
                n = complex(w.n_glass, 0.0)
            nre[li, m] = n.real
            nim[li, m] = n.imag
    rng = np.random.Generator(np.random.PCG64(w.seed))
    D, M, Lm = w.n_designs, w.n_mirrors, w.max_layers
    thk = np.zeros((D, M, Lm))
    mat = np.zeros((D, M, Lm), dtype=np.uint8)
    nlay = np.zeros((D, M), dtype=np.int32)
    for d in range(D):
        for m in range(M):
            if w.variable_layers is not None:
                nl = int(rng.integers(w.variable_layers[0], w.variable_layers[1] + 1))
            else:
                nl = w.n_layers
            for j in range(w.n_layers):
                mat[d, m, j] = w.cycle[j % len(w.cycle)]
            thk[d, m, :nl] = rng.uniform(w.thk_range[0], w.thk_range[1], size=nl)
            # slots beyond the drawn layer count are padding with zero thickness
            nlay[d, m] = nl
            if w.ag_layer_at is not None:
                k = w.ag_layer_at
                thk[d, m, k + 1:] = thk[d, m, k:-1].copy()
                mat[d, m, k + 1:] = mat[d, m, k:-1].copy()
                mat[d, m, k] = MAT_AG
                thk[d, m, k] = rng.uniform(*w.ag_thk_range)
                nlay[d, m] = Lm
    if w.fov_mode == 0:
        fov = _fov_grid(w.fov_n, w.fov_half_deg)
    else:
        h = w.fov_half_deg
        fov = np.array([[-h, h], [-h, h]], dtype=np.float64)
    px0, pxw, pyh = w.pupil
    ex0, ey0, ew, eh = w.eyebox
    out = dict(
        lambda_nm=lam, n_re=nre, n_im=nim, thk=thk, mat=mat, n_layers=nlay,
        omega=default_omega(M), fov=fov, lambda_sel=np.arange(len(lam), dtype=np.int32),
        pupil=(px0, pxw, pyh), eyebox=(ex0, ey0, ew, eh),
    )
    if w.eye_pupil_grid > 0:
        out["eye_pupils"] = w.eye_pupils
        out["eye_pupil_r"] = 0.5 * w.eye_pupil_diam_mm
    return out


def _cfg(i: int, **kw) -> Workload:
    return Workload(seed=20260100 + i, **kw)


#: The five workloads, shaped like the configurations the paper describes (stack sizes,
#: materials, wavelengths, field of view, ray counts).
WORKLOADS = {
    "plain_fp64": _cfg(
        1, name="plain_fp64", n_mirrors=4, n_layers=8, thk_range=(0.0, 200.0),
        cycle=(MAT_SIO2, MAT_TIO2), dispersion=False, lambdas_nm=(550.0,),
        fov_mode=1, fov_half_deg=10.0, rays_per_point=100_000, bins=(10, 10)),
    "fwd_scale": _cfg(
        2, name="fwd_scale", n_mirrors=6, n_layers=40, thk_range=(0.0, 250.0),
        rays_per_point=500_000, bins=(32, 32)),
    # 8192 rays per (wavelength, FoV) point: about 1e8 ray-surface interactions per step
    "diff_1200": _cfg(
        3, name="diff_1200", n_mirrors=6, n_layers=200, thk_range=(0.0, 300.0),
        rays_per_point=8192, bins=(32, 32)),
    "precision_ag": _cfg(
        4, name="precision_ag", n_mirrors=6, n_layers=200, thk_range=(0.0, 300.0),
        ag_layer_at=100, rays_per_point=4096, bins=(32, 32)),
    # the pupil-image objective: diff_1200's stacks, nine wavelengths (three
    # per colour channel), a 3 x 3 grid of 4 mm eye pupils over the eyebox;
    # the rays per point keep the interactions per step near diff_1200's
    "pupil_rgb": _cfg(
        6, name="pupil_rgb", n_mirrors=6, n_layers=200, thk_range=(0.0, 300.0),
        lambdas_nm=(450.0, 470.0, 490.0, 500.0, 530.0, 560.0, 620.0, 660.0, 700.0),
        rays_per_point=2752, bins=(9, 1), eye_pupil_grid=3, eye_pupil_diam_mm=4.0,
        loss_kind=2, loss_wf=10.0, loss_we=3.0),
    "batched": _cfg(
        5, name="batched", n_mirrors=6, n_designs=64, n_layers=250,
        variable_layers=(10, 250), thk_range=(20.0, 200.0),
        lambdas_nm=tuple(float(x) for x in range(400, 701, 10)), fov_n=11,
        rays_per_point=200_000, bins=(16, 16)),
}


def workload(name: str) -> Workload:
    return dataclasses.replace(WORKLOADS[name])


def small_variant(name: str, **kw) -> Workload:
    """A reduced copy of a workload (fewer rays / FoV points) for tests."""
    return dataclasses.replace(WORKLOADS[name], **kw)


def all_names() -> List[str]:
    return list(WORKLOADS)
