"""Coating optimisation with discrete thickness constraints and layer pruning,
and the pre-optimisation of the mirrors' reflection probabilities.

``learn_reflection_probabilities`` is the step before the trace (Methods,
learned reflection probabilities): omega per mirror is optimised for eyebox
throughput with every coating idealised as a scalar reflectance, using the
library's score-function gradient (``gwg_omega_gradient``); the learned
omega then drives the Monte Carlo sampling of the polarization trace.

The step after the differentiable trace (Results: stacks are optimised from a
random start inside thickness bounds, over-parameterised stacks are pruned by
driving layers to zero thickness; Eq. 1 with w_f = 10 and w_e = 3).  Every
iteration draws fresh paths (the Philox key includes the iteration), and the
library does all of the trace work:

  1. ``gwg_trace_forward`` with the gradient flag (optionally memoized);
  2. ``gwg_loss``: Eq. 1 and dL/dI on the device;
  3. ``gwg_trace_backward``: dL/dthk.

The host then adds the soft-gap penalty's gradient, takes an Adam step on the
thicknesses (nm) and projects them onto the feasible set.

The paper gives the bounds (20-200 nm) and says that a soft gap between 0
and 20 nm lets layers be eliminated; it does not give the mechanism.
Reading taken here:

  - feasible thicknesses are {0} U [t_min, t_max];
  - while optimising, thicknesses live in [0, t_max]; inside the gap
    (0, t_min) they pay mu * phi(t) with phi(t) = t (t_min - t) / t_min^2,
    zero at both ends and largest mid-gap, which pushes a layer either down
    to 0 (pruned) or up to t_min;
  - every ``snap_every`` iterations and at the end, thicknesses still in the
    gap are snapped to 0 below t_min / 2 and to t_min otherwise;
  - thicknesses start from a Gaussian centred at the midpoint of
    [t_min, t_max] (sigma = a sixth of the range), clipped to the range.

Metrics (Eq. 1's terms, population statistics): mean eyebox throughput Ibar,
CV_FoV of the per-FoV throughput and CV_eyebox of the per-bin eyebox
profile, averaged over designs; reported designs are evaluated on several
seeds and averaged (the paper averages five Monte Carlo runs).  With eye
pupils (Results: the images of a grid of pupil positions are the
objective) the "bins" are the pupils: Ibar is the mean throughput into one
pupil (averaged over pupils, FoV samples and wavelengths, hence colour
channels), CV_eyebox the CV over pupils, and the loss is Eq. 1's pupil form
(``gwg_loss`` kind 2).
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Optional

import numpy as np

from .gwg import FP64, Context, SceneSpec


@dataclasses.dataclass
class OptimConfig:
    iters: int = 1000
    lr: float = 2.0                 # Adam step size, nm
    t_min: float = 20.0
    t_max: float = 200.0
    gap_weight: float = 1e-3        # mu of the soft-gap penalty (per layer)
    snap_every: int = 50
    w_f: float = 10.0
    w_e: float = 3.0
    precision: int = FP64
    memo: bool = False              # memoized thin film (exact, faster)
    eval_seeds: int = 5
    loss_kind: int = 1              # Eq. 1 (1), or its pupil-image form (2)


def init_thicknesses(n_layers: np.ndarray, l_max: int, t_min: float = 20.0, t_max: float = 200.0,
                     seed: int = 0) -> np.ndarray:
    """[D][M][Lmax] thicknesses: Gaussian at the midpoint of the bounds,
    sigma = (t_max - t_min) / 6, clipped; padding slots are 0."""
    rng = np.random.default_rng(seed)
    D, M = n_layers.shape
    mid, sig = 0.5 * (t_min + t_max), (t_max - t_min) / 6.0
    thk = np.clip(rng.normal(mid, sig, size=(D, M, l_max)), t_min, t_max)
    for d in range(D):
        for m in range(M):
            thk[d, m, int(n_layers[d, m]):] = 0.0
    return thk


def gap_penalty(t, t_min: float):
    """(phi(t), dphi/dt) elementwise: t (t_min - t) / t_min^2 inside (0, t_min), else 0."""
    inside = (t > 0) & (t < t_min)
    phi = t * (t_min - t) / (t_min * t_min)
    dphi = (t_min - 2 * t) / (t_min * t_min)
    zero = phi * 0
    return (phi * inside + zero, dphi * inside + zero)


def project(t, t_max: float, mask):
    """Box [0, t_max] on real layers, 0 on padding (mask: 1 for real layers)."""
    return t.clamp(0.0, t_max) * mask


def snap(t, t_min: float):
    """Thicknesses in the gap go to 0 (below t_min / 2) or t_min."""
    inside = (t > 0) & (t < t_min)
    up = inside & (t >= 0.5 * t_min)
    down = inside & (t < 0.5 * t_min)
    return t * (~inside) + t_min * up + 0 * down


def metrics(irr, pupils: bool = False) -> dict:
    """Ibar, CV_FoV, CV_eyebox of irradiance [D][n_l][F][by][bx], averaged
    over designs (pupils: the last axes are pupils, and Ibar is the mean
    throughput into one pupil)."""
    import torch
    I = irr.reshape(irr.shape[0], irr.shape[1], irr.shape[2], -1).to(torch.float64)
    eta = I.sum(dim=3)                               # [D][n_l][F]
    ibar = eta.mean(dim=(1, 2))                      # [D]
    if pupils:
        return {"ibar": float((ibar / I.shape[3]).mean()), **_cvs(I, eta, ibar)}
    return {"ibar": float(ibar.mean()), **_cvs(I, eta, ibar)}


def _cvs(I, eta, ibar) -> dict:
    phi = eta.mean(dim=1)                            # [D][F]
    eyeb = I.mean(dim=(1, 2))                        # [D][B]
    cv_f = phi.std(dim=1, unbiased=False) / ibar
    cv_e = eyeb.std(dim=1, unbiased=False) / eyeb.mean(dim=1)
    return {"cv_fov": float(cv_f.mean()), "cv_eyebox": float(cv_e.mean())}


class CoatingOptimizer:
    """Adam on the layer thicknesses of ``scene`` through the library's
    forward, loss and adjoint; the thickness tensor lives on the context's GPU."""

    def __init__(self, ctx: Context, scene: SceneSpec, thk0: np.ndarray, n_layers: np.ndarray, seed: int,
                 cfg: OptimConfig):
        import torch
        self.torch = torch
        self.ctx, self.scene, self.seed, self.cfg = ctx, scene, seed, cfg
        dev = torch.device("cuda", ctx.device)
        self.mask = torch.zeros(thk0.shape, dtype=torch.float64, device=dev)
        for d in range(n_layers.shape[0]):
            for m in range(n_layers.shape[1]):
                self.mask[d, m, : int(n_layers[d, m])] = 1.0
        self.thk = torch.tensor(thk0, dtype=torch.float64, device=dev) * self.mask
        self.param = self.thk.clone().requires_grad_(False)
        self.opt = torch.optim.Adam([self.param], lr=cfg.lr)
        self.history = []

    def step(self, k: int) -> dict:
        torch, ctx, cfg = self.torch, self.ctx, self.cfg
        thk = self.param.detach().clone().contiguous()
        _, _, irr, _, _ = ctx.trace_forward(self.scene, thk, self.seed, k, cfg.precision, grad=True, memo=cfg.memo)
        L, dLdI = ctx.loss(irr, cfg.loss_kind, cfg.w_f, cfg.w_e)
        g = ctx.trace_backward(dLdI, self.scene)
        phi, dphi = gap_penalty(thk, cfg.t_min)
        g = (g + cfg.gap_weight * dphi) * self.mask
        self.param.grad = g
        self.opt.step()
        with torch.no_grad():
            self.param.copy_(project(self.param, cfg.t_max, self.mask))
            if cfg.snap_every and (k + 1) % cfg.snap_every == 0:
                self.param.copy_(snap(self.param, cfg.t_min))
        rec = {"iter": k, "loss": float(L) + cfg.gap_weight * float(phi.sum()),
               **metrics(irr, cfg.loss_kind == 2),
               "pruned": int(((self.param == 0) & (self.mask > 0)).sum())}
        self.history.append(rec)
        return rec

    def run(self, callback: Optional[Callable[[dict], None]] = None) -> np.ndarray:
        for k in range(self.cfg.iters):
            rec = self.step(k)
            if callback:
                callback(rec)
        with self.torch.no_grad():
            self.param.copy_(snap(project(self.param, self.cfg.t_max, self.mask), self.cfg.t_min))
        return self.param.detach().cpu().numpy()

    def evaluate(self, thk: Optional[np.ndarray] = None, seeds=None, step: int = 10 ** 6) -> dict:
        """Eq. 1 terms of a design averaged over Monte Carlo runs with different seeds."""
        torch, ctx, cfg = self.torch, self.ctx, self.cfg
        t = self.param.detach().clone() if thk is None else torch.tensor(thk, dtype=torch.float64,
                                                                          device=self.param.device)
        seeds = seeds if seeds is not None else [self.seed + 1000 + i for i in range(cfg.eval_seeds)]
        acc = {"ibar": 0.0, "cv_fov": 0.0, "cv_eyebox": 0.0, "loss": 0.0}
        for s in seeds:
            _, _, irr, _, _ = ctx.trace_forward(self.scene, t.contiguous(), s, step, cfg.precision, memo=cfg.memo)
            L, _ = ctx.loss(irr, cfg.loss_kind, cfg.w_f, cfg.w_e, want_grad=False)
            m = metrics(irr, cfg.loss_kind == 2)
            for key in ("ibar", "cv_fov", "cv_eyebox"):
                acc[key] += m[key] / len(seeds)
            acc["loss"] += float(L) / len(seeds)
        return acc


def learn_reflection_probabilities(ctx: Context, w, inp: dict, iters: int = 100, lr: float = 0.2, seed: int = 0,
                                   objective: str = "throughput", w_f: float = 10.0, w_e: float = 3.0,
                                   omega0: Optional[np.ndarray] = None, p_min: float = 0.02, p_max: float = 0.98,
                                   callback: Optional[Callable[[dict], None]] = None) -> np.ndarray:
    """Pre-optimisation of the mirrors' reflection probabilities (Methods,
    learned reflection probabilities): every coating idealised as a scalar
    reflectance equal to omega, geometry only.  Each iteration traces fresh
    paths (the forward's bin counts are geometry, so the cheapest thin-film
    mode serves), forms the scalar irradiance I = counts / N, and takes an
    Adam step on logit(omega) with the score-function gradient of the
    objective (gwg_omega_gradient):
      - "throughput" (the paper's): maximise the mean eyebox throughput;
      - "eq1": minimise Eq. 1 (w_f, w_e) at the scalar irradiance.
    omega stays in [p_min, p_max].  Returns omega [M]."""
    import torch
    dev = torch.device("cuda", ctx.device)
    om = np.clip(np.asarray(inp["omega"] if omega0 is None else omega0, dtype=np.float64), p_min, p_max)
    theta = np.log(om / (1.0 - om))
    m1, m2 = np.zeros_like(theta), np.zeros_like(theta)
    b1, b2, eps = 0.9, 0.999, 1e-8
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device=dev)
    saved = ctx.get_tuning()
    try:
        ctx.set_tuning(**{**saved, "table_nodes": 4})
        for k in range(iters):
            om = np.clip(1.0 / (1.0 + np.exp(-theta)), p_min, p_max)
            scene = SceneSpec.from_workload(w, {**inp, "omega": om})
            _, counts, _, _, _ = ctx.trace_forward(scene, thk, seed, k, FP64, table=True, want_irradiance=False)
            I = counts.to(torch.float64) / float(w.rays_per_point)
            n_pts = I.shape[0] * I.shape[1] * I.shape[2]
            if objective == "throughput":
                W = torch.ones_like(I)
                value = float(I.sum()) / n_pts
                sign = -1.0                               # ascent
            elif objective == "eq1":
                L, W = ctx.loss(I, 1, w_f, w_e)
                value = float(L)
                sign = 1.0
            else:
                raise ValueError(f"unknown objective {objective!r}")
            g = ctx.omega_gradient(W, counts, scene).cpu().numpy()
            if objective == "throughput":
                g = g / n_pts
            gt = sign * g * om * (1.0 - om)               # d/dlogit, as a descent direction
            m1 = b1 * m1 + (1 - b1) * gt
            m2 = b2 * m2 + (1 - b2) * gt * gt
            theta = theta - lr * (m1 / (1 - b1 ** (k + 1))) / (np.sqrt(m2 / (1 - b2 ** (k + 1))) + eps)
            if callback:
                callback({"iter": k, "objective": value, "omega": om.tolist()})
    finally:
        ctx.set_tuning(**saved)
    return np.clip(1.0 / (1.0 + np.exp(-theta)), p_min, p_max)


def main():
    import argparse
    import json
    import os
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import inputs

    ap = argparse.ArgumentParser(description="optimise the coating stacks of a synthetic workload")
    ap.add_argument("--workload", default="diff_1200")
    ap.add_argument("--rays-per-point", type=int, default=0)
    ap.add_argument("--designs", type=int, default=0, help="keep the first n designs of the workload")
    ap.add_argument("--iters", type=int, default=1000)
    ap.add_argument("--lr", type=float, default=2.0)
    ap.add_argument("--memo", action="store_true")
    ap.add_argument("--log-every", type=int, default=10)
    a = ap.parse_args()
    w = inputs.workload(a.workload)
    if a.rays_per_point:
        w = dataclasses.replace(w, rays_per_point=a.rays_per_point)
    if a.designs:
        w = dataclasses.replace(w, n_designs=a.designs)
    inp = inputs.make_inputs(w)
    cfg = OptimConfig(iters=a.iters, lr=a.lr, memo=a.memo, loss_kind=2 if w.eye_pupil_grid > 0 else 1)
    thk0 = init_thicknesses(inp["n_layers"], inp["thk"].shape[2], cfg.t_min, cfg.t_max, seed=w.seed)
    ctx = Context(0)
    scene = SceneSpec.from_workload(w, inp)
    opt = CoatingOptimizer(ctx, scene, thk0, inp["n_layers"], w.seed, cfg)
    before = opt.evaluate(thk0)
    print(json.dumps({"initial": before}), flush=True)
    t0 = time.perf_counter()

    def log(rec):
        if rec["iter"] % a.log_every == 0 or rec["iter"] == cfg.iters - 1:
            print(json.dumps({**rec, "elapsed_s": round(time.perf_counter() - t0, 2)}), flush=True)

    thk = opt.run(log)
    after = opt.evaluate(thk)
    n_real = int(inp["n_layers"].sum())
    print(json.dumps({"final": after, "pruned_layers": int(((thk == 0) & (opt.mask.cpu().numpy() > 0)).sum()),
                      "layers": n_real, "s_per_iter": (time.perf_counter() - t0) / cfg.iters,
                      "workload": a.workload, "designs": w.n_designs, "rays_per_point": w.rays_per_point,
                      "loss_kind": cfg.loss_kind, "memo": cfg.memo, "iters": cfg.iters,
                      "eval_seeds": cfg.eval_seeds}), flush=True)


if __name__ == "__main__":
    main()
