"""The coating optimiser on the GPU: a short run lowers Eq. 1 (evaluated on
the same held-out seeds before and after), keeps every thickness feasible
({0} or [20, 200] nm, padding 0), and the memoized and per-hit thin films
take the same steps (their gradients agree to rounding)."""
import numpy as np
import pytest

import inputs
import paper_2601_04370_amd as gwg
from paper_2601_04370_amd import optim

pytestmark = pytest.mark.gpu


def _setup(gctx, rays=512, iters=40, memo=True):
    w = inputs.small_variant("diff_1200", rays_per_point=rays, fov_n=3)
    inp = inputs.make_inputs(w)
    cfg = optim.OptimConfig(iters=iters, lr=5.0, memo=memo, snap_every=20, eval_seeds=3)
    thk0 = optim.init_thicknesses(inp["n_layers"], inp["thk"].shape[2], cfg.t_min, cfg.t_max, seed=w.seed)
    scene = gwg.SceneSpec.from_workload(w, inp)
    return w, inp, cfg, thk0, optim.CoatingOptimizer(gctx, scene, thk0, inp["n_layers"], w.seed, cfg)


def test_optimizer_lowers_loss_and_stays_feasible(gctx):
    w, inp, cfg, thk0, opt = _setup(gctx)
    before = opt.evaluate(thk0)
    thk = opt.run()
    after = opt.evaluate(thk)
    print(f"  loss {before['loss']:.4f} -> {after['loss']:.4f}; Ibar {before['ibar']:.4f} -> {after['ibar']:.4f}; "
          f"CV_FoV {before['cv_fov']:.3f} -> {after['cv_fov']:.3f}; CV_eyebox {before['cv_eyebox']:.3f} -> "
          f"{after['cv_eyebox']:.3f}", flush=True)
    assert after["loss"] < before["loss"]
    nl = inp["n_layers"]
    for m in range(nl.shape[1]):
        real = thk[0, m, : nl[0, m]]
        assert np.all((real == 0.0) | ((real >= cfg.t_min) & (real <= cfg.t_max)))
        assert np.all(thk[0, m, nl[0, m]:] == 0.0)
    losses = [r["loss"] for r in opt.history]
    assert np.all(np.isfinite(losses))


def test_memoized_and_per_hit_steps_agree(gctx):
    runs = []
    for memo in (False, True):
        _, _, _, _, opt = _setup(gctx, rays=256, iters=3, memo=memo)
        runs.append(opt.run())
    assert np.allclose(runs[0], runs[1], rtol=0, atol=1e-9)
