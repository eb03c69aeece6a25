"""Parity of the pupil-image objective on the GPU with the oracle (Results,
"System Architecture": a 3 x 3 grid of eye pupils, three wavelengths per
colour channel, the pupil images and Eq. 1 on them as the objective).

The eyebox outputs hold one value per pupil; the forward (plain and with the
gradient flag), the pupil form of the loss (kind 2) and the gradient through
the trace are compared with the oracle on the same seeded inputs.
"""
import numpy as np
import pytest
import torch

import inputs
import paper_2601_04370_amd as gwg

pytestmark = pytest.mark.gpu

SMALL = dict(rays_per_point=500, fov_n=3, lambdas_nm=(450.0, 530.0, 700.0))


def _scene(**kw):
    w = inputs.small_variant("pupil_rgb", **kw)
    inp = inputs.make_inputs(w)
    return w, inp, gwg.SceneSpec.from_workload(w, inp)


@pytest.mark.parametrize("grad", [False, True])
def test_pupil_forward_matches_oracle(gctx, orc, grad):
    w, inp, scene = _scene(**SMALL)
    print(f"pupil forward grad={grad}", flush=True)
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")
    q, c, irr, rec, st = gctx.trace_forward(scene, thk, w.seed, 0, gwg.FP64, record_stride=1, stats=True,
                                            grad=grad)
    torch.cuda.synchronize()
    q, c, irr = q.cpu().numpy().astype(np.int64), c.cpu().numpy(), irr.cpu().numpy()
    rec = gwg.records_view(rec)
    assert q.shape == (1, 3, 9, 1, 9)
    osc = orc.OracleScene(w, inp)
    oq, oc, ows, ost = osc.forward()
    assert np.array_equal(c, oc.astype(np.int32))
    assert np.all(np.abs(q - oq.astype(np.int64)) <= oc.astype(np.int64))
    orec = osc.trace_rays(np.arange(w.n_rays))
    assert np.array_equal(rec["bin"], [r.bin for r in orec])
    assert np.array_equal(rec["category"], [r.category for r in orec])
    assert np.array_equal(rec["n_events"], [r.n_events for r in orec])
    ow = np.array([r.w for r in orec])
    assert np.max(np.abs(rec["w"] - ow)) <= 1e-11 * max(1.0, ow.max())
    oirr = osc.forward_sampled(1)
    rel = np.abs(irr - oirr).max() / oirr.max()
    print(f"  rays in pupils {c.sum()} of {w.n_rays}; irradiance rel err {rel:.2e}", flush=True)
    assert rel < 1e-6 and c.sum() > 100 and np.count_nonzero(c.sum(axis=(0, 1, 2))) == 9


def test_pupil_loss_matches_oracle(gctx, orc):
    rng = np.random.default_rng(12)
    I = rng.uniform(0, 0.02, size=(2, 9, 25, 1, 9))
    L, g = gctx.loss(torch.tensor(I), 2, 10.0, 3.0)
    oL, og = orc.loss(I, 2, 10.0, 3.0)
    assert abs(L.item() - oL) <= 1e-12 * max(1.0, abs(oL))
    assert np.max(np.abs(g.cpu().numpy() - og)) <= 1e-12 * np.max(np.abs(og))


@pytest.mark.parametrize("mode", ["entries", "regen", "memo"])
def test_pupil_gradient_matches_oracle(gctx, orc, mode):
    w, inp, scene = _scene(rays_per_point=96, fov_n=3, lambdas_nm=(470.0, 560.0, 660.0))
    print(f"pupil gradient {mode}", flush=True)
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")
    osc = orc.OracleScene(w, inp)
    oirr = osc.forward_sampled(1)
    oL, odLdI = orc.loss(oirr, 2, 10.0, 3.0)
    gctx.trace_forward(scene, thk, w.seed, 0, gwg.FP64, grad=(mode != "regen"), memo=(mode == "memo"))
    g = gctx.trace_backward(torch.tensor(odLdI), scene).cpu().numpy()
    og = osc.backward(odLdI, 1)
    scale = np.max(np.abs(og))
    err = np.abs(g - og)
    print(f"  max |g| {scale:.3e} max abs err {err.max():.2e}", flush=True)
    assert scale > 0
    assert np.all(err <= 1e-4 * np.maximum(np.abs(og), 1e-3 * scale))


def test_pupil_step_on_gpu_matches_oracle_step(gctx, orc):
    """One training step of the pupil objective on the GPU (forward, loss
    kind 2, adjoint) against the oracle's: loss and gradient."""
    w, inp, scene = _scene(rays_per_point=128, fov_n=3, lambdas_nm=(490.0, 530.0, 620.0))
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")
    _, _, irr, _, _ = gctx.trace_forward(scene, thk, w.seed, 0, gwg.FP64, grad=True)
    L, dLdI = gctx.loss(irr, 2, 10.0, 3.0)
    g = gctx.trace_backward(dLdI, scene).cpu().numpy()
    osc = orc.OracleScene(w, inp)
    oirr = osc.forward_sampled(1)
    oL, odLdI = orc.loss(oirr, 2, 10.0, 3.0)
    og = osc.backward(odLdI, 1)
    assert abs(L.item() - oL) <= 1e-4 * abs(oL)
    assert np.max(np.abs(g - og)) <= 1e-4 * np.max(np.abs(og))


def test_pupil_scene_validation(gctx):
    w, inp, scene = _scene(rays_per_point=8, fov_n=1, lambdas_nm=(530.0,))
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")
    bad = dict(inp)
    bad["eye_pupils"] = np.array([[15.0, 0.0], [17.0, 0.0]])      # 2 mm apart, radius 2: overlap
    sc = gwg.SceneSpec.from_workload(inputs.small_variant("pupil_rgb", rays_per_point=8, fov_n=1,
                                                          lambdas_nm=(530.0,), bins=(2, 1)), bad)
    with pytest.raises(gwg.GwgError, match="overlap"):
        gctx.trace_forward(sc, thk, w.seed, 0, gwg.FP64)
    sc = gwg.SceneSpec.from_workload(inputs.small_variant("pupil_rgb", rays_per_point=8, fov_n=1,
                                                          lambdas_nm=(530.0,), bins=(3, 3)), inp)
    with pytest.raises(gwg.GwgError, match="bins"):
        gctx.trace_forward(sc, thk, w.seed, 0, gwg.FP64)
