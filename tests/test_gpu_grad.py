"""Parity of gwg_trace_backward (adjoint kernel) with the oracle's adjoint, and
of gwg_loss with the oracle's loss.

The oracle differentiates its own recursive-Airy solve and stores the whole
path; the GPU runs the characteristic-matrix adjoint with segment
recomputation.  Both receive the same dL/dI.
"""
import numpy as np
import pytest
import torch

import inputs
import paper_2601_04370_amd as gwg

pytestmark = pytest.mark.gpu


# backward modes: adjoint entries recorded by the forward; paths regenerated
# by the backward; entry regions too small for some items (both kernels run)
MODES = {"entries": (True, 0), "regen": (False, 0), "mixed": (True, 2), "memo": (True, 0)}


def _grad_case(gctx, orc, w, inp, precision=0, stride=1, tile=0, bwd_wg=0, mode="entries"):
    scene = gwg.SceneSpec.from_workload(w, inp)
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")
    osc = orc.OracleScene(w, inp)
    oirr = osc.forward_sampled(stride)
    L, dLdI = orc.loss(oirr, 0)
    grad, per_ray = MODES[mode]
    gctx.set_tuning(bwd_rays_per_block=tile, bwd_block_threads=bwd_wg, adj_entries_per_ray=per_ray)
    try:
        gctx.trace_forward(scene, thk, w.seed, 0, precision, grad=grad, memo=(mode == "memo"))
        assert gctx.forward_kept_entries() == grad
        g, st = gctx.trace_backward(torch.tensor(dLdI), scene, sample_stride=stride, stats=True)
        g = g.cpu().numpy()
        print(f"  mode {mode}: regenerated rays {st['rays']}, adjoint hits {st['adjoint_hits']}", flush=True)
    finally:
        gctx.set_tuning()
    og = osc.backward(dLdI, stride)
    return g, og


GCASES = [
    ("plain_fp64", dict(rays_per_point=4000), 1, 0),
    ("diff_1200", dict(rays_per_point=96, fov_n=3), 1, 640),
    ("precision_ag", dict(rays_per_point=64, fov_n=3, lambdas_nm=(530.0,)), 1, 0),
    ("batched", dict(n_designs=2, rays_per_point=48, fov_n=3, lambdas_nm=(420.0, 680.0)), 1, 0),
]


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("name,kw,stride,tile", GCASES)
def test_backward_fp64_matches_oracle(gctx, orc, name, kw, stride, tile, mode):
    w = inputs.small_variant(name, **kw)
    inp = inputs.make_inputs(w)
    print(f"backward fp64 {name} {kw} {mode}", flush=True)
    g, og = _grad_case(gctx, orc, w, inp, 0, stride, tile, mode=mode)
    scale = np.max(np.abs(og))
    assert scale > 0
    err = np.abs(g - og)
    print(f"  max |g| {scale:.3e}  max abs err {err.max():.3e}  rel {err.max() / scale:.2e}", flush=True)
    # elementwise, relative with a floor at 1e-3 of the largest component
    assert np.all(err <= 1e-4 * np.maximum(np.abs(og), 1e-3 * scale))
    # padding slots are exactly zero
    for d in range(inp["thk"].shape[0]):
        for m in range(w.n_mirrors):
            assert np.all(g[d, m, inp["n_layers"][d, m]:] == 0.0)


@pytest.mark.parametrize("wg,tile", [(64, 1280), (128, 2150)])
def test_backward_pooled_rounds_match_oracle(gctx, orc, wg, tile):
    """The per-hit forward takes a wave's rays in pools of at most 8 rounds of
    64: with 64-thread workgroups and 1280-ray tiles a wave walks 20 rounds of
    a point's first item (pools of 8, 8 and 4) and 14 of its second (8 and 6,
    the last round partial); with 128 threads and one 2150-ray tile per point
    17 rounds (8, 8 and 1, partial in the second wave), so entries, checkpoint
    slots and the field-pass order cross pools.  Forward counts and gradient
    against the oracle."""
    w = inputs.small_variant("diff_1200", rays_per_point=2150, fov_n=2, lambdas_nm=(530.0,))
    inp = inputs.make_inputs(w)
    scene = gwg.SceneSpec.from_workload(w, inp)
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")
    osc = orc.OracleScene(w, inp)
    oq, oc, ows, ost = osc.forward()
    oirr = osc.forward_sampled(1)
    L, dLdI = orc.loss(oirr, 0)
    print(f"pooled rounds wg={wg} tile={tile}", flush=True)
    gctx.set_tuning(block_threads=wg, rays_per_block=tile)
    try:
        q, c, irr, _, _ = gctx.trace_forward(scene, thk, w.seed, 0, 0, grad=True)
        assert gctx.forward_kept_entries()
        g = gctx.trace_backward(torch.tensor(dLdI), scene).cpu().numpy()
    finally:
        gctx.set_tuning()
    assert np.array_equal(c.cpu().numpy().astype(np.uint32), oc)
    og = osc.backward(dLdI, 1)
    scale = np.max(np.abs(og))
    err = np.abs(g - og)
    print(f"  max |g| {scale:.3e}  rel err {err.max() / scale:.2e}", flush=True)
    assert np.all(err <= 1e-4 * np.maximum(np.abs(og), 1e-3 * scale))


@pytest.mark.parametrize("grad,memo", [(True, False), (False, False), (True, True)])
def test_backward_is_deterministic(gctx, orc, grad, memo):
    w = inputs.small_variant("diff_1200", rays_per_point=128, fov_n=3)
    inp = inputs.make_inputs(w)
    scene = gwg.SceneSpec.from_workload(w, inp)
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")
    rng = np.random.default_rng(0)
    dLdI = torch.tensor(rng.standard_normal(scene.shape))
    gctx.trace_forward(scene, thk, w.seed, 0, 0, grad=grad, memo=memo)
    a = gctx.trace_backward(dLdI, scene).cpu().numpy()
    b = gctx.trace_backward(dLdI, scene).cpu().numpy()
    assert np.array_equal(a, b)
    gctx.trace_forward(scene, thk, w.seed, 0, 0, grad=grad, memo=memo)
    c = gctx.trace_backward(dLdI, scene).cpu().numpy()
    assert np.array_equal(a, c)


def test_backward_full_size_sampled(gctx, orc):
    """Full differentiation workload, default launch configuration; only rays
    with id % 4099 == 0 contribute on both sides."""
    w = inputs.workload("diff_1200")
    inp = inputs.make_inputs(w)
    stride = 4099
    g, og = _grad_case(gctx, orc, w, inp, 0, stride)
    scale = np.max(np.abs(og))
    err = np.abs(g - og)
    print(f"full size sampled: max |g| {scale:.3e} rel err {err.max() / scale:.2e}", flush=True)
    assert np.all(err <= 1e-4 * np.maximum(np.abs(og), 1e-3 * scale))


def test_backward_full_size_entries_match_regeneration(gctx):
    """Full differentiation workload in the launch configuration the bench
    times (adjoint entries from the forward, every ray contributing): the
    gradient equals that of the regenerating backward (checked against the
    oracle above on every ray of small cases and on sampled rays at full
    size) up to summation order."""
    w = inputs.workload("diff_1200")
    inp = inputs.make_inputs(w)
    scene = gwg.SceneSpec.from_workload(w, inp)
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")
    _, _, irr, _, _ = gctx.trace_forward(scene, thk, w.seed, 3, 0, grad=True)
    _, dLdI = gctx.loss(irr, 0)
    ge, st = gctx.trace_backward(dLdI, scene, stats=True)
    gctx.trace_forward(scene, thk, w.seed, 3, 0, grad=False)
    gr = gctx.trace_backward(dLdI, scene)
    gctx.trace_forward(scene, thk, w.seed, 3, 0, grad=True, memo=True)
    gm, sm = gctx.trace_backward(dLdI, scene, stats=True)
    ge, gr, gm = ge.cpu().numpy(), gr.cpu().numpy(), gm.cpu().numpy()
    print(f"memoized: {sm['adjoint_hits']} thin-film adjoints for {st['adjoint_hits']} hits, "
          f"max diff {np.max(np.abs(gm - gr)):.2e}", flush=True)
    assert np.all(np.abs(gm - gr) <= 1e-10 * np.maximum(np.abs(gr), 1e-3 * np.max(np.abs(gr))))
    scale = np.max(np.abs(gr))
    print(f"full size entries vs regeneration: max |g| {scale:.3e} max diff {np.max(np.abs(ge - gr)):.2e} "
          f"regenerated rays {st['rays']} adjoint hits {st['adjoint_hits']}", flush=True)
    assert st["rays"] == 0
    assert np.all(np.abs(ge - gr) <= 1e-10 * np.maximum(np.abs(gr), 1e-3 * scale))


def test_autograd_function(gctx, orc):
    w = inputs.small_variant("plain_fp64", rays_per_point=3000)
    inp = inputs.make_inputs(w)
    scene = gwg.SceneSpec.from_workload(w, inp)
    GWGTrace = gwg.make_trace_function()
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0", requires_grad=True)
    irr = GWGTrace.apply(thk, gctx, scene, w.seed, 0, gwg.FP64)
    weights = torch.linspace(0.5, 1.5, irr.numel(), dtype=torch.float64, device="cuda:0").view_as(irr)
    (irr * weights).sum().backward()
    osc = orc.OracleScene(w, inp)
    og = osc.backward(weights.cpu().numpy(), 1)
    g = thk.grad.cpu().numpy()
    assert np.max(np.abs(g - og)) <= 1e-6 * np.max(np.abs(og))


def test_autograd_function_non_contiguous_leaf(gctx):
    """A non-contiguous thickness leaf: the library reads a contiguous copy in
    the forward and again in the backward; the copy must stay alive in
    between even when the allocator is busy, so the gradient equals that of
    a contiguous leaf bit for bit."""
    w = inputs.small_variant("diff_1200", rays_per_point=64, fov_n=3)
    inp = inputs.make_inputs(w)
    scene = gwg.SceneSpec.from_workload(w, inp)
    GWGTrace = gwg.make_trace_function()
    grads = []
    for contiguous in (True, False):
        if contiguous:
            thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0", requires_grad=True)
        else:
            base = torch.tensor(np.ascontiguousarray(inp["thk"].transpose(2, 1, 0)), dtype=torch.float64,
                                device="cuda:0")
            thk = base.permute(2, 1, 0).detach().requires_grad_(True)
            assert not thk.is_contiguous() and thk.is_leaf
            del base
        irr = GWGTrace.apply(thk, gctx, scene, w.seed, 0, gwg.FP64)
        # churn the caching allocator between forward and backward
        junk = [torch.full(inp["thk"].shape, 1e3, dtype=torch.float64, device="cuda:0") for _ in range(8)]
        weights = torch.linspace(0.5, 1.5, irr.numel(), dtype=torch.float64, device="cuda:0").view_as(irr)
        (irr * weights).sum().backward()
        del junk
        grads.append(thk.grad.cpu().numpy())
    assert np.array_equal(grads[0], grads[1])


@pytest.mark.parametrize("kind", [0, 1])
def test_loss_matches_oracle(gctx, orc, kind):
    rng = np.random.default_rng(kind)
    I = rng.uniform(0, 1e-3, size=(2, 3, 9, 8, 8))
    wf, we = (10.0, 3.0) if kind else (1.0, 1.0)
    L, g = gctx.loss(torch.tensor(I), kind, wf, we)
    oL, og = orc.loss(I, kind, wf, we)
    assert abs(L.item() - oL) <= 1e-12 * max(1.0, abs(oL))
    assert np.max(np.abs(g.cpu().numpy() - og)) <= 1e-12 * np.max(np.abs(og))


def test_backward_requires_forward(orc):
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    ctx = gwg.Context(0)
    w = inputs.small_variant("plain_fp64", rays_per_point=10)
    scene = gwg.SceneSpec.from_workload(w, inputs.make_inputs(w))
    with pytest.raises(gwg.GwgError) as e:
        ctx.trace_backward(_t.zeros(scene.shape, dtype=_t.float64), scene)
    assert e.value.code == 4
    ctx.close()


@pytest.mark.parametrize("name,kw", [
    ("diff_1200", dict(rays_per_point=160, fov_n=3)),
    ("plain_fp64", dict(rays_per_point=3000)),
    ("batched", dict(n_designs=2, rays_per_point=64, fov_n=3, lambdas_nm=(420.0, 680.0))),
])
def test_stored_sweep_checkpoints_give_the_same_gradient(gctx, name, kw):
    """The FP64 forward keeps the adjoint's sweep checkpoints for (some or
    all) entries; the adjoint then skips that sweep.  Same arithmetic, so
    the gradient is identical bit for bit to the recomputing adjoint."""
    w = inputs.small_variant(name, **kw)
    inp = inputs.make_inputs(w)
    scene = gwg.SceneSpec.from_workload(w, inp)
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")
    rng = np.random.default_rng(11)
    dLdI = torch.tensor(rng.standard_normal(scene.shape))
    out = []
    for per in (-1, 0, 1):
        gctx.set_tuning(ck_entries_per_ray=per)
        try:
            gctx.trace_forward(scene, thk, w.seed, 0, 0, grad=True)
            out.append(gctx.trace_backward(dLdI, scene).cpu().numpy())
        finally:
            gctx.set_tuning()
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


@pytest.mark.parametrize("n_layers", [1, 15, 16, 17, 31, 32, 33, 65])
def test_checkpoint_schedule_layer_counts(gctx, orc, n_layers):
    """Stacks with no checkpoint (L at most the interval) and with L - 1 just
    below, at and above a multiple of either checkpoint interval (16 layers
    for hits that meet an evanescent layer, 32 for the others): the gradient
    with the forward's stored sweep checkpoints matches the oracle and equals
    the recomputing adjoint's bit for bit."""
    w = inputs.small_variant("diff_1200", rays_per_point=96, fov_n=3, n_layers=n_layers)
    inp = inputs.make_inputs(w)
    print(f"checkpoint schedule diff_1200 n_layers={n_layers}", flush=True)
    g, og = _grad_case(gctx, orc, w, inp, 0, 1, 0, mode="entries")
    scale = np.max(np.abs(og))
    assert scale > 0
    err = np.abs(g - og)
    assert np.all(err <= 1e-4 * np.maximum(np.abs(og), 1e-3 * scale))
    scene = gwg.SceneSpec.from_workload(w, inp)
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")
    dLdI = torch.tensor(np.random.default_rng(5).standard_normal(scene.shape))
    out = []
    for per in (-1, 0):
        gctx.set_tuning(ck_entries_per_ray=per)
        try:
            gctx.trace_forward(scene, thk, w.seed, 0, 0, grad=True)
            out.append(gctx.trace_backward(dLdI, scene).cpu().numpy())
        finally:
            gctx.set_tuning()
    assert np.array_equal(out[0], out[1])


def test_gradient_on_a_quarter_wave_stack(gctx, orc):
    """Every layer of an SiO2/TiO2 stack a quarter wave thick at the first
    mirror incidence of the centre field (kappa = n_glass sin 25 deg): the
    hits there lie deep in the stack's reflection band, where the transfer
    matrix grows fastest over a checkpoint interval and the adjoint's walk
    down each interval with inverse layer matrices loses the most digits.
    Gradient against the oracle elementwise to 1e-7 (relative, with a floor
    at 1e-3 of the largest component)."""
    lam = 530.0
    w = inputs.small_variant("diff_1200", rays_per_point=512, fov_n=3, lambdas_nm=(lam,),
                             cycle=(inputs.MAT_SIO2, inputs.MAT_TIO2))
    inp = inputs.make_inputs(w)
    kap = w.n_glass * np.sin(np.radians(w.tilt_deg))
    for m in range(w.n_mirrors):
        for j in range(w.n_layers):
            n = inp["n_re"][0, inp["mat"][0, m, j]]
            inp["thk"][0, m, j] = lam / (4.0 * np.sqrt(n * n - kap * kap))
    print(f"quarter-wave stack: thicknesses {inp['thk'][0, 0, :2]} nm", flush=True)
    g, og = _grad_case(gctx, orc, w, inp, 0, 1, 0, mode="entries")
    scale = np.max(np.abs(og))
    assert scale > 0
    err = np.abs(g - og)
    rel = err / np.maximum(np.abs(og), 1e-3 * scale)
    print(f"  max |g| {scale:.3e}  max abs err {err.max():.3e}  max rel {rel.max():.2e}", flush=True)
    assert np.all(err <= 1e-7 * np.maximum(np.abs(og), 1e-3 * scale))


def test_work_order_does_not_change_results(gctx):
    """Work items are taken largest first: the forward by the mirror hits its
    previous forward of the same decomposition recorded, the adjoint by the
    entry counts.  Every output is indexed by item, so a fresh context (item
    order) and a context whose previous forward traced another step give the
    same bits: bins, counts, ray records and gradient."""
    w = inputs.small_variant("diff_1200", rays_per_point=1024, fov_n=3)
    inp = inputs.make_inputs(w)
    scene = gwg.SceneSpec.from_workload(w, inp)
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")
    dLdI = torch.tensor(np.random.default_rng(3).standard_normal(scene.shape))
    outs = []
    for warm in (False, True):
        ctx = gwg.Context(0)
        if warm:
            ctx.trace_forward(scene, thk, w.seed, 7, 0, grad=True)
        q, c, _, rec, _ = ctx.trace_forward(scene, thk, w.seed, 0, 0, record_stride=3, grad=True)
        g = ctx.trace_backward(dLdI, scene)
        outs.append((q.cpu().numpy(), c.cpu().numpy(), gwg.records_view(rec), g.cpu().numpy()))
        del ctx
    (qa, ca, ra, ga), (qb, cb, rb, gb) = outs
    assert np.array_equal(qa, qb) and np.array_equal(ca, cb)
    for k in ra:
        assert np.array_equal(ra[k], rb[k]), k
    assert np.array_equal(ga, gb)
    assert np.any(ga != 0.0)
