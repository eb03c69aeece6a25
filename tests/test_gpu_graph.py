"""Batched scheduling, graph capture and autotuning of the trace step.

A captured step (forward with adjoint entries, loss, adjoint, device step
counter advanced) is replayed several times with eager work and
synchronizations in between; every replay must reproduce, bit for bit, the
eager step with the same step index.  The autotuner must pick a launch
configuration without changing any result.
"""
import numpy as np
import pytest
import torch

import inputs
import paper_2601_04370_amd as gwg

pytestmark = pytest.mark.gpu


def _scene(name="diff_1200", **kw):
    w = inputs.small_variant(name, **kw)
    inp = inputs.make_inputs(w)
    scene = gwg.SceneSpec.from_workload(w, inp)
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device="cuda:0")
    return w, inp, scene, thk


def _step(ctx, scene, thk, seed, step):
    _, _, irr, _, _ = ctx.trace_forward(scene, thk, seed, step, gwg.FP64, grad=True)
    _, dLdI = ctx.loss(irr, 0)
    g = ctx.trace_backward(dLdI, scene)
    return irr, g


def test_graph_replays_match_eager_steps(gctx):
    w, inp, scene, thk = _scene(rays_per_point=256, fov_n=3)
    ref = [tuple(t.clone() for t in _step(gctx, scene, thk, w.seed, 5 + k)) for k in range(3)]
    d_step = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    gctx.set_step_source(d_step)
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):          # sizes every buffer before capture
            _step(gctx, scene, thk, w.seed, 5)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            irr_g, g_g = _step(gctx, scene, thk, w.seed, 5)
            d_step.add_(1)
        torch.cuda.synchronize()
        # the captured forward kept the adjoint entries (nothing allocated during capture)
        assert gctx.forward_kept_entries()
        d_step.zero_()
        torch.cuda.synchronize()
        for k in range(3):
            print(f"replay {k}", flush=True)
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(irr_g, ref[k][0]), f"irradiance of replay {k}"
            assert torch.equal(g_g, ref[k][1]), f"gradient of replay {k}"
            # eager work of the program between replays
            e_irr, _ = _step(gctx, scene, thk, w.seed, 40 + k)
            assert float(e_irr.sum()) > 0.0
        assert int(d_step.item()) == 3
    finally:
        gctx.set_step_source(None)


def test_autotune_keeps_results(gctx, tmp_path):
    w, inp, scene, thk = _scene("batched", n_designs=3, rays_per_point=300, fov_n=3,
                                lambdas_nm=(450.0, 550.0, 650.0))
    q0, c0, irr0, _, _ = gctx.trace_forward(scene, thk, w.seed, 2, gwg.FP64)
    q0, c0 = q0.cpu().numpy(), c0.cpu().numpy()
    cache = str(tmp_path / "tune.txt")
    try:
        t = gctx.autotune(scene, thk, w.seed, gwg.FP64, grad=True, cache_path=cache)
        print("tuned", t, flush=True)
        assert t["block_threads"] in (128, 256) and t["bwd_block_threads"] in (64, 128)
        assert t["rays_per_block"] > 0
        q1, c1, _, _, _ = gctx.trace_forward(scene, thk, w.seed, 2, gwg.FP64)
        assert np.array_equal(q1.cpu().numpy(), q0) and np.array_equal(c1.cpu().numpy(), c0)
        lines = open(cache).read().split("\n")
        assert len([x for x in lines if x.strip()]) == 1
        # a second context reads the cache file instead of timing again
        ctx2 = gwg.Context(0)
        t2 = ctx2.autotune(scene, thk, w.seed, gwg.FP64, grad=True, cache_path=cache)
        assert t2 == t
        ctx2.close()
        assert len([x for x in open(cache).read().split("\n") if x.strip()]) == 1
    finally:
        gctx.set_tuning()


def test_design_chunks_in_one_graph(gctx):
    """A batch traced as chunks of consecutive designs (each chunk's forward,
    loss and adjoint before the next chunk's) gives the single launch's
    irradiance bit for bit and its gradient to rounding (the loss is a sum
    over designs; only the work items differ).  The context keeps every
    chunk's scene, so the chunked step captures in one graph, whose replays
    reproduce the eager chunked steps bit for bit."""
    w, inp, scene, thk = _scene("batched", n_designs=4, rays_per_point=200, fov_n=3,
                                lambdas_nm=(450.0, 550.0, 650.0))
    chunks = []
    for d0 in (0, 2):
        inp_c = dict(inp)
        for k in ("thk", "mat", "n_layers"):
            inp_c[k] = inp[k][d0:d0 + 2].copy()
        sc_c = gwg.SceneSpec.from_workload(w, inp_c)
        sc_c.first_design = d0                 # the batch's random streams
        chunks.append((sc_c, torch.tensor(inp_c["thk"], dtype=torch.float64, device="cuda:0")))

    def chunked(step):
        out = [tuple(t.clone() for t in _step(gctx, sc, th, w.seed, step)) for sc, th in chunks]
        return torch.cat([o[0] for o in out]), torch.cat([o[1] for o in out])

    irr_full, g_full = _step(gctx, scene, thk, w.seed, 3)
    irr_c, g_c = chunked(3)
    assert torch.equal(irr_c, irr_full)
    scale = float(g_full.abs().max())
    assert scale > 0 and float((g_c - g_full).abs().max()) <= 1e-12 * scale
    ref = [chunked(5 + k) for k in range(2)]
    d_step = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    gctx.set_step_source(d_step)
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for sc, th in chunks:
                _step(gctx, sc, th, w.seed, 5)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            outs = [_step(gctx, sc, th, w.seed, 5) for sc, th in chunks]
            d_step.add_(1)
        torch.cuda.synchronize()
        d_step.zero_()
        torch.cuda.synchronize()
        for k in range(2):
            print(f"chunked replay {k}", flush=True)
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(torch.cat([o[0] for o in outs]), ref[k][0])
            assert torch.equal(torch.cat([o[1] for o in outs]), ref[k][1])
            # eager work in between, on a chunk's scene (its buffers were
            # sized before the capture, so nothing the graph points to moves)
            sc, th = chunks[k % 2]
            _step(gctx, sc, th, w.seed, 60 + k)
    finally:
        gctx.set_step_source(None)
