#!/usr/bin/env python3
"""Throughput of one optimisation step of the differentiable waveguide trace.

A step is the whole hot path on one batch: forward Monte Carlo trace with
per-hit thin-film solves and fixed-point eyebox scatter, the eyebox loss and
its dL/dI, and the adjoint trace down to every layer thickness (plus the
fixed-order gradient reduction).  Each step draws fresh paths (the Philox
key includes the step index).  The metric is forward ray-surface
interactions per second of whole steps.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed|fp32]
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd ray-surface interactions/s @1200 layers; mixed vs FP64, |dR|<=1e-5"
UNIT = "interactions/s"
# MI355X vector peaks (TFLOP/s): FP64 78.6; FP32 157.3 (packed dual-issue)
PEAK_FP64 = 78.6
# Algorithmic FLOPs per (mirror hit, layer) of a lossless layer, counting an
# FMA as two and one sine/cosine pair as zero (reported separately):
#   forward solve 29 = phase 1 + four X/Y products 4 + two real-coefficient
#     complex 2x2 matrix-vector products 2 x 12;
#   adjoint 125 = exit-to-incident sweep 29 + inverse step back down 29 +
#     contraction u^T D w for s and p 39 + covector step for s and p 28;
#     96 where the forward solve stored the sweep's checkpoints (its 29 are
#     then part of the forward's work).
# Adjoint layer steps are counted per hit that enters the thin-film adjoint;
# regenerated hits (items whose entry regions overflowed) add 29 each.
FLOP_FWD_LAYER = 29.0
FLOP_ADJ_LAYER = 125.0


def source_hash() -> str:
    """Hash of the library's sources (the one compiled into libgwg.so)."""
    from paper_2601_04370_amd import build
    return build.source_hash()


def load_traffic(kernel: str, workload: str, precision: str):
    """HBM bytes per launch measured by rocprofv3 PMC runs (profiles/traffic.json),
    valid only for the kernel sources they were measured on."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    e = t.get(f"{kernel}/{workload}/{precision}")
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get("bytes_per_launch")


def _oracle_workers(name, rays_per_point, chunks, forward_only):
    """Run the oracle on each chunk of whole points in its own process
    (`oracle.points`), all released together once every one has built its
    scenes; returns the wall time from release to the last result and the
    per-process results."""
    import subprocess
    procs = []
    try:
        for pts in chunks:
            arg = json.dumps({"workload": name, "rays_per_point": rays_per_point,
                              "points": [list(p) for p in pts], "forward_only": forward_only})
            procs.append(subprocess.Popen([sys.executable, "-m", "oracle.points", arg], cwd=ROOT,
                                          stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True))
        for p in procs:
            if p.stdout.readline().strip() != "ready":
                raise RuntimeError("oracle worker failed to start")
        t = time.perf_counter()
        for p in procs:
            p.stdin.write("go\n")
            p.stdin.flush()
        res = [json.loads(p.stdout.readline()) for p in procs]
        wall = time.perf_counter() - t
        for p in procs:
            if p.wait(timeout=60) != 0:
                raise RuntimeError("oracle worker failed")
        return wall, res
    finally:
        for p in procs:
            if p.poll() is None:
                p.kill()


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, inp, name: str, rays_per_point: int, interactions_per_point: float,
                 forward_only: bool = False, min_interactions: float = 1e6, max_cores: int = 16):
    """The FP64 oracle (plain C, as it stands) on whole (wavelength, FoV)
    points of the same workload, forward + loss + adjoint (or forward only):

    - one thread: the fewest points spread over the grid that hold at least
      `min_interactions` interactions;
    - all host cores: one worker process per core (at most `max_cores`, the
      host's share for one GPU), each running whole points of its own, the
      same number of points per core, released together and timed by the
      wall clock from release to the last result.

    The point loop runs the oracle's own calls; only the points differ
    between workers (each point's rays are those of a workload holding that
    point alone)."""
    import math
    n_l = len(w.lambdas_nm)
    F = w.n_fov
    n_pts = n_l * F
    ipp = max(interactions_per_point, 1.0)
    k1 = max(1, min(n_pts, math.ceil(min_interactions / ipp)))
    pts = [divmod(int(j * n_pts / k1), F) for j in range(k1)]
    el1, r1 = _oracle_workers(name, rays_per_point, [pts], forward_only)
    int1 = r1[0]["interactions"]
    el1 = r1[0]["seconds"]
    cores = max(1, min(len(os.sched_getaffinity(0)), max_cores))
    per_core = max(1, math.ceil(min_interactions / (ipp * cores)))
    total = min(n_pts, per_core * cores)
    allpts = [divmod(int(j * n_pts / total), F) for j in range(total)]
    chunks = [allpts[c::cores] for c in range(cores)]
    chunks = [c for c in chunks if c]
    wall, res = _oracle_workers(name, rays_per_point, chunks, forward_only)
    intn = sum(r["interactions"] for r in res)
    what = "forward" if forward_only else "forward + loss + adjoint"
    return {"value": intn / wall, "unit": UNIT, "cores": len(chunks), "kind": "oracle",
            "sample": f"{len(allpts)} whole (wavelength, FoV) points of the workload ({intn} interactions, "
                      f"{w.rays_per_point} rays each), {what}, FP64 C, one worker process per core, "
                      f"{wall:.1f} s wall",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "single_thread": {"value": int1 / el1, "unit": UNIT, "cores": 1,
                              "sample": f"{len(pts)} whole points ({int1} interactions), {what}, "
                                        f"{el1:.1f} s"}}


def copy_probe(torch, mib: int = 1024, reps: int = 5):
    """A plain device-to-device copy of `mib` MiB, `reps` times: each launch
    reads and writes exactly mib MiB, which scales the FETCH_SIZE and
    WRITE_SIZE counters to bytes."""
    n = mib * 1024 * 1024 // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": reps}))


def progress(msg: str) -> None:
    """One line on stderr as each phase of the run ends (stdout carries only
    the result line)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


# Per-ray storage the forward keeps for the adjoint (gwg_api.cpp): entry
# regions of 8 entries of 6 doubles, checkpoints of 4 entries of
# (Lmax / 16 + 1) blocks of 64 bytes; and their budgets.
ENTRY_BYTES_PER_RAY = 8 * 6 * 8
ENTRY_BUDGET = 96 * 2**30
CHECKPOINT_BUDGET = 128 * 2**30


def auto_design_chunks(w) -> int:
    """Fewest consecutive-design chunks whose entries and sweep checkpoints
    both fit the library's budgets at full per-ray counts."""
    rays_per_design = len(w.lambdas_nm) * w.fov_n * w.fov_n * w.rays_per_point
    ck_per_ray = 4 * (w.n_layers // 16 + 1) * 64
    per_design = rays_per_design * max(ENTRY_BYTES_PER_RAY / ENTRY_BUDGET, ck_per_ray / CHECKPOINT_BUDGET)
    fit = max(1, int(1.0 / per_design))                # designs per chunk
    return -(-w.n_designs // fit)


def design_slice(inp, d, n=1):
    """Inputs of designs d .. d + n - 1 alone (per-design or per-chunk launches)."""
    out = dict(inp)
    for k in ("thk", "mat", "n_layers"):
        out[k] = inp[k][d:d + n].copy()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "fp32"])
    ap.add_argument("--workload", default="diff_1200")
    ap.add_argument("--rays-per-point", type=int, default=0, help="override the workload's rays per point")
    ap.add_argument("--forward-only", action="store_true", help="time the forward trace alone")
    ap.add_argument("--graph", action="store_true",
                    help="capture one step in a graph (device step counter) and time its replays")
    ap.add_argument("--autotune", action="store_true", help="autotune launch parameters first")
    ap.add_argument("--memo", action="store_true",
                    help="memoized thin film: one solve per distinct hit key of a work item in the forward, one "
                         "adjoint per key in the backward (reported separately from the per-hit metric)")
    ap.add_argument("--table", action="store_true",
                    help="angle-table thin film (interpolated model, reported separately with its error against "
                         "the per-hit solve)")
    ap.add_argument("--table-nodes", type=int, default=0, help="incidence angles of the table (0: library default)")
    ap.add_argument("--rays-per-block", type=int, default=0,
                    help="rays per work item (tuning rays_per_block; 0: the library's choice)")
    ap.add_argument("--per-design", action="store_true",
                    help="also time one launch per design (the batched workload) for comparison")
    ap.add_argument("--design-chunks", type=int, default=0,
                    help="also time the batch as this many launches of consecutive designs (each chunk's "
                         "forward, loss and adjoint before the next chunk's, so its stored sweeps fit); "
                         "-1: the fewest chunks whose adjoint entries and sweep checkpoints fit the library's "
                         "budgets")
    ap.add_argument("--cpu-interactions", type=float, default=1e6,
                    help="interactions in each CPU-baseline sample (whole points)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of known size (calibrates HBM byte counters)")
    a = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print(json.dumps({"error": "only one GPU is measured: the per-GPU kernel at its real shape is the whole "
                                   "measured path; sharding over GPUs is not built", "n_gpus": a.gpus}))
        sys.exit(2)

    import dataclasses

    import numpy as np
    import torch

    if a.copy_probe:
        copy_probe(torch)
        return

    import inputs
    import paper_2601_04370_amd as gwg

    w = inputs.workload(a.workload)
    if a.rays_per_point:
        w = dataclasses.replace(w, rays_per_point=a.rays_per_point)
    inp = inputs.make_inputs(w)
    scene = gwg.SceneSpec.from_workload(w, inp)
    prec = gwg.PRECISIONS[a.precision]
    ctx = gwg.Context(0)
    dev = torch.device("cuda", 0)
    thk = torch.tensor(inp["thk"], dtype=torch.float64, device=dev)
    fo = a.forward_only
    extra = {}
    if a.autotune:
        t = time.perf_counter()
        extra["tuning"] = ctx.autotune(scene, thk, w.seed, prec, grad=not fo)
        extra["autotune_s"] = time.perf_counter() - t

    if a.rays_per_block:
        t = ctx.get_tuning()
        t["rays_per_block"] = a.rays_per_block
        ctx.set_tuning(**t)
        extra["rays_per_block"] = a.rays_per_block
    if a.memo and a.table:
        sys.exit("--memo and --table exclude each other")
    if a.table and a.table_nodes:
        t = ctx.get_tuning()
        t["table_nodes"] = a.table_nodes
        ctx.set_tuning(**t)

    def step(k, ev=None, sc=scene, th=thk, table=a.table):
        if ev:
            ev[0].record()
        _, _, irr, _, _ = ctx.trace_forward(sc, th, w.seed, k, prec, grad=not fo, memo=a.memo, table=table)
        if ev:
            ev[1].record()
        if fo:
            if ev:
                ev[2].record()
                ev[3].record()
            return irr
        _, dLdI = ctx.loss(irr, w.loss_kind, w.loss_wf, w.loss_we)
        if ev:
            ev[2].record()
        g = ctx.trace_backward(dLdI, sc)
        if ev:
            ev[3].record()
        return g

    for k in range(a.warmup):
        step(k)
    torch.cuda.synchronize()
    progress(f"{a.warmup} warm-up steps done")
    ctx.set_timing(True)
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step(a.warmup + i, events[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    progress(f"{a.steps} timed steps done: {wall / a.steps * 1e3:.2f} ms per step")
    fwd_ms = [e[0].elapsed_time(e[1]) for e in events]
    loss_ms = [e[1].elapsed_time(e[2]) for e in events]
    bwd_ms = [e[2].elapsed_time(e[3]) for e in events]
    # durations of the trace kernel launches themselves (library HIP events on
    # the launch stream), for the roofline
    n_t = min(a.steps, gwg.TIMING_RING)
    kfwd_ms = ctx.kernel_times(gwg.KERNEL_FORWARD, n_t)
    kbwd_ms = ctx.kernel_times(gwg.KERNEL_ADJOINT, n_t) if not fo else [0.0]
    ctx.set_timing(False)

    if a.graph:
        # one captured step (device step counter advanced inside), replayed
        d_step = torch.zeros(1, dtype=torch.int32, device=dev)
        ctx.set_step_source(d_step)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step(a.warmup + a.steps)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step(a.warmup + a.steps)
            d_step.add_(1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(a.steps):
            graph.replay()
        torch.cuda.synchronize()
        g_wall = time.perf_counter() - tg
        ctx.set_step_source(None)
        extra["graph_ms_per_step"] = g_wall / a.steps * 1e3
        extra["eager_ms_per_step"] = wall / a.steps * 1e3
        progress(f"graph replays done: {extra['graph_ms_per_step']:.2f} ms per step")

    if a.table:
        # the interpolated model against the per-hit solve on the same paths
        # (untimed): irradiance and, for a full step, the gradient
        k = a.warmup
        _, _, irr_t, _, _ = ctx.trace_forward(scene, thk, w.seed, k, prec, grad=not fo, table=True)
        irr_t = irr_t.clone()
        g_t = None
        if not fo:
            _, dLdI_t = ctx.loss(irr_t, w.loss_kind, w.loss_wf, w.loss_we)
        _, _, irr_e, _, _ = ctx.trace_forward(scene, thk, w.seed, k, prec, grad=not fo)
        e_irr = float((irr_t - irr_e).abs().max() / irr_e.abs().max())
        tab = {"nodes": ctx.get_tuning()["table_nodes"] or 8192, "irradiance_max_rel_err": e_irr,
               "irradiance_mean_abs_rel_err": float((irr_t - irr_e).abs().sum() / irr_e.abs().sum())}
        if not fo:
            g_e = ctx.trace_backward(dLdI_t, scene).clone()
            ctx.trace_forward(scene, thk, w.seed, k, prec, grad=True, table=True)
            g_t = ctx.trace_backward(dLdI_t, scene)
            tab["grad_max_rel_err"] = float((g_t - g_e).abs().max() / g_e.abs().max())
        extra["table"] = tab

    # counters of the timed steps (recomputed untimed: same seeds, same paths)
    inter = hits = lay_f = lay_b = lay_a = lay_s = fp64h = 0
    for i in range(a.steps):
        _, _, irr, _, st = ctx.trace_forward(scene, thk, w.seed, a.warmup + i, prec, stats=True, grad=not fo,
                                             memo=a.memo, table=a.table)
        inter += st["interactions"]
        hits += st["prma_hits"]
        lay_f += st["layer_steps"]
        fp64h += st["fp64_hits"]
        if not fo:
            _, dLdI = ctx.loss(irr, w.loss_kind, w.loss_wf, w.loss_we)
            _, bst = ctx.trace_backward(dLdI, scene, stats=True)
            lay_b += bst["layer_steps"]
            lay_a += bst["adjoint_layer_steps"]
            lay_s += bst["adjoint_stored_layer_steps"]
    progress("step counters recomputed")
    K = a.steps
    if a.graph:
        wall = extra["graph_ms_per_step"] * 1e-3 * K
    value = inter / wall

    if a.per_design:
        # the same batch as one launch per design (64 forward + 64 adjoint launches)
        scenes = []
        for d in range(w.n_designs):
            inp_d = design_slice(inp, d)
            sc_d = gwg.SceneSpec.from_workload(w, inp_d)
            sc_d.first_design = d
            scenes.append((sc_d, torch.tensor(inp_d["thk"], dtype=torch.float64, device=dev)))
        for sc_d, th_d in scenes:
            step(0, sc=sc_d, th=th_d)
        torch.cuda.synchronize()
        progress("per-design warm-up done")
        tp = time.perf_counter()
        for i in range(K):
            for sc_d, th_d in scenes:
                step(a.warmup + i, sc=sc_d, th=th_d)
            torch.cuda.synchronize()
            progress(f"per-design step {i + 1} of {K} done")
        pd_wall = time.perf_counter() - tp
        extra["per_design_ms_per_step"] = pd_wall / K * 1e3
        extra["batched_speedup_vs_per_design"] = pd_wall / wall

    if a.design_chunks:
        # the same batch as a few launches of consecutive designs: the loss is a
        # sum over designs, so chunking by design changes no result
        nc = a.design_chunks if a.design_chunks > 0 else auto_design_chunks(w)
        nc = max(1, min(nc, w.n_designs))
        bounds = [round(i * w.n_designs / nc) for i in range(nc + 1)]
        chunks = []
        for c0, c1 in zip(bounds[:-1], bounds[1:]):
            inp_c = design_slice(inp, c0, c1 - c0)
            sc_c = gwg.SceneSpec.from_workload(w, inp_c)
            sc_c.first_design = c0          # the batch's random streams: the same results
            chunks.append((sc_c, torch.tensor(inp_c["thk"], dtype=torch.float64, device=dev)))
        for sc_c, th_c in chunks:
            step(0, sc=sc_c, th=th_c)
        torch.cuda.synchronize()
        progress("design-chunk warm-up done")
        tp = time.perf_counter()
        for i in range(K):
            for sc_c, th_c in chunks:
                step(a.warmup + i, sc=sc_c, th=th_c)
            torch.cuda.synchronize()
            progress(f"design-chunk step {i + 1} of {K} done")
        ch_wall = time.perf_counter() - tp
        extra["design_chunks"] = nc
        extra["chunked_ms_per_step"] = ch_wall / K * 1e3
        extra["chunked_speedup_vs_single_launch"] = wall / ch_wall
        if a.graph:
            # the whole chunked step in one graph (every chunk's scene was
            # built above, so the capture rebuilds nothing)
            d_step = torch.zeros(1, dtype=torch.int32, device=dev)
            ctx.set_step_source(d_step)
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                for sc_c, th_c in chunks:
                    step(a.warmup + K, sc=sc_c, th=th_c)
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            cgraph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(cgraph):
                for sc_c, th_c in chunks:
                    step(a.warmup + K, sc=sc_c, th=th_c)
                d_step.add_(1)
            torch.cuda.synchronize()
            cgraph.replay()
            torch.cuda.synchronize()
            tg = time.perf_counter()
            for _ in range(K):
                cgraph.replay()
            torch.cuda.synchronize()
            extra["chunked_graph_ms_per_step"] = (time.perf_counter() - tg) / K * 1e3
            progress(f"design-chunk graph replays done: {extra['chunked_graph_ms_per_step']:.1f} ms per step")
            ctx.set_step_source(None)
        if a.per_design:
            extra["chunked_speedup_vs_per_design"] = extra["per_design_ms_per_step"] / extra["chunked_ms_per_step"]

    f_fwd = FLOP_FWD_LAYER * lay_f / K
    f_bwd = (FLOP_FWD_LAYER * lay_b + FLOP_ADJ_LAYER * lay_a - FLOP_FWD_LAYER * lay_s) / K
    t_fwd = float(np.mean(kfwd_ms)) * 1e-3
    t_bwd = float(np.mean(kbwd_ms)) * 1e-3
    # the adjoint launch is the entry kernel (plus the regenerating kernel,
    # which only runs for items whose entry regions overflowed)
    if not fo and t_bwd >= t_fwd:
        kname, flops, tk = ("k_adj_memo" if a.memo else "k_table_adj" if a.table else "k_adj_entries"), f_bwd, t_bwd
    else:
        kname, flops, tk = "k_trace_fwd", f_fwd, t_fwd
    achieved = flops / tk / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64, "traffic": load_traffic(kname, a.workload, a.precision),
            "kernel": kname, "kernel_ms": tk * 1e3}
    extra.update({"interactions_per_step": inter / K, "mirror_hits_per_step": hits / K,
                  "fwd_layer_steps_per_step": lay_f / K, "adj_layer_steps_per_step": lay_a / K,
                  "adj_stored_sweep_layer_steps_per_step": lay_s / K,
                  "mirror_hits_per_s": hits / wall, "fp64_hit_fraction": fp64h / max(hits, 1),
                  "fwd_ms": float(np.mean(fwd_ms)), "loss_ms": float(np.mean(loss_ms)),
                  "bwd_ms": float(np.mean(bwd_ms)), "fwd_kernel_ms": t_fwd * 1e3,
                  "fwd_tflops": f_fwd / t_fwd / 1e12})
    if not fo:
        extra.update({"bwd_kernel_ms": t_bwd * 1e3, "bwd_tflops": f_bwd / t_bwd / 1e12})
    out = {
        "metric": (METRIC + (" (memoized thin film)" if a.memo else " (angle-table thin film)" if a.table else "")
                   + (" (pupil-image objective)" if w.eye_pupil_grid > 0 else ""))
        if not fo else "fwd ray-surface interactions/s",
        "value": value, "unit": UNIT, "n_gpus": 1, "steps": K, "warmup": a.warmup,
        "ms_per_step": wall / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == gwg.FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": a.workload, "designs": w.n_designs, "mirrors": w.n_mirrors,
                   "layers_per_mirror": w.max_layers, "thickness_params": w.n_params,
                   "wavelengths": len(w.lambdas_nm), "fov_points": w.n_fov,
                   "rays_per_point": w.rays_per_point, "rays_per_step": w.n_rays,
                   "bins": list(w.bins), "max_events": w.max_events, "precision": a.precision,
                   "step": "forward" if fo else "forward+loss+adjoint",
                   "thin_film": ("memoized per distinct hit key" if a.memo else
                                 "angle table, Catmull-Rom interpolation" if a.table else "per hit"),
                   "launch": "graph" if a.graph else "eager",
                   "objective": ({"pupils": f"{w.eye_pupil_grid}x{w.eye_pupil_grid}, "
                                            f"{w.eye_pupil_diam_mm:g} mm diameter",
                                  "loss": "Eq. 1 on pupil images (kind 2)", "w_f": w.loss_wf, "w_e": w.loss_we}
                                 if w.eye_pupil_grid > 0 else
                                 {"loss": f"kind {w.loss_kind}", "w_f": w.loss_wf, "w_e": w.loss_we}),
                   "library_source_hash": gwg.source_hash()},
        "roofline": roof,
        "extra": extra,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, inp, a.workload, a.rays_per_point, inter / K / w.n_points,
                                           forward_only=fo, min_interactions=a.cpu_interactions)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
