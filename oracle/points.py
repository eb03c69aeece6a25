"""Timing harness of the oracle on whole (wavelength, FoV) points of a
workload (test infrastructure: the CPU baseline of the benchmark).

Run as `python -m oracle.points '<json>'` with
{"workload": name, "rays_per_point": n (0 = the workload's), "points":
[[lambda_index, fov_index], ...], "forward_only": bool}.  The process builds
one oracle scene per point (a workload holding that point alone), prints
"ready", waits for one line on stdin, then runs the oracle's forward (+ loss
+ adjoint) on every point and prints one JSON line with the seconds spent in
the oracle and the forward interactions it traced.  The barrier lets a
caller start several of these on separate cores and time them together.
"""
import dataclasses
import json
import sys
import time

import numpy as np


def main():
    args = json.loads(sys.argv[1])
    import inputs
    import oracle
    w = inputs.workload(args["workload"])
    if args.get("rays_per_point"):
        w = dataclasses.replace(w, rays_per_point=int(args["rays_per_point"]))
    inp = inputs.make_inputs(w)
    scenes = []
    for li, f in args["points"]:
        sub = dict(inp)
        sub["lambda_sel"] = np.array([li], dtype=np.int32)
        if w.fov_mode == 0:
            sub["fov"] = inp["fov"][f:f + 1].copy()
        scenes.append(oracle.OracleScene(w, sub))
    oracle.lib()
    print("ready", flush=True)
    sys.stdin.readline()
    el = 0.0
    n_int = 0
    for osc in scenes:
        t = time.perf_counter()
        _, _, wsum, st = osc.forward()
        if not args.get("forward_only"):
            _, g = oracle.loss(wsum / osc.s.rays_per_point, w.loss_kind, w.loss_wf, w.loss_we)
            osc.backward(g, 1)
        el += time.perf_counter() - t
        n_int += int(st.counters[1])
    print(json.dumps({"seconds": el, "interactions": n_int}), flush=True)


if __name__ == "__main__":
    main()
