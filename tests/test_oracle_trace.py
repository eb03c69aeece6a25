"""Pins of the oracle's Monte Carlo trace (Methods, "Polarization ray tracing"
and "Differentiable Monte Carlo non-sequential ray tracing").

Pinned against closed-form geometry, exact enumeration of sampled paths,
brute-force deterministic splitting, energy bookkeeping and degenerate stacks.
"""
import dataclasses
import math

import numpy as np
import pytest

import inputs

EV_TIR, EV_EXIT, EV_LEAK, EV_END, EV_MIRROR = 1, 2, 3, 4, 5


def scene(orc, name="plain_fp64", inp_mut=None, **kw):
    w = inputs.small_variant(name, **kw)
    inp = inputs.make_inputs(w)
    if inp_mut:
        inp_mut(inp)
    return orc.OracleScene(w, inp), w, inp


def centre_only(w_kw):
    return dict(fov_mode=0, fov_n=1, **w_kw)


def test_centre_field_angles_of_incidence(orc):
    """Centre field: guided at 2*tilt = 50 deg; until its first mirror
    reflection a ray meets the mirrors at exactly tilt = 25 deg (down-going)
    or 3*tilt = 75 deg (up-going); a back-side reflection at 75 deg turns it
    into a ghost guided at 80 deg."""
    sc, w, inp = scene(orc, "fwd_scale", **centre_only(dict(rays_per_point=200, lambdas_nm=(530.0,))))
    seen = set()
    ghosts = 0
    for rid in range(200):
        ev = sc.events(rid)
        for e in ev:
            if e[0] == EV_MIRROR:
                aoi = e[8]
                assert min(abs(aoi - 25.0), abs(aoi - 75.0)) < 1e-9, aoi
                seen.add(round(aoi))
                if e[9] == 1:
                    if round(aoi) == 75:
                        ghosts += 1
                        assert abs(math.degrees(math.acos(abs(e[7]))) - 80.0) < 1e-9
                    break
        # first event: the injected ray is guided at 50 deg from the face normal
    ev = sc.events(0)
    d0 = ev[0][5:8]
    assert abs(math.degrees(math.acos(abs(d0[2]))) - 50.0) < 1e-9
    assert seen == {25, 75}
    assert ghosts > 0


def test_single_reflection_exits_along_field_direction(orc):
    """With the in-coupler parallel to the mirrors, a ray out-coupled by a
    single mirror reflection leaves the top face along the field direction
    a = normalize(tan tx, tan ty, 1) (mirror reflections commute with TIR)."""
    sc, w, inp = scene(orc, "plain_fp64", rays_per_point=3000)
    ids = np.arange(3000)
    rec = sc.trace_rays(ids)
    key = [(20260101 & 0xFFFFFFFF), (20260101 >> 32)]
    checked = 0
    for r in rec:
        if r.category not in (0, 1):
            continue
        ev = sc.events(r.ray_id)
        n_refl = sum(1 for e in ev if e[0] == EV_MIRROR and e[9] == 1)
        if n_refl != 1:
            continue
        wd = orc.philox([r.ray_id & 0xFFFFFFFF, r.ray_id >> 32, 0, 0], key)
        u = (wd >> 8) / 2.0 ** 24
        tx = math.tan(math.radians(-10 + 20 * u[2]))
        ty = math.tan(math.radians(-10 + 20 * u[3]))
        a = np.array([tx, ty, 1.0]) / math.sqrt(tx * tx + ty * ty + 1)
        assert np.max(np.abs(np.array(r.exit_dir[:]) - a)) < 1e-12
        checked += 1
    assert checked > 500


def test_tir_bounce_positions(orc):
    """Between mirrors the ray zig-zags: successive face hits advance by
    T * |d_xy / d_z| and alternate between z = T and z = 0."""
    sc, w, inp = scene(orc, "fwd_scale", rays_per_point=50, lambdas_nm=(460.0,), fov_n=3)
    for rid in range(0, 9 * 50, 7):
        ev = sc.events(rid)
        pos = np.array([0.5, 0.0, w.T_mm])  # not used for the first (birth on the face)
        for a, b in zip(ev[:-1], ev[1:]):
            if a[0] == EV_TIR and b[0] == EV_TIR:
                d = a[5:8]
                step = w.T_mm / abs(d[2])
                assert abs(b[2] - (a[2] + step * d[0])) < 1e-12
                assert abs(b[3] - (a[3] + step * d[1])) < 1e-12
                assert {a[4], b[4]} == {0.0, w.T_mm}
        del pos


def test_events_lie_on_their_surfaces(orc):
    sc, w, inp = scene(orc, "diff_1200", rays_per_point=20, fov_n=5, lambdas_nm=(620.0,))
    beta = math.radians(w.tilt_deg)
    n = np.array([-math.sin(beta), 0, math.cos(beta)])
    M = w.n_mirrors
    for rid in range(25 * 20):
        for e in sc.events(rid):
            p = e[2:5]
            if e[0] == EV_MIRROR:
                m = int(e[1])
                xm = w.center_x_mm + (m - (M - 1) / 2) * w.pitch_mm
                assert abs(n @ (p - np.array([xm, 0, w.T_mm / 2]))) < 1e-12
                assert -1e-12 <= p[2] <= w.T_mm + 1e-12
            elif e[0] in (EV_TIR, EV_EXIT, EV_LEAK):
                assert p[2] in (0.0, w.T_mm)
                assert 0 <= p[0] <= w.L_mm
            elif e[0] == EV_END:
                assert p[0] in (0.0, w.L_mm)


def _enumerate(sc, rid, B):
    """Exact expectation of the MC weight per bin over all decision sequences."""
    exp = np.zeros(B)
    total_p = 0.0
    stack = [(0, 0)]
    while stack:
        bits, n = stack.pop()
        b, wmc, p, used = sc.forced(rid, bits, n)
        if used > n:
            stack.append((bits, n + 1))
            stack.append((bits | (1 << n), n + 1))
            continue
        total_p += p
        if b >= 0:
            exp[b] += p * wmc
    return exp, total_p


def _toy(**kw):
    base = dict(n_mirrors=2, n_layers=6, L_mm=18.0, center_x_mm=9.0, rays_per_point=60,
                lambdas_nm=(530.0,), fov_n=3, fov_half_deg=8.0, max_events=40, bins=(6, 6))
    base.update(kw)
    return base


def test_sampled_paths_are_unbiased_exactly(orc):
    """Eq. 6 rescaling: sum over decision sequences of P(path) * w_MC(path)
    equals the unsampled split sum of |E_path|^2 for every birth and bin."""
    sc, w, inp = scene(orc, "fwd_scale", **_toy())
    B = w.bins[0] * w.bins[1]
    for rid in range(0, 9 * 60, 13):
        d, rem = divmod(rid, 9 * 60)
        f, i = divmod(rem, 60)
        exp, tp = _enumerate(sc, rid, B)
        assert abs(tp - 1.0) < 1e-12
        split, npaths = sc.split(0, 0, f, 1, first=i)
        assert np.max(np.abs(exp - split)) < 1e-12 * max(1.0, split.max())


def test_mc_matches_bruteforce_splitting(orc):
    """Two-mirror toy waveguide: MC bin estimates agree with deterministic
    splitting within 5 standard errors."""
    sc, w, inp = scene(orc, "fwd_scale", **_toy(rays_per_point=4000, fov_n=1))
    B = w.bins[0] * w.bins[1]
    N = w.rays_per_point
    rec = sc.trace_rays(np.arange(N))
    mc = np.zeros((N, B))
    for k, r in enumerate(rec):
        if r.bin >= 0:
            mc[k, r.bin] = r.w
    # per-birth exact expectation
    ex = np.zeros((N, B))
    for i in range(N):
        ex[i], _ = sc.split(0, 0, 0, 1, first=i)
    diff = (mc - ex).sum(0)
    se = np.sqrt(((mc - ex) ** 2).sum(0))
    active = ex.sum(0) > 1e-3
    assert active.sum() >= 4
    z = np.abs(diff[active]) / np.maximum(se[active], 1e-12)
    assert np.all(z < 5.0), z
    # and the estimator is not trivially equal to the expectation
    assert np.max(se) > 1e-3


def test_energy_bookkeeping(orc):
    """Lossless stacks: summed tallies of every termination category (eyebox,
    missed, leaked, absorbed at the ends, truncated, dropped face reflection)
    average to the injected power 1 per ray."""
    sc, w, inp = scene(orc, "fwd_scale", rays_per_point=2000, fov_n=3, lambdas_nm=(530.0,))
    N = 9 * 2000
    rec = sc.trace_rays(np.arange(N))
    q, c, ws, st = sc.forward()
    tot = sum(st.power[k] for k in range(8))
    assert st.counters[0] == N
    mean = tot / N
    assert abs(mean - 1.0) < 0.05
    # per-ray final weights (every category but the dropped face reflection)
    per = np.array([r.w for r in rec])
    cats = np.array([r.category for r in rec])
    for k in range(6):
        assert abs(per[cats == k].sum() - st.power[k]) <= 1e-9 * max(1.0, st.power[k])
    se = per.std() / math.sqrt(N)
    assert abs(mean - 1.0) < 5 * se + 1e-3
    assert st.power[0] > 0 and st.power[6] > 0


def test_zero_stacks_are_invisible(orc):
    """All-zero-thickness stacks are bare glass/glass interfaces (r = 0,
    t = 1): nothing is out-coupled, and the Eq. 6 weights of the rays that
    transmit to the far end face average to the injected power."""
    def zero(inp):
        inp["thk"][:] = 0.0
    w = inputs.small_variant("plain_fp64", rays_per_point=4000, fov_half_deg=5.0)
    inp = inputs.make_inputs(w)
    zero(inp)
    sc = orc.OracleScene(w, inp, omega=np.full(w.n_mirrors, 0.1))
    q, c, ws, st = sc.forward()
    # reflected rays still land (the counts are pure geometry) but carry w ~ 0
    assert q.sum() == 0 and ws.sum() < 1e-20 and c.sum() > 0
    rec = sc.trace_rays(np.arange(4000))
    w_end = np.array([r.w if r.category == 3 else 0.0 for r in rec])
    assert all(r.w < 1e-25 for r in rec if r.category == 0)
    assert np.count_nonzero(w_end) > 0.5 * 4000
    se = w_end.std() / math.sqrt(len(w_end))
    assert abs(w_end.mean() - 1.0) < 5 * se


def test_zero_thickness_layers_do_not_change_bins(orc):
    def pad(inp):
        th, mt = inp["thk"], inp["mat"]
        inp["thk"] = np.concatenate([th, np.zeros(th.shape[:2] + (3,))], axis=2)
        inp["mat"] = np.concatenate([mt, np.full(mt.shape[:2] + (3,), 3, np.uint8)], axis=2)
        # the padded zero layers sit at the end of the listed layers
        inp["n_layers"] = inp["n_layers"] + 3
    sc0, w, _ = scene(orc, "plain_fp64", rays_per_point=3000)
    sc1, _, _ = scene(orc, "plain_fp64", inp_mut=pad, rays_per_point=3000)
    q0, c0, ws0, _ = sc0.forward()
    q1, c1, ws1, _ = sc1.forward()
    assert np.array_equal(c0, c1)
    assert np.max(np.abs(ws0 - ws1)) < 1e-12 * ws0.max()


def test_reproducible_and_step_dependent(orc):
    sc, w, inp = scene(orc, "plain_fp64", rays_per_point=2000)
    a = sc.forward()
    b = sc.forward()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    sc2 = orc.OracleScene(w, inp, step=1)
    c = sc2.forward()
    assert not np.array_equal(a[1], c[1])


def test_fixed_point_bins_round_half_even(orc):
    """Q = sum of rne(w 2^S): identical to the per-ray records re-quantised."""
    sc, w, inp = scene(orc, "plain_fp64", rays_per_point=5000)
    q, c, ws, st = sc.forward()
    rec = sc.trace_rays(np.arange(5000))
    Q = np.zeros(100, dtype=np.uint64)
    for r in rec:
        if r.bin >= 0:
            Q[r.bin] += np.uint64(np.rint(r.w * 2.0 ** 24))
    assert np.array_equal(Q, q.reshape(-1))


def test_first_design_selects_the_batch_streams(orc):
    """Designs traced on their own with first_design set draw the streams
    they draw inside the whole batch: bins, counts and weights equal that
    batch's slice (a batch traced in chunks of designs is the same batch)."""
    w = inputs.small_variant("batched", n_designs=3, rays_per_point=60, fov_n=3, lambdas_nm=(450.0, 600.0))
    inp = inputs.make_inputs(w)
    q, c, ws, _ = orc.OracleScene(w, inp).forward()
    for d0, n in ((1, 2), (2, 1)):
        sub = dict(inp)
        for k in ("thk", "mat", "n_layers"):
            sub[k] = inp[k][d0:d0 + n].copy()
        qs, cs, wss, _ = orc.OracleScene(w, sub, first_design=d0).forward()
        assert np.array_equal(qs, q[d0:d0 + n]) and np.array_equal(cs, c[d0:d0 + n])
        assert np.array_equal(wss, ws[d0:d0 + n])
        q0, _, _, _ = orc.OracleScene(w, sub).forward()      # without it: other streams
        assert not np.array_equal(q0, q[d0:d0 + n])
