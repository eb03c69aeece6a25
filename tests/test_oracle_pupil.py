"""Pins of the oracle's pupil-image objective (Results, "System
Architecture": a 3 x 3 grid of pupil positions in the eyebox, three
wavelengths per colour channel, the pupil images as the objective; Eq. 1 on
them).

- Aperture membership by brute force: from every ray's own exit position and
  direction the test finds its crossing of the eyebox plane and the pupil
  containing it, and sums the rays' weights per (point, pupil); the oracle's
  pupil images must equal these sums.
- Pupils that tile the eyebox: pupils whose discs cover the whole eyebox
  rectangle partition it into cells (each ray is given to the first disc that
  holds it), so their images add up to the image of a single aperture
  covering the eyebox, ray for ray.
- The pupil form of Eq. 1 (loss kind 2): closed forms, its relation to the
  eyebox form, and central differences.
- The gradient through the trace with the pupil loss against same-seed
  central differences of the whole estimator.
"""
import dataclasses

import numpy as np
import pytest

import inputs


def _scene(orc, **kw):
    w = inputs.small_variant("pupil_rgb", **kw)
    inp = inputs.make_inputs(w)
    return orc.OracleScene(w, inp), w, inp


def test_workload_pupils_follow_the_paper():
    w = inputs.workload("pupil_rgb")
    # three wavelengths per colour channel: blue, green, red
    assert w.lambdas_nm == (450.0, 470.0, 490.0, 500.0, 530.0, 560.0, 620.0, 660.0, 700.0)
    inp = inputs.make_inputs(w)
    xy = inp["eye_pupils"]
    assert xy.shape == (9, 2) and w.bins == (9, 1)
    ex0, ey0, ew, eh = inp["eyebox"]
    # a 3 x 3 grid of pupil positions inside the eyebox, not overlapping
    assert np.all((xy[:, 0] > ex0) & (xy[:, 0] < ex0 + ew) & (xy[:, 1] > ey0) & (xy[:, 1] < ey0 + eh))
    d = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1)) + np.eye(9) * 1e9
    assert d.min() >= 2 * inp["eye_pupil_r"]


def _brute_force_images(sc, w, inp, n_rays):
    """Per-point pupil sums from each ray's exit position and direction."""
    rec = sc.trace_rays(np.arange(n_rays))
    xy = inp["eye_pupils"]
    r2 = inp["eye_pupil_r"] * inp["eye_pupil_r"]
    P = np.zeros((n_rays // w.rays_per_point, xy.shape[0]))
    C = np.zeros_like(P, dtype=np.int64)
    for r in rec:
        if r.category not in (0, 1):     # binned or missed: left the top face
            continue
        px, py = r.exit_pos[0], r.exit_pos[1]
        ax, ay, az = r.exit_dir[0], r.exit_dir[1], r.exit_dir[2]
        xe = px + w.eye_relief_mm * (ax / az)
        ye = py + w.eye_relief_mm * (ay / az)
        hit = -1
        for q in range(xy.shape[0]):
            dx, dy = xe - xy[q, 0], ye - xy[q, 1]
            if dx * dx + dy * dy < r2:
                hit = q
                break
        assert (hit >= 0) == (r.category == 0) and r.bin == hit
        if hit >= 0:
            pt = r.ray_id // w.rays_per_point
            P[pt, hit] += r.w
            C[pt, hit] += 1
    return P, C


def test_pupil_images_by_brute_force(orc):
    sc, w, inp = _scene(orc, rays_per_point=600, fov_n=3, lambdas_nm=(470.0, 530.0, 660.0))
    q, c, ws, st = sc.forward()
    P, C = _brute_force_images(sc, w, inp, w.n_rays)
    assert np.array_equal(c.reshape(P.shape), C)
    assert np.max(np.abs(ws.reshape(P.shape) - P)) <= 1e-14 * max(1.0, P.max())
    assert C.sum() > 200 and np.count_nonzero(C) >= 9


def _with_pupils(w, inp, xy, r):
    inp = dict(inp)
    inp["eye_pupils"] = np.asarray(xy, dtype=np.float64)
    inp["eye_pupil_r"] = r
    return dataclasses.replace(w, bins=(len(xy), 1)), inp


def test_pupils_tiling_the_eyebox_sum_to_the_whole(orc):
    """Nine discs centred on a 3 x 3 partition of the eyebox with the cell's
    half diagonal as radius cover the eyebox; each ray goes to the first disc
    holding it, so the discs act as nine apertures that tile their union.
    Their images, summed, equal the image of one disc covering that union:
    every ray is counted once, none is lost."""
    sc, w, inp = _scene(orc, rays_per_point=800, fov_n=3, lambdas_nm=(530.0,))
    ex0, ey0, ew, eh = inp["eyebox"]
    cells = w.eye_pupils
    r_cell = 0.5 * np.hypot(ew / 3, eh / 3)
    w9, inp9 = _with_pupils(w, inp, cells, r_cell)
    big = np.hypot(ew, eh)                # holds every disc of the nine
    w1, inp1 = _with_pupils(w, inp, [[ex0 + ew / 2, ey0 + eh / 2]], big)
    q9, c9, s9, _ = orc.OracleScene(w9, inp9).forward()
    q1, c1, s1, _ = orc.OracleScene(w1, inp1).forward()
    # each ray lands in at most one of the nine, and in the big disc if in any
    assert np.all(c9.sum(-1) <= c1.sum(-1))
    P9, C9 = _brute_force_images(orc.OracleScene(w9, inp9), w9, inp9, w.n_rays)
    rec = orc.OracleScene(w1, inp1).trace_rays(np.arange(w.n_rays))
    union = np.zeros(P9.shape[0])
    n_union = np.zeros(P9.shape[0], dtype=np.int64)
    for r in rec:
        if r.category not in (0, 1):
            continue
        xe = r.exit_pos[0] + w.eye_relief_mm * (r.exit_dir[0] / r.exit_dir[2])
        ye = r.exit_pos[1] + w.eye_relief_mm * (r.exit_dir[1] / r.exit_dir[2])
        if any((xe - x) ** 2 + (ye - y) ** 2 < r_cell ** 2 for x, y in cells):
            union[r.ray_id // w.rays_per_point] += r.w
            n_union[r.ray_id // w.rays_per_point] += 1
    assert np.array_equal(C9.sum(-1), n_union)
    assert np.allclose(P9.sum(-1), union, rtol=1e-13, atol=0)
    assert np.allclose(s9.reshape(P9.shape).sum(-1), union, rtol=1e-13, atol=0)
    # and the eyebox rectangle lies inside the union: every ray binned in the
    # 1 x 1 eyebox is in one of the nine discs
    wb = dataclasses.replace(w, bins=(1, 1), eye_pupil_grid=0)
    inpb = dict(inp)
    inpb.pop("eye_pupils")
    inpb.pop("eye_pupil_r")
    _, cb, sb, _ = orc.OracleScene(wb, inpb).forward()
    assert np.all(cb.reshape(-1) <= c9.sum(-1).reshape(-1))
    assert np.all(sb.reshape(-1) <= s9.sum(-1).reshape(-1) * (1 + 1e-13))


def test_pupil_loss_closed_forms(orc):
    D, nl, F, B = 1, 9, 5, 9
    # identical images: both CVs vanish (up to the rounding of the means),
    # L = -mean I (the CV's derivative is singular there, so only L is checked)
    I = np.full((D, nl, F, 1, B), 0.02)
    L, g = orc.loss(I, 2, 10.0, 3.0)
    assert abs(L + 0.02) < 1e-13
    # a variance-form loss of the same images has the plain brightness gradient
    L0, g0 = orc.loss(I, 0, 1.0, 1.0)
    assert np.allclose(g0, -1.0 / (nl * F), rtol=1e-12, atol=1e-18)
    # relation to the eyebox form: the same CV terms, brightness divided by B
    rng = np.random.default_rng(4)
    I = rng.uniform(0.0, 0.05, size=(2, nl, F, 1, B))
    L1, g1 = orc.loss(I, 1, 10.0, 3.0)
    L2, g2 = orc.loss(I, 2, 10.0, 3.0)
    ibar = I.sum(-1).sum(-1).mean(axis=(1, 2))      # mean over points of sum over pupils, per design
    assert abs((L2 - L1) - (ibar.sum() - ibar.sum() / B)) < 1e-13
    assert np.allclose(g2 - g1, (1.0 - 1.0 / B) / (nl * F), rtol=1e-12, atol=1e-15)
    # CV_eyebox alone: one pupil twice as bright as the rest, w_f = 0
    I = np.full((1, nl, F, 1, B), 0.01)
    I[..., 4] = 0.02
    L, _ = orc.loss(I, 2, 0.0, 1.0)
    Ep = np.full(B, 0.01)
    Ep[4] = 0.02
    cv = Ep.std() / Ep.mean()
    assert abs(L - (-I.mean() + cv)) < 1e-14


def test_pupil_loss_central_differences(orc):
    rng = np.random.default_rng(9)
    I = rng.uniform(0.001, 0.05, size=(1, 9, 4, 1, 9))
    L, g = orc.loss(I, 2, 10.0, 3.0)
    h = 1e-7
    for k in rng.choice(I.size, size=12, replace=False):
        Ip, Im = I.copy().reshape(-1), I.copy().reshape(-1)
        Ip[k] += h
        Im[k] -= h
        fd = (orc.loss(Ip.reshape(I.shape), 2, 10.0, 3.0)[0] - orc.loss(Im.reshape(I.shape), 2, 10.0, 3.0)[0]) / (2 * h)
        assert abs(fd - g.reshape(-1)[k]) <= 1e-6 * abs(g.reshape(-1)[k]) + 1e-9


def test_pupil_gradient_matches_central_fd(orc):
    """dL/d(thickness) through the trace with the pupil loss, against same-seed
    central differences of the whole estimator."""
    w = inputs.small_variant("pupil_rgb", rays_per_point=64, fov_n=3, lambdas_nm=(470.0, 530.0, 660.0))
    inp = inputs.make_inputs(w)
    thk = inp["thk"].copy()

    def loss_of(t):
        irr = orc.OracleScene(w, inp, thk=t).forward_sampled(1)
        return orc.loss(irr, 2, 10.0, 3.0)

    L0, dLdI = loss_of(thk)
    g = orc.OracleScene(w, inp, thk=thk).backward(dLdI, 1)
    gmax = np.max(np.abs(g))
    assert gmax > 0
    rng = np.random.default_rng(w.seed)
    h = 1e-3
    for idx in rng.choice(thk.size, size=10, replace=False):
        tp, tm = thk.copy().reshape(-1), thk.copy().reshape(-1)
        tp[idx] += h
        tm[idx] -= h
        fd = (loss_of(tp.reshape(thk.shape))[0] - loss_of(tm.reshape(thk.shape))[0]) / (2 * h)
        ad = g.reshape(-1)[idx]
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-7 * gmax, (idx, fd, ad)
