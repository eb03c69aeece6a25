"""Pins of the oracle's angle-table thin film (Methods, memory-saving
strategies: the response is precomputed on a discrete set of incidence
angles and interpolated differentiably in between).

Reading: n angles uniform in [0, pi/2], a Catmull-Rom cubic in the angle
through the four surrounding angles, the response taken as even in the
angle below theta_0 and the last segment clamped.  Pins:
  - the interpolant: weights sum to one, reproduce the table at the angles
    themselves, and reproduce quadratics exactly (a property of the
    Catmull-Rom cubic: its central-difference slopes are exact for them);
  - the table trace converges to the exact per-hit trace as the table
    refines, at the cubic's third-order rate on a smooth 8-layer stack;
  - the table adjoint is the derivative of the table forward: same-seed
    central finite differences.
"""
import math

import numpy as np
import pytest

import inputs


def test_weights_partition_of_unity_and_nodes(orc):
    n = 37
    h = (math.pi / 2) / (n - 1)
    for theta in np.linspace(0.0, math.pi / 2, 211):
        idx, w = orc.table_weights(theta, n)
        assert abs(w.sum() - 1.0) < 1e-14
        assert np.all((idx >= 0) & (idx < n))
    for j in range(n - 1):
        idx, w = orc.table_weights(j * h, n)
        # at a table angle the interpolant returns that angle's entry
        val = np.zeros(n)
        np.add.at(val, idx, w)
        expect = np.zeros(n)
        expect[j] = 1.0
        assert np.allclose(val, expect, atol=1e-13), j


def _interp(orc, f, theta, n):
    h = (math.pi / 2) / (n - 1)
    idx, w = orc.table_weights(theta, n)
    return float(sum(wi * f(i * h) for i, wi in zip(idx, w)))


def test_weights_reproduce_quadratics(orc):
    n = 50
    h = (math.pi / 2) / (n - 1)
    rng = np.random.default_rng(1)
    a, b, c = rng.standard_normal(3)
    # a general quadratic away from both ends
    for theta in rng.uniform(h, math.pi / 2 - 2 * h, 200):
        f = lambda x: a + b * x + c * x * x
        assert abs(_interp(orc, f, theta, n) - f(theta)) < 1e-12 * (1 + abs(f(theta)))
    # an even quadratic also in the first segment (mirrored angle)
    for theta in rng.uniform(0.0, h, 50):
        f = lambda x: a + c * x * x
        assert abs(_interp(orc, f, theta, n) - f(theta)) < 1e-12 * (1 + abs(f(theta)))
    # a cubic is not reproduced (the slopes are only second-order)
    f = lambda x: x ** 3
    errs = [abs(_interp(orc, f, t, n) - f(t)) for t in rng.uniform(h, 1.0, 20)]
    assert max(errs) > 1e-9


def _rays(orc, w, inp, n_tab, ids):
    sc = orc.OracleScene(w, inp, table_nodes=n_tab)
    return np.array([r.w for r in sc.trace_rays(ids)])


def test_table_trace_converges_to_exact(orc):
    w = inputs.small_variant("plain_fp64", rays_per_point=400)
    inp = inputs.make_inputs(w)
    ids = np.arange(0, 400, 3)
    exact = _rays(orc, w, inp, 0, ids)
    errs = []
    for n in (64, 128, 256, 512):
        errs.append(np.max(np.abs(_rays(orc, w, inp, n, ids) - exact)))
    print("table error by n", errs)
    assert errs[-1] < 5e-6 * max(1.0, exact.max())
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < e0 / 5.0          # third order: about 8x per halving


@pytest.mark.parametrize("name,kw,n_tab", [
    ("plain_fp64", dict(rays_per_point=1500), 64),
    ("diff_1200", dict(rays_per_point=40, fov_n=3, lambdas_nm=(530.0,)), 2048),
])
def test_table_adjoint_matches_central_fd(orc, name, kw, n_tab):
    w = inputs.small_variant(name, **kw)
    inp = inputs.make_inputs(w)
    thk = inp["thk"].copy()

    def loss(t):
        irr = orc.OracleScene(w, inp, thk=t, table_nodes=n_tab).forward_sampled(1)
        return orc.loss(irr, 0)

    L0, dLdI = loss(thk)
    g = orc.OracleScene(w, inp, thk=thk, table_nodes=n_tab).backward(dLdI, 1)
    gmax = np.max(np.abs(g))
    assert gmax > 0 and np.all(np.isfinite(g))
    rng = np.random.default_rng(w.seed)
    h = 1e-3
    for idx in rng.choice(thk.size, size=8, replace=False):
        tp, tm = thk.copy().reshape(-1), thk.copy().reshape(-1)
        tp[idx] += h
        tm[idx] -= h
        fd = (loss(tp.reshape(thk.shape))[0] - loss(tm.reshape(thk.shape))[0]) / (2 * h)
        ad = g.reshape(-1)[idx]
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-7 * gmax, (idx, fd, ad)
