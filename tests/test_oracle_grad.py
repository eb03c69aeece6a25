"""Pins of the oracle's adjoint (gradient of the eyebox loss with respect to
every layer thickness) against same-seed central finite differences.

The reflect/transmit choice depends only on the random word and the mirror's
probability (Methods, reparameterization), so a thickness perturbation never
changes a path and central differences of the sampled estimator converge as
O(h^2) to the pathwise derivative that the adjoint computes.
"""
import numpy as np
import pytest

import inputs


def _setup(orc, name, **kw):
    w = inputs.small_variant(name, **kw)
    inp = inputs.make_inputs(w)
    return w, inp


def _loss_of(orc, w, inp, thk, kind, wf, we, stride):
    sc = orc.OracleScene(w, inp, thk=thk)
    irr = sc.forward_sampled(stride)
    return orc.loss(irr, kind, wf, we)


@pytest.mark.parametrize("name,kw,kind,stride", [
    ("plain_fp64", dict(rays_per_point=3000), 1, 1),
    ("diff_1200", dict(rays_per_point=48, fov_n=3), 0, 1),
    ("precision_ag", dict(rays_per_point=96, fov_n=3), 0, 2),
])
def test_adjoint_matches_central_fd(orc, name, kw, kind, stride):
    w, inp = _setup(orc, name, **kw)
    thk = inp["thk"].copy()
    wf, we = (10.0, 3.0) if kind == 1 else (1.0, 1.0)
    L0, dLdI = _loss_of(orc, w, inp, thk, kind, wf, we, stride)
    sc = orc.OracleScene(w, inp, thk=thk)
    g = sc.backward(dLdI, stride)
    assert np.all(np.isfinite(g))
    rng = np.random.default_rng(w.seed)
    flat = rng.choice(thk.size, size=16, replace=False)
    h = 1e-3
    gmax = np.max(np.abs(g))
    assert gmax > 0
    for idx in flat:
        tp, tm = thk.copy().reshape(-1), thk.copy().reshape(-1)
        tp[idx] += h
        tm[idx] -= h
        Lp, _ = _loss_of(orc, w, inp, tp.reshape(thk.shape), kind, wf, we, stride)
        Lm, _ = _loss_of(orc, w, inp, tm.reshape(thk.shape), kind, wf, we, stride)
        fd = (Lp - Lm) / (2 * h)
        ad = g.reshape(-1)[idx]
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-7 * gmax, (idx, fd, ad)


def test_directional_derivative_all_parameters(orc):
    w, inp = _setup(orc, "diff_1200", rays_per_point=32, fov_n=3, lambdas_nm=(530.0,))
    thk = inp["thk"].copy()
    L0, dLdI = _loss_of(orc, w, inp, thk, 0, 1.0, 1.0, 1)
    g = orc.OracleScene(w, inp, thk=thk).backward(dLdI, 1)
    v = np.random.default_rng(3).standard_normal(thk.shape)
    h = 1e-4
    Lp, _ = _loss_of(orc, w, inp, thk + h * v, 0, 1.0, 1.0, 1)
    Lm, _ = _loss_of(orc, w, inp, thk - h * v, 0, 1.0, 1.0, 1)
    fd = (Lp - Lm) / (2 * h)
    ad = float((g * v).sum())
    assert abs(fd - ad) <= 1e-6 * abs(ad)


def test_padding_slots_have_zero_gradient(orc):
    """Slots beyond a mirror's layer count are not layers: zero gradient."""
    w, inp = _setup(orc, "batched", n_designs=2, rays_per_point=16, fov_n=3,
                    lambdas_nm=(450.0, 600.0))
    irr = orc.OracleScene(w, inp).forward_sampled(1)
    L, dLdI = orc.loss(irr, 0)
    g = orc.OracleScene(w, inp).backward(dLdI, 1)
    for d in range(2):
        for m in range(w.n_mirrors):
            nl = inp["n_layers"][d, m]
            assert np.all(g[d, m, nl:] == 0.0)
    assert np.count_nonzero(g) > 0


def test_gradient_is_linear_in_dLdI(orc):
    w, inp = _setup(orc, "plain_fp64", rays_per_point=2000)
    sc = orc.OracleScene(w, inp)
    sh = sc.shape
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal(sh), rng.standard_normal(sh)
    ga, gb = sc.backward(a), sc.backward(b)
    gab = sc.backward(2.0 * a - 0.5 * b)
    assert np.max(np.abs(gab - (2.0 * ga - 0.5 * gb))) < 1e-12 * np.max(np.abs(gab))
    # a one-hot dL/dI gives the derivative of that bin's irradiance
    one = np.zeros(sh)
    flat_irr = sc.forward_sampled(1).reshape(-1)
    k = int(np.argmax(flat_irr))
    one.reshape(-1)[k] = 1.0
    g1 = sc.backward(one)
    h = 1e-3
    th = inp["thk"]
    j = (0, 1, 3)
    tp, tm = th.copy(), th.copy()
    tp[j] += h
    tm[j] -= h
    fd = (orc.OracleScene(w, inp, thk=tp).forward_sampled(1).reshape(-1)[k]
          - orc.OracleScene(w, inp, thk=tm).forward_sampled(1).reshape(-1)[k]) / (2 * h)
    assert abs(fd - g1[j]) <= 1e-6 * abs(g1[j]) + 1e-12
