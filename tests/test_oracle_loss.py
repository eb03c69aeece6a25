"""Pins of the oracle's eyebox loss (Eq. 1 and the variance form) and of its
gradient with respect to the irradiance."""
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _brute(I, kind, wf, we):
    """The loss written directly with numpy reductions (population moments)."""
    total = 0.0
    for Id in I:
        nl, F = Id.shape[:2]
        Ib = Id.reshape(nl, F, -1)
        eta = Ib.sum(2)
        ibar = eta.mean()
        E = Ib.mean((0, 1))
        phi = eta.mean(0)
        if kind == 0:
            total += -ibar + we * E.var() + wf * phi.var()
        else:
            total += -ibar + wf * phi.std() / phi.mean() + we * E.std() / E.mean()
    return total


@pytest.mark.parametrize("kind", [0, 1])
def test_loss_value_and_gradient(orc, kind):
    rng = np.random.default_rng(kind)
    I = rng.uniform(0.0, 1e-3, size=(2, 3, 5, 4, 4))
    wf, we = (10.0, 3.0) if kind else (1.0, 1.0)
    L, g = orc.loss(I, kind, wf, we)
    assert abs(L - _brute(I, kind, wf, we)) < 1e-14
    h = 1e-9
    for _ in range(40):
        idx = tuple(rng.integers(0, s) for s in I.shape)
        Ip, Im = I.copy(), I.copy()
        Ip[idx] += h
        Im[idx] -= h
        fd = (orc.loss(Ip, kind, wf, we)[0] - orc.loss(Im, kind, wf, we)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-6 * max(1.0, abs(g[idx]))


def test_uniform_irradiance(orc):
    """Uniform over bins, FoV and wavelength: no non-uniformity penalty, and
    the loss is minus the throughput per point."""
    I = np.full((1, 3, 9, 4, 4), 2e-3)
    for kind in (0, 1):
        L, g = orc.loss(I, kind, 10.0, 3.0)
        assert abs(L + 16 * 2e-3) < 1e-12
        if kind == 0:
            assert np.allclose(g, -1.0 / 27, rtol=0, atol=1e-14)


def test_cv_is_scale_invariant(orc):
    rng = np.random.default_rng(9)
    I = rng.uniform(0, 1, size=(1, 2, 6, 3, 3))
    L1, _ = orc.loss(I, 1, 10.0, 3.0)
    L2, _ = orc.loss(5.0 * I, 1, 10.0, 3.0)
    eta = I.sum((3, 4)).mean()
    # only the brightness term scales
    assert abs((L2 + 5 * eta) - (L1 + eta)) < 1e-12


def test_paper_weights(orc):
    with open(os.path.join(HERE, "golden", "paper_constants.json")) as f:
        pc = json.load(f)
    assert pc["loss_weights"] == {"w_f": 10.0, "w_e": 3.0}
