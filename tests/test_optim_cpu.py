"""Host logic of the coating optimiser (paper_2601_04370_amd.optim): the
soft-gap penalty, projection and snapping of thicknesses, the Gaussian
initialisation, and the Eq. 1 metrics pinned against the oracle's loss."""
import numpy as np
import torch

import inputs
from paper_2601_04370_amd import optim


def test_gap_penalty_values_and_derivative():
    t_min = 20.0
    t = torch.tensor([0.0, 5.0, 10.0, 15.0, 20.0, 50.0, 200.0], dtype=torch.float64)
    phi, dphi = optim.gap_penalty(t, t_min)
    assert torch.allclose(phi, torch.tensor([0.0, 0.1875, 0.25, 0.1875, 0.0, 0.0, 0.0], dtype=torch.float64))
    # central differences inside the gap
    for x in (1.0, 7.5, 12.0, 19.0):
        h = 1e-6
        fp = optim.gap_penalty(torch.tensor([x + h], dtype=torch.float64), t_min)[0]
        fm = optim.gap_penalty(torch.tensor([x - h], dtype=torch.float64), t_min)[0]
        d = optim.gap_penalty(torch.tensor([x], dtype=torch.float64), t_min)[1]
        assert abs(float((fp - fm) / (2 * h)) - float(d)) < 1e-7
    assert float(dphi[0]) == 0.0 and float(dphi[4]) == 0.0


def test_snap_and_project():
    t = torch.tensor([-3.0, 0.0, 5.0, 9.999, 10.0, 15.0, 20.0, 150.0, 250.0], dtype=torch.float64)
    mask = torch.ones_like(t)
    mask[-1] = 0.0
    p = optim.project(t, 200.0, mask)
    assert p.tolist() == [0.0, 0.0, 5.0, 9.999, 10.0, 15.0, 20.0, 150.0, 0.0]
    s = optim.snap(p, 20.0)
    assert s.tolist() == [0.0, 0.0, 0.0, 0.0, 20.0, 20.0, 20.0, 150.0, 0.0]


def test_init_thicknesses():
    nl = np.array([[200, 150, 3], [10, 0, 200]], dtype=np.int32)
    thk = optim.init_thicknesses(nl, 200, 20.0, 200.0, seed=3)
    for d in range(2):
        for m in range(3):
            assert np.all(thk[d, m, nl[d, m]:] == 0.0)
            real = thk[d, m, : nl[d, m]]
            assert np.all((real >= 20.0) & (real <= 200.0))
    real = np.concatenate([thk[d, m, : nl[d, m]] for d in range(2) for m in range(3)])
    assert abs(real.mean() - 110.0) < 3.0


def test_metrics_match_oracle_loss(orc):
    rng = np.random.default_rng(7)
    for D in (1, 3):
        irr = rng.uniform(0.0, 1e-3, size=(D, 2, 5, 4, 4))
        m = [optim.metrics(torch.tensor(irr[d:d + 1])) for d in range(D)]
        L, _ = orc.loss(irr, 1, 10.0, 3.0)
        mine = sum(-x["ibar"] + 10.0 * x["cv_fov"] + 3.0 * x["cv_eyebox"] for x in m)
        assert abs(mine - L) < 1e-12 * max(1.0, abs(L))
        avg = optim.metrics(torch.tensor(irr))
        for key in ("ibar", "cv_fov", "cv_eyebox"):
            assert abs(avg[key] - np.mean([x[key] for x in m])) < 1e-14


def test_pupil_metrics_match_oracle_loss(orc):
    """With eye pupils the metrics are Eq. 1's pupil form (loss kind 2)."""
    rng = np.random.default_rng(8)
    irr = rng.uniform(0.0, 0.02, size=(2, 9, 5, 1, 9))
    m = [optim.metrics(torch.tensor(irr[d:d + 1]), pupils=True) for d in range(2)]
    L, _ = orc.loss(irr, 2, 10.0, 3.0)
    mine = sum(-x["ibar"] + 10.0 * x["cv_fov"] + 3.0 * x["cv_eyebox"] for x in m)
    assert abs(mine - L) < 1e-12 * max(1.0, abs(L))
