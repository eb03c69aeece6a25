"""Pins of the oracle's learned-reflection-probability estimator (Methods,
learned reflection probabilities): with every coating a scalar reflectance
equal to omega, the score-function estimate of dJ/domega (J = sum_b W I) is
unbiased.  The exact J for the same births comes from enumerating every
reflect/transmit sequence with forced traces (a polynomial in the sampling
probabilities), and its central differences must agree with the estimator
within its Monte Carlo error."""
import numpy as np
import pytest

import inputs


def _exact_derivative(orc, w, inp, W, ids, h=1e-3):
    om = np.asarray(inp["omega"], dtype=np.float64)
    out = np.zeros(len(om))
    for m in range(len(om)):
        up, dn = om.copy(), om.copy()
        up[m] += h
        dn[m] -= h
        Jp = orc.scalar_expectation(orc.OracleScene(w, inp, omega=up), W, ids)
        Jm = orc.scalar_expectation(orc.OracleScene(w, inp, omega=dn), W, ids)
        out[m] = (Jp - Jm) / (orc.p_eff(up)[m] - orc.p_eff(dn)[m])
    return out


@pytest.mark.parametrize("weights", ["throughput", "random"])
def test_score_gradient_is_unbiased(orc, weights):
    w = inputs.small_variant("plain_fp64", rays_per_point=3000)
    inp = inputs.make_inputs(w)
    osc = orc.OracleScene(w, inp)
    shape = osc.shape
    W = np.ones(shape) if weights == "throughput" else np.random.default_rng(4).uniform(0.0, 2.0, shape)
    _, counts, _, _ = osc.forward()
    ids = np.arange(w.rays_per_point)
    g, contrib = orc.omega_score_gradient(osc, W, counts)
    sigma = contrib.std(axis=0) * np.sqrt(len(ids))
    exact = _exact_derivative(orc, w, inp, W, ids)
    print("estimate", g, "exact", exact, "sigma", sigma)
    assert np.all(np.abs(g - exact) <= 5.0 * sigma + 1e-12)
    assert np.all(sigma < 0.5 * np.abs(exact) + 0.05)   # the test has resolving power


def test_exact_expectation_matches_sampling(orc):
    """The enumerated expectation and the sampled forward agree within the
    binomial error, and the path probabilities of a birth sum to one."""
    w = inputs.small_variant("plain_fp64", rays_per_point=2000)
    inp = inputs.make_inputs(w)
    osc = orc.OracleScene(w, inp)
    W = np.ones(osc.shape)
    J = orc.scalar_expectation(osc, W, np.arange(w.rays_per_point))
    _, counts, _, _ = osc.forward()
    mc = counts.sum() / w.rays_per_point
    assert abs(J - mc) < 5.0 * np.sqrt(J * (1 - J) / w.rays_per_point)
    # every path of one birth (W = 1 on every outcome, bins or not)
    total = 0.0
    stack = [(0, 0)]
    while stack:
        bits, k = stack.pop()
        _, _, prob, used = osc.forced(7, bits, 64)
        total += prob
        for j in range(k, min(used, 64)):
            stack.append((bits | (1 << j), j + 1))
    assert abs(total - 1.0) < 1e-12
