"""Parity of gwg_tmm_rt (per-hit thin-film solve on the GPU) with the oracle.

FP64: within 1e-12 of the oracle's recursive-Airy solve (an independent
formulation) on lossless stacks of 0 to 200 layers, and within 2e-11 on the
201-layer stack with an absorbing Ag layer, where two independent CPU
formulations already differ by 4.2e-12 (`tmm_cases.FP64_TOL`).  FP32: the
error distribution is measured and reported; the tracer's re-solve rule is
exercised through the mixed mode.
"""
import numpy as np
import pytest
import torch

import inputs
import tmm_cases
from inputs import MAT_AG, MAT_AIR, MAT_AL2O3, MAT_GLASS, MAT_SIO2, MAT_TIO2

pytestmark = pytest.mark.gpu


def _tables(lams=(460.0, 530.0, 620.0)):
    return tmm_cases.tables(lams)


def _oracle(orc, thk, mat, nre, nim, lam, mat_in, mat_out, li, th):
    N = nre[li, mat] + 1j * nim[li, mat]
    n_out = nre[li, mat_out] + 1j * nim[li, mat_out]
    return orc.tmm_rt(thk, N, nre[li, mat_in], n_out, lam[li], theta=th)


_queries = tmm_cases.queries


@pytest.mark.parametrize("L,with_ag", [(0, False), (1, False), (8, False), (40, False), (200, False), (201, True)])
def test_tmm_fp64_matches_oracle(gctx, orc, L, with_ag):
    lam, nre, nim = _tables()
    mat, thk, li, th, sample = tmm_cases.fp64_case(L, with_ag)
    tol = tmm_cases.FP64_TOL[(L, with_ag)]
    n = len(li)
    print(f"tmm fp64 L={L} ag={with_ag} n={n} tol={tol:g}", flush=True)
    got = gctx.tmm_rt(torch.tensor(thk), mat, MAT_GLASS, MAT_GLASS, lam, nre, nim,
                      torch.tensor(li), torch.tensor(th), precision=0).cpu().numpy()
    worst = 0.0
    for q in sample:
        ref = _oracle(orc, thk, mat, nre, nim, lam, MAT_GLASS, MAT_GLASS, li[q], th[q])
        err = np.max(np.abs(got[q] - ref)) / max(1.0, np.max(np.abs(ref)))
        worst = max(worst, err)
        assert err < tol, (q, got[q], ref)
    print(f"  max rel error {worst:.3e}", flush=True)


def test_tmm_exit_media(gctx, orc):
    """Glass -> stack -> air (slab face) and glass -> stack -> Ag."""
    rng = np.random.default_rng(3)
    lam, nre, nim = _tables()
    mat = np.array([MAT_SIO2, MAT_TIO2] * 5, dtype=np.uint8)
    thk = rng.uniform(0, 200, 10)
    for mat_out in (MAT_AIR, MAT_AG):
        li, th = _queries(rng, 300, len(lam), 0.0, 0.0, 85.0)
        got = gctx.tmm_rt(torch.tensor(thk), mat, MAT_GLASS, mat_out, lam, nre, nim,
                          torch.tensor(li), torch.tensor(th), precision=0).cpu().numpy()
        for q in range(300):
            ref = _oracle(orc, thk, mat, nre, nim, lam, MAT_GLASS, mat_out, li[q], th[q])
            assert np.max(np.abs(got[q] - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_tmm_zero_thickness_layers_are_exact_identity(gctx):
    rng = np.random.default_rng(4)
    lam, nre, nim = _tables()
    mat = np.array([MAT_SIO2, MAT_TIO2, MAT_AL2O3] * 10, dtype=np.uint8)
    thk = rng.uniform(0, 300, 30)
    li, th = _queries(rng, 500, len(lam))
    a = gctx.tmm_rt(torch.tensor(thk), mat, MAT_GLASS, MAT_GLASS, lam, nre, nim, torch.tensor(li),
                    torch.tensor(th), precision=0).cpu().numpy()
    thk2 = np.insert(thk, [0, 5, 17, 30], 0.0)
    mat2 = np.insert(mat, [0, 5, 17, 30], MAT_TIO2).astype(np.uint8)
    b = gctx.tmm_rt(torch.tensor(thk2), mat2, MAT_GLASS, MAT_GLASS, lam, nre, nim, torch.tensor(li),
                    torch.tensor(th), precision=0).cpu().numpy()
    assert np.array_equal(a, b)


def test_tmm_energy_and_invalid_queries(gctx):
    rng = np.random.default_rng(5)
    lam, nre, nim = _tables()
    mat = np.array([MAT_SIO2, MAT_TIO2, MAT_AL2O3] * 67, dtype=np.uint8)[:200]
    thk = rng.uniform(0, 300, 200)
    li, th = _queries(rng, 2000, len(lam))
    li[5] = 7          # out of range -> NaN
    th[6] = 2.0        # beyond 90 degrees -> NaN
    c = gctx.tmm_rt(torch.tensor(thk), mat, MAT_GLASS, MAT_GLASS, lam, nre, nim, torch.tensor(li),
                    torch.tensor(th), precision=0).cpu().numpy()
    assert np.all(np.isnan(c[5])) and np.all(np.isnan(c[6]))
    ok = np.ones(2000, bool)
    ok[[5, 6]] = False
    R = np.abs(c[ok, :2]) ** 2
    T = np.abs(c[ok, 2:]) ** 2
    assert np.max(np.abs(R + T - 1)) < 1e-10


def test_tmm_fp32_error_distribution(gctx):
    """FP32 vs FP64 on 200-layer hits: the bulk agrees to single precision; the
    tail (ill-conditioned hits) is what the mixed mode must re-solve."""
    rng = np.random.default_rng(6)
    lam, nre, nim = _tables()
    mat = np.array([MAT_SIO2, MAT_TIO2, MAT_AL2O3] * 67, dtype=np.uint8)[:200]
    thk = rng.uniform(0, 300, 200)
    li, th = _queries(rng, 20000, len(lam), 0.2, 0.0, 88.0)
    args = (torch.tensor(thk), mat, MAT_GLASS, MAT_GLASS, lam, nre, nim, torch.tensor(li), torch.tensor(th))
    c64 = gctx.tmm_rt(*args, precision=0).cpu().numpy()
    c32 = gctx.tmm_rt(*args, precision=2).cpu().numpy()
    cmx = gctx.tmm_rt(*args, precision=1).cpu().numpy()
    dR = np.abs(np.abs(c32[:, :2]) ** 2 - np.abs(c64[:, :2]) ** 2).max(1)
    dRm = np.abs(np.abs(cmx[:, :2]) ** 2 - np.abs(c64[:, :2]) ** 2).max(1)
    q = np.quantile(dR, [0.5, 0.99, 0.9999])
    print(f"fp32 |dR|: median {q[0]:.2e} p99 {q[1]:.2e} p99.99 {q[2]:.2e} max {dR.max():.2e} "
          f"frac>1e-5 {np.mean(dR > 1e-5):.4f}; mixed max {dRm.max():.2e} frac>1e-5 {np.mean(dRm > 1e-5):.4f}",
          flush=True)
    assert q[0] < 1e-5
    assert np.all(np.isfinite(c32))
