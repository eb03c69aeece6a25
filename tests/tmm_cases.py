"""Seeded thin-film query sets shared by the GPU parity tests and the CPU
measurement that sizes their tolerance (input generation only)."""
import numpy as np

import inputs
from inputs import MAT_AG, MAT_AL2O3, MAT_SIO2, MAT_TIO2

#: FP64 tolerance of gwg_tmm_rt against the oracle, relative to max(1, |c|),
#: sized from the largest difference between two independent CPU
#: double-precision formulations (the oracle's Rouard recursion and a numpy
#: characteristic-matrix product) on the same queries: 2.3e-13 on the
#: 200-layer lossless stack, tolerance 1e-12 for every lossless stack; 4.2e-12
#: on the 201-layer stack with an Ag layer, whose absorbing layer amplifies
#: the chain's rounding, tolerance 2e-11.  Each tolerance is at least four
#: times that spread (`test_oracle_tmm.test_fp64_formulation_spread`).
FP64_TOL = {(0, False): 1e-12, (1, False): 1e-12, (8, False): 1e-12, (40, False): 1e-12,
            (200, False): 1e-12, (201, True): 2e-11}


def tables(lams=(460.0, 530.0, 620.0)):
    w = inputs.small_variant("diff_1200", lambdas_nm=lams)
    inp = inputs.make_inputs(w)
    return inp["lambda_nm"], inp["n_re"], inp["n_im"]


def queries(rng, n, nlam, crit_frac=0.2, lo=0.0, hi=89.0):
    li = rng.integers(0, nlam, size=n).astype(np.int32)
    th = np.radians(rng.uniform(lo, hi, size=n))
    k = int(crit_frac * n)
    # near the SiO2/glass critical angle (about 73.9 deg)
    th[:k] = np.radians(rng.uniform(71.5, 76.5, size=k))
    return li, th


def fp64_case(L, with_ag):
    """Stack, queries and the sampled query indices of one FP64 parity case."""
    rng = np.random.default_rng(L)
    cyc = [MAT_SIO2, MAT_TIO2, MAT_AL2O3]
    mat = np.array([cyc[j % 3] for j in range(L)], dtype=np.uint8)
    thk = rng.uniform(0, 300, L)
    if with_ag:
        mat[100] = MAT_AG
        thk[100] = 25.0
    n = 256 * 5 + 37          # several workgroups and a ragged tail
    lam = tables()[0]
    li, th = queries(rng, n, len(lam))
    return mat, thk, li, th, range(0, n, 7)
