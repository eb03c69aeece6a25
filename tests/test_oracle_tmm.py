"""Pins of the oracle's thin-film solver (Methods, "Multilayer thin-film solver").

The oracle evaluates Eq. 3/Eq. 4 recursively (Rouard).  It is pinned here to
things other than itself: an independent characteristic-matrix (Abeles /
Heavens) evaluation written in numpy below, the textbook quarter-wave-stack
reflectance, Brewster's angle, total internal reflection, energy
conservation, reciprocity, absentee layers, zero-thickness invariance and
finite differences of its own derivative.
"""
import json
import os

import numpy as np
import pytest

from numpy_ref import charmatrix, maxwell_event, qz

HERE = os.path.dirname(os.path.abspath(__file__))


def rand_stack(rng, L, mats=(1.46, 2.35, 1.63), hi=300.0):
    thk = rng.uniform(0, hi, L)
    N = np.array([mats[j % len(mats)] for j in range(L)], dtype=np.complex128)
    return thk, N


@pytest.mark.parametrize("L", [0, 1, 2, 8, 40, 200])
def test_rouard_matches_characteristic_matrix(orc, L):
    rng = np.random.default_rng(100 + L)
    for _ in range(20):
        thk, N = rand_stack(rng, L)
        lam = rng.choice([460.0, 530.0, 620.0])
        theta = np.radians(rng.uniform(0, 89))
        k = 1.52 * np.sin(theta)
        a = orc.tmm_rt(thk, N, 1.52, 1.52, lam, kappa=k)
        b = charmatrix(thk, N, 1.52, 1.52, lam, k)
        # the characteristic matrix grows with evanescent layers; compare relative
        # to the coefficient scale
        assert np.max(np.abs(a - b)) < 1e-9 * max(1.0, np.max(np.abs(b))), (L, np.degrees(theta))


def test_rouard_matches_characteristic_matrix_absorbing(orc):
    rng = np.random.default_rng(5)
    for _ in range(30):
        thk, N = rand_stack(rng, 21)
        N[10] = 0.12 + 3.3j
        thk[10] = rng.uniform(10, 40)
        k = 1.52 * np.sin(np.radians(rng.uniform(0, 85)))
        a = orc.tmm_rt(thk, N, 1.52, 1.52, 530.0, kappa=k)
        b = charmatrix(thk, N, 1.52, 1.52, 530.0, k)
        assert np.max(np.abs(a - b)) < 1e-10


def test_different_exit_medium(orc):
    """Air exit (slab top face) and an absorbing exit medium."""
    rng = np.random.default_rng(8)
    for ns in (1.0, 2.0 + 0.1j):
        for _ in range(10):
            thk, N = rand_stack(rng, 5)
            k = 1.52 * np.sin(np.radians(rng.uniform(0, 40)))
            a = orc.tmm_rt(thk, N, 1.52, ns, 550.0, kappa=k)
            b = charmatrix(thk, N, 1.52, ns, 550.0, k)
            assert np.max(np.abs(a - b)) < 1e-12


def test_quarter_wave_stack_closed_form(orc):
    """(HL)^N H on a substrate at its design wavelength and normal incidence:
    R = ((n0 - Y) / (n0 + Y))^2 with Y = (nH/nL)^(2N) nH^2 / ns (Macleod)."""
    for nH, nL, n0, ns, lam0 in [(2.35, 1.46, 1.52, 1.52, 550.0), (2.13, 1.46, 1.9, 1.9, 530.0),
                                 (2.35, 1.63, 1.0, 1.52, 460.0)]:
        for Np in range(0, 6):
            thk, N = [], []
            for _ in range(Np):
                thk += [lam0 / (4 * nH), lam0 / (4 * nL)]
                N += [nH, nL]
            thk.append(lam0 / (4 * nH))
            N.append(nH)
            c = orc.tmm_rt(thk, N, n0, ns, lam0, kappa=0.0)
            Y = (nH / nL) ** (2 * Np) * nH ** 2 / ns
            R = ((n0 - Y) / (n0 + Y)) ** 2
            assert abs(abs(c[0]) ** 2 - R) < 1e-13
            assert abs(abs(c[1]) ** 2 - R) < 1e-13
            # (HL)^N: Y = (nH/nL)^(2N) ns
            c2 = orc.tmm_rt(thk[:-1], N[:-1], n0, ns, lam0, kappa=0.0)
            Y2 = (nH / nL) ** (2 * Np) * ns
            assert abs(abs(c2[0]) ** 2 - ((n0 - Y2) / (n0 + Y2)) ** 2) < 1e-13


def test_paper_materials_quarter_wave(orc):
    """The paper's own coating materials (Ta2O5 / SiO2 on n = 1.9 glass)."""
    with open(os.path.join(HERE, "golden", "paper_constants.json")) as f:
        pc = json.load(f)
    nH, nL, ng = pc["ta2o5_index"], pc["sio2_index"], pc["substrate_index"]
    lam0 = 530.0
    n_pairs = (pc["layers_per_mirror"] - 1) // 2       # 23 layers = (HL)^11 H
    thk, N = [], []
    for _ in range(n_pairs):
        thk += [lam0 / (4 * nH), lam0 / (4 * nL)]
        N += [nH, nL]
    thk.append(lam0 / (4 * nH))
    N.append(nH)
    assert len(thk) == pc["layers_per_mirror"]
    c = orc.tmm_rt(thk, N, ng, ng, lam0, kappa=0.0)
    Y = (nH / nL) ** (2 * n_pairs) * nH ** 2 / ng
    assert abs(abs(c[0]) ** 2 - ((ng - Y) / (ng + Y)) ** 2) < 1e-13


def test_energy_conservation_lossless(orc):
    rng = np.random.default_rng(11)
    for L in (1, 7, 40, 200):
        for _ in range(10):
            thk, N = rand_stack(rng, L)
            th = np.radians(rng.uniform(0, 89.5))
            c = orc.tmm_rt(thk, N, 1.52, 1.52, 530.0, theta=th)
            assert abs(abs(c[0]) ** 2 + abs(c[2]) ** 2 - 1) < 1e-11
            assert abs(abs(c[1]) ** 2 + abs(c[3]) ** 2 - 1) < 1e-11
    # different exit medium: T = Re(q_s)/q_0 |t|^2 for both polarizations
    for _ in range(10):
        thk, N = rand_stack(rng, 9)
        th = np.radians(rng.uniform(0, 40))
        k = 1.52 * np.sin(th)
        c = orc.tmm_rt(thk, N, 1.52, 1.0, 530.0, kappa=k)
        f = qz(1.0, k).real / qz(1.52, k).real
        assert abs(abs(c[0]) ** 2 + f * abs(c[2]) ** 2 - 1) < 1e-12
        assert abs(abs(c[1]) ** 2 + f * abs(c[3]) ** 2 - 1) < 1e-12


def test_absorbing_layer_absorbs(orc):
    rng = np.random.default_rng(12)
    for _ in range(30):
        thk, N = rand_stack(rng, 31)
        N[15] = 0.12 + 3.3j
        thk[15] = rng.uniform(10, 40)
        c = orc.tmm_rt(thk, N, 1.52, 1.52, 460.0, theta=np.radians(rng.uniform(0, 85)))
        for r, t in ((c[0], c[2]), (c[1], c[3])):
            A = 1 - abs(r) ** 2 - abs(t) ** 2
            assert A > 0.0


def test_single_interface_limits(orc):
    # Brewster: glass -> TiO2, tan(theta_B) = n2 / n1 gives r_p = 0
    n1, n2 = 1.52, 2.35
    c = orc.tmm_rt([], [], n1, n2, 550.0, theta=np.arctan(n2 / n1))
    assert abs(c[1]) < 1e-15 and abs(c[0]) > 0.1
    # normal incidence: r_s = (n1 - n2)/(n1 + n2), r_p = -r_s (Eq. 3 convention), t = 2 n1/(n1+n2)
    c = orc.tmm_rt([], [], n1, n2, 550.0, theta=0.0)
    assert abs(c[0] - (n1 - n2) / (n1 + n2)) < 1e-16
    assert abs(c[1] + c[0]) < 1e-16
    assert abs(c[2] - 2 * n1 / (n1 + n2)) < 1e-16 and abs(c[3] - c[2]) < 1e-16
    # total internal reflection glass -> air beyond 41.1 deg: |r| = 1, nonzero phase
    for deg in (41.5, 50.0, 60.0, 80.0):
        c = orc.tmm_rt([], [], 1.52, 1.0, 550.0, theta=np.radians(deg))
        assert abs(abs(c[0]) - 1) < 1e-15 and abs(abs(c[1]) - 1) < 1e-15
        assert abs(np.angle(c[0])) > 1e-3
    # below critical: no TIR
    c = orc.tmm_rt([], [], 1.52, 1.0, 550.0, theta=np.radians(40.0))
    assert abs(c[0]) < 0.9
    # the s-phase on TIR: with exp(-i w t) and a transmitted wave that decays
    # into the air (Im q >= 0), r_s = (a - i b)/(a + i b), a = cos, b =
    # sqrt(sin^2 - n^2) (n = n2/n1), so arg r_s = -2 atan(b / a): signed
    th = np.radians(55.0)
    nrel = 1.0 / 1.52
    phi = 2 * np.arctan(np.sqrt(np.sin(th) ** 2 - nrel ** 2) / np.cos(th))
    c = orc.tmm_rt([], [], 1.52, 1.0, 550.0, theta=th)
    assert abs(np.angle(c[0]) + phi) < 1e-13


@pytest.mark.parametrize("n_out", [1.0, 1.46, 2.35, 0.12 + 3.3j])
def test_single_interface_solves_maxwell(orc, n_out):
    """0 layers: r_s, r_p, t_s, t_p (Eq. 3 amplitudes, p = k x s) equal the
    field ratios of a laboratory-frame solve of Maxwell's boundary conditions,
    signs and phases included, below and above the critical angle."""
    n0, lam = 1.52, 550.0
    for deg in np.linspace(0.5, 88.0, 23):
        th = np.radians(deg)
        d = np.array([np.sin(th), 0.0, np.cos(th)])
        u = np.array([0.0, 0.0, 1.0])
        s = np.cross(d, u) / np.linalg.norm(np.cross(d, u))
        c = orc.tmm_rt([], [], n0, n_out, lam, theta=th)
        Er, kr, Et, kt = maxwell_event(d, s.astype(complex), u, n0, [], n_out, lam)
        assert abs(Er @ s - c[0]) < 1e-14 and abs(Et @ s - c[2]) < 1e-14, deg
        p_in = np.cross(d, s)
        Er, kr, Et, kt = maxwell_event(d, p_in.astype(complex), u, n0, [], n_out, lam)
        # outgoing p = k x s on each wave's own (possibly complex) unit wave vector
        p_r = np.cross(kr / n0, s)
        p_t = np.cross(kt / np.sqrt(kt @ kt), s)
        assert abs(Er @ p_r - c[1]) < 1e-14, deg
        assert abs(Et @ p_t / (p_t @ p_t) - c[3]) < 1e-13, deg


def test_single_layer_is_conjugate_airy(orc):
    """Eq. 4 as printed uses exp(-2 i delta); our exp(-i w t) convention gives
    its complex conjugate for a lossless layer (same |r|, |t|)."""
    n1, n2, n3, d, lam = 1.52, 2.35, 1.52, 83.0, 550.0
    th = np.radians(30.0)
    k = n1 * np.sin(th)
    c = orc.tmm_rt([d], [n2], n1, n3, lam, kappa=k)
    q1, q2, q3 = qz(n1, k), qz(n2, k), qz(n3, k)
    delta = 2 * np.pi / lam * q2 * d
    r12 = (q1 - q2) / (q1 + q2)
    r23 = (q2 - q3) / (q2 + q3)
    t12 = 2 * q1 / (q1 + q2)
    t23 = 2 * q2 / (q2 + q3)
    e = np.exp(-2j * delta)
    r_airy = (r12 + r23 * e) / (1 + r12 * r23 * e)
    t_airy = t12 * t23 * np.exp(-1j * delta) / (1 + r12 * r23 * e)
    assert abs(c[0] - np.conj(r_airy)) < 1e-15
    assert abs(c[2] - np.conj(t_airy)) < 1e-15


def test_zero_thickness_invariance(orc):
    rng = np.random.default_rng(13)
    for _ in range(20):
        thk, N = rand_stack(rng, 12)
        k = 1.52 * np.sin(np.radians(rng.uniform(0, 85)))
        a = orc.tmm_rt(thk, N, 1.52, 1.52, 530.0, kappa=k)
        pos = rng.integers(0, 13, size=3)
        thk2, N2 = list(thk), list(N)
        for p in sorted(pos, reverse=True):
            thk2.insert(p, 0.0)
            N2.insert(p, rng.choice([1.46, 2.35, 1.63, 0.12 + 3.3j]))
        b = orc.tmm_rt(thk2, N2, 1.52, 1.52, 530.0, kappa=k)
        assert np.max(np.abs(a - b)) < 1e-13


def test_half_wave_absentee(orc):
    """A half-wave layer at normal incidence leaves r unchanged and flips t."""
    rng = np.random.default_rng(14)
    lam = 550.0
    for _ in range(10):
        thk, N = rand_stack(rng, 6)
        a = orc.tmm_rt(thk, N, 1.52, 1.52, lam, kappa=0.0)
        nh = 2.35
        thk2 = list(thk) + [lam / (2 * nh)]
        N2 = list(N) + [nh]
        b = orc.tmm_rt(thk2, N2, 1.52, 1.52, lam, kappa=0.0)
        assert abs(a[0] - b[0]) < 1e-13 and abs(a[2] + b[2]) < 1e-13


def test_reciprocity(orc):
    rng = np.random.default_rng(15)
    for absorbing in (False, True):
        for _ in range(10):
            thk, N = rand_stack(rng, 15)
            if absorbing:
                N[7] = 0.12 + 3.3j
                thk[7] = 25.0
            k = 1.52 * np.sin(np.radians(rng.uniform(0, 85)))
            f = orc.tmm_rt(thk, N, 1.52, 1.52, 460.0, kappa=k)
            b = orc.tmm_rt(thk[::-1], N[::-1], 1.52, 1.52, 460.0, kappa=k)
            assert abs(f[2] - b[2]) < 1e-12 and abs(f[3] - b[3]) < 1e-12
            if not absorbing:
                assert abs(abs(f[0]) - abs(b[0])) < 1e-12
            else:
                assert abs(abs(f[0]) - abs(b[0])) > 1e-6


def _fd(orc, thk, N, k, lam, j, h):
    tp, tm = np.array(thk, dtype=float), np.array(thk, dtype=float)
    tp[j] += h
    tm[j] -= h
    return (orc.tmm_rt(tp, N, 1.52, 1.52, lam, kappa=k) - orc.tmm_rt(tm, N, 1.52, 1.52, lam, kappa=k)) / (2 * h)


def test_derivative_matches_central_differences(orc):
    rng = np.random.default_rng(16)
    for L, absorbing in ((1, False), (9, False), (40, False), (25, True)):
        thk, N = rand_stack(rng, L)
        thk += 5.0
        if absorbing:
            N[12] = 0.12 + 3.3j
            thk[12] = 20.0
        for deg in (10.0, 50.0, 74.0, 80.0):
            k = 1.52 * np.sin(np.radians(deg))
            g = orc.tmm_dthk(thk, N, 1.52, 1.52, 530.0, kappa=k)
            for j in range(0, L, max(1, L // 7)):
                fd = _fd(orc, thk, N, k, 530.0, j, 1e-4)
                scale = max(1e-3, np.max(np.abs(g)))
                assert np.max(np.abs(g[j] - fd)) < 1e-6 * scale, (L, deg, j)


def test_quarter_wave_stationarity(orc):
    """At the design wavelength and normal incidence dR/dd_j = 0 for every layer
    of a quarter-wave stack (R is at an extremum)."""
    nH, nL, lam0 = 2.35, 1.46, 550.0
    thk = [lam0 / (4 * nH), lam0 / (4 * nL)] * 4 + [lam0 / (4 * nH)]
    N = [nH, nL] * 4 + [nH]
    c = orc.tmm_rt(thk, N, 1.52, 1.52, lam0, kappa=0.0)
    g = orc.tmm_dthk(thk, N, 1.52, 1.52, lam0, kappa=0.0)
    dR = 2 * np.real(np.conj(c[0]) * g[:, 0])
    assert np.max(np.abs(dR)) < 1e-13
    # but the phase of r is not stationary
    assert np.max(np.abs(g[:, 0])) > 1e-4


@pytest.mark.parametrize("case", [(40, False), (200, False), (201, True)])
def test_fp64_formulation_spread(orc, case):
    """Sizes the GPU thin-film tolerance: on the GPU parity test's own queries,
    two independent double-precision formulations (the oracle's Rouard
    recursion and the numpy characteristic-matrix product) differ by at most a
    quarter of the tolerance that test applies (`tmm_cases.FP64_TOL`)."""
    import tmm_cases
    from inputs import MAT_GLASS
    lam, nre, nim = tmm_cases.tables()
    mat, thk, li, th, sample = tmm_cases.fp64_case(*case)
    worst = 0.0
    for q in sample:
        N = nre[li[q], mat] + 1j * nim[li[q], mat]
        ng = nre[li[q], MAT_GLASS]
        a = orc.tmm_rt(thk, N, ng, ng + 0j, lam[li[q]], theta=th[q])
        b = charmatrix(thk, N, ng, ng, lam[li[q]], ng * np.sin(th[q]))
        worst = max(worst, np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(a))))
    assert worst <= tmm_cases.FP64_TOL[case] / 4, worst


def test_batch_equals_single_queries(orc):
    """orc_tmm_rt_batch (threaded) is the single-query solve, query by query."""
    rng = np.random.default_rng(21)
    thk, N = rand_stack(rng, 30)
    N[7] = 0.12 + 3.3j
    Nl = np.stack([N, N * 1.01, N * 0.99])
    n_in = np.array([1.52, 1.53, 1.51])
    n_out = np.array([1.52, 1.0, 2.0 + 0.1j])
    lam = np.array([460.0, 530.0, 620.0])
    li = rng.integers(0, 3, size=500).astype(np.int32)
    th = np.radians(rng.uniform(0, 85, size=500))
    b = orc.tmm_rt_batch(thk, Nl, n_in, n_out, lam, li, th, threads=4)
    for q in range(0, 500, 7):
        a = orc.tmm_rt(thk, Nl[li[q]], n_in[li[q]], n_out[li[q]], lam[li[q]], theta=th[q])
        assert np.array_equal(a, b[q])
