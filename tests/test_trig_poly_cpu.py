"""The layer sine/cosine's polynomial coefficients (csrc/gwg_trig_poly.h).

The thin-film sweeps evaluate cos/sin (circular layers) and cosh/sinh
(evanescent layers) of the phase thickness with one pair of minimax
polynomials: after a quarter-period reduction with an exact quadrant
rotation (the sweeps through absorbing stacks), or after a half-period
reduction that leaves the sign (-1)^n to the caller (the lossless sweeps of
the forward and the adjoint).  These CPU tests check
that

- the committed header is what its generator writes (Remez fit, 60 digits);
- the device routine's steps, replayed here in exact arithmetic with every
  fused multiply-add and product rounded once to double as the GPU does,
  meet the accuracy the FP64 path is built for: about one unit in the last
  place for circular arguments over many periods, a few for hyperbolic ones
  after the argument halvings and doublings.  The reference values are
  series summed to 70 digits, independent of the fitted coefficients.
"""
import decimal
import math
import os
import random
import re
import subprocess
import sys
from decimal import Decimal as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2601_04370_amd")
HEADER = os.path.join(PKG, "csrc", "gwg_trig_poly.h")

CTX = decimal.Context(prec=80)


def _coeffs(name=""):
    src = open(HEADER).read()
    hexf = r"(-?0x[0-9a-f.]+p[-+]?\d+)"

    def arr(key):
        body = src.split(f"double kTrig{name}Poly{key}[")[1].split("};")[0]
        return [float.fromhex(x) for x in re.findall(hexf, body.split("=", 1)[1])]

    return arr("F"), arr("G")


def _fma(a, b, c):
    return float(CTX.add(CTX.multiply(D(a), D(b)), D(c)))


def _mul(a, b):
    return float(CTX.multiply(D(a), D(b)))


def _device_trig(a, hyper, F, G):
    """The device routine's operations in order, each rounded once."""
    n = float(round(_mul(a, 0.63661977236758134308)))
    k = 0
    if hyper:
        _, e = math.frexp(_mul(a, 2.5464790894703255))
        k, n = max(e, 0), 0.0
    r = _fma(-n, 1.5707963267948966, a)
    r = _fma(-n, 6.123233995736766e-17, r)
    r = math.ldexp(r, -k)
    u = _mul(r, r) if hyper else -_mul(r, r)
    ps = F[-1]
    for c in reversed(F[:-1]):
        ps = _fma(ps, u, c)
    sn = _fma(_mul(r, u), ps, r)
    pc = G[-1]
    for c in reversed(G[:-1]):
        pc = _fma(pc, u, c)
    cs = _fma(u, pc, 1.0)
    q = int(n) & 3
    so, co = (cs, sn) if q & 1 else (sn, cs)
    if q & 2:
        so = -so
    if (q + 1) & 2:
        co = -co
    sn, cs = so, co
    for _ in range(k):
        s2 = _mul(_mul(2.0, sn), cs)
        cs = _fma(cs, cs, _mul(sn, sn))
        sn = s2
    return cs, sn


def _device_trig_half(a, hyper, F, G):
    """The half-period routine's operations in order, each rounded once;
    returns (C, S, n) with cos a = (-1)^n C, sin a = (-1)^n S."""
    n = float(round(_mul(a, 0.31830988618379067154)))
    k = 0
    if hyper:
        _, e = math.frexp(_mul(a, 2.5464790894703255))
        k, n = max(e, 0), 0.0
    r = _fma(-n, 3.141592653589793116, a)
    r = _fma(-n, 1.2246467991473532072e-16, r)
    r = math.ldexp(r, -k)
    u = _mul(r, r) if hyper else -_mul(r, r)
    ps = F[-1]
    for c in reversed(F[:-1]):
        ps = _fma(ps, u, c)
    sn = _fma(_mul(r, u), ps, r)
    pc = G[-1]
    for c in reversed(G[:-1]):
        pc = _fma(pc, u, c)
    cs = _fma(u, pc, 1.0)
    for _ in range(k):
        s2 = _mul(_mul(2.0, sn), cs)
        cs = _fma(cs, cs, _mul(sn, sn))
        sn = s2
    return cs, sn, int(n)


def _series_sin_cos(x):
    x = D(x)
    tiny = D(10) ** -70
    s, t, k = D(0), x, 1
    while abs(t) > tiny:
        s = CTX.add(s, t)
        t = CTX.divide(CTX.multiply(CTX.multiply(-t, x), x), (2 * k) * (2 * k + 1))
        k += 1
    c, t, k = D(0), D(1), 1
    while abs(t) > tiny:
        c = CTX.add(c, t)
        t = CTX.divide(CTX.multiply(CTX.multiply(-t, x), x), (2 * k - 1) * (2 * k))
        k += 1
    return c, s


def test_header_matches_generator():
    out = subprocess.run([sys.executable, os.path.join(PKG, "gen_trig_poly.py"), "--check"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr


def test_coefficients_near_taylor():
    # minimax coefficients stay close to the Taylor ones they replace; the
    # top one absorbs the dropped terms (a few %), the low ones barely move
    for name, nF, nG in (("", 6, 7), ("Half", 8, 8)):
        F, G = _coeffs(name)
        assert len(F) == nF and len(G) == nG
        for P, first in ((F, 3), (G, 2)):
            for j, c in enumerate(P):
                t = 1.0 / math.factorial(2 * j + first)
                bound = 5e-2 if j == len(P) - 1 else 1e-3
                assert abs(c - t) <= bound * t, (name, first, j, c, t)
        # the device code writes the constant term of G as the literal 0.5
        assert G[0] == 0.5


def test_circular_accuracy():
    F, G = _coeffs()
    rng = random.Random(11)
    worst_c = worst_s = 0.0
    args = [rng.uniform(0.0, 12.0) for _ in range(1500)] + [rng.uniform(0.0, 0.8) for _ in range(500)]
    args += [j * math.pi / 4 for j in range(17)] + [0.0, 1e-300, 1e-8]
    for a in args:
        c, s = _device_trig(a, False, F, G)
        ce, se = _series_sin_cos(a)
        worst_c = max(worst_c, abs(float(D(c) - ce)))
        worst_s = max(worst_s, abs(float(D(s) - se)))
    # |cos|, |sin| <= 1: one ulp of 1 is 2.2e-16
    assert worst_c <= 2.5e-16 and worst_s <= 2.5e-16, (worst_c, worst_s)


def test_hyperbolic_accuracy():
    F, G = _coeffs()
    rng = random.Random(12)
    worst = 0.0
    args = [rng.uniform(0.0, 6.0) for _ in range(800)] + [rng.uniform(0.0, 0.4) for _ in range(200)]
    args += [math.pi / 8, math.pi / 4, 1.0, 2.0, 4.0]
    for a in args:
        c, s = _device_trig(a, True, F, G)
        ea, eb = D(a).exp(CTX), (-D(a)).exp(CTX)
        ch, sh = (ea + eb) / 2, (ea - eb) / 2
        worst = max(worst, float(abs(D(c) - ch) / ch))
        if a > 0:
            worst = max(worst, float(abs(D(s) - sh) / sh))
    # the k doublings each add about an ulp of relative error
    assert worst <= 4e-15, worst


def test_half_period_circular_accuracy():
    F, G = _coeffs("Half")
    rng = random.Random(13)
    worst_c = worst_s = 0.0
    args = [rng.uniform(0.0, 12.0) for _ in range(1500)] + [rng.uniform(0.0, 1.7) for _ in range(500)]
    args += [j * math.pi / 4 for j in range(17)] + [0.0, 1e-300, 1e-8]
    for a in args:
        c, s_, n = _device_trig_half(a, False, F, G)
        sg = -1 if n & 1 else 1
        ce, se = _series_sin_cos(a)
        worst_c = max(worst_c, abs(float(D(sg * c) - ce)))
        worst_s = max(worst_s, abs(float(D(sg * s_) - se)))
        assert abs(a - n * math.pi) <= math.pi / 2 + 1e-12
    assert worst_c <= 2.5e-16 and worst_s <= 2.5e-16, (worst_c, worst_s)


def test_half_period_hyperbolic_accuracy():
    F, G = _coeffs("Half")
    rng = random.Random(14)
    worst = 0.0
    for a in [rng.uniform(0.0, 6.0) for _ in range(600)] + [math.pi / 8, 1.0, 4.0]:
        c, s_, n = _device_trig_half(a, True, F, G)
        assert n == 0
        ea, eb = D(a).exp(CTX), (-D(a)).exp(CTX)
        ch, sh = (ea + eb) / 2, (ea - eb) / 2
        worst = max(worst, float(abs(D(c) - ch) / ch), float(abs(D(s_) - sh) / sh))
    assert worst <= 4e-15, worst
