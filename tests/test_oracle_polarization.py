"""Pins of the oracle's polarization transport (Methods, "Polarization ray
tracing", Eq. 5; "Multilayer thin-film solver", Eq. 3) against physics the
oracle does not use.

The reference here is `numpy_ref.maxwell_event`: a plane wave meeting a planar
multilayer, solved from Maxwell's boundary conditions in laboratory
coordinates (transverse fields, continuous tangential E and H), with no s/p
basis, no Fresnel formula and no sign convention.  Against it:

- every single event of the oracle (bare-face total internal reflection and
  exit, coated-mirror reflection and transmission from either side) must give
  the same outgoing field vector;
- at normal incidence every event must act as one scalar on any field
  (isotropy; this fixes r_p(0) = -r_s(0) together with p = k x s);
- a whole Monte Carlo path, replayed event by event from the oracle's own
  event log and the paper's birth reading, must end with the oracle's |E|^2;
- a centre-field ray, whose s axis is the same (+-y) at every surface, must
  carry exactly the product of |c_s|^2 (pure s) or |c_p|^2 (pure p) of the
  events on its path, divided by the branch probabilities (Eq. 6).

Swapping the s and p coefficients anywhere in the event update, or taking the
other evanescent branch at a totally reflecting face (a conjugated phase),
fails these tests.
"""
import math

import numpy as np
import pytest

import inputs
from inputs import MAT_AIR, MAT_GLASS
from numpy_ref import charmatrix, maxwell_event, normal_flux

EV_TIR, EV_EXIT, EV_LEAK, EV_END, EV_MIRROR = 1, 2, 3, 4, 5


def _scene(orc, name, **kw):
    w = inputs.small_variant(name, **kw)
    inp = inputs.make_inputs(w)
    return orc.OracleScene(w, inp), w, inp


def _index(inp, li, mat):
    return complex(inp["n_re"][li, mat], inp["n_im"][li, mat])


def _mirror_normal(w):
    b = math.radians(w.tilt_deg)
    return np.array([-math.sin(b), 0.0, math.cos(b)])


def _stack_as_met(w, inp, li, m, d_in, dsg=0):
    """Layers of mirror m in the order a ray with direction d_in meets them,
    and the unit normal along its travel.  Layer 0 lies on the +n side of the
    mirror plane, so a ray arriving from that side (d . n < 0) meets it
    first; a ray from the other side meets the layers in reverse order."""
    n = _mirror_normal(w)
    L = int(inp["n_layers"][dsg, m])
    lay = [(_index(inp, li, int(inp["mat"][dsg, m, j])), float(inp["thk"][dsg, m, j])) for j in range(L)]
    if d_in @ n < 0:
        return lay, -n
    return lay[::-1], n


def _rand_field(rng, d):
    """Random complex field transverse to d."""
    a = rng.normal(size=3)
    e1 = a - (a @ d) * d
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    c = rng.normal(size=2) + 1j * rng.normal(size=2)
    return c[0] * e1 + c[1] * e2


def _rand_dir(rng, theta_deg, axis):
    """Unit vector at angle theta from `axis`, random azimuth."""
    a = rng.normal(size=3)
    t = a - (a @ axis) * axis
    t /= np.linalg.norm(t)
    th = math.radians(theta_deg)
    return math.cos(th) * axis + math.sin(th) * t


def _expected_face(E, d, ng, na, lam, top):
    """Face event from Maxwell's boundary conditions: (kind, field, direction)."""
    u = np.array([0.0, 0.0, 1.0 if d[2] > 0 else -1.0])
    Er, kr, Et, kt = maxwell_event(d, E, u, ng, [], na, lam)
    if abs(kt.imag @ u) > 0:                  # evanescent exit wave: total reflection
        return EV_TIR, Er, (kr / ng).real
    if not top:
        return EV_LEAK, E, d
    # |E_out|^2 is the transmitted power: scale by the normal power fluxes
    frac = normal_flux(Et, kt, u) / normal_flux(E, ng * d, u)
    scale = math.sqrt(frac * np.vdot(E, E).real / np.vdot(Et, Et).real)
    return EV_EXIT, Et * scale, (kt / na).real


def _expected_mirror(E, d, w, inp, li, m, reflect):
    lay, u = _stack_as_met(w, inp, li, m, d)
    ng = inp["n_re"][li, MAT_GLASS]
    Er, kr, Et, kt = maxwell_event(d, E, u, ng, lay, ng, inp["lambda_nm"][li])
    if reflect:
        return Er, (kr / ng).real
    return Et, (kt / ng).real


# ---------------------------------------------------------------- single events
def test_face_events_solve_maxwell(orc):
    """Bare glass/air faces (Eq. 3 at the slab faces): total internal
    reflection, exit and leak, for arbitrary directions and complex fields."""
    sc, w, inp = _scene(orc, "fwd_scale", rays_per_point=1, fov_n=1)
    rng = np.random.default_rng(11)
    kinds = set()
    for li in range(len(w.lambdas_nm)):
        ng = inp["n_re"][li, MAT_GLASS]
        na = inp["n_re"][li, MAT_AIR]
        lam = inp["lambda_nm"][li]
        for k in range(60):
            up = k % 2 == 0
            th = rng.uniform(0.0, 85.0)
            d = _rand_dir(rng, th, np.array([0.0, 0.0, 1.0 if up else -1.0]))
            E = _rand_field(rng, d)
            surf = orc.SURF_TOP if up else orc.SURF_BOTTOM
            ev, dout, Eout = sc.event(surf, d, E, li=li)
            kind, Ex, dx = _expected_face(E, d, ng, na, lam, up)
            kinds.add(kind)
            assert ev == kind, (th, up)
            scale = np.linalg.norm(E)
            assert np.max(np.abs(Eout - Ex)) < 1e-13 * scale, (ev, th, Eout, Ex)
            assert np.max(np.abs(dout - dx)) < 1e-13
    assert kinds == {EV_TIR, EV_EXIT, EV_LEAK}


def test_face_tir_phase_sign(orc):
    """A field with equal real s and p parts (45 deg linear) acquires, on total
    internal reflection, an s/p phase difference whose sign fixes the
    handedness of the reflected ellipse; Maxwell's boundary conditions with a
    transmitted wave that decays into the air fix it.  Checked as the complex
    ratio of the reflected components, not only its modulus."""
    sc, w, inp = _scene(orc, "fwd_scale", rays_per_point=1, fov_n=1)
    ng = inp["n_re"][1, MAT_GLASS]
    na = inp["n_re"][1, MAT_AIR]
    lam = inp["lambda_nm"][1]
    crit = math.degrees(math.asin(na / ng))
    for th in np.linspace(crit + 0.5, 85.0, 9):
        d = np.array([math.sin(math.radians(th)), 0.0, math.cos(math.radians(th))])
        s = np.array([0.0, 1.0, 0.0])
        p = np.cross(d, s)
        E = (s + p) / math.sqrt(2.0)
        ev, dout, Eout = sc.event(orc.SURF_TOP, d, E, li=1)
        assert ev == EV_TIR
        Er, kr, _, _ = maxwell_event(d, E, np.array([0.0, 0.0, 1.0]), ng, [], na, lam)
        pr = np.cross((kr / ng).real, s)
        want = (Er @ pr) / (Er @ s)
        got = (Eout @ pr) / (Eout @ s)
        assert abs(abs(want) - 1.0) < 1e-13
        assert abs(got - want) < 1e-13, (th, got, want)
        # the s/p phase difference is a retardation, nonzero above the critical angle
        assert abs(np.angle(want)) > 1e-3


@pytest.mark.parametrize("name,kw,tol", [
    ("plain_fp64", dict(rays_per_point=1), 1e-12),
    ("fwd_scale", dict(rays_per_point=1, fov_n=1), 1e-12),
    ("precision_ag", dict(rays_per_point=1, fov_n=1, n_layers=20, ag_layer_at=10), 1e-11),
])
def test_mirror_events_solve_maxwell(orc, name, kw, tol):
    """Coated mirrors (Eq. 3-5): reflection and transmission from both sides,
    arbitrary directions and complex fields, including evanescent layers
    beyond their critical angle and an absorbing layer."""
    sc, w, inp = _scene(orc, name, **kw)
    rng = np.random.default_rng(hash(name) % 2 ** 32)
    n = _mirror_normal(w)
    for li in range(len(w.lambdas_nm)):
        for k in range(24):
            m = int(rng.integers(0, w.n_mirrors))
            front = k % 2 == 0
            th = rng.uniform(0.0, 85.0)
            d = _rand_dir(rng, th, -n if front else n)
            E = _rand_field(rng, d)
            for refl in (1, 0):
                ev, dout, Eout = sc.event(m, d, E, reflect=refl, li=li)
                assert ev == EV_MIRROR
                Ex, dx = _expected_mirror(E, d, w, inp, li, m, refl)
                scale = np.linalg.norm(E)
                assert np.max(np.abs(Eout - Ex)) < tol * scale, (name, li, m, front, th, refl)
                assert np.max(np.abs(dout - dx)) < 1e-13


@pytest.mark.parametrize("offset", [0.0, 3e-7, 3e-5])
def test_normal_incidence_is_isotropic(orc, offset):
    """At normal incidence s and p are indistinguishable, so every event must
    multiply any incoming field by one complex scalar (in laboratory
    coordinates), equal to the normal-incidence solution of Maxwell's
    equations.  Holds on both sides of the tiny-|k x n| fallback basis."""
    sc, w, inp = _scene(orc, "plain_fp64", rays_per_point=1)
    rng = np.random.default_rng(5)
    n = _mirror_normal(w)
    ng = inp["n_re"][0, MAT_GLASS]
    na = inp["n_re"][0, MAT_AIR]
    lam = inp["lambda_nm"][0]
    cases = [(orc.SURF_TOP, np.array([0.0, 0.0, 1.0]), 0)]
    for m in range(w.n_mirrors):
        for axis in (-n, n):
            cases += [(m, axis, 1), (m, axis, 0)]
    for surf, axis, refl in cases:
        d = axis + offset * np.cross(axis, np.array([0.0, 1.0, 0.0]))
        d /= np.linalg.norm(d)
        for _ in range(3):
            E = _rand_field(rng, d)
            ev, dout, Eout = sc.event(surf, d, E, reflect=refl)
            if surf == orc.SURF_TOP:
                _, Ex, _ = _expected_face(E, d, ng, na, lam, True)
            else:
                Ex, _ = _expected_mirror(E, d, w, inp, 0, surf, refl)
            assert np.max(np.abs(Eout - Ex)) < 1e-12 * np.linalg.norm(E)
            if offset == 0.0:
                tau = np.vdot(E, Eout) / np.vdot(E, E)
                assert np.max(np.abs(Eout - tau * E)) < 1e-13 * np.linalg.norm(E), (surf, refl)


# ----------------------------------------------------------------- whole paths
def _birth(w, inp, ray_id, orc):
    """Birth direction and field per the readings: field angle a =
    normalize(tan tx, tan ty, 1) refracted into the glass and mirrored by an
    in-coupler parallel to the mirrors; pure s or p (word 0, bit 0) with
    respect to the top face's basis."""
    pt = ray_id // w.rays_per_point
    F = w.n_fov
    f = pt % F
    li = (pt // F) % len(w.lambdas_nm)
    key = [w.seed & 0xFFFFFFFF, (w.seed >> 32) & 0xFFFFFFFF]
    wd = orc.philox([ray_id & 0xFFFFFFFF, ray_id >> 32, 0, 0], key)
    if w.fov_mode == 1:
        u = (wd >> 8) / 2.0 ** 24
        b = inp["fov"]
        tx = b[0, 0] + u[2] * (b[0, 1] - b[0, 0])
        ty = b[1, 0] + u[3] * (b[1, 1] - b[1, 0])
    else:
        tx, ty = inp["fov"][f]
    a = np.array([math.tan(math.radians(tx)), math.tan(math.radians(ty)), 1.0])
    a /= np.linalg.norm(a)
    ng = inp["n_re"][li, MAT_GLASS]
    g = np.array([a[0] / ng, a[1] / ng, math.sqrt(1.0 - (a[0] ** 2 + a[1] ** 2) / ng ** 2)])
    n = _mirror_normal(w)
    d = g - 2.0 * (g @ n) * n
    s0 = np.cross(d, [0.0, 0.0, 1.0])
    s0 /= np.linalg.norm(s0)
    E = np.cross(d, s0) if (wd[0] & 1) else s0
    return li, d, E.astype(np.complex128), int(wd[0] & 1)


def _p_eff(omega):
    return np.floor(np.asarray(omega) * 4294967296.0) / 4294967296.0


def _replay(w, inp, ev, li, d, E):
    """Field along a logged path, event by event, from Maxwell's equations and
    the Monte Carlo rescaling of Eq. 6.  Returns the final |E|^2."""
    ng = inp["n_re"][li, MAT_GLASS]
    na = inp["n_re"][li, MAT_AIR]
    lam = inp["lambda_nm"][li]
    pe = _p_eff(inp["omega"])
    for e in ev:
        kind, surf, dlog = int(e[0]), int(e[1]), e[5:8]
        if kind in (EV_TIR, EV_EXIT, EV_LEAK):
            k2, E, d2 = _expected_face(E, d, ng, na, lam, surf == 1000)
            assert k2 == kind
        elif kind == EV_MIRROR:
            refl = int(e[9])
            E, d2 = _expected_mirror(E, d, w, inp, li, surf, refl)
            p = pe[surf] if refl else 1.0 - pe[surf]
            E = E / math.sqrt(p)
        else:
            d2 = d
        assert np.max(np.abs(d2 - dlog)) < 1e-12
        d = dlog
    return float(np.vdot(E, E).real)


@pytest.mark.parametrize("name,kw", [
    ("plain_fp64", dict(rays_per_point=160)),
    ("fwd_scale", dict(rays_per_point=12, fov_n=3, fov_half_deg=9.0)),
])
def test_paths_replayed_from_maxwell(orc, name, kw):
    """Whole Monte Carlo paths: the oracle's final |E|^2 equals a replay of its
    logged events with fields from Maxwell's boundary conditions (random
    field angles, so s and p mix between surfaces)."""
    sc, w, inp = _scene(orc, name, **kw)
    ids = np.arange(w.n_rays)
    rec = sc.trace_rays(ids)
    mixed = 0
    for r in rec:
        ev = sc.events(r.ray_id, cap=w.max_events)
        li, d, E, _ = _birth(w, inp, r.ray_id, orc)
        wr = _replay(w, inp, ev, li, d, E)
        assert abs(wr - r.w) <= 1e-11 * max(wr, 1e-300) + 1e-300, (r.ray_id, wr, r.w)
        mixed += int(sum(1 for e in ev if e[0] == EV_MIRROR) >= 2)
    assert mixed > len(rec) // 4


def test_centre_field_rays_carry_one_polarization(orc):
    """A centre-field ray moves in the x-z plane, so its s axis is +-y at every
    surface: a pure-s ray ends with the product of |c_s|^2 over its mirror
    events (c = r or t of the branch taken, from the characteristic-matrix
    solve), over the branch probabilities, times the exit transmittance; a
    pure-p ray with |c_p|^2.  Total internal reflections have |r_s| = |r_p| = 1."""
    sc, w, inp = _scene(orc, "fwd_scale", rays_per_point=400, fov_n=1, lambdas_nm=(530.0,))
    pe = _p_eff(inp["omega"])
    n = _mirror_normal(w)
    ng = inp["n_re"][0, MAT_GLASS]
    na = inp["n_re"][0, MAT_AIR]
    lam = inp["lambda_nm"][0]
    rec = sc.trace_rays(np.arange(w.n_rays))
    seen = {0: 0, 1: 0}
    contrast = 0.0
    for r in rec:
        if r.category != 0:
            continue
        ev = sc.events(r.ray_id, cap=w.max_events)
        _, d, _, pol = _birth(w, inp, r.ray_id, orc)
        prod = 1.0
        other = 1.0
        for e in ev:
            kind, surf = int(e[0]), int(e[1])
            if kind == EV_MIRROR:
                assert abs(d[1]) == 0.0
                lay, _ = _stack_as_met(w, inp, 0, surf, d)
                kap = ng * np.linalg.norm(np.cross(d, n))
                c = charmatrix([t for _, t in lay], [N for N, _ in lay], ng, ng, lam, kap)
                refl = int(e[9])
                cs, cp = (c[0], c[1]) if refl else (c[2], c[3])
                p = pe[surf] if refl else 1.0 - pe[surf]
                mine, theirs = (cs, cp) if pol == 0 else (cp, cs)
                prod *= abs(mine) ** 2 / p
                other *= abs(theirs) ** 2 / p
            elif kind == EV_EXIT:
                s = np.array([0.0, 1.0, 0.0])
                Ein = s if pol == 0 else np.cross(d, s)
                u = np.array([0.0, 0.0, 1.0])
                Er, kr, Et, kt = maxwell_event(d, Ein.astype(complex), u, ng, [], na, lam)
                prod *= normal_flux(Et, kt, u) / normal_flux(Ein.astype(complex), ng * d, u)
            d = e[5:8]
        assert abs(prod - r.w) <= 1e-12 * prod, (r.ray_id, pol, prod, r.w)
        seen[pol] += 1
        contrast = max(contrast, abs(prod - other) / prod)
    assert seen[0] > 20 and seen[1] > 20
    # the test discriminates: s and p products differ along these paths
    assert contrast > 1e-2
