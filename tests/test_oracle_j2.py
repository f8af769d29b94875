"""Pins of the oracle's J2 oblateness term (App. A.3, Eq. A.4) against
what the mathematics fixes, independently of the way the oracle writes it:

- the term is minus the gradient of the J2 potential
  Phi = mu J2 R^2 (3 z^2 - d^2) / (2 d^5), d the object's offset from the
  body and z its component along the pole (numerical gradient here);
- on the pole axis it is 3 J2 mu R^2 / d^4 away from the body, in the
  equatorial plane 3 J2 mu R^2 / (2 d^4) towards it;
- the oracle's Jacobian matches finite differences of its force;
- a near-circular orbit about an oblate Sun regresses its node about the
  pole at the secular rate dOmega/dt = -(3/2) n J2 (R / p)^2 cos i.
"""
import math

import numpy as np
import pytest

from paper_2509_04666_amd import synth

GM = synth.GM_SUN


def _pole(rng):
    p = rng.normal(size=3)
    return p / np.linalg.norm(p)


def _eph(j2, radius, pole, n_seg=20, t_start=-8.0):
    return synth.sun_only_ephemeris(t_start, n_seg, j2=(j2, radius, pole))


def _a_j2(orc, eph, eph0, x):
    """The J2 part of the oracle's force: with the term less without it
    (exact up to a few ulps of the Newtonian term)."""
    v = np.array([0.0, 0.01, 0.0])
    return orc.accel(eph, 0.0, x, v) - orc.accel(eph0, 0.0, x, v)


def _phi(x, j2, radius, pole):
    d = np.asarray(x, float)
    r2 = float(d @ d)
    z = float(d @ pole)
    return GM * j2 * radius ** 2 * (3.0 * z * z - r2) / (2.0 * r2 ** 2.5)


def test_j2_force_is_minus_the_potential_gradient(orc):
    rng = np.random.default_rng(41)
    j2, radius = 1e-3, 0.01
    pole = _pole(rng)
    eph = _eph(j2, radius, pole)
    eph0 = synth.sun_only_ephemeris(-8.0, 20)
    for _ in range(20):
        x = rng.normal(size=3)
        x *= rng.uniform(0.05, 2.0) / np.linalg.norm(x)
        a = _a_j2(orc, eph, eph0, x)
        h = 1e-5 * np.linalg.norm(x)
        g = np.array([(_phi(x + h * e, j2, radius, pole) - _phi(x - h * e, j2, radius, pole)) / (2 * h)
                      for e in np.eye(3)])
        np.testing.assert_allclose(a, -g, rtol=1e-7, atol=1e-9 * np.abs(g).max())


def test_j2_on_the_pole_and_in_the_equator(orc):
    rng = np.random.default_rng(42)
    j2, radius = 2e-3, 0.02
    pole = _pole(rng)
    eph = _eph(j2, radius, pole)
    eph0 = synth.sun_only_ephemeris(-8.0, 20)
    for d in (0.1, 0.7, 3.0):
        tol = 8 * np.finfo(float).eps * GM / d ** 2           # rounding of the Newtonian term
        a = _a_j2(orc, eph, eph0, d * pole)
        np.testing.assert_allclose(a, 3.0 * j2 * GM * radius ** 2 / d ** 4 * pole, rtol=1e-12, atol=tol)
        a = _a_j2(orc, eph, eph0, -d * pole)
        np.testing.assert_allclose(a, -3.0 * j2 * GM * radius ** 2 / d ** 4 * pole, rtol=1e-12, atol=tol)
        e = np.cross(pole, rng.normal(size=3))
        e /= np.linalg.norm(e)
        a = _a_j2(orc, eph, eph0, d * e)
        np.testing.assert_allclose(a, -1.5 * j2 * GM * radius ** 2 / d ** 4 * e, rtol=1e-12, atol=tol)


def test_j2_jacobian_matches_finite_differences(orc):
    rng = np.random.default_rng(43)
    eph = _eph(5e-3, 0.05, _pole(rng))
    for _ in range(10):
        x = rng.normal(size=3)
        x *= rng.uniform(0.2, 1.5) / np.linalg.norm(x)
        v = rng.normal(size=3) * 0.01
        _, jx, _ = orc.accel(eph, 0.0, x, v, jac=True)
        h = 1e-6 * np.linalg.norm(x)
        fd = np.stack([(orc.accel(eph, 0.0, x + h * e, v) - orc.accel(eph, 0.0, x - h * e, v)) / (2 * h)
                       for e in np.eye(3)], axis=1)
        np.testing.assert_allclose(jx, fd, rtol=1e-6, atol=1e-8 * np.abs(fd).max())


def _node(state, pole, ex, ey):
    h = np.cross(state[:3], state[3:])
    n = np.cross(pole, h)
    return math.atan2(n @ ey, n @ ex), math.acos(np.clip(h @ pole / np.linalg.norm(h), -1, 1))


@pytest.mark.parametrize("inc_deg", [30.0, 120.0])
def test_j2_secular_nodal_regression(orc, inc_deg):
    rng = np.random.default_rng(44)
    j2, radius, a = 1e-2, 0.02, 0.2
    pole = _pole(rng)
    ex = np.cross(pole, [0.3, 0.5, 0.8])
    ex /= np.linalg.norm(ex)
    ey = np.cross(pole, ex)
    inc = math.radians(inc_deg)
    n = math.sqrt(GM / a ** 3)
    period = 2 * math.pi / n
    span = 40 * period
    eph = _eph(j2, radius, pole, n_seg=int(span / synth.SEG_DAYS) + 4)
    # circular orbit of radius a inclined by inc to the body's equator
    r0 = a * ex
    v0 = n * a * (math.cos(inc) * ey + math.sin(inc) * pole)
    t = np.linspace(0.0, span, 641)[1:]
    xs, st, _ = orc.propagate(eph, np.concatenate([r0, v0])[None], 0.0, t, eps=1e-10)
    assert st[0] == 0
    om, incs = zip(*[_node(xs[k, 0], pole, ex, ey) for k in range(t.size)])
    om = np.unwrap(np.array(om))
    slope = np.polyfit(t, om, 1)[0]
    want = -1.5 * n * j2 * (radius / a) ** 2 * math.cos(inc)
    assert abs(slope / want - 1.0) < 5e-3, (slope, want)
    assert np.ptp(incs) < 1e-3
