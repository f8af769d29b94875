"""Pins of the CPU oracle against values fixed by the paper and by the
mathematics: polynomial reproduction, analytic planet motion, potential
gradients, the relativistic perihelion advance, Kepler's equation,
conservation laws, time reversal, self-convergence, brute-force and
closed-form field-of-view membership, and the symplectic structure of
the state transition matrix.  None of these re-types an oracle formula."""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npc
from numpy.polynomial import legendre as npl

from paper_2509_04666_amd import synth

GM = synth.GM_SUN


# ---------------------------------------------------------------- nodes
def test_radau_nodes_are_legendre_roots(orc):
    # roots of P7 + P8 from numpy's Legendre class, mapped to [0, 1]
    c = np.zeros(9); c[7] = 1; c[8] = 1
    r = np.sort(npl.legroots(c))
    r = r[r > -1 + 1e-9]
    ref = np.concatenate([[0.0], 0.5 * (r + 1.0)])
    np.testing.assert_allclose(orc.radau_nodes(), ref, rtol=0, atol=1e-15)


def test_radau_quadrature_degree(orc):
    # the left Radau rule on 8 nodes integrates polynomials of degree <= 14 exactly
    s = orc.radau_nodes()
    V = np.vander(s, 8, increasing=True).T
    w = np.linalg.solve(V, 1.0 / np.arange(1, 9))
    for k in range(15):
        assert abs(np.dot(w, s ** k) - 1.0 / (k + 1)) < 1e-13, k


# ---------------------------------------------------------------- Chebyshev
def test_cheb_reproduces_polynomials(orc):
    rng = np.random.default_rng(0)
    eph = synth.polynomial_ephemeris(rng, 2, -8.0, 4)
    # replace segment contents by Chebyshev series of random monomial polynomials
    polys = rng.normal(size=(2, 4, 3, 13))
    for b in range(2):
        for k in range(4):
            for c in range(3):
                eph.coef[b, k, c] = npc.poly2cheb(polys[b, k, c])
    for t in rng.uniform(-8.0, 24.0, 40):
        k = min(int((t + 8.0) // 8.0), 3)
        tau = 2 * (t - (-8.0 + 8.0 * k)) / 8.0 - 1.0
        for b in range(2):
            st, p, v = orc.cheb(eph, b, t)
            assert st == 0
            ref = [np.polynomial.polynomial.polyval(tau, polys[b, k, c]) for c in range(3)]
            dref = [np.polynomial.polynomial.polyval(tau, np.polynomial.polynomial.polyder(polys[b, k, c])) * 2 / 8.0
                    for c in range(3)]
            np.testing.assert_allclose(p, ref, rtol=1e-13, atol=1e-13)
            np.testing.assert_allclose(v, dref, rtol=1e-12, atol=1e-12)


def test_cheb_matches_analytic_planets(orc):
    case = synth.survey_case(n_obj=1, n_frames=0)
    rng = np.random.default_rng(1)
    # the Moon's 27-day orbit fits degree 12 over 8 days to about 4 cm
    # (its table is the tightest; planets stay at the rounding level)
    tol = {"moon": (1e-12, 2e-11)}
    for t in rng.uniform(0.0, 365.0, 50):
        ref = case.model.bary(np.array(t))
        for b in range(case.ephem.n_body):
            st, p, v = orc.cheb(case.ephem, b, t)
            tp, tv = tol.get(case.ephem.names[b], (2e-13, 1e-12))
            assert st == 0
            assert np.max(np.abs(p - ref[b, :3])) < tp
            assert np.max(np.abs(v - ref[b, 3:])) < tv


def test_cheb_joint_continuity_and_range(orc):
    case = synth.tiny_case(n_obj=1, n_frames=1)
    e = case.ephem
    for k in range(1, e.n_seg):
        t = e.t_start + k * e.seg_days
        _, p1, _ = orc.cheb(e, 1, t - 1e-9)
        _, p2, _ = orc.cheb(e, 1, t)
        assert np.max(np.abs(p1 - p2)) < 1e-10  # 1e-9 day of motion at ~0.01 au/day
    assert orc.cheb(e, 1, e.t_start - 1e-6)[0] == -2
    assert orc.cheb(e, 1, e.t_end + 1e-6)[0] == -2
    assert orc.cheb(e, 1, e.t_end)[0] == 0


# ---------------------------------------------------------------- force
def test_newtonian_force_is_potential_gradient(orc):
    case = synth.survey_case(n_obj=20, n_frames=0)
    e = case.ephem
    e.flags[:] = 0
    t = 17.3
    pos = np.array([orc.cheb(e, b, t)[1] for b in range(e.n_body)])

    def phi(x):  # gravitational potential energy per unit mass
        return -np.sum(e.gm / np.linalg.norm(x[None, :] - pos, axis=1))

    for x in case.x0[:5, :3]:
        a = orc.accel(e, t, x, np.zeros(3))
        h = 1e-5
        g = np.array([(phi(x + h * np.eye(3)[i]) - phi(x - h * np.eye(3)[i])) / (2 * h) for i in range(3)])
        np.testing.assert_allclose(a, -g, rtol=1e-8, atol=1e-16)


def test_jacobians_match_finite_differences(orc):
    case = synth.survey_case(n_obj=6, n_frames=0)
    e = case.ephem
    t = 40.0
    c_red = 20.0     # enlarge the relativistic part so its Jacobian is visible
    for s in case.x0[:6]:
        a, jx, jv = orc.accel(e, t, s[:3], s[3:], c_light=c_red, jac=True)
        h = 1e-6
        for i in range(3):
            dx = np.eye(3)[i] * h
            fx = (orc.accel(e, t, s[:3] + dx, s[3:], c_light=c_red) - orc.accel(e, t, s[:3] - dx, s[3:], c_light=c_red)) / (2 * h)
            fv = (orc.accel(e, t, s[:3], s[3:] + dx, c_light=c_red) - orc.accel(e, t, s[:3], s[3:] - dx, c_light=c_red)) / (2 * h)
            np.testing.assert_allclose(jx[:, i], fx, rtol=1e-6, atol=1e-6 * np.abs(jx).max())
            np.testing.assert_allclose(jv[:, i], fv, rtol=1e-6, atol=1e-5 * np.abs(jv).max())


def test_relativistic_perihelion_advance(orc):
    # Sun-only, reduced c: the eps=0 term advances the perihelion by
    # 6 pi mu / (c^2 a (1 - e^2)) per orbit.  Perihelia are located as the
    # sign changes of r.v on a fine time grid.
    a, ecc = 1.0, 0.5
    c_red = 2.0
    eph = synth.sun_only_ephemeris(-8.0, 300, gr=True)
    x0 = synth.elements_to_state(a, ecc, 0.0, 0.0, 0.0, 0.0, GM)
    P = 2 * np.pi * math.sqrt(a ** 3 / GM)

    def perihelion_angle(center, half):
        ts = np.linspace(center - half, center + half, 4001)
        xs, st, _ = orc.propagate(eph, x0[None], 0.0, ts, eps=1e-11, c_light=c_red)
        assert st[0] == 0
        rv = np.sum(xs[:, 0, :3] * xs[:, 0, 3:], axis=1)
        i = np.nonzero((rv[:-1] < 0) & (rv[1:] >= 0))[0][0]
        w = -rv[i] / (rv[i + 1] - rv[i])
        ang = np.arctan2(xs[:, 0, 1], xs[:, 0, 0])
        return ts[i] + w * (ts[i + 1] - ts[i]), ang[i] + w * (ang[i + 1] - ang[i])

    t1, a1 = perihelion_angle(P, 5.0)
    drift = t1 - P
    angs = [0.0, a1]
    for k in (2, 3, 4):
        angs.append(perihelion_angle(k * (P + drift), 2.0)[1])
    rate = np.polyfit(np.arange(5), np.unwrap(angs), 1)[0]
    expect = 6 * np.pi * GM / (c_red ** 2 * a * (1 - ecc ** 2))
    assert abs(rate / expect - 1.0) < 2e-3, (rate, expect)


# ---------------------------------------------------------------- integrator
def _kepler_analytic(el, dt):
    n = np.sqrt(GM / el[:, 0] ** 3)
    return synth.elements_to_state(el[:, 0], el[:, 1], el[:, 2], el[:, 3], el[:, 4], el[:, 5] + n * dt, GM)


def test_sun_only_matches_analytic_kepler(orc):
    rng = np.random.default_rng(3)
    el = np.concatenate([synth.main_belt_elements(rng, 30), synth.neo_elements(rng, 10)])
    eph = synth.sun_only_ephemeris(-8.0, 60)
    x0 = synth.elements_to_state(el[:, 0], el[:, 1], el[:, 2], el[:, 3], el[:, 4], el[:, 5], GM)
    ts = np.array([91.0, 200.5, 365.25])
    xs, st, _ = orc.propagate(eph, x0, 0.0, ts)
    assert np.all(st == 0)
    for k, t in enumerate(ts):
        ref = _kepler_analytic(el, t)
        assert np.max(np.abs(xs[k, :, :3] - ref[:, :3])) < 1e-12
        assert np.max(np.abs(xs[k, :, 3:] - ref[:, 3:])) < 1e-14


def test_conservation_and_time_reversal(orc):
    rng = np.random.default_rng(4)
    el = np.concatenate([synth.main_belt_elements(rng, 10), synth.neo_elements(rng, 10)])
    eph = synth.sun_only_ephemeris(-400.0, 110)
    x0 = synth.elements_to_state(el[:, 0], el[:, 1], el[:, 2], el[:, 3], el[:, 4], el[:, 5], GM)
    xs, st, _ = orc.propagate(eph, x0, 0.0, [365.25, 0.0])
    assert np.all(st == 0)

    def energy(s): return 0.5 * np.sum(s[:, 3:] ** 2, 1) - GM / np.linalg.norm(s[:, :3], axis=1)
    def angmom(s): return np.cross(s[:, :3], s[:, 3:])
    def lrl(s):
        return np.cross(s[:, 3:], angmom(s)) / GM - s[:, :3] / np.linalg.norm(s[:, :3], axis=1)[:, None]

    assert np.max(np.abs(energy(xs[0]) / energy(x0) - 1)) < 1e-13
    assert np.max(np.abs(angmom(xs[0]) - angmom(x0))) < 1e-15
    assert np.max(np.abs(lrl(xs[0]) - lrl(x0))) < 1e-12
    assert np.max(np.abs(xs[1, :, :3] - x0[:, :3])) < 1e-11


def test_self_convergence_full_perturbers(orc):
    case = synth.survey_case(n_obj=24, n_frames=0, neo_frac=0.25)
    ts = np.linspace(30.0, 365.25, 12)
    # the b6 round-off floor (~1e-11 of |a|) bounds eps from below, so the
    # reference run instead caps the step at a quarter day
    a, sa, _ = orc.propagate(case.ephem, case.x0, 0.0, ts, eps=1e-9)
    b, sb, _ = orc.propagate(case.ephem, case.x0, 0.0, ts, eps=1e-9, h_max=0.25)
    assert np.all(sa == 0) and np.all(sb == 0)
    assert np.max(np.abs(a[:, :, :3] - b[:, :, :3])) < 1e-12


def test_epoch_chaining_matches_direct(orc):
    # landing on intermediate epochs does not change the result beyond round-off
    case = synth.survey_case(n_obj=16, n_frames=0, neo_frac=0.25)
    a, _, _ = orc.propagate(case.ephem, case.x0, 0.0, np.arange(3.0, 366.0, 3.0))
    b, _, _ = orc.propagate(case.ephem, case.x0, 0.0, [a.shape[0] * 3.0])
    assert np.max(np.abs(a[-1, :, :3] - b[0, :, :3])) < 1e-12


# ---------------------------------------------------------------- Kepler
def test_kepler_elliptic_vs_eccentric_anomaly(orc):
    rng = np.random.default_rng(5)
    el = np.concatenate([synth.main_belt_elements(rng, 40), synth.neo_elements(rng, 40)])
    s0 = synth.elements_to_state(el[:, 0], el[:, 1], el[:, 2], el[:, 3], el[:, 4], el[:, 5], GM)
    for dt in (-1.6, -0.02, 1e-6, 0.7, 1.5, 30.0, 800.0):
        ref = _kepler_analytic(el, dt)
        for j in range(el.shape[0]):
            st, r, v = orc.kepler(GM, s0[j, :3], s0[j, 3:], dt)
            assert st == 0
            tol = 1e-14 * max(1.0, abs(dt) / 10)
            assert np.max(np.abs(r - ref[j, :3])) < tol, (dt, j)
            assert np.max(np.abs(v - ref[j, 3:])) < tol


def test_kepler_hyperbolic_vs_hyperbolic_anomaly(orc):
    # e sinh H - H = M, r = a (1 - e cosh H) with a < 0, in the orbital plane
    mu = GM
    for ecc, q in [(1.3, 0.5), (2.5, 1.2), (1.05, 0.3)]:
        a = q / (1 - ecc)
        n = math.sqrt(mu / (-a) ** 3)

        def st_at(M):
            H = math.asinh(M / ecc) if abs(M) > 0 else 0.0
            for _ in range(100):
                H -= (ecc * math.sinh(H) - H - M) / (ecc * math.cosh(H) - 1)
            r = a * (1 - ecc * math.cosh(H))
            x = a * (math.cosh(H) - ecc)
            y = -a * math.sqrt(ecc ** 2 - 1) * math.sinh(H)
            Hd = n / (ecc * math.cosh(H) - 1)
            vx = a * math.sinh(H) * Hd
            vy = -a * math.sqrt(ecc ** 2 - 1) * math.cosh(H) * Hd
            return np.array([x, y, 0.0]), np.array([vx, vy, 0.0]), r

        r0, v0, _ = st_at(-0.3)
        for dt in (0.5, 5.0, 50.0):
            r1, v1, _ = st_at(-0.3 + n * dt)
            st, r, v = orc.kepler(mu, r0, v0, dt)
            assert st == 0
            np.testing.assert_allclose(r, r1, rtol=0, atol=2e-13 * max(1, np.linalg.norm(r1)))
            np.testing.assert_allclose(v, v1, rtol=0, atol=2e-14)


def test_kepler_reversibility_and_invariants(orc):
    rng = np.random.default_rng(6)
    el = synth.neo_elements(rng, 50)
    s0 = synth.elements_to_state(el[:, 0], el[:, 1], el[:, 2], el[:, 3], el[:, 4], el[:, 5], GM)
    for j in range(50):
        _, r, v = orc.kepler(GM, s0[j, :3], s0[j, 3:], 1.3)
        _, r2, v2 = orc.kepler(GM, r, v, -1.3)
        assert np.max(np.abs(r2 - s0[j, :3])) < 1e-14
        h0 = np.cross(s0[j, :3], s0[j, 3:]); h1 = np.cross(r, v)
        assert np.max(np.abs(h1 - h0)) < 1e-17
        e0 = 0.5 * s0[j, 3:] @ s0[j, 3:] - GM / np.linalg.norm(s0[j, :3])
        e1 = 0.5 * v @ v - GM / np.linalg.norm(r)
        assert abs(e1 / e0 - 1) < 1e-13


# ---------------------------------------------------------------- light time
def test_light_time_vs_independent_root(orc):
    from scipy.optimize import brentq
    rng = np.random.default_rng(7)
    el = synth.main_belt_elements(rng, 20)
    eph = synth.sun_only_ephemeris(-8.0, 10)
    s0 = synth.elements_to_state(el[:, 0], el[:, 1], el[:, 2], el[:, 3], el[:, 4], el[:, 5], GM)
    c = synth.C_AU_PER_DAY
    for j in range(20):
        t_ref, t_obs = 5.0, 6.2
        o = np.array([math.cos(0.3 * j), math.sin(0.3 * j), 0.01])
        st, d, tau, xe = orc.lighttime(eph, t_ref, s0[j], t_obs, o)
        assert st == 0

        def pos(t):  # elements are valid at t_ref here
            return _kepler_analytic(el[j:j + 1], t - t_ref)[0, :3]

        tau_ref = brentq(lambda x: c * x - np.linalg.norm(pos(t_obs - x) - o), 0.0, 0.2, xtol=1e-18, rtol=1e-15)
        assert abs(tau - tau_ref) < 1e-15
        np.testing.assert_allclose(d, pos(t_obs - tau_ref) - o, rtol=0, atol=1e-13)
        assert abs(c * tau - np.linalg.norm(d)) < 1e-13


# ---------------------------------------------------------------- FoV
def _gnomonic_inside(fr, f, s, d):
    c, u, w = fr.center[f, s], fr.u[f, s], fr.w[f, s]
    dc = d @ c
    if dc <= 0:
        return False
    return abs(d @ u / dc) < math.tan(fr.half_u[f, s]) and abs(d @ w / dc) < math.tan(fr.half_w[f, s])


def _gnomonic_margin(fr, f, s, d):
    c, u, w = fr.center[f, s], fr.u[f, s], fr.w[f, s]
    dc = d @ c
    if dc <= 0:
        return -1.0
    return min(math.tan(fr.half_u[f, s]) - abs(d @ u / dc), math.tan(fr.half_w[f, s]) - abs(d @ w / dc))


def test_membership_equals_gnomonic_box(orc):
    rng = np.random.default_rng(8)
    case = synth.tiny_case(n_obj=1, n_frames=40)
    fr = case.frames
    for f in range(fr.n_frames):
        for _ in range(200):
            d = fr.center[f, 0] + rng.normal(scale=0.02, size=3)
            ins, _ = orc.inside(fr.normals[f], d)
            assert ins[0] == _gnomonic_inside(fr, f, 0, d)


def test_membership_edge_band(orc):
    # directions 2 mas inside / outside each edge midpoint and near corners
    case = synth.tiny_case(n_obj=1, n_frames=10)
    fr = case.frames
    mas = math.radians(1 / 3.6e6)
    for f in range(fr.n_frames):
        c, u, w = fr.center[f, 0], fr.u[f, 0], fr.w[f, 0]
        hu, hw = fr.half_u[f, 0], fr.half_w[f, 0]
        for axis, h in ((u, hu), (w, hw)):
            for sgn in (1, -1):
                for delta, want in ((-2 * mas, True), (2 * mas, False)):
                    ang = h + delta
                    d = math.cos(ang) * c + sgn * math.sin(ang) * axis
                    ins, edge = orc.inside(fr.normals[f], d)
                    assert ins[0] == want
                    assert abs(abs(edge[0]) - 2 * mas) < 1e-3 * mas


def _rotate_ephem(eph, R):
    import copy
    e2 = copy.deepcopy(eph)
    e2.coef = np.einsum("ij,bsjk->bsik", R, eph.coef)
    return e2


def test_fov_bruteforce_definition_and_rotation_invariance(orc):
    case = synth.tiny_case(n_obj=300, n_frames=20, n_targeted=40)
    fr = case.frames
    order, off, t_ref = orc.make_batches(fr.t)
    xe, st, _ = orc.propagate(case.ephem, case.x0, 0.0, t_ref)
    pf, ps, po, edge = orc.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals)
    assert pf.size > 20
    # definition: recompute membership directly from the (pinned) light-time
    # directions and the gnomonic closed form
    pairs, ambiguous = set(), set()
    for b in range(t_ref.size):
        for q in range(off[b], off[b + 1]):
            f = order[q]
            d, _ = orc.directions(case.ephem, xe[b], t_ref[b], fr.t[f], fr.obs[f])
            for j in range(case.x0.shape[0]):
                if _gnomonic_inside(fr, f, 0, d[j]):
                    pairs.add((f, 0, j))
                if abs(_gnomonic_margin(fr, f, 0, d[j])) < 1e-12:
                    ambiguous.add((f, 0, j))
    got = set(zip(pf.tolist(), ps.tolist(), po.tolist()))
    assert (got ^ pairs) <= ambiguous
    # global rotation of every vector leaves the pair set unchanged
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    eph_r = _rotate_ephem(case.ephem, Q)
    xr = xe.copy()
    xr[..., :3] = xe[..., :3] @ Q.T
    xr[..., 3:] = xe[..., 3:] @ Q.T
    nr = fr.normals @ Q.T
    pf2, ps2, po2, edge2 = orc.fov(eph_r, xr, st, order, off, t_ref, fr.t, fr.obs @ Q.T, nr)
    got2 = set(zip(pf2.tolist(), ps2.tolist(), po2.tolist()))
    far = {(f, s, j) for f, s, j, e in zip(pf, ps, po, edge) if abs(e) > 1e-9}
    assert far <= got2
    assert len(got2 ^ got) <= len([e for e in edge if abs(e) < 1e-9]) + len([e for e in edge2 if abs(e) < 1e-9])


def test_batching_rule(orc):
    rng = np.random.default_rng(10)
    t = np.round(rng.uniform(0, 30, 300), 1)   # many ties
    order, off, t_ref = orc.make_batches(t, 3.0)
    ts = t[order]
    assert np.all(np.diff(ts) >= 0)
    for b in range(off.size - 1):
        seg = ts[off[b]:off[b + 1]]
        assert seg[-1] - seg[0] <= 3.0
        if off[b + 1] < ts.size:
            assert ts[off[b + 1]] - seg[0] > 3.0
        assert t_ref[b] == 0.5 * (seg[0] + seg[-1])
    # ties keep index order
    for i in range(1, order.size):
        if ts[i] == ts[i - 1]:
            assert order[i] > order[i - 1]


# ---------------------------------------------------------------- magnitudes
def test_hg_magnitude_closed_forms(orc):
    ln10 = math.log(10.0)
    rng = np.random.default_rng(30)
    for _ in range(20):
        H, G = rng.uniform(5, 20), rng.uniform(-0.1, 0.6)
        r, d = rng.uniform(0.5, 5), rng.uniform(0.05, 6)
        # zero phase: both phase functions are 1, only the distances remain
        assert abs(orc.hg_mag(H, G, r, d, 0.0) - (H + 5 * math.log10(r) + 5 * math.log10(d))) < 1e-12
    assert orc.hg_mag(7.25, 0.15, 1.0, 1.0, 0.0) == 7.25
    # tan(alpha/2) = 1 fixes A1 (G = 0) and A2 (G = 1); tan(alpha/2) = 2 adds B1, B2
    assert abs(orc.hg_mag(0.0, 0.0, 1, 1, math.pi / 2) - 2.5 * 3.33 / ln10) < 1e-12
    assert abs(orc.hg_mag(0.0, 1.0, 1, 1, math.pi / 2) - 2.5 * 1.87 / ln10) < 1e-12
    a2 = 2 * math.atan(2.0)
    assert abs(orc.hg_mag(0.0, 0.0, 1, 1, a2) - 2.5 * 3.33 * 2 ** 0.63 / ln10) < 1e-12
    assert abs(orc.hg_mag(0.0, 1.0, 1, 1, a2) - 2.5 * 1.87 * 2 ** 1.22 / ln10) < 1e-12


def test_hg_magnitude_flux_linear_in_slope_and_monotone(orc):
    # the reduced flux 10^(-0.4 (V - H)) at r = Delta = 1 is the G-weighted
    # mix of two phase functions: affine in G; V grows with the phase angle
    alphas = np.linspace(0.0, math.radians(120), 41)
    for a in alphas[1:]:
        fl = [10 ** (-0.4 * orc.hg_mag(0.0, g, 1, 1, a)) for g in (0.0, 0.3, 0.6)]
        assert abs(fl[1] - 0.5 * (fl[0] + fl[2])) < 1e-14
        assert 0 < fl[0] < 1 and 0 < fl[2] < 1
    for g in (-0.1, 0.15, 0.6):
        v = [orc.hg_mag(0.0, g, 1, 1, a) for a in alphas]
        assert np.all(np.diff(v) > 0)


def test_pair_magnitude_geometry(orc):
    # over the pairs of a small survey: the phase angle is the angle at the
    # body of the Sun-body-observer triangle (law of cosines with the
    # Sun-observer distance taken from the ephemeris separately), Delta is
    # c times the light time, r_H the body's distance from the Sun at
    # emission, and V the H-G value at that geometry
    case = synth.tiny_case(n_obj=300, n_frames=30, n_targeted=40)
    fr = case.frames
    order, off, t_ref = orc.make_batches(fr.t)
    xe, st, _ = orc.propagate(case.ephem, case.x0, 0.0, t_ref)
    pf, ps, po, _ = orc.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals)
    assert pf.size > 20
    H, G = synth.hg_params(np.random.default_rng(31), case.x0.shape[0])
    v, geom = orc.pair_mags(case.ephem, xe, order, off, t_ref, fr.t, fr.obs, pf, po, H, G)
    fb = np.empty(fr.t.size, np.int64)
    for b in range(t_ref.size):
        fb[order[off[b]:off[b + 1]]] = b
    for i in range(pf.size):
        f, j = pf[i], po[i]
        b = fb[f]
        _, d, tau, x_emit = orc.lighttime(case.ephem, t_ref[b], xe[b, j], fr.t[f], fr.obs[f])
        _, sun, _ = orc.cheb(case.ephem, 0, fr.t[f] - tau)
        rh, dl, al = geom[i]
        R = np.linalg.norm(np.asarray(sun) - fr.obs[f])
        assert abs(dl - orc.C_AU_PER_DAY * tau) < 1e-12
        assert abs(rh - np.linalg.norm(x_emit[:3] - np.asarray(sun))) < 1e-13
        assert abs(math.cos(al) - (rh ** 2 + dl ** 2 - R ** 2) / (2 * rh * dl)) < 1e-12
        assert abs(v[i] - orc.hg_mag(H[j], G[j], rh, dl, al)) < 1e-12
    assert np.all(np.isfinite(v)) and geom[:, 2].max() < math.pi / 2


# ---------------------------------------------------------------- variational
def test_stm_symplectic_newtonian(orc):
    case = synth.survey_case(n_obj=4, n_frames=0, neo_frac=0.5)
    e = case.ephem
    e.flags[:] = 0
    J = np.zeros((6, 6)); J[:3, 3:] = np.eye(3); J[3:, :3] = -np.eye(3)
    for s in case.x0:
        _, phi = orc.stm(e, s, 0.0, 60.0)
        assert abs(np.linalg.det(phi) - 1) < 1e-10
        np.testing.assert_allclose(phi.T @ J @ phi, J, atol=1e-9)


def test_stm_matches_state_finite_differences(orc):
    case = synth.survey_case(n_obj=3, n_frames=0, neo_frac=0.34)
    for s in case.x0:
        _, phi = orc.stm(case.ephem, s, 0.0, 40.0)
        fd = np.zeros((6, 6))
        for c in range(6):
            # steps well above the noise of the adaptive step control (1e-7 au
            # and 1e-9 au/day sat at the tolerance) and well below curvature
            h = 1e-6 if c < 3 else 1e-8
            sp = s.copy(); sp[c] += h
            sm = s.copy(); sm[c] -= h
            xp, _, _ = orc.propagate(case.ephem, sp[None], 0.0, [40.0], h_max=0.5)
            xm, _, _ = orc.propagate(case.ephem, sm[None], 0.0, [40.0], h_max=0.5)
            fd[:, c] = (xp[0, 0] - xm[0, 0]) / (2 * h)
        np.testing.assert_allclose(phi, fd, rtol=2e-5, atol=2e-7)


def test_loss_gradient_vs_frozen_step_fd(orc):
    g = synth.gradient_case(n_obj=4, k_obs=6, arc=30.0)
    for j in range(4):
        args = (g.ephem, g.x0[j], 0.0, g.t_obs[j], g.obs_pos[j], g.radec_obs[j])
        _, _, grad, st = orc.sky_grad(g.ephem, g.x0[j:j + 1], 0.0, g.t_obs[j:j + 1], g.obs_pos[j:j + 1],
                                      g.radec_obs[j:j + 1])
        assert st[0] == 0
        L0, steps = orc.loss_steps(*args)
        fd = np.zeros(6)
        for c in range(6):
            h = 1e-8 if c < 3 else 1e-10
            xp = g.x0[j].copy(); xp[c] += h
            xm = g.x0[j].copy(); xm[c] -= h
            Lp, _ = orc.loss_steps(g.ephem, xp, 0.0, g.t_obs[j], g.obs_pos[j], g.radec_obs[j], replay=steps)
            Lm, _ = orc.loss_steps(g.ephem, xm, 0.0, g.t_obs[j], g.obs_pos[j], g.radec_obs[j], replay=steps)
            fd[c] = (Lp - Lm) / (2 * h)
        np.testing.assert_allclose(grad[0], fd, rtol=1e-6, atol=1e-6 * np.max(np.abs(fd)))


# ---------------------------------------------------------------- RA/Dec and residual
OBLIQ = math.radians(84381.448 / 3600.0)     # IAU 1980 J2000 mean obliquity


def test_radec_closed_forms(orc):
    """Ecliptic J2000 -> equatorial RA/Dec: the equinox direction is
    (0, 0); the ecliptic +y axis is the point of the ecliptic at longitude
    90 deg, which lies at RA 90 deg and Dec +eps; the ecliptic north pole is
    at RA 270 deg, Dec 90 deg - eps; the equatorial north pole written in
    ecliptic coordinates, (0, sin eps, cos eps), has Dec 90 deg.  A wrong
    obliquity sign, a swapped axis or a missing RA wrap fails one of these."""
    e = OBLIQ
    cases = [((1.0, 0.0, 0.0), 0.0, 0.0),
             ((0.0, 1.0, 0.0), math.pi / 2, e),
             ((0.0, 0.0, 1.0), 3 * math.pi / 2, math.pi / 2 - e),
             ((-1.0, 0.0, 0.0), math.pi, 0.0),
             ((0.0, -1.0, 0.0), 3 * math.pi / 2, -e)]
    for d, ra0, dec0 in cases:
        for scale in (1.0, 3.7):          # the length of d does not matter
            ra, dec, _ = orc.radec(np.array(d) * scale)
            assert abs(ra - ra0) < 1e-15 and abs(dec - dec0) < 1e-15, (d, ra, dec)
    ra, dec, _ = orc.radec(np.array([0.0, math.sin(e), math.cos(e)]))
    assert abs(dec - math.pi / 2) < 1e-8
    # RA lies in [0, 2 pi): a direction just below the equinox on the equator
    ra, dec, _ = orc.radec(np.array([1.0, -1e-9 * math.cos(e), 1e-9 * math.sin(e)]))
    assert 2 * math.pi - 2e-9 < ra < 2 * math.pi and abs(dec) < 1e-15
    # a point of the ecliptic at longitude lam: sin(dec) = sin(eps) sin(lam),
    # tan(ra) = cos(eps) tan(lam) (spherical trigonometry of the ecliptic)
    for lam in np.linspace(0.1, 6.2, 17):
        ra, dec, _ = orc.radec(np.array([math.cos(lam), math.sin(lam), 0.0]))
        assert abs(math.sin(dec) - math.sin(e) * math.sin(lam)) < 1e-15
        assert abs(math.sin(ra) * math.cos(lam) - math.cos(e) * math.sin(lam) * math.cos(ra)) < 1e-15
        assert (ra < math.pi) == (math.sin(lam) > 0)


def test_radec_jacobian_matches_finite_differences(orc):
    rng = np.random.default_rng(61)
    for _ in range(20):
        d = rng.normal(size=3) * rng.uniform(0.5, 4.0)
        _, _, J = orc.radec(d)
        num = np.zeros((2, 3))
        for i in range(3):
            h = 1e-6 * np.linalg.norm(d)
            dp, dm = d.copy(), d.copy()
            dp[i] += h
            dm[i] -= h
            rp, xp, _ = orc.radec(dp)
            rm, xm, _ = orc.radec(dm)
            dra = (rp - rm + math.pi) % (2 * math.pi) - math.pi
            num[:, i] = [dra / (2 * h), (xp - xm) / (2 * h)]
        assert np.abs(num - J).max() < 1e-7 * np.abs(J).max()


def test_sky_residual_wraps_across_ra_zero(orc):
    """r = ((ra - ra_obs) cos dec, dec - dec_obs) with the RA difference in
    (-pi, pi]: two points 2 microradians apart across RA = 0 are 2 urad
    apart, not 2 pi; the cos(dec) factor uses the computed declination."""
    dec = 0.7
    r = orc.sky_residual(2 * math.pi - 1e-6, dec, 1e-6, dec - 3e-7)
    # (2 pi - 1e-6 carries the rounding of 2 pi, a few 1e-16)
    assert abs(r[0] - (-2e-6 * math.cos(dec))) < 1e-15 and abs(r[1] - 3e-7) < 1e-15
    r = orc.sky_residual(1e-6, -dec, 2 * math.pi - 1e-6, -dec)
    assert abs(r[0] - 2e-6 * math.cos(dec)) < 1e-15 and r[1] == 0.0
    r = orc.sky_residual(math.pi + 0.1, 0.0, 0.0, 0.0)
    assert abs(r[0] - (0.1 - math.pi)) < 1e-15
    r = orc.sky_residual(1.0, 0.2, 1.0, 0.2)
    assert r[0] == 0.0 and r[1] == 0.0


def test_kepler_iteration_cap_reports_failure(orc):
    """Host-forced non-convergence: with one Newton iteration allowed the
    universal-variable solve reports KEPLER_NOCONV; the membership test
    then drops every pair of such an object and reports its status; with
    the default cap nothing fails."""
    case = synth.tiny_case(n_obj=200, n_frames=20, n_targeted=60)
    fr = case.frames
    order, off, t_ref = orc.make_batches(fr.t)
    xe, st, _ = orc.propagate(case.ephem, case.x0, 0.0, t_ref)
    r0 = xe[0, 0, :3] - orc.cheb(case.ephem, 0, t_ref[0])[1]
    v0 = xe[0, 0, 3:] - orc.cheb(case.ephem, 0, t_ref[0])[2]
    mu = float(case.ephem.gm[0])
    assert orc.kepler(mu, r0, v0, 1.2)[0] == orc.ST_OK
    base = orc.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals, return_status=True)
    assert len(base[0]) > 20 and not base[4].any()
    try:
        orc.set_kepler_max_iter(1)
        assert orc.kepler(mu, r0, v0, 1.2)[0] == orc.ST_KEPLER_NOCONV
        assert orc.kepler(mu, r0, v0, 0.0)[0] == orc.ST_OK          # no hop, nothing to solve
        capped = orc.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals, return_status=True)
    finally:
        orc.set_kepler_max_iter(0)
    assert len(capped[0]) == 0
    assert np.all(capped[4] == orc.ST_KEPLER_NOCONV)
    again = orc.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals)
    assert len(again[0]) == len(base[0])


# ---------------------------------------------------------------- RADAU predictor
def test_predictor_reexpands_the_polynomial(orc):
    """b' from predict_b describes the same acceleration polynomial about
    the step end: a(1 + q sigma) - a(1) = sum_k b'_k sigma^(k+1) for any
    sigma, checked by evaluating both sides as plain polynomials."""
    rng = np.random.default_rng(71)
    for _ in range(20):
        b = rng.normal(size=7)
        q = rng.uniform(0.1, 3.0)
        bn = orc.predict_b(b, q)
        a = lambda s: sum(b[j] * s ** (j + 1) for j in range(7))
        for sig in rng.uniform(0.0, 1.0, 5):
            lhs = a(1.0 + q * sig) - a(1.0)
            rhs = sum(bn[k] * sig ** (k + 1) for k in range(7))
            assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs)) * (1 + q) ** 7
    # q = 1, b = e_6: (1 + sigma)^7 - 1 has the binomial coefficients 7, 21, 35, 35, 21, 7, 1
    e6 = np.zeros(7); e6[6] = 1.0
    np.testing.assert_array_equal(orc.predict_b(e6, 1.0), [7, 21, 35, 35, 21, 7, 1])


def test_predictor_start_reaches_the_same_solution(orc):
    """Starting each corrector from the extrapolated polynomial changes the
    number of sweeps, not the collocation solution: one year of survey-like
    bodies agrees with the zero start (the paper's) within 1e-12 au, with
    far fewer sweeps per step."""
    case = synth.survey_case(n_obj=120, n_frames=0, neo_frac=0.25)
    t_out = [365.25]
    xz, sz, stz = orc.propagate(case.ephem, case.x0, 0.0, t_out)
    xp, sp, stp = orc.propagate(case.ephem, case.x0, 0.0, t_out, opts=orc.make_opts(extrapolate=1))
    assert not sz.any() and not sp.any()
    err = np.abs(xz[..., :3] - xp[..., :3]).max()
    sw_z, sw_p = stz[1] / stz[0], stp[1] / stp[0]
    print(f"zero start {stz[0]} steps {sw_z:.2f} sweeps/step; extrapolated {stp[0]} steps {sw_p:.2f} "
          f"sweeps/step ({stp[4]} predicted); max |dx| {err:.2e} au")
    assert err < 1e-12
    assert stz[4] == 0 and stp[4] > 0.9 * stp[0]
    assert sw_p < 0.7 * sw_z
