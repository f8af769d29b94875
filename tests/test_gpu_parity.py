"""GPU parity tests: every kernel of the path, called through the C ABI,
against the CPU oracle on the same seeded inputs.

Tolerances: positions within 1e-10 au after a year of integration; the
light-time direction from a given state within 1e-12 rad; pair sets
identical except pairs whose oracle edge distance is below 1 mas."""
import dataclasses
import math
import sys

import numpy as np
import pytest

from paper_2509_04666_amd import synth

pytestmark = pytest.mark.gpu

MAS = math.radians(1.0 / 3.6e6)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_04666_amd import api
    return torch, api


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev_x(torch, x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


# ---------------------------------------------------------------- ephemeris
def test_ephem_eval_matches_oracle(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.survey_case(n_obj=1, n_frames=0)
    e = case.ephem
    rng = np.random.default_rng(11)
    joints = e.t_start + e.seg_days * np.arange(1, e.n_seg)
    t = np.concatenate([rng.uniform(e.t_start, e.t_end, 300), joints, [e.t_start, e.t_end]])
    out = api.ephem_eval(api.DeviceEphemeris.from_synth(e), t).cpu().numpy()
    err_p = err_v = 0.0
    for q, tq in enumerate(t):
        for b in range(e.n_body):
            st, p, v = orc.cheb(e, b, tq)
            assert st == 0
            err_p = max(err_p, np.max(np.abs(out[q, b, :3] - p)))
            err_v = max(err_v, np.max(np.abs(out[q, b, 3:] - v)))
    _say(f"ephem max |dp| {err_p:.3e} au, |dv| {err_v:.3e} au/d")
    assert err_p < 1e-13 and err_v < 1e-14


# ---------------------------------------------------------------- light time
def test_lighttime_matches_oracle(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.survey_case(n_obj=300, n_frames=0, neo_frac=0.2)
    rng = np.random.default_rng(12)
    t_ref = 40.0
    xs, st, _ = orc.propagate(case.ephem, case.x0, 0.0, [t_ref])
    states = xs[0]
    t_obs = t_ref + rng.uniform(-1.6, 1.6, 12)
    obs = synth.circular_observer(case.model, t_obs)
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    d, tau = api.lighttime_directions(eph, _dev_x(torch, states), t_ref, _dev_x(torch, t_obs), _dev_x(torch, obs))
    d = d.cpu().numpy(); tau = tau.cpu().numpy()
    worst_ang = worst_tau = 0.0
    for q in range(t_obs.size):
        dref, tref = orc.directions(case.ephem, states, t_ref, t_obs[q], obs[q])
        cosang = np.sum(d[q] * dref, 1) / np.linalg.norm(d[q], axis=1) / np.linalg.norm(dref, axis=1)
        ang = np.arccos(np.clip(cosang, -1, 1))
        cr = np.linalg.norm(np.cross(d[q], dref), axis=1) / np.linalg.norm(d[q], axis=1) / np.linalg.norm(dref, axis=1)
        worst_ang = max(worst_ang, np.max(np.minimum(ang, cr)))
        worst_tau = max(worst_tau, np.max(np.abs(tau[q] - tref)))
        np.testing.assert_allclose(d[q], dref, rtol=0, atol=1e-13)
    _say(f"light-time max angle {worst_ang:.3e} rad, max |dtau| {worst_tau:.3e} d")
    assert worst_ang < 1e-12 and worst_tau < 1e-15


def test_lighttime_extreme_geometries(torch_cuda, orc):
    """Bodies far and near, slow and fast, and hops of up to 8 days: distant
    (40 au) and very distant (400 au) bodies, bodies 0.002 au from the
    observer, a Sun-grazer near perihelion and fast hyperbolic bodies.  The
    light time reaches 2.3 days for the farthest; the directions must match
    the oracle's plain iteration to the same bar as the survey bodies."""
    torch, api = torch_cuda
    case = synth.survey_case(n_obj=1, n_frames=0)
    rng = np.random.default_rng(13)
    t_ref = 40.0
    gm = synth.GM_SUN
    sun = case.model.sun(np.array([t_ref]))[0]
    rows = []
    def add(r, v):
        rows.append(np.concatenate([np.asarray(r, float) + sun[:3], np.asarray(v, float) + sun[3:]]))
    for dist in (40.0, 400.0):
        for _ in range(8):
            u = rng.normal(size=3); u /= np.linalg.norm(u)
            w = np.cross(u, rng.normal(size=3)); w /= np.linalg.norm(w)
            add(dist * u, math.sqrt(gm / dist) * w * rng.uniform(0.5, 1.3))
    for _ in range(8):                                   # fast hyperbolic bodies at 1-3 au
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        w = rng.normal(size=3); w /= np.linalg.norm(w)
        add(rng.uniform(1.0, 3.0) * u, rng.uniform(0.03, 0.08) * w)
    for _ in range(4):                                   # Sun-grazers near perihelion
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        w = np.cross(u, rng.normal(size=3)); w /= np.linalg.norm(w)
        q = rng.uniform(0.02, 0.1)
        add(q * u, math.sqrt(1.9 * gm / q) * w)
    t_obs = t_ref + np.concatenate([rng.uniform(-8.0, 8.0, 6), [0.0, 1e-9]])
    obs = synth.circular_observer(case.model, t_obs)
    o_ref = synth.circular_observer(case.model, np.array([t_ref]))[0]
    for _ in range(6):                                   # bodies 0.002 au from the observer at t_ref
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        w = rng.normal(size=3); w /= np.linalg.norm(w)
        rows.append(np.concatenate([o_ref + 0.002 * u, sun[3:] + 0.02 * w]))
    states = np.array(rows)
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    d, tau = api.lighttime_directions(eph, _dev_x(torch, states), t_ref, _dev_x(torch, t_obs), _dev_x(torch, obs))
    d = d.cpu().numpy(); tau = tau.cpu().numpy()
    worst_ang = worst_tau = 0.0
    for q in range(t_obs.size):
        dref, tref = orc.directions(case.ephem, states, t_ref, t_obs[q], obs[q])
        assert np.all(np.isfinite(dref)) and np.all(np.isfinite(d[q]))
        n1, n2 = np.linalg.norm(d[q], axis=1), np.linalg.norm(dref, axis=1)
        cr = np.linalg.norm(np.cross(d[q], dref), axis=1) / n1 / n2
        worst_ang = max(worst_ang, float(np.max(cr)))
        worst_tau = max(worst_tau, float(np.max(np.abs(tau[q] - tref))))
        np.testing.assert_allclose(d[q], dref, rtol=1e-14, atol=1e-13)
    _say(f"light-time (extreme geometries) max angle {worst_ang:.3e} rad, max |dtau| {worst_tau:.3e} d, "
         f"max tau {tau.max():.3f} d")
    assert worst_ang < 1e-12 and worst_tau < 3e-15


# ---------------------------------------------------------------- propagation
def _propagate_both(torch, api, orc, ephem, x0, t0, t_out, **opts):
    eph = api.DeviceEphemeris.from_synth(ephem)
    o = api.default_opts(**opts)
    xg, sg = api.propagate(eph, _dev_x(torch, x0), t0, t_out, o)
    xo, so, _ = orc.propagate(ephem, x0, t0, t_out)
    return xg.cpu().numpy(), sg.cpu().numpy(), xo, so


def test_propagate_sun_only_one_year(torch_cuda, orc):
    torch, api = torch_cuda
    rng = np.random.default_rng(13)
    el = np.concatenate([synth.main_belt_elements(rng, 200), synth.neo_elements(rng, 56)])
    x0 = synth.elements_to_state(*[el[:, k] for k in range(6)], synth.GM_SUN)
    eph = synth.sun_only_ephemeris(-8.0, 60)
    t_out = np.arange(30.0, 366.0, 30.0)
    xg, sg, xo, so = _propagate_both(torch, api, orc, eph, x0, 0.0, t_out)
    assert np.all(sg == 0) and np.all(so == 0)
    err = np.max(np.abs(xg[..., :3] - xo[..., :3]))
    _say(f"sun-only 1 yr max |dx| {err:.3e} au")
    assert err < 1e-10


def test_propagate_j2_enlarged(torch_cuda, orc):
    # Eq. A.4 (App. A.3): an oblate Sun with J2 and radius enlarged so that
    # the term moves close-in bodies far beyond the tolerance, about a
    # tilted pole; the post-Newtonian term on as well
    torch, api = torch_cuda
    rng = np.random.default_rng(31)
    pole = rng.normal(size=3)
    pole /= np.linalg.norm(pole)
    eph = synth.sun_only_ephemeris(-8.0, 45, gr=True, j2=(1e-2, 0.02, pole))
    el = synth.main_belt_elements(rng, 256)
    el[:, 0] = rng.uniform(0.15, 0.8, 256)
    x0 = synth.elements_to_state(*[el[:, k] for k in range(6)], synth.GM_SUN)
    t_out = np.arange(10.0, 340.0, 15.0)
    xg, sg, xo, so = _propagate_both(torch, api, orc, eph, x0, 0.0, t_out)
    assert np.all(sg == 0) and np.all(so == 0)
    err = np.max(np.abs(xg[..., :3] - xo[..., :3]))
    xn, _ = api.propagate(api.DeviceEphemeris.from_synth(synth.sun_only_ephemeris(-8.0, 45, gr=True)),
                          torch.as_tensor(x0).cuda(), 0.0, t_out)
    shift = np.max(np.abs(xn.cpu().numpy()[..., :3] - xg[..., :3]))
    _say(f"enlarged solar J2, 330 d: max |dx| vs oracle {err:.3e} au, J2 shift {shift:.3e} au")
    assert err < 1e-10
    assert shift > 1e-4


def test_propagate_default_model_j2_moon(torch_cuda, orc):
    # the default force model: Sun, planets and the Moon, the Eq. A.3 term
    # for the Sun, Jupiter and the Earth, Eq. A.4 for the Sun and Jupiter;
    # bodies passing close to Jupiter and to the Earth-Moon system
    torch, api = torch_cuda
    model = synth.PlanetModel.make()
    assert model.names[-1] == "moon"
    eph = synth.make_ephemeris(model, -8.0, 50)
    assert eph.j2 is not None and eph.j2[model.names.index("jupiter"), 0] > 0
    rng = np.random.default_rng(32)
    st = model.bary(np.array([100.0]))[0]
    near = []
    # hyperbolic flybys across the offset (closest approach near `dist`),
    # whose straight path keeps clear of the Earth and the Moon
    ie, im = model.names.index("earth"), model.names.index("moon")
    for nm, dist, n, speed in (("jupiter", 0.01, 24, 0.0225), ("earth", 0.003, 24, 5e-3), ("moon", 0.002, 16, 1e-2)):
        b = st[model.names.index(nm)]
        rows = []
        while len(rows) < n:
            off = rng.normal(size=3)
            if nm == "moon":                      # start on the far side from the Earth
                off = 0.3 * off + (b[:3] - st[ie, :3]) / np.linalg.norm(b[:3] - st[ie, :3])
            off *= dist / np.linalg.norm(off)
            dv = np.cross(off, rng.normal(size=3))
            dv *= speed / np.linalg.norm(dv)
            x = np.concatenate([b[:3] + off, b[3:] + dv])
            clear = True
            for k in (ie, im):
                rel, w = x[:3] - st[k, :3], x[3:] - st[k, 3:]
                s = max(0.0, -(rel @ w) / (w @ w))
                clear &= np.linalg.norm(rel + s * w) > 1e-3
            if clear:
                rows.append(x)
        near.append(np.array(rows))
    near = np.concatenate(near)
    far = synth.bodies_from_elements(model, synth.main_belt_elements(rng, 100), 100.0)
    x0 = np.concatenate([near, far])
    t_out = np.arange(103.0, 380.0, 12.0)
    xg, sg, xo, so = _propagate_both(torch, api, orc, eph, x0, 100.0, t_out)
    assert np.all(sg == 0) and np.all(so == 0)
    err = np.max(np.abs(xg[..., :3] - xo[..., :3]))
    _say(f"default model (10 bodies, J2, Moon), flybys of Jupiter, the Earth and the Moon: max |dx| {err:.3e} au")
    assert err < 1e-10


def test_propagate_tiny_config(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.tiny_case(n_obj=1000, n_frames=100)
    order, off, t_ref = orc.make_batches(case.frames.t)
    xg, sg, xo, so = _propagate_both(torch, api, orc, case.ephem, case.x0, 0.0, t_ref)
    assert np.all(sg == 0) and np.all(so == 0)
    err = np.max(np.abs(xg[..., :3] - xo[..., :3]))
    _say(f"tiny config ({t_ref.size} epochs) max |dx| {err:.3e} au")
    assert err < 1e-10


def test_propagate_survey_mix_one_year(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.survey_case(n_obj=3000, n_frames=0, neo_frac=0.05)
    t_out = np.arange(1.5, 365.25, 3.0)
    xg, sg, xo, so = _propagate_both(torch, api, orc, case.ephem, case.x0, 0.0, t_out)
    _say(f"survey mix 1 yr: status gpu {np.bincount(sg)}, oracle {np.bincount(so)}")
    np.testing.assert_array_equal(sg, so)
    ok = so == 0
    err = np.abs(xg[..., :3] - xo[..., :3]).max(axis=(0, 2))
    _say(f"survey mix 1 yr: max |dx| {err[ok].max():.3e} au over {ok.sum()} bodies")
    assert ok.all() and err.max() < 1e-10


@pytest.mark.parametrize("n_ast", [4, 7])
def test_propagate_extra_perturbers(torch_cuda, orc, n_ast):
    # Sun + 8 planets + the largest asteroids as extra perturbers: 13
    # bodies, and 16, the most the ABI takes (the run-time body count path)
    torch, api = torch_cuda
    model = synth.PlanetModel.make(synth.PLANET_NAMES + synth.ASTEROID_NAMES[:n_ast], moon=False)
    assert len(model.names) == 9 + n_ast
    eph = synth.make_ephemeris(model, -8.0, 20)
    rng = np.random.default_rng(16 + n_ast)
    x0 = synth.bodies_from_elements(model, np.concatenate([synth.main_belt_elements(rng, 600),
                                                           synth.neo_elements(rng, 30)]), 0.0)
    t_out = np.arange(1.5, 120.0, 3.0)
    xg, sg, xo, so = _propagate_both(torch, api, orc, eph, x0, 0.0, t_out)
    ok = (sg == 0) & (so == 0)
    assert ok.all()
    err = np.abs(xg[..., :3] - xo[..., :3]).max()
    # the asteroids move the bodies measurably against the planets alone
    xp, _ = api.propagate(api.DeviceEphemeris.from_synth(
        synth.make_ephemeris(synth.PlanetModel.make(moon=False), -8.0, 20)), _dev_x(torch, x0), 0.0, t_out)
    shift = np.abs(xp.cpu().numpy()[..., :3] - xg[..., :3]).max()
    _say(f"{len(model.names)} perturbers, 120 d: max |dx| vs oracle {err:.3e} au, shift from the asteroids "
         f"{shift:.3e} au")
    assert err < 1e-10
    assert shift > 1e-11


def test_propagate_backward(torch_cuda, orc):
    torch, api = torch_cuda
    model = synth.PlanetModel.make()
    e = synth.make_ephemeris(model, -216.0, 40)
    rng = np.random.default_rng(14)
    x0, _, _ = synth.make_population(rng, model, 500, 0.1, 0.0)
    t_out = np.array([-3.0, -50.0, -120.5, -200.0])
    xg, sg, xo, so = _propagate_both(torch, api, orc, e, x0, 0.0, t_out)
    assert np.all(sg == 0) and np.all(so == 0)
    err = np.max(np.abs(xg[..., :3] - xo[..., :3]))
    _say(f"backward 200 d max |dx| {err:.3e} au")
    assert err < 1e-10


def test_propagate_configuration_invariance(torch_cuda):
    torch, api = torch_cuda
    case = synth.survey_case(n_obj=777, n_frames=0, neo_frac=0.2)
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    x0 = _dev_x(torch, case.x0)
    t_out = np.arange(3.0, 100.0, 3.0)
    ref, st = api.propagate(eph, x0, 0.0, t_out, api.default_opts())
    ref2, _ = api.propagate(eph, x0, 0.0, t_out, api.default_opts())
    assert torch.equal(ref, ref2), "propagation is not deterministic"
    for kw in (dict(n_buckets=1), dict(block=64), dict(block=128, n_buckets=4), dict(rebucket_epochs=1),
               dict(window_segs=1), dict(rebucket_epochs=0), dict(rebucket_epochs=16), dict(lanes_per_body=7),
               dict(lanes_per_body=8), dict(lanes_per_body=7, block=256), dict(lanes_per_body=1),
               dict(zero_start=1), dict(zero_start=1, lanes_per_body=8)):
        x, s = api.propagate(eph, x0, 0.0, t_out, api.default_opts(**kw))
        d = (x - ref).abs().max().item()
        _say(f"config {kw}: max |dx| vs default {d:.3e}")
        assert d < 1e-11
        assert torch.equal(s, st)


def test_extrapolated_corrector_start(torch_cuda, orc):
    """The grouped integrators start each corrector from the previous
    step's increments extrapolated: nearly every step after the first is
    counted as predicted, the corrector needs fewer sweeps than from zero,
    and both starts agree with the oracle (which starts from zero)."""
    torch, api = torch_cuda
    case = synth.survey_case(n_obj=600, n_frames=0, neo_frac=0.2)
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    x0 = _dev_x(torch, case.x0)
    t_out = np.arange(3.0, 121.0, 3.0)
    xp, sp, stp = api.propagate(eph, x0, 0.0, t_out, api.default_opts(), stats=True)
    xz, sz, stz = api.propagate(eph, x0, 0.0, t_out, api.default_opts(zero_start=1), stats=True)
    stp, stz = stp.cpu().numpy(), stz.cpu().numpy()
    sweeps_p, sweeps_z = stp[4] / stp[3], stz[4] / stz[3]
    _say(f"sweeps per body-step: extrapolated start {sweeps_p:.2f}, zero start {sweeps_z:.2f}; "
         f"predicted steps {stp[7] / stp[3]:.3f}")
    assert stz[7] == 0
    assert stp[7] > 0.9 * stp[3]
    assert sweeps_p < 0.8 * sweeps_z
    assert torch.equal(sp, sz)
    sel = np.arange(0, 600, 25)
    xo, so, _ = orc.propagate(case.ephem, case.x0[sel], 0.0, t_out)
    for x in (xp, xz):
        xs = x[:, torch.as_tensor(sel, device="cuda")].cpu().numpy()
        assert np.max(np.abs(xs[..., :3] - xo[..., :3])) < 1e-10


def test_dense_epochs_match_landing(torch_cuda, orc):
    """Epochs read off the step polynomials (the default) against landing on
    every epoch and against the oracle, which lands: an epoch equal to the
    start, epochs a fraction of a step apart, backward integration and runs
    split over several launches."""
    torch, api = torch_cuda
    case = synth.survey_case(n_obj=300, n_frames=0, neo_frac=0.2)
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    x0 = _dev_x(torch, case.x0)
    sel = np.arange(0, 300, 7)
    for t0, t_out in ((0.0, [0.0, 0.7, 3.1, 3.2, 10.0, 17.5, 40.0, 61.25]), (30.0, [29.5, 21.0, 20.9, 2.0])):
        xd, sd, std = api.propagate(eph, x0, t0, t_out, api.default_opts(), stats=True)
        xl, sl, stl = api.propagate(eph, x0, t0, t_out, api.default_opts(land_epochs=1), stats=True)
        xr, sr = api.propagate(eph, x0, t0, t_out, api.default_opts(rebucket_epochs=3))
        assert torch.equal(sd, sl) and torch.equal(sd, sr)
        ok = (sd == 0).cpu().numpy()
        d_land = (xd - xl)[:, torch.as_tensor(ok, device="cuda")].abs().max().item()
        d_split = (xd - xr)[:, torch.as_tensor(ok, device="cuda")].abs().max().item()
        xo, so, _ = orc.propagate(case.ephem, case.x0[sel], t0, t_out)
        xs = xd[:, torch.as_tensor(sel, device="cuda")].cpu().numpy()
        d_orc = np.abs(xs[:, so == 0, :3] - xo[:, so == 0, :3]).max()
        _say(f"t0 {t0}: dense vs landing {d_land:.2e}, vs split launches {d_split:.2e}, vs oracle {d_orc:.2e} au; "
             f"body-steps {std.cpu().numpy()[3]} vs {stl.cpu().numpy()[3]} landing")
        assert d_land < 1e-11 and d_split < 1e-11 and d_orc < 1e-11
        assert std.cpu().numpy()[3] < stl.cpu().numpy()[3]
        # the epoch at the start time is the initial state itself
        if t_out[0] == t0:
            assert torch.equal(xd[0], x0)


def test_propagate_ragged_sizes(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.survey_case(n_obj=130, n_frames=0, neo_frac=0.3)
    t_out = [2.0, 9.5]
    for lanes in (7, 8, 1):
        for n in (1, 8, 9, 10, 17, 63, 65, 130):
            xg, sg, xo, so = _propagate_both(torch, api, orc, case.ephem, case.x0[:n], 0.0, t_out,
                                             lanes_per_body=lanes)
            assert np.max(np.abs(xg - xo)) < 1e-12, (lanes, n)
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    x, s = api.propagate(eph, torch.zeros((0, 6), dtype=torch.float64, device="cuda"), 0.0, t_out)
    assert x.shape == (2, 0, 6)


def test_propagate_status_codes(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.survey_case(n_obj=200, n_frames=0)
    x0 = case.x0.copy()
    x0[7] = np.nan
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    x, s = api.propagate(eph, _dev_x(torch, x0), 0.0, [10.0, 20.0])
    s = s.cpu().numpy(); x = x.cpu().numpy()
    assert s[7] == 1 and np.all(np.isnan(x[:, 7]))
    good = np.arange(200) != 7
    assert np.all(s[good] == 0)
    xo, so, _ = orc.propagate(case.ephem, case.x0[good], 0.0, [10.0, 20.0])
    assert np.max(np.abs(x[:, good] - xo)) < 1e-12
    _, s2 = api.propagate(eph, _dev_x(torch, case.x0), 0.0, [300.0], api.default_opts(max_steps=3))
    assert np.all(s2.cpu().numpy() == 3)
    _, s3 = api.propagate(eph, _dev_x(torch, case.x0), 0.0, [300.0], api.default_opts(h_min=200.0))
    assert np.all(s3.cpu().numpy() == 2)


# ---------------------------------------------------------------- FoV
def _pair_set(pf, ps, po):
    return set(zip(np.asarray(pf).tolist(), np.asarray(ps).tolist(), np.asarray(po).tolist()))


def _compare_pairs(gpu, orc_pairs, edge, label):
    g = _pair_set(*gpu)
    o = _pair_set(*orc_pairs)
    near = {k for k, e in zip(zip(*[np.asarray(a).tolist() for a in orc_pairs]), edge) if abs(e) < MAS}
    missing = o - g - near
    extra = g - o
    _say(f"{label}: oracle {len(o)} pairs, gpu {len(g)}, missing {len(missing)}, extra {len(extra)}")
    assert not missing, sorted(missing)[:10]
    # an extra GPU pair must sit within 1 mas of an edge of its frame
    return extra


def _edge_of(orc, ephem, x_epoch, order, off, t_ref, fr, pair):
    f, s, j = pair
    q = int(np.nonzero(order == f)[0][0])
    b = int(np.searchsorted(off, q, side="right") - 1)
    st, d, tau, _ = orc.lighttime(ephem, t_ref[b], x_epoch[b, j], fr.t[f], fr.obs[f])
    ins, edge = orc.inside(fr.normals[f], d)
    return edge[s]


def _fov_case(torch, api, orc, case, x_epoch_host, order, off, t_ref, opts=None, status=None):
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    fr = api.DeviceFrames.from_synth(case.frames)
    b = api.Batches.from_host(order.astype(np.int32), off.astype(np.int32), t_ref)
    pf, ps, po, stats = api.fov_check(eph, _dev_x(torch, x_epoch_host), b, fr, status, opts, return_stats=True)
    _say(f"fov stats (candidates, exact, brute-force objects): {stats[:3].tolist()}")
    return pf.cpu().numpy(), ps.cpu().numpy(), po.cpu().numpy()


def test_fov_given_oracle_states(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.tiny_case(n_obj=1000, n_frames=100, n_targeted=400)
    fr = case.frames
    order, off, t_ref = orc.make_batches(fr.t)
    xe, st, _ = orc.propagate(case.ephem, case.x0, 0.0, t_ref)
    opairs = orc.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals)
    gp = _fov_case(torch, api, orc, case, xe, order, off, t_ref)
    assert np.all(np.diff(gp[0].astype(np.int64) * 2 ** 32 + gp[1].astype(np.int64) * 2 ** 25 + gp[2]) > 0)
    extra = _compare_pairs(gp, opairs[:3], opairs[3], "tiny+targeted given oracle states")
    for p in extra:
        assert abs(_edge_of(orc, case.ephem, xe, order, off, t_ref, fr, p)) < MAS
    assert len(opairs[0]) > 200


def test_fov_distant_bodies(torch_cuda, orc):
    """Bodies from 30 au to 400 au (light times up to 2.3 days, where the
    exact test's Sun cubic is re-expanded about each body's emission time)
    among main-belt bodies, with frames aimed at them: the pair sets must
    match the oracle's."""
    torch, api = torch_cuda
    case = synth.tiny_case(n_obj=600, n_frames=40)
    rng = np.random.default_rng(16)
    n_far = 240
    a = np.concatenate([rng.uniform(30.0, 60.0, n_far - 40), rng.uniform(150.0, 400.0, 40)])
    e = rng.uniform(0.0, 0.2, n_far)
    inc = rng.rayleigh(math.radians(10.0), n_far)
    ang = rng.uniform(0.0, 2.0 * np.pi, (3, n_far))
    el_far = np.stack([a, e, inc, ang[0], ang[1], ang[2]], axis=1)
    x_far = synth.bodies_from_elements(case.model, el_far, 0.0)
    x0 = np.concatenate([case.x0, x_far])
    fr = synth.Frames.concat([case.frames, synth.frames_targeted(rng, case.model, el_far, 0.0, case.span, 160)])
    fr = fr.subset(np.argsort(fr.t, kind="stable"))
    case = synth.PropagationCase("tiny-far", case.ephem, case.model, x0, None, np.zeros(x0.shape[0], bool), 0.0,
                                 case.span, fr, 16)
    order, off, t_ref = orc.make_batches(fr.t)
    xe, st, _ = orc.propagate(case.ephem, x0, 0.0, t_ref)
    opairs = orc.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals)
    gp = _fov_case(torch, api, orc, case, xe, order, off, t_ref)
    extra = _compare_pairs(gp, opairs[:3], opairs[3], "distant bodies given oracle states")
    for p in extra:
        assert abs(_edge_of(orc, case.ephem, xe, order, off, t_ref, fr, p)) < MAS
    far_pairs = int(np.sum(np.asarray(opairs[2]) >= 600))
    _say(f"pairs of the distant bodies: {far_pairs}")
    assert far_pairs > 100


def test_fov_full_chain_tiny(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.tiny_case(n_obj=1000, n_frames=100, n_targeted=300)
    fr = case.frames
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    pf, ps, po, xg, sg, bt = api.predict(eph, _dev_x(torch, case.x0), 0.0, api.DeviceFrames.from_synth(fr), fr.t)
    order, off, t_ref = orc.make_batches(fr.t)
    np.testing.assert_array_equal(bt.t_ref_host, t_ref)
    xe, st, _ = orc.propagate(case.ephem, case.x0, 0.0, t_ref)
    assert np.max(np.abs(xg.cpu().numpy() - xe)) < 1e-10
    opairs = orc.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals)
    extra = _compare_pairs((pf.cpu().numpy(), ps.cpu().numpy(), po.cpu().numpy()), opairs[:3], opairs[3],
                           "tiny full chain")
    for p in extra:
        assert abs(_edge_of(orc, case.ephem, xe, order, off, t_ref, fr, p)) < MAS


def test_fov_survey_geometry(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.survey_case(n_obj=20000, n_frames=20000, span=20.0, neo_frac=0.05)
    fr = case.frames
    order, off, t_ref = orc.make_batches(fr.t)
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    xg, sg = api.propagate(eph, _dev_x(torch, case.x0), 0.0, t_ref)
    b = api.Batches.from_host(order.astype(np.int32), off.astype(np.int32), t_ref)
    pf, ps, po, stats = api.fov_check(eph, xg, b, api.DeviceFrames.from_synth(fr), sg, return_stats=True)
    _say(f"survey geometry stats {stats.tolist()}, pairs {pf.numel()}")
    # oracle on a sample of objects, all frames
    rng = np.random.default_rng(15)
    sample = np.sort(rng.choice(case.x0.shape[0], 600, replace=False))
    xe, st, _ = orc.propagate(case.ephem, case.x0[sample], 0.0, t_ref)
    opf, ops, opo, oedge = orc.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals)
    opo = sample[opo]
    keep = np.isin(po.cpu().numpy(), sample)
    gp = (pf.cpu().numpy()[keep], ps.cpu().numpy()[keep], po.cpu().numpy()[keep])
    extra = _compare_pairs(gp, (opf, ops, opo), oedge, "survey geometry sample")
    # an extra GPU pair lies within 1 mas of an edge, measured from the oracle's states
    loc = {int(j): i for i, j in enumerate(sample)}
    for f, s, j in extra:
        assert abs(_edge_of(orc, case.ephem, xe, order, off, t_ref, fr, (f, s, loc[j]))) < MAS, (f, s, j)


def test_fov_capacity_and_empty(torch_cuda, orc):
    torch, api = torch_cuda
    from paper_2509_04666_amd import _lib
    case = synth.tiny_case(n_obj=500, n_frames=50, n_targeted=100)
    fr = case.frames
    order, off, t_ref = orc.make_batches(fr.t)
    xe, st, _ = orc.propagate(case.ephem, case.x0, 0.0, t_ref)
    opairs = orc.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals)
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    b = api.Batches.from_host(order.astype(np.int32), off.astype(np.int32), t_ref)
    with pytest.raises(_lib.KeteError) as e:
        api.fov_check(eph, _dev_x(torch, xe), b, api.DeviceFrames.from_synth(fr), pairs_cap=3)
    assert e.value.code == _lib.KETE_ECAPACITY
    # objects far from every frame: no pairs
    far = xe.copy()
    far[..., :3] += 500.0
    pf, ps, po = api.fov_check(eph, _dev_x(torch, far), b, api.DeviceFrames.from_synth(fr))
    assert pf.numel() == 0
    # failed objects are skipped
    status = torch.zeros(500, dtype=torch.int32, device="cuda")
    status[opairs[2]] = 1
    pf, ps, po = api.fov_check(eph, _dev_x(torch, xe), b, api.DeviceFrames.from_synth(fr), status)
    assert pf.numel() == 0


def test_kepler_cap_forced_from_the_host(torch_cuda, orc):
    """Host-forced non-convergence (kepler_iter = 1): every object whose
    hop the membership test needs (pairs the linear-motion bound leaves
    undecided) gets KETE_ST_KEPLER_NOCONV and loses all of its pairs, so
    what remains is a subset of the default run's pairs from unflagged
    objects only (the oracle, which hops every pair, fails everything with
    its own cap); magnitudes, light-time directions and the adjoint report
    NaN / the status; with the default cap nothing fails."""
    torch, api = torch_cuda
    from paper_2509_04666_amd import _lib
    case = synth.tiny_case(n_obj=400, n_frames=40, n_targeted=120)
    # 24 more frames, each with an edge through the oracle's apparent
    # direction of one body: no motion bound decides such a pair, so each
    # of these bodies needs a hop
    rng = np.random.default_rng(11)
    pick = rng.choice(400, 24, replace=False)
    te = rng.uniform(1.0, case.span - 1.0, 24)
    oe = synth.circular_observer(case.model, te)
    h = np.full(24, math.radians(0.75))
    nrm = np.zeros((24, 1, 4, 3))
    fr = synth.Frames.concat([case.frames, synth.Frames(te, oe, None, None, None, None, None, nrm)])
    srt = np.argsort(fr.t, kind="stable")
    fr = fr.subset(srt)
    order, off, t_ref = orc.make_batches(fr.t)
    xe, st, _ = orc.propagate(case.ephem, case.x0, 0.0, t_ref)
    pos = np.argsort(srt)[case.frames.t.size:]      # where the new frames went
    for k, f in enumerate(pos):
        b = int(np.searchsorted(off, int(np.nonzero(order == f)[0][0]), side="right") - 1)
        d = orc.lighttime(case.ephem, t_ref[b], xe[b, pick[k]], fr.t[f], fr.obs[f])[1]
        d = d / np.linalg.norm(d)
        e = synth.tangent_basis(d)[0]
        c = math.cos(h[k]) * d + math.sin(h[k]) * e
        u = math.cos(h[k]) * e - math.sin(h[k]) * d
        fr.normals[f, 0] = synth.rect_normals(c, u, np.cross(c, u), h[k], h[k])
        assert abs(fr.normals[f, 0, 1] @ d) < 1e-15
    case = dataclasses.replace(case, frames=fr)
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    dfr = api.DeviceFrames.from_synth(fr)
    b = api.Batches.from_host(order.astype(np.int32), off.astype(np.int32), t_ref)
    xd = _dev_x(torch, xe)
    s0 = torch.zeros(400, dtype=torch.int32, device="cuda")
    pf, ps, po = api.fov_check(eph, xd, b, dfr, s0)
    assert pf.numel() > 50 and int(s0.abs().sum()) == 0
    o = orc.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals, return_status=True)
    assert not o[4].any()
    _say(f"kepler cap: default run {pf.numel()} pairs (oracle {len(o[0])})")
    capped = api.default_opts(kepler_iter=1)
    s1 = torch.zeros(400, dtype=torch.int32, device="cuda")
    pf1, ps1, po1 = api.fov_check(eph, xd, b, dfr, s1, capped)
    s1h = s1.cpu().numpy()
    had = np.unique(po.cpu().numpy())
    _say(f"kepler cap 1: {pf1.numel()} pairs, {np.count_nonzero(s1h)} objects flagged, {had.size} had pairs")
    assert np.count_nonzero(s1h) > 0 and np.all(s1h[pick] != 0)
    assert set(np.unique(s1h).tolist()) <= {0, _lib.ST_KEPLER_NOCONV}
    kept = set(zip(pf1.cpu().tolist(), ps1.cpu().tolist(), po1.cpu().tolist()))
    assert kept <= set(zip(pf.cpu().tolist(), ps.cpu().tolist(), po.cpu().tolist()))
    assert all(s1h[j] == 0 for _, _, j in kept)
    # the same without a status array: the same pairs
    pf2, ps2, po2 = api.fov_check(eph, xd, b, dfr, None, capped)
    assert set(zip(pf2.cpu().tolist(), ps2.cpu().tolist(), po2.cpu().tolist())) == kept
    # magnitudes of the default run's pairs: NaN under the cap, finite without it
    H, G = synth.hg_params(np.random.default_rng(42), 400)
    Hd = torch.as_tensor(H, device="cuda")
    Gd = torch.as_tensor(G, device="cuda")
    v = api.pair_magnitudes(eph, xd, b, dfr, pf, po, Hd, Gd)
    v1 = api.pair_magnitudes(eph, xd, b, dfr, pf, po, Hd, Gd, opts=capped)
    assert torch.isfinite(v).all() and torch.isnan(v1).all()
    # light-time directions
    d, tau = api.lighttime_directions(eph, xd[0], float(t_ref[0]), torch.as_tensor(fr.t[:3], device="cuda"),
                                      torch.as_tensor(fr.obs[:3], device="cuda"), capped)
    assert torch.isnan(d).all() and torch.isnan(tau).all()
    # adjoint: every object's hops fail, so status NOCONV, NaN sky, zero gradient
    g = synth.gradient_case(n_obj=64, k_obs=5, arc=20.0)
    ctx = api.AdjointContext(api.DeviceEphemeris.from_synth(g.ephem), g.t0, g.arc,
                             torch.as_tensor(g.t_obs, device="cuda"), torch.as_tensor(g.obs_pos, device="cuda"),
                             5.0, capped)
    x0 = torch.as_tensor(g.x0, device="cuda").requires_grad_(True)
    sky = api.AdjointSky.apply(x0, ctx)
    assert torch.isnan(sky).all()
    assert np.all(ctx.status.cpu().numpy() == _lib.ST_KEPLER_NOCONV)
    sky.nan_to_num(0.0).sum().backward()
    assert torch.equal(x0.grad, torch.zeros_like(x0))


def _random_layout_frames(rng, fr, n_sub=16):
    """The frames of `fr` with their sub-frames replaced by n_sub
    rectangles of random size (0.2-1.5 deg half-sides), roll and place
    (within 4 deg of the frame centre): overlaps and gaps, no grid."""
    from paper_2509_04666_amd import synth as S
    F = fr.t.size
    # frame centre: the normalised sum of the first sub-frame's inward normals
    c = fr.normals[:, 0].sum(axis=1)
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    e, n = S.tangent_basis(c)
    out = np.empty((F, n_sub, 4, 3))
    for s in range(n_sub):
        off = rng.uniform(-np.radians(4.0), np.radians(4.0), (F, 2))
        cs = c + off[:, :1] * e + off[:, 1:] * n
        cs /= np.linalg.norm(cs, axis=1, keepdims=True)
        es, ns = S.tangent_basis(cs)
        roll = rng.uniform(0, np.pi, F)[:, None]
        u = np.cos(roll) * es + np.sin(roll) * ns
        w = -np.sin(roll) * es + np.cos(roll) * ns
        hu = np.radians(rng.uniform(0.2, 1.5, F))
        hw = np.radians(rng.uniform(0.2, 1.5, F))
        out[:, s] = S.rect_normals(cs, u, w, hu, hw)
    return S.Frames(fr.t, fr.obs, None, None, None, None, None, out)


def test_fov_multi_subframe_layouts(torch_cuda, orc):
    """Frames of many sub-frames, which the sub-frame locator prunes:
    ground footprints of 8 x 8 sub-frames, and the same frames with 16 or
    120 rectangles of random size, roll and place (overlapping, with gaps;
    120 fills both mask words and gives pairs more candidate sub-frames
    than the drains list in LDS), against the oracle's brute force, given
    the oracle's states."""
    torch, api = torch_cuda
    case = synth.footprint_case(n_obj=4000, n_frames=1500, span=12.0)
    layouts = [("footprints 8x8", case.frames),
               ("random 16", _random_layout_frames(np.random.default_rng(81), case.frames)),
               ("random 120", _random_layout_frames(np.random.default_rng(82), case.frames, n_sub=120))]
    order, off, t_ref = orc.make_batches(case.frames.t)
    xe, st, _ = orc.propagate(case.ephem, case.x0, 0.0, t_ref)
    assert not st.any()
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    b = api.Batches.from_host(order.astype(np.int32), off.astype(np.int32), t_ref)
    for label, fr in layouts:
        opf, ops, opo, oedge = orc.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals)
        pf, ps, po, stats = api.fov_check(eph, _dev_x(torch, xe), b, api.DeviceFrames.from_synth(fr), None,
                                          return_stats=True)
        _say(f"{label}: stats {stats.tolist()}")
        gp = (pf.cpu().numpy(), ps.cpu().numpy(), po.cpu().numpy())
        assert np.all(np.diff(gp[0].astype(np.int64) * 2 ** 32 + gp[1].astype(np.int64) * 2 ** 25 + gp[2]) > 0)
        extra = _compare_pairs(gp, (opf, ops, opo), oedge, label)
        for p in extra:
            assert abs(_edge_of(orc, case.ephem, xe, order, off, t_ref, fr, p)) < MAS
        assert len(opf) > 500
