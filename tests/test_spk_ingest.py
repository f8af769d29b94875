"""SPK ingest (Sect. 3.2: perturbers from precomputed kernels): type-2 and
type-3 files written from the analytic planet model with per-body record
lengths and degrees, in the equatorial J2000 frame (NAIF frame 1, as in
DE440) or the ecliptic J2000 frame (17), read back, rotated to the
ecliptic frame the library integrates in (App. A.1), chained to the
barycentre and resampled into the library's uniform table.  The fixtures
are fitted here with numpy's own Chebyshev routines and rotated to the
equator with this file's own rotation; the checks compare against the
analytic (ecliptic) model."""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npc

from paper_2509_04666_amd import spk, synth

DAY = 86400.0


EPS = math.radians(84381.448 / 3600.0)


def _to_equatorial(p):
    """Ecliptic J2000 vectors [..., 3] (or position-velocity [..., 6]) in the
    equatorial J2000 frame: the ecliptic north pole goes to
    (0, -sin eps, cos eps)."""
    p = np.asarray(p, float)
    out = p.copy()
    for k in range(0, p.shape[-1], 3):
        y, z = p[..., k + 1], p[..., k + 2]
        out[..., k + 1] = math.cos(EPS) * y - math.sin(EPS) * z
        out[..., k + 2] = math.sin(EPS) * y + math.cos(EPS) * z
    return out


def _fit_records(fun, t0_day, t1_day, rec_days, deg, frame):
    """Type-2 records (fun -> km [..., 3]) or type-3 records (fun -> km and
    km/s [..., 6]) of fun(t_days) over [t0, t1], labelled with `frame`."""
    n = int(math.ceil((t1_day - t0_day) / rec_days))
    x = np.cos(np.pi * (np.arange(4 * deg) + 0.5) / (4 * deg))
    coef = None
    for i in range(n):
        a = t0_day + i * rec_days
        p = fun(a + 0.5 * rec_days * (x + 1.0))
        if coef is None:
            coef = np.empty((n, p.shape[-1], deg + 1))
        for c in range(p.shape[-1]):
            coef[i, c] = npc.chebfit(x, p[:, c], deg)
    return dict(init=t0_day * DAY, intlen=rec_days * DAY, coef=coef, frame=frame)


def test_equatorial_to_ecliptic_closed_forms():
    """The equator's north pole lies at ecliptic (0, sin eps, cos eps); the
    ecliptic pole at equatorial (0, -sin eps, cos eps); the equinox stays."""
    from paper_2509_04666_amd import spk as S
    got = S.equatorial_to_ecliptic(np.array([[0.0, 0.0, 1.0], [0.0, -math.sin(EPS), math.cos(EPS)],
                                             [1.0, 0.0, 0.0]]))
    np.testing.assert_allclose(got, [[0.0, math.sin(EPS), math.cos(EPS)], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]],
                               atol=1e-16)


@pytest.fixture(scope="module")
def fixture_file(tmp_path_factory):
    model = synth.PlanetModel.make()
    bary = lambda t: model.bary(t)[..., :3] * spk.AU_KM          # [..., body, 3] km
    idx = {n: i for i, n in enumerate(model.names)}
    # Earth-Moon barycentre = Earth + a small circular offset; Earth stored relative to it
    off = lambda t: np.stack([4e-5 * np.cos(2 * np.pi * t / 27.3), 4e-5 * np.sin(2 * np.pi * t / 27.3),
                              0 * t], -1) * spk.AU_KM
    # Jupiter as a type-3 segment: positions (km) and velocities (km/s)
    bary6 = lambda t: np.concatenate([model.bary(t)[..., :3] * spk.AU_KM,
                                      model.bary(t)[..., 3:] * spk.AU_KM / DAY], -1)
    eq = lambda f: (lambda t: _to_equatorial(f(t)))
    t0, t1 = -40.0, 140.0
    # DE440-like: equatorial J2000 (frame 1), except Mercury in ecliptic J2000 (frame 17)
    segs = [dict(target=10, center=0, **_fit_records(eq(lambda t: bary(t)[:, idx["sun"]]), t0, t1, 16.0, 11, 1)),
            dict(target=1, center=0, **_fit_records(lambda t: bary(t)[:, idx["mercury"]], t0, t1, 4.0, 10, 17)),
            dict(target=3, center=0, **_fit_records(eq(lambda t: bary(t)[:, idx["earth"]] + off(t)), t0, t1, 8.0,
                                                    12, 1)),
            dict(target=399, center=3, **_fit_records(eq(lambda t: -off(t)), t0, t1, 4.0, 12, 1)),
            dict(target=5, center=0, **_fit_records(eq(lambda t: bary6(t)[:, idx["jupiter"]]), t0, t1, 32.0, 9,
                                                    1))]
    path = str(tmp_path_factory.mktemp("spk") / "planets.bsp")
    spk.write_spk(path, segs)
    return path, model


def test_spk_round_trip_and_chaining(fixture_file):
    path, model = fixture_file
    segs = spk.read_segments(path)
    assert [(s.target, s.center, s.dtype, s.frame) for s in segs] == [(10, 0, 2, 1), (1, 0, 2, 17), (3, 0, 2, 1),
                                                                     (399, 3, 2, 1), (5, 0, 3, 1)]
    names = ["sun", "mercury", "earth", "jupiter"]
    sel = [model.names.index(n) for n in names]
    eph = spk.load_spk([path], [10, 1, 399, 5], model.gm[sel], -8.0, 120.0, names=names)
    assert eph.coef.shape == (4, 16, 3, synth.CHEB_DEGREE + 1)
    assert eph.flags.tolist() == [1, 0, 1, 1]
    t = np.random.default_rng(60).uniform(-8.0, 120.0, 400)
    seg = np.minimum(((t - eph.t_start) // eph.seg_days).astype(int), eph.n_seg - 1)
    tau = 2.0 * (t - (eph.t_start + seg * eph.seg_days)) / eph.seg_days - 1.0
    ref = model.bary(t)[..., :3]
    worst = 0.0
    for b, i in enumerate(sel):
        got = np.stack([npc.chebval(tau[q], eph.coef[b, seg[q], :, :].T) for q in range(t.size)])
        worst = max(worst, np.abs(got - ref[:, i]).max())
    # the Earth came through its barycentre chain: the offset cancels; the
    # equatorial segments came back to the ecliptic.  The bound is the two
    # Chebyshev fits (file records, then 8-day degree-12 segments) of
    # Mercury's orbit, about 1e-12 au
    print(f"ingested table vs analytic model: max |dx| {worst:.3e} au")
    assert worst < 1e-11, worst


def test_spk_errors(fixture_file, tmp_path):
    path, model = fixture_file
    with pytest.raises(ValueError):
        spk.load_spk([path], [10, 6], model.gm[:2], -8.0, 120.0)           # no Saturn segment
    with pytest.raises(ValueError):
        spk.load_spk([path], [10], model.gm[:1], -8.0, 400.0)              # beyond the coverage
    # a frame the reader does not know (13: galactic) is refused
    gal = tmp_path / "galactic.bsp"
    spk.write_spk(str(gal), [dict(target=10, center=0, init=0.0, intlen=8 * DAY, coef=np.zeros((4, 3, 5)), frame=13)])
    with pytest.raises(ValueError, match="frame 13"):
        spk.load_spk([str(gal)], [10], model.gm[:1], 0.0, 16.0)
    # type-3 velocities ride along: the reader keeps positions only
    s3 = [sg for sg in spk.read_segments(path) if sg.dtype == 3][0]
    assert s3.n_comp == 6 and s3.coef.shape[1] == 6
    bad = tmp_path / "bad.bsp"
    bad.write_bytes(b"NAIF/DAF" + bytes(2048))
    with pytest.raises(ValueError):
        spk.read_segments(str(bad))


@pytest.mark.gpu
def test_spk_ephemeris_drives_the_gpu_path(fixture_file, orc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_04666_amd import api
    path, model = fixture_file
    names = ["sun", "mercury", "earth", "jupiter"]
    sel = [model.names.index(n) for n in names]
    eph = spk.load_spk([path], [10, 1, 399, 5], model.gm[sel], -8.0, 120.0, names=names)
    rng = np.random.default_rng(61)
    x0 = synth.bodies_from_elements(model, synth.main_belt_elements(rng, 300), 0.0)
    t_out = np.arange(2.0, 100.0, 7.0)
    xg, sg = api.propagate(api.DeviceEphemeris.from_synth(eph), torch.as_tensor(x0, device="cuda"), 0.0, t_out)
    xo, so, _ = orc.propagate(eph, x0, 0.0, t_out)
    assert np.all(sg.cpu().numpy() == 0) and np.all(so == 0)
    assert np.abs(xg.cpu().numpy()[..., :3] - xo[..., :3]).max() < 1e-10
