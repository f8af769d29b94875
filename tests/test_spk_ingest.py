"""SPK ingest (Sect. 3.2: perturbers from precomputed kernels): type-2
files written from the analytic planet model with per-body record lengths
and degrees, read back, chained to the barycentre and resampled into the
library's uniform table.  The fixtures are fitted here with numpy's own
Chebyshev routines; the checks compare against the analytic model."""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npc

from paper_2509_04666_amd import spk, synth

DAY = 86400.0


def _fit_records(fun, t0_day, t1_day, rec_days, deg):
    """Type-2 records of fun(t_days) -> km [..., 3] over [t0, t1]."""
    n = int(math.ceil((t1_day - t0_day) / rec_days))
    coef = np.empty((n, 3, deg + 1))
    x = np.cos(np.pi * (np.arange(4 * deg) + 0.5) / (4 * deg))
    for i in range(n):
        a = t0_day + i * rec_days
        p = fun(a + 0.5 * rec_days * (x + 1.0))
        for c in range(3):
            coef[i, c] = npc.chebfit(x, p[:, c], deg)
    return dict(init=t0_day * DAY, intlen=rec_days * DAY, coef=coef)


@pytest.fixture(scope="module")
def fixture_file(tmp_path_factory):
    model = synth.PlanetModel.make()
    bary = lambda t: model.bary(t)[..., :3] * spk.AU_KM          # [..., body, 3] km
    idx = {n: i for i, n in enumerate(model.names)}
    # Earth-Moon barycentre = Earth + a small circular offset; Earth stored relative to it
    off = lambda t: np.stack([4e-5 * np.cos(2 * np.pi * t / 27.3), 4e-5 * np.sin(2 * np.pi * t / 27.3),
                              0 * t], -1) * spk.AU_KM
    t0, t1 = -40.0, 140.0
    segs = [dict(target=10, center=0, **_fit_records(lambda t: bary(t)[:, idx["sun"]], t0, t1, 16.0, 11)),
            dict(target=1, center=0, **_fit_records(lambda t: bary(t)[:, idx["mercury"]], t0, t1, 4.0, 10)),
            dict(target=3, center=0, **_fit_records(lambda t: bary(t)[:, idx["earth"]] + off(t), t0, t1, 8.0, 12)),
            dict(target=399, center=3, **_fit_records(lambda t: -off(t), t0, t1, 4.0, 12)),
            dict(target=5, center=0, **_fit_records(lambda t: bary(t)[:, idx["jupiter"]], t0, t1, 32.0, 9))]
    path = str(tmp_path_factory.mktemp("spk") / "planets.bsp")
    spk.write_spk(path, segs)
    return path, model


def test_spk_round_trip_and_chaining(fixture_file):
    path, model = fixture_file
    segs = spk.read_segments(path)
    assert [(s.target, s.center, s.dtype) for s in segs] == [(10, 0, 2), (1, 0, 2), (3, 0, 2), (399, 3, 2), (5, 0, 2)]
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
    # the Earth came through its barycentre chain: the offset cancels.  The
    # bound is the two Chebyshev fits (file records, then 8-day degree-12
    # segments) of Mercury's orbit, about 1e-12 au
    print(f"ingested table vs analytic model: max |dx| {worst:.3e} au")
    assert worst < 1e-11, worst


def test_spk_errors(fixture_file, tmp_path):
    path, model = fixture_file
    with pytest.raises(ValueError):
        spk.load_spk([path], [10, 6], model.gm[:2], -8.0, 120.0)           # no Saturn segment
    with pytest.raises(ValueError):
        spk.load_spk([path], [10], model.gm[:1], -8.0, 400.0)              # beyond the coverage
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
