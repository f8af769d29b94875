"""H-G magnitudes of the pairs (Sect. 3.3) through the C ABI against the
CPU oracle: on the oracle's own states (so only the magnitude step is
compared), along the full GPU chain, and on the degenerate inputs (pairs
in any order, pairs naming a frame outside every batch or an index out of
range, no pairs, a ragged count).

Tolerances: given the same states the two sides differ by rounding only:
1e-9 mag, 1e-11 au in r_H and Delta, 1e-10 rad in the phase angle.  Along
the chain the states themselves differ by up to 1e-10 au, which moves V
by 5 / ln 10 * 1e-10 / r in the distance term plus at most about 2e-9 mag
through the phase term at the smallest phase angles here: 1e-8 mag."""
import math
import sys

import numpy as np
import pytest

from paper_2509_04666_amd import synth

pytestmark = pytest.mark.gpu


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


def _dev(torch, a, dtype=None):
    import torch as _t
    return _t.as_tensor(np.ascontiguousarray(a), dtype=dtype or _t.float64).cuda()


def test_magnitudes_given_oracle_states(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.tiny_case(n_obj=1000, n_frames=100, n_targeted=400)
    fr = case.frames
    order, off, t_ref = orc.make_batches(fr.t)
    xe, st, _ = orc.propagate(case.ephem, case.x0, 0.0, t_ref)
    H, G = synth.hg_params(np.random.default_rng(40), case.x0.shape[0])
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    dfr = api.DeviceFrames.from_synth(fr)
    b = api.Batches.from_host(order.astype(np.int32), off.astype(np.int32), t_ref)
    xd = _dev(torch, xe)
    pf, ps, po = api.fov_check(eph, xd, b, dfr, _dev(torch, st, torch.int32))
    n = pf.numel()
    assert n > 200 and n % 256 != 0
    Hd, Gd = _dev(torch, H), _dev(torch, G)
    v, geom = api.pair_magnitudes(eph, xd, b, dfr, pf, po, Hd, Gd, geometry=True)
    torch.cuda.synchronize()
    ov, og = orc.pair_mags(case.ephem, xe, order, off, t_ref, fr.t, fr.obs, pf.cpu().numpy(), po.cpu().numpy(), H, G)
    vg, gg = v.cpu().numpy(), geom.cpu().numpy()
    dv = np.abs(vg - ov).max()
    _say(f"magnitudes of {n} pairs given oracle states: max |dV| {dv:.3e} mag, max |d r_H| "
         f"{np.abs(gg[:, 0] - og[:, 0]).max():.3e}, |d Delta| {np.abs(gg[:, 1] - og[:, 1]).max():.3e} au, "
         f"|d alpha| {np.abs(gg[:, 2] - og[:, 2]).max():.3e} rad; V in [{vg.min():.2f}, {vg.max():.2f}]")
    assert dv < 1e-9
    assert np.abs(gg[:, :2] - og[:, :2]).max() < 1e-11
    assert np.abs(gg[:, 2] - og[:, 2]).max() < 1e-10
    # the geometry-free call returns the same magnitudes
    v2 = api.pair_magnitudes(eph, xd, b, dfr, pf, po, Hd, Gd)
    assert torch.equal(v2, v)
    # pairs in another order: the same value per pair, bit for bit
    perm = torch.as_tensor(np.random.default_rng(41).permutation(n), device="cuda")
    vp = api.pair_magnitudes(eph, xd, b, dfr, pf[perm], po[perm], Hd, Gd)
    assert torch.equal(vp, v[perm])
    # a ragged prefix
    vr = api.pair_magnitudes(eph, xd, b, dfr, pf[:77], po[:77], Hd, Gd)
    assert torch.equal(vr, v[:77])


def test_magnitudes_degenerate_inputs(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.tiny_case(n_obj=50, n_frames=30)
    fr = case.frames
    order, off, t_ref = orc.make_batches(fr.t)
    xe, st, _ = orc.propagate(case.ephem, case.x0, 0.0, t_ref)
    H, G = synth.hg_params(np.random.default_rng(42), 50)
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    dfr = api.DeviceFrames.from_synth(fr)
    # drop the last batch's frames from the batch list: their pairs name no batch
    nb = t_ref.size - 1
    b = api.Batches.from_host(order[:off[nb]].astype(np.int32), off[:nb + 1].astype(np.int32), t_ref[:nb])
    last = int(order[off[nb]])
    first = int(order[0])
    F = fr.t.size
    pf = np.array([first, -1, F, first, last, first], np.int32)
    po = np.array([3, 3, 3, 50, 3, -2], np.int32)
    xd = _dev(torch, xe[:nb])
    v, geom = api.pair_magnitudes(eph, xd, b, dfr, _dev(torch, pf, torch.int32), _dev(torch, po, torch.int32),
                                  _dev(torch, H), _dev(torch, G), geometry=True)
    vg, gg = v.cpu().numpy(), geom.cpu().numpy()
    ov, og = orc.pair_mags(case.ephem, xe[:nb], order[:off[nb]], off[:nb + 1], t_ref[:nb], fr.t, fr.obs,
                           pf[:1], po[:1], H, G)
    assert abs(vg[0] - ov[0]) < 1e-9 and np.abs(gg[0] - og[0]).max() < 1e-10
    assert np.all(np.isnan(vg[1:])) and np.all(np.isnan(gg[1:]))
    # no pairs: nothing to do, no error
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    assert api.pair_magnitudes(eph, xd, b, dfr, e, e, _dev(torch, H), _dev(torch, G)).numel() == 0


def test_magnitudes_full_chain_survey_geometry(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.survey_case(n_obj=20000, n_frames=20000, span=20.0, neo_frac=0.05)
    fr = case.frames
    order, off, t_ref = orc.make_batches(fr.t)
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    dfr = api.DeviceFrames.from_synth(fr)
    xg, sg = api.propagate(eph, _dev(torch, case.x0), 0.0, t_ref)
    b = api.Batches.from_host(order.astype(np.int32), off.astype(np.int32), t_ref)
    pf, ps, po = api.fov_check(eph, xg, b, dfr, sg)
    H, G = synth.hg_params(np.random.default_rng(43), case.x0.shape[0])
    v, geom = api.pair_magnitudes(eph, xg, b, dfr, pf, po, _dev(torch, H), _dev(torch, G), geometry=True)
    torch.cuda.synchronize()
    assert pf.numel() > 1000 and bool(torch.isfinite(v).all())
    rng = np.random.default_rng(44)
    sample = np.sort(rng.choice(case.x0.shape[0], 600, replace=False))
    pos = np.full(case.x0.shape[0], -1, np.int64)
    pos[sample] = np.arange(sample.size)
    pfh, poh = pf.cpu().numpy(), po.cpu().numpy()
    keep = pos[poh] >= 0
    xo, so, _ = orc.propagate(case.ephem, case.x0[sample], 0.0, t_ref)
    ov, og = orc.pair_mags(case.ephem, xo, order, off, t_ref, fr.t, fr.obs, pfh[keep], pos[poh[keep]], H[sample],
                           G[sample])
    vg, gg = v.cpu().numpy()[keep], geom.cpu().numpy()[keep]
    dv = np.abs(vg - ov).max()
    _say(f"survey geometry: {pf.numel()} pairs, {keep.sum()} of the sampled bodies: max |dV| {dv:.3e} mag, "
         f"phase angles {math.degrees(og[:, 2].min()):.3f}..{math.degrees(og[:, 2].max()):.1f} deg")
    assert keep.sum() > 20
    assert dv < 1e-8
    assert np.abs(gg[:, :2] - og[:, :2]).max() < 1e-9
