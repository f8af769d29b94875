"""Parity at the full sizes of the workloads, in the configuration the
benchmark runs (default options, whole workload in one call), checked on
outputs sampled so that the CPU oracle can compute them one by one:
sampled bodies over every epoch, and their pairs over sampled batches.

Tolerances as in the small parity tests: positions 1e-10 au, pair sets
identical outside the 1 mas edge band, sky positions 1e-3 mas, gradients
1e-8 relative."""
import math
import sys
import time

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


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).cuda()


def _sample_bodies(rng, is_neo, n_mb, n_neo):
    mb = np.nonzero(~is_neo)[0]
    neo = np.nonzero(is_neo)[0]
    return np.sort(np.concatenate([rng.choice(mb, n_mb, replace=False), rng.choice(neo, n_neo, replace=False)]))


def _check_sampled(torch, api, orc, case, xg, sg, pairs, order, off, t_ref, sample, batches, label):
    """Sampled bodies against the oracle: states at every epoch, and pairs
    over the frames of the sampled batches."""
    fr = case.frames
    xo, so, _ = orc.propagate(case.ephem, case.x0[sample], case.t0, t_ref)
    xs = xg[:, torch.as_tensor(sample, device="cuda")].cpu().numpy()
    ss = sg[torch.as_tensor(sample, device="cuda")].cpu().numpy()
    np.testing.assert_array_equal(ss, so)
    ok = so == 0
    assert ok.all()
    err = np.abs(xs[:, ok, :3] - xo[:, ok, :3]).max()
    _say(f"{label}: {sample.size} sampled bodies over {t_ref.size} epochs, max |dx| {err:.3e} au")
    assert err < 1e-10
    # pairs of the sampled bodies over the sampled batches
    sub_order = np.concatenate([order[off[b]:off[b + 1]] for b in batches])
    sub_off = np.concatenate([[0], np.cumsum([off[b + 1] - off[b] for b in batches])]).astype(np.int32)
    opf, ops, opo, oedge = orc.fov(case.ephem, xo[batches], so, sub_order, sub_off, t_ref[batches], fr.t, fr.obs,
                                   fr.normals)
    opo = sample[opo]
    pf, ps, po = pairs
    frames_sel = np.zeros(fr.t.size, bool)
    frames_sel[sub_order] = True
    keep = frames_sel[pf] & np.isin(po, sample)
    g = set(zip(pf[keep].tolist(), ps[keep].tolist(), po[keep].tolist()))
    o = set(zip(opf.tolist(), ops.tolist(), opo.tolist()))
    near = {p for p, e in zip(zip(opf.tolist(), ops.tolist(), opo.tolist()), oedge) if abs(e) < MAS}
    missing, extra = o - g - near, g - o
    _say(f"{label}: {len(batches)} batches, {sub_order.size} frames: oracle {len(o)} pairs, gpu {len(g)}, "
         f"missing {len(missing)}, extra {len(extra)}")
    assert not missing, sorted(missing)[:5]
    pos = {int(f): i for i, f in enumerate(sub_order)}
    for f, s, j in extra:
        q = pos[f]
        bi = int(np.searchsorted(sub_off, q, side="right") - 1)
        js = int(np.nonzero(sample == j)[0][0])
        _, d, _, _ = orc.lighttime(case.ephem, t_ref[batches[bi]], xo[batches[bi], js], fr.t[f], fr.obs[f])
        _, edge = orc.inside(fr.normals[f], d)
        assert abs(edge[s]) < MAS
    return len(o)


def _run_full(torch, api, case, label):
    fr = case.frames
    t0 = time.perf_counter()
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    frames = api.DeviceFrames.from_synth(fr)
    order, off, t_ref = api.make_batches(fr.t)
    b = api.Batches.from_host(order, off, t_ref)
    xg, sg = api.propagate(eph, _dev(torch, case.x0), case.t0, t_ref)
    pf, ps, po = api.fov_check(eph, xg, b, frames, sg)
    torch.cuda.synchronize()
    _say(f"{label}: {case.x0.shape[0]} bodies, {fr.t.size} frames x {fr.n_sub} sub-frames, {t_ref.size} batches: "
         f"{pf.numel()} pairs ({time.perf_counter() - t0:.1f} s with uploads)")
    # every pair once, in (frame, sub-frame, body) order, at full size
    key = (pf.long() << 32) | (ps.long() << 25) | po.long()
    assert bool((key[1:] > key[:-1]).all())
    del key
    return xg, sg, (pf, ps, po), order, off, t_ref


def _pairs_of(torch, pairs, sample):
    pf, ps, po = pairs
    keep = torch.isin(po, torch.as_tensor(sample, dtype=po.dtype, device=po.device))
    return pf[keep].cpu().numpy(), ps[keep].cpu().numpy(), po[keep].cpu().numpy()


def test_survey_full_size_sampled(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.survey_case()
    xg, sg, pairs, order, off, t_ref = _run_full(torch, api, case, "survey")
    rng = np.random.default_rng(21)
    sample = _sample_bodies(rng, case.is_neo, 400, 100)
    batches = np.sort(rng.choice(t_ref.size, 12, replace=False))
    n = _check_sampled(torch, api, orc, case, xg, sg, _pairs_of(torch, pairs, sample), order, off, t_ref, sample,
                       batches, "survey")
    assert n > 0
    # H-G magnitudes of every pair, sampled bodies on the sampled batches against the oracle
    fr = case.frames
    H, G = synth.hg_params(np.random.default_rng(25), case.x0.shape[0])
    b = api.Batches.from_host(order, off, t_ref)
    pf, ps, po = pairs
    v = api.pair_magnitudes(api.DeviceEphemeris.from_synth(case.ephem), xg, b, api.DeviceFrames.from_synth(fr),
                            pf, po, _dev(torch, H), _dev(torch, G))
    torch.cuda.synchronize()
    pfh, poh, vh = pf.cpu().numpy(), po.cpu().numpy(), v.cpu().numpy()
    bad = np.nonzero(~np.isfinite(vh))[0]
    _say(f"survey: {bad.size} non-finite magnitudes; first (frame, body): "
         f"{list(zip(pfh[bad[:5]].tolist(), poh[bad[:5]].tolist()))}")
    assert bad.size == 0
    loc = np.full(case.x0.shape[0], -1, np.int64)
    loc[sample] = np.arange(sample.size)
    in_b = np.zeros(fr.t.size, bool)
    for bb in batches:
        in_b[order[off[bb]:off[bb + 1]]] = True
    keep = (loc[poh] >= 0) & in_b[pfh]
    xo, _, _ = orc.propagate(case.ephem, case.x0[sample], case.t0, t_ref)
    ov, _ = orc.pair_mags(case.ephem, xo, order, off, t_ref, fr.t, fr.obs, pfh[keep], loc[poh[keep]], H[sample],
                          G[sample])
    dv = np.abs(vh[keep] - ov).max()
    _say(f"survey: magnitudes of {vh.size} pairs, {keep.sum()} sampled against the oracle: max |dV| {dv:.3e} mag")
    assert keep.sum() > 0 and dv < 1e-8


def test_footprint_full_size_sampled(torch_cuda, orc):
    torch, api = torch_cuda
    t0 = time.perf_counter()
    case = synth.footprint_case()
    _say(f"footprint case generated in {time.perf_counter() - t0:.1f} s")
    xg, sg, pairs, order, off, t_ref = _run_full(torch, api, case, "footprints")
    rng = np.random.default_rng(22)
    sample = _sample_bodies(rng, case.is_neo, 400, 100)
    batches = np.sort(rng.choice(t_ref.size, 12, replace=False))
    n = _check_sampled(torch, api, orc, case, xg, sg, _pairs_of(torch, pairs, sample), order, off, t_ref, sample,
                       batches, "footprints")
    assert n > 0


def test_gradient_full_size_sampled(torch_cuda, orc):
    torch, api = torch_cuda
    g = synth.gradient_case()
    eph = api.DeviceEphemeris.from_synth(g.ephem)
    ctx = api.AdjointContext(eph, g.t0, g.arc, _dev(torch, g.t_obs), _dev(torch, g.obs_pos), 5.0)
    x0 = _dev(torch, g.x0).requires_grad_(True)
    sky = api.AdjointSky.apply(x0, ctx)
    loss = api.sky_residual_loss(sky, _dev(torch, g.radec_obs))
    loss.backward()
    rng = np.random.default_rng(23)
    sample = np.sort(rng.choice(g.x0.shape[0], 60, replace=False))
    radec, oloss, og, ost = orc.sky_grad(g.ephem, g.x0[sample], g.t0, g.t_obs[sample], g.obs_pos[sample],
                                         g.radec_obs[sample])
    gs = sky.detach()[torch.as_tensor(sample, device="cuda")].cpu().numpy()
    gg = x0.grad[torch.as_tensor(sample, device="cuda")].cpu().numpy()
    st = ctx.status[torch.as_tensor(sample, device="cuda")].cpu().numpy()
    np.testing.assert_array_equal(st, ost)
    ok = ost == 0
    assert ok.all()
    dra = (gs[..., 0] - radec[..., 0] + np.pi) % (2 * np.pi) - np.pi
    dsky = np.hypot(dra * np.cos(radec[..., 1]), gs[..., 1] - radec[..., 1])[ok].max()
    rel = np.linalg.norm(gg[ok] - og[ok], axis=1) / np.linalg.norm(og[ok], axis=1)
    _say(f"gradient workload ({g.x0.shape[0]} bodies): sampled max sky difference {dsky / MAS:.3e} mas, "
         f"max rel gradient difference {rel.max():.3e}")
    assert dsky < 1e-3 * MAS
    assert rel.max() < 1e-8


def test_batched_full_size_sampled(torch_cuda, orc):
    torch, api = torch_cuda
    t0 = time.perf_counter()
    ephem, jobs = synth.batched_jobs()
    eph = api.DeviceEphemeris.from_synth(ephem)
    runner = api.BatchRunner(eph, jobs)
    runner.run()
    torch.cuda.synchronize()
    pf, ps, po = runner.pairs()
    _say(f"batched: {len(jobs)} jobs, {int(runner.obj_off[-1])} bodies, {int(runner.frame_off[-1])} frames, "
         f"{pf.numel()} pairs ({time.perf_counter() - t0:.1f} s with generation)")
    rng = np.random.default_rng(24)
    sizes = np.array([j[0].shape[0] * j[2].t.size for j in jobs])
    picks = list(np.argsort(sizes)[-3:]) + list(rng.choice(len(jobs), 5, replace=False))
    total = 0
    for k in picks:
        x0, t0j, fr = jobs[k]
        if x0.shape[0] == 0 or fr.t.size == 0:
            continue
        n_s = min(12, x0.shape[0])
        sample = np.sort(rng.choice(x0.shape[0], n_s, replace=False))
        ep = runner.job_epochs[k]
        xb = runner.job_states(k)[:, torch.as_tensor(sample, device="cuda")].cpu().numpy()
        xo, so, _ = orc.propagate(ephem, x0[sample], t0j, ep)
        err = np.abs(xb[..., :3] - xo[..., :3])[:, so == 0].max()
        assert err < 1e-10, (k, err)
        # pairs of the sampled bodies over at most 4 of the job's batches
        order, off, t_ref = orc.make_batches(fr.t)
        bsel = np.sort(rng.choice(t_ref.size, min(4, t_ref.size), replace=False))
        pos = np.array([int(np.nonzero(ep == t_ref[b])[0][0]) for b in bsel])
        sub_order = np.concatenate([order[off[b]:off[b + 1]] for b in bsel])
        sub_off = np.concatenate([[0], np.cumsum([off[b + 1] - off[b] for b in bsel])]).astype(np.int32)
        opf, ops, opo, oedge = orc.fov(ephem, xo[pos], so, sub_order, sub_off, t_ref[bsel], fr.t, fr.obs,
                                       fr.normals)
        f0, o0 = int(runner.frame_off[k]), int(runner.obj_off[k])
        gsel = torch.isin(po, torch.as_tensor(o0 + sample, dtype=po.dtype, device="cuda")) & \
            torch.isin(pf, torch.as_tensor(f0 + sub_order, dtype=pf.dtype, device="cuda"))
        g = set(zip((pf[gsel] - f0).tolist(), ps[gsel].tolist(), (po[gsel] - o0).tolist()))
        o = set(zip(opf.tolist(), ops.tolist(), sample[opo].tolist()))
        near = {p for p, e in zip(zip(opf.tolist(), ops.tolist(), sample[opo].tolist()), oedge) if abs(e) < MAS}
        assert not (o - g - near), (k, sorted(o - g - near)[:5])
        fpos = {int(f): i for i, f in enumerate(sub_order)}
        for f, s, j in g - o:
            bi = int(np.searchsorted(sub_off, fpos[f], side="right") - 1)
            js = int(np.nonzero(sample == j)[0][0])
            _, d, _, _ = orc.lighttime(ephem, t_ref[bsel[bi]], xo[pos[bi], js], fr.t[f], fr.obs[f])
            _, edge = orc.inside(fr.normals[f], d)
            assert abs(edge[s]) < MAS, (k, f, s, j)
        total += len(o)
        _say(f"  job {k}: {x0.shape[0]} bodies, {fr.t.size} frames, span {ep.max() - t0j:.1f} d: max |dx| "
             f"{err:.2e} au, {len(o)} oracle pairs on {len(bsel)} batches")
    assert total > 0
