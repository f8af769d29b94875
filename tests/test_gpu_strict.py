"""Strict n-body mode (Sect. 2: the two-body interval set to zero): with a
batch span of zero every distinct frame time is its own batch epoch, the
integrator reaches each exposure time and the hop covers the light time
alone.  Checked against the oracle in the same mode, and used to measure
the two-body approximation error of the default 3-day batches."""
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


def _directions(torch, api, eph, x_epoch, bt, frame_batch, fr, pairs):
    """Light-time directions of the pairs (f, j) hopping from the state of
    the frame's batch epoch."""
    out = {}
    by_frame = {}
    for f, j in pairs:
        by_frame.setdefault(f, []).append(j)
    for f, js in by_frame.items():
        b = frame_batch[f]
        xs = x_epoch[b][torch.as_tensor(js, device="cuda")].contiguous()
        d, _ = api.lighttime_directions(eph, xs, float(bt.t_ref_host[b]),
                                        torch.as_tensor([fr.t[f]], dtype=torch.float64, device="cuda"),
                                        torch.as_tensor(fr.obs[f:f + 1], dtype=torch.float64, device="cuda"))
        for j, dj in zip(js, d[0].cpu().numpy()):
            out[(f, j)] = dj
    return out


def _frame_batch(bt, n_frames):
    order = bt.frame_order.cpu().numpy()
    off = bt.batch_off.cpu().numpy()
    fb = np.empty(n_frames, np.int64)
    for b in range(off.size - 1):
        fb[order[off[b]:off[b + 1]]] = b
    return fb


def test_strict_nbody_mode(torch_cuda, orc):
    torch, api = torch_cuda
    case = synth.survey_case(n_obj=5000, n_frames=2400, span=4.0, neo_frac=0.05)
    fr = case.frames
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    dfr = api.DeviceFrames.from_synth(fr)
    x0 = torch.as_tensor(case.x0, dtype=torch.float64, device="cuda")
    pf, ps, po, xg, sg, bt = api.predict(eph, x0, 0.0, dfr, fr.t)
    spf, sps, spo, sxg, ssg, sbt = api.predict(eph, x0, 0.0, dfr, fr.t, api.default_opts(batch_span=0.0))
    torch.cuda.synchronize()
    assert sbt.t_ref_host.size == np.unique(fr.t).size
    assert int((sg != 0).sum()) == 0 and int((ssg != 0).sum()) == 0
    _say(f"default: {bt.t_ref_host.size} batches, {pf.numel()} pairs; strict: {sbt.t_ref_host.size} batches, "
         f"{spf.numel()} pairs")

    # strict mode against the oracle in the same mode, on sampled bodies
    order, off, t_ref = orc.make_batches(fr.t, 0.0)
    np.testing.assert_array_equal(sbt.t_ref_host, t_ref)
    rng = np.random.default_rng(50)
    sample = np.sort(np.concatenate([rng.choice(np.nonzero(~case.is_neo)[0], 150, replace=False),
                                     rng.choice(np.nonzero(case.is_neo)[0], 50, replace=False)]))
    xo, so, _ = orc.propagate(case.ephem, case.x0[sample], 0.0, t_ref)
    err = np.abs(sxg[:, torch.as_tensor(sample, device="cuda")].cpu().numpy()[..., :3] - xo[..., :3]).max()
    _say(f"strict mode: {sample.size} sampled bodies at {t_ref.size} frame times, max |dx| {err:.3e} au")
    assert err < 1e-10
    opf, ops, opo, oedge = orc.fov(case.ephem, xo, so, order, off, t_ref, fr.t, fr.obs, fr.normals)
    opo = sample[opo]
    keep = np.isin(spo.cpu().numpy(), sample)
    g = set(zip(spf.cpu().numpy()[keep].tolist(), sps.cpu().numpy()[keep].tolist(), spo.cpu().numpy()[keep].tolist()))
    o = set(zip(opf.tolist(), ops.tolist(), opo.tolist()))
    near = {p for p, e in zip(zip(opf.tolist(), ops.tolist(), opo.tolist()), oedge) if abs(e) < MAS}
    assert not (o - g - near), sorted(o - g - near)[:5]
    loc = {int(j): k for k, j in enumerate(sample)}
    pos = {int(f): q for q, f in enumerate(order)}
    for f, s_, j in g - o:
        b = int(np.searchsorted(off, pos[f], side="right") - 1)
        _, d, _, _ = orc.lighttime(case.ephem, t_ref[b], xo[b, loc[j]], fr.t[f], fr.obs[f])
        _, edge = orc.inside(fr.normals[f], d)
        assert abs(edge[s_]) < MAS
    assert len(o) > 0

    # two-body approximation error of the default batches: the direction of
    # every pair of either mode under both modes
    dset = set(zip(pf.cpu().numpy().tolist(), po.cpu().numpy().tolist()))
    sset = set(zip(spf.cpu().numpy().tolist(), spo.cpu().numpy().tolist()))
    union = sorted(dset | sset)
    dd = _directions(torch, api, eph, xg, bt, _frame_batch(bt, fr.t.size), fr, union)
    ds = _directions(torch, api, eph, sxg, sbt, _frame_batch(sbt, fr.t.size), fr, union)
    ang = {}
    for p in union:
        a, b = dd[p], ds[p]
        ang[p] = math.atan2(np.linalg.norm(np.cross(a, b)), float(a @ b))
    v = np.array(list(ang.values())) / MAS
    neo = np.array([case.is_neo[j] for _, j in union])
    _say(f"two-body approximation error over {len(union)} pairs: main belt max {v[~neo].max():.3f} mas, "
         f"median {np.median(v[~neo]):.3f} mas; NEO-like max {v[neo].max() if neo.any() else 0:.3f} mas")
    # pairs found by one mode only lie within that pair's approximation error of an edge
    for f, j in sorted(dset ^ sset):
        _, edge = orc.inside(fr.normals[f], ds[(f, j)])
        assert np.abs(edge).min() <= ang[(f, j)] + MAS, (f, j, edge, ang[(f, j)])
    _say(f"pairs in one mode only: {len(dset ^ sset)} of {len(union)}")
