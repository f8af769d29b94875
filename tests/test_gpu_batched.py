"""Batched uneven jobs: one persistent propagation launch over every job
plus the field-of-view stages over all their batches, called through the
C ABI, against the CPU oracle job by job, against the per-job GPU path,
and as a captured HIP graph replayed several times."""
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


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).cuda()


def _jobs():
    """Uneven jobs plus the degenerate ones: a single body, no bodies, no
    frames, a ragged 65-body tile, and a job whose frames all precede its
    start epoch (integrated backward)."""
    eph, jobs = synth.batched_jobs(seed=7, n_jobs=18, max_obj=400, max_span=90.0, max_frames=160)
    model = synth.PlanetModel.make()
    rng = np.random.default_rng(70)
    el = synth.main_belt_elements(rng, 65)
    fr = synth.Frames.concat([synth.frames_tiny(rng, model, 20, 5.0, 25.0, 1.5),
                              synth.frames_targeted(rng, model, el, 5.0, 25.0, 40)])
    fr = fr.subset(np.argsort(fr.t, kind="stable"))
    jobs.append((synth.bodies_from_elements(model, el, 40.0), 40.0, fr))          # backward
    jobs.append((synth.bodies_from_elements(model, el[:1], 3.0), 3.0,
                 synth.frames_targeted(rng, model, el[:1], 3.0, 10.0, 6)))        # one body
    jobs.append((np.zeros((0, 6)), 1.0, synth.frames_tiny(rng, model, 9, 1.0, 5.0, 1.5)))   # no bodies
    jobs.append((synth.bodies_from_elements(model, el, 2.0), 2.0, fr.subset(np.zeros(0, np.int64))))  # no frames
    return eph, jobs


def _job_epochs_in_batch_order(runner, k, t_ref):
    ep = runner.job_epochs[k]
    return np.array([int(np.nonzero(ep == t)[0][0]) for t in t_ref], dtype=np.int64)


@pytest.fixture(scope="module")
def batched(torch_cuda):
    torch, api = torch_cuda
    ephem, jobs = _jobs()
    eph = api.DeviceEphemeris.from_synth(ephem)
    runner = api.BatchRunner(eph, jobs)
    _say(f"batched case: {len(jobs)} jobs, {int(runner.obj_off[-1])} bodies, {int(runner.frame_off[-1])} frames, "
         f"{runner.bjob.size} batches, {runner.n_x // 6} states")
    runner.run()
    torch.cuda.synchronize()
    pf, ps, po = runner.pairs()
    pairs = (pf.cpu().numpy(), ps.cpu().numpy(), po.cpu().numpy())
    return ephem, jobs, eph, runner, runner.x_out.clone(), runner.status.clone(), pairs


def test_batched_states_match_oracle(torch_cuda, orc, batched):
    torch, api = torch_cuda
    ephem, jobs, eph, runner, x_out, status, _ = batched
    worst = 0.0
    n_bad = 0
    for k, (x0, t0, fr) in enumerate(jobs):
        if x0.shape[0] == 0 or runner.job_epochs[k].size == 0:
            continue
        xg = runner.job_states(k).cpu().numpy()
        sg = status[runner.obj_off[k]:runner.obj_off[k + 1]].cpu().numpy()
        xo, so, _ = orc.propagate(ephem, x0, t0, runner.job_epochs[k])
        ok = (sg == 0) & (so == 0)
        n_bad += int((~ok).sum())
        assert np.array_equal(sg != 0, np.isnan(xg).any(axis=(0, 2)))
        worst = max(worst, float(np.abs(xg[:, ok, :3] - xo[:, ok, :3]).max()))
    _say(f"batched states vs oracle: max |dx| {worst:.3e} au, {n_bad} bodies not both ok")
    assert worst < 1e-10
    assert n_bad == 0


def test_batched_pairs_match_oracle(torch_cuda, orc, batched):
    torch, api = torch_cuda
    ephem, jobs, eph, runner, x_out, status, pairs = batched
    gf, gs, go = pairs
    key = gf.astype(np.int64) * 2 ** 32 + gs.astype(np.int64) * 2 ** 25 + go
    assert np.all(np.diff(key) > 0), "pairs not sorted by (frame, sub-frame, body)"
    total_o = 0
    for k, (x0, t0, fr) in enumerate(jobs):
        f0, f1 = runner.frame_off[k], runner.frame_off[k + 1]
        o0, o1 = runner.obj_off[k], runner.obj_off[k + 1]
        sel = (gf >= f0) & (gf < f1)
        assert np.all((go[sel] >= o0) & (go[sel] < o1)), "pair links a frame to another job's body"
        if x0.shape[0] == 0 or fr.t.size == 0:
            assert sel.sum() == 0
            continue
        order, off, t_ref = orc.make_batches(fr.t)
        xe, st, _ = orc.propagate(ephem, x0, t0, t_ref)
        opf, ops, opo, oedge = orc.fov(ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals)
        total_o += opf.size
        g = set(zip((gf[sel] - f0).tolist(), gs[sel].tolist(), (go[sel] - o0).tolist()))
        o = set(zip(opf.tolist(), ops.tolist(), opo.tolist()))
        near = {p for p, e in zip(zip(opf.tolist(), ops.tolist(), opo.tolist()), oedge) if abs(e) < MAS}
        assert not (o - g - near), (k, sorted(o - g - near)[:5])
        for f, s, j in g - o:
            q = int(np.nonzero(order == f)[0][0])
            b = int(np.searchsorted(off, q, side="right") - 1)
            _, d, _, _ = orc.lighttime(ephem, t_ref[b], xe[b, j], fr.t[f], fr.obs[f])
            _, edge = orc.inside(fr.normals[f], d)
            assert abs(edge[s]) < MAS
    _say(f"batched pairs: gpu {gf.size}, oracle {total_o}")
    assert total_o > 100


def test_batched_equals_per_job_path(torch_cuda, batched):
    torch, api = torch_cuda
    ephem, jobs, eph, runner, x_out, status, pairs = batched
    gf, gs, go = pairs
    worst = 0.0
    n_diff = 0
    for k, (x0, t0, fr) in enumerate(jobs):
        ep = runner.job_epochs[k]
        if x0.shape[0] == 0 or ep.size == 0:
            continue
        xj, sj = api.propagate(eph, _dev(torch, x0), t0, ep)
        xb = runner.job_states(k)
        assert torch.equal(sj, status[runner.obj_off[k]:runner.obj_off[k + 1]])
        ok = sj == 0
        worst = max(worst, (xj[:, ok] - xb[:, ok]).abs().max().item())
        order, off, t_ref = api.make_batches(fr.t)
        pos = _job_epochs_in_batch_order(runner, k, t_ref)
        b = api.Batches.from_host(order, off, t_ref)
        pf, ps, po = api.fov_check(eph, xj[torch.as_tensor(pos, device="cuda")].contiguous(), b,
                                   api.DeviceFrames.from_synth(fr), sj)
        f0, o0 = runner.frame_off[k], runner.obj_off[k]
        sel = (gf >= f0) & (gf < runner.frame_off[k + 1])
        g = set(zip((gf[sel] - f0).tolist(), gs[sel].tolist(), (go[sel] - o0).tolist()))
        j = set(zip(pf.cpu().numpy().tolist(), ps.cpu().numpy().tolist(), po.cpu().numpy().tolist()))
        n_diff += len(g ^ j)
    _say(f"batched vs per-job GPU path: max |dx| {worst:.3e} au, {n_diff} pairs differ")
    assert worst < 1e-11
    assert n_diff == 0


def test_batched_graph_replays(torch_cuda, batched):
    torch, api = torch_cuda
    ephem, jobs, eph, runner, x_out, status, pairs = batched
    runner.capture()
    rng = np.random.default_rng(3)
    for rep in range(3):
        runner.x_out.fill_(0.0)
        runner.status.fill_(-7)
        # unrelated eager work on the same stream between replays
        a = torch.randn(256, 256, dtype=torch.float64, device="cuda")
        _ = (a @ a).sum().item()
        x, _s = api.propagate(eph, _dev(torch, jobs[0][0][:10]), jobs[0][1], [jobs[0][1] + 1.0 + rep])
        torch.cuda.synchronize()
        runner.replay()
        torch.cuda.synchronize()
        assert torch.equal(runner.status, status), rep
        same = torch.equal(runner.x_out.nan_to_num(123.0), x_out.nan_to_num(123.0))
        assert same, rep
        pf, ps, po = runner.pairs()
        for got, ref in zip((pf, ps, po), pairs):
            assert np.array_equal(got.cpu().numpy(), ref), rep
        _say(f"graph replay {rep}: states and {pf.numel()} pairs identical to the eager run")
    # eager run after the replays still agrees
    runner.run()
    torch.cuda.synchronize()
    assert torch.equal(runner.x_out.nan_to_num(123.0), x_out.nan_to_num(123.0))


def test_batched_configurations_agree(torch_cuda, batched):
    torch, api = torch_cuda
    ephem, jobs, eph, runner, x_out, status, pairs = batched
    for kw in (dict(n_buckets=1), dict(window_segs=1), dict(fov_block=128), dict(cell_chord=0.3)):
        r = api.BatchRunner(eph, jobs, api.default_opts(**kw))
        r.run()
        torch.cuda.synchronize()
        pf, ps, po = r.pairs()
        d = (r.x_out - x_out)[torch.isfinite(x_out)].abs().max().item()
        same = all(np.array_equal(g.cpu().numpy(), p) for g, p in zip((pf, ps, po), pairs))
        _say(f"batched config {kw}: max |dx| vs default {d:.3e}, pairs identical {same}")
        assert d < 1e-11
        assert torch.equal(r.status, status)
        assert same


def test_batched_autotune_and_cache(torch_cuda, batched, tmp_path):
    torch, api = torch_cuda
    ephem, jobs, eph, runner, x_out, status, pairs = batched
    r = api.BatchRunner(eph, jobs)
    cache = str(tmp_path / "tune.json")
    best, ms, hit = r.autotune(reps=1, cache=cache)
    assert not hit and ms > 0
    _say(f"autotune: n_buckets {best.n_buckets}, persist_waves {best.persist_waves}, window_segs {best.window_segs}, "
         f"fov_block {best.fov_block}, cell_chord {best.cell_chord}: {ms:.3f} ms per run")
    r.run()
    torch.cuda.synchronize()
    pf, ps, po = r.pairs()
    assert all(np.array_equal(g.cpu().numpy(), p) for g, p in zip((pf, ps, po), pairs))
    assert (r.x_out - x_out)[torch.isfinite(x_out)].abs().max().item() < 1e-11
    r2 = api.BatchRunner(eph, jobs)
    best2, ms2, hit2 = r2.autotune(cache=cache)
    assert hit2 and ms2 == ms
    for k in ("n_buckets", "persist_waves", "window_segs", "fov_block", "cell_chord"):
        assert getattr(best2, k) == getattr(best, k)
