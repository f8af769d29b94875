#!/usr/bin/env python3
"""Benchmark of the known-object prediction path on one MI355X.

One step is the whole path over the survey workload: 100,000 bodies
(95% main belt, 5% NEO-like) with the Sun and 8 planets as 8-day
degree-12 Chebyshev segments, 500,000 frames of 0.78 deg x 0.78 deg
over one year from a space observer (1 au orbit plus a 7,000 km offset
orbit) in 11 s sequences of 12 along great circles:
  frame batching (<= 3 days) -> n-body integration of every body to every
  batch epoch -> universal-variable light-time hops and the sky-binned
  membership test -> (frame, sub-frame, object) pairs sorted.
Inputs are resident in device memory before the timed region.

Prints one JSON line.  `value` is object-days propagated per second of
the whole step.  The roofline block covers the dominant kernel, timed
live with HIP events on the stream it runs on.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X vector FP64: 256 CU x 64 lanes x 2 flop x 2.4 GHz
HBM_PEAK_GBS = 8000.0

# Algorithmic flop weights (FMA = 2, add/sub/mul = 1, rsqrt/sqrt/div = 1).
CLENSHAW_CHAIN_FLOPS = lambda deg1: 7 * (deg1 - 1) + 12     # value and derivative
CLENSHAW_VALUE_FLOPS = lambda deg1: 3 * (deg1 - 1) + 9      # value only
# Extrapolated corrector start, per body-step: 7 nodes x (sig 2, 7 differences,
# 7 prefix products, 7 x (basis product 1, weight FMA 2, three FMAs 6, suffix
# product 1)), and q.
PREDICT_FLOPS = 7 * (2 + 7 + 7 + 7 * 10) + 1
# Epoch read off a step's collocation polynomial, per body: 6 components x
# (7 FMAs + 4), plus the wavefront's 14 weight polynomials (8 FMAs and a
# product each) shared by its 9 bodies.
DENSE_FLOPS = 6 * (7 * 2 + 4) + (14 * 17 + 8) // 9


def node_flops(n_body: int, n_gr: int) -> int:
    pred_x = 3 * (1 + 14 + 4) + 1          # half_s2 F0 + 7 FMA + 2 FMA, s h
    pred_v = 3 * (1 + 14 + 2) if n_gr else 0
    force = 18 * n_body + 27 * n_gr        # per-body Newtonian and Eq. A.3 terms
    return pred_x + pred_v + force + 3     # + D update


def integrator_flops(stats, n_body: int, n_gr: int, deg1: int) -> float:
    """Algorithmic FP64 flops from the kernel's own counters:
    stats = [wave steps, wave iterations, rejections, body-steps,
    body-sweeps, Clenshaw chains with derivative, value-only chains,
    body-steps started from an extrapolated corrector]."""
    lane_steps, lane_iter, chains, vchains = float(stats[3]), float(stats[4]), float(stats[5]), float(stats[6])
    pred = float(stats[7]) if len(stats) > 7 else 0.0
    per_iter = 7 * node_flops(n_body, n_gr) + 3 * 14 + 12
    per_step = 3 * (1 + 28 + 4 + 2) + (18 * n_body + 27 * n_gr) + 10
    return (lane_iter * per_iter + lane_steps * per_step + chains * CLENSHAW_CHAIN_FLOPS(deg1)
            + vchains * CLENSHAW_VALUE_FLOPS(deg1) + pred * PREDICT_FLOPS)


def measured_traffic(path=os.path.join(ROOT, "profiles", "traffic_k_nbody_g8_survey.md")):
    """HBM bytes per integrator launch from the committed counter summary,
    or None when the summary is missing or the kernel sources changed
    since it was taken."""
    import hashlib
    import re
    try:
        txt = open(path).read()
        val = float(re.search(r"^traffic_bytes_per_launch: (\S+)$", txt, re.M).group(1))
        sha = re.search(r"^sources_sha1: (\S+)$", txt, re.M).group(1)
        files = re.search(r"^sources: (.+)$", txt, re.M).group(1).split()
    except (OSError, AttributeError, ValueError):
        return None
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(ROOT, "paper_2509_04666_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return val if h.hexdigest() == sha else None


def workload_name(case, F):
    return ("survey: %d bodies (95%% main belt, 5%% NEO-like), Sun + 8 planets as 8-day degree-12 "
            "Chebyshev segments, %.2f days, %d frames of 0.78 deg in 11 s sequences of 12" %
            (case.x0.shape[0], case.span, F))


def cpu_baseline(case, t_ref, order, off, n_obj_prop=10000, n_obj_fov=4000, n_batches_fov=3):
    """The CPU oracle as it stands, on a bounded sample of the same
    workload, extrapolated to the whole step."""
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    opts = O.make_opts(n_threads=threads)
    rng = np.random.default_rng(7)
    N = case.x0.shape[0]
    sel = np.sort(rng.choice(N, n_obj_prop, replace=False))
    t0 = time.perf_counter()
    xe, st, _ = O.propagate(case.ephem, case.x0[sel], 0.0, t_ref, opts=opts)
    t_prop = time.perf_counter() - t0
    rate_prop = n_obj_prop * case.span / t_prop                # object-days/s
    fr = case.frames
    nb = n_batches_fov
    sub_off = off[:nb + 1]
    sub_order = order[:off[nb]]
    xs = xe[:nb, :n_obj_fov]
    t1 = time.perf_counter()
    O.fov(case.ephem, xs, st[:n_obj_fov], sub_order, sub_off, t_ref[:nb], fr.t, fr.obs, fr.normals,
          n_threads=threads)
    t_fov = time.perf_counter() - t1
    tests = n_obj_fov * int(off[nb]) * fr.n_sub
    rate_fov = tests / t_fov
    F = fr.n_frames
    t_total = N * case.span / rate_prop + N * F * fr.n_sub / rate_fov
    return {
        "value": N * case.span / t_total, "unit": "object-days/s", "cores": threads, "kind": "oracle",
        "sample": (f"propagation of {n_obj_prop} bodies over all {len(t_ref)} batch epochs "
                   f"({t_prop:.2f} s, {rate_prop:.3e} object-days/s) and brute-force membership of "
                   f"{n_obj_fov} bodies x {int(off[nb])} frames ({t_fov:.2f} s, {rate_fov:.3e} tests/s), "
                   f"extrapolated to {N} bodies x {F} frames"),
        "propagation_object_days_per_s": rate_prop, "fov_tests_per_s": rate_fov,
    }


def strict_component(api, torch, case, eph, x0, log, days=1.0, reps=3):
    """Strict n-body mode (the two-body interval set to zero, Sect. 2) on
    the first `days` of the survey's frames, every body: a batch span of
    zero makes each distinct frame time a batch epoch.  Timed beside the
    default 3-day batching of the same frames."""
    fr = case.frames.subset(np.nonzero(case.frames.t < days)[0])
    frames = api.DeviceFrames.from_synth(fr)
    res = {"frames": int(fr.t.size), "days": days}
    for name, span in (("default", 3.0), ("strict", 0.0)):
        opts = api.default_opts(batch_span=span)
        out = api.predict(eph, x0, 0.0, frames, fr.t, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = api.predict(eph, x0, 0.0, frames, fr.t, opts)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        res[name] = {"batches": int(out[5].t_ref_host.size), "pairs": int(out[0].numel()), "ms": ms,
                     "object_days_per_s": x0.shape[0] * days / (ms / 1e3)}
        del out
        log(f"strict component: {name} {res[name]}")
    res["strict_over_default"] = res["strict"]["ms"] / res["default"]["ms"]
    return res


def adjoint_component(api, synth, torch, n_obj, log, reps=10):
    """Forward sky positions and the backward gradient of the summed squared
    sky residual: 100,000 bodies, 20 observations each over a 60-day arc,
    checkpoints every 5 days."""
    t_setup = time.perf_counter()
    g = synth.gradient_case(n_obj=n_obj, k_obs=20, arc=60.0)
    dev = torch.device("cuda:0")
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(dev)
    eph = api.DeviceEphemeris.from_synth(g.ephem)
    ctx = api.AdjointContext(eph, g.t0, g.arc, f(g.t_obs), f(g.obs_pos), 5.0, api.default_opts())
    x0 = f(g.x0)
    radec = f(g.radec_obs)
    log(f"adjoint setup {time.perf_counter() - t_setup:.1f} s")

    def fwd():
        return ctx.forward(x0)

    def bwd(sky):
        s = sky.detach().requires_grad_(True)
        loss = api.sky_residual_loss(s, radec)
        (gs,) = torch.autograd.grad(loss, s)
        return ctx.backward(x0, gs)

    sky = fwd()
    bwd(sky)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sky = fwd()
    torch.cuda.synchronize()
    t_f = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        grad = bwd(sky)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / reps
    n_fail = int((ctx.status != 0).sum().item())
    return {
        "workload": f"{n_obj} bodies x 20 observations over 60 days, Sun + 8 planets, checkpoints every 5 days",
        "forward_ms": t_f * 1e3, "backward_ms": t_b * 1e3, "backward_over_forward": t_b / t_f,
        "gradient_over_forward": (t_f + t_b) / t_f,
        "forward_object_days_per_s": n_obj * 60.0 / t_f, "failed_objects": n_fail,
        "grad_finite": bool(torch.isfinite(grad).all().item()),
    }


def batched_component(api, synth, torch, n_jobs, log, reps=2, tune_cache=None):
    """Uneven jobs (log-uniform 1-20,000 bodies, 1 day-10 years, 1-5,000
    frames): the whole set as one captured graph replay against one
    propagation call and one FoV call per job."""
    from paper_2509_04666_amd import _lib
    import ctypes as C
    t_setup = time.perf_counter()
    ephem, jobs = synth.batched_jobs(n_jobs=n_jobs)
    dev = torch.device("cuda:0")
    eph = api.DeviceEphemeris.from_synth(ephem)
    runner = api.BatchRunner(eph, jobs)
    n_bodies = int(runner.obj_off[-1])
    obj_days = float(sum(x0.shape[0] * np.abs(np.concatenate([[t0], runner.job_epochs[k]]) -
                                              np.concatenate([runner.job_epochs[k], [t0]]))[:-1].sum()
                         for k, (x0, t0, fr) in enumerate(jobs)))
    log(f"batched setup {time.perf_counter() - t_setup:.1f} s: {len(jobs)} jobs, {n_bodies} bodies, "
        f"{int(runner.frame_off[-1])} frames, {runner.bjob.size} batches")
    t_tune = time.perf_counter()
    best, tune_ms, hit = runner.autotune(reps=1, cache=tune_cache,
                                         progress=lambda o, t: log(f"  tune {o}: {t:.1f} ms"))
    log(f"autotune {'(cached) ' if hit else ''}{time.perf_counter() - t_tune:.1f} s: {tune_ms:.1f} ms per run")
    runner.capture()
    runner.replay()
    torch.cuda.synchronize()
    L = _lib.lib()
    L.kete_timing_enable(1)
    t0 = time.perf_counter()
    for _ in range(reps):
        runner.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    L.kete_timing_enable(0)
    ms = np.zeros(4); cnt = np.zeros(4, np.int64)
    _lib.check(L.kete_timing_read(ms.ctypes.data_as(C.c_void_p), cnt.ctypes.data_as(C.c_void_p)))
    pf, ps, po = runner.pairs()
    n_pairs_batched = pf.numel()

    # one propagation call and one FoV call per job, inputs already on the device
    opts = api.default_opts()
    x0_dev = [runner.x0[runner.obj_off[k]:runner.obj_off[k + 1]] for k in range(len(jobs))]
    fr_dev, bt_dev, ws_p, ws_f = [], [], 0, 0
    for k, (x0, t0, fr) in enumerate(jobs):
        f0, f1 = int(runner.frame_off[k]), int(runner.frame_off[k + 1])
        fr_dev.append(api.DeviceFrames(runner.frames.t[f0:f1], runner.frames.obs[f0:f1],
                                       runner.frames.normals[f0:f1]))
        order, off, t_ref = api.make_batches(fr.t, opts.batch_span)
        bt_dev.append(api.Batches.from_host(order, off, t_ref, dev))
        n, nb = x0.shape[0], t_ref.size
        ws_p = max(ws_p, L.kete_propagate_workspace_size(n, nb, C.byref(opts)))
        ws_f = max(ws_f, L.kete_fov_workspace_size(n, f1 - f0, nb, fr.n_sub, max(1 << 16, 8 * (f1 - f0)),
                                                   C.byref(opts)))
    wp = torch.empty(max(ws_p, 256), dtype=torch.uint8, device=dev)
    wf = torch.empty(max(ws_f, 256), dtype=torch.uint8, device=dev)

    def per_job():
        n_pairs = 0
        for k, (x0, t0, fr) in enumerate(jobs):
            if x0.shape[0] == 0 or fr.t.size == 0:
                continue
            b = bt_dev[k]
            x, st = api.propagate(eph, x0_dev[k], t0, b.t_ref_host, opts, workspace=wp)
            pf, ps, po = api.fov_check(eph, x, b, fr_dev[k], st, opts, workspace=wf)
            n_pairs += pf.numel()
        return n_pairs

    t0 = time.perf_counter()
    n_pairs_job = per_job()
    torch.cuda.synchronize()
    t_job = time.perf_counter() - t0
    return {
        "workload": (f"{len(jobs)} uneven jobs: log-uniform 1-20,000 bodies, 1 day-10 years, 1-5,000 frames; "
                     f"{n_bodies} bodies, {int(runner.frame_off[-1])} frames"),
        "object_days": obj_days, "graph_ms": t_graph * 1e3, "per_job_ms": t_job * 1e3,
        "speedup_vs_per_job": t_job / t_graph, "object_days_per_s": obj_days / t_graph,
        "graph_launch_event_ms": ms[3] / max(cnt[3], 1),
        "pairs": n_pairs_batched, "pairs_per_job_path": n_pairs_job,
        "tuned": {k: getattr(best, k) for k in ("n_buckets", "persist_waves", "window_segs", "fov_block",
                                                "cell_chord")},
        "tuning_from_cache": hit,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--objects", type=int, default=100_000)
    ap.add_argument("--frames", type=int, default=500_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint-objects", type=int, default=100_000)
    ap.add_argument("--batched-jobs", type=int, default=4096)
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2509_04666_amd", "tuning.json"))
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-strict", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="copy a buffer of this size once before timing (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the objects are independent "
              "and the path would shard them over GPUs; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_04666_amd import api, synth, _lib
    import ctypes as C

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    t_setup = time.perf_counter()
    case = synth.survey_case(n_obj=args.objects, n_frames=args.frames)
    fr = case.frames
    N, F, S = case.x0.shape[0], fr.n_frames, fr.n_sub
    dev = torch.device("cuda:0")
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    frames = api.DeviceFrames.from_synth(fr)
    x0 = torch.as_tensor(case.x0).to(dev)
    frame_t_host = np.ascontiguousarray(fr.t)
    opts = api.default_opts()
    # one launch per call that reads every epoch but the last off the step polynomials
    dense_epochs_read = not opts.land_epochs and opts.lanes_per_body != 1 and opts.rebucket_epochs == 0
    n_gr = int(np.sum(case.ephem.flags & 1))
    log(f"setup {time.perf_counter() - t_setup:.1f} s: N={N} F={F}")

    order, off, t_ref = api.make_batches(frame_t_host, opts.batch_span)
    B = t_ref.size
    cap = 8 * F

    # Consecutive steps alternate between two streams (both at the default
    # priority), each with its own workspaces: step i's integrator runs
    # while step i - 1's field-of-view stages do, and their kernels fill
    # each other's tails.  Every step batches its own frames (a1) on the host.
    streams = [torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)]
    ws = [(torch.empty(_lib.lib().kete_propagate_workspace_size(N, B, C.byref(opts)), dtype=torch.uint8, device=dev),
           torch.empty(_lib.lib().kete_fov_workspace_size(N, F, B, S, cap, C.byref(opts)), dtype=torch.uint8,
                       device=dev)) for _ in streams]

    def run_steps(K, stats=None, marks=None):
        """K survey steps, pipelined over the two streams; stats (one [8]
        counter tensor per stream) accumulate the integrator counters."""
        pending, out = None, None
        for i in range(K + 1):
            nxt = None
            if i < K:
                k = i % 2
                with torch.cuda.stream(streams[k]):
                    order, off, t_ref = api.make_batches(frame_t_host, opts.batch_span)
                    batches = api.Batches.from_host(order, off, t_ref, dev)
                    res = api.propagate(eph, x0, 0.0, t_ref, opts, stats=stats[k] if stats is not None else False,
                                        workspace=ws[k][0])
                nxt = (k, batches, res[0], res[1])
            if pending is not None:
                k, batches, x_epoch, status = pending
                with torch.cuda.stream(streams[k]):
                    pf, ps, po, fst = api.fov_check(eph, x_epoch, batches, frames, status, opts, pairs_cap=cap,
                                                    workspace=ws[k][1], return_stats=True)
                out = (pf.numel(), fst, status)
                if marks is not None:
                    marks.append(time.perf_counter())
            pending = nxt
        for st in streams:
            st.synchronize()
        return out

    if args.copy_calibration_mib > 0:
        # a plain device copy of known size, for scaling the HBM byte counters
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # warm-up steps run the same calls as the timed ones (counters included),
    # so every kernel's code is loaded before the clock starts
    warm_stats = [torch.zeros(8, dtype=torch.int64, device=dev) for _ in streams]
    if args.warmup > 0:
        run_steps(args.warmup, warm_stats)
    torch.cuda.synchronize()
    stats_s = [torch.zeros(8, dtype=torch.int64, device=dev) for _ in streams]
    L = _lib.lib()
    L.kete_timing_enable(1)
    # as timeit does: collect first, then keep the interpreter's collector
    # out of the timed steps
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks = []
    n_pairs, fst, status = run_steps(args.steps, stats_s, marks)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gc.enable()
    stats = stats_s[0] + stats_s[1]
    # host-side return times of the steps (each ends with its pair count read; the
    # first also covers the second step's launch, as the steps are pipelined)
    log("step host times (ms): " + " ".join("%.1f" % (1e3 * (b - a)) for a, b in zip([t0] + marks[:-1], marks)))
    L.kete_timing_enable(0)
    ms = np.zeros(4); cnt = np.zeros(4, np.int64)
    _lib.check(L.kete_timing_read(ms.ctypes.data_as(C.c_void_p), cnt.ctypes.data_as(C.c_void_p)))
    st = stats.cpu().numpy()
    n_fail = int((status != 0).sum().item())
    # after the timed region: one step on its own (nothing overlaps its
    # kernels), for the integrator's launch time without a neighbour
    L.kete_timing_enable(1)
    iso_stats = [torch.zeros(8, dtype=torch.int64, device=dev) for _ in streams]
    run_steps(1, iso_stats)
    L.kete_timing_enable(0)
    ms_iso = np.zeros(4); cnt_iso = np.zeros(4, np.int64)
    _lib.check(L.kete_timing_read(ms_iso.ctypes.data_as(C.c_void_p), cnt_iso.ctypes.data_as(C.c_void_p)))

    # H-G magnitudes of one step's pairs (Sect. 3.3), an epilogue timed on
    # its own with events on the launching stream
    hg_h, hg_g = synth.hg_params(np.random.default_rng(11), N)
    hg_h, hg_g = torch.as_tensor(hg_h, device=dev), torch.as_tensor(hg_g, device=dev)
    mb = api.Batches.from_host(order, off, t_ref, dev)
    mx, mst = api.propagate(eph, x0, 0.0, t_ref, opts, workspace=ws[0][0])
    mpf, _, mpo = api.fov_check(eph, mx, mb, frames, mst, opts, pairs_cap=cap, workspace=ws[0][1])
    mws = torch.empty(L.kete_magnitudes_workspace_size(F), dtype=torch.uint8, device=dev)
    v_mag = api.pair_magnitudes(eph, mx, mb, frames, mpf, mpo, hg_h, hg_g, opts=opts, workspace=mws)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_mag_reps = 5
    ev0.record()
    for _ in range(n_mag_reps):
        api.pair_magnitudes(eph, mx, mb, frames, mpf, mpo, hg_h, hg_g, opts=opts, workspace=mws)
    ev1.record()
    torch.cuda.synchronize()
    mag_ms = ev0.elapsed_time(ev1) / n_mag_reps
    mag = {"pairs": int(mpf.numel()), "ms": mag_ms, "pairs_per_s": mpf.numel() / (mag_ms / 1e3),
           "finite": bool(torch.isfinite(v_mag).all().item()),
           "v_range": [float(v_mag.min().item()), float(v_mag.max().item())] if mpf.numel() else None}
    del mx, mst, mpf, mpo, v_mag, mws

    ms_step = elapsed * 1e3 / args.steps
    obj_days = N * case.span
    value = obj_days / (ms_step / 1e3)
    # integrator roofline (FP64 vector ALU)
    # every epoch but the last of a launch is read off the step polynomials
    dense_epochs = (B - 1) * N if dense_epochs_read else 0
    flops = (integrator_flops(st, case.ephem.n_body, n_gr, case.ephem.degree + 1) / max(cnt[0], 1)
             + dense_epochs * DENSE_FLOPS)
    t_launch_nb = ms[0] / max(cnt[0], 1) / 1e3
    achieved_tf = flops / t_launch_nb / 1e12
    # FoV candidate kernel: compulsory HBM bytes (states per batch, frames, pair keys)
    fov_bytes = B * N * 48 + F * (8 + 24 + 96 * S) + n_pairs * 8
    t_launch_fov = ms[1] / max(cnt[1], 1) / 1e3
    fov_gbs = fov_bytes / t_launch_fov / 1e9
    integ_ms_step = ms[0] / args.steps
    fov_ms_step = ms[1] / args.steps
    iso_ms = ms_iso[0] / max(cnt_iso[0], 1)
    iso_flops = (integrator_flops((iso_stats[0] + iso_stats[1]).cpu().numpy(), case.ephem.n_body, n_gr,
                                  case.ephem.degree + 1) / max(cnt_iso[0], 1) + dense_epochs * DENSE_FLOPS)
    iso_tf = iso_flops / (iso_ms / 1e3) / 1e12 if iso_ms > 0 else None
    if integ_ms_step >= fov_ms_step:
        roof = {"kernel": "k_nbody_g8 (integrator)", "bound": "alu", "achieved": achieved_tf,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved_tf / FP64_PEAK_TFLOPS,
                "traffic": measured_traffic(),
                "launches_per_step": int(cnt[0] // args.steps), "avg_launch_ms": t_launch_nb * 1e3,
                "algorithmic_flops_per_launch": flops}
    else:
        roof = {"kernel": "k_fov_cells + k_fov_wide (candidates)", "bound": "hbm", "achieved": fov_gbs,
                "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": fov_gbs / HBM_PEAK_GBS, "traffic": None,
                "launches_per_step": int(cnt[1] // args.steps), "avg_launch_ms": t_launch_fov * 1e3,
                "algorithmic_bytes_per_launch": fov_bytes}
    out = {
        "metric": "FP64 object-days/s propagated + FoV tests/s; adjoint grad cost vs forward",
        "value": value, "unit": "object-days/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": workload_name(case, F), "bodies": N, "frames": F, "sub_frames": S,
                   "batches": B, "span_days": case.span, "parallelism": "single GPU"},
        "roofline": roof,
        "components": {
            "integrator_ms_per_step": integ_ms_step, "fov_kernel_ms_per_step": fov_ms_step,
            "integrator_TFLOPs": achieved_tf, "integrator_frac_fp64_peak": achieved_tf / FP64_PEAK_TFLOPS,
            "integrator_alone_ms": iso_ms, "integrator_alone_TFLOPs": iso_tf,
            "integrator_alone_frac_fp64_peak": iso_tf / FP64_PEAK_TFLOPS if iso_tf else None,
            "fov_kernel_GBs": fov_gbs, "fov_frac_hbm": fov_gbs / HBM_PEAK_GBS,
            "fov_tests_per_s_bruteforce_equiv": N * F * S / (fov_ms_step / 1e3) if fov_ms_step > 0 else None,
            "pairs": n_pairs, "fov_candidates": int(fst[0]), "fov_exact_tests": int(fst[1]),
            "fov_bruteforce_objects": int(fst[2]), "failed_objects": n_fail,
            "integrator_counters": st[:8].tolist(),
            "magnitudes": mag,
        },
    }
    if not args.no_strict:
        log("strict n-body component ...")
        out["components"]["strict_nbody"] = strict_component(api, torch, case, eph, x0, log)
    if not args.no_adjoint:
        log("adjoint component ...")
        out["components"]["adjoint"] = adjoint_component(api, synth, torch, args.adjoint_objects, log)
    if not args.no_batched:
        log("batched component ...")
        out["components"]["batched"] = batched_component(api, synth, torch, args.batched_jobs, log,
                                                         tune_cache=args.tune_cache)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample ...")
        out["cpu_baseline"] = cpu_baseline(case, t_ref, order, off)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
