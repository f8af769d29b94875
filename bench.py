#!/usr/bin/env python3
"""Benchmark of the known-object prediction path on one MI355X.

One step is the whole path over one workload:
  frame batching (<= 3 days, host) -> n-body integration of every body to
  every batch epoch -> universal-variable light-time hops and the
  sky-binned membership test -> (frame, sub-frame, object) pairs sorted.
Inputs are resident in device memory before the timed region.

The headline workload is the full-scale one: 750,000 bodies (95% main
belt, 5% NEO-like), the default force model (Sun, 8 planets and the Moon
as 8-day degree-12 Chebyshev segments; the post-Newtonian term of the Sun,
Jupiter and the Earth; the J2 term of the Sun and Jupiter), one year,
2,000,000 ground footprints of 7 x 7.3 deg made of 8 x 8 sub-frames of
0.87 deg.  Its steps run one after the other on one stream.
The survey workload (100,000 bodies, 500,000 frames of 0.78 deg) is a
component; its steps alternate between two streams so that one step's
integrator overlaps the previous step's field-of-view kernels (stated in
its record).

Prints one JSON line.  `value` is object-days propagated per second of the
whole headline step.  The roofline block covers the headline step's
dominant kernel, timed live with HIP events on the stream it runs on;
both workloads also report the integrator's FP64 rate against the
algorithmic flop count fixed by the oracle's natural step and sweep counts
(tests/golden/oracle_counts.json).
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X vector FP64: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
HBM_PEAK_GBS = 8000.0

# Flop weights (FMA = 2, add/sub/mul = 1, reciprocal square root = 1).
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


def force_flops(n_body: int, n_gr: int, n_j2: int) -> int:
    """One force evaluation: per body the Newtonian term, the Eq. A.3 term
    for n_gr of them and the Eq. A.4 term for n_j2 of them (offset, its
    inverse norm, pole component, the two coefficients, three FMAs)."""
    return 18 * n_body + 27 * n_gr + 45 * n_j2


def node_flops(n_body: int, n_gr: int, n_j2: int = 0) -> int:
    """Predictor and force at one collocation node of one body."""
    pred_x = 3 * (1 + 14 + 4) + 1          # half_s2 F0 + 7 FMA + 2 FMA, s h
    pred_v = 3 * (1 + 14 + 2) if n_gr else 0
    return pred_x + pred_v + force_flops(n_body, n_gr, n_j2) + 3     # + D update


def sweep_flops(n_body: int, n_gr: int, n_j2: int = 0) -> int:
    """One corrector sweep of one body: 7 nodes plus b6 and the test."""
    return 7 * node_flops(n_body, n_gr, n_j2) + 3 * 14 + 12


def step_flops(n_body: int, n_gr: int, n_j2: int = 0) -> int:
    """Step end of one body: position and velocity sums, force, control."""
    return 3 * (1 + 28 + 4 + 2) + force_flops(n_body, n_gr, n_j2) + 10


def algorithmic_flops(counts: dict, n_obj: int, span: float, n_body: int, n_gr: int, n_epochs: int,
                      n_j2: int = 0) -> float:
    """FP64 flops of the method for n_obj bodies over `span` days: the
    oracle's natural steps, sweeps and extrapolated starts per body-day
    (each body integrated alone), weighted per operation, plus the epochs
    read off the step polynomials.  The perturber ephemeris is not counted:
    a wavefront evaluates it once for its bodies."""
    c = counts["extrapolated_start"]
    body_days = n_obj * span
    return (body_days * (c["steps_per_body_day"] * step_flops(n_body, n_gr, n_j2)
                         + c["sweeps_per_body_day"] * sweep_flops(n_body, n_gr, n_j2)
                         + c["extrapolated_starts_per_body_day"] * PREDICT_FLOPS)
            + max(n_epochs - 1, 0) * n_obj * DENSE_FLOPS)


def executed_flops(stats, n_body: int, n_gr: int, deg1: int, dense_epochs: int, n_j2: int = 0) -> float:
    """FP64 flops the kernel executes by its own counters: stats = [wave
    steps, wave sweeps, rejections, body-steps, body-sweeps, Clenshaw
    chains with derivative, value-only chains, body-steps started from an
    extrapolated corrector]."""
    lane_steps, lane_iter, chains, vchains = float(stats[3]), float(stats[4]), float(stats[5]), float(stats[6])
    pred = float(stats[7]) if len(stats) > 7 else 0.0
    return (lane_iter * sweep_flops(n_body, n_gr, n_j2) + lane_steps * step_flops(n_body, n_gr, n_j2)
            + chains * CLENSHAW_CHAIN_FLOPS(deg1) + vchains * CLENSHAW_VALUE_FLOPS(deg1)
            + pred * PREDICT_FLOPS + dense_epochs * DENSE_FLOPS)


def oracle_counts(name: str):
    path = os.path.join(ROOT, "tests", "golden", "oracle_counts.json")
    with open(path) as f:
        return json.load(f)[name]


def profile_figure(name: str, key: str):
    """A figure recorded in a committed profile summary, or None when the
    summary is missing or the sources it names changed since."""
    import hashlib
    import re
    try:
        txt = open(os.path.join(ROOT, "profiles", name)).read()
        val = float(re.search(r"^%s: (\S+)$" % re.escape(key), txt, re.M).group(1))
        sha = re.search(r"^sources_sha1: (\S+)$", txt, re.M).group(1)
        files = re.search(r"^sources: (.+)$", txt, re.M).group(1).split()
    except (OSError, AttributeError, ValueError):
        return None
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(ROOT, "paper_2509_04666_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return val if h.hexdigest() == sha else None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def force_model_name(eph) -> str:
    names = list(eph.names)
    planets = [n for n in names if n not in ("sun", "moon")]
    j2 = [] if eph.j2 is None else [names[i].capitalize() for i in np.nonzero(eph.j2[:, 0])[0]]
    return ("Sun + %d planets%s as %g-day degree-%d Chebyshev segments, J2 of %s"
            % (len(planets), " + Moon" if "moon" in names else "", eph.seg_days, eph.degree,
               " and ".join(j2) if j2 else "none"))


def workload_name(case) -> str:
    fr = case.frames
    if case.name == "footprint":
        return ("full-scale footprints: %d bodies (95%% main belt, 5%% NEO-like), %s, %.2f days, %d ground "
                "footprints of 7 x 7.3 deg in %d sub-frames of 0.87 deg, six sites at latitude 33 deg, 30 s "
                "exposures in 8 h nights"
                % (case.x0.shape[0], force_model_name(case.ephem), case.span, fr.n_frames, fr.n_sub))
    return ("survey: %d bodies (95%% main belt, 5%% NEO-like), %s, %.2f days, %d frames of 0.78 deg in 11 s "
            "sequences of 12 from a 1 au orbit with a 7,000 km offset orbit"
            % (case.x0.shape[0], force_model_name(case.ephem), case.span, fr.n_frames))


class Workload:
    """One workload's device inputs, workspaces and step machinery."""

    def __init__(self, api, torch, case, streams: int, log):
        import ctypes as C
        from paper_2509_04666_amd import _lib
        self.api, self.torch, self.case, self.log, self.C, self.L = api, torch, case, log, C, _lib.lib()
        self._lib = _lib
        fr = case.frames
        self.N, self.F, self.S = case.x0.shape[0], fr.n_frames, fr.n_sub
        dev = torch.device("cuda:0")
        self.dev = dev
        self.eph = api.DeviceEphemeris.from_synth(case.ephem)
        self.frames = api.DeviceFrames.from_synth(fr)
        self.x0 = torch.as_tensor(case.x0).to(dev)
        self.frame_t_host = np.ascontiguousarray(fr.t)
        self.opts = api.default_opts()
        order, off, t_ref = api.make_batches(self.frame_t_host, self.opts.batch_span)
        self.order, self.off, self.t_ref = order, off, t_ref
        self.B = t_ref.size
        self.n_gr = int(np.sum(case.ephem.flags & 1))
        self.n_j2 = 0 if case.ephem.j2 is None else int(np.count_nonzero(case.ephem.j2[:, 0]))
        # learn the pair count once, then size the pair buffers to it
        b = api.Batches.from_host(order, off, t_ref, dev)
        x, st = api.propagate(self.eph, self.x0, case.t0, t_ref, self.opts)
        pf, ps, po = api.fov_check(self.eph, x, b, self.frames, st, self.opts)
        self.cap = max(1 << 16, int(pf.numel() * 1.02) + 4096)
        del x, st, pf, ps, po
        torch.cuda.empty_cache()
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(streams)]
        size_p = self.L.kete_propagate_workspace_size(self.N, self.B, C.byref(self.opts))
        size_f = self.L.kete_fov_workspace_size(self.N, self.F, self.B, self.S, self.cap, C.byref(self.opts))
        self.ws = [(torch.empty(size_p, dtype=torch.uint8, device=dev),
                    torch.empty(size_f, dtype=torch.uint8, device=dev)) for _ in self.streams]
        log(f"{case.name}: N={self.N} F={self.F} x {self.S} sub-frames, {self.B} batches, pair capacity {self.cap}, "
            f"workspaces {size_p / 1e9:.2f} + {size_f / 1e9:.2f} GB per stream")

    def run_steps(self, K, stats=None, marks=None):
        """K steps.  With one stream each step's FoV call follows its
        propagation; with two, consecutive steps alternate between the
        streams and step i's propagation is issued before step i-1's FoV
        call, so the two overlap on the GPU."""
        api, case, opts = self.api, self.case, self.opts
        ns = len(self.streams)
        pending, out = None, None
        for i in range(K + (1 if ns > 1 else 0)):
            nxt = None
            if i < K:
                k = i % ns
                with self.torch.cuda.stream(self.streams[k]):
                    order, off, t_ref = api.make_batches(self.frame_t_host, opts.batch_span)
                    batches = api.Batches.from_host(order, off, t_ref, self.dev)
                    res = api.propagate(self.eph, self.x0, case.t0, t_ref, opts,
                                        stats=stats[k] if stats is not None else False, workspace=self.ws[k][0])
                nxt = (k, batches, res[0], res[1])
            if ns == 1:
                cur = nxt
            else:
                cur, pending = pending, nxt
            if cur is not None:
                k, batches, x_epoch, status = cur
                with self.torch.cuda.stream(self.streams[k]):
                    pf, ps, po = api.fov_check(self.eph, x_epoch, batches, self.frames, status, opts,
                                               pairs_cap=self.cap, workspace=self.ws[k][1])
                counts = np.zeros(8, np.int64)
                self.L.kete_fov_last_counts(counts.ctypes.data_as(self.C.c_void_p))
                out = (pf.numel(), counts, status)
                del pf, ps, po
                if marks is not None:
                    marks.append(time.perf_counter())
        for st in self.streams:
            st.synchronize()
        return out

    def timing_read(self):
        ms = np.zeros(8)
        cnt = np.zeros(8, np.int64)
        self._lib.check(self.L.kete_timing_read_all(ms.ctypes.data_as(self.C.c_void_p),
                                                   cnt.ctypes.data_as(self.C.c_void_p)))
        return ms, cnt

    def measure(self, steps, warmup):
        torch, case, log = self.torch, self.case, self.log
        ns = len(self.streams)
        if warmup > 0:
            self.run_steps(warmup, [torch.zeros(8, dtype=torch.int64, device=self.dev) for _ in range(ns)])
        torch.cuda.synchronize()
        stats_s = [torch.zeros(8, dtype=torch.int64, device=self.dev) for _ in range(ns)]
        self.L.kete_timing_enable(1)
        # as timeit does: collect first, then keep the collector out of the timed steps
        gc.collect()
        gc.disable()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        marks = []
        n_pairs, fcounts, status = self.run_steps(steps, stats_s, marks)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        gc.enable()
        self.L.kete_timing_enable(0)
        ms, cnt = self.timing_read()
        log(f"{case.name} step host times (ms): " +
            " ".join("%.1f" % (1e3 * (b - a)) for a, b in zip([t0] + marks[:-1], marks)))
        st = sum(s for s in stats_s).cpu().numpy()
        n_fail = int((status != 0).sum().item())
        # one more step with nothing beside it, for the integrator alone
        self.L.kete_timing_enable(1)
        iso_stats = [torch.zeros(8, dtype=torch.int64, device=self.dev) for _ in range(ns)]
        t1 = time.perf_counter()
        self.run_steps(1, iso_stats)
        torch.cuda.synchronize()
        serial_ms = (time.perf_counter() - t1) * 1e3
        self.L.kete_timing_enable(0)
        ms_iso, cnt_iso = self.timing_read()

        N, B, F, S = self.N, self.B, self.F, self.S
        eph = case.ephem
        ms_step = elapsed * 1e3 / steps
        obj_days = N * case.span
        alg = algorithmic_flops(oracle_counts("survey" if case.name == "survey" else "footprints"), N, case.span,
                                eph.n_body, self.n_gr, B, self.n_j2)
        exe = executed_flops(st, eph.n_body, self.n_gr, eph.degree + 1, (B - 1) * N * int(cnt[0]),
                             self.n_j2) / max(cnt[0], 1)
        t_int = ms[0] / max(cnt[0], 1) / 1e3
        t_int_iso = ms_iso[0] / max(cnt_iso[0], 1) / 1e3
        fov_ms = ms[1] / steps
        join_ms = ms[4] / steps
        # compulsory HBM bytes of the FoV stage: states at every epoch,
        # frames (time, observer, normals) and the sorted pair keys
        fov_bytes = B * N * 48 + F * (8 + 24 + 96 * S) + n_pairs * 8
        steps_body_yr = st[3] / max(N, 1) / steps * (365.25 / case.span)
        rec = {
            "workload": workload_name(case),
            "ms_per_step": ms_step, "object_days_per_s": obj_days / (ms_step / 1e3),
            "step_ms_one_after_another": serial_ms,
            "integrator": {
                "kernel": "k_nbody_g8", "bound": "alu", "avg_launch_ms": t_int * 1e3,
                "alone_ms": t_int_iso * 1e3,
                "algorithmic_flops_per_launch": alg,
                "algorithmic_TFLOPs": alg / t_int / 1e12, "algorithmic_frac_fp64_peak": alg / t_int / 1e12 / FP64_PEAK_TFLOPS,
                "algorithmic_frac_fp64_peak_alone": alg / t_int_iso / 1e12 / FP64_PEAK_TFLOPS,
                "kernel_counted_flops_per_launch": exe,
                "kernel_counted_TFLOPs": exe / t_int / 1e12,
                "steps_per_body_year": steps_body_yr,
                "sweeps_per_step": float(st[4]) / max(float(st[3]), 1.0),
                "oracle_natural_steps_per_body_year":
                    oracle_counts("survey" if case.name == "survey" else "footprints")["extrapolated_start"][
                        "steps_per_body_year"],
                "counters": st[:8].tolist(),
            },
            "fov": {
                "ms_per_step": fov_ms, "join_ms_per_step": join_ms,
                "algorithmic_bytes": fov_bytes, "GBs": fov_bytes / (fov_ms / 1e3) / 1e9 if fov_ms > 0 else None,
                "frac_hbm": fov_bytes / (fov_ms / 1e3) / 1e9 / HBM_PEAK_GBS if fov_ms > 0 else None,
                "tests_per_s_bruteforce_equiv": N * F * S / (fov_ms / 1e3) if fov_ms > 0 else None,
                "pairs": n_pairs, "cap_hits": int(fcounts[0]), "exact_tests": int(fcounts[1]),
                "bruteforce_objects": int(fcounts[2]), "wide_items": int(fcounts[5]),
            },
            "failed_objects": n_fail,
            "pipelining": ("consecutive steps alternate between two streams at the default priority; step i's "
                           "integrator runs beside step i-1's field-of-view kernels" if len(self.streams) > 1
                           else "none: steps run one after the other on one stream"),
        }
        return rec


def cpu_baseline(case, t_ref, order, off, n_obj_prop=8000, n_obj_fov=40000, n_frames_fov=240, serial_frac=0.25):
    """The CPU oracle as it stands, on a bounded sample of the headline
    workload: propagation of a body sample over every batch epoch, and
    brute-force membership of a body sample against the first frames of
    the first batch, on every host thread and on one (a quarter of the
    sample), each extrapolated to the whole step."""
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rng = np.random.default_rng(7)
    N = case.x0.shape[0]
    fr = case.frames
    res = {}
    for label, nt, scale in (("all_threads", threads, 1.0), ("one_thread", 1, serial_frac)):
        npp = max(50, int(n_obj_prop * scale))
        sel = np.sort(rng.choice(N, npp, replace=False))
        t0 = time.perf_counter()
        xe, st, _ = O.propagate(case.ephem, case.x0[sel], case.t0, t_ref, opts=O.make_opts(n_threads=nt))
        t_prop = time.perf_counter() - t0
        rate_prop = npp * case.span / t_prop
        nfo = min(N, max(200, int(n_obj_fov * scale)))
        nfr = min(int(off[1]), max(10, int(n_frames_fov * scale)))
        sel_f = np.sort(rng.choice(N, nfo, replace=False))
        xf, sf, _ = O.propagate(case.ephem, case.x0[sel_f], case.t0, t_ref[:1], opts=O.make_opts(n_threads=threads))
        t1 = time.perf_counter()
        O.fov(case.ephem, xf, sf, order[:nfr], np.array([0, nfr]), t_ref[:1], fr.t, fr.obs, fr.normals, n_threads=nt)
        t_fov = time.perf_counter() - t1
        rate_fov = nfo * nfr * fr.n_sub / t_fov
        t_total = N * case.span / rate_prop + N * fr.n_frames * fr.n_sub / rate_fov
        res[label] = {"threads": nt, "object_days_per_s": N * case.span / t_total,
                      "propagation_object_days_per_s": rate_prop, "fov_tests_per_s": rate_fov,
                      "sample": (f"propagation of {npp} bodies over all {t_ref.size} batch epochs ({t_prop:.2f} s) "
                                 f"and brute-force membership of {nfo} bodies x {nfr} frames x {fr.n_sub} "
                                 f"sub-frames ({t_fov:.2f} s)")}
    a = res["all_threads"]
    return {
        "value": a["object_days_per_s"], "unit": "object-days/s", "cores": threads, "kind": "oracle",
        "sample": a["sample"] + f", extrapolated to {N} bodies x {fr.n_frames} frames",
        "cpu_model": cpu_model(), "logical_cpus_seen": os.cpu_count(),
        "propagation_object_days_per_s": a["propagation_object_days_per_s"],
        "fov_tests_per_s": a["fov_tests_per_s"],
        "one_thread": res["one_thread"],
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
        "workload": f"{n_obj} bodies x 20 observations over 60 days, {force_model_name(g.ephem)}, "
                    "checkpoints every 5 days",
        "forward_ms": t_f * 1e3, "backward_ms": t_b * 1e3, "backward_over_forward": t_b / t_f,
        "gradient_over_forward": (t_f + t_b) / t_f,
        "forward_object_days_per_s": n_obj * 60.0 / t_f, "failed_objects": n_fail,
        "grad_finite": bool(torch.isfinite(grad).all().item()),
    }


def batched_component(api, synth, torch, n_jobs, log, reps=2, tune_cache=None):
    """Uneven jobs (log-uniform 1-20,000 bodies, 1 day-10 years, 1-5,000
    frames): the whole set as one captured graph replay against one
    propagation call and one FoV call per job, each path warmed up once and
    run with the tuned options."""
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
    ms = np.zeros(8); cnt = np.zeros(8, np.int64)
    _lib.check(L.kete_timing_read_all(ms.ctypes.data_as(C.c_void_p), cnt.ctypes.data_as(C.c_void_p)))
    pf, ps, po = runner.pairs()
    n_pairs_batched = pf.numel()

    # one propagation call and one FoV call per job, inputs already on the
    # device, with the same tuned options
    opts = best
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

    per_job()                                   # warm-up pass
    torch.cuda.synchronize()
    t_jobs = []
    for _ in range(reps):
        t0 = time.perf_counter()
        n_pairs_job = per_job()
        torch.cuda.synchronize()
        t_jobs.append(time.perf_counter() - t0)
    t_job = min(t_jobs)
    return {
        "workload": (f"{len(jobs)} uneven jobs: log-uniform 1-20,000 bodies, 1 day-10 years, 1-5,000 frames; "
                     f"{n_bodies} bodies, {int(runner.frame_off[-1])} frames"),
        "object_days": obj_days, "graph_ms": t_graph * 1e3, "per_job_ms": t_job * 1e3,
        "per_job_ms_runs": [t * 1e3 for t in t_jobs],
        "speedup_vs_per_job": t_job / t_graph, "object_days_per_s": obj_days / t_graph,
        "graph_launch_event_ms": ms[3] / max(cnt[3], 1),
        "pairs": n_pairs_batched, "pairs_per_job_path": n_pairs_job,
        "tuned": {k: getattr(best, k) for k in ("n_buckets", "persist_waves", "window_segs", "fov_block",
                                                "cell_chord")},
        "tuning_from_cache": hit,
    }


def magnitudes_component(api, synth, torch, wl, L, log, reps=5):
    """H-G magnitudes of one step's pairs (Sect. 3.3), an epilogue timed on
    its own with events on the launching stream."""
    N, dev = wl.N, wl.dev
    hg_h, hg_g = synth.hg_params(np.random.default_rng(11), N)
    hg_h, hg_g = torch.as_tensor(hg_h, device=dev), torch.as_tensor(hg_g, device=dev)
    mb = api.Batches.from_host(wl.order, wl.off, wl.t_ref, dev)
    mx, mst = api.propagate(wl.eph, wl.x0, wl.case.t0, wl.t_ref, wl.opts, workspace=wl.ws[0][0])
    mpf, _, mpo = api.fov_check(wl.eph, mx, mb, wl.frames, mst, wl.opts, pairs_cap=wl.cap, workspace=wl.ws[0][1])
    mws = torch.empty(L.kete_magnitudes_workspace_size(wl.F), dtype=torch.uint8, device=dev)
    v_mag = api.pair_magnitudes(wl.eph, mx, mb, wl.frames, mpf, mpo, hg_h, hg_g, opts=wl.opts, workspace=mws)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        api.pair_magnitudes(wl.eph, mx, mb, wl.frames, mpf, mpo, hg_h, hg_g, opts=wl.opts, workspace=mws)
    ev1.record()
    torch.cuda.synchronize()
    mag_ms = ev0.elapsed_time(ev1) / reps
    return {"pairs": int(mpf.numel()), "ms": mag_ms, "pairs_per_s": mpf.numel() / (mag_ms / 1e3),
            "finite": bool(torch.isfinite(v_mag).all().item()),
            "v_range": [float(v_mag.min().item()), float(v_mag.max().item())] if mpf.numel() else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=("footprints", "survey"), default="footprints",
                    help="headline workload (the other one, when run, is a component)")
    ap.add_argument("--survey-steps", type=int, default=20)
    ap.add_argument("--no-survey", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint-objects", type=int, default=100_000)
    ap.add_argument("--batched-jobs", type=int, default=4096)
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2509_04666_amd", "tuning.json"))
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-strict", action="store_true")
    ap.add_argument("--no-magnitudes", action="store_true")
    ap.add_argument("--head-streams", type=int, default=0,
                    help="streams the headline steps alternate over (0: the workload's default)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="copy a buffer of this size once before timing (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the objects are independent "
              "and the path would shard them over GPUs; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_04666_amd import api, synth, _lib

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    L = _lib.lib()
    t_setup = time.perf_counter()
    survey = synth.survey_case()
    head_case = synth.footprint_case() if args.workload == "footprints" else survey
    log(f"generated in {time.perf_counter() - t_setup:.1f} s")
    if args.copy_calibration_mib > 0:
        # a plain device copy of known size, for scaling the HBM byte counters
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    head_streams = args.head_streams if args.head_streams > 0 else (1 if head_case.name == "footprint" else 2)
    head = Workload(api, torch, head_case, head_streams, log)
    hrec = head.measure(args.steps, args.warmup)
    components = {}
    if head_case.name == "footprint" and not args.no_magnitudes:
        log("magnitudes component ...")
        components["magnitudes"] = magnitudes_component(api, synth, torch, head, L, log)
    head_cpu = (head_case, head.t_ref, head.order, head.off)
    del head
    torch.cuda.empty_cache()

    if head_case.name == "footprint" and not args.no_survey:
        log("survey component ...")
        sw = Workload(api, torch, survey, 2, log)
        components["survey"] = sw.measure(args.survey_steps, 3)
        if not args.no_strict:
            log("strict n-body component ...")
            components["strict_nbody"] = strict_component(api, torch, survey, sw.eph, sw.x0, log)
        del sw
        torch.cuda.empty_cache()
    if not args.no_adjoint:
        log("adjoint component ...")
        components["adjoint"] = adjoint_component(api, synth, torch, args.adjoint_objects, log)
    if not args.no_batched:
        log("batched component ...")
        components["batched"] = batched_component(api, synth, torch, args.batched_jobs, log,
                                                  tune_cache=args.tune_cache)
        torch.cuda.empty_cache()

    # roofline of the headline step's dominant kernel; valu_issue_frac is the
    # share of its time the SIMDs spend issuing its vector instructions (SQ
    # counters in the committed profile, None once its sources changed)
    integ, fov = hrec["integrator"], hrec["fov"]
    if integ["avg_launch_ms"] >= fov["join_ms_per_step"]:
        roof = {"kernel": "k_nbody_g8 (integrator)", "bound": "alu", "achieved": integ["algorithmic_TFLOPs"],
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": integ["algorithmic_frac_fp64_peak"],
                "traffic": profile_figure("traffic_k_nbody_g8_%s.md" % head_case.name, "traffic_bytes_per_launch"),
                "valu_issue_frac": profile_figure("sq_counters_%s.md" % head_case.name,
                                                  "valu_issue_share_integrator"),
                "launches_per_step": 1, "avg_launch_ms": integ["avg_launch_ms"],
                "algorithmic_flops_per_launch": integ["algorithmic_flops_per_launch"]}
    else:
        # the join (k_fov_cells + k_fov_wide, with its item kernels) reads the
        # epoch states, the frames and writes the surely-inside pair keys
        jb = fov["algorithmic_bytes"]
        roof = {"kernel": "k_fov_cells + k_fov_wide (field-of-view join)", "bound": "hbm",
                "achieved": jb / (fov["join_ms_per_step"] / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": jb / (fov["join_ms_per_step"] / 1e3) / 1e9 / HBM_PEAK_GBS,
                "traffic": profile_figure("traffic_fov_join_%s.md" % head_case.name, "traffic_bytes_per_step"),
                "valu_issue_frac": profile_figure("sq_counters_%s.md" % head_case.name, "valu_issue_share_join"),
                "launches_per_step": 1, "avg_launch_ms": fov["join_ms_per_step"],
                "algorithmic_bytes_per_launch": jb}
    out = {
        "metric": "FP64 object-days/s propagated + FoV tests/s; adjoint grad cost vs forward",
        "value": hrec["object_days_per_s"], "unit": "object-days/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": hrec["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": hrec["workload"], "bodies": head_case.x0.shape[0],
                   "frames": head_case.frames.n_frames, "sub_frames": head_case.frames.n_sub,
                   "span_days": head_case.span, "parallelism": "single GPU", "pipelining": hrec["pipelining"]},
        "roofline": roof,
        "headline": hrec,
        "components": components,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample ...")
        out["cpu_baseline"] = cpu_baseline(*head_cpu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
