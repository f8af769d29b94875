"""Python entry points over the C ABI.  Torch supplies device memory and
streams; every step of the path runs in the library's HIP kernels."""
from __future__ import annotations

import copy
import ctypes as C
import dataclasses
import hashlib
import json
import math
import os
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import EphemT, FramesT, OptsT, check, lib

DEV = "cuda"


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_opts(**kw) -> OptsT:
    o = OptsT()
    lib().kete_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class DeviceEphemeris:
    """A Chebyshev ephemeris with its coefficient table in device memory."""

    def __init__(self, coef, gm, flags, t_start: float, seg_days: float, device=DEV, j2=None):
        """j2: None, or [n_body, 5] rows {J2, radius au, unit pole} of the
        App. A.3 term (J2 = 0: none)."""
        self.coef = torch.as_tensor(np.ascontiguousarray(coef), dtype=torch.float64).to(device).contiguous()
        self.gm = np.ascontiguousarray(gm, dtype=np.float64)
        self.flags = np.ascontiguousarray(flags, dtype=np.uint32)
        self.t_start = float(t_start)
        self.seg_days = float(seg_days)
        nb, ns, three, m = self.coef.shape
        assert three == 3
        self.j2 = None if j2 is None else np.ascontiguousarray(np.asarray(j2, dtype=np.float64).reshape(nb, 5))
        self.c = EphemT(nb, ns, m - 1, 0, self.t_start, self.seg_days, self.coef.data_ptr(),
                        self.gm.ctypes.data_as(C.POINTER(C.c_double)),
                        self.flags.ctypes.data_as(C.POINTER(C.c_uint32)),
                        None if self.j2 is None else self.j2.ctypes.data_as(C.POINTER(C.c_double)))

    @staticmethod
    def from_synth(e, device=DEV) -> "DeviceEphemeris":
        return DeviceEphemeris(e.coef, e.gm, e.flags, e.t_start, e.seg_days, device, getattr(e, "j2", None))

    @property
    def n_body(self): return self.coef.shape[0]

    @property
    def t_end(self): return self.t_start + self.coef.shape[1] * self.seg_days


def _workspace(nbytes: int, device=DEV) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def propagate(eph: DeviceEphemeris, x0: torch.Tensor, t0: float, t_out: Sequence[float],
              opts: Optional[OptsT] = None, stats=False, workspace: Optional[torch.Tensor] = None):
    """States at every epoch: (x_out [E, N, 6], status [N] int32[, stats [8] int64]).  stats may be
    an int64 [8] device tensor that the kernels add their counters into."""
    opts = opts or default_opts()
    x0 = x0.contiguous()
    assert x0.dtype == torch.float64 and x0.is_cuda and x0.dim() == 2 and x0.shape[1] == 6
    t_out = np.ascontiguousarray(np.atleast_1d(np.asarray(t_out, dtype=np.float64)))
    n, E = x0.shape[0], t_out.size
    x_out = torch.empty((E, n, 6), dtype=torch.float64, device=x0.device)
    status = torch.empty(n, dtype=torch.int32, device=x0.device)
    if isinstance(stats, torch.Tensor):
        assert stats.dtype == torch.int64 and stats.numel() == 8 and stats.device == x0.device
        st = stats
    else:
        st = torch.zeros(8, dtype=torch.int64, device=x0.device) if stats else None
    need = lib().kete_propagate_workspace_size(n, E, C.byref(opts))
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, x0.device)
    check(lib().kete_propagate_nbody(C.byref(eph.c), _ptr(x0), float(t0), n,
                                     t_out.ctypes.data_as(C.c_void_p), E, _ptr(x_out), _ptr(status), _ptr(st),
                                     C.byref(opts), _ptr(ws), ws.numel(), _stream()))
    return (x_out, status, st) if st is not None else (x_out, status)


def make_batches(t: np.ndarray, span: float = 3.0):
    """(frame_order int32 [F], batch_off int32 [B+1], t_ref float64 [B]) on the host."""
    t = np.ascontiguousarray(t, dtype=np.float64)
    F = t.size
    order = np.empty(F, np.int32)
    off = np.empty(F + 1, np.int32)
    t_ref = np.empty(max(F, 1), np.float64)
    nb = C.c_int64(0)
    check(lib().kete_make_batches(t.ctypes.data_as(C.c_void_p), F, float(span), order.ctypes.data_as(C.c_void_p),
                                  off.ctypes.data_as(C.c_void_p), t_ref.ctypes.data_as(C.c_void_p), C.byref(nb)))
    B = nb.value
    return order, off[:B + 1].copy(), t_ref[:B].copy()


@dataclasses.dataclass
class DeviceFrames:
    t: torch.Tensor          # [F]
    obs: torch.Tensor        # [F, 3]
    normals: torch.Tensor    # [F, S, 4, 3]

    @staticmethod
    def from_synth(fr, device=DEV) -> "DeviceFrames":
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(device).contiguous()
        return DeviceFrames(f(fr.t), f(fr.obs), f(fr.normals))

    def c(self) -> FramesT:
        return FramesT(self.t.shape[0], self.normals.shape[1], 0, self.t.data_ptr(), self.obs.data_ptr(),
                       self.normals.data_ptr())


@dataclasses.dataclass
class Batches:
    frame_order: torch.Tensor   # device int32 [F]
    batch_off: torch.Tensor     # device int32 [B+1]
    t_ref: torch.Tensor         # device float64 [B]
    t_ref_host: np.ndarray

    @staticmethod
    def from_host(order, off, t_ref, device=DEV) -> "Batches":
        return Batches(torch.as_tensor(order).to(device), torch.as_tensor(off).to(device),
                       torch.as_tensor(t_ref).to(device), np.asarray(t_ref))


def fov_check(eph: DeviceEphemeris, x_epoch: torch.Tensor, batches: Batches, frames: DeviceFrames,
              status: Optional[torch.Tensor] = None, opts: Optional[OptsT] = None, pairs_cap: Optional[int] = None,
              workspace: Optional[torch.Tensor] = None, return_stats: bool = False):
    """Pairs sorted by (frame, sub-frame, object): (pf, ps, po) int32 tensors.
    status [N] int32 (optional) is read (objects to skip) and updated in
    place: an object whose hop ends on the Kepler iteration cap gets
    KETE_ST_KEPLER_NOCONV and loses all of its pairs."""
    opts = opts or default_opts()
    x_epoch = x_epoch.contiguous()
    B, N = x_epoch.shape[0], x_epoch.shape[1]
    F, S = frames.t.shape[0], frames.normals.shape[1]
    cap = int(pairs_cap) if pairs_cap is not None else max(1 << 16, 4 * F)
    fc = frames.c()
    for attempt in range(3):
        need = lib().kete_fov_workspace_size(N, F, B, S, cap, C.byref(opts))
        if need == 0:
            check(_lib.KETE_EINVAL)
        ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, x_epoch.device)
        pf = torch.empty(max(cap, 1), dtype=torch.int32, device=x_epoch.device)
        ps = torch.empty_like(pf)
        po = torch.empty_like(pf)
        n_pairs = C.c_int64(0)
        rc = lib().kete_fov_check(C.byref(eph.c), _ptr(x_epoch), _ptr(status), N, B, _ptr(batches.t_ref),
                                  _ptr(batches.batch_off), _ptr(batches.frame_order), C.byref(fc), C.byref(opts),
                                  _ptr(pf), _ptr(ps), _ptr(po), cap, C.byref(n_pairs), _ptr(ws), ws.numel(),
                                  _stream())
        if rc == _lib.KETE_ECAPACITY and pairs_cap is None and attempt < 2:
            cap = int(n_pairs.value)
            ws = None
            continue
        check(rc)
        break
    n = n_pairs.value
    out = (pf[:n], ps[:n], po[:n])
    if return_stats:
        st = np.zeros(4, np.int64)
        lib().kete_fov_last_stats(st.ctypes.data_as(C.c_void_p))
        return out + (st,)
    return out


def pair_magnitudes(eph: DeviceEphemeris, x_epoch: torch.Tensor, batches: Batches, frames: DeviceFrames,
                    pf: torch.Tensor, po: torch.Tensor, h_mag: torch.Tensor, g_slope: torch.Tensor,
                    geometry: bool = False, opts: Optional[OptsT] = None, workspace: Optional[torch.Tensor] = None):
    """H-G apparent V magnitude of every pair (pf[i], po[i]): a float64
    tensor [P], plus {r_H, Delta, phase angle} [P, 3] with geometry=True."""
    opts = opts or default_opts()
    x_epoch = x_epoch.contiguous()
    B, N = x_epoch.shape[0], x_epoch.shape[1]
    P = pf.shape[0]
    dev = x_epoch.device
    v = torch.empty(P, dtype=torch.float64, device=dev)
    geom = torch.empty((P, 3), dtype=torch.float64, device=dev) if geometry else None
    need = lib().kete_magnitudes_workspace_size(frames.t.shape[0])
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, dev)
    fc = frames.c()
    check(lib().kete_pair_magnitudes(C.byref(eph.c), _ptr(x_epoch), N, B, _ptr(batches.t_ref),
                                     _ptr(batches.batch_off), _ptr(batches.frame_order), C.byref(fc),
                                     _ptr(pf.contiguous()), _ptr(po.contiguous()), P, _ptr(h_mag.contiguous()),
                                     _ptr(g_slope.contiguous()), _ptr(v), _ptr(geom), C.byref(opts), _ptr(ws),
                                     ws.numel(), _stream()))
    return (v, geom) if geometry else v


def pair_magnitudes_noalloc(eph: DeviceEphemeris, x_epoch: torch.Tensor, batches: Batches, frames: DeviceFrames,
                            pf: torch.Tensor, po: torch.Tensor, h_mag: torch.Tensor, g_slope: torch.Tensor,
                            v_mag: torch.Tensor, geom: Optional[torch.Tensor] = None,
                            opts: Optional[OptsT] = None) -> None:
    """pair_magnitudes into caller-allocated outputs v_mag [P] (and geom
    [P, 3]) through the entry point that allocates no device memory (its
    frame-to-batch map is the library's static array)."""
    opts = opts or default_opts()
    x_epoch = x_epoch.contiguous()
    B, N = x_epoch.shape[0], x_epoch.shape[1]
    P = pf.shape[0]
    if v_mag.numel() < P or (geom is not None and geom.numel() < 3 * P):
        raise ValueError("output tensors are smaller than the pair count")
    fc = frames.c()
    check(lib().kete_pair_magnitudes_noalloc(C.byref(eph.c), _ptr(x_epoch), N, B, _ptr(batches.t_ref),
                                             _ptr(batches.batch_off), _ptr(batches.frame_order), C.byref(fc),
                                             _ptr(pf.contiguous()), _ptr(po.contiguous()), P,
                                             _ptr(h_mag.contiguous()), _ptr(g_slope.contiguous()), _ptr(v_mag),
                                             _ptr(geom), C.byref(opts), _stream()))


def lighttime_directions(eph: DeviceEphemeris, x_ref: torch.Tensor, t_ref: float, t_obs: torch.Tensor,
                         obs: torch.Tensor, opts: Optional[OptsT] = None):
    """(d [Q, N, 3], tau [Q, N]) for states x_ref [N, 6] at t_ref."""
    opts = opts or default_opts()
    N, Q = x_ref.shape[0], t_obs.shape[0]
    d = torch.empty((Q, N, 3), dtype=torch.float64, device=x_ref.device)
    tau = torch.empty((Q, N), dtype=torch.float64, device=x_ref.device)
    check(lib().kete_lighttime_directions(C.byref(eph.c), _ptr(x_ref.contiguous()), float(t_ref), N,
                                          _ptr(t_obs.contiguous()), _ptr(obs.contiguous()), Q, _ptr(d), _ptr(tau),
                                          C.byref(opts), _stream()))
    return d, tau


def ephem_eval(eph: DeviceEphemeris, t: np.ndarray) -> torch.Tensor:
    """Positions and velocities [Q, n_body, 6] of every perturber at times t."""
    t = np.ascontiguousarray(np.atleast_1d(t), dtype=np.float64)
    td = torch.as_tensor(t).to(eph.coef.device)
    out = torch.empty((t.size, eph.n_body, 6), dtype=torch.float64, device=eph.coef.device)
    check(lib().kete_ephem_eval(C.byref(eph.c), _ptr(td), t.ctypes.data_as(C.c_void_p), t.size, _ptr(out),
                                _stream()))
    return out


def predict(eph: DeviceEphemeris, x0: torch.Tensor, t0: float, frames: DeviceFrames, frame_t_host: np.ndarray,
            opts: Optional[OptsT] = None, pairs_cap: Optional[int] = None):
    """The whole path: batch the frames, integrate to every batch epoch,
    test membership.  Returns (pf, ps, po, x_epoch, status, batches)."""
    opts = opts or default_opts()
    order, off, t_ref = make_batches(frame_t_host, opts.batch_span)
    batches = Batches.from_host(order, off, t_ref, x0.device)
    x_epoch, status = propagate(eph, x0, t0, t_ref, opts)
    pf, ps, po = fov_check(eph, x_epoch, batches, frames, status, opts, pairs_cap)
    return pf, ps, po, x_epoch, status, batches


class AdjointContext:
    """Inputs and workspace shared by the forward and backward adjoint calls.

    The forward call leaves its checkpoints, light times and status in the
    shared workspace, and the backward call reads them.  Each forward bumps
    `generation`; AdjointSky records it and its backward refuses to run
    once a later forward on the same context has overwritten that state
    (use one context per pending backward)."""

    def __init__(self, eph: DeviceEphemeris, t0: float, t_end: float, t_obs: torch.Tensor, obs_pos: torch.Tensor,
                 ckpt_days: float = 5.0, opts: Optional[OptsT] = None):
        self.eph, self.t0, self.t_end, self.ckpt_days = eph, float(t0), float(t_end), float(ckpt_days)
        self.t_obs = t_obs.contiguous()
        self.obs_pos = obs_pos.contiguous()
        self.opts = opts or default_opts()
        self.n_obj, self.k_obs = self.t_obs.shape
        need = lib().kete_adjoint_workspace_size(self.n_obj, self.k_obs, self.t0, self.t_end, self.ckpt_days,
                                                 C.byref(self.opts))
        if need == 0:
            check(_lib.KETE_EINVAL)
        self.workspace = _workspace(need, self.t_obs.device)
        self.status = torch.zeros(self.n_obj, dtype=torch.int32, device=self.t_obs.device)
        self.generation = 0

    def forward(self, x0: torch.Tensor) -> torch.Tensor:
        """Sky positions [N, K, 2]; the workspace now belongs to this call."""
        self.generation += 1
        return self._run_forward(x0)

    def backward(self, x0: torch.Tensor, dL_dsky: torch.Tensor) -> torch.Tensor:
        """dL/dx0 [N, 6] of the latest forward call."""
        return self._run_backward(x0, dL_dsky)

    def _run_forward(self, x0: torch.Tensor) -> torch.Tensor:
        sky = torch.empty((self.n_obj, self.k_obs, 2), dtype=torch.float64, device=x0.device)
        check(lib().kete_propagate_adjoint(C.byref(self.eph.c), _lib.ADJ_FWD, _ptr(x0.contiguous()), self.t0,
                                           self.t_end, self.n_obj, self.k_obs, _ptr(self.t_obs), _ptr(self.obs_pos),
                                           None, self.ckpt_days, _ptr(sky), None, _ptr(self.status),
                                           C.byref(self.opts), _ptr(self.workspace), self.workspace.numel(),
                                           _stream()))
        return sky

    def _run_backward(self, x0: torch.Tensor, dL_dsky: torch.Tensor) -> torch.Tensor:
        grad = torch.empty((self.n_obj, 6), dtype=torch.float64, device=x0.device)
        check(lib().kete_propagate_adjoint(C.byref(self.eph.c), _lib.ADJ_BWD, _ptr(x0.contiguous()), self.t0,
                                           self.t_end, self.n_obj, self.k_obs, _ptr(self.t_obs), _ptr(self.obs_pos),
                                           _ptr(dL_dsky.contiguous()), self.ckpt_days, None, _ptr(grad),
                                           _ptr(self.status), C.byref(self.opts), _ptr(self.workspace),
                                           self.workspace.numel(), _stream()))
        return grad


class AdjointSky(torch.autograd.Function):
    """sky = AdjointSky.apply(x0, ctx): RA/Dec [N, K, 2] of every
    observation; backward runs the library's adjoint kernel."""

    @staticmethod
    def forward(fctx, x0: torch.Tensor, actx: AdjointContext):
        fctx.actx = actx
        fctx.save_for_backward(x0)
        sky = actx.forward(x0.detach())
        fctx.generation = actx.generation
        return sky

    @staticmethod
    def backward(fctx, g_sky):
        (x0,) = fctx.saved_tensors
        if fctx.generation != fctx.actx.generation:
            raise RuntimeError("AdjointSky backward: a later forward call on the same AdjointContext has "
                               "overwritten the checkpoints this gradient needs; use one context per pending "
                               "backward")
        return fctx.actx.backward(x0.detach(), g_sky), None


def sky_residual_loss(sky: torch.Tensor, radec_obs: torch.Tensor) -> torch.Tensor:
    """Sum over objects and observations of ((ra - ra_obs) cos dec)^2 + (dec - dec_obs)^2,
    with the RA difference wrapped to (-pi, pi]."""
    dra = torch.remainder(sky[..., 0] - radec_obs[..., 0] + math.pi, 2 * math.pi) - math.pi
    r1 = dra * torch.cos(sky[..., 1])
    r2 = sky[..., 1] - radec_obs[..., 1]
    return (r1 * r1 + r2 * r2).sum()


class BatchRunner:
    """Many independent jobs (bodies + frames) run as one batch: a
    persistent propagation launch over all jobs, then the field-of-view
    stages over every job's batches.  `jobs` is a list of
    (x0 [n, 6] numpy, t0, frames) with frames a synth.Frames-like object.
    Device tables are built once here (setup); run() and graph replays only
    launch work.  Body and frame numbers in the pairs are global: job k's
    body i is row obj_off[k] + i, its frame f is frame_off[k] + f."""

    def __init__(self, eph: DeviceEphemeris, jobs, opts: Optional[OptsT] = None, pairs_cap: Optional[int] = None,
                 device=DEV):
        self.eph = eph
        self.opts = opts or default_opts()
        n_obj = [j[0].shape[0] for j in jobs]
        self.obj_off = np.concatenate([[0], np.cumsum(n_obj)]).astype(np.int64)
        n_fr = [j[2].t.shape[0] for j in jobs]
        self.frame_off = np.concatenate([[0], np.cumsum(n_fr)]).astype(np.int64)
        job_rows, epochs, orders, offs, bjob, bep, trefs = [], [], [], [0], [], [], []
        ep_off, xo = 0, 0
        self.job_epochs = []
        for k, (x0, t0, fr) in enumerate(jobs):
            order, off, t_ref = make_batches(fr.t, self.opts.batch_span)
            # epochs visited away from t0: later ones ascending, then earlier ones descending
            idx = np.arange(t_ref.size)
            visit = np.concatenate([idx[t_ref >= t0], idx[t_ref < t0][::-1]])
            pos = np.empty_like(idx)
            pos[visit] = np.arange(visit.size)
            job_rows.append((int(self.obj_off[k]), ep_off, xo, x0.shape[0], t_ref.size, float(t0)))
            epochs.append(t_ref[visit])
            self.job_epochs.append(t_ref[visit])
            orders.append(order.astype(np.int64) + self.frame_off[k])
            offs.extend((off[1:] + self.frame_off[k]).tolist())
            bjob.extend([k] * t_ref.size)
            bep.extend(pos.tolist())
            trefs.append(t_ref)
            ep_off += t_ref.size
            xo += 6 * x0.shape[0] * t_ref.size
        self.n_x = xo
        self.jobs_host = (_lib.JobT * len(jobs))(*[_lib.JobT(*r) for r in job_rows])
        jb = np.frombuffer(self.jobs_host, dtype=np.uint8).copy()
        f = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a, dtype=dt)).to(device)
        self.jobs_dev = torch.as_tensor(jb).to(device)
        self.x0 = f(np.concatenate([j[0] for j in jobs]), np.float64)
        self.epochs_host = np.ascontiguousarray(np.concatenate(epochs), dtype=np.float64)
        self.epochs = f(self.epochs_host, np.float64)
        self.bjob = np.ascontiguousarray(bjob, dtype=np.int32)
        self.bep = np.ascontiguousarray(bep, dtype=np.int32)
        self.boff_host = np.ascontiguousarray(offs, dtype=np.int32)
        self.t_ref = f(np.concatenate(trefs), np.float64)
        self.boff = f(self.boff_host, np.int32)
        self.order = f(np.concatenate(orders), np.int32)
        cat = lambda name: np.concatenate([getattr(j[2], name) for j in jobs])
        self.frames = DeviceFrames(f(cat("t"), np.float64), f(cat("obs"), np.float64), f(cat("normals"), np.float64))
        self.fc = self.frames.c()
        self.c = _lib.BatchT(len(jobs), 0, int(self.obj_off[-1]), int(ep_off), int(self.bjob.size),
                             C.addressof(self.jobs_host), self.jobs_dev.data_ptr(), self.x0.data_ptr(),
                             self.epochs.data_ptr(), self.epochs_host.ctypes.data, self.bjob.ctypes.data,
                             self.bep.ctypes.data,
                             self.boff_host.ctypes.data, self.t_ref.data_ptr(), self.boff.data_ptr(),
                             self.order.data_ptr(), self.fc)
        F = int(self.frame_off[-1])
        self.pairs_cap = int(pairs_cap) if pairs_cap is not None else max(1 << 16, 8 * F)
        self.device = device
        self.x_out = torch.empty(max(self.n_x, 1), dtype=torch.float64, device=device)
        self.status = torch.zeros(max(int(self.obj_off[-1]), 1), dtype=torch.int32, device=device)
        self.pf = torch.empty(self.pairs_cap, dtype=torch.int32, device=device)
        self.ps = torch.empty_like(self.pf)
        self.po = torch.empty_like(self.pf)
        self.workspace = None
        self.graph = None
        self.set_opts(self.opts)

    def _ws_size(self, opts) -> int:
        need = lib().kete_batch_workspace_size(C.byref(self.eph.c), C.byref(self.c), self.pairs_cap, C.byref(opts))
        if need == 0:
            raise _lib.KeteError(_lib.KETE_EINVAL, lib().kete_last_error().decode())
        return need

    def set_opts(self, opts: OptsT, workspace_bytes: int = 0):
        """Adopt `opts`: (re)allocate the workspace if it is too small and plan."""
        self.drop_graph()
        self.opts = opts
        need = max(self._ws_size(opts), int(workspace_bytes))
        if self.workspace is None or self.workspace.numel() < need:
            self.workspace = None
            self.workspace = _workspace(need, self.device)
        check(lib().kete_batch_plan(C.byref(self.eph.c), C.byref(self.c), self.pairs_cap, C.byref(opts),
                                    _ptr(self.workspace), self.workspace.numel(), _stream()))

    def signature(self) -> str:
        """Hash of the batch description (jobs, epochs and batch tables)."""
        h = hashlib.sha1()
        for a in (np.frombuffer(self.jobs_host, dtype=np.uint8), self.epochs_host, self.bjob, self.bep,
                  self.boff_host):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(np.int64([self.pairs_cap, self.fc.n_sub]).tobytes())
        return h.hexdigest()

    def autotune(self, reps: int = 1, cache: Optional[str] = None, progress=None):
        """Pick launch parameters with the library's autotuner.  With `cache`
        (a JSON file), a result stored under this device and batch is reused
        and a new one is stored.  Returns (opts, ms per run, from_cache)."""
        props = torch.cuda.get_device_properties(self.device)
        key = f"{getattr(props, 'gcnArchName', props.name)}|cu{props.multi_processor_count}|{self.signature()}"
        tuned = ("n_buckets", "persist_waves", "window_segs", "fov_block", "cell_chord")
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                entry = json.load(fh).get(key)
            if entry:
                o = copy.copy(self.opts)
                for k in tuned:
                    setattr(o, k, entry[k])
                self.set_opts(o)
                return o, float(entry["ms"]), True
        # room for the largest candidate grid (smaller sky cells need more keys)
        probe = copy.copy(self.opts)
        probe.cell_chord = 0.04
        self.set_opts(self.opts, max(self._ws_size(probe), self._ws_size(self.opts)))
        best = OptsT()
        ms = C.c_double(0.0)

        def report(o, t, _user):
            if progress is not None:
                progress({k: getattr(o.contents, k) for k in tuned}, t)

        cb = _lib.TUNE_PROGRESS(report)
        check(lib().kete_batch_autotune(C.byref(self.eph.c), C.byref(self.c), self.pairs_cap, C.byref(self.opts),
                                        int(reps), _ptr(self.x_out), _ptr(self.status), _ptr(self.workspace),
                                        self.workspace.numel(), _stream(), cb, None, C.byref(best), C.byref(ms)))
        self.opts = best
        if cache:
            data = {}
            if os.path.exists(cache):
                with open(cache) as fh:
                    data = json.load(fh)
            data[key] = {k: getattr(best, k) for k in tuned}
            data[key]["ms"] = ms.value
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            with open(cache, "w") as fh:
                json.dump(data, fh, indent=1, sort_keys=True)
        return best, ms.value, False

    def drop_graph(self):
        if getattr(self, "graph", None) is not None:
            lib().kete_batch_graph_destroy(self.graph)
            self.graph = None

    def run(self):
        check(lib().kete_batch_run(C.byref(self.eph.c), C.byref(self.c), self.pairs_cap, C.byref(self.opts),
                                   _ptr(self.x_out), _ptr(self.status), _ptr(self.workspace),
                                   self.workspace.numel(), _stream()))

    def capture(self):
        self.drop_graph()
        g = C.c_void_p(0)
        check(lib().kete_batch_graph_create(C.byref(self.eph.c), C.byref(self.c), self.pairs_cap,
                                            C.byref(self.opts), _ptr(self.x_out), _ptr(self.status),
                                            _ptr(self.workspace), self.workspace.numel(), _stream(), C.byref(g)))
        self.graph = g

    def replay(self):
        check(lib().kete_batch_graph_launch(self.graph, _stream()))

    def pairs(self):
        n = C.c_int64(0)
        check(lib().kete_batch_pairs(C.byref(self.c), self.pairs_cap, C.byref(self.opts), _ptr(self.pf),
                                     _ptr(self.ps), _ptr(self.po), C.byref(n), _ptr(self.workspace),
                                     self.workspace.numel(), _stream()))
        return self.pf[:n.value], self.ps[:n.value], self.po[:n.value]

    def job_states(self, k: int) -> torch.Tensor:
        """States of job k [n_epoch, n_obj, 6] at self.job_epochs[k]."""
        r = self.jobs_host[k]
        return self.x_out[r.xout_off:r.xout_off + 6 * r.n_obj * r.n_epoch].view(r.n_epoch, r.n_obj, 6)

    def __del__(self):
        try:
            self.drop_graph()
        except Exception:
            pass
