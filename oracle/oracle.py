"""ctypes wrapper around the plain C oracle (kete_oracle.c).

TEST INFRASTRUCTURE: only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The GPU product
path never imports it and shares no code with it.

The frame batching rule of Sect. 2 (batches of frames spanning at most
3 days, each integrated to its mid time) is restated here in plain Python
for the oracle's own use.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kete_oracle.c")
LIB = os.path.join(HERE, "libkete_oracle.so")

ST_OK, ST_NONFINITE, ST_STEP_UNDERFLOW, ST_MAX_STEPS, ST_KEPLER_NOCONV, ST_ERANGE = range(6)
C_AU_PER_DAY = 173.14463267424034


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no contraction, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Ephem(C.Structure):
    _fields_ = [("n_body", C.c_int32), ("n_seg", C.c_int32), ("degree", C.c_int32), ("pad", C.c_int32),
                ("t_start", C.c_double), ("seg_days", C.c_double),
                ("coef", C.POINTER(C.c_double)), ("gm", C.POINTER(C.c_double)),
                ("flags", C.POINTER(C.c_uint32)), ("j2", C.POINTER(C.c_double))]


class Opts(C.Structure):
    _fields_ = [("eps", C.c_double), ("h_init", C.c_double), ("h_min", C.c_double),
                ("safety", C.c_double), ("c_light", C.c_double), ("max_iter", C.c_int32),
                ("n_threads", C.c_int32), ("max_steps", C.c_int64), ("h_max", C.c_double),
                ("extrapolate", C.c_int32), ("pad", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        _lib = C.CDLL(LIB)
    return _lib


def _p(a, ct=C.c_double):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleEphem:
    """Holds numpy buffers alive for the C struct."""

    def __init__(self, eph):
        self.coef = _f64(eph.coef)
        self.gm = _f64(eph.gm)
        self.flags = np.ascontiguousarray(eph.flags, dtype=np.uint32)
        nb, ns, _, m = self.coef.shape
        j2 = getattr(eph, "j2", None)
        self.j2 = None if j2 is None else _f64(j2).reshape(nb, 5)
        self.s = Ephem(nb, ns, m - 1, 0, float(eph.t_start), float(eph.seg_days),
                       _p(self.coef), _p(self.gm), _p(self.flags, C.c_uint32),
                       None if self.j2 is None else _p(self.j2))

    @property
    def ref(self):
        return C.byref(self.s)


def _eph(e):
    return e if isinstance(e, OracleEphem) else OracleEphem(e)


def make_opts(eps=1e-9, h_init=1.0, h_min=1e-9, safety=0.25, c_light=0.0, max_iter=12,
              n_threads=0, max_steps=10_000_000, h_max=0.0, extrapolate=0):
    return Opts(eps, h_init, h_min, safety, c_light, max_iter, n_threads, max_steps, h_max, extrapolate, 0)


DEFAULT_OPTS = dict(eps=1e-9, h_init=1.0)


def predict_b(b, q):
    """RADAU's predictor for one coordinate: the coefficients b' of the
    previous step's acceleration polynomial about its end, for a step q
    times as long."""
    bn = np.zeros(7)
    lib().orc_predict_b(_p(_f64(b)), C.c_double(q), _p(bn))
    return bn


def radau_nodes():
    out = np.zeros(8)
    lib().orc_radau_nodes(_p(out))
    return out


def cheb(eph, body, t):
    e = _eph(eph)
    pos = np.zeros(3); vel = np.zeros(3)
    st = lib().orc_cheb(e.ref, C.c_int(body), C.c_double(t), _p(pos), _p(vel))
    return st, pos, vel


def accel(eph, t, x, v, c_light=C_AU_PER_DAY, jac=False):
    e = _eph(eph)
    x = _f64(x); v = _f64(v)
    a = np.zeros(3); jx = np.zeros(9); jv = np.zeros(9)
    st = lib().orc_accel_jac(e.ref, C.c_double(c_light), C.c_double(t), _p(x), _p(v), _p(a),
                             _p(jx) if jac else None, _p(jv) if jac else None)
    if st:
        raise ValueError(f"oracle accel status {st}")
    return (a, jx.reshape(3, 3), jv.reshape(3, 3)) if jac else a


def kepler(mu, r0, v0, dt):
    r = np.zeros(3); v = np.zeros(3)
    st = lib().orc_kepler(C.c_double(mu), _p(_f64(r0)), _p(_f64(v0)), C.c_double(dt), _p(r), _p(v))
    return st, r, v


def lighttime(eph, t_ref, state, t_obs, obs, c_light=C_AU_PER_DAY):
    e = _eph(eph)
    d = np.zeros(3); tau = C.c_double(0); xe = np.zeros(6)
    st = lib().orc_lighttime(e.ref, C.c_double(c_light), C.c_double(t_ref), _p(_f64(state)),
                             C.c_double(t_obs), _p(_f64(obs)), _p(d), C.byref(tau), _p(xe))
    return st, d, tau.value, xe


def directions(eph, states, t_ref, t_obs, obs, c_light=C_AU_PER_DAY):
    e = _eph(eph)
    states = _f64(states)
    n = states.shape[0]
    d = np.zeros((n, 3)); tau = np.zeros(n)
    st = lib().orc_directions(e.ref, C.c_double(c_light), C.c_int64(n), _p(states), C.c_double(t_ref),
                              C.c_double(t_obs), _p(_f64(obs)), _p(d), _p(tau))
    if st:
        raise ValueError(f"oracle directions status {st}")
    return d, tau


def propagate(eph, x0, t0, t_out, opts=None, **kw):
    """States at each t_out: returns (x_out [E, N, 6], status [N], stats[5]:
    steps, corrector sweeps, rejections, force evaluations, steps started
    from the extrapolated polynomial)."""
    e = _eph(eph)
    o = opts if opts is not None else make_opts(**{**DEFAULT_OPTS, **kw})
    x0 = _f64(x0); t_out = _f64(np.atleast_1d(t_out))
    n = x0.shape[0]; E = t_out.shape[0]
    x_out = np.zeros((E, n, 6)); status = np.zeros(n, np.int32); stats = np.zeros(5, np.int64)
    rc = lib().orc_propagate(e.ref, C.byref(o), C.c_int64(n), _p(x0), C.c_double(t0), C.c_int64(E),
                             _p(t_out), _p(x_out), _p(status, C.c_int32), _p(stats, C.c_int64))
    if rc:
        raise ValueError(f"oracle propagate rc {rc}")
    return x_out, status, stats


def step_trace(eph, x0, t0, t1, opts=None, **kw):
    """Accepted step sizes (days, signed) of one object integrated alone
    from t0 to t1."""
    e = _eph(eph)
    o = opts if opts is not None else make_opts(**{**DEFAULT_OPTS, **kw})
    rec = np.zeros(1 << 16); n = C.c_int64(0)
    st = lib().orc_step_trace(e.ref, C.byref(o), _p(_f64(x0)), C.c_double(t0), C.c_double(t1), _p(rec),
                              C.c_int64(rec.size), C.byref(n))
    if st:
        raise ValueError(f"oracle step trace status {st}")
    return rec[:min(n.value, rec.size)].copy()


def make_batches(t, span=3.0):
    """Greedy batching of frames (Sect. 2): sort by (time, index); a batch
    starts at its first frame and takes every following frame within
    `span` days of it; the batch epoch is the midpoint of its first and
    last frame times.  Returns (frame_order, batch_off, t_ref)."""
    t = np.asarray(t, float)
    order = np.lexsort((np.arange(t.size), t))
    off = [0]
    ts = t[order]
    i = 0
    while i < ts.size:
        j = i
        while j + 1 < ts.size and ts[j + 1] - ts[i] <= span:
            j += 1
        off.append(j + 1)
        i = j + 1
    off = np.array(off, np.int64)
    t_ref = np.array([0.5 * (ts[off[b]] + ts[off[b + 1] - 1]) for b in range(off.size - 1)])
    return order.astype(np.int64), off, t_ref


def fov(eph, x_epoch, status, frame_order, batch_off, t_ref, frames_t, frames_obs, normals,
        cap=None, c_light=C_AU_PER_DAY, n_threads=0, return_status=False):
    """Brute-force pairs sorted by (frame, sub, object), with edge distances
    (and, with return_status, the per-object status of the light-time hops:
    an object with a failed hop has no pairs)."""
    e = _eph(eph)
    x_epoch = _f64(x_epoch)
    n_batch, n_obj = x_epoch.shape[:2]
    normals = _f64(normals)
    n_sub = normals.shape[1]
    status = np.zeros(n_obj, np.int32) if status is None else np.ascontiguousarray(status, np.int32)
    fo = np.ascontiguousarray(frame_order, np.int64); bo = np.ascontiguousarray(batch_off, np.int64)
    tr = _f64(t_ref); ft = _f64(frames_t); fobs = _f64(frames_obs)
    n_pairs = C.c_int64(0)
    st_out = np.zeros(n_obj, np.int32)
    for attempt in range(2):
        cap_ = cap if cap is not None else 1 << 16
        if attempt == 1:
            cap_ = max(int(n_pairs.value), 1)
        pf = np.zeros(cap_, np.int32); ps = np.zeros(cap_, np.int32); po = np.zeros(cap_, np.int32)
        edge = np.zeros(cap_)
        rc = lib().orc_fov(e.ref, C.c_double(c_light), C.c_int64(n_obj), _p(x_epoch), _p(status, C.c_int32),
                           C.c_int64(n_batch), _p(tr), _p(bo, C.c_int64), _p(fo, C.c_int64), _p(ft), _p(fobs),
                           C.c_int32(n_sub), _p(normals), C.c_int64(cap_), _p(pf, C.c_int32), _p(ps, C.c_int32),
                           _p(po, C.c_int32), _p(edge), C.byref(n_pairs), C.c_int32(n_threads),
                           _p(st_out, C.c_int32))
        if rc == 0:
            break
        if cap is not None:
            raise ValueError("oracle fov capacity")
    n = int(n_pairs.value)
    pf, ps, po, edge = pf[:n], ps[:n], po[:n], edge[:n]
    order = np.lexsort((po, ps, pf))
    if return_status:
        return pf[order], ps[order], po[order], edge[order], st_out
    return pf[order], ps[order], po[order], edge[order]


def set_kepler_max_iter(n: int) -> None:
    """Newton iterations one Kepler solve may take (0 restores the default,
    200); fewer force the not-converged report in tests."""
    lib().orc_set_kepler_max_iter(C.c_int(n))


def sky_grad(eph, x0, t0, t_obs, obs_pos, radec_obs, want_grad=True, opts=None, **kw):
    e = _eph(eph)
    o = opts if opts is not None else make_opts(**{**DEFAULT_OPTS, **kw})
    x0 = _f64(x0); t_obs = _f64(t_obs); obs_pos = _f64(obs_pos); radec_obs = _f64(radec_obs)
    n, k = t_obs.shape
    radec = np.zeros((n, k, 2)); loss = np.zeros(n); grad = np.zeros((n, 6)); status = np.zeros(n, np.int32)
    lib().orc_sky_grad(e.ref, C.byref(o), C.c_int64(n), _p(x0), C.c_double(t0), C.c_int32(k), _p(t_obs),
                       _p(obs_pos), _p(radec_obs), _p(radec), _p(loss), _p(grad) if want_grad else None,
                       C.c_int32(1 if want_grad else 0), _p(status, C.c_int32))
    return radec, loss, grad, status


def loss_steps(eph, x0, t0, t_obs, obs_pos, radec_obs, replay=None, opts=None, **kw):
    """Loss of one object; returns (loss, steps) where steps is the recorded
    sequence (replay=None) or the replayed one."""
    e = _eph(eph)
    o = opts if opts is not None else make_opts(**{**DEFAULT_OPTS, **kw})
    loss = C.c_double(0)
    rec = np.zeros(1 << 16); rec_n = C.c_int64(0)
    rp = None if replay is None else _f64(replay)
    st = lib().orc_loss_steps(e.ref, C.byref(o), _p(_f64(x0)), C.c_double(t0), C.c_int32(len(t_obs)),
                              _p(_f64(t_obs)), _p(_f64(obs_pos)), _p(_f64(radec_obs)), C.byref(loss),
                              _p(rec), C.c_int64(rec.size), C.byref(rec_n),
                              _p(rp) if rp is not None else None, C.c_int64(0 if rp is None else rp.size))
    if st:
        raise ValueError(f"oracle loss status {st}")
    return loss.value, (rec[:rec_n.value].copy() if replay is None else rp)


def radec(d):
    """(ra, dec) in the equatorial J2000 frame of an ecliptic direction d,
    and the Jacobian d(ra, dec)/dd [2, 3]."""
    out = np.zeros(2); jac = np.zeros(6)
    lib().orc_radec_of(_p(_f64(d)), _p(out), _p(jac))
    return out[0], out[1], jac.reshape(2, 3)


def sky_residual(ra, dec, ra_obs, dec_obs):
    """((ra - ra_obs) cos dec, dec - dec_obs), the RA difference wrapped to (-pi, pi]."""
    r = np.zeros(2)
    lib().orc_sky_residual(C.c_double(ra), C.c_double(dec), C.c_double(ra_obs), C.c_double(dec_obs), _p(r))
    return r


def inside(normals, d):
    """Membership of direction d in each sub-frame of one frame: (inside[S], edge[S])."""
    n = _f64(normals)
    S = n.shape[0]
    ins = np.zeros(S, np.int32); edge = np.zeros(S)
    lib().orc_inside(C.c_int32(S), _p(n), _p(_f64(d)), _p(ins, C.c_int32), _p(edge))
    return ins.astype(bool), edge


def hg_mag(H, G, r_h, delta, alpha):
    """H-G apparent magnitude (Sect. 3.3) of one body from r_H, Delta (au), alpha (rad)."""
    f = lib().orc_hg_mag
    f.restype = C.c_double
    return f(C.c_double(H), C.c_double(G), C.c_double(r_h), C.c_double(delta), C.c_double(alpha))


def pair_mags(eph, x_epoch, frame_order, batch_off, t_ref, frames_t, frames_obs, pf, po, H, G,
              c_light=C_AU_PER_DAY):
    """V magnitude and {r_H, Delta, alpha} of every (frame, object) pair."""
    e = _eph(eph)
    x_epoch = _f64(x_epoch)
    n_batch, n_obj = x_epoch.shape[:2]
    pf = np.ascontiguousarray(pf, np.int32); po = np.ascontiguousarray(po, np.int32)
    n = pf.size
    v = np.zeros(n); geom = np.zeros((n, 3))
    ft = _f64(frames_t)
    rc = lib().orc_pair_mags(e.ref, C.c_double(c_light), C.c_int64(n_obj), _p(x_epoch), C.c_int64(n_batch),
                             _p(_f64(t_ref)), _p(np.ascontiguousarray(batch_off, np.int64), C.c_int64),
                             _p(np.ascontiguousarray(frame_order, np.int64), C.c_int64), C.c_int64(ft.size),
                             _p(ft), _p(_f64(frames_obs)), C.c_int64(n), _p(pf, C.c_int32), _p(po, C.c_int32),
                             _p(_f64(H)), _p(_f64(G)), _p(v), _p(geom))
    if rc:
        raise ValueError("oracle pair_mags: bad pair or frame")
    return v, geom


def stm(eph, x0, t0, t1, opts=None, **kw):
    """(state [6], Phi [6, 6]) at t1 from the variational equations."""
    e = _eph(eph)
    o = opts if opts is not None else make_opts(**{**DEFAULT_OPTS, **kw})
    out = np.zeros(6); phi = np.zeros(36)
    st = lib().orc_stm(e.ref, C.byref(o), _p(_f64(x0)), C.c_double(t0), C.c_double(t1), _p(out), _p(phi))
    if st:
        raise ValueError(f"oracle stm status {st}")
    return out, phi.reshape(6, 6)
