"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every function declared in include/kete_mi.h, host batching
matches the oracle's batching rule, and invalid arguments are rejected
before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2509_04666_amd import _lib, api
from paper_2509_04666_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            src = open(os.path.join(inc, fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(kete_\w+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    declared = _declared_functions()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(L, name), name
    assert set(_lib.exported_symbols()) == declared


def test_make_batches_matches_oracle(orc):
    rng = np.random.default_rng(1)
    for t in (rng.uniform(0, 40, 500), np.round(rng.uniform(0, 10, 300), 1), np.array([5.0]), np.zeros(7)):
        o1, off1, tr1 = api.make_batches(t, 3.0)
        o2, off2, tr2 = orc.make_batches(t, 3.0)
        np.testing.assert_array_equal(o1, o2)
        np.testing.assert_array_equal(off1, off2)
        np.testing.assert_array_equal(tr1, tr2)


def test_make_batches_empty_and_errors():
    o, off, tr = api.make_batches(np.zeros(0), 3.0)
    assert off.tolist() == [0] and tr.size == 0
    with pytest.raises(_lib.KeteError) as e:
        api.make_batches(np.array([1.0, np.nan]), 3.0)
    assert e.value.code == _lib.KETE_EINVAL


def _host_ephem():
    e = synth.tiny_case(n_obj=1, n_frames=1).ephem
    gm = np.ascontiguousarray(e.gm)
    fl = np.ascontiguousarray(e.flags)
    # coefficient pointer is never dereferenced on these error paths
    et = _lib.EphemT(e.n_body, e.n_seg, e.degree, 0, e.t_start, e.seg_days, 0x1000,
                     gm.ctypes.data_as(C.POINTER(C.c_double)), fl.ctypes.data_as(C.POINTER(C.c_uint32)))
    return e, et, (gm, fl)


def test_propagate_argument_errors():
    L = _lib.lib()
    e, et, keep = _host_ephem()
    o = api.default_opts()
    fake = C.c_void_p(0x1000)
    t_out = np.array([5.0, 10.0])
    tp = t_out.ctypes.data_as(C.c_void_p)
    # ERANGE: epoch beyond the ephemeris
    bad = np.array([5.0, e.t_end + 1.0])
    rc = L.kete_propagate_nbody(C.byref(et), fake, 0.0, 10, bad.ctypes.data_as(C.c_void_p), 2, fake, fake, None,
                                C.byref(o), fake, 1 << 30, None)
    assert rc == _lib.KETE_ERANGE
    assert b"outside ephemeris" in L.kete_last_error()
    # ERANGE: t0 before the ephemeris
    rc = L.kete_propagate_nbody(C.byref(et), fake, e.t_start - 1.0, 10, tp, 2, fake, fake, None, C.byref(o),
                                fake, 1 << 30, None)
    assert rc == _lib.KETE_ERANGE
    # EINVAL: non-monotone epochs, null pointers, bad block size, too many bodies
    nm = np.array([10.0, 5.0])
    assert L.kete_propagate_nbody(C.byref(et), fake, 0.0, 10, nm.ctypes.data_as(C.c_void_p), 2, fake, fake, None,
                                  C.byref(o), fake, 1 << 30, None) == _lib.KETE_EINVAL
    assert L.kete_propagate_nbody(C.byref(et), None, 0.0, 10, tp, 2, fake, fake, None, C.byref(o), fake, 1 << 30,
                                  None) == _lib.KETE_EINVAL
    o2 = api.default_opts(block=96)
    assert L.kete_propagate_nbody(C.byref(et), fake, 0.0, 10, tp, 2, fake, fake, None, C.byref(o2), fake, 1 << 30,
                                  None) == _lib.KETE_EINVAL
    et2 = _lib.EphemT(17, et.n_seg, et.degree, 0, et.t_start, et.seg_days, 0x1000, et.gm, et.flags)
    assert L.kete_propagate_nbody(C.byref(et2), fake, 0.0, 10, tp, 2, fake, fake, None, C.byref(o), fake, 1 << 30,
                                  None) == _lib.KETE_EINVAL
    # EINVAL: bad J2 rows (non-unit pole, zero radius, more than KETE_MAX_J2 bodies)
    nb = e.n_body
    for row in ([1e-3, 0.01, 0.0, 0.0, 2.0], [1e-3, 0.0, 0.0, 0.0, 1.0], [np.nan, 0.01, 0.0, 0.0, 1.0]):
        j2 = np.zeros((nb, 5))
        j2[0] = row
        et3 = _lib.EphemT(nb, et.n_seg, et.degree, 0, et.t_start, et.seg_days, 0x1000, et.gm, et.flags,
                          j2.ctypes.data_as(C.POINTER(C.c_double)))
        assert L.kete_propagate_nbody(C.byref(et3), fake, 0.0, 10, tp, 2, fake, fake, None, C.byref(o), fake,
                                      1 << 30, None) == _lib.KETE_EINVAL
        assert b"j2[0]" in L.kete_last_error()
    gm5, fl5, j25 = np.full(5, 1e-10), np.zeros(5, np.uint32), np.tile([1e-3, 0.01, 0.0, 0.0, 1.0], (5, 1))
    many = _lib.EphemT(5, et.n_seg, et.degree, 0, et.t_start, et.seg_days, 0x1000,
                       gm5.ctypes.data_as(C.POINTER(C.c_double)), fl5.ctypes.data_as(C.POINTER(C.c_uint32)),
                       j25.ctypes.data_as(C.POINTER(C.c_double)))
    assert L.kete_propagate_nbody(C.byref(many), fake, 0.0, 10, tp, 2, fake, fake, None, C.byref(o), fake, 1 << 30,
                                  None) == _lib.KETE_EINVAL
    # EWORKSPACE
    need = L.kete_propagate_workspace_size(10, 2, C.byref(o))
    assert need > 0
    assert L.kete_propagate_nbody(C.byref(et), fake, 0.0, 10, tp, 2, fake, fake, None, C.byref(o), fake, need - 1,
                                  None) == _lib.KETE_EWORKSPACE
    # empty input is a no-op
    assert L.kete_propagate_nbody(C.byref(et), None, 0.0, 0, tp, 2, None, None, None, C.byref(o), None, 0,
                                  None) == _lib.KETE_OK


def test_fov_argument_errors():
    L = _lib.lib()
    e, et, keep = _host_ephem()
    o = api.default_opts()
    fake = C.c_void_p(0x1000)
    n = C.c_int64(0)
    fr = _lib.FramesT(10, 0, 0, 0x1000, 0x1000, 0x1000)
    assert L.kete_fov_check(C.byref(et), fake, None, 10, 2, fake, fake, fake, C.byref(fr), C.byref(o), fake, fake,
                            fake, 10, C.byref(n), fake, 1 << 30, None) == _lib.KETE_EINVAL
    fr = _lib.FramesT(10, 1, 0, 0x1000, 0x1000, 0x1000)
    assert L.kete_fov_check(C.byref(et), fake, None, 10, 2, fake, fake, fake, C.byref(fr), C.byref(o), fake, fake,
                            fake, 10, None, fake, 1 << 30, None) == _lib.KETE_EINVAL
    need = L.kete_fov_workspace_size(10, 10, 2, 1, 10, C.byref(o))
    assert need > 0
    assert L.kete_fov_check(C.byref(et), fake, None, 10, 2, fake, fake, fake, C.byref(fr), C.byref(o), fake, fake,
                            fake, 10, C.byref(n), fake, need - 1, None) == _lib.KETE_EWORKSPACE
    # a negative Kepler iteration cap is refused before any device work
    ob = api.default_opts(kepler_iter=-1)
    assert L.kete_fov_check(C.byref(et), fake, None, 10, 2, fake, fake, fake, C.byref(fr), C.byref(ob), fake, fake,
                            fake, 10, C.byref(n), fake, 1 << 30, None) == _lib.KETE_EINVAL
    assert b"kepler_iter" in L.kete_last_error()
    assert api.default_opts().kepler_iter == 60
    # no objects / frames: nothing to do
    assert L.kete_fov_check(C.byref(et), None, None, 0, 2, None, None, None, C.byref(fr), C.byref(o), None, None,
                            None, 0, C.byref(n), None, 0, None) == _lib.KETE_OK
    assert n.value == 0


def test_magnitudes_argument_errors():
    L = _lib.lib()
    e, et, keep = _host_ephem()
    o = api.default_opts()
    fake = C.c_void_p(0x1000)
    fr = _lib.FramesT(10, 1, 0, 0x1000, 0x1000, 0x1000)
    assert L.kete_magnitudes_workspace_size(-1) == 0
    need = L.kete_magnitudes_workspace_size(10)
    assert need >= 40 and need % 256 == 0
    args = lambda n_pairs, frames, pf, ws, ws_bytes: (C.byref(et), fake, 10, 2, fake, fake, fake, frames, pf, fake,
                                                      n_pairs, fake, fake, fake, None, C.byref(o), ws, ws_bytes,
                                                      None)
    assert L.kete_pair_magnitudes(*args(5, None, fake, fake, need)) == _lib.KETE_EINVAL      # no frames
    assert L.kete_pair_magnitudes(*args(-1, C.byref(fr), fake, fake, need)) == _lib.KETE_EINVAL
    assert L.kete_pair_magnitudes(*args(5, C.byref(fr), None, fake, need)) == _lib.KETE_EINVAL
    assert L.kete_pair_magnitudes(*args(5, C.byref(fr), fake, None, need)) == _lib.KETE_EWORKSPACE
    assert L.kete_pair_magnitudes(*args(5, C.byref(fr), fake, fake, need - 1)) == _lib.KETE_EWORKSPACE
    # no pairs: nothing to do
    assert L.kete_pair_magnitudes(*args(0, C.byref(fr), None, None, 0)) == _lib.KETE_OK


def test_ephem_eval_range_check():
    L = _lib.lib()
    e, et, keep = _host_ephem()
    t = np.array([e.t_end + 0.5])
    rc = L.kete_ephem_eval(C.byref(et), C.c_void_p(0x1000), t.ctypes.data_as(C.c_void_p), 1, C.c_void_p(0x1000), None)
    assert rc == _lib.KETE_ERANGE


def _host_batch(jobs_rows, n_bodies, n_epochs, bjob, bep, boff, n_frames, n_sub=1):
    jobs = (_lib.JobT * len(jobs_rows))(*[_lib.JobT(*r) for r in jobs_rows])
    bjob = np.ascontiguousarray(bjob, dtype=np.int32)
    bep = np.ascontiguousarray(bep, dtype=np.int32)
    boff = np.ascontiguousarray(boff, dtype=np.int32)
    fr = _lib.FramesT(n_frames, n_sub, 0, 0x1000, 0x1000, 0x1000)
    bt = _lib.BatchT(len(jobs_rows), 0, n_bodies, n_epochs, bjob.size, C.addressof(jobs), 0x1000, 0x1000, 0x1000,
                     None, bjob.ctypes.data, bep.ctypes.data, boff.ctypes.data, 0x1000, 0x1000, 0x1000, fr)
    return bt, (jobs, bjob, bep, boff)


def test_batch_description_checks():
    L = _lib.lib()
    e, et, keep = _host_ephem()
    o = api.default_opts()
    # two jobs: 100 bodies over 3 epochs, 5 bodies over 1 epoch; 4 batches over 12 frames
    rows = [(0, 0, 0, 100, 3, 0.0), (100, 3, 1800, 5, 1, 2.0)]
    bt, k1 = _host_batch(rows, 105, 4, [0, 0, 0, 1], [0, 1, 2, 0], [0, 3, 6, 9, 12], 12)
    good = L.kete_batch_workspace_size(C.byref(et), C.byref(bt), 64, C.byref(o))
    assert good > 0
    # larger pair capacity -> larger workspace
    assert L.kete_batch_workspace_size(C.byref(et), C.byref(bt), 1 << 20, C.byref(o)) > good
    bad_cases = [
        ([(0, 0, 0, 100, 3, 0.0), (100, 3, 1800, 6, 1, 2.0)], 105, 4, [0, 0, 0, 1], [0, 1, 2, 0]),   # rows past n_bodies
        ([(0, 0, 0, 100, 3, 0.0), (100, 3, 1800, 5, 2, 2.0)], 105, 4, [0, 0, 0, 1], [0, 1, 2, 0]),   # epochs past n_epochs
        (rows, 105, 4, [0, 0, 0, 2], [0, 1, 2, 0]),                                                # batch of no job
        (rows, 105, 4, [0, 0, 0, 1], [0, 1, 3, 0]),                                                # epoch out of range
        ([(0, 0, 0, 100, 3, e.t_start - 1.0), (100, 3, 1800, 5, 1, 2.0)], 105, 4, [0, 0, 0, 1], [0, 1, 2, 0]),
    ]
    for r, nb, ne, bj, be in bad_cases:
        b2, k2 = _host_batch(r, nb, ne, bj, be, [0, 3, 6, 9, 12], 12)
        assert L.kete_batch_workspace_size(C.byref(et), C.byref(b2), 64, C.byref(o)) == 0
        assert L.kete_last_error() != b""
    # plan/run reject a short workspace before touching the device
    assert L.kete_batch_plan(C.byref(et), C.byref(bt), 64, C.byref(o), C.c_void_p(0x1000), good - 1,
                             None) == _lib.KETE_EWORKSPACE
    assert L.kete_batch_run(C.byref(et), C.byref(bt), 64, C.byref(o), C.c_void_p(0x1000), C.c_void_p(0x1000),
                            C.c_void_p(0x1000), good - 1, None) == _lib.KETE_EWORKSPACE
    best = _lib.OptsT()
    assert L.kete_batch_autotune(C.byref(et), C.byref(bt), 64, C.byref(o), 0, None, None, None, 0, None,
                                 _lib.TUNE_PROGRESS(), None, C.byref(best), None) == _lib.KETE_EINVAL
    assert L.kete_batch_graph_launch(None, None) == _lib.KETE_EINVAL
    assert L.kete_batch_graph_destroy(None) == _lib.KETE_OK


def test_noalloc_magnitudes_rejects_too_many_frames():
    """The magnitude entry point without a workspace holds its
    frame-to-batch map in a static device array: more frames than it holds
    is a clear error raised before any device work (the fake pointers are
    never dereferenced on this path)."""
    L = _lib.lib()
    e, et, keep = _host_ephem()
    fake = C.c_void_p(0x1000)
    fr = _lib.FramesT(_lib.MAG_NOALLOC_MAX_FRAMES + 1, 1, 0, 0x1000, 0x1000, 0x1000)
    rc = L.kete_pair_magnitudes_noalloc(C.byref(et), fake, 10, 2, fake, fake, fake, C.byref(fr), fake, fake, 5,
                                        fake, fake, fake, None, None, None)
    assert rc == _lib.KETE_EWORKSPACE
    assert b"static scratch" in L.kete_last_error()
    # no pairs: nothing to do, no device work, no error
    rc = L.kete_pair_magnitudes_noalloc(C.byref(et), fake, 10, 2, fake, fake, fake, C.byref(fr), fake, fake, 0,
                                        fake, fake, fake, None, None, None)
    assert rc == _lib.KETE_OK


def test_adjoint_sky_refuses_a_stale_backward():
    """Two forwards on one adjoint context before backward: the first
    graph's backward would read the second call's checkpoints, so it must
    raise; the latest one still runs.  The device calls are replaced by
    host stand-ins: this checks the binding's bookkeeping only."""
    import torch

    class HostCtx(api.AdjointContext):
        def __init__(self):
            self.n_obj, self.k_obs, self.generation = 3, 2, 0

        def _run_forward(self, x0):
            return torch.zeros((self.n_obj, self.k_obs, 2), dtype=torch.float64)

        def _run_backward(self, x0, g):
            return torch.ones((self.n_obj, 6), dtype=torch.float64)

    ctx = HostCtx()
    x = torch.zeros((3, 6), dtype=torch.float64, requires_grad=True)
    s1 = api.AdjointSky.apply(x, ctx)
    s2 = api.AdjointSky.apply(x, ctx)
    s2.sum().backward()
    assert torch.equal(x.grad, torch.ones((3, 6), dtype=torch.float64))
    with pytest.raises(RuntimeError, match="later forward"):
        s1.sum().backward()
