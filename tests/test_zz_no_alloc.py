"""The magnitude entry point that allocates nothing
(kete_pair_magnitudes_noalloc, its frame-to-batch map in the library's
static device array) against the workspace entry point
(kete_pair_magnitudes) on the same pairs, both called through the C ABI.
They share the kernels, so the results must agree bit for bit.  Two calls
in a row, the second with fewer frames, batches and pairs, check that the
static map keeps nothing of the earlier call that the later one reads."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2509_04666_amd import _lib, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64).cuda()


def _case(n_obj, n_frames, n_targeted, seed):
    import torch
    from paper_2509_04666_amd import api
    case = synth.tiny_case(n_obj=n_obj, n_frames=n_frames, n_targeted=n_targeted, seed=seed)
    fr = case.frames
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    dfr = api.DeviceFrames.from_synth(fr)
    pf, ps, po, xg, st, b = api.predict(eph, _dev(case.x0), 0.0, dfr, fr.t)
    H, G = synth.hg_params(np.random.default_rng(seed + 7), n_obj)
    torch.cuda.synchronize()
    return eph, dfr, b, xg, pf, po, _dev(H), _dev(G)


def _both(case):
    """(v, geom) from the workspace entry point and from the static one."""
    import torch
    from paper_2509_04666_amd import api
    eph, dfr, b, xg, pf, po, H, G = case
    L = _lib.lib()
    P = pf.numel()
    B, N = xg.shape[0], xg.shape[1]
    fc = dfr.c()
    opts = api.default_opts()
    out = []
    for static in (False, True):
        v = torch.full((P,), -7.0, dtype=torch.float64, device="cuda")
        geom = torch.full((P, 3), -7.0, dtype=torch.float64, device="cuda")
        args = [C.byref(eph.c), xg.data_ptr(), N, B, b.t_ref.data_ptr(), b.batch_off.data_ptr(),
                b.frame_order.data_ptr(), C.byref(fc), pf.data_ptr(), po.data_ptr(), P, H.data_ptr(), G.data_ptr(),
                v.data_ptr(), geom.data_ptr(), C.byref(opts)]
        stream = torch.cuda.current_stream().cuda_stream
        if static:
            rc = L.kete_pair_magnitudes_noalloc(*args, stream)
        else:
            need = L.kete_magnitudes_workspace_size(dfr.t.shape[0])
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
            rc = L.kete_pair_magnitudes(*args, ws.data_ptr(), ws.numel(), stream)
        _lib.check(rc)
        torch.cuda.synchronize()
        out.append((v.cpu().numpy(), geom.cpu().numpy()))
    return out


def test_noalloc_magnitudes_match_workspace_entry_point():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sizes = [(900, 120, 400, 21), (300, 37, 90, 22)]     # the second call is smaller
    for n_obj, n_fr, n_tg, seed in sizes:
        _say(f"noalloc magnitudes: {n_obj} bodies, {n_fr + n_tg} frames, seed {seed}")
        case = _case(n_obj, n_fr, n_tg, seed)
        P = case[4].numel()
        assert P > 50
        (vw, gw), (vs, gs) = _both(case)
        _say(f"  {P} pairs, finite {np.isfinite(vs).mean():.3f}")
        np.testing.assert_array_equal(vs, vw)
        np.testing.assert_array_equal(gs, gw)
        assert np.isfinite(vs).all()
