"""Stored expected values (tests/golden/tiny_case.json, written by
tests/golden/make_golden.py from the oracle): the oracle must keep
reproducing them, and the GPU path must match them at the parity
tolerances."""
import json
import math
import os

import numpy as np
import pytest

from paper_2509_04666_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tiny_case.json")
MAS = math.radians(1.0 / 3.6e6)


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def case():
    return synth.tiny_case(n_obj=1000, n_frames=100, n_targeted=300)


def test_oracle_reproduces_stored_values(orc, golden, case):
    fr = case.frames
    order, off, t_ref = orc.make_batches(fr.t)
    np.testing.assert_array_equal(t_ref, golden["t_ref"])
    xe, st, _ = orc.propagate(case.ephem, case.x0, 0.0, t_ref)
    s = golden["sample"]
    assert np.abs(xe[:, s] - np.array(golden["states"])).max() < 1e-13
    pf, ps, po, edge = orc.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals)
    gp = golden["pairs"]
    assert pf.tolist() == gp["frame"] and ps.tolist() == gp["sub"] and po.tolist() == gp["body"]
    assert np.allclose(edge, gp["edge"], rtol=1e-5, atol=1e-15)
    for d in golden["directions"]:
        f = d["frame"]
        dd, tau = orc.directions(case.ephem, xe[0, s[:8]], t_ref[0], fr.t[f], fr.obs[f])
        assert np.abs(dd - np.array(d["d"])).max() < 1e-14
        assert np.abs(tau - np.array(d["tau"])).max() < 1e-16
    for hop in golden["hops"]:
        st_h, r, v = orc.kepler(synth.GM_SUN, case.x0[hop["body"], :3] - case.model.sun(0.0)[:3],
                                case.x0[hop["body"], 3:] - case.model.sun(0.0)[3:], hop["dt"])
        assert st_h == hop["status"]
        assert np.abs(r - np.array(hop["r"])).max() < 1e-14 and np.abs(v - np.array(hop["v"])).max() < 1e-15


@pytest.mark.gpu
def test_gpu_matches_stored_values(orc, golden, case):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_04666_amd import api
    fr = case.frames
    eph = api.DeviceEphemeris.from_synth(case.ephem)
    pf, ps, po, xg, sg, bt = api.predict(eph, torch.as_tensor(case.x0).cuda(), 0.0, api.DeviceFrames.from_synth(fr),
                                         fr.t)
    np.testing.assert_array_equal(bt.t_ref_host, golden["t_ref"])
    s = golden["sample"]
    err = np.abs(xg.cpu().numpy()[:, s] - np.array(golden["states"])).max()
    assert err < 1e-10
    g = set(zip(pf.cpu().tolist(), ps.cpu().tolist(), po.cpu().tolist()))
    gp = golden["pairs"]
    o = set(zip(gp["frame"], gp["sub"], gp["body"]))
    near = {k for k, e in zip(zip(gp["frame"], gp["sub"], gp["body"]), gp["edge"]) if abs(e) < MAS}
    assert not (o - g - near)
    # an extra pair must lie within 1 mas of an edge (oracle light-time direction)
    order, off, t_ref = orc.make_batches(fr.t)
    xe, st, _ = orc.propagate(case.ephem, case.x0, 0.0, t_ref)
    for f, sub, j in g - o:
        q = int(np.nonzero(order == f)[0][0])
        b = int(np.searchsorted(off, q, side="right") - 1)
        _, d, _, _ = orc.lighttime(case.ephem, t_ref[b], xe[b, j], fr.t[f], fr.obs[f])
        _, edge = orc.inside(fr.normals[f], d)
        assert abs(edge[sub]) < MAS
    print(f"stored tiny case: max |dx| {err:.3e} au, {len(o)} stored pairs, gpu {len(g)}", flush=True)
