"""Writes the stored expected values under tests/golden/ from the CPU
oracle alone (inputs from the seeded generators).  Run from the
repository root:  python tests/golden/make_golden.py

tiny_case.json: the tiny workload (1,000 main-belt bodies, Sun + Jupiter
+ Saturn, 30 days, 100 frames plus 300 targeted frames): states of 16
sampled bodies at every batch epoch, every (frame, sub-frame, body) pair
with its signed edge distance, the light-time direction of 8 bodies for
4 frames, and two universal-variable hops."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2509_04666_amd import synth  # noqa: E402

SAMPLE = [0, 7, 42, 99, 123, 256, 300, 333, 404, 512, 600, 701, 777, 850, 901, 999]


def tiny_golden():
    case = synth.tiny_case(n_obj=1000, n_frames=100, n_targeted=300)
    fr = case.frames
    order, off, t_ref = O.make_batches(fr.t)
    xe, st, _ = O.propagate(case.ephem, case.x0, 0.0, t_ref)
    pf, ps, po, edge = O.fov(case.ephem, xe, st, order, off, t_ref, fr.t, fr.obs, fr.normals)
    dirs = []
    for f in range(4):
        d, tau = O.directions(case.ephem, xe[0, SAMPLE[:8]], t_ref[0], fr.t[order[f]], fr.obs[order[f]])
        dirs.append({"frame": int(order[f]), "d": d.tolist(), "tau": tau.tolist()})
    hops = []
    for dt in (3.5, -40.0):
        s, r, v = O.kepler(synth.GM_SUN, case.x0[5, :3] - case.model.sun(0.0)[:3],
                           case.x0[5, 3:] - case.model.sun(0.0)[3:], dt)
        hops.append({"body": 5, "dt": dt, "status": int(s), "r": r.tolist(), "v": v.tolist()})
    return {
        "source": "written by tests/golden/make_golden.py from the CPU oracle (oracle/kete_oracle.c)",
        "workload": "synth.tiny_case(n_obj=1000, n_frames=100, n_targeted=300)",
        "t_ref": t_ref.tolist(),
        "sample": SAMPLE,
        "states": xe[:, SAMPLE].tolist(),
        "status": st[SAMPLE].tolist(),
        "pairs": {"frame": pf.tolist(), "sub": ps.tolist(), "body": po.tolist(),
                  "edge": [float(f"{e:.6e}") for e in edge]},
        "directions": dirs,
        "hops": hops,
    }


if __name__ == "__main__":
    O.build(force=False)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_case.json")
    with open(out, "w") as fh:
        json.dump(tiny_golden(), fh, indent=0)
    print("wrote", out, os.path.getsize(out), "bytes")
