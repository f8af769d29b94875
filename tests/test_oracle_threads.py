"""The oracle gives the same results on one thread and on many, from a
fresh process (no state shared between objects)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, %r)
from oracle import oracle as O
from paper_2509_04666_amd import synth
g = synth.gradient_case(n_obj=64, k_obs=8, arc=20.0, neo_frac=0.2)
radec, loss, grad, st = O.sky_grad(g.ephem, g.x0, 0.0, g.t_obs, g.obs_pos, g.radec_obs,
                                   opts=O.make_opts(n_threads=int(sys.argv[1])))
np.save(sys.argv[2], np.concatenate([radec.ravel(), loss, grad.ravel()]))
"""


def test_oracle_thread_count_does_not_change_results(tmp_path):
    outs = []
    for nt in (1, 8):
        f = str(tmp_path / f"o{nt}.npy")
        subprocess.check_call([sys.executable, "-c", SCRIPT % ROOT, str(nt), f])
        outs.append(np.load(f))
    assert np.array_equal(outs[0], outs[1])
