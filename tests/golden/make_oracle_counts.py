"""Natural step and sweep counts of the integration method on the
benchmark workloads, measured with the CPU oracle (App. A.6: Gauss-Radau
steps under IAS15 control).  Each sampled body is integrated on its own
from the start epoch to the end of the span in one go (the epochs in
between are read off the step polynomials, so they do not cut steps), once
with the corrector started from the previous step's extrapolated polynomial
(the start the GPU kernels use) and once from zero (the paper's start).
The per-body-day rates scale to any number of bodies of the same mix and
fix the algorithmic flop count of the benchmark's roofline.

Writes tests/golden/oracle_counts.json.  Calls only the oracle and the
seeded input generators.

    python tests/golden/make_oracle_counts.py [--sample 10000]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2509_04666_amd import synth  # noqa: E402

WORKLOADS = {
    "survey": lambda: synth.survey_case(n_frames=0),
    "footprints": lambda: synth.footprint_case(n_frames=0),
}


def counts(case, sample, seed=17):
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(case.x0.shape[0], sample, replace=False))
    out = {"bodies_in_workload": int(case.x0.shape[0]), "sample": int(sample), "sample_seed": seed,
           "span_days": case.span, "neo_in_sample": int(case.is_neo[sel].sum())}
    for name, extrap in (("extrapolated_start", 1), ("zero_start", 0)):
        t0 = time.perf_counter()
        _, st, s = O.propagate(case.ephem, case.x0[sel], case.t0, [case.t0 + case.span],
                               opts=O.make_opts(extrapolate=extrap))
        body_days = float(sample * case.span)
        out[name] = {
            "failed": int(np.count_nonzero(st)),
            "steps_per_body_day": s[0] / body_days, "sweeps_per_body_day": s[1] / body_days,
            "rejections_per_body_day": s[2] / body_days, "extrapolated_starts_per_body_day": s[4] / body_days,
            "steps_per_body_year": s[0] / body_days * 365.25, "sweeps_per_step": s[1] / s[0],
            "oracle_seconds": time.perf_counter() - t0,
        }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sample", type=int, default=10000)
    args = ap.parse_args()
    res = {"source": "tests/golden/make_oracle_counts.py (CPU oracle, eps 1e-9, one run per body over the span)"}
    for name, mk in WORKLOADS.items():
        res[name] = counts(mk(), args.sample)
        print(name, json.dumps(res[name]["extrapolated_start"]), flush=True)
    with open(os.path.join(HERE, "oracle_counts.json"), "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
