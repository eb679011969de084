"""Writes tests/golden/oracle_workload1.json: the FP64 oracle's -2 ln L_spec (Sec. 2.1,
eq. spectral_likelihood, constant dropped) and its gradient (Sec. 3.3.1) for the first four
parameter points of workload 1.  Calls only the seeded generator and oracle/ (regression
fixture for the oracle; the paper prints no worked numeric example of the likelihood)."""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import skygen  # noqa: E402
from oracle import oracle  # noqa: E402


def main():
    sky = skygen.make_config(1)
    pr = oracle.Problem.from_sky(sky, 0)
    out = {"source": "oracle/cs_oracle.c via tests/golden/make_golden.py", "points": []}
    for b in range(4):
        f, g, cf, st = pr.likelihood_grad(sky.x[b])
        out["points"].append({"x": sky.x[b].tolist(), "neg2logL": f, "grad": g.tolist(), "status": st})
    with open(os.path.join(HERE, "oracle_workload1.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
