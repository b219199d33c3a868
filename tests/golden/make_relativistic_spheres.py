"""Writes relativistic_spheres_oracle.json: the FP64 reference's stationary
state of the three relativistic radiating spheres (boost, lapse well, both;
Sec. 4.2 set-ups in relativistic_spheres.json) as the per-zone invariants
(1+v)/(1-v) L_rs and gamma (1+v) alpha <eps> and the moments they come from.
Calls only the reference (oracle/); takes several minutes."""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle                             # noqa: E402
from paper_2003_02845_amd import workloads as W      # noqa: E402

STEPS_PER_RMAX = 1.6          # run for 1.6 light-crossing times of the grid


def invariants(w, zm):
    rc = 0.5 * (w.r_edges[1:] + w.r_edges[:-1])
    H, NF = zm[:, 0, 2], zm[:, 0, 4]
    v, a, p = w.v_r, w.alpha, w.psi
    g = 1.0 / np.sqrt(1.0 - v * v)
    lrs = 16.0 * math.pi * a ** 2 * p ** 4 * H * rc ** 2
    return rc, (1 + v) / (1 - v) * lrs, g * (1 + v) * a * H / NF


def main():
    params = json.load(open(os.path.join(HERE, "relativistic_spheres.json")))
    out = {"_source": "written by make_relativistic_spheres.py from the FP64 reference (oracle/)"}
    for test in (1, 2, 3):
        w = W.relativistic_sphere(test, params)
        o = oracle.Oracle(w)
        dt = o.max_dt(0.4)
        steps = int(STEPS_PER_RMAX * w.r_edges[-1] / dt)
        o.step(dt, steps)
        zm, tot = o.moments()
        rc, i1, i2 = invariants(w, zm)
        out[str(test)] = {"dt": dt, "steps": steps, "r": rc.tolist(), "I_lum": i1.tolist(),
                          "I_eps": i2.tolist(), "H": zm[:, 0, 2].tolist(), "number_flux": zm[:, 0, 4].tolist()}
        print(f"test {test}: {steps} steps", flush=True)
    json.dump(out, open(os.path.join(HERE, "relativistic_spheres_oracle.json"), "w"))


if __name__ == "__main__":
    main()
