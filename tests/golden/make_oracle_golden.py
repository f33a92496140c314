"""Write the stored oracle references used by the GPU parity tests.

Calls only the FP64 oracle (oracle/) on inputs from heom_inputs; nothing here
touches the GPU library.  Full-length FMO-like runs take minutes in the oracle,
so their records are computed once and stored as text:

  fmo_like_fp64_records.txt      2000 RK4 steps of the 7-site FMO-like system
                                 (depth 4, 3060 ADOs), every 10th record
                                 [step, populations (7), Re Tr, Im Tr, herm]
  fmo_like_absorption_P.txt      1000 steps of the three dipole-correlation
                                 runs (N = 8): [step, Re P_x, Im P_x, Re P_y,
                                 Im P_y, Re P_z, Im P_z] at every step

Run:  python tests/golden/make_oracle_golden.py
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import heom_inputs as hi  # noqa: E402
import oracle  # noqa: E402


def fmo_population():
    prob = hi.fmo_like()
    t0 = time.time()
    _, rec = oracle.run(prob)
    steps = np.arange(len(rec))[:, None]
    out = np.hstack([steps, rec])[::10]
    np.savetxt(os.path.join(HERE, "fmo_like_fp64_records.txt"), out, fmt="%.17g",
               header="oracle: fmo_like (seed 7), FP64 RK4 dt=1 fs, 2000 steps, every 10th "
                      "record: step, P_1..P_7, Re Tr, Im Tr, max|rho-rho^+|")
    print("fmo_like population: %.1f s" % (time.time() - t0), flush=True)


def fmo_absorption():
    runs = hi.fmo_like_absorption()
    t0 = time.time()
    cols = []
    for r in runs:
        _, rec = oracle.run(r)
        cols += [rec[:, 0], rec[:, 1]]
    steps = np.arange(len(cols[0]))
    out = np.column_stack([steps] + cols)
    np.savetxt(os.path.join(HERE, "fmo_like_absorption_P.txt"), out, fmt="%.17g",
               header="oracle: fmo_like_absorption (seeds 7, 70), FP64 RK4 dt=1 fs, 1000 steps: "
                      "step, Re/Im P_x, Re/Im P_y, Re/Im P_z")
    print("fmo_like absorption: %.1f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["population", "absorption"]
    if "population" in which:
        fmo_population()
    if "absorption" in which:
        fmo_absorption()
