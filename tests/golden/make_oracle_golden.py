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
  aggregate24_prefix_*.txt       the first 10 RK4 steps of the 24-site aggregate
                                 (depth 4, 20475 ADOs of 24x24)
  aggregate48_prefix_*.txt       the first 2 RK4 steps of the 48-site aggregate
                                 (96 modes, depth 3, 156849 ADOs of 48x48; the
                                 oracle needs ~35 GB and several minutes)
      *_records.txt  [step, P_1..P_N, Re Tr, Im Tr, max|rho-rho^+|] every step
      *_ados.txt     [u, part, k, Re, Im] of sampled ADOs u after the last
                     step: part 0 = row 0 (k = column), part 1 = diagonal

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


def sampled_ados(W, D, n, n_spread):
    """ADO indices sampled for the stored prefixes: the first ADOs of every
    level (the largest ones, next to sigma_0) and an even spread over the
    whole hierarchy (mostly the top level, which holds most ADOs)."""
    from math import comb
    starts = [comb(W + L - 1, W) if L > 0 else 0 for L in range(D + 1)]
    first = [s + k for s in starts[1:] for k in range(3)]
    spread = np.linspace(1, n - 1, n_spread).astype(np.int64).tolist()
    return sorted(set(u for u in first + spread if 0 < u < n))


def aggregate_prefix(name, prob, n_steps, n_spread):
    W, n = oracle.sizes(prob)
    N = prob["H"].shape[0]
    t0 = time.time()
    x = np.zeros((n, N, N), np.complex128)
    x[0] = prob["rho0"]
    _, rec = oracle.propagate(prob, x, prob["dt_fs"], n_steps, 1, prob["observable"],
                              inplace=True)
    steps = np.arange(len(rec))[:, None]
    np.savetxt(os.path.join(HERE, name + "_prefix_records.txt"), np.hstack([steps, rec]),
               fmt="%.17g",
               header="oracle: %s, FP64 RK4 dt=%g fs, first %d steps, every step: step, "
                      "P_1..P_%d, Re Tr, Im Tr, max|rho-rho^+|" % (name, prob["dt_fs"], n_steps, N))
    rows = []
    for u in sampled_ados(W, prob["depth"], n, n_spread):
        for k in range(N):
            rows.append([u, 0, k, x[u, 0, k].real, x[u, 0, k].imag])
        for k in range(N):
            rows.append([u, 1, k, x[u, k, k].real, x[u, k, k].imag])
    np.savetxt(os.path.join(HERE, name + "_prefix_ados.txt"), np.array(rows),
               fmt=["%d", "%d", "%d", "%.17g", "%.17g"],
               header="oracle: %s after %d FP64 RK4 steps of dt=%g fs from rho0=|0><0|: "
                      "u, part (0 = row 0, 1 = diagonal), k, Re, Im" % (name, n_steps, prob["dt_fs"]))
    print("%s prefix (%d steps): %.1f s" % (name, n_steps, time.time() - t0), flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["population", "absorption", "aggregate24", "aggregate48"]
    if "population" in which:
        fmo_population()
    if "absorption" in which:
        fmo_absorption()
    if "aggregate24" in which:
        aggregate_prefix("aggregate24", hi.aggregate24(), 10, 21)
    if "aggregate48" in which:
        aggregate_prefix("aggregate48", hi.aggregate48(), 2, 13)
