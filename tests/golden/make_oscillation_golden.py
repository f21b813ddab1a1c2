"""Write the FP64 oracle's droplet-oscillation reference (Sec. IV.C) to
tests/golden/oscillation_1024_tau<tau>.json.

Workload: 1024 x 1024 periodic lattice, elliptical droplet with semi-axes 160
(x) and 120 (y) lattice units (Eqs. ISD, REL), W = 2, Carnahan-Starling EOS
with a = b = c = k = 1 at T_r = 0.7, Maxwell densities, U(+-1e-3) noise of
seed 8, BGK, eps = 1.73, sigma = 1, G = -1, 40000 steps.

Stored: the +x extent through the centre every 20 steps (the rho_m crossing of
the two rows next to y0), the mass at t = 0 and at the end, the period of a
damped cosine fitted to the extent series, and the density at 256 seeded
cells and along the two centre rows at t = 10000, 20000, 30000 and 40000.

Only the CPU oracle (oracle/) computes the run; the extent and the fit are
the measurement helpers of the tests.  One tau takes about 40 minutes on 8
cores.  Usage:  python -m tests.golden.make_oscillation_golden 1.0
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import lbmref  # noqa: E402
from paper_2003_07968_amd import workloads as W  # noqa: E402
from tests.helpers import fit_damped_period, oracle_params, x_extent  # noqa: E402

N, STEPS, EVERY = 1024, 40000, 20
SNAP_TIMES = (10000, 20000, 30000, 40000)
N_CELLS, CELL_SEED = 256, 12


def sample_cells():
    """Seeded cell indices (y * N + x) at which the density is stored."""
    rng = np.random.default_rng(CELL_SEED)
    return sorted(int(v) for v in rng.choice(N * N, size=N_CELLS, replace=False))


def path_for(tau):
    return os.path.join(HERE, f"oscillation_1024_tau{tau:.1f}.json")


def main(tau):
    p, rho0 = W.ellipse_case(n=N, tr=0.7, tau=tau)
    rg, rl = W.unit_cs_coexistence(0.7)
    rho_m = 0.5 * (rg + rl)
    P = oracle_params(lbmref, p)
    f = lbmref.init(P, rho0)
    cells = sample_cells()
    ts, rs, snaps = [], [], {}
    mass0 = None
    t0 = time.perf_counter()
    for k in range(STEPS // EVERY + 1):
        if k:
            lbmref.step(P, f, EVERY)
        rho = lbmref.moments(P, f)["rho"]
        t = k * EVERY
        if mass0 is None:
            mass0 = float(rho.sum())
        ts.append(t)
        rs.append(x_extent(rho[N // 2 - 1:N // 2 + 1], rho_m))
        if t in SNAP_TIMES:
            snaps[str(t)] = {"cells": [float(rho.flat[c]) for c in cells],
                             "centre_rows": rho[N // 2 - 1:N // 2 + 1].tolist()}
            print(f"t={t}: extent {rs[-1]:.6f}, {time.perf_counter() - t0:.0f} s", flush=True)
    mass1 = float(rho.sum())
    period, popt = fit_damped_period(ts, rs)
    out = {
        "_about": "FP64 CPU oracle, droplet oscillation of Sec. IV.C (BGK): 1024x1024 periodic, "
                  "ellipse 160 (x) / 120 (y), W=2, Carnahan-Starling a=b=c=k=1 at T_r=0.7, "
                  "Maxwell densities, U(+-1e-3) noise seed 8, eps=1.73, sigma=1, G=-1. "
                  "Written by tests/golden/make_oscillation_golden.py from oracle/ only.",
        "tau": tau, "n": N, "steps": STEPS, "every": EVERY,
        "oracle_threads": lbmref.threads(),
        "t": ts, "extent": rs,
        "mass0": mass0, "mass_end": mass1, "drift": abs(mass1 / mass0 - 1),
        "period": period, "fit": [float(v) for v in popt],
        "sample_cells": cells, "snapshots": snaps,
        "wall_s": round(time.perf_counter() - t0, 1),
    }
    with open(path_for(tau), "w") as fh:
        json.dump(out, fh, separators=(",", ":"))
    print(f"tau={tau}: period {period:.2f}, drift {out['drift']:.2e}, "
          f"{out['wall_s']} s -> {path_for(tau)}", flush=True)


if __name__ == "__main__":
    for arg in sys.argv[1:] or ["1.0"]:
        main(float(arg))
