"""Writes tests/golden/poiseuille_steady.json: the FP64 oracle's steady state
of a force-driven Poiseuille case of the headline's kind at a density inside
the stable range of the scheme (the headline's eta0 = 0.3 has growing wall
modes): Nx = 96 tanh-stretched, 2x4 half-range x 6 x 4 velocities (K = 192),
Kn = 0.05, eta0 = 0.2, a_y = 0.05, walls at rest at T = 1, Shakhov with the
dense Pr; stepped from its uniform initial state until the residual (the
largest change of n, u_x, u_y, T per unit time over one step) is below 1e-8.

Calls only the oracle (oracle/fdlb_oracle.c through oracle/oracle.py); the
GPU path takes the same number of steps from the same start and compares.

    python tests/golden/make_poiseuille_steady.py [--tol 1e-8] [--chunk 1000]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fdlb_inputs as I  # noqa: E402
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "poiseuille_steady.json")
OVERRIDES = dict(nx=96, qx_half=4, eta0=0.2)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--chunk", type=int, default=1000)
    ap.add_argument("--max-steps", type=int, default=400000)
    a = ap.parse_args()
    cfg = I.config("C3", precision=0, **OVERRIDES)
    o = O.Oracle(**{k: v for k, v in cfg.items() if k != "precision"})
    cfg["dt"] = o.dt     # the comparison passes the same time step explicitly
    t0 = time.time()
    steps, r = 0, float("inf")
    while steps < a.max_steps:
        # plain steps, then one step with the residual
        o.step(a.chunk - 1)
        r = o.step_resid()
        steps += a.chunk
        print("steps %d residual %.3e (%.0f s)" % (steps, r, time.time() - t0), flush=True)
        if r < a.tol:
            break
    m = o.moments()
    json.dump({"workload": "force-driven Poiseuille, Nx 96, K 192, eta0 0.2, FP64 oracle, uniform initial state",
               "config": cfg, "steps": steps, "residual": r, "tol": a.tol,
               "threads": O.lib().orc_threads(),
               "moments": {nm: [float(v) for v in m[i]] for i, nm in
                           enumerate(("n", "ux", "uy", "T", "qx", "qy", "Pxx", "Pxy", "Pyy", "Pzz"))}},
              open(OUT, "w"), indent=0)
    print("wrote %s: %d steps, residual %.3e" % (OUT, steps, r), flush=True)


if __name__ == "__main__":
    main()
