"""Writes tests/golden/c3_divergence.json: the FP64 oracle's trajectory of the
full-size Poiseuille workload (Nx = 512 tanh-stretched, 2x16 half-range x 6 x 4
velocities, Kn = 0.05, eta0 = 0.3, a_y = 0.05, Shakhov with the dense Pr) from
its uniform initial state: max |u_x| and max |u_y| every 100 steps until the
moments are no longer finite.  At this density the discretised operator has
growing modes at the walls (WENO-5 advection with sixth-order gradients in J1
next to diffuse walls), so u_x, zero in exact arithmetic, grows about tenfold
per 100 steps and the run ends non-finite; the GPU path must follow the same
trajectory.

Calls only the oracle (oracle/fdlb_oracle.c through oracle/oracle.py).

    python tests/golden/make_c3_divergence.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fdlb_inputs as I  # noqa: E402
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_divergence.json")


def main():
    cfg = I.config("C3", precision=0)
    o = O.Oracle(**{k: v for k, v in cfg.items() if k != "precision"})
    cfg["dt"] = o.dt
    t0 = time.time()
    steps, rows = 0, []
    while steps < 4000:
        o.step(100)
        steps += 100
        m = o.moments()
        finite = bool(np.all(np.isfinite(m)))
        rows.append({"step": steps, "max_abs_ux": float(np.max(np.abs(m[1]))) if finite else None,
                     "max_abs_uy": float(np.max(np.abs(m[2]))) if finite else None, "finite": finite})
        print(rows[-1], "%.0f s" % (time.time() - t0), flush=True)
        if not finite:
            break
    json.dump({"workload": "C3 Poiseuille full size, FP64 oracle, uniform initial state", "config": cfg,
               "every": 100, "trajectory": rows}, open(OUT, "w"), indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
