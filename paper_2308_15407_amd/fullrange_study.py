"""Full-range against half-range Gauss-Hermite rules on the x axis (App. A,
fig:full_vs_half).

The paper's comparison: Fourier (walls at T = 1 -/+ 0.5), Couette (walls
moving at u_y = -/+ 1) and Poiseuille (a_y = 0.001) flows at R = 10 and
eta0 = 0.01 (Kn = 1/(6 sqrt2 eta0 chi(eta0) R) = 1.17, transition regime),
steady profiles on a full-range x rule of order Q^H (x_rule = 1, Q^H = 2
qx_half nodes) against the half-range rule of order Q_x^h = 8 (16 nodes).
The paper finds that Q^H of the order of 200 is needed for relative errors
below 1 %.

Everything but the x rule is shared by the two families: the Shakhov model
with the dense Prandtl number, the local contact value, Q_y = 5 (Couette,
Poiseuille) or 4 (Fourier), Q_z = 4, a uniform grid with CELLS_PER_SIGMA
cells per molecular diameter, FP64.  Each profile is compared with a
converged half-range reference (Q_x^h = 100) and with the paper's
comparator (Q_x^h = 8):

    eps_M = max_x |M(x) - M_ref(x)| / (max_x M_ref - min_x M_ref),

M = T (Fourier) or u_y (Couette, Poiseuille), the measure of the quadrature
convergence test.

    python -m paper_2308_15407_amd.fullrange_study run [--out PATH] [--cells-per-sigma N]
"""
import argparse
import json
import os
import time

import numpy as np

from . import quad_study as QS

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "fullrange_results.json")

R = 10.0
ETA0 = 0.01
CELLS_PER_SIGMA = 20
HALF_ORDERS = (8, 16, 32, 100)          # Q_x^h (nodes per half)
HALF_REF = 100
HALF_PAPER = 8
FULL_ORDERS = (8, 16, 24, 32, 48, 64, 80, 100, 128, 150, 176, 200)   # Q^H (total nodes)


def case(flow, q_half=None, q_full=None, cells_per_sigma=CELLS_PER_SIGMA):
    if q_full is not None:
        if q_full % 2:
            raise ValueError("the full-range x rule takes an even order")
        d = QS.case(flow, R, ETA0, q_full // 2, cells_per_sigma)
        d["x_rule"] = 1
    else:
        d = QS.case(flow, R, ETA0, q_half, cells_per_sigma)
        d["x_rule"] = 0
    return d


def run_flow(flow, cells_per_sigma=CELLS_PER_SIGMA, max_steps=600000, chunk=50000, log=print):
    from .solver import Solver
    spec = QS.FLOWS[flow]
    keys = [("half", q) for q in HALF_ORDERS] + [("full", q) for q in FULL_ORDERS]
    cfgs = [case(flow, q_half=q, cells_per_sigma=cells_per_sigma) if kind == "half"
            else case(flow, q_full=q, cells_per_sigma=cells_per_sigma) for kind, q in keys]
    log("%s: %d cases, Nx = %d, Kn = %.4f" % (flow, len(cfgs), cfgs[0]["nx"], cfgs[0]["kn"]))
    s = Solver(cfgs, graph_steps=100)
    t0 = time.perf_counter()
    nc = len(cfgs)
    total = np.zeros(nc, dtype=np.int64)
    steps = np.full(nc, -1, dtype=np.int64)
    done = np.zeros(nc, dtype=bool)
    k = 0
    while k < max_steps and not np.all(done):
        st, resid, _ = s.run_to_steady(spec["tol"], min(chunk, max_steps - k), check_every=1000)
        k += chunk
        total += st
        ok = resid < spec["tol"]
        steps = np.where(ok & ~done, total, steps)
        done |= ok
        log("  %s: %d steps, %d of %d converged (%.1f s)" % (flow, k, int(np.sum(done)), nc,
                                                              time.perf_counter() - t0))
    prof = {key: s.moments(i)[spec["m"]] for i, key in enumerate(keys)}
    wall = time.perf_counter() - t0
    ref, paper = prof[("half", HALF_REF)], prof[("half", HALF_PAPER)]
    out = {"tol": spec["tol"], "wall_s": round(wall, 2), "nx": cfgs[0]["nx"], "kn": cfgs[0]["kn"],
           "moment": "T" if spec["m"] == 3 else "u_y",
           "half": {"q": list(HALF_ORDERS), "eps_ref": [QS.eps(prof[("half", q)], ref) for q in HALF_ORDERS]},
           "full": {"q": list(FULL_ORDERS),
                    "eps_ref": [QS.eps(prof[("full", q)], ref) for q in FULL_ORDERS],
                    "eps_half8": [QS.eps(prof[("full", q)], paper) for q in FULL_ORDERS]},
           "converged": {"%s%d" % key: bool(done[i]) for i, key in enumerate(keys)},
           "steps": {"%s%d" % key: int(steps[i]) for i, key in enumerate(keys)},
           "profiles": {"%s%d" % key: [round(float(v), 10) for v in prof[key]] for key in keys}}
    out["full"]["q_min_ref"] = QS.q_min(FULL_ORDERS, out["full"]["eps_ref"])
    out["full"]["q_min_half8"] = QS.q_min(FULL_ORDERS, out["full"]["eps_half8"])
    log("%s: %.1f s; full-range eps vs Q_x^h = %d: %s" % (flow, wall, HALF_REF,
                                                         " ".join("%d:%.2e" % (q, e) for q, e in
                                                                  zip(FULL_ORDERS, out["full"]["eps_ref"]))))
    log("  half-range eps vs Q_x^h = %d: %s" % (HALF_REF, " ".join("%d:%.2e" % (q, e) for q, e in
                                                                  zip(HALF_ORDERS, out["half"]["eps_ref"]))))
    return out


def run(out=DEFAULT_OUT, cells_per_sigma=CELLS_PER_SIGMA, flows=tuple(QS.FLOWS), max_steps=600000, log=print):
    result = {"R": R, "eta0": ETA0, "cells_per_sigma": cells_per_sigma, "half_ref": HALF_REF,
              "half_paper": HALF_PAPER, "eps_limit": QS.EPS_LIMIT, "flows": {}}
    for flow in flows:
        result["flows"][flow] = run_flow(flow, cells_per_sigma, max_steps=max_steps, log=log)
        with open(out, "w") as f:
            json.dump(result, f, indent=1)
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["run"])
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--cells-per-sigma", type=int, default=CELLS_PER_SIGMA)
    ap.add_argument("--flows", default=",".join(QS.FLOWS))
    ap.add_argument("--max-steps", type=int, default=600000)
    a = ap.parse_args()
    run(a.out, a.cells_per_sigma, tuple(a.flows.split(",")), a.max_steps, log=lambda msg: print(msg, flush=True))


if __name__ == "__main__":
    main()
