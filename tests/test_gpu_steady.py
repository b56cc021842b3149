"""Steady states against the FP64 oracle's, each stored by the generator of
the same name under tests/golden/ (the oracle run from the uniform initial
state until the residual was below 1e-8):

  c2_steady.json          the full-size Couette workload (Nx = 256
                          tanh-stretched, K = 256, Kn = 0.1, eta0 = 0.2,
                          walls T = 1 at u_y = -/+0.2, Shakhov Pr = 2/3);
  poiseuille_steady.json  force-driven Poiseuille of the headline's kind
                          (Kn = 0.05, a_y = 0.05, 6 x 4 transverse rule,
                          Shakhov with the dense Pr) at Nx = 96, K = 192 and
                          eta0 = 0.2, inside the density range where the
                          scheme reaches a steady state.

The GPU takes the same number of steps with the same time step from the same
start: FP64 within 1e-10 per moment, FP32 bulk within 1e-5."""
import json
import os

import numpy as np
import pytest

from tests.gpu_util import assert_fp32_moments, rel_moment_errors

pytestmark = pytest.mark.gpu

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GOLDEN = os.path.join(GOLDEN_DIR, "c2_steady.json")
NAMES = ("n", "ux", "uy", "T", "qx", "qy", "Pxx", "Pxy", "Pyy", "Pzz")


def _golden(path=GOLDEN):
    d = json.load(open(path))
    ref = np.array([d["moments"][k] for k in NAMES])
    return d, ref


def test_c2_steady_state_fp64_matches_oracle():
    from paper_2308_15407_amd.solver import Solver
    d, ref = _golden()
    cfg = dict(d["config"], precision=0)
    s = Solver(cfg, graph_steps=1000)
    assert s.dt(0) == cfg["dt"]
    steps = d["steps"]
    s.step(steps)
    r = s.residual()[0]
    m = s.moments(0)
    print("C2 steady, FP64: %d steps, residual %.3e (oracle %.3e)" % (steps, r, d["residual"]), flush=True)
    err = rel_moment_errors(m, ref)
    print("FP64 steady vs oracle:", {k: "%.1e" % v for k, v in err.items()}, flush=True)
    for k in NAMES:
        assert err[k] < 1e-10, (k, err[k])
    assert r < 2 * d["tol"]


def test_c2_steady_state_fp32_bulk_run_matches_oracle():
    """FP32 bulk from the same start, run to the same tolerance.  The FP32 map
    comes to rest at a fixed point of its own (sub-ulp increments of the
    stored deviations are lost; C2 loses 4e-5 of its mass on the way), so the
    run promotes the case when its residual reaches the tolerance or 0 and
    finishes in FP64 at the initial mass; that state is the scheme's steady
    state, within the FP32 bound of the oracle's."""
    from paper_2308_15407_amd.solver import Solver
    d, ref = _golden()
    cfg = dict(d["config"], precision=1)
    s = Solver(cfg, graph_steps=500)
    st, res, code = s.run_to_steady(tol=d["tol"], max_steps=400000, check_every=500)
    print("C2 FP32 bulk run to steady: %d steps, residual %.2e, final storage %s" %
          (st[0], res[0], "FP64" if s.precision(0) == 0 else "FP32"), flush=True)
    assert code == 0 and res[0] < d["tol"] and s.precision(0) == 0
    assert_fp32_moments(s.moments(0), ref, "C2 steady after the FP64 finish")


POISEUILLE = os.path.join(GOLDEN_DIR, "poiseuille_steady.json")


def test_poiseuille_steady_state_fp64_matches_oracle():
    from paper_2308_15407_amd.solver import Solver
    d, ref = _golden(POISEUILLE)
    cfg = dict(d["config"], precision=0)
    s = Solver(cfg, graph_steps=1000)
    assert s.dt(0) == cfg["dt"]
    steps = d["steps"]
    s.step(steps)
    r = s.residual()[0]
    m = s.moments(0)
    print("Poiseuille steady, FP64: %d steps, residual %.3e (oracle %.3e)" % (steps, r, d["residual"]),
          flush=True)
    err = rel_moment_errors(m, ref)
    print("FP64 steady vs oracle:", {k: "%.1e" % v for k, v in err.items()}, flush=True)
    for k in NAMES:
        assert err[k] < 1e-10, (k, err[k])
    assert r < 2 * d["tol"]
    # the force drives a flow along y only, symmetric about the channel middle
    assert np.max(np.abs(m[1])) < 1e-6 and np.min(m[2]) > 0.0
    np.testing.assert_allclose(m[2], m[2][::-1], rtol=1e-10, atol=1e-12)


def test_poiseuille_steady_state_fp32_bulk_run_matches_oracle():
    """FP32 bulk from the same start, run to the same tolerance; the run is
    promoted to FP64 storage when its residual stalls or reaches the
    tolerance and finishes there at its initial mass."""
    from paper_2308_15407_amd.solver import Solver
    d, ref = _golden(POISEUILLE)
    cfg = dict(d["config"], precision=1)
    s = Solver(cfg, graph_steps=500)
    st, res, code = s.run_to_steady(tol=d["tol"], max_steps=200000, check_every=500)
    print("Poiseuille FP32 bulk run to steady: %d steps, residual %.2e, final storage %s" %
          (st[0], res[0], "FP64" if s.precision(0) == 0 else "FP32"), flush=True)
    assert code == 0 and res[0] < d["tol"] and s.precision(0) == 0
    assert_fp32_moments(s.moments(0), ref, "Poiseuille steady after the FP64 finish")
