"""Full-range Gauss-Hermite rule on the x axis (App. A, fig:full_vs_half):
x_rule = 1 puts the 2 qx_half roots of He_{2 qx_half} on x, in the layout of
the half-range lattice, with the full-range projections (eq:g_H, eq:H_gk)
taken through the NB_WIDE base rule of the wide table pass.

Parity with the oracle (whose full-range x projection is pinned in
tests/test_oracle_pins.py) at orders the oracle supports (2 qx_half <= 96);
at the paper's order 200, properties that hold at any order.
"""
import numpy as np
import pytest

import fdlb_inputs as I
from tests.gpu_util import assert_fp32_moments, seeded_state
from tests.test_gpu_parity import TOL64, _compare, _pair

pytestmark = pytest.mark.gpu


def _solver(cfgs, **kw):
    from paper_2308_15407_amd.solver import Solver
    return Solver(cfgs, **kw)


@pytest.mark.parametrize("flow,kw,prec", [("C1", dict(nx=24, qx_half=4), 0),
                                          ("C2", dict(nx=40, qx_half=8), 0),
                                          ("C3", dict(nx=36, qx_half=20, qy=4, qz=4), 0),
                                          ("C1", dict(nx=30, qx_half=48, qy=2, qz=2), 0),
                                          ("C2", dict(nx=40, qx_half=8), 1)])
def test_full_range_x_matches_oracle(flow, kw, prec):
    cfg = dict(I.config(flow, x_rule=1, **kw), precision=prec)
    s, o = _pair(cfg, 80)
    s.step(6)
    o.step(6)
    label = "%s full-range Q=%d" % (flow, 2 * kw["qx_half"])
    if prec == 0:
        _compare(s, o, TOL64, label)
    else:
        assert_fp32_moments(s.moments(0), o.moments(), label)


@pytest.mark.parametrize("qh", [16, 50, 100])
def test_full_range_x_projection_reproduces_the_fields(qh):
    """The projected Grad-13-type state on a full-range x rule of order 2 qh
    carries the moments it was built from (the rule resolves the cubic)."""
    nx = 40
    s = _solver(dict(I.config("C2", nx=nx, qx_half=qh, qy=4, qz=4, x_rule=1)))
    fields = I.smooth_fields(90 + qh, nx, amp=0.08)
    s.set_state(0, fields, None)
    m = s.moments(0)
    err = {"n": np.max(np.abs(m[0] - fields[0]) / fields[0]),
           "ux": np.max(np.abs(m[1] - fields[1])), "uy": np.max(np.abs(m[2] - fields[2])),
           "T": np.max(np.abs(m[3] - fields[3]) / fields[3]),
           "qx": np.max(np.abs(m[4] - fields[4])), "Pxy": np.max(np.abs(m[7] - fields[5]))}
    print("full-range Q=%d" % (2 * qh), {k: "%.1e" % v for k, v in err.items()}, flush=True)
    for k, v in err.items():
        assert v < 1e-12, (k, v)


def test_full_range_x_order_200_conserves_mass_and_stays_finite():
    nx = 36
    cfg = I.config("C3", nx=nx, qx_half=100, qy=4, qz=4, x_rule=1, ay=0.01)
    s = _solver(cfg)
    fields, noise = seeded_state(95, nx, 2 * 100 * 16)
    s.set_state(0, fields, noise)
    m0 = s.mass(0)
    s.step(150)
    m = s.moments(0)
    assert np.all(np.isfinite(m))
    assert abs(s.mass(0) - m0) < 1e-13 * m0


def test_batch_mixing_half_and_full_range_x_matches_single_bitwise():
    cfgs = [I.config("C2", nx=40, qx_half=8), I.config("C2", nx=45, qx_half=8, x_rule=1),
            I.config("C1", nx=30, qx_half=24, x_rule=1, precision=1)]
    b = _solver(cfgs)
    singles = [_solver(c) for c in cfgs]
    for i, c in enumerate(cfgs):
        K = 2 * c["qx_half"] * c["qy"] * c["qz"]
        fields, noise = seeded_state(80 + i, c["nx"], K)
        b.set_state(i, fields, noise)
        singles[i].set_state(0, fields, noise)
    b.step(17)
    for i, s in enumerate(singles):
        s.step(17)
        assert np.array_equal(b.get_f(i), s.get_f(0)), i
