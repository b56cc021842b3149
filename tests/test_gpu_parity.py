"""GPU path (libfdlb.so through the C ABI) against the FP64 CPU oracle.

FP64 parity bar: 1e-10 per moment (n, T pointwise relative; velocities,
heat fluxes and shear stress relative to their channel maximum), and the same
bound on the populations relative to their maximum.
"""
import numpy as np
import pytest

import fdlb_inputs as I
from oracle import oracle as O
from tests.gpu_util import assert_fp32_moments, rel_moment_errors, seeded_state

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _pair(cfg, seed, amp=0.05, eps=1e-3):
    from paper_2308_15407_amd.solver import Solver
    s = Solver(cfg)
    o = O.Oracle(**{k: v for k, v in cfg.items() if k != "precision"})
    fields, noise = seeded_state(seed, cfg["nx"], o.K, amp, eps)
    s.set_state(0, fields, noise)
    o.set_state(fields, noise)
    return s, o


def _compare(s, o, tol, label):
    m_g, m_o = s.moments(0), o.moments()
    err = rel_moment_errors(m_g, m_o)
    f_g, f_o = s.get_f(0), o.get_f()
    ferr = np.max(np.abs(f_g - f_o)) / np.max(np.abs(f_o))
    print(label, "f err %.2e" % ferr, {k: "%.1e" % v for k, v in err.items()}, flush=True)
    assert ferr < tol, (label, ferr)
    for k, v in err.items():
        assert v < tol, (label, k, v)


def test_initial_state_matches():
    cfg = I.config("C1")
    s, o = _pair(cfg, 1)
    _compare(s, o, TOL64, "C1 init")


@pytest.mark.parametrize("steps", [1, 10, 60])
def test_c1_fourier_bgk_steps(steps):
    cfg = I.config("C1")
    s, o = _pair(cfg, 2)
    s.step(steps)
    o.step(steps)
    _compare(s, o, TOL64, "C1 %d steps" % steps)


def test_couette_shakhov_stretched_ragged():
    # 80 cells: two update tiles (63 + 17) and five table tiles of 16
    cfg = I.config("C2", nx=80, qx_half=6)
    s, o = _pair(cfg, 3)
    s.step(20)
    o.step(20)
    _compare(s, o, TOL64, "Couette nx=80")


def test_poiseuille_dense_pr_force():
    cfg = I.config("C3", nx=40, qx_half=5, qy=6, qz=4)
    s, o = _pair(cfg, 4)
    s.step(20)
    o.step(20)
    _compare(s, o, TOL64, "Poiseuille nx=40")


def test_free_molecular_and_tiny_grid():
    cfg = dict(I.BASE, nx=7, qx_half=3, qy=3, qz=3, kn=0.0, eta0=0.0, t_left=1.0, t_right=1.3, t_init=1.1)
    s, o = _pair(cfg, 5)
    s.step(30)
    o.step(30)
    _compare(s, o, TOL64, "free molecular nx=7")


@pytest.mark.parametrize("kxc,waves", [(1, 1), (3, 2), (0, 8)])
def test_tiling_does_not_change_results(kxc, waves):
    cfg = I.config("C2", nx=70, qx_half=4)
    s, o = _pair(cfg, 6)
    s.set_tiling(kxc, waves)
    s.step(10)
    o.step(10)
    _compare(s, o, TOL64, "tiling %d/%d" % (kxc, waves))


def test_graph_replay_matches_direct_launches():
    from paper_2308_15407_amd.solver import Solver
    cfg = I.config("C1", nx=40)
    fields, noise = seeded_state(7, 40, 72)
    a = Solver(cfg)
    b = Solver(cfg, graph_steps=5)
    for s in (a, b):
        s.set_state(0, fields, noise)
    a.step(23)
    b.step(23)
    fa, fb = a.get_f(0), b.get_f(0)
    assert np.array_equal(fa, fb)


def test_full_size_c2_and_c3_few_steps():
    for name, steps in (("C2", 3), ("C3", 2)):
        cfg = I.config(name)
        s, o = _pair(cfg, 8)
        s.step(steps)
        o.step(steps)
        _compare(s, o, TOL64, "%s full size %d steps" % (name, steps))


def test_sweep_batch_at_full_size_matches_oracle_on_sampled_cases():
    """The 256-case sweep batch as bench.py runs it (one launch map, FP32 bulk,
    tiling 8 x 8, graph replay): sampled small cases agree with the FP64
    oracle to the FP32-bulk tolerances, and with the same case run alone
    bit for bit."""
    from paper_2308_15407_amd import sweep
    from paper_2308_15407_amd.solver import Solver
    cases = sweep.sweep_cases(256)
    steps = 40
    s = Solver(cases, tiling=(8, 8), graph_steps=20)
    s.step(steps)
    picks = [i for i, c in enumerate(cases) if c["nx"] == 64 and c["qx_half"] <= 8][:4]
    assert len(picks) == 4
    for i in picks:
        cfg = cases[i]
        o = O.Oracle(**{k: v for k, v in cfg.items() if k != "precision"})
        o.step(steps)
        assert_fp32_moments(s.moments(i), o.moments(), "sweep case %d" % i)
        alone = Solver(cfg, tiling=(8, 8))
        alone.step(steps)
        assert np.array_equal(alone.moments(0), s.moments(i))


@pytest.mark.parametrize("flow,prec", [("C2", 0), ("C3", 0), ("C2", 1)])
def test_largest_velocity_sets(flow, prec):
    """Q_x^h = 32 (the largest half-range order) and Q_y = Q_z = 8 (the largest
    full-range orders), K = 4096: the projection tables no longer fit the
    update block's LDS and are read from global memory; with body force the
    force kernel spans 8 y-nodes.  140 cells: three update tiles."""
    cfg = dict(I.config(flow, nx=140, qx_half=32, qy=8, qz=8), precision=prec)
    s, o = _pair(cfg, 9)
    s.step(4)
    o.step(4)
    if prec == 0:
        _compare(s, o, TOL64, "%s K=4096" % flow)
    else:
        assert_fp32_moments(s.moments(0), o.moments(), "%s K=4096" % flow)


@pytest.mark.parametrize("base,kw,prec", [("C2", dict(nx=80, qx_half=6), 0), ("C1", dict(nx=64), 0),
                                          ("C3", dict(nx=48, qx_half=5, qy=6, qz=4), 0),
                                          ("C2", dict(nx=80, qx_half=6), 1)])
def test_revised_enskog_chi(base, kw, prec):
    """chi_mode 1: chi from the revised Enskog (Fischer-Methfessel) average
    density, computed on the GPU by its own pass from the chunk partials."""
    cfg = dict(I.config(base, **kw), chi_mode=1, precision=prec)
    s, o = _pair(cfg, 12)
    s.step(15)
    o.step(15)
    if prec == 0:
        _compare(s, o, TOL64, "%s chi_mode 1" % base)
    else:
        assert_fp32_moments(s.moments(0), o.moments(), "%s chi_mode 1" % base)
