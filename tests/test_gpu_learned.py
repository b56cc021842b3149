"""Learned warm start, end to end on the device at a small scale: steady
states computed by the solver train the network (library kernels); on
held-out cases the warm-started solve needs fewer steps to the 1e-8
residual than the cold start and reaches the same steady state."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_warm_start_reduces_steps_to_steady():
    from paper_2308_15407_amd import learned as LW
    train = LW.draw_cases(1, 96, kn_min=0.1, nx=32, qx_max=4)
    held = LW.draw_cases(100001, 6, kn_min=0.1, nx=32, qx_max=4)
    X, Y, kept = LW.build_dataset(train, tol=1e-6, max_steps=200000, batch=96, log=print)
    assert len(kept) >= 80
    model = LW.WarmStartModel().fit(X, Y, epochs=1500, batch=32, lr=2e-3, log=None)
    pred = model.predict(held)
    fields = [LW.warm_fields(c, p) for c in held for p in [pred[held.index(c)]]]
    assert all(f is not None for f in fields)
    mc, _, st_c, rc, _ = LW.solve_steady(held, 1e-8, 400000, check_every=50, precision=0)
    mw, _, st_w, rw, _ = LW.solve_steady(held, 1e-8, 400000, check_every=50, precision=0, fields=fields)
    print("cold steps", st_c, "warm steps", st_w)
    assert np.all(rc < 1e-8) and np.all(rw < 1e-8)
    assert np.sum(st_w) < 0.9 * np.sum(st_c)
    for a, b in zip(mc, mw):        # same steady state (same mass)
        assert np.max(np.abs(a[0] - b[0])) < 1e-6 and np.max(np.abs(a[3] - b[3])) < 1e-6
