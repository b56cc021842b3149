"""Helpers shared by the GPU tests (seeded inputs, oracle runs, comparisons)."""
import numpy as np

import fdlb_inputs as I


def rel_moment_errors(gpu, ref, floor=1e-4):
    """Per-moment error with the normalisation of the parity target:
    n and T pointwise relative; u, q and stresses relative to max |ref|.
    Fields that vanish by symmetry (e.g. u_y in Fourier flow) are compared
    against `floor` in the reduced units (thermal speed and density ~ 1)."""
    out = {}
    names = ("n", "ux", "uy", "T", "qx", "qy", "Pxx", "Pxy", "Pyy", "Pzz")
    for i, nm in enumerate(names):
        if nm in ("n", "T", "Pxx", "Pyy", "Pzz"):
            e = np.max(np.abs(gpu[i] - ref[i]) / np.abs(ref[i]))
        else:
            scale = max(np.max(np.abs(ref[i])), floor)
            e = np.max(np.abs(gpu[i] - ref[i])) / scale
        out[nm] = float(e)
    return out


def seeded_state(seed, nx, K, amp=0.05, eps=1e-3):
    return I.smooth_fields(seed, nx, amp=amp), I.noise(seed + 1000, K, nx, eps)


# Tolerance of the FP32-bulk mode against the FP64 oracle, per moment.  The
# normalisation is that of rel_moment_errors, with the scale of a field that
# crosses zero taken as max(max |ref|, FP32_FLOOR): in reduced units the
# thermal speed, density, pressure and heat-flux scales are 1, and a field
# that has not formed yet or vanishes to second order in the drive (u_x and
# q_x of a Poiseuille flow from rest: 1e-8 and 2e-7 after 40 steps) is held
# to an absolute 1e-8 of the thermal scale, a sixth of FP32's unit roundoff.
TOL32 = 1e-5
FP32_FLOOR = 1e-3
MOMENTS = ("n", "ux", "uy", "T", "qx", "qy", "Pxx", "Pxy", "Pyy", "Pzz")


def assert_fp32_moments(gpu, ref, label, tol=TOL32):
    """Every moment (n, u, T, q and the stresses) of an FP32-bulk run within
    `tol` of the FP64 oracle; returns the errors."""
    err = rel_moment_errors(gpu, ref, floor=FP32_FLOOR)
    print("FP32 bulk %s:" % label, {k: "%.1e" % v for k, v in err.items()}, flush=True)
    bad = {k: err[k] for k in MOMENTS if not err[k] < tol}
    assert not bad, (label, bad)
    return err
