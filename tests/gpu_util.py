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
