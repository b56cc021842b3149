"""fdlb_init_static: the set-up that allocates no device memory (its workspace
is the library's static per-device array) evolves cases exactly as fdlb_init
with a caller-owned workspace does, on two calls in a row, the second with a
smaller input; it rejects a second live handle on the device and cases that
do not fit."""
import numpy as np
import pytest
import torch

import fdlb_inputs as I
from paper_2308_15407_amd import fdlb as F

pytestmark = pytest.mark.gpu


def _run_workspace(cases, steps):
    nbytes = F.fdlb_workspace_bytes(cases)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    h = F.fdlb_init(cases, ws.data_ptr(), nbytes, stream.cuda_stream)
    try:
        F.fdlb_step(h, steps)
        mom = [F.fdlb_moments(h, c, cases[c]["nx"]) for c in range(len(cases))]
        f = [F.fdlb_get_f(h, c, 2 * cases[c]["qx_half"] * cases[c]["qy"] * cases[c]["qz"], cases[c]["nx"])
             for c in range(len(cases))]
    finally:
        F.fdlb_destroy(h)
    return mom, f


def _run_static(cases, steps):
    stream = torch.cuda.current_stream()
    h = F.fdlb_init_static(cases, stream.cuda_stream)
    try:
        # the device array is held: a second static set-up must be refused
        with pytest.raises(F.FdlbError) as e:
            F.fdlb_init_static([I.config("C1", nx=16)], stream.cuda_stream)
        assert e.value.code == F.FDLB_ESTATE
        F.fdlb_step(h, steps)
        mom = [F.fdlb_moments(h, c, cases[c]["nx"]) for c in range(len(cases))]
        f = [F.fdlb_get_f(h, c, 2 * cases[c]["qx_half"] * cases[c]["qy"] * cases[c]["qz"], cases[c]["nx"])
             for c in range(len(cases))]
    finally:
        F.fdlb_destroy(h)
    return mom, f


@pytest.mark.parametrize("first,second", [
    # full-size Poiseuille (FP32 bulk, 17.8 MiB of the 32 MiB array), then a
    # smaller batch: full-size Couette in FP64 plus a ragged Fourier case
    ([I.config("C3", precision=1)], [I.config("C2", precision=0), I.config("C1", nx=37)]),
])
def test_static_workspace_matches_caller_workspace(first, second):
    assert F.fdlb_workspace_bytes(second) < F.fdlb_workspace_bytes(first)
    for cases in (first, second):
        steps = 12
        ms, fs = _run_static(cases, steps)
        mw, fw = _run_workspace(cases, steps)
        for c in range(len(cases)):
            print("static vs workspace, case %d (nx=%d): max |dm| %.1e" %
                  (c, cases[c]["nx"], np.max(np.abs(ms[c] - mw[c]))), flush=True)
            assert np.array_equal(ms[c], mw[c])
            assert np.array_equal(fs[c], fw[c])


def test_static_workspace_rejects_cases_that_do_not_fit():
    stream = torch.cuda.current_stream()
    big = [I.config("R2")]
    assert F.fdlb_workspace_bytes(big) > F.FDLB_STATIC_WORKSPACE_BYTES
    with pytest.raises(F.FdlbError) as e:
        F.fdlb_init_static(big, stream.cuda_stream)
    assert e.value.code == F.FDLB_ENOMEM
    # nothing was left held: a set-up that fits still succeeds
    h = F.fdlb_init_static([I.config("C1", nx=16)], stream.cuda_stream)
    F.fdlb_destroy(h)
