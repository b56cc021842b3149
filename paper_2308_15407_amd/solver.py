"""Solver: a batch of FDLB channel cases on one MI355X.

PyTorch supplies the device workspace (one uint8 tensor) and the stream; all
arithmetic happens in libfdlb.so.  Fails loudly when no HIP device or no
built library is present.
"""
import numpy as np
import torch

from . import fdlb as F


class Solver:
    def __init__(self, cases, device="cuda:0", stream=None, graph_steps=0, tiling=None):
        if isinstance(cases, dict):
            cases = [cases]
        if not torch.cuda.is_available():
            raise RuntimeError("the FDLB solver needs a HIP device (torch.cuda.is_available() is False)")
        self.cases = [dict(c) for c in cases]
        self.device = torch.device(device)
        nbytes = F.fdlb_workspace_bytes(self.cases)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.handle = F.fdlb_init(self.cases, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
        self.nx = [c["nx"] for c in self.cases]
        self.K = [2 * c["qx_half"] * c["qy"] * c["qz"] for c in self.cases]
        if tiling is not None:
            F.fdlb_set_tiling(self.handle, *tiling)
        if graph_steps:
            F.fdlb_set_graph_steps(self.handle, graph_steps)

    @property
    def ncases(self):
        return len(self.cases)

    def close(self):
        if getattr(self, "handle", None):
            F.fdlb_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        F.fdlb_step(self.handle, n)

    def synchronize(self):
        self.stream.synchronize()

    def moments(self, c=0):
        return F.fdlb_moments(self.handle, c, self.nx[c])

    def grid(self, c=0):
        return F.fdlb_grid_coords(self.handle, c, self.nx[c])

    def lattice(self, c=0):
        return F.fdlb_lattice(self.handle, c, self.K[c])

    def geometry(self, c=0):
        return F.fdlb_geometry(self.handle, c)

    def dt(self, c=0):
        return F.fdlb_dt(self.handle, c)

    def residual(self):
        return F.fdlb_residual(self.handle, self.ncases)

    def run_to_steady(self, tol=1e-8, max_steps=10 ** 6, check_every=100):
        return F.fdlb_run_to_steady(self.handle, self.ncases, tol, max_steps, check_every)

    def promote(self, c=0):
        F.fdlb_promote(self.handle, c)

    def set_restart_on_nonfinite(self, on=True):
        F.fdlb_set_restart_on_nonfinite(self.handle, on)

    def restarts(self):
        return F.fdlb_restarts(self.handle, self.ncases)

    def set_stall_checks(self, checks):
        F.fdlb_set_stall_checks(self.handle, checks)

    def set_state(self, c, fields, noise=None):
        F.fdlb_set_state(self.handle, c, fields, noise)

    def get_f(self, c=0):
        return F.fdlb_get_f(self.handle, c, self.K[c], self.nx[c])

    def set_f(self, c, f):
        F.fdlb_set_f(self.handle, c, f)

    def precision(self, c=0):
        return F.fdlb_case_precision(self.handle, c)

    def set_tiling(self, kx_per_chunk=0, waves=4):
        F.fdlb_set_tiling(self.handle, kx_per_chunk, waves)

    def set_graph_steps(self, n):
        F.fdlb_set_graph_steps(self.handle, n)

    def profile(self, nrep=50):
        """Per-kernel average ms: [table, update1..3 (FP64), update1..3 (FP32)]."""
        return F.fdlb_profile(self.handle, nrep)

    def mass(self, c=0):
        x, jac = self.grid(c)
        return float(np.sum(self.moments(c)[0] * jac) * 2.0 / self.nx[c])


class ReducedSolver:
    """A batch of cases in the paper's reduced form (include/fdlb.h, fdlb_r1_*),
    FP64: Fourier cases as phi and theta on the 2 qx_half x-nodes (1D),
    Couette and Poiseuille cases on the 2 qx_half x qy (x, y) nodes (2D); one
    dimension per batch."""

    def __init__(self, cases, device="cuda:0", stream=None):
        if isinstance(cases, dict):
            cases = [cases]
        if not torch.cuda.is_available():
            raise RuntimeError("the FDLB solver needs a HIP device (torch.cuda.is_available() is False)")
        self.cases = [dict(c) for c in cases]
        self.device = torch.device(device)
        nbytes = F.fdlb_r1_workspace_bytes(self.cases)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.handle = F.fdlb_r1_init(self.cases, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
        self.nx = [c["nx"] for c in self.cases]
        self.rows = [4 * c["qx_half"] * (c.get("qy", 3) if c.get("flow", 0) != 0 else 1) for c in self.cases]

    @property
    def ncases(self):
        return len(self.cases)

    def close(self):
        if getattr(self, "handle", None):
            F.fdlb_r1_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        F.fdlb_r1_step(self.handle, n)

    def synchronize(self):
        self.stream.synchronize()

    def moments(self, c=0):
        return F.fdlb_r1_moments(self.handle, c, self.nx[c])

    def set_state(self, c, fields, noise=None):
        F.fdlb_r1_set_state(self.handle, c, fields, noise)

    def get_f(self, c=0):
        """[rows][nx]: phi rows (kx qy + ky in 2D), then theta rows."""
        return F.fdlb_r1_get_f(self.handle, c, self.rows[c], self.nx[c])

    def dt(self, c=0):
        return F.fdlb_r1_dt(self.handle, c)

    def grid(self, c=0):
        """Cell centres and metric dx/deta of case c."""
        return F.fdlb_case_grid(self.cases[c])
