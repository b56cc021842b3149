"""Short, fixed run of one workload for profilers (rocprofv3 kernel traces and
hardware counters):

  python -m paper_2308_15407_amd.profile_case --workload R2 --precision 0 --steps 3

runs `steps` RK3 steps of the named configuration (after one untimed step)
with the given update tiling, then one device copy of --copy-mib MiB (the
calibration kernel for memory-traffic counters).  --reduced runs the same
case in the reduced 1D form (phi, theta; Fourier workloads, FP64)."""
import argparse
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="R2")
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--tiling", type=int, nargs=2, default=None, metavar=("KX_PER_CHUNK", "WAVES"))
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--reduced", action="store_true")
    a = ap.parse_args(argv)
    import torch
    import fdlb_inputs as I
    from . import fdlb as F
    from .solver import ReducedSolver, Solver
    if a.reduced:
        s = ReducedSolver(I.config(a.workload, precision=0))
    elif a.workload == "sweep":
        from . import sweep
        cfg = sweep.sweep_cases(256, precision=a.precision)
    else:
        cfg = I.config(a.workload, precision=a.precision)
    if not a.reduced:
        s = Solver(cfg)
        if a.tiling:
            s.set_tiling(*a.tiling)
        else:
            from . import autotune
            autotune.tune(s)
    s.step(1)
    torch.cuda.synchronize()
    s.step(a.steps)
    torch.cuda.synchronize()
    if a.copy_mib > 0:
        n = a.copy_mib << 20
        buf = torch.empty(2 * n, dtype=torch.uint8, device="cuda")
        F.fdlb_copy_probe(buf.data_ptr(), buf.data_ptr() + n, n, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    print("profile_case done: %s%s precision %d, %d steps" % (a.workload, " reduced" if a.reduced else "",
                                                               a.precision, a.steps), flush=True)


if __name__ == "__main__":
    main()
