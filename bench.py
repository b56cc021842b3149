"""Benchmark: node-velocity updates per second of the FDLB time step on one MI355X.

Workload (default): the plain Couette configuration -- Nx = 256 wall-refined
cells, 2x8 half-range x 4 x 4 full-range velocities (K = 256), Kn = 0.1,
eta0 = 0.2, walls T = 1 moving at u_y = -/+0.2, Shakhov Pr = 2/3, FP64.  One
step = one TVD-RK3 step (three stages of table + update launches) of the whole
case; inputs are resident in device memory before timing starts.

Also reported: the FP32-bulk variant of the same case, a large single case
(Nx = 32768, K = 512) that sizes the memory-bound roofline, the roofline
object for the dominant kernel (the update launch of RK stage 2) with its
time measured by HIP events, and the CPU oracle timed on this host.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="only the main workload")
    ap.add_argument("--large-steps", type=int, default=60)
    ap.add_argument("--retune", action="store_true")
    ap.add_argument("--sweep-steps", type=int, default=100)
    ap.add_argument("--r1-steps", type=int, default=20)
    ap.add_argument("--tts-batch", type=int, default=64, help="held-out cases in the learned time-to-steady leg")
    ap.add_argument("--tts-seq", type=int, default=8, help="cases solved one at a time by the plain FP64 leg")
    return ap.parse_args()


def kernel_src_hash():
    h = hashlib.sha1()
    for f in ("fdlb_kernels.hip", "fdlb_common.h"):
        h.update(open(os.path.join(ROOT, "paper_2308_15407_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:12]


def read_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        parts = line.split()
        if len(parts) >= 6 and parts[0] == "TRAFFIC" and parts[1] == kernel and parts[2] == workload:
            if parts[3] != kernel_src_hash():
                return None
            return float(parts[4]) + float(parts[5])
    return None


def timed_run(solver, steps, warmup):
    import torch
    solver.step(warmup)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(solver.stream)
    solver.step(steps)
    b.record(solver.stream)
    b.synchronize()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def measure(cfg, steps, warmup, retune, graph_steps=50):
    from paper_2308_15407_amd.solver import Solver
    from paper_2308_15407_amd import autotune
    s = Solver(cfg)
    tile = autotune.tune(s, use_cache=True, refresh=retune)
    s.set_graph_steps(graph_steps)
    ms = timed_run(s, steps, warmup)
    cases = cfg if isinstance(cfg, list) else [cfg]
    nodes = sum(c["nx"] * 2 * c["qx_half"] * c["qy"] * c["qz"] for c in cases)
    prof = s.profile(nrep=20)
    return s, ms, nodes, tile, prof


def roofline(prof, nodes, prec, kernel_name, workload):
    """The kernel whose bytes scale with the nodes: the stage-2 update (reads
    f^(1) and f^n, writes f^(2)): 3 passes x bytes per population x nodes,
    algorithmic.  (At small sizes the per-cell table pass can take as long,
    as a latency chain of little traffic.)"""
    s_bytes = 8 if prec == 0 else 4
    t_ms = prof[2] if prec == 0 else prof[5]
    alg = 3.0 * s_bytes * nodes
    achieved = alg / (t_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": read_traffic(kernel_name, workload),
            "kernel": kernel_name, "launch_ms": round(t_ms, 5), "algorithmic_bytes_per_launch": alg}


def cpu_baseline(cfg, budget_s=15.0):
    from oracle import oracle as O
    o = O.Oracle(**{k: v for k, v in cfg.items() if k != "precision"})
    t0 = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t0
    n = max(1, min(2000, int(budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    nodes = cfg["nx"] * o.K
    return {"value": nodes * n / dt, "unit": "node-velocity updates/s", "cores": 1, "kind": "oracle",
            "sample": "%d RK3 steps of the same case (Nx=%d, K=%d) on one host thread, %.1f s" % (n, cfg["nx"], o.K, dt)}


def sweep_leg(steps, retune):
    """All cases of the seeded sweep (256 cases, FP32 bulk) advance together in
    one launch map per stage, replayed from a HIP graph."""
    from paper_2308_15407_amd import sweep
    cases = sweep.sweep_cases(256)
    s, ms, _, tile, prof = measure(cases, steps, 10, retune, graph_steps=20)
    nodes = sum(c["nx"] * 2 * c["qx_half"] * c["qy"] * c["qz"] for c in cases)
    return {"workload": "sweep: 256 seeded cases (PCG64 %d, R >= 2), Nx 64-512, Q_x^h 4-16 x 4 x 4, FP32 bulk"
                        % sweep.SWEEP_SEED,
            "value": round(nodes / (ms * 1e-3), 1), "unit": "node-velocity updates/s", "ms_per_step": round(ms, 5),
            "nodes": nodes, "tiling": {"kx_per_chunk": tile[0], "waves": tile[1]}}


def sweep_r1_leg(steps, retune, ncases=1024):
    """The sweep generator at 1024 cases (FP32 bulk, about 0.3 GB per population
    array, beyond the 256 MB Infinity Cache): whole-step throughput, and the
    algorithmic bytes of a step (8 passes x 4 B per node) over its time as an
    effective bandwidth (the table passes included, so a lower bound on the
    update kernels' rate)."""
    from paper_2308_15407_amd import sweep
    cases = sweep.sweep_cases(ncases)
    s, ms, nodes, tile, prof = measure(cases, steps, 5, retune, graph_steps=10)
    eff = 8 * 4 * nodes / (ms * 1e-3) / 1e9
    return {"workload": "sweep: %d seeded cases (PCG64 %d, R >= 2), Nx 64-512, Q_x^h 4-16 x 4 x 4, FP32 bulk"
                        % (ncases, sweep.SWEEP_SEED),
            "value": round(nodes / (ms * 1e-3), 1), "unit": "node-velocity updates/s", "ms_per_step": round(ms, 5),
            "nodes": nodes, "f_array_bytes": 4 * sum(c["nx"] * 2 * c["qx_half"] * c["qy"] * c["qz"] for c in cases),
            "effective_GBps_whole_step": round(eff, 1), "frac_of_hbm_peak": round(eff / HBM_PEAK_GBS, 4),
            "tiling": {"kx_per_chunk": tile[0], "waves": tile[1]}}


def reduced_leg(steps, workload="R2", warmup=5):
    """A workload in the paper's reduced form, FP64: R2 (Fourier, Nx=32768,
    Q_x^h=16) as the 1D model, 64 rows per cell against the 3D lattice's K = 512
    (the large_case_f64 leg); C2 (Couette, Nx=256) as the 2D model, 2 x 16 x 4
    x 2 = 128 rows per cell against K = 256 (the main line).  A step is three
    launches of the fused stage kernel; its algorithmic bytes are eight passes
    over the rows (each stage reads its input and writes its output, stages 2
    and 3 also read f^n) of 8 B each."""
    import torch
    import fdlb_inputs as I
    from paper_2308_15407_amd.solver import ReducedSolver
    cfg = I.config(workload, precision=0)
    s = ReducedSolver(cfg)
    vals = s.rows[0] * cfg["nx"]
    s.step(warmup)
    s.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s.stream)
    s.step(steps)
    b.record(s.stream)
    b.synchronize()
    ms = a.elapsed_time(b) / steps
    eff = 8 * 8 * vals / (ms * 1e-3) / 1e9
    names = {"R2": "reduced 1D Fourier Nx=32768 uniform, phi/theta on 2x16 x-nodes (64 rows), FP64",
             "C2": "reduced 2D Couette Nx=256 tanh-stretched, phi/theta on 2x8 x 4 (x, y) nodes (128 rows), FP64"}
    return {"workload": names.get(workload, workload),
            "value": round(vals / (ms * 1e-3), 1), "unit": "row-cell updates/s", "ms_per_step": round(ms, 5),
            "values": vals, "effective_GBps_whole_step": round(eff, 1), "frac_of_hbm_peak": round(eff / HBM_PEAK_GBS, 4)}


def time_to_steady_leg(n_batch, n_seq, tol=1e-8, max_steps=400000):
    """Wall-clock time to r < tol per case: plain FP64 cold start (one case at a
    time, a sample of n_seq cases) against batched FP32 bulk + learned warm
    start (n_batch held-out cases in one batch, inference included)."""
    import numpy as np
    import torch
    from paper_2308_15407_amd import learned as LW
    path = LW.default_weights_path()
    if not os.path.exists(path):
        return {"skipped": "no trained warm-start weights in the package"}
    model = LW.WarmStartModel.load(path)
    evp = LW.default_eval_path()
    if not os.path.exists(evp):
        return {"skipped": "no held-out evaluation summary next to the weights"}
    # held-out cases that the plain FP64 solve converges on (fixed by the evaluation)
    held = LW.cases_from_seeds(json.load(open(evp))["seeds"][:n_batch])
    seq_t, seq_st = [], []
    for c in held[:n_seq]:
        _, _, st, res, wall = LW.solve_steady([c], tol, max_steps, check_every=100, precision=0)
        seq_t.append(wall)
        seq_st.append(int(st[0]))
    arms = {}
    for name, prec, learned in (("batched_fp32_learned", 1, True), ("batched_fp32_cold", 1, False),
                                ("batched_fp64_learned", 0, True), ("batched_fp64_cold", 0, False)):
        if learned:
            _, _, st, res, wall, nfb, t_inf = LW.solve_steady_learned(held, model, tol, max_steps, check_every=100,
                                                                      precision=prec)
        else:
            _, _, st, res, wall = LW.solve_steady(held, tol, max_steps, check_every=100, precision=prec)
            nfb = 0
        arms[name] = {"s_per_case": round(wall / len(held), 5), "mean_steps": float(np.mean(st)),
                      "converged": int(np.sum(res < tol)), "fallbacks": int(nfb)}
    plain = float(np.mean(seq_t))
    return {"workload": "held-out sweep cases (first %d of the evaluation set): Nx=64 uniform, Q_x^h<=8 x 4 x 4, "
                        "Kn>=0.05, tol %g" % (len(held), tol),
            "plain_fp64_cold_s_per_case": round(plain, 4), "plain_sample_cases": len(seq_t),
            "plain_mean_steps": float(np.mean(seq_st)), "batched": arms,
            "speedup_batched_fp32_learned_vs_plain": round(plain / arms["batched_fp32_learned"]["s_per_case"], 2)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only; this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import fdlb_inputs as I
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    cfg = I.config(args.workload, precision=0)
    s, ms, nodes, tile, prof = measure(cfg, args.steps, args.warmup, args.retune)
    value = nodes / (ms * 1e-3)
    out = {
        "metric": "node-velocity updates/s",
        "value": round(value, 1),
        "unit": "node-velocity updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "%s Couette: Nx=256 tanh-stretched, 2x8 half-range x 4 x 4 (K=256), Kn=0.1, "
                               "eta0=0.2, walls T=1 at u_y=-/+0.2, Shakhov Pr=2/3, FP64" % args.workload,
                   "nodes": nodes, "tiling": {"kx_per_chunk": tile[0], "waves": tile[1]}},
        "roofline": roofline(prof, nodes, 0, "k_update<double,2>", args.workload),
    }
    if not args.no_extra:
        cfg32 = I.config(args.workload, precision=1)
        _, ms32, _, tile32, prof32 = measure(cfg32, args.steps, args.warmup, args.retune)
        out["fp32_bulk"] = {"value": round(nodes / (ms32 * 1e-3), 1), "ms_per_step": round(ms32, 6),
                            "roofline": roofline(prof32, nodes, 1, "k_update<float,2>", args.workload)}
        for prec in (0, 1):
            cfgL = I.config("R2", precision=prec)
            _, msL, nodesL, tileL, profL = measure(cfgL, args.large_steps, 5, args.retune, graph_steps=10)
            out["large_case_" + ("f64" if prec == 0 else "f32")] = {
                "workload": "Fourier Nx=32768 uniform, 2x16 x 4 x 4 (K=512), %s" % ("FP64" if prec == 0 else "FP32 bulk"),
                "value": round(nodesL / (msL * 1e-3), 1), "ms_per_step": round(msL, 5),
                "tiling": {"kx_per_chunk": tileL[0], "waves": tileL[1]},
                "roofline": roofline(profL, nodesL, prec, "k_update<%s,2>" % ("double" if prec == 0 else "float"), "R2"),
                "kernel_ms": {"table": round(profL[0], 5), "update": [round(x, 5) for x in profL[1 + 3 * prec:4 + 3 * prec]]}}
        out["reduced_1d"] = reduced_leg(args.large_steps, "R2")
        out["reduced_2d"] = reduced_leg(args.steps, "C2", warmup=args.warmup)
        out["sweep"] = sweep_leg(args.sweep_steps, args.retune)
        out["sweep_r1"] = sweep_r1_leg(args.r1_steps, args.retune)
        out["time_to_steady"] = time_to_steady_leg(args.tts_batch, args.tts_seq)
    out["cpu_baseline"] = None if args.no_cpu else cpu_baseline(cfg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
