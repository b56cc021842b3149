"""Benchmark: node-velocity updates per second of the FDLB time step on one MI355X.

Workload (default): the plain force-driven Poiseuille configuration, the
largest single-GPU case -- Nx = 512 wall-refined cells, 2x16 half-range x 6 x 4
full-range velocities (K = 768), Kn = 0.05, eta0 = 0.3, a_y = 0.05, walls T = 1
at rest, Shakhov with the dense Prandtl number, FP64.  One step = one TVD-RK3
step (three stages of table + update launches) of the whole case; inputs are
resident in device memory before timing starts.

Also reported: the FP32-bulk variant of the same case, the Couette case (Nx =
256, K = 256), a large single case (Nx = 32768, K = 512) that sizes the
memory-bound roofline, the sweeps, the reduced models, time to steady state,
the roofline object for the dominant kernel (its time measured by HIP events
on the solver's stream), and the CPU oracle timed on this host's cores.

--profile-case WORKLOAD runs a short fixed run for profilers instead (no JSON
line): one untimed step, --steps steps, then a plain device copy of --copy-mib
MiB that calibrates memory-traffic counters.
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
BF16_MFMA_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix peak


WORKLOADS = {
    "C1": "C1 Fourier: Nx=64 uniform, 2x4 half-range x 3 x 3 (K=72), Kn=0.1, eta0=0.05, walls T=1.0/1.1 at rest, "
          "BGK + J1",
    "C2": "C2 Couette: Nx=256 tanh-stretched, 2x8 half-range x 4 x 4 (K=256), Kn=0.1, eta0=0.2, walls T=1 at "
          "u_y=-/+0.2, Shakhov Pr=2/3",
    "C3": "C3 Poiseuille: Nx=512 tanh-stretched, 2x16 half-range x 6 x 4 (K=768), Kn=0.05, eta0=0.3, a_y=0.05, "
          "walls T=1 at rest, Shakhov dense Pr",
    "R2": "R2 Fourier: Nx=32768 uniform, 2x16 half-range x 4 x 4 (K=512), Kn=0.1, eta0=0.05, walls T=1.0/1.1, BGK + J1",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="C3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="only the main workload")
    ap.add_argument("--no-pmc", action="store_true", help="skip the counter passes of the headline kernel")
    ap.add_argument("--large-steps", type=int, default=60)
    ap.add_argument("--retune", action="store_true")
    ap.add_argument("--sweep-steps", type=int, default=100)
    ap.add_argument("--r1-steps", type=int, default=20)
    ap.add_argument("--tts-cases", type=int, default=16,
                    help="held-out cases of the time-to-steady leg (every arm solves the same cases)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the all-cores oracle sample")
    # profiler mode
    ap.add_argument("--profile-case", default=None, help="short fixed run of a workload (R2, C2, C3, sweep, sweep1024, mlp)")
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--tiling", type=int, nargs=2, default=None, metavar=("KX_PER_CHUNK", "WAVES"))
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--reduced", action="store_true", help="profile the reduced 1D/2D form of the workload")
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


def measure_traffic(workload, prec, tile, timeout_s=150):
    """HBM bytes per launch of the stage-2 update, measured in this run: two
    rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) over
    a short child run of the same workload and tiling, each scaled by what the
    same counter reads for a 256 MiB device copy in that child run.  Returns
    (bytes, detail) or (None, reason) when the profiler is not usable here."""
    import glob
    import shutil
    import sqlite3
    import subprocess
    import tempfile
    kname = "k_update<%s, 2," % ("double" if prec == 0 else "float")
    per = {}
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        d = tempfile.mkdtemp(prefix="fdlb_pmc_", dir="/tmp")
        try:
            cmd = ["timeout", "-s", "KILL", str(timeout_s), "rocprofv3", "--pmc", counter, "-d", d, "-o", "pmc", "--",
                   sys.executable, os.path.join(ROOT, "bench.py"), "--profile-case", workload, "--precision",
                   str(prec), "--steps", "3", "--tiling", str(tile[0]), str(tile[1]), "--copy-mib", "256"]
            env = dict(os.environ, TMPDIR="/tmp")
            r = subprocess.run(cmd, cwd=ROOT, env=env, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
            # the profiler can exit non-zero after a complete run; the samples decide
            dbs = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
            if not dbs:
                return None, "rocprofv3 --pmc %s: exit %d, no result file" % (counter, r.returncode)
            vals = {"k": [], "copy": []}
            con = sqlite3.connect(dbs[0])
            for n, cn, v in con.execute("select kernel_name, counter_name, value from counters_collection"):
                if cn != counter:
                    continue
                if kname in n:
                    vals["k"].append(v)
                elif "k_copy_probe" in n:
                    vals["copy"].append(v)
            con.close()
            if not vals["k"] or not vals["copy"]:
                return None, "rocprofv3 --pmc %s: exit %d, no samples for the update or the copy" % (counter,
                                                                                                  r.returncode)
            kib = sum(vals["k"]) / len(vals["k"])
            factor = 262144.0 / (sum(vals["copy"]) / len(vals["copy"]))
            per[counter] = {"kib_per_dispatch": round(kib, 1), "copy_factor": round(factor, 4),
                            "bytes": round(kib * factor * 1024)}
        except (OSError, sqlite3.Error) as e:
            return None, "rocprofv3 --pmc %s: %s" % (counter, e)
        finally:
            shutil.rmtree(d, ignore_errors=True)
    return per["FETCH_SIZE"]["bytes"] + per["WRITE_SIZE"]["bytes"], per


def attach_traffic(roof, workload, prec, tile):
    """Replace a roofline object's traffic by the counters of measure_traffic
    (this run); the committed profile's value stands if the profiler fails."""
    t, detail = measure_traffic(workload, prec, tile)
    if t is not None:
        roof["traffic"] = t
        roof["traffic_source"] = "rocprofv3 --pmc FETCH_SIZE, WRITE_SIZE in this run, copy-calibrated"
        roof["traffic_counters"] = detail
    else:
        roof["traffic_source"] = ("committed profile (%s)" % detail) if roof["traffic"] is not None else detail


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


def update_roofline(prof, nodes, prec, workload):
    """The stage-2 update (reads f^(1) and f^n, writes f^(2)): 3 passes x bytes
    per population x nodes, algorithmic, over its mean launch time."""
    s_bytes = 8 if prec == 0 else 4
    t_ms = prof[2] if prec == 0 else prof[5]
    kernel = "k_update<%s,2>" % ("double" if prec == 0 else "float")
    alg = 3.0 * s_bytes * nodes
    achieved = alg / (t_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": read_traffic(kernel, workload),
            "kernel": kernel, "launch_ms": round(t_ms, 5), "algorithmic_bytes_per_launch": alg}


def table_roofline(prof, cases, prec, workload, chunks):
    """The table pass (per cell: moments from the chunk partials, closure,
    gradients, projection tables): it reads 9 FP64 raw sums per cell and chunk
    and writes 4 (2 Q_x^h + Q_y Q_z) table values plus 1/tau per cell."""
    s_bytes = 8 if prec == 0 else 4
    alg = 0.0
    for c, nch in zip(cases, chunks):
        alg += 8.0 * 9 * nch * c["nx"] + s_bytes * (4 * (2 * c["qx_half"] + c["qy"] * c["qz"]) + 1) * c["nx"]
    t_ms = prof[0]
    achieved = alg / (t_ms * 1e-3) / 1e9
    kernel = "k_table<%s>" % ("double" if prec == 0 else "float")
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": read_traffic(kernel, workload),
            "kernel": kernel, "launch_ms": round(t_ms, 5), "algorithmic_bytes_per_launch": alg}


def dominant_roofline(tile, prof, cfg, nodes, prec, workload):
    """Roofline object of the kernel that takes the largest share of a step:
    the stage-2 update or the table pass (three launches per step each)."""
    upd = update_roofline(prof, nodes, prec, workload)
    cases = cfg if isinstance(cfg, list) else [cfg]
    kxc = tile[0]
    chunks = [-(-2 * c["qx_half"] // min(kxc, 2 * c["qx_half"])) for c in cases]
    tab = table_roofline(prof, cases, prec, workload, chunks)
    up_ms = sum(prof[1 + 3 * prec:4 + 3 * prec])
    table_dominant = 3 * prof[0] > up_ms
    dom, other = (tab, upd) if table_dominant else (upd, tab)
    dom = dict(dom)
    dom["share_of_kernel_time"] = round((3 * prof[0] if table_dominant else up_ms) / (3 * prof[0] + up_ms), 3)
    dom["other_kernel"] = other
    return dom


def cpu_baseline(cfg, budget_s=12.0, single_s=4.0):
    """The FP64 oracle on this host: all cores (OpenMP over cells and
    velocities), then one thread, each on a bounded number of steps of the
    same case."""
    from oracle import oracle as O
    L = O.lib()
    cores = L.orc_threads()
    res = {}
    for label, threads, budget in (("all", cores, budget_s), ("one", 1, single_s)):
        L.orc_set_threads(threads)
        o = O.Oracle(**{k: v for k, v in cfg.items() if k != "precision"})
        t0 = time.perf_counter()
        o.step(1)
        one = time.perf_counter() - t0
        n = max(1, min(2000, int(budget / max(one, 1e-6))))
        t0 = time.perf_counter()
        o.step(n)
        dt = time.perf_counter() - t0
        res[label] = (cfg["nx"] * o.K * n / dt, n, dt)
    L.orc_set_threads(cores)
    v, n, dt = res["all"]
    v1, n1, dt1 = res["one"]
    return {"value": round(v, 1), "unit": "node-velocity updates/s", "cores": cores, "kind": "oracle",
            "sample": "%d RK3 steps of the same case (Nx=%d, K=%d) on %d host threads, %.1f s" %
                      (n, cfg["nx"], 2 * cfg["qx_half"] * cfg["qy"] * cfg["qz"], cores, dt),
            "single_thread": {"value": round(v1, 1), "sample": "%d steps on one thread, %.1f s" % (n1, dt1)}}


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


def mlp_flops_per_step(batch, n_in=10, width=256, depth=4, n_out=640):
    """GEMM flops of one training step of the warm-start network: per layer the
    forward product and the weight gradient, and the input gradient of every
    layer but the first (2 flops per multiply-add)."""
    dims = [n_in] + [width] * depth + [n_out]
    f = 0
    for l in range(len(dims) - 1):
        mac = batch * dims[l] * dims[l + 1]
        f += 2 * mac * (3 if l > 0 else 2)
    return f


def mlp_leg(steps=50, batch=4096, gemm_n=4096, gemm_reps=5):
    """The warm-start network's training step at its full shape (10 -> 4 x 256
    GELU -> 640, BF16 on MFMA with FP32 accumulation, AdamW), batch 4096: its
    GEMM flops over the step time against the dense BF16 MFMA peak; and the
    library's BF16 GEMM kernel alone on a square product of edge gemm_n."""
    import time
    import torch
    from paper_2308_15407_amd import fdlb as F
    from paper_2308_15407_amd.mlp import WarmStartNet
    net = WarmStartNet(n_in=10, width=256, depth=4, n_out=640, max_batch=batch)
    g = torch.Generator(device="cuda")
    g.manual_seed(20230829)
    x = torch.randn(batch, 10, device="cuda", generator=g)
    t = torch.randn(batch, 640, device="cuda", generator=g)
    for _ in range(5):
        net.train_step(x, t, 1e-4)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(net.stream)
    for _ in range(steps):
        net.train_step(x, t, 1e-4)
    b.record(net.stream)
    b.synchronize()
    ms = a.elapsed_time(b) / steps
    flops = mlp_flops_per_step(batch)
    net.close()
    # the GEMM kernel alone (each call synchronises; wall clock over gemm_reps calls)
    n = gemm_n
    A = torch.randn(n, n, device="cuda", generator=g).to(torch.bfloat16)
    B = torch.randn(n, n, device="cuda", generator=g).to(torch.bfloat16)
    Cm = torch.empty(n, n, device="cuda", dtype=torch.float32)
    st = torch.cuda.current_stream().cuda_stream
    F.fdlb_mlp_gemm_bf16(A.data_ptr(), B.data_ptr(), Cm.data_ptr(), n, n, n, n, 1, n, 1, n, st)
    t0 = time.perf_counter()
    for _ in range(gemm_reps):
        F.fdlb_mlp_gemm_bf16(A.data_ptr(), B.data_ptr(), Cm.data_ptr(), n, n, n, n, 1, n, 1, n, st)
    gms = (time.perf_counter() - t0) / gemm_reps * 1e3
    step_tf = flops / (ms * 1e-3) / 1e12
    gemm_tf = 2.0 * n ** 3 / (gms * 1e-3) / 1e12
    return {"workload": "warm-start MLP 10 -> 4 x 256 GELU -> 640, BF16 MFMA, batch %d, one AdamW training step"
                        % batch,
            "ms_per_step": round(ms, 5), "gemm_flops_per_step": flops,
            "roofline": {"bound": "mfma", "achieved": round(step_tf, 2), "peak": BF16_MFMA_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(step_tf / BF16_MFMA_PEAK_TFLOPS, 5)},
            "gemm_kernel": {"shape": "%d^3" % n, "ms": round(gms, 4), "achieved": round(gemm_tf, 1),
                            "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": round(gemm_tf / BF16_MFMA_PEAK_TFLOPS, 4)}}


def time_to_steady_leg(n_cases, tol=1e-8, max_steps=400000):
    """Wall-clock time to r < tol per case on one sample of held-out cases:
    plain FP64 cold start (one case at a time) against the batched arms (all
    the sample's cases in one batch, FP32 bulk or FP64, cold or learned warm
    start with inference included)."""
    import numpy as np
    from paper_2308_15407_amd import learned as LW
    path = LW.default_weights_path()
    if not os.path.exists(path):
        return {"skipped": "no trained warm-start weights in the package"}
    model = LW.WarmStartModel.load(path)
    evp = LW.default_eval_path()
    if not os.path.exists(evp):
        return {"skipped": "no held-out evaluation summary next to the weights"}
    ev = json.load(open(evp))
    held = LW.cases_from_seeds(ev["seeds"][:n_cases])
    seq_t, seq_st = [], []
    for c in held:
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
    return {"workload": "the first %d held-out cases of the warm-start evaluation set (%s), tol %g; every arm "
                        "solves these same cases" % (len(held), ev.get("generator", "C4 generator"), tol),
            "plain_fp64_cold_s_per_case": round(plain, 4), "plain_mean_steps": float(np.mean(seq_st)),
            "batched": arms,
            "speedup_batched_fp32_learned_vs_plain": round(plain / arms["batched_fp32_learned"]["s_per_case"], 2),
            "speedup_learned_vs_cold_batched_fp32": round(arms["batched_fp32_cold"]["s_per_case"] /
                                                          arms["batched_fp32_learned"]["s_per_case"], 3)}


def profile_case(a):
    """Short fixed run of one workload for rocprofv3 (kernel traces, counters)."""
    import torch
    import fdlb_inputs as I
    from paper_2308_15407_amd import fdlb as F
    from paper_2308_15407_amd.solver import ReducedSolver, Solver
    if a.profile_case == "mlp":
        print(json.dumps(mlp_leg(steps=a.steps, gemm_reps=3)), flush=True)
        return
    if a.reduced:
        s = ReducedSolver(I.config(a.profile_case, precision=0))
    else:
        if a.profile_case in ("sweep", "sweep1024"):
            from paper_2308_15407_amd import sweep
            cfg = sweep.sweep_cases(1024 if a.profile_case == "sweep1024" else 256, precision=a.precision)
        else:
            cfg = I.config(a.profile_case, precision=a.precision)
        s = Solver(cfg)
        if a.tiling:
            s.set_tiling(*a.tiling)
        else:
            from paper_2308_15407_amd import autotune
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
    print("profile case done: %s%s precision %d, %d steps" % (a.profile_case, " reduced" if a.reduced else "",
                                                              a.precision, a.steps), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only; this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import fdlb_inputs as I
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.profile_case:
        profile_case(args)
        return
    wl = args.workload
    cfg = I.config(wl, precision=0)
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
        "config": {"workload": WORKLOADS[wl] + ", FP64", "nodes": nodes,
                   "tiling": {"kx_per_chunk": tile[0], "waves": tile[1]}},
        "roofline": dominant_roofline(tile, prof, cfg, nodes, 0, wl),
        "kernel_ms": {"table": round(prof[0], 5), "update": [round(x, 5) for x in prof[1:4]]},
    }
    del s
    torch.cuda.synchronize()
    if not args.no_pmc:
        # the headline kernel's HBM traffic from counters taken in this run (the
        # committed profile's value stands only if the profiler is unusable)
        upd = out["roofline"] if out["roofline"]["kernel"].startswith("k_update") else out["roofline"]["other_kernel"]
        attach_traffic(upd, wl, 0, tile)
    if not args.no_extra:
        cfg32 = I.config(wl, precision=1)
        s32, ms32, _, tile32, prof32 = measure(cfg32, args.steps, args.warmup, args.retune)
        del s32
        out["fp32_bulk"] = {"workload": WORKLOADS[wl] + ", FP32 bulk with FP64 reductions",
                            "value": round(nodes / (ms32 * 1e-3), 1), "ms_per_step": round(ms32, 6),
                            "tiling": {"kx_per_chunk": tile32[0], "waves": tile32[1]},
                            "roofline": dominant_roofline(tile32, prof32, cfg32, nodes, 1, wl),
                            "kernel_ms": {"table": round(prof32[0], 5), "update": [round(x, 5) for x in prof32[4:7]]}}
        other = "C2" if wl != "C2" else "C3"
        for prec in (0, 1):
            cfgO = I.config(other, precision=prec)
            sO, msO, nodesO, tileO, profO = measure(cfgO, args.steps, args.warmup, args.retune)
            del sO
            out["%s_%s" % (other, "f64" if prec == 0 else "f32")] = {
                "workload": WORKLOADS[other] + (", FP64" if prec == 0 else ", FP32 bulk"),
                "value": round(nodesO / (msO * 1e-3), 1), "ms_per_step": round(msO, 6),
                "roofline": dominant_roofline(tileO, profO, cfgO, nodesO, prec, other)}
        for prec in (0, 1):
            cfgL = I.config("R2", precision=prec)
            sL, msL, nodesL, tileL, profL = measure(cfgL, args.large_steps, 5, args.retune, graph_steps=10)
            del sL
            out["large_case_" + ("f64" if prec == 0 else "f32")] = {
                "workload": WORKLOADS["R2"] + (", FP64" if prec == 0 else ", FP32 bulk"),
                "value": round(nodesL / (msL * 1e-3), 1), "ms_per_step": round(msL, 5),
                "effective_GBps_whole_step": round(8 * (8 if prec == 0 else 4) * nodesL / (msL * 1e-3) / 1e9, 1),
                "tiling": {"kx_per_chunk": tileL[0], "waves": tileL[1]},
                "roofline": update_roofline(profL, nodesL, prec, "R2"),
                "kernel_ms": {"table": round(profL[0], 5), "update": [round(x, 5) for x in profL[1 + 3 * prec:4 + 3 * prec]]}}
            if not args.no_pmc:
                torch.cuda.synchronize()
                attach_traffic(out["large_case_" + ("f64" if prec == 0 else "f32")]["roofline"], "R2", prec, tileL)
        out["reduced_1d"] = reduced_leg(args.large_steps, "R2")
        out["reduced_2d"] = reduced_leg(args.steps, "C2", warmup=args.warmup)
        out["sweep"] = sweep_leg(args.sweep_steps, args.retune)
        out["sweep_r1"] = sweep_r1_leg(args.r1_steps, args.retune)
        out["time_to_steady"] = time_to_steady_leg(args.tts_cases)
        out["mlp"] = mlp_leg()
    out["cpu_baseline"] = None if args.no_cpu else cpu_baseline(cfg, budget_s=args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
