"""In-project autotuner for the update launch shape.

Chooses, for a solver's batch, the velocity chunk (kx values per block, i.e.
how many y-lines of velocities each block covers) and the waves per update
block, by timing graph-replayed trial steps on the device.  Decisions are
cached in a JSON file keyed by the batch shape.
"""
import json
import os

import torch

# decisions cache (FDLB_TUNING_CACHE overrides the location)
CACHE = os.environ.get("FDLB_TUNING_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json"))


def _key(solver):
    shapes = sorted({(c["nx"], c["qx_half"], c["qy"], c["qz"], c.get("precision", 0)) for c in solver.cases})
    return "n%d:" % solver.ncases + ";".join("%d-%d-%d-%d-%d" % s for s in shapes[:8]) + (
        ";+%d" % (len(shapes) - 8) if len(shapes) > 8 else "")


def candidates(solver):
    qh_max = max(c["qx_half"] for c in solver.cases)
    out = []
    for waves in (1, 2, 4, 8):
        for kxc in (1, 2, 4, 8, 16, 32):
            if kxc <= 2 * qh_max:
                out.append((kxc, waves))
    return out


def time_steps(solver, nsteps):
    stream = solver.stream
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    solver.step(nsteps)               # warm (and capture the graph)
    a.record(stream)
    solver.step(nsteps)
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / nsteps


def tune(solver, trial_steps=20, use_cache=True, verbose=False, refresh=False):
    """Pick and apply the fastest (kx_per_chunk, waves); returns it.  With
    use_cache a cached decision is reused and a new one is stored; refresh
    times the candidates again and overwrites the cached decision."""
    key = _key(solver)
    cache = {}
    if use_cache and os.path.exists(CACHE):
        try:
            cache = json.load(open(CACHE))
        except ValueError:
            cache = {}
    if use_cache and not refresh and key in cache:
        kxc, waves = cache[key]
        solver.set_tiling(kxc, waves)
        return kxc, waves
    solver.set_graph_steps(trial_steps)
    best = None
    for kxc, waves in candidates(solver):
        solver.set_tiling(kxc, waves)
        ms = time_steps(solver, trial_steps)
        if verbose:
            print("  tile kx/chunk=%d waves=%d: %.4f ms/step" % (kxc, waves, ms), flush=True)
        if best is None or ms < best[0]:
            best = (ms, kxc, waves)
    _, kxc, waves = best
    solver.set_tiling(kxc, waves)
    if use_cache:
        cache[key] = [kxc, waves]
        try:
            json.dump(cache, open(CACHE, "w"), indent=1, sort_keys=True)
        except OSError:
            pass
    return kxc, waves
