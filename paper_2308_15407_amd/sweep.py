"""Parameter-sweep batches: seeded cases from the sweep generator, filtered
by the library's own validation (confinement ratio R >= r_min)."""
import fdlb_inputs as I

from . import fdlb as F

SWEEP_SEED = 20230829


def accepted(case, r_min=2.0):
    try:
        return F.fdlb_case_info(case)["R"] >= r_min
    except F.FdlbError:
        return False


def sweep_cases(n=256, seed=SWEEP_SEED, r_min=2.0, precision=1):
    """The first n accepted draws of PCG64(seed) (draws with R < r_min are
    skipped), as case dicts with the given storage precision."""
    out, k = [], 0
    while len(out) < n:
        draws = I.c4_draws(seed, 4 * n + k)
        for d in draws[k:]:
            c = dict(I.c4_params(d), precision=precision)
            if accepted(c, r_min):
                out.append(c)
                if len(out) == n:
                    break
        k = len(draws)
    return out
