"""Driver of the learned-warm-start study (data generation, training,
evaluation of time to steady state).

  python -m paper_2308_15407_amd.warmstart_study data  --start 1 --count 2048 --out D.npz
  python -m paper_2308_15407_amd.warmstart_study train --data D1.npz D2.npz --out W.npz
  python -m paper_2308_15407_amd.warmstart_study eval  --weights W.npz --count 512 --out R.json

Cases come from the sweep generator (flow, Kn, eta0, wall data, force) on a
64-cell uniform grid with Q_x^h <= 8 and Q_y = Q_z = 4; draws with R < 2 or
Kn < 0.05 are rejected.  Training seeds start at 1, held-out seeds at 100001.
--nx 0 --qx-max 0 keeps the generator's own grids and orders (Nx 64-512,
Q_x^h 4-16); --kn-min 0.01 its whole Knudsen range.
"""
import argparse
import json
import sys
import time

import numpy as np


def log(*a):
    print(*a, flush=True)


def cmd_data(args):
    from . import learned as LW
    cases = LW.draw_cases(args.start, args.count, kn_min=args.kn_min, nx=args.nx, qx_max=args.qx_max)
    X, Y, kept = [], [], []
    for b0 in range(0, len(cases), args.batch):
        Xb, Yb, kb = LW.build_dataset(cases[b0:b0 + args.batch], tol=args.tol, max_steps=args.max_steps,
                                      batch=args.batch, log=log)
        X.append(Xb); Y.append(Yb)
        ks = set(c["_seed"] for c in kb)
        drop = [c["_seed"] for c in cases[b0:b0 + args.batch] if c["_seed"] not in ks]
        if drop:
            log("data: dropped seeds (diverged or unconverged):", drop)
        kept += kb
        log("data: %d / %d cases kept" % (len(kept), b0 + len(cases[b0:b0 + args.batch])))
    np.savez(args.out, X=np.concatenate(X), Y=np.concatenate(Y), seeds=np.array([c["_seed"] for c in kept]))


def cmd_train(args):
    from . import learned as LW
    Xs, Ys = [], []
    for f in args.data:
        z = np.load(f)
        Xs.append(z["X"]); Ys.append(z["Y"])
    X, Y = np.concatenate(Xs), np.concatenate(Ys)
    log("training on %d steady states" % len(X))
    model = LW.WarmStartModel().fit(X, Y, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    model.save(args.out)
    log("train seconds %.1f" % model.train_seconds)


def cmd_eval(args):
    """Time to steady state on held-out cases.  The evaluation set is the
    held-out draws that the plain FP64 cold solve brings below tol within
    max_steps (run batched to find them); every arm is then timed on that set."""
    import torch
    from . import learned as LW
    model = LW.WarmStartModel.load(args.weights)
    held = LW.draw_cases(100001, args.count, kn_min=args.kn_min, nx=args.nx, qx_max=args.qx_max)
    out = {"n_drawn": len(held), "tol": args.tol, "max_steps": args.max_steps, "kn_min": args.kn_min,
           "generator": "sweep generator, %s, %s, Kn >= %g, R >= 2" % (
               "its own grids (Nx 64-512)" if not args.nx else "Nx = %d uniform" % args.nx,
               "Q_x^h 4-16" if not args.qx_max else "Q_x^h <= %d" % args.qx_max, args.kn_min)}
    moms, grids, st, res, wall = LW.solve_steady(held, args.tol, args.max_steps, check_every=args.check, precision=0)
    ok = [i for i in range(len(held)) if res[i] < args.tol]
    out["not_converged_plain_seeds"] = [held[i]["_seed"] for i in range(len(held)) if not (res[i] < args.tol)]
    cases = [held[i] for i in ok]
    ref = [moms[i] for i in ok]
    out["n_cases"] = len(cases)
    out["seeds"] = [c["_seed"] for c in cases]
    log("evaluation set: %d of %d held-out cases converge under the plain FP64 solve" % (len(cases), len(held)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = model.predict(cases)
    fields = [LW.warm_fields(c, p) for c, p in zip(cases, pred)]
    t_pred = time.perf_counter() - t0
    out["inference_seconds"] = t_pred
    out["nonphysical_predictions"] = int(sum(f is None for f in fields))
    errs = []
    for f, m in zip(fields, ref):
        if f is not None:
            errs.append([np.max(np.abs(f[0] - m[0]) / m[0]), np.max(np.abs(f[3] - m[3]) / m[3]),
                         np.max(np.abs(f[2] - m[2])) / max(np.max(np.abs(m[2])), 1e-3)])
    e = np.array(errs)
    out["prediction_max_rel_err"] = {k: {"median": float(np.median(e[:, j])), "p90": float(np.percentile(e[:, j], 90))}
                                     for j, k in enumerate(("n", "T", "uy"))}
    runs, steps = {}, {}
    arms = (("batched_fp64_cold", 0, None), ("batched_fp32_cold", 1, None),
            ("batched_fp32_learned", 1, True), ("batched_fp64_learned", 0, True),
            ("batched_fp32_learned_maxwellian", 1, False), ("batched_fp64_learned_maxwellian", 0, False))
    if args.short:
        arms = arms[:4]
    for name, prec, g13 in arms:
        nfb = 0
        if g13 is not None:
            _, _, st, res, wall, nfb, t_inf = LW.solve_steady_learned(cases, model, args.tol, args.max_steps,
                                                                      check_every=args.check, precision=prec,
                                                                      grad13=g13)
            log("  %s inference %.3f s" % (name, t_inf))
        else:
            _, _, st, res, wall = LW.solve_steady(cases, args.tol, args.max_steps, check_every=args.check,
                                                  precision=prec)
        steps[name] = st
        runs[name] = dict(wall_s=wall, s_per_case=wall / len(cases), steps_mean=float(np.mean(st)),
                          steps_median=float(np.median(st)), steps_max=int(np.max(st)),
                          converged=int(np.sum(res < args.tol)), fallbacks=nfb)
        log("%s: %.2f s (%.4f s/case), steps mean %.0f median %.0f max %d, converged %d/%d, fallbacks %d"
            % (name, wall, wall / len(cases), np.mean(st), np.median(st), np.max(st), runs[name]["converged"],
               len(cases), nfb))
    for p in ("fp32", "fp64"):
        for v in ("", "_maxwellian") if not args.short else ("",):
            r = steps["batched_%s_learned%s" % (p, v)] / np.maximum(steps["batched_%s_cold" % p], 1)
            runs["step_ratio_learned%s_over_cold_%s" % (v, p)] = {"mean": float(np.mean(r)),
                                                                   "median": float(np.median(r))}
    # the plain method: FP64 cold start, one case at a time (a sample of the set)
    rng = np.random.default_rng(7)
    pick = sorted(rng.choice(len(cases), size=min(args.seq_count, len(cases)), replace=False).tolist())
    t_seq, st_seq = [], []
    for k, i in enumerate(pick):
        _, _, st, res, wall = LW.solve_steady([cases[i]], args.tol, args.max_steps, check_every=args.check, precision=0)
        t_seq.append(wall)
        st_seq.append(int(st[0]))
        log("plain FP64 cold, one case %d/%d: %.2f s, %d steps" % (k + 1, len(pick), wall, st[0]))
    runs["plain_fp64_cold_sequential"] = dict(n_cases=len(pick), s_per_case=float(np.mean(t_seq)),
                                              steps_mean=float(np.mean(st_seq)))
    out["runs"] = runs
    plain = float(np.mean(t_seq))
    out["speedup_vs_plain_fp64_cold"] = {k: plain / runs[k]["s_per_case"] for k, _, _ in arms}
    json.dump(out, open(args.out, "w"), indent=1)
    log(json.dumps({k: v for k, v in out.items() if k not in ("seeds", "not_converged_plain_seeds")}))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    for name in ("data", "train", "eval"):
        p = sub.add_parser(name)
        p.add_argument("--out", required=True)
        p.add_argument("--kn-min", type=float, default=0.05)
        p.add_argument("--nx", type=int, default=64)
        p.add_argument("--qx-max", type=int, default=8)
        p.add_argument("--tol", type=float, default=1e-6 if name == "data" else 1e-8)
        p.add_argument("--max-steps", type=int, default=400000)
        p.add_argument("--batch", type=int, default=256)
        if name == "data":
            p.add_argument("--start", type=int, default=1)
            p.add_argument("--count", type=int, default=2048)
        if name == "train":
            p.add_argument("--data", nargs="+", required=True)
            p.add_argument("--epochs", type=int, default=1500)
            p.add_argument("--lr", type=float, default=1e-3)
        if name == "eval":
            p.add_argument("--weights", required=True)
            p.add_argument("--count", type=int, default=512)
            p.add_argument("--seq-count", type=int, default=24)
            p.add_argument("--check", type=int, default=100)
            p.add_argument("--short", action="store_true", help="only the Grad-13 learned and cold arms")
    args = ap.parse_args(argv)
    {"data": cmd_data, "train": cmd_train, "eval": cmd_eval}[args.cmd](args)


if __name__ == "__main__":
    main()
