"""Driver of the learned-warm-start study (data generation, training,
evaluation of time to steady state).

  python -m paper_2308_15407_amd.warmstart_study data  --start 1 --count 2048 --out D.npz
  python -m paper_2308_15407_amd.warmstart_study train --data D1.npz D2.npz --out W.npz
  python -m paper_2308_15407_amd.warmstart_study eval  --weights W.npz --count 512 --out R.json

Cases come from the sweep generator (flow, Kn, eta0, wall data, force) on a
64-cell uniform grid with Q_x^h <= 8 and Q_y = Q_z = 4; draws with R < 2 or
Kn < 0.05 are rejected.  Training seeds start at 1, held-out seeds at 100001.
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
    import torch
    from . import learned as LW
    model = LW.WarmStartModel.load(args.weights)
    held = LW.draw_cases(100001, args.count, kn_min=args.kn_min, nx=args.nx, qx_max=args.qx_max)
    out = {"n_cases": len(held), "tol": args.tol}
    # prediction accuracy against the converged steady states
    t0 = time.perf_counter()
    pred = model.predict(held)
    fields = [LW.warm_fields(c, p) for c, p in zip(held, pred)]
    t_pred = time.perf_counter() - t0
    out["fallback_cold"] = int(sum(f is None for f in fields))
    out["inference_seconds"] = t_pred
    runs = {}
    for name, prec, warm in (("batched_fp32_learned", 1, True), ("batched_fp32_cold", 1, False),
                             ("batched_fp64_cold", 0, False), ("batched_fp64_learned", 0, True)):
        nfb = 0
        if warm:
            moms, grids, st, res, wall, nfb = LW.solve_steady_warm(held, fields, args.tol, args.max_steps,
                                                                   check_every=args.check, precision=prec)
        else:
            moms, grids, st, res, wall = LW.solve_steady(held, args.tol, args.max_steps, check_every=args.check,
                                                         precision=prec)
        runs[name] = dict(wall_s=wall + (t_pred if warm else 0.0), steps_mean=float(np.mean(st)),
                          steps_max=int(np.max(st)), converged=int(np.sum(res < args.tol)), fallbacks=nfb)
        log("%s: %.2f s, mean steps %.0f, converged %d/%d" % (name, runs[name]["wall_s"], np.mean(st),
                                                                runs[name]["converged"], len(held)))
        if name == "batched_fp64_cold":
            ref = moms
            # accuracy of the prediction on the grid
            errs = []
            for c, f, m in zip(held, fields, ref):
                if f is None:
                    continue
                errs.append([np.max(np.abs(f[0] - m[0])) / np.max(m[0]), np.max(np.abs(f[3] - m[3])) / np.max(m[3]),
                             np.max(np.abs(f[2] - m[2])) / max(np.max(np.abs(m[2])), 1e-3)])
            out["prediction_max_rel_err_median"] = dict(zip(("n", "T", "uy"), np.median(np.array(errs), axis=0).tolist()))
    # plain FP64 cold start, one case at a time, on a sample of the held-out cases
    seq = held[:args.seq_count]
    t_seq, st_seq = 0.0, []
    for i, c in enumerate(seq):
        _, _, st, res, wall = LW.solve_steady([c], args.tol, args.max_steps, check_every=args.check, precision=0)
        t_seq += wall
        st_seq.append(int(st[0]))
        log("sequential fp64 cold %d/%d: %.2f s, %d steps" % (i + 1, len(seq), wall, st[0]))
    runs["sequential_fp64_cold_sample"] = dict(n_cases=len(seq), wall_s=t_seq, per_case_s=t_seq / len(seq),
                                               steps_mean=float(np.mean(st_seq)))
    out["runs"] = runs
    out["per_case_seconds"] = {
        "plain_fp64_cold_sequential": t_seq / len(seq),
        "batched_fp32_learned": runs["batched_fp32_learned"]["wall_s"] / len(held),
        "batched_fp32_cold": runs["batched_fp32_cold"]["wall_s"] / len(held),
        "batched_fp64_cold": runs["batched_fp64_cold"]["wall_s"] / len(held)}
    out["speedup_vs_plain_fp64_cold"] = out["per_case_seconds"]["plain_fp64_cold_sequential"] / \
        out["per_case_seconds"]["batched_fp32_learned"]
    json.dump(out, open(args.out, "w"), indent=1)
    log(json.dumps(out))


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
            p.add_argument("--seq-count", type=int, default=16)
            p.add_argument("--check", type=int, default=100)
    args = ap.parse_args(argv)
    {"data": cmd_data, "train": cmd_train, "eval": cmd_eval}[args.cmd](args)


if __name__ == "__main__":
    main()
