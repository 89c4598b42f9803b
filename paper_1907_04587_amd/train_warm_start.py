"""Train and evaluate the learned contact warm start.

    python -m paper_1907_04587_amd.train_warm_start --dist grasp --out weights/warm_start_grasp

1. Dataset: a batch of seeded scenes of the chosen distribution is stepped by the
   plain solver (previous-step warm start, tight tolerance 1e-6, at most 50 Newton x
   40 PCR iterations).  Every contact of every step contributes its 12 step-start
   features and its final multipliers (lambda_n, lambda_f1, lambda_f2).
2. Training: the 12 -> 64 -> 64 -> 64 -> 3 MLP with the library's BF16-MFMA forward /
   backward kernels and its Adam kernel, inputs and targets z-scored.
3. Evaluation on held-out seeds (disjoint from the training and validation seeds):
   the ZERO, PREV, LEARNED and HYBRID (previous-step multipliers for persisting
   contacts, the network for new ones) starts step identical initial states in residual mode
   (r_ncp <= 1e-4, at most 50 Newton x 40 PCR); reported per arm: mean Newton and PCR
   iterations, converged fraction, start residual, final residual, contact residual.

Writes <out>.npy (the weights blob) and <out>.json (dataset size, losses, evaluation).
Distributions: "grasp" (4-finger capsule hand on a 6-DoF arm squeezing an FEM sphere,
h = 1/120) and "batched" (the uneven box / joint / tet-block envs, h = 1/60).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def _envs(dist, seeds):
    import scene_inputs as si
    if dist == "grasp":
        return [si.grasp_scene(seed=int(s), sphere_cell=0.02) for s in seeds]
    return [si.batched_env(seed=int(s), tets_max=3000) for s in seeds]


def _h(dist):
    return 1.0 / 120.0 if dist == "grasp" else 1.0 / 60.0


def evaluate(dist, blob, seeds, steps, warmup, log=print):
    """Step identical held-out scenes with each warm start; per-arm statistics."""
    import scene_inputs as si
    from .scene import Scene

    envs = _envs(dist, seeds)
    h = _h(dist)
    out = {}
    for arm, mode in [("zero", si.WARM_ZERO), ("prev", si.WARM_PREV), ("learned", si.WARM_LEARNED),
                      ("hybrid", si.WARM_HYBRID)]:
        sc = Scene(envs, si.SolverParams(warm=mode))
        if mode in (si.WARM_LEARNED, si.WARM_HYBRID):
            sc.set_warm_start_model(blob)
        for _ in range(warmup):
            sc.step(h, 50, 40, 1e-4)
        sc.reset_accumulators()
        r_first, r_fin, r_con = [], [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            sc.step(h, 50, 40, 1e-4)
            st = sc.stats()
            r_first.append(st["r_ncp_first"].copy())
            r_fin.append(st["r_ncp"].copy())
            r_con.append(st["r_contact"].copy())
        sc.synchronize()
        wall = time.perf_counter() - t0
        acc = sc.accumulators()
        n = max(int(acc["steps"].sum()), 1)
        out[arm] = {
            "env_steps_per_s": n / wall,
            "mean_newton_iters": float(acc["newton_iters"].sum()) / n,
            "mean_cr_iters": float(acc["cr_iters"].sum()) / n,
            "converged_frac": float(acc["converged"].sum()) / n,
            "nonfinite_steps": int(acc["nonfinite"].sum()),
            "median_r_first": float(np.median(np.concatenate(r_first))),
            "median_r_final": float(np.median(np.concatenate(r_fin))),
            "median_r_contact": float(np.median(np.concatenate(r_con))),
        }
        log(f"eval {arm}: {out[arm]}")
        del sc
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dist", choices=["grasp", "batched"], default="grasp")
    ap.add_argument("--out", default=None)
    ap.add_argument("--train-envs", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-envs", type=int, default=256)
    ap.add_argument("--eval-steps", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)

    from .warmstart import generate_dataset, predict, train_mlp

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    # disjoint seed ranges: train [base, base + n), validation and test above
    base = 10_000 if args.dist == "grasp" else 20_000
    train_seeds = np.arange(base, base + args.train_envs)
    val_seeds = np.arange(base + 100_000, base + 100_000 + max(args.train_envs // 8, 16))
    test_seeds = np.arange(base + 200_000, base + 200_000 + args.eval_envs)
    h = _h(args.dist)

    t0 = time.perf_counter()
    x, t = generate_dataset(_envs(args.dist, train_seeds), args.steps, h, warmup=args.warmup, log=log)
    xv, tv = generate_dataset(_envs(args.dist, val_seeds), max(args.steps // 2, 4), h, warmup=args.warmup, log=log)
    t_data = time.perf_counter() - t0
    log(f"dataset: {len(x)} training / {len(xv)} validation contacts in {t_data:.1f}s")

    t0 = time.perf_counter()
    blob, hist = train_mlp(x, t, epochs=args.epochs, batch=args.batch, lr=args.lr, seed=args.seed, log=log)
    t_train = time.perf_counter() - t0
    pv = predict(blob, xv)
    ss_res = ((pv - tv) ** 2).sum(0)
    ss_tot = ((tv - tv.mean(0)) ** 2).sum(0)
    r2 = (1.0 - ss_res / np.maximum(ss_tot, 1e-30)).tolist()
    # the previous-step multipliers (features 4..6) as a predictor, for comparison
    ss_prev = ((xv[:, 4:7] - tv) ** 2).sum(0)
    r2_prev = (1.0 - ss_prev / np.maximum(ss_tot, 1e-30)).tolist()
    log(f"validation R^2 learned {r2}, previous-step {r2_prev}")

    ev = evaluate(args.dist, blob, test_seeds, args.eval_steps, args.warmup, log=log)
    report = {
        "dist": args.dist,
        "h": h,
        "train_contacts": int(len(x)),
        "val_contacts": int(len(xv)),
        "train_seeds": [int(train_seeds[0]), int(train_seeds[-1])],
        "val_seeds": [int(val_seeds[0]), int(val_seeds[-1])],
        "test_seeds": [int(test_seeds[0]), int(test_seeds[-1])],
        "epochs": args.epochs,
        "loss_history": [float(v) for v in hist],
        "val_r2_learned": r2,
        "val_r2_previous_step": r2_prev,
        "dataset_seconds": t_data,
        "train_seconds": t_train,
        "eval": ev,
    }
    out = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", f"warm_start_{args.dist}")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    np.save(out + ".npy", blob.astype(np.float32))
    with open(out + ".json", "w") as f:
        json.dump(report, f, indent=1)
    print(json.dumps({k: report[k] for k in ["dist", "train_contacts", "val_r2_learned", "val_r2_previous_step"]}))
    print(json.dumps(report["eval"]))


if __name__ == "__main__":
    main()
