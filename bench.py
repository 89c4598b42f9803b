#!/usr/bin/env python
"""Benchmark: env-steps/s at NCP residual 1e-4 on one MI355X.

Workload: 4096 independent environments of uneven size (5-40 boxes, 0-12 revolute
joints, 0-3000 neo-Hookean tets, mu in [0.3, 1]), stepped together by the persistent
per-env Newton kernel (one launch per step, replayed from a hipGraph), h = 1/60 s,
residual mode: every env stops when r_ncp <= 1e-4 or after 50 Newton iterations of 40
PCR iterations.  Inputs are seeded and synthetic and already resident in HBM.

Prints ONE JSON line.  `value` is env-steps/s of the headline arm (the faster of the
two learned warm starts when the trained model is available: "learned" takes the
network's multipliers for every contact, "hybrid" keeps the previous step's for
contacts that persist and takes the network's for new ones; else the stronger plain
start); every arm is reported under "arms".  `roofline` covers the dominant kernel (the Newton kernel):
algorithmic bytes of its PCR loop per launch divided by its launch duration, the
latter read from the GPU wall clock inside the kernel for every timed step.
`cpu_baseline` times the FP64 oracle on a bounded sample of the same envs on the
host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
H = 1.0 / 60.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_arm(envs, arm, args, model_blob=None):
    import numpy as np
    import torch

    import scene_inputs as si
    from paper_1907_04587_amd import Scene

    warm = {"zero": si.WARM_ZERO, "prev": si.WARM_PREV, "learned": si.WARM_LEARNED,
            "hybrid": si.WARM_HYBRID}[arm]
    p = si.SolverParams(warm=si.WARM_ZERO, islands=int(args.islands))
    sc = Scene(envs, p)
    if model_blob is not None:
        sc.set_warm_start_model(model_blob)
    if args.schedule:
        from paper_1907_04587_amd.autotune import autotune
        sched = autotune(sc, H, args.newton, args.cr, args.tol, log=log)
        log(f"[{arm}] schedule {sched}")
    p.warm = warm
    sc.set_params(p)
    for i in range(args.warmup):
        sc.step(H, args.newton, args.cr, args.tol)
        if i == 0 or (i + 1) % 10 == 0:
            sc.synchronize()
            log(f"[{arm}] warmup {i + 1}/{args.warmup}")
    sc.reset_accumulators()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        sc.step(H, args.newton, args.cr, args.tol)
        if (i + 1) % max(1, args.steps // 5) == 0:
            log(f"[{arm}] timed step {i + 1}/{args.steps} enqueued")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    acc = sc.accumulators()
    kt = sc.kernel_times_ms(cap=args.steps)
    n = len(envs)
    steps_total = int(acc["steps"].sum())
    res = {
        "env_steps_per_s": steps_total / wall,
        "ms_per_step": 1e3 * wall / args.steps,
        "converged_frac": float(acc["converged"].sum()) / max(steps_total, 1),
        "mean_newton_iters": float(acc["newton_iters"].sum()) / max(steps_total, 1),
        "mean_cr_iters": float(acc["cr_iters"].sum()) / max(steps_total, 1),
        "env_cr_iters_per_s": float(acc["cr_iters"].sum()) / wall,
        "nonfinite_steps": int(acc["nonfinite"].sum()),
        "newton_kernel_ms": float(np.mean(kt)) if len(kt) else None,
        "cr_bytes_per_launch": float(acc["cr_bytes"].sum()) / args.steps,
        "n_envs": n,
    }
    if res["newton_kernel_ms"]:
        res["achieved_gbs"] = res["cr_bytes_per_launch"] / (res["newton_kernel_ms"] * 1e-3) / 1e9
    del sc
    torch.cuda.empty_cache()
    return res


def cpu_baseline(envs, args):
    """FP64 oracle, as it stands, on a bounded sample of the same envs (a few steps of
    residual mode each, one env per thread)."""
    import concurrent.futures as cf

    import numpy as np

    from oracle import oracle as O
    import scene_inputs as si

    cores = min(16, os.cpu_count() or 1)
    rng = np.random.default_rng(123)
    idx = rng.choice(len(envs), size=min(args.cpu_envs, len(envs)), replace=False)
    params = O.make_params(si.SolverParams(warm=si.WARM_PREV))

    def work(i):
        e = O.OracleEnv(envs[i])
        for _ in range(args.cpu_steps):
            e.step(H, args.newton, args.cr, args.tol, params)
        return args.cpu_steps

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        done = sum(ex.map(work, idx))
    wall = time.perf_counter() - t0
    return {"value": done / wall, "unit": "env-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(idx)} randomly chosen envs of the same 4096-env batch x {args.cpu_steps} steps "
                      f"from their initial state, residual mode (tol {args.tol}, <= {args.newton} Newton x "
                      f"{args.cr} PCR), previous-step warm start, one env per thread, {wall:.1f} s"}


def traffic_from_profile(tet_model):
    """HBM traffic of the Newton kernel from the committed rocprofv3 counter summary of
    the same workload (tet model), if it was taken on the current kernel sources; else
    None."""
    import hashlib
    name = "newton_kernel_traffic.json" if tet_model == "neohookean" else f"newton_kernel_traffic_{tet_model}.json"
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    h = hashlib.sha256()
    for name in sorted(os.listdir(os.path.join(ROOT, "paper_1907_04587_amd", "csrc"))):
        if name.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(ROOT, "paper_1907_04587_amd", "csrc", name), "rb") as f:
                h.update(f.read())
    if prof.get("sources_sha256") != h.hexdigest():
        return None
    return prof.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--envs", type=int, default=4096)
    ap.add_argument("--newton", type=int, default=50)
    ap.add_argument("--cr", type=int, default=40)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--arms", default="zero,prev,learned,hybrid")
    ap.add_argument("--islands", action="store_true", help="one PCR per island of an env (Sec. 11 option)")
    ap.add_argument("--tets-max", type=int, default=3000, help="largest tet block of an env (0: rigid only)")
    ap.add_argument("--tet-model", choices=["neohookean", "linear"], default="neohookean",
                    help="material of the envs' tet blocks (linear: six co-rotated strain rows per tet)")
    ap.add_argument("--schedule", action="store_true", help="autotune the launch schedule first")
    ap.add_argument("--cpu-envs", type=int, default=256)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 launches): the reference for "
                         "scaling the HBM byte counters of a profiler")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: environments are independent, so each GPU would "
              "step its own share of the batch in its own workspace with no per-step "
              "communication; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import scene_inputs as si

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 5}))
        return
    log(f"generating {args.envs} envs")
    tet_model = si.TET_LINEAR if args.tet_model == "linear" else si.TET_NEOHOOKEAN
    envs = si.batched_envs(args.envs, base_seed=1000, tet_model=tet_model, tets_max=args.tets_max)
    blobs = {}
    model_path = os.path.join(ROOT, "paper_1907_04587_amd", "weights", "warm_start_batched.npy")
    if os.path.exists(model_path):
        blobs["learned"] = blobs["hybrid"] = np.load(model_path, allow_pickle=False)
    arms = [a for a in args.arms.split(",") if a and (a not in ("learned", "hybrid") or a in blobs)]
    results = {}
    for arm in arms:
        log(f"arm {arm}")
        results[arm] = run_arm(envs, arm, args, blobs.get(arm))
        log(f"arm {arm}: {json.dumps(results[arm])}")
    plains = [a for a in results if a in ("zero", "prev")]
    plain = max(plains, key=lambda a: results[a]["env_steps_per_s"]) if plains else None
    learned = [a for a in results if a in ("learned", "hybrid")]
    head = max(learned, key=lambda a: results[a]["env_steps_per_s"]) if learned else plain
    if head is None:
        sys.exit("bench.py: no arm to report (--arms)")
    r = results[head]
    roof = None
    if r.get("achieved_gbs"):
        traffic = traffic_from_profile(args.tet_model)
        roof = {"bound": "hbm", "achieved": round(r["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "nsn::k_newton", "kernel_ms": round(r["newton_kernel_ms"], 3),
                "algorithmic_bytes_per_launch": r["cr_bytes_per_launch"]}
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(envs, args)
    out = {
        "metric": "env-steps/s at NCP residual 1e-4 (plain vs learned warm start); CR iters/s",
        "value": round(r["env_steps_per_s"], 2),
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.envs} uneven envs (5-40 boxes, 0-12 revolute joints, 0-{args.tets_max} "
                               f"{'linear co-rotated' if args.tet_model == 'linear' else 'neo-Hookean'} "
                               f"tets), h=1/60, residual mode tol={args.tol}, "
                               f"{'one PCR per island, ' if args.islands else ''}"
                               f"<= {args.newton} Newton x {args.cr} PCR",
                   "n_envs": args.envs, "arm": head, "plain_arm": plain},
        "cr_iters_per_s": round(r["env_cr_iters_per_s"], 1),
        "arms": {a: {k: (round(v, 6) if isinstance(v, float) else v) for k, v in results[a].items()}
                 for a in results},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
