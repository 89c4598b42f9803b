#!/usr/bin/env python
"""Benchmark: env-steps/s at NCP residual 1e-4 on one MI355X.

Workload: 4096 independent environments of uneven size (5-40 boxes, 0-12 revolute
joints, 0-3000 neo-Hookean tets, mu in [0.3, 1]), stepped together by the persistent
per-env Newton kernel (one launch per step, replayed from a hipGraph), h = 1/60 s,
residual mode: every env stops when r_ncp <= 1e-4 or after 50 Newton iterations of 40
PCR iterations.  Inputs are seeded and synthetic and already resident in HBM.

Before the timed steps the autotuner picks the launch schedule and the form of the
PCR loop by env-steps/s, replaying the same steps from one state snapshot per
candidate (--no-tune keeps the library's defaults); every arm then runs under them.

Prints ONE JSON line.  `value` is env-steps/s of the headline arm: of the two learned
warm starts ("learned" takes the network's multipliers for every contact, "hybrid"
keeps the previous step's for contacts that persist and takes the network's for new
ones), the one with more env-steps/s reaching the residual, when the trained model is
available; else the stronger plain start.  Each arm reports its env-steps/s, the
env-steps/s that reached the residual, and the distribution of the last step's exit
residuals; `learned_vs_plain` compares the headline arm with each plain arm.
`roofline` covers the dominant kernel (the Newton kernel): algorithmic bytes of its
PCR loop per launch divided by its launch duration, the latter read from the GPU wall
clock inside the kernel for every timed step, with a plain device copy's bandwidth
beside it.  `cpu_baseline` times the FP64 oracle in the headline arm and step window
on a bounded sample of the same envs on the host cores.
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


def run_arm(envs, arm, args, model_blob=None, tuned=None):
    """One arm: warm-up steps, then (first arm only: tuned None and tuning on) the
    autotuner from the post-warm-up state, then the timed steps from that same state.
    tuned: (schedule, PCR form) to run under.  Returns (results, (schedule, PCR form)
    used, tuner report or None)."""
    import numpy as np
    import torch

    import scene_inputs as si
    from paper_1907_04587_amd import Scene

    warm = {"zero": si.WARM_ZERO, "prev": si.WARM_PREV, "learned": si.WARM_LEARNED,
            "hybrid": si.WARM_HYBRID}[arm]
    p = si.SolverParams(warm=si.WARM_ZERO, islands=int(args.islands), watchdog=int(args.watchdog))
    sc = Scene(envs, p, stream=None if args.stream == "private" else torch.cuda.current_stream())
    if model_blob is not None:
        sc.set_warm_start_model(model_blob)
    if args.graphs >= 0:
        sc.set_use_graphs(bool(args.graphs))
    if tuned is not None:
        if tuned[0] is not None:
            sc.set_schedule(tuned[0])
        if tuned[1] is not None:
            sc.set_pcr_form(tuned[1])
    p.warm = warm
    sc.set_params(p)
    if args.pcr_form >= 0:
        sc.set_pcr_form(args.pcr_form)
    for i in range(args.warmup):
        sc.step(H, args.newton, args.cr, args.tol)
        if i == 0 or (i + 1) % 10 == 0:
            sc.synchronize()
            log(f"[{arm}] warmup {i + 1}/{args.warmup}")
    report = None
    if tuned is None and not args.no_tune:
        from paper_1907_04587_amd.autotune import autotune
        sched, form, report = autotune(sc, H, args.newton, args.cr, args.tol, steps=args.tune_steps,
                                       forms=(0, 1, 2) if args.pcr_form < 0 else (), log=log)
        log(f"[{arm}] tuned schedule {sched}, PCR form {form}")
    used = ([tuple(b) for b in sc.schedule()], sc.pcr_form)
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
    st = sc.stats()  # the last timed step's per-env exit record
    n = len(envs)
    steps_total = int(acc["steps"].sum())
    conv_total = int(acc["converged"].sum())
    res = {
        "env_steps_per_s": steps_total / wall,
        "converged_env_steps_per_s": conv_total / wall,
        "ms_per_step": 1e3 * wall / args.steps,
        "converged_frac": conv_total / max(steps_total, 1),
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
    res["residual_last_step"] = residual_distribution(envs, st, args.tol)
    del sc
    torch.cuda.empty_cache()
    return res, used, report


def residual_distribution(envs, st, tol):
    """Exit residuals r_ncp of one step over the batch: quantiles, the fraction at or
    below tol, and the same for the envs with and without a tet block."""
    import numpy as np

    r = np.asarray(st["r_ncp"], np.float64)
    fem = np.array([d.n_tets > 0 for d in envs])

    def summ(m):
        if not m.any():
            return None
        q = np.quantile(r[m], [0.1, 0.5, 0.9, 0.99])
        return {"n": int(m.sum()), "p10": float(q[0]), "p50": float(q[1]), "p90": float(q[2]),
                "p99": float(q[3]), "max": float(r[m].max()), "frac_at_tol": float((r[m] <= tol).mean())}

    return {"all": summ(np.ones(len(r), bool)), "with_tets": summ(fem), "rigid_only": summ(~fem)}


WARM_OF_ARM = {"zero": 0, "prev": 1, "learned": 2, "hybrid": 3}


def host_cores():
    """Cores this process may use, bounded by the host's share per GPU (16)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(envs, args, arm, blob):
    """FP64 oracle, as it stands, on a bounded sample of the same batch, in the headline's
    arm (same warm start, same weights) and step window (args.warmup untimed steps from
    the initial state, then the timed steps), one env per thread on every usable core.
    The sample is stratified over the launch order of work (evenly spaced ranks of
    rows + DOFs), so its mean work per env follows the batch's."""
    import concurrent.futures as cf

    import numpy as np

    from oracle import oracle as O
    import scene_inputs as si

    cores = host_cores()
    work = np.array([6 * d.n_joints + 3 * d.n_tets + 6 * d.n_rigid + 3 * d.n_particles for d in envs])
    order = np.argsort(-work, kind="stable")
    m = min(args.cpu_envs, len(envs))
    idx = order[np.linspace(0, len(envs) - 1, m).round().astype(int)]
    params = O.make_params(si.SolverParams(warm=WARM_OF_ARM[arm]))
    oes = {}

    def warm_up(i):
        e = O.OracleEnv(envs[i])
        if blob is not None:
            e.set_mlp(blob)
        for _ in range(args.warmup):
            e.step(H, args.newton, args.cr, args.tol, params)
        oes[i] = e

    def timed(i):
        e = oes[i]
        for _ in range(args.cpu_steps):
            e.step(H, args.newton, args.cr, args.tol, params)
        return args.cpu_steps

    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(warm_up, idx))
        t0 = time.perf_counter()
        done = sum(ex.map(timed, idx))
        wall = time.perf_counter() - t0
    return {"value": done / wall, "unit": "env-steps/s", "cores": cores, "nproc": os.cpu_count(),
            "kind": "oracle",
            "sample": f"{m} envs of the same {len(envs)}-env batch at evenly spaced ranks of work, arm {arm}, "
                      f"{args.warmup} untimed steps from the initial state then {args.cpu_steps} timed steps "
                      f"(steps {args.warmup + 1}-{args.warmup + args.cpu_steps} of the window the GPU times), "
                      f"residual mode (tol {args.tol}, <= {args.newton} Newton x {args.cr} PCR), one env per "
                      f"thread on {cores} threads, {wall:.1f} s timed"}


def copy_gbs(mib=2048, reps=10):
    """Bandwidth of a plain device copy (read + write bytes over time, HIP events): what
    a pure streaming kernel reaches on this GPU, next to the roofline's peak."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * 4 * n / (ms * 1e-3) / 1e9


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
    ap.add_argument("--watchdog", type=int, default=0, choices=[0, 1],
                    help="1: a diverging step returns its lowest-merit iterate (not in the paper); "
                         "0: the paper's iteration (default)")
    ap.add_argument("--stream", choices=["private", "current"], default="private",
                    help="the scene's stream: its own (graph replay, buckets on forked streams; default) or "
                         "torch's current one")
    ap.add_argument("--graphs", type=int, default=-1, choices=[-1, 0, 1],
                    help="1: replay each step from a hipGraph; 0: launch directly; -1: the library's default")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the library's default schedule (no autotuning before the timed steps)")
    ap.add_argument("--tune-steps", type=int, default=1, help="replayed steps per autotuner candidate")
    ap.add_argument("--schedule", default=None, metavar="FIRST:COUNT:BLOCK,...",
                    help="launch every arm under this schedule (buckets of the launch order) instead of tuning")
    ap.add_argument("--pcr-form", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="0: streaming two-pass PCR; 1: register-resident where an env's elements fit; "
                         "2: one-pass; -1: the library's default, or the tuner's choice")
    ap.add_argument("--cpu-envs", type=int, default=48, help="envs of the oracle's sample")
    ap.add_argument("--cpu-steps", type=int, default=2, help="timed oracle steps per sampled env")
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
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 5
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 5,
                          "ms_per_launch": ms, "copy_gbs": 2 * 4 * n / (ms * 1e-3) / 1e9}))
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
    tuned, tune_report = None, None
    if args.schedule:
        tuned = ([tuple(int(v) for v in b.split(":")) for b in args.schedule.split(",")], None)
    for arm in arms:
        log(f"arm {arm}")
        results[arm], tuned, rep = run_arm(envs, arm, args, blobs.get(arm), tuned)
        tune_report = tune_report or rep
        log(f"arm {arm}: {json.dumps(results[arm])}")
    # arms ranked by env-steps/s that reach the residual, then by all env-steps/s
    rank = lambda a: (results[a]["converged_env_steps_per_s"], results[a]["env_steps_per_s"])  # noqa: E731
    plains = [a for a in results if a in ("zero", "prev")]
    plain = max(plains, key=rank) if plains else None
    learned = [a for a in results if a in ("learned", "hybrid")]
    head = max(learned, key=rank) if learned else plain
    if head is None:
        sys.exit("bench.py: no arm to report (--arms)")
    r = results[head]
    roof = None
    if r.get("achieved_gbs"):
        traffic = traffic_from_profile(args.tet_model)
        roof = {"bound": "hbm", "achieved": round(r["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "nsn::k_newton", "kernel_ms": round(r["newton_kernel_ms"], 3),
                "algorithmic_bytes_per_launch": r["cr_bytes_per_launch"],
                "copy_kernel_gbs": round(copy_gbs(), 1)}
    verdict = None
    if plain is not None and head != plain:
        def versus(rp):
            ratio = r["env_steps_per_s"] / rp["env_steps_per_s"]
            cratio = (r["converged_env_steps_per_s"] / rp["converged_env_steps_per_s"]
                      if rp["converged_env_steps_per_s"] > 0 else None)
            return {"env_steps_ratio": round(ratio, 4),
                    "converged_env_steps_ratio": round(cratio, 4) if cratio is not None else None,
                    "newton_iters_ratio": round(r["mean_newton_iters"] / max(rp["mean_newton_iters"], 1e-30), 4),
                    # beats: more env-steps/s reach the residual, by a 5% margin (the
                    # converged counts of one arm move by about 3% between runs), at no
                    # loss of env-steps/s overall (1%)
                    "beats": bool(cratio is not None and cratio > 1.05 and ratio > 0.99)}
        verdict = {"learned_arm": head, "plain_arm": plain, **versus(results[plain]),
                   "per_plain_arm": {a: versus(results[a]) for a in plains}}
        verdict["beats_plain"] = verdict.pop("beats")
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(envs, args, head, blobs.get(head))
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
                               f"{'watchdog on, ' if args.watchdog else ''}"
                               f"<= {args.newton} Newton x {args.cr} PCR",
                   "n_envs": args.envs, "arm": head, "plain_arm": plain,
                   "schedule": [list(b) for b in tuned[0]], "pcr_form": tuned[1]},
        "cr_iters_per_s": round(r["env_cr_iters_per_s"], 1),
        "converged_env_steps_per_s": round(r["converged_env_steps_per_s"], 2),
        "learned_vs_plain": verdict,
        "arms": {a: {k: (round(v, 6) if isinstance(v, float) else v) for k, v in results[a].items()}
                 for a in results},
        "autotune": None if tune_report is None else {
            "objective": "env-steps/s over replayed steps from one state snapshot",
            "default_env_steps_per_s": round(tune_report[0]["env_steps_per_s"], 2),
            "best_env_steps_per_s": round(max(c["env_steps_per_s"] for c in tune_report), 2),
            "candidates": [[c["family"], [list(b) for b in c["schedule"]], c["pcr_form"],
                            round(c["env_steps_per_s"], 2)]
                           for c in tune_report]},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
