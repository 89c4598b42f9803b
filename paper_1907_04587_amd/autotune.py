"""Autotuner of the batched launch schedule.

Environments are launched in decreasing order of work (rows + DOFs).  A schedule cuts
that order into consecutive buckets; each bucket is one grid, launched concurrently
with the others on forked streams, in one of two families:

  tile:                one workgroup of 128 to 1024 threads (2 to 16 wavefronts) per
                       env, cooperating over the env's rows through LDS and barriers;
  wavefront per env:   one 64-thread workgroup per env, the whole env in a single
                       wavefront (no cross-wave barrier or LDS reduction); the CU holds
                       as many of them side by side as registers allow, so several
                       small envs share a CU without waiting on one another.

Objective: env-steps/s.  Every candidate replays the same steps from one snapshot of
the scene's state (nsn_save_state / nsn_load_state), so candidates see identical work;
the scene is left at the snapshot with the best schedule set.  Candidates run as direct
launches (a capture per candidate would only be thrown away); the scene's graph
setting is restored afterwards.
"""
from __future__ import annotations

import time

BLOCKS = (64, 128, 256, 512, 1024)


def _valid(buckets, n):
    at = 0
    for first, count, block in buckets:
        if first != at or count <= 0 or block not in BLOCKS:
            return False
        at += count
    return at == n


def _score(scene, snap, sched, h, newton, cr, tol, steps):
    """env-steps/s of `steps` steps from the snapshot under `sched`."""
    scene.set_schedule([tuple(b) for b in sched])
    scene.load_state(snap)
    scene.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        scene.step(h, newton, cr, tol)
    scene.synchronize()
    return scene.n_envs * steps / (time.perf_counter() - t0)


def candidates(current, n):
    """The schedules tried after `current`: each bucket's block size moved to its
    neighbours (coordinate search of the tile family, 64 threads included for the
    lightest bucket), then the wavefront-per-env family on the light tail of the
    order (the last 1/8 or 1/4 of the envs at 64 threads, split off the last bucket)."""
    out = []
    for k, (_, _, blk) in enumerate(current):
        i = BLOCKS.index(blk)
        for j in (i - 1, i + 1):
            if 0 <= j < len(BLOCKS) and (BLOCKS[j] != 64 or k == len(current) - 1):
                trial = [list(b) for b in current]
                trial[k][2] = BLOCKS[j]
                out.append(("tile" if BLOCKS[j] != 64 else "wavefront", trial))
    last_first, last_count, last_blk = current[-1]
    for frac in (1 / 8, 1 / 4):
        tail = int(round(frac * n))
        if last_blk != 64 and 0 < tail < last_count:
            trial = [list(b) for b in current[:-1]]
            trial.append([last_first, last_count - tail, last_blk])
            trial.append([last_first + last_count - tail, tail, 64])
            out.append(("wavefront", trial))
    return [(fam, t) for fam, t in out if _valid(t, n)]


def autotune(scene, h, newton, cr, tol, steps=2, rounds=2, forms=(), log=None):
    """Tune the scene's schedule by env-steps/s over `steps` replayed steps per candidate.
    Starts from the scene's current schedule (the library's default) and repeats the
    neighbourhood search `rounds` times from the best so far; then, under the best
    schedule, tries each PCR form in `forms` (nsn_set_pcr_form).  Returns (schedule,
    PCR form, report) where report lists every candidate's family, schedule, form and
    env-steps/s."""
    n = scene.n_envs
    graphs = scene.use_graphs
    scene.set_use_graphs(False)
    try:
        return _search(scene, n, h, newton, cr, tol, steps, rounds, forms, log)
    finally:
        scene.set_use_graphs(graphs)


def _search(scene, n, h, newton, cr, tol, steps, rounds, forms, log):
    snap = scene.save_state()
    current = [list(b) for b in scene.schedule()]
    form = scene.pcr_form
    best = _score(scene, snap, current, h, newton, cr, tol, steps)
    report = [{"family": "default", "schedule": [tuple(b) for b in current], "pcr_form": form,
               "env_steps_per_s": best}]
    if log:
        log(f"autotune default {current}: {best:.1f} env-steps/s")
    seen = {tuple(map(tuple, current))}
    for _ in range(rounds):
        improved = False
        for fam, trial in candidates(current, n):
            key = tuple(map(tuple, trial))
            if key in seen:
                continue
            seen.add(key)
            v = _score(scene, snap, trial, h, newton, cr, tol, steps)
            report.append({"family": fam, "schedule": [tuple(b) for b in trial], "pcr_form": form,
                           "env_steps_per_s": v})
            if log:
                log(f"autotune {fam} {trial}: {v:.1f} env-steps/s (best {best:.1f})")
            if v > best * 1.01:  # a candidate must beat the timing noise to replace the best
                best, current, improved = v, trial, True
        if not improved:
            break
    for f in forms:
        if f == form:
            continue
        scene.set_pcr_form(f)
        v = _score(scene, snap, current, h, newton, cr, tol, steps)
        report.append({"family": f"pcr form {f}", "schedule": [tuple(b) for b in current], "pcr_form": f,
                       "env_steps_per_s": v})
        if log:
            log(f"autotune PCR form {f}: {v:.1f} env-steps/s (best {best:.1f})")
        if v > best * 1.01:
            best, form = v, f
    scene.set_pcr_form(form)
    scene.set_schedule([tuple(b) for b in current])
    scene.load_state(snap)
    scene.synchronize()
    return [tuple(b) for b in current], form, report


def default_vs(scene, snap, sched, form, h, newton, cr, tol, steps, default, default_form):
    """(env-steps/s of `default` with PCR form `default_form`, of `sched` with `form`)
    replayed from the same snapshot; the scene is left at the snapshot under `sched`."""
    scene.set_pcr_form(default_form)
    a = _score(scene, snap, default, h, newton, cr, tol, steps)
    scene.set_pcr_form(form)
    b = _score(scene, snap, sched, h, newton, cr, tol, steps)
    scene.load_state(snap)
    return a, b


__all__ = ["autotune", "candidates", "default_vs", "BLOCKS"]
