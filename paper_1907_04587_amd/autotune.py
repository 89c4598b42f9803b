"""Autotuner of the batched launch schedule.

Environments are launched in decreasing order of work (rows + DOFs).  A schedule cuts
that order into consecutive buckets; each bucket is one grid with its own workgroup
size: 64 threads = one wavefront per env (no cross-wave barrier, many envs per CU),
up to 1024 threads = a 16-wave workgroup per env (large envs).  Buckets run
concurrently on forked streams.

The tuner measures candidates on live steps of the scene (they double as warm-up
steps) and scores each by Newton-kernel time per algorithmic byte of the PCR loop,
which normalises away the step-to-step change of work while the simulation evolves.
"""
from __future__ import annotations

import numpy as np

BLOCKS = (64, 128, 256, 512, 1024)


def _work(envs, order):
    w = []
    for i in order:
        d = envs[i]
        tet_rows = getattr(d, "tet_rows", 3)
        w.append(6 * d.n_joints + tet_rows * d.n_tets + 3 * d.max_contacts + 6 * d.n_rigid + 3 * d.n_particles)
    return np.array(w)


def _start_block(elements):
    b = 64
    while b < 1024 and b * 4 < elements:
        b *= 2
    return b


def _measure(scene, h, newton, cr, tol, steps):
    scene.reset_accumulators()
    for _ in range(steps):
        scene.step(h, newton, cr, tol)
    kt = scene.kernel_times_ms(cap=steps)
    acc = scene.accumulators()
    by = float(acc["cr_bytes"].sum())
    return float(np.sum(kt)) / max(by, 1.0) * 1e9  # ms per GB


def autotune(scene, h, newton, cr, tol, bucket_counts=(1, 2, 4), steps=2, log=None):
    """The scene's current schedule is the first candidate (the library's default for
    large batches is itself a measured choice), then equal-count cuts into
    `bucket_counts` buckets with a coordinate search over each bucket's block size."""
    order = scene.env_order()
    n = len(order)
    work = _work(scene.envs, order)
    current = scene.schedule()
    best = (_measure(scene, h, newton, cr, tol, steps), current)
    if log:
        log(f"autotune current {current}: {best[0]:.3f} ms/GB")
    for nb in bucket_counts:
        if nb > n:
            continue
        cuts = [int(round(k * n / nb)) for k in range(nb + 1)]
        buckets = [[cuts[k], cuts[k + 1] - cuts[k], _start_block(int(work[cuts[k]] // 3 + 1))]
                   for k in range(nb) if cuts[k + 1] > cuts[k]]
        scene.set_schedule([tuple(b) for b in buckets])
        cost = _measure(scene, h, newton, cr, tol, steps)
        for k in range(len(buckets)):
            for blk in BLOCKS:
                if blk == buckets[k][2]:
                    continue
                trial = [list(b) for b in buckets]
                trial[k][2] = blk
                scene.set_schedule([tuple(b) for b in trial])
                c = _measure(scene, h, newton, cr, tol, steps)
                if log:
                    log(f"autotune nb={nb} bucket {k} block {blk}: {c:.3f} ms/GB (best {cost:.3f})")
                if c < cost:
                    cost, buckets = c, trial
        if cost < best[0]:
            best = (cost, [tuple(b) for b in buckets])
        if log:
            log(f"autotune nb={nb}: {best}")
    scene.set_schedule(best[1])
    return best[1]
