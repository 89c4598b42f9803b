"""Per-row parity of one Newton iteration (assembly, residual, geometric stiffness,
Schur right-hand side, preconditioner and one Schur product) between the HIP path and
the FP64 oracle, from identical iterates and one contact set (the oracle's, injected
with nsn_set_contacts), on the workloads the benchmark and the configurations run at
their stated sizes:

  * sampled envs of the 4096-env batch in the benchmark's launch configuration
    (every schedule bucket's first and last env plus seeded random ones);
  * the 12^3-hex tet block (8640 tets) under 16 dropped boxes;
  * the articulated hand grasping a ~2k-tet sphere (2160 tets);
  * the 8-cube stack.

Iterations k = 0 (assembly at the start iterate), 1 and 3 (with the secant of the
geometric stiffness, which needs iterate k-1) of a step taken after a few ordinary
steps.  Tolerances as in tests/rows_util.py; every line printed shows, per field and
group, the worst error over the group's scale, the count of elements and of
ill-conditioned ones.
"""
import numpy as np
import pytest

import scene_inputs as si
from oracle import oracle as O
from tests.parity_util import bucket_sample
from tests.rows_util import compare_iteration, inject, oracle_contacts

pytestmark = pytest.mark.gpu

H = 1.0 / 60.0


def _scene(envs, params):
    from paper_1907_04587_amd import Scene
    return Scene(envs, params)


def _run(sc, envs, ids, p, h, ks, M=40, label=""):
    op = O.make_params(p)
    pre = {e: sc.read_state(e) for e in ids}
    failures = []
    for k in ks:
        for e in ids:
            inject(sc, e, oracle_contacts(envs[e], pre[e], h, op))
        sc.dump_iteration(h, k, M)
        for e in ids:
            rep, bad = compare_iteration(sc, e, envs[e], pre[e], h, k, M, op)
            line = {f: f"{r['err']:.1e} ({r['n']}, ill {r['illcond']})" for f, r in rep.items()}
            print(f"{label} env {e} k {k}:", line, flush=True)
            failures += [f"{label} env {e} k {k}: {b}" for b in bad]
        for e in ids:  # back to the pre-step state
            sc.write_state(e, pre[e])
    assert not failures, "\n".join(failures[:20])


def _advance(sc, steps, h, N=10, M=40):
    for _ in range(steps):
        sc.step(h, N, M, 0.0)
    st = sc.stats()
    assert not st["nonfinite"].any()


def test_rows_bench_batch_sampled():
    envs = si.batched_envs(4096, base_seed=1000)
    p = si.SolverParams()
    sc = _scene(envs, p)
    assert len(sc.schedule()) == 3
    _advance(sc, 3, H)
    ids = bucket_sample(sc, n_random=8, seed=5)
    _run(sc, envs, ids, p, H, [0, 1, 3], label="bench")


def test_rows_tet_block_8640():
    envs = [si.tet_block_with_boxes(seed=0)]
    assert envs[0].n_tets == 8640 and envs[0].n_rigid == 16
    p = si.SolverParams()
    sc = _scene(envs, p)
    _advance(sc, 12, H)
    _run(sc, envs, [0], p, H, [0, 1, 3], label="block")


def test_rows_grasp_2k_tets():
    envs = [si.grasp_scene(seed=0)]
    assert envs[0].n_tets > 2000
    p = si.SolverParams()
    h = 1.0 / 120.0
    sc = _scene(envs, p)
    _advance(sc, 6, h)
    _run(sc, envs, [0], p, h, [0, 1, 3], label="grasp")


def test_rows_cube_stack_and_warm_start():
    envs = [si.cube_stack(seed=s) for s in range(2)]
    p = si.SolverParams(warm=si.WARM_PREV)
    sc = _scene(envs, p)
    _advance(sc, 4, H)
    _run(sc, envs, [0, 1], p, H, [0, 1, 3], label="stack")
