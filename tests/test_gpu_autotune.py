"""State snapshot (nsn_save_state / nsn_load_state) and the schedule autotuner on the
GPU: a restored snapshot repeats the following steps bit for bit; the tuner returns a
valid schedule that is no slower than the default on the benchmark's 4096-env batch,
and the envs it launches differently still match the FP64 oracle row by row."""
import numpy as np
import pytest

import scene_inputs as si
from tests.parity_util import bucket_sample
from tests.test_gpu_rows import _run

pytestmark = pytest.mark.gpu

H = 1.0 / 60.0


def _snapshot_of(sc, n):
    out = []
    for e in range(n):
        st = sc.read_state(e)
        st["lam"] = sc.lambdas(e)
        c = sc.contacts(e)
        st["keys"], st["clam"] = c["key"], c["lam"]
        out.append(st)
    return out


def _equal(a, b):
    for x, y in zip(a, b):
        for k in x:
            assert np.array_equal(np.asarray(x[k]), np.asarray(y[k])), k


@pytest.mark.parametrize("warm", [si.WARM_ZERO, si.WARM_PREV])
def test_snapshot_repeats_steps_bitwise(warm):
    from paper_1907_04587_amd import Scene

    envs = si.batched_envs(96, base_seed=1000, tets_max=600)
    sc = Scene(envs, si.SolverParams(warm=warm))
    for _ in range(2):
        sc.step(H, 12, 20, 1e-4)
    before = _snapshot_of(sc, len(envs))
    snap = sc.save_state()
    for _ in range(3):
        sc.step(H, 12, 20, 1e-4)
    first = _snapshot_of(sc, len(envs))
    sc.load_state(snap)
    restored = [{k: v for k, v in s.items() if k not in ("lam", "keys", "clam")} for s in _snapshot_of(sc, len(envs))]
    _equal(restored, [{k: v for k, v in s.items() if k not in ("lam", "keys", "clam")} for s in before])
    for _ in range(3):
        sc.step(H, 12, 20, 1e-4)
    _equal(_snapshot_of(sc, len(envs)), first)


def test_autotune_bench_batch_valid_not_slower_with_row_parity():
    from paper_1907_04587_amd import Scene
    from paper_1907_04587_amd.autotune import BLOCKS, autotune, default_vs

    envs = si.batched_envs(4096, base_seed=1000)
    p = si.SolverParams()
    sc = Scene(envs, p)
    for _ in range(2):
        sc.step(H, 50, 40, 1e-4)
    default, default_form = [tuple(b) for b in sc.schedule()], sc.pcr_form
    sched, form, report = autotune(sc, H, 50, 40, 1e-4, steps=1, rounds=1, forms=(0, 1, 2), log=print)
    assert form in (0, 1, 2) and sc.pcr_form == form
    # valid: consecutive buckets covering the launch order once, known block sizes
    at = 0
    for first, count, block in sched:
        assert first == at and count > 0 and block in BLOCKS
        at += count
    assert at == len(envs)
    assert [tuple(b) for b in sc.schedule()] == [tuple(b) for b in sched]
    assert {c["family"] for c in report} >= {"default", "tile", "wavefront"} | {
        f"pcr form {f}" for f in (0, 1, 2) if f != default_form}
    # not slower than the default on the same replayed steps (a timing-noise margin)
    snap = sc.save_state()
    d, t = default_vs(sc, snap, sched, form, H, 50, 40, 1e-4, 2, default, default_form)
    print(f"default {default} form {default_form}: {d:.1f} env-steps/s; tuned {sched} form {form}: {t:.1f}")
    assert t >= 0.97 * d
    # row parity on sampled envs of every bucket of the tuned schedule
    sc.set_schedule(sched)
    ids = bucket_sample(sc, n_random=4, seed=11)
    _run(sc, envs, ids, p, H, [0, 1], label="tuned")
