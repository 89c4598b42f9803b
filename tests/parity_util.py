"""Helpers comparing the HIP path with the FP64 oracle on identical pre-step states."""
import numpy as np

from oracle import oracle as O


def state_close(gpu, orc, L_scene=1.0, h=1 / 60, g=9.81, tol=1e-4):
    """Relative errors of R22 style: positions over max(|x|_inf, L_scene), quaternions
    absolute after fixing the sign to w >= 0, velocities over max(|u|_inf, g h).
    Returns a dict of the error of each field."""
    out = {}
    for k in ["rigid_x", "particle_x"]:
        a, b = np.asarray(gpu[k], np.float64), np.asarray(orc[k], np.float64)
        if a.size:
            out[k] = np.abs(a - b).max() / max(np.abs(b).max(), L_scene)
    if np.asarray(gpu["rigid_q"]).size:
        a, b = np.asarray(gpu["rigid_q"], np.float64), np.asarray(orc["rigid_q"], np.float64)
        a = a * np.where(a[:, :1] < 0, -1, 1)
        b = b * np.where(b[:, :1] < 0, -1, 1)
        out["rigid_q"] = np.abs(a - b).max()
    for k in ["rigid_v", "rigid_w", "particle_v"]:
        a, b = np.asarray(gpu[k], np.float64), np.asarray(orc[k], np.float64)
        if a.size:
            out[k] = np.abs(a - b).max() / max(np.abs(b).max(), g * h)
    return out


FP32_REL = 1.2e-7  # about one FP32 ulp, relative
STATE_TOL_CAP = 1e-3  # largest conditioning-based state tolerance that is still asserted


class History(list):
    """Per-step worst errors of a lockstep run, with the comparisons whose
    conditioning-based tolerance exceeded STATE_TOL_CAP (not asserted: capped)."""

    def __init__(self):
        super().__init__()
        self.capped = []


def skip_if_capped(hist):
    """Mark a test skipped (after every decidable comparison has passed) when some of
    its comparisons were above the cap, naming them."""
    import pytest
    if hist.capped:
        cases = "; ".join(f"step {s} env {e} {k}: tol {t:.1e} (err {v:.1e})" for s, e, k, t, v in hist.capped[:8])
        pytest.skip(f"{len(hist.capped)} comparisons not decidable at the {STATE_TOL_CAP:g} cap "
                    f"(the FP64 oracle itself moves more under FP32-sized input changes): {cases}")


def oracle_sensitivity(desc, pre, op, h, N, M, tol, trials=3, L_scene=1.0, prev=None):
    """How far the oracle's own step moves when its input state is perturbed at the
    level of FP32 rounding (relative noise of about one ulp on positions and
    velocities, plus one ulp of g h on velocities, which are often exact zeros at
    rest): the spread that an FP32 implementation cannot be expected to beat.
    prev = (keys, lam3, lam_joint) loads previous-step multipliers for warm starts.
    Returns {field: worst relative change} in the metric of state_close."""
    base = O.OracleEnv(desc)
    if prev is not None:
        base.set_prev(*prev)
    st0 = {k: np.asarray(v, np.float64) for k, v in pre.items() if k != "time"}
    base.set_state(st0)
    base.time = pre["time"]
    base.step(h, N, M, tol, op)
    ref = base.get_state()
    worst = {}
    for t in range(trials):
        rng = np.random.default_rng(100 + t)
        st = {k: v.copy() for k, v in st0.items()}
        for k in ["rigid_x", "particle_x", "rigid_v", "rigid_w", "particle_v"]:
            if st[k].size:
                st[k] = st[k] * (1.0 + FP32_REL * rng.standard_normal(st[k].shape))
                if k.endswith(("_v", "_w")):  # velocities at rest are exact zeros: add ulp(g h)
                    st[k] = st[k] + FP32_REL * 9.81 * h * rng.standard_normal(st[k].shape)
        oe = O.OracleEnv(desc)
        if prev is not None:
            oe.set_prev(*prev)
        oe.set_state(st)
        oe.time = pre["time"]
        oe.step(h, N, M, tol, op)
        for k, v in state_close(oe.get_state(), ref, L_scene=L_scene, h=h).items():
            worst[k] = max(worst.get(k, 0.0), v)
    return worst


def lockstep(scene, envs, params, h, N, M, tol=0.0, steps=1, env_ids=None, check_contacts=True,
             err_tol=1e-4, L_scene=1.0, sens_factor=None, prev_from_gpu=False, sens_trials=3):
    """Step the GPU scene `steps` times; before each step copy every checked env's
    state into a fresh oracle env and step it too; compare after each step.

    With sens_factor set, the tolerance of each field is
    max(err_tol, sens_factor * oracle_sensitivity(...)): where the unconverged
    iterate amplifies rounding (global Krylov scalars shared by stiff and soft parts,
    the per-DOF secant of the geometric stiffness), FP32 and FP64 cannot agree closer
    than the problem's own conditioning; elsewhere err_tol applies unchanged.  A
    tolerance above STATE_TOL_CAP is not asserted: the comparison is recorded in the
    returned history's `capped` list (see skip_if_capped).
    prev_from_gpu: from the second step on, the oracle's previous-step multipliers
    (the warm start's input) are the GPU's, so both sides start from the same lambda0.
    sens_trials: perturbed oracle runs per estimate (more trials, a larger and less
    state-dependent estimate of the spread).
    Returns the list of per-step dicts {field: (worst error, its env, its tolerance)}."""
    if env_ids is None:
        env_ids = list(range(len(envs)))
    op = O.make_params(params)
    orcs = {e: O.OracleEnv(envs[e]) for e in env_ids}
    history = History()
    for s in range(steps):
        pre = {e: scene.read_state(e) for e in env_ids}
        prev = {}
        if prev_from_gpu and s > 0:
            for e in env_ids:
                c = scene.contacts(e)
                lj = scene.lambdas(e)[:6 * envs[e].n_joints]
                prev[e] = (c["key"], np.asarray(c["lam"], np.float64), np.asarray(lj, np.float64))
        scene.step(h, N, M, tol)
        stats = scene.stats()
        worst = {}
        for e in env_ids:
            oe = orcs[e]
            oe.set_state({k: np.asarray(v, np.float64) for k, v in pre[e].items() if k != "time"})
            oe.time = pre[e]["time"]
            if e in prev:
                oe.set_prev(*prev[e])
            ost = oe.step(h, N, M, tol, op)
            post = scene.read_state(e)
            if check_contacts:
                gk = scene.contacts(e)["key"]
                ok = oe.contacts()["key"]
                assert np.array_equal(gk, ok), f"step {s} env {e}: contact sets differ " \
                    f"({len(gk)} vs {len(ok)}, sym diff {sorted(set(gk) ^ set(ok))[:10]})"
            err = state_close(post, oe.get_state(), L_scene=L_scene, h=h)
            err["stats_gpu"] = stats[e]
            err["stats_orc"] = ost
            tols = {k: err_tol for k in err}
            if sens_factor is not None:
                sens = oracle_sensitivity(envs[e], pre[e], op, h, N, M, tol, trials=sens_trials, L_scene=L_scene,
                                          prev=prev.get(e))
                # by group: a rounding-level branch flip (a kink of the NCP function, a
                # friction mode) lands in linear or angular velocity depending on geometry
                for group in [("rigid_v", "rigid_w", "particle_v"), ("rigid_x", "rigid_q", "particle_x")]:
                    g = max([sens.get(k, 0.0) for k in group])
                    for k in group:
                        if k in tols:
                            tols[k] = max(err_tol, sens_factor * g)
                err["stats_sens"] = sens
            for k, v in err.items():
                if k.startswith("stats"):
                    continue
                if tols[k] > STATE_TOL_CAP:
                    history.capped.append((s, e, k, tols[k], v))
                    continue
                if v > worst.get(k, (-1, None, None))[0]:
                    worst[k] = (v, e, tols[k])
            bad = {k: (v, tols[k]) for k, v in err.items()
                   if not k.startswith("stats") and tols[k] <= STATE_TOL_CAP and v > tols[k]}
            assert not bad, f"step {s} env {e}: (err, tol) {bad}; gpu stats {stats[e]}; oracle {ost}"
        history.append(worst)
    return history


def bucket_sample(scene, n_random=12, seed=0):
    """Envs to check in a full-size batch: a seeded random sample plus the first and
    the last env of every schedule bucket (each block size the launch uses, and the
    largest and smallest env of the batch)."""
    rng = np.random.default_rng(seed)
    n = scene.n_envs
    order = scene.env_order()
    ids = set(int(i) for i in rng.choice(n, size=min(n_random, n), replace=False))
    for first, count, _ in scene.schedule():
        if count > 0:
            ids.add(int(order[first]))
            ids.add(int(order[first + count - 1]))
    return sorted(ids)
