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


def lockstep(scene, envs, params, h, N, M, tol=0.0, steps=1, env_ids=None, check_contacts=True,
             err_tol=1e-4, L_scene=1.0):
    """Step the GPU scene `steps` times; before each step copy every checked env's
    state into a fresh oracle env and step it too; compare after each step.
    Returns the list of per-step error dicts (worst over envs)."""
    if env_ids is None:
        env_ids = list(range(len(envs)))
    op = O.make_params(params)
    orcs = {e: O.OracleEnv(envs[e]) for e in env_ids}
    history = []
    for s in range(steps):
        pre = {e: scene.read_state(e) for e in env_ids}
        scene.step(h, N, M, tol)
        stats = scene.stats()
        worst = {}
        for e in env_ids:
            oe = orcs[e]
            oe.set_state({k: np.asarray(v, np.float64) for k, v in pre[e].items() if k != "time"})
            oe.time = pre[e]["time"]
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
            for k, v in err.items():
                if k.startswith("stats"):
                    continue
                if v > worst.get(k, (-1, None))[0]:
                    worst[k] = (v, e)
            bad = {k: v for k, v in err.items() if not k.startswith("stats") and v > err_tol}
            assert not bad, f"step {s} env {e}: {bad}; gpu stats {stats[e]}; oracle {ost}"
        history.append(worst)
    return history
