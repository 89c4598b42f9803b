"""Learned warm start on the GPU: feature parity with the oracle, parity of the
projected MLP start multipliers, and what the trained network gains.

The gain is measured where the network acts: how close its start multipliers are to
the multipliers the solver ends a step with, against the previous step's multipliers
(the plain warm start), and in Newton / PCR iterations to r_ncp <= 1e-4 on held-out
rigid batches against the paper's zero start.  On the grasp distribution no start
reaches r_ncp <= 1e-4 within 50 Newton iterations (the friction and tet rows of the
soft sphere stall), so the iteration counts there are reported, not asserted."""
import os

import numpy as np
import pytest

import scene_inputs as si
from oracle import oracle as O

pytestmark = pytest.mark.gpu

H_GRASP = 1.0 / 120.0
WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1907_04587_amd",
                       "weights", "warm_start_grasp.npy")


def _scene(envs, p):
    from paper_1907_04587_amd import Scene
    return Scene(envs, p)


def _blob():
    return np.load(WEIGHTS, allow_pickle=False)


def _prev_of(sc, e, d):
    c = sc.contacts(e)
    lj = sc.lambdas(e)[:6 * d.n_joints]
    return c["key"], np.asarray(c["lam"], np.float64), np.asarray(lj, np.float64)


def test_contact_features_match_oracle():
    """The 12 step-start features (normal and tangential velocity under u~,
    penetration, previous multipliers, inverse masses, mu, n_z, previous-contact flag)
    against the oracle given the same state and previous-step multipliers."""
    envs = [si.grasp_scene(seed=5, sphere_cell=0.02), si.batched_env(seed=1500, tets_max=300), si.cube_stack(seed=3)]
    p = si.SolverParams(warm=si.WARM_PREV)
    sc = _scene(envs, p)
    sc.enable_features(True)
    for _ in range(3):
        sc.step(H_GRASP, 10, 40, 0.0)
    prev = [_prev_of(sc, e, d) for e, d in enumerate(envs)]
    pre = [sc.read_state(e) for e in range(len(envs))]
    sc.step(H_GRASP, 10, 40, 0.0)
    for e, d in enumerate(envs):
        fg = sc.features(e)
        kg = sc.contacts(e)["key"]
        oe = O.OracleEnv(d)
        oe.set_state({k: np.asarray(v, np.float64) for k, v in pre[e].items() if k != "time"})
        oe.time = pre[e]["time"]
        oe.set_prev(*prev[e])
        fo, ko = oe.contact_features(H_GRASP, O.make_params(p))
        assert np.array_equal(kg, ko), e
        assert len(fg) == len(fo) and len(fg) > 0
        # floors: velocities g h, penetration 1 m (a millimetre gap is the difference of
        # metre-scale FP32 positions), multipliers and the rest their own scale
        floor = np.array([9.81 * H_GRASP] * 3 + [1.0] + [1e-6] * 8)
        scale = np.maximum(np.abs(fo).max(0), floor)
        err = (np.abs(fg - fo) / scale).max(0)
        print("features env", e, "max rel err per column", np.array2string(err, precision=1), flush=True)
        assert (err < 2e-5).all(), (e, err)


@pytest.mark.parametrize("mode", [si.WARM_LEARNED, si.WARM_HYBRID])
def test_learned_start_multipliers_match_oracle(mode):
    """Zero Newton iterations leave the start multipliers in the state: the projected
    BF16-MFMA prediction (in hybrid mode only for new contacts; persisting ones keep
    the previous-step multipliers) against the oracle's FP64 MLP on the same features.
    BF16 rounds weights and activations to 2^-9 relative; 3e-2 of the output scale is
    several times that and far below a layout or projection mistake.  The check is
    made after 3 to 6 steps; in hybrid mode some of them must hold both new and
    persisting contacts."""
    blob = _blob()
    envs = [si.grasp_scene(seed=6, sphere_cell=0.02), si.grasp_scene(seed=7, sphere_cell=0.02)]
    p = si.SolverParams(warm=mode)
    mixed = 0
    for n_pre in (3, 4, 5, 6):
        sc = _scene(envs, p)
        sc.set_warm_start_model(blob)
        for _ in range(n_pre):
            sc.step(H_GRASP, 10, 40, 0.0)
        prev = [_prev_of(sc, e, d) for e, d in enumerate(envs)]
        pre = [sc.read_state(e) for e in range(len(envs))]
        sc.step(H_GRASP, 0, 40, 0.0)
        for e, d in enumerate(envs):
            cg = sc.contacts(e)
            oe = O.OracleEnv(d)
            oe.set_mlp(blob)
            oe.set_state({k: np.asarray(v, np.float64) for k, v in pre[e].items() if k != "time"})
            oe.time = pre[e]["time"]
            oe.set_prev(*prev[e])
            oe.step(H_GRASP, 0, 40, 0.0, O.make_params(p))
            co = oe.contacts()
            assert np.array_equal(cg["key"], co["key"])
            lg, lo = np.asarray(cg["lam"], np.float64), co["lam"]
            scale = np.abs(lo).max() + 1e-9
            err = np.abs(lg - lo).max() / scale
            known = np.isin(cg["key"], prev[e][0])
            print("start multipliers after", n_pre, "steps, env", e, "contacts", len(lo), "new",
                  int((~known).sum()), "max err / scale", f"{err:.2e}", flush=True)
            assert err < 3e-2
            if mode == si.WARM_HYBRID:
                # persisting contacts keep the previous-step multipliers exactly
                pk = dict(zip(prev[e][0].tolist(), prev[e][1]))
                for k, l in zip(cg["key"][known], lg[known]):
                    p0 = pk[int(k)]
                    lim = d.mu * max(p0[0], 0.0)
                    if np.hypot(p0[1], p0[2]) <= lim * (1 - 1e-5):  # inside the cone: kept as is
                        # (the start projection clamps lambda_n at zero: a slightly
                        # negative previous lambda_n starts from 0)
                        want = p0.astype(np.float32).astype(np.float64)
                        want[0] = max(want[0], 0.0)
                        np.testing.assert_array_equal(l, want)
                mixed += int(known.any() and (~known).any())
            # the cone projection holds exactly on the GPU side too
            lf = np.hypot(lg[:, 1], lg[:, 2])
            assert (lg[:, 0] >= 0).all() and (lf <= d.mu * lg[:, 0] * (1 + 1e-5) + 1e-7).all()
    if mode == si.WARM_HYBRID:
        assert mixed > 0


def test_trained_network_gain_on_held_out_grasps():
    """Held-out grasp seeds (disjoint from training and validation): the network's
    start multipliers are closer to the solver's final multipliers than the previous
    step's are (coefficient of determination per component)."""
    from paper_1907_04587_amd.warmstart import predict
    blob = _blob()
    envs = [si.grasp_scene(seed=300_000 + i, sphere_cell=0.02) for i in range(32)]
    p = si.SolverParams(warm=si.WARM_PREV)
    sc = _scene(envs, p)
    sc.enable_features(True)
    xs, ts = [], []
    for s in range(12):
        sc.step(H_GRASP, 50, 40, 1e-6)
        if s < 4:
            continue
        for e in range(len(envs)):
            f = sc.features(e)
            if len(f):
                xs.append(f)
                ts.append(sc.contacts(e)["lam"][:len(f)])
    x, t = np.concatenate(xs), np.concatenate(ts).astype(np.float64)
    pred = predict(blob, x).astype(np.float64)
    ss_tot = ((t - t.mean(0)) ** 2).sum(0)
    r2_net = 1 - ((pred - t) ** 2).sum(0) / ss_tot
    r2_prev = 1 - ((x[:, 4:7] - t) ** 2).sum(0) / ss_tot
    print("held-out contacts", len(x), "R^2 network", np.round(r2_net, 3), "previous step", np.round(r2_prev, 3),
          flush=True)
    assert r2_net[0] > r2_prev[0] and r2_net[0] > 0.5
    assert (r2_net > r2_prev).all()
    # iterations at r_ncp <= 1e-4 (reported)
    for name, mode in [("zero", si.WARM_ZERO), ("prev", si.WARM_PREV), ("learned", si.WARM_LEARNED)]:
        sc2 = _scene(envs, si.SolverParams(warm=mode))
        if mode == si.WARM_LEARNED:
            sc2.set_warm_start_model(blob)
        for _ in range(8):
            sc2.step(H_GRASP, 50, 40, 1e-4)
        st = sc2.stats()
        print(f"arm {name}: mean Newton iterations {st['newton_iters'].mean():.1f}, converged "
              f"{st['converged'].mean():.2f}, median r_first {np.median(st['r_ncp_first']):.2e}, "
              f"median r_contact {np.median(st['r_contact']):.2e}", flush=True)
        assert not st["nonfinite"].any()


def test_nonfinite_learned_start_falls_back_to_plain_start():
    """A model that predicts lambda_n = 3e38 overflows the FP32 residual; each such
    step is rerun from the plain start and then equals the plain step bitwise."""
    from paper_1907_04587_amd.warmstart import N_PARAMS
    blob = np.zeros(N_PARAMS + 30, np.float32)
    blob[N_PARAMS + 12:N_PARAMS + 24] = 1.0  # x_std
    blob[N_PARAMS + 24] = 3e38               # y_mean of lambda_n
    blob[N_PARAMS + 27:N_PARAMS + 30] = 1.0  # y_std
    envs = [si.cube_stack(seed=4, n=3), si.cube_stack(seed=5, n=2)]
    sw = _scene(envs, si.SolverParams(warm=si.WARM_LEARNED))
    sw.set_warm_start_model(blob)
    sz = _scene(envs, si.SolverParams(warm=si.WARM_ZERO))
    for s in range(3):
        sw.step(1 / 60, 6, 30, 0.0)
        sz.step(1 / 60, 6, 30, 0.0)
        st = sw.stats()
        assert (st["fallback"] == 1).all() and not st["nonfinite"].any(), st
        for e in range(len(envs)):
            a, b = sw.read_state(e), sz.read_state(e)
            for k in a:
                if k != "time":
                    assert np.array_equal(a[k], b[k]), (s, e, k)
    assert (sw.accumulators()["fallbacks"] == 3).all()


def test_learned_mode_needs_a_model():
    """Stepping in a learned mode before a model is set is refused (no launch)."""
    from paper_1907_04587_amd._lib import NSNError
    for mode in (si.WARM_LEARNED, si.WARM_HYBRID):
        sc = _scene([si.cube_stack(seed=1, n=2)], si.SolverParams(warm=mode))
        with pytest.raises(NSNError):
            sc.step(1 / 60, 2, 10, 0.0)
        sc.set_warm_start_model(_blob())
        sc.step(1 / 60, 2, 10, 0.0)
        assert not sc.stats()["nonfinite"].any()


def test_learned_start_iterations_saved_on_held_out_rigid_batches():
    """Newton and PCR iterations per env-step to reach r_ncp <= 1e-4 (cap 50 x 40) on
    two held-out sets of 512 rigid envs (seeds disjoint from the training, validation,
    test and benchmark seeds), after three settling steps, over eight steps.  Asserted:
    the learned and hybrid starts save at least 25% of the Newton iterations of the
    paper's start (zero), on each set.  Reported: the previous-step start, which stays
    ahead of both learned starts on these envs (persisting contacts make the previous
    multipliers nearly exact; the network's prediction is percent-level), so the
    learned starts do not beat the stronger plain start here."""
    blob = np.load(os.path.join(os.path.dirname(WEIGHTS), "warm_start_batched.npy"), allow_pickle=False)
    for base in (500_000, 600_000):
        envs = si.batched_envs(512, base_seed=base, tets_max=0)
        out = {}
        for name, mode in [("zero", si.WARM_ZERO), ("prev", si.WARM_PREV), ("learned", si.WARM_LEARNED),
                           ("hybrid", si.WARM_HYBRID)]:
            sc = _scene(envs, si.SolverParams(warm=mode))
            if mode in (si.WARM_LEARNED, si.WARM_HYBRID):
                sc.set_warm_start_model(blob)
            for _ in range(3):
                sc.step(1 / 60, 50, 40, 1e-4)
            sc.reset_accumulators()
            for _ in range(8):
                sc.step(1 / 60, 50, 40, 1e-4)
                assert not sc.stats()["nonfinite"].any()
            acc = sc.accumulators()
            steps = max(int(acc["steps"].sum()), 1)
            out[name] = (float(acc["newton_iters"].sum()) / steps, float(acc["cr_iters"].sum()) / steps,
                         int(acc["converged"].sum()) / steps)
            print(f"seeds {base}+: arm {name}: Newton {out[name][0]:.2f}, PCR {out[name][1]:.1f} per env-step, "
                  f"converged {100 * out[name][2]:.2f}%", flush=True)
        for arm in ("learned", "hybrid"):
            assert out[arm][0] <= 0.75 * out["zero"][0], (base, arm, out)
