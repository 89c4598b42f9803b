"""Parity of the HIP path (through the C ABI) with the FP64 oracle on identical
pre-step states.  Tolerance 1e-4 relative: positions over max(|x|, 1 m), velocities
over max(|u|, g h), quaternions absolute.

Regimes:
  * per Newton iteration: 1..3 Newton updates of 40 PCR iterations from the same
    pre-step state, on every scene type (every kernel path, incl. geometric
    stiffness at k >= 1 and the warm-start paths).  Where the oracle itself moves by
    more than 1e-5 under FP32-sized perturbations of its input (unconverged
    iterates of FEM + rigid scenes, which share one set of Krylov scalars; kinks of
    the NCP functions), the tolerance of the velocities (or of the positions) is
    10x that group's spread instead;
  * the grasp scene with one PCR iteration per Newton update, where its iterate is
    far better determined than at 40 (same tolerance rule);
  * whole steps at the fixed 10 x 40 budget, several steps in lockstep, on scenes
    whose iterate path is smooth (joints, drives, free bodies, sliding, sticking);
  * converged steps (residual mode) on rigid contact stacks.
"""
import numpy as np
import pytest

import scene_inputs as si
from tests.parity_util import bucket_sample, lockstep, skip_if_capped

pytestmark = pytest.mark.gpu

H = 1.0 / 60.0


def _scene(envs, params=None):
    from paper_1907_04587_amd import Scene
    return Scene(envs, params or si.SolverParams())


def _print(name, hist):
    for s, w in enumerate(hist):
        print(name, s, {k: f"{v[0]:.2e}@{v[1]} (tol {v[2]:.1e})" for k, v in w.items()}, flush=True)


def _driven_chain():
    d = si.batched_env(seed=11, tets_max=0, joints_max=12)
    d.joint_drive[:, 0] = 3.0
    d.joint_drive[:, 1] = 0.1
    d.joint_drive[:, 2] = 0.4
    d.joint_drive[:, 3] = 1.0
    return d


def _rigid_kinds():
    return [
        si.cube_stack(seed=1),
        si.box_on_incline(0.5, 0.3),
        si.particles_vs_planes_lcp(seed=1),
        _driven_chain(),
        si.pendulum_drive(),
    ]


def _all_kinds():
    return _rigid_kinds() + [
        si.tet_block_with_boxes(seed=0, cells=3, n_boxes=3),
        si.single_tet(n_tets=5, deform=[[1.1, 0.02, 0.0], [0.0, 1.0, 0.03], [0.01, 0.0, 0.9]]),
        si.grasp_scene(seed=0, sphere_cell=0.02),
        si.batched_env(seed=1000, tets_max=600),
        si.batched_env(seed=1001, tets_max=600),
    ]


def test_single_particle_worked_example():
    """Fig. rscalingvis: lambda = 1/2 after one r-scaled min-map Newton step (t = 1)."""
    h = 0.5
    d = si.particle_on_plane(v=(0.0, 0.0, -0.25), mass=4 * h * h, mu=0.0, gravity=(0, 0, 0))
    p = si.SolverParams(ncp=1, damping=1.0, eps=0.0)
    sc = _scene([d], p)
    sc.step(h, 1, 10, 0.0)
    c = sc.contacts(0)
    assert len(c["key"]) == 1
    assert c["lam"][0, 0] == pytest.approx(0.5, abs=1e-6)


@pytest.mark.parametrize("newton", [1, 2, 3])
@pytest.mark.parametrize("ncp", [0, 1])
def test_per_newton_iteration_rigid_kinds(newton, ncp):
    """The rigid, contact and joint scenes alone (their states are decidable at 1e-4
    or at the conditioning tolerance below the cap)."""
    envs = _rigid_kinds()
    p = si.SolverParams(ncp=ncp)
    sc = _scene(envs, p)
    hist = lockstep(sc, envs, p, H, newton, 40, steps=1, sens_factor=10.0)
    _print(f"rigid{newton}", hist)
    skip_if_capped(hist)


@pytest.mark.parametrize("newton", [1, 2, 3])
@pytest.mark.parametrize("ncp", [0, 1])
def test_per_newton_iteration_all_scene_kinds(newton, ncp):
    """Every scene kind together; FEM-bearing states often move more than the cap in
    the oracle itself (they are decided row by row in tests/test_gpu_rows.py)."""
    envs = _all_kinds()
    p = si.SolverParams(ncp=ncp)
    sc = _scene(envs, p)
    hist = lockstep(sc, envs, p, H, newton, 40, steps=1, sens_factor=10.0)
    _print(f"iter{newton}", hist)
    skip_if_capped(hist)


@pytest.mark.parametrize("newton", [1, 2])
def test_grasp_single_cr_iteration(newton):
    """Every row type of the grasp scene (prismatic and revolute drives on a 6-DoF
    arm, capsule fingers, FEM sphere on the ground, geometric stiffness) with one PCR
    iteration per Newton update, where the iterate is far better determined than at
    40 (the global Krylov scalars amplify rounding there): 1e-4, or 10x the oracle's
    own spread on sticking-friction particles."""
    envs = [si.grasp_scene(seed=0, sphere_cell=0.02), si.grasp_scene(seed=1, sphere_cell=0.02)]
    p = si.SolverParams()
    sc = _scene(envs, p)
    for s in range(3):  # let the sphere settle on the ground: active contacts and friction
        sc.step(1.0 / 120.0, 10, 40, 0.0)
    hist = lockstep(sc, envs, p, 1.0 / 120.0, newton, 1, steps=1, sens_factor=10.0)
    _print(f"grasp{newton}", hist)
    skip_if_capped(hist)


@pytest.mark.parametrize("newton", [1, 2])
def test_per_newton_iteration_warm_start(newton):
    """Warm-start path (projected previous contact multipliers, previous joint
    multipliers, start-configuration tet stresses, u0 = u^-): the oracle is given the
    GPU's previous-step multipliers, so both sides start from the same lambda0.
    The FEM batched env is checked at N = 1 only: its second update diverges on both
    sides (r_ncp 1.3 -> 9..12), where rounding decides the iterate."""
    envs = [si.cube_stack(seed=2, n=3), _driven_chain(), si.box_on_incline(0.3, 0.6)]
    if newton == 1:
        envs.append(si.batched_env(seed=1002, tets_max=300))
    p = si.SolverParams(warm=si.WARM_PREV)
    sc = _scene(envs, p)
    hist = lockstep(sc, envs, p, H, newton, 40, steps=3, sens_factor=10.0, prev_from_gpu=True)
    _print(f"warm{newton}", hist)
    skip_if_capped(hist)


@pytest.mark.parametrize("newton", [2, 4, 8])
def test_line_search_frictionless(newton):
    """Sec. 8.1's back-tracking line search (full step first, halved on insufficient
    merit decrease) on frictionless contact scenes, against the oracle.  (On the stiff
    driven chain the rounding-level PCR stop falls on different iterations in FP32 and
    FP64, and full steps amplify that; it is left to the damped tests.)"""
    envs = [si.particles_vs_planes_lcp(seed=3), si.cube_stack(seed=4, n=4, mu=0.0),
            si.tet_block_with_boxes(seed=1, cells=3, n_boxes=2, mu=0.0)]
    p = si.SolverParams(line_search=1, damping=1.0)
    sc = _scene(envs, p)
    hist = lockstep(sc, envs, p, H, newton, 40, steps=2, sens_factor=10.0)
    _print(f"linesearch{newton}", hist)
    skip_if_capped(hist)


def test_line_search_converges_in_fewer_iterations():
    """Residual mode on frictionless contact: the line-searched full steps reach
    r_ncp <= 1e-4 (the FP32 floor of a frictionless stack is about 4e-5) in fewer Newton iterations
    than the constant damping t = 0.75."""
    envs = [si.particles_vs_planes_lcp(seed=4), si.cube_stack(seed=6, n=4, mu=0.0)]
    its = {}
    for ls in [0, 1]:
        sc = _scene(envs, si.SolverParams(line_search=ls, damping=1.0 if ls else 0.75))
        tot = np.zeros(len(envs))
        for _ in range(5):
            sc.step(H, 100, 60, 1e-4)
            st = sc.stats()
            assert st["converged"].all(), st
            tot += st["newton_iters"]
        its[ls] = tot
    print("Newton iterations over 5 steps, damped / line search:", its[0], its[1], flush=True)
    assert (its[1] < its[0]).all()


def test_fixed_budget_lockstep_smooth_scenes():
    envs = [si.free_particle(), si.particle_on_plane(v=(0.5, 0.2, 0.0)), si.spinning_box(),
            _driven_chain(), si.pendulum_drive(), si.box_on_incline(0.3, 0.6), si.cube_stack(seed=1, n=2)]
    p = si.SolverParams()
    sc = _scene(envs, p)
    hist = lockstep(sc, envs, p, H, 10, 40, steps=4)
    _print("fixed", hist)


def test_converged_rigid_stack():
    """Residual mode on the 8-cube stack: both sides converge (the GPU to its FP32
    floor) and the states agree."""
    envs = [si.cube_stack(seed=s) for s in range(2)]
    p = si.SolverParams()
    sc = _scene(envs, p)
    hist = lockstep(sc, envs, p, H, 100, 40, tol=1e-5, steps=3, err_tol=3e-4)
    _print("converged", hist)


def test_full_size_batch_sampled():
    """The 4096-env uneven batch at full size, launched as the benchmark launches it
    (default schedule of three block sizes): sampled envs, with the first and last env
    of every bucket, are checked one by one against the oracle (2 Newton iterations)."""
    envs = si.batched_envs(4096, base_seed=1000)
    p = si.SolverParams()
    sc = _scene(envs, p)
    assert len(sc.schedule()) == 3
    sample = bucket_sample(sc)
    hist = lockstep(sc, envs, p, H, 2, 40, steps=1, env_ids=sample, sens_factor=10.0)
    _print("full", hist)
    st = sc.stats()
    assert not st["nonfinite"].any()
    skip_if_capped(hist)


def test_full_size_rigid_batch_sampled():
    """The same 4096 envs without tet blocks: no env carries 1024 rows + DOFs besides
    its contact slots, so the default schedule is one launch of 128 threads per env;
    sampled envs and the ends of the bucket against the oracle (2 Newton iterations)."""
    envs = si.batched_envs(4096, base_seed=1000, tets_max=0)
    p = si.SolverParams()
    sc = _scene(envs, p)
    assert sc.schedule() == [(0, 4096, 128)]
    sample = bucket_sample(sc, seed=3)
    hist = lockstep(sc, envs, p, H, 2, 40, steps=1, env_ids=sample, sens_factor=10.0)
    _print("rigidfull", hist)
    assert not sc.stats()["nonfinite"].any()
    skip_if_capped(hist)


def test_empty_env_and_overflow():
    """An env with no bodies, and contact overflow (capacity below the contact count)."""
    empty = si.scenes._empty(name="empty").finalize()
    over = si.cube_stack(seed=0, n=3)
    over.max_contacts = 5
    envs = [empty, over]
    p = si.SolverParams()
    sc = _scene(envs, p)
    lockstep(sc, envs, p, H, 2, 20, steps=2)
    st = sc.stats()
    assert st["n_contacts"][1] == 5 and st["overflow"][1] > 0
    assert st["n_contacts"][0] == 0 and st["newton_iters"][0] == 2


def test_residual_mode_early_exit():
    """tol > 0: an env stops as soon as r_ncp <= tol; a free particle converges in a
    few iterations while the budget is larger."""
    envs = [si.free_particle(), si.cube_stack(seed=0, n=2)]
    sc = _scene(envs)
    sc.step(H, 50, 40, 1e-4)
    st = sc.stats()
    assert st["converged"][0] == 1 and st["r_ncp"][0] <= 1e-4 and st["newton_iters"][0] < 50


def test_bitwise_deterministic():
    envs = [si.batched_env(seed=2000 + i, tets_max=300) for i in range(4)]
    p = si.SolverParams()
    out = []
    for _ in range(2):
        sc = _scene(envs, p)
        for _ in range(3):
            sc.step(H, 6, 30, 0.0)
        out.append([sc.read_state(e) for e in range(len(envs))])
    for a, b in zip(*out):
        for k in a:
            if k != "time":
                assert np.array_equal(a[k], b[k]), k


def test_graph_replay_matches_direct_launch():
    envs = [si.batched_env(seed=3000 + i, tets_max=300) for i in range(3)]
    res = []
    for graphs in [True, False]:
        sc = _scene(envs)
        sc.set_use_graphs(graphs)
        for _ in range(3):
            sc.step(H, 4, 20, 0.0)
        res.append([sc.read_state(e) for e in range(len(envs))])
    for a, b in zip(*res):
        for k in a:
            if k != "time":
                assert np.array_equal(a[k], b[k]), k


def test_write_read_state_roundtrip_and_resume():
    envs = [si.batched_env(seed=4000, tets_max=200)]
    sc = _scene(envs)
    sc.step(H, 4, 20, 0.0)
    s0 = sc.read_state(0)
    sc.step(H, 4, 20, 0.0)
    s1 = sc.read_state(0)
    sc2 = _scene(envs)
    sc2.write_state(0, s0)
    assert sc2.read_state(0)["time"] == s0["time"]
    sc2.step(H, 4, 20, 0.0)
    # zero warm start: the step depends only on (q, u, t), so the resume is bit-exact
    for k in s1:
        if k != "time":
            assert np.array_equal(sc2.read_state(0)[k], s1[k]), k


@pytest.mark.parametrize("block", [1024, 512, 128])
@pytest.mark.parametrize("ext", [False, True])
def test_lds_modes_bitwise_equal(ext, block):
    """The tets' contributions in LDS (mode 2), the body-space vector alone in LDS (1)
    and everything in global memory (0) sum the same terms in the same order:
    identical states.  ext: linear tets and islands (the
    extended kernel)."""
    envs = [si.batched_env(seed=2100 + i, tets_max=600) for i in range(4)]
    if ext:
        envs += [si.tet_block_with_boxes(seed=1, cells=3, n_boxes=3, tet_model=si.TET_LINEAR)]
    p = si.SolverParams(islands=1 if ext else 0)
    out = []
    for mode in [2, 1, 0]:
        sc = _scene(envs, p)
        sc.set_schedule([(0, len(envs), block)])
        sc.set_lds_mode(mode)
        assert sc.lds_modes() == [mode], (mode, sc.lds_modes())
        for _ in range(3):
            sc.step(H, 6, 30, 0.0)
        out.append([sc.read_state(e) for e in range(len(envs))])
    for other in out[1:]:
        for a, b in zip(out[0], other):
            for k in a:
                if k != "time":
                    assert np.array_equal(a[k], b[k]), k


def test_lds_mode_falls_back_for_large_envs():
    """A 5000-tet env does not fit LDS mode 2 (about 156 KB per workgroup): its bucket
    runs in mode 1, with the same results as in global memory."""
    envs = [si.tet_block_with_boxes(seed=2, cells=10, n_boxes=4)]
    assert envs[0].n_tets == 5000
    out = []
    for mode in [2, 0]:
        sc = _scene(envs)
        sc.set_schedule([(0, 1, 1024)])
        sc.set_lds_mode(mode)
        assert sc.lds_modes() == [1 if mode == 2 else 0]
        sc.step(H, 3, 20, 0.0)
        out.append(sc.read_state(0))
    for k in out[0]:
        if k != "time":
            assert np.array_equal(out[0][k], out[1][k]), k


@pytest.mark.parametrize("block", [512, 256, 128])
def test_register_resident_pcr_bitwise_equal(block):
    """The register-resident PCR (rows of every tet and contact in registers for all the
    PCR iterations of a Newton iteration) and the streaming form sum the same terms in
    the same order: identical states, also with envs too large for their slots (those
    take the streaming form inside the same launch), with the previous-step start and in
    residual mode."""
    envs = [si.batched_env(seed=2200 + i, tets_max=500) for i in range(5)] + [si.cube_stack(seed=3),
                                                                               _driven_chain()]
    for p, tol, n in [(si.SolverParams(), 0.0, 6), (si.SolverParams(warm=si.WARM_PREV), 1e-4, 50)]:
        out = []
        for form in [1, 0]:
            sc = _scene(envs, p)
            sc.set_schedule([(0, len(envs), block)])
            sc.set_pcr_form(form)
            for _ in range(3):
                sc.step(H, n, 30, tol)
            out.append(([sc.read_state(e) for e in range(len(envs))], sc.stats()))
        (sa, ta), (sb, tb) = out
        assert np.array_equal(ta["cr_iters"], tb["cr_iters"])
        for a, b in zip(sa, sb):
            for k in a:
                if k != "time":
                    assert np.array_equal(a[k], b[k]), (block, k)
