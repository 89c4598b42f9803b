"""Linear Hookean tets (Sec. 9.2, six co-rotated strain rows per tet) on the GPU:
parity with the FP64 oracle per Newton iteration and over converged steps, the
uniaxial Poisson ratio of a stretched bar, and the material-extension comparison
with the neo-Hookean model.

Scenes that hold linear tets run the linear-capable instantiation of the Newton
kernel, which must also keep the neo-Hookean and rigid envs of the same batch exact;
the mixed batch below checks that."""
import numpy as np
import pytest

import scene_inputs as si
from oracle import oracle as O
from tests.parity_util import bucket_sample, lockstep, skip_if_capped

pytestmark = pytest.mark.gpu

H = 1.0 / 60.0
NU = 0.45
DEFORM = [[1.1, 0.02, 0.0], [0.0, 1.0, 0.03], [0.01, 0.0, 0.9]]


def _scene(envs, params=None):
    from paper_1907_04587_amd import Scene
    return Scene(envs, params or si.SolverParams())


def _print(name, hist):
    for s, w in enumerate(hist):
        print(name, s, {k: f"{v[0]:.2e}@{v[1]} (tol {v[2]:.1e})" for k, v in w.items()}, flush=True)


def _linear_kinds():
    return [
        si.single_tet(n_tets=5, deform=DEFORM, tet_model=si.TET_LINEAR),
        si.single_tet(n_tets=1, perturb=1e-3, seed=3, deform=DEFORM, tet_model=si.TET_LINEAR),
        si.tet_block_with_boxes(seed=0, cells=3, n_boxes=3, tet_model=si.TET_LINEAR),
        si.extension_bar(0.3, si.TET_LINEAR, nx=6),
        # the same batch also holds a neo-Hookean tet env and a rigid stack
        si.single_tet(n_tets=5, deform=DEFORM),
        si.cube_stack(seed=1),
    ]


@pytest.mark.parametrize("newton", [1, 2, 3])
@pytest.mark.parametrize("ncp", [0, 1])
def test_per_newton_iteration_linear_tets(newton, ncp):
    envs = _linear_kinds()
    p = si.SolverParams(ncp=ncp)
    sc = _scene(envs, p)
    lam = sc.lambdas(0)
    assert len(lam) == 6 * envs[0].n_tets
    hist = lockstep(sc, envs, p, H, newton, 40, steps=1, sens_factor=10.0)
    _print(f"lin{newton}", hist)
    skip_if_capped(hist)


@pytest.mark.parametrize("newton", [1, 2])
def test_per_newton_iteration_linear_tets_warm_start(newton):
    """Warm start: the start-configuration stress -V_e K_e s(q^-) of every linear tet."""
    envs = _linear_kinds()
    p = si.SolverParams(warm=si.WARM_PREV)
    sc = _scene(envs, p)
    hist = lockstep(sc, envs, p, H, newton, 40, steps=3, sens_factor=10.0, prev_from_gpu=True)
    _print(f"linwarm{newton}", hist)
    skip_if_capped(hist)


def test_converged_linear_steps_lockstep():
    """Residual mode (r_ncp <= 1e-4, the FP32 path's level: its residual stalls at a few
    1e-5 here), several steps in lockstep: linear tets converge in a few Newton
    iterations (constant compliance), so whole steps agree to 1e-4."""
    envs = [si.extension_bar(0.3, si.TET_LINEAR, nx=6),
            si.single_tet(n_tets=5, deform=DEFORM, tet_model=si.TET_LINEAR)]
    p = si.SolverParams(warm=si.WARM_PREV)
    sc = _scene(envs, p)
    hist = lockstep(sc, envs, p, H, 50, 100, tol=1e-4, steps=3, prev_from_gpu=True)
    _print("linconv", hist)
    st = sc.stats()
    assert st["converged"].all(), st


def _mid_section(d, x, cell=0.05):
    r = d.particle_rest
    nx = int(round(r[:, 0].max() / cell))
    sel = lambda i: np.abs(r[:, 0] - i * cell) < 1e-6
    c = sel(nx // 2)
    wy = r[:, 1].max() - r[:, 1].min()
    wz = r[:, 2].max() - r[:, 2].min()
    lat = 0.5 * ((x[c, 1].max() - x[c, 1].min()) / wy + (x[c, 2].max() - x[c, 2].min()) / wz)
    ax = (x[sel(nx // 2 + 1), 0].mean() - x[sel(nx // 2 - 1), 0].mean()) / (2 * cell)
    return ax, lat, ax * lat * lat


def test_extension_bar_uniaxial_poisson_ratio_gpu():
    """The middle of a pre-stretched linear bar relaxes to uniaxial stress: lateral
    strain = -nu * axial strain (closed form of linear elasticity).  At twice the
    length the elastic forces over the particle masses put the FP32 residual's floor
    near 1e-4, so the residual is only required to be far below the elastic scale."""
    envs = [si.extension_bar(s, si.TET_LINEAR) for s in (0.1, 1.0)]
    sc = _scene(envs, si.SolverParams(warm=si.WARM_PREV))
    for _ in range(40):
        sc.step(H, 50, 100, 1e-4)
    st = sc.stats()
    assert (st["r_ncp"] < 1e-3).all(), st
    for e, d in enumerate(envs):
        ax, lat, _ = _mid_section(d, sc.read_state(e)["particle_x"])
        nu_eff = -(lat - 1) / (ax - 1)
        print("stretch", [0.1, 1.0][e], "axial", ax, "lateral", lat, "nu_eff", nu_eff, flush=True)
        assert nu_eff == pytest.approx(NU, abs=3e-3)


def test_material_extension_volume_gpu():
    """Bars pulled to about twice their length, linear and neo-Hookean in one batch:
    the linear middle section follows (1 + e)(1 - nu e)^2 (about half the volume), the
    neo-Hookean one keeps its volume within 10%; the linear bar also matches the
    oracle's end state."""
    envs = [si.extension_bar(0.0, si.TET_LINEAR, speed=0.25), si.extension_bar(0.0, si.TET_NEOHOOKEAN, speed=0.25)]
    p = si.SolverParams(warm=si.WARM_PREV)
    sc = _scene(envs, p)
    for _ in range(72):
        sc.step(H, 50, 100, 1e-4)
        assert not sc.stats()["nonfinite"].any()
    ax, lat, J = _mid_section(envs[0], sc.read_state(0)["particle_x"])
    print("linear: axial", ax, "lateral", lat, "J", J, flush=True)
    assert ax > 2.0
    assert J == pytest.approx(ax * (1 - NU * (ax - 1)) ** 2, rel=1e-2)
    _, _, Jn = _mid_section(envs[1], sc.read_state(1)["particle_x"])
    print("neo-Hookean: J", Jn, flush=True)
    assert abs(Jn - 1.0) < 0.1
    oe = O.OracleEnv(envs[0])
    op = O.make_params(p)
    for _ in range(72):
        oe.step(H, 50, 100, 1e-4, op)
    xo, xg = oe.get_state()["particle_x"], sc.read_state(0)["particle_x"]
    assert np.abs(xo - xg).max() / np.abs(xo).max() < 1e-4


def test_full_size_linear_batch_sampled():
    """The 4096-env uneven batch with linear tet blocks at full size, in the default
    schedule (the extended instantiation, 512 and 128 threads): sampled envs and the
    ends of every bucket against the oracle, 2 Newton iterations."""
    envs = si.batched_envs(4096, base_seed=1000, tet_model=si.TET_LINEAR)
    p = si.SolverParams()
    sc = _scene(envs, p)
    assert [b[2] for b in sc.schedule()] == [512, 128]  # linear tets: no 1024-thread bucket
    sample = bucket_sample(sc, seed=1)
    hist = lockstep(sc, envs, p, H, 2, 40, steps=1, env_ids=sample, sens_factor=10.0)
    _print("linfull", hist)
    assert not sc.stats()["nonfinite"].any()
    skip_if_capped(hist)
