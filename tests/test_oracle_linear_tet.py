"""Pins of the oracle's linear Hookean tet (Sec. 9.2, linear materials) and of the
material-extension test (Sec. 11): six co-rotated strains per element, constant
compliance (V_e K_e)^-1.

Independent references: SciPy's polar decomposition for the stretch S (F = R S), the
textbook isotropic energy mu e:e + lambda tr(e)^2 / 2 on the full strain tensor, finite
differences, and the closed-form uniaxial-stress state of linear elasticity (lateral
strain = -nu * axial strain).  All CPU."""
import numpy as np
import pytest
from scipy.linalg import polar
from scipy.spatial.transform import Rotation

import scene_inputs as si
from oracle import oracle as O

E_Y, NU = 1e5, 0.45
MU = E_Y / (2 * (1 + NU))
LA = E_Y * NU / ((1 + NU) * (1 - 2 * NU))
PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]  # Sec. 9.2 order xx yy zz yz xz xy
REST = np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0], [0.0, 0.1, 0.0], [0.02, 0.01, 0.1]])


def _Dm(rest):
    return np.stack([rest[k] - rest[0] for k in (1, 2, 3)], axis=1)


def _F(x, rest):
    return np.stack([x[k] - x[0] for k in (1, 2, 3)], axis=1) @ np.linalg.inv(_Dm(rest))


def _energy(x, rest):
    """V_e (mu |S - I|^2 + lambda tr(S - I)^2 / 2), S from SciPy's polar decomposition."""
    _, S = polar(_F(x, rest))
    e = S - np.eye(3)
    Ve = abs(np.linalg.det(_Dm(rest))) / 6
    return Ve * (MU * (e * e).sum() + 0.5 * LA * np.trace(e) ** 2)


def _tet(x, rest=REST):
    Ve = abs(np.linalg.det(_Dm(rest))) / 6
    return O.linear_tet(np.linalg.inv(_Dm(rest)), x, E_Y, NU, Ve)


def _deformed(seed, scale=0.15):
    rng = np.random.default_rng(seed)
    F = np.eye(3) + rng.uniform(-scale, scale, (3, 3))
    R = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    c = REST.mean(0)
    return c + (REST - c) @ (R @ F).T + rng.normal(scale=1e-3, size=(4, 3)), R


def test_rest_and_rigid_motion_are_strain_free():
    """Co-rotation: a rigid rotation plus translation produces no strain and no stress."""
    eps, _, c, _ = _tet(REST)
    np.testing.assert_allclose(eps, 0.0, atol=1e-14)
    for seed in range(5):
        R = Rotation.from_rotvec(np.random.default_rng(seed).normal(size=3) * 2).as_matrix()
        eps, _, c, _ = _tet(REST @ R.T + [0.3, -1.0, 2.0])
        np.testing.assert_allclose(eps, 0.0, atol=1e-13)
        np.testing.assert_allclose(c, 0.0, atol=1e-8)


@pytest.mark.parametrize("seed", range(4))
def test_strain_is_polar_stretch_minus_identity(seed):
    """s = S - I of the polar decomposition F = R S (SciPy), tensor shear components in
    the paper's order."""
    x, _ = _deformed(seed)
    _, S = polar(_F(x, REST))
    eps, _, _, _ = _tet(x)
    ref = [S[a, b] - (a == b) for a, b in PAIRS]
    np.testing.assert_allclose(eps, ref, atol=1e-12)


def test_stress_and_compliance_of_isotropic_hooke():
    """c = V_e K_e s: s.c / 2 is the textbook energy V_e (mu e:e + lambda tr(e)^2 / 2) of
    the full strain tensor, and the compliance is the inverse of V_e K_e."""
    x, _ = _deformed(7)
    eps, _, c, Cm = _tet(x)
    e = np.zeros((3, 3))
    for q, (a, b) in enumerate(PAIRS):
        e[a, b] = e[b, a] = eps[q]
    Ve = abs(np.linalg.det(_Dm(REST))) / 6
    assert 0.5 * eps @ c == pytest.approx(Ve * (MU * (e * e).sum() + 0.5 * LA * np.trace(e) ** 2), rel=1e-12)
    # K_e from the stress of unit strains (the oracle's c is linear in s)
    K = np.zeros((6, 6))
    for q in range(6):
        u = np.zeros(6); u[q] = 1.0
        ue = np.zeros((3, 3))
        a, b = PAIRS[q]
        ue[a, b] = ue[b, a] = 1.0
        sig = 2 * MU * ue + LA * np.trace(ue) * np.eye(3)   # Hooke's law on the tensor
        K[:, q] = [sig[a2, b2] * (1 if a2 == b2 else 2) for a2, b2 in PAIRS]
    np.testing.assert_allclose(Cm @ (Ve * K), np.eye(6), atol=1e-12)
    np.testing.assert_allclose(c, Ve * K @ eps, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("seed", range(4))
def test_rows_are_strain_derivative_at_fixed_rotation(seed):
    """Rows ds/dx with R frozen: e_R(x) = sym(R^T F(x)) - I is linear in x, so central
    differences of it are exact up to rounding."""
    x, _ = _deformed(seed)
    R, _ = polar(_F(x, REST))
    _, rows, _, _ = _tet(x)

    def eR(xx):
        G = R.T @ _F(xx, REST)
        G = 0.5 * (G + G.T) - np.eye(3)
        return np.array([G[a, b] for a, b in PAIRS])

    h = 1e-6
    for j in range(4):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[j, k] += h; xm[j, k] -= h
            np.testing.assert_allclose(rows[:, j, k], (eR(xp) - eR(xm)) / (2 * h), atol=1e-7)


@pytest.mark.parametrize("seed", range(4))
def test_force_is_exact_energy_gradient(seed):
    """For isotropic K_e the fixed-rotation rows give the exact elastic force:
    J^T c = dU/dx with U from SciPy's polar stretch (central differences)."""
    x, _ = _deformed(seed, scale=0.3)
    _, rows, c, _ = _tet(x)
    f = np.einsum("qjk,q->jk", rows, c)
    h = 1e-7
    g = np.zeros((4, 3))
    for j in range(4):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[j, k] += h; xm[j, k] -= h
            g[j, k] = (_energy(xp, REST) - _energy(xm, REST)) / (2 * h)
    assert np.abs(g).max() > 10.0
    np.testing.assert_allclose(f, g, rtol=1e-6, atol=1e-6 * np.abs(g).max())


@pytest.mark.parametrize("n_tets", [1, 5])
def test_linear_fem_step_is_variational_implicit_euler(n_tets):
    """A converged contact-free step with linear tets satisfies
    M (u+ - u~) + h grad U(x- + h u+) = 0, U the sum of the co-rotated energies above."""
    h = 1 / 60
    F = [[1.15, 0.05, 0.0], [0.0, 1.0, 0.03], [0.02, 0.0, 0.85]]
    d = si.single_tet(perturb=1e-3, seed=n_tets, n_tets=n_tets, deform=F, tet_model=si.TET_LINEAR)
    env = O.OracleEnv(d)
    st = env.step(h, 100, 60, 1e-10, O.make_params(si.SolverParams(warm=si.WARM_ZERO)))
    assert st["r_ncp"] < 1e-8, st
    S = env.get_state()
    x, u = S["particle_x"], S["particle_v"]
    m = np.zeros(d.n_particles)
    for t in d.tet_ids:
        m[t] += 1000.0 * abs(np.linalg.det(_Dm(d.particle_rest[t]))) / 6 / 4

    def U(xx):
        return sum(_energy(xx[t], d.particle_rest[t]) for t in d.tet_ids)

    grad = np.zeros_like(x)
    e = 1e-7
    for p in range(d.n_particles):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[p, a] += e; xm[p, a] -= e
            grad[p, a] = (U(xp) - U(xm)) / (2 * e)
    res = (m[:, None] * (u - d.particle_v) + h * grad) / m[:, None]
    assert np.abs(h * grad / m[:, None]).max() > 0.1
    assert np.abs(res).max() < 1e-5


@pytest.mark.parametrize("stretch", [0.1, 1.0])
def test_extension_bar_uniaxial_poisson_ratio(stretch):
    """A pre-stretched linear bar held at its ends relaxes to uniaxial stress in its
    middle, where linear elasticity fixes lateral strain = -nu * axial strain (the
    co-rotated strain makes this hold at any stretch)."""
    d = si.extension_bar(stretch, si.TET_LINEAR)
    env = O.OracleEnv(d)
    p = O.make_params(si.SolverParams(warm=si.WARM_PREV))
    for _ in range(40):
        st = env.step(1 / 60, 50, 100, 1e-5, p)
        assert st["r_ncp"] < 1e-5
    ax, lat, _ = _mid_section(d, env.get_state()["particle_x"])
    assert ax - 1 == pytest.approx(stretch, rel=0.15)
    assert -(lat - 1) / (ax - 1) == pytest.approx(NU, abs=2e-3)


def _mid_section(d, x, cell=0.05):
    r = d.particle_rest
    nx = int(round(r[:, 0].max() / cell))
    sel = lambda i: np.abs(r[:, 0] - i * cell) < 1e-6
    c = sel(nx // 2)
    ny = (r[:, 1].max() - r[:, 1].min())
    nz = (r[:, 2].max() - r[:, 2].min())
    lat = 0.5 * ((x[c, 1].max() - x[c, 1].min()) / ny + (x[c, 2].max() - x[c, 2].min()) / nz)
    ax = (x[sel(nx // 2 + 1), 0].mean() - x[sel(nx // 2 - 1), 0].mean()) / (2 * cell)
    return ax, lat, ax * lat * lat


def test_material_extension_linear_loses_volume_hyperelastic_keeps_it():
    """The material-extension test: a bar pulled to about twice its length.  The linear
    co-rotated model follows (1 + e)(1 - nu e)^2 in the middle (a 47% volume loss at
    e = 1.1); the stable neo-Hookean model keeps the volume within a few percent."""
    out = {}
    for model in (si.TET_LINEAR, si.TET_NEOHOOKEAN):
        d = si.extension_bar(0.0, model, speed=0.25)
        env = O.OracleEnv(d)
        p = O.make_params(si.SolverParams(warm=si.WARM_PREV))
        for _ in range(72):
            st = env.step(1 / 60, 50, 100, 1e-5, p)
            assert not st["nonfinite"]
        out[model] = _mid_section(d, env.get_state()["particle_x"])
    ax, lat, J = out[si.TET_LINEAR]
    assert ax > 2.0
    assert J == pytest.approx(ax * (1 - NU * (ax - 1)) ** 2, rel=1e-2)
    assert J < 0.6
    assert abs(out[si.TET_NEOHOOKEAN][2] - 1.0) < 0.1
