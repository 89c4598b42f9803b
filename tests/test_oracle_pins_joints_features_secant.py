"""Pins of three oracle functions that the state-level pins do not reach, each with
a planted-mistake check: a copy of the oracle source with one plausible mistake
(a flipped sign, a wrong frame vector, a wrong operand) is compiled on the CPU and
the same pin must fail on it.

  * prismatic joint rows (Sec. 3 hard bilateral rows; the paper gives no formulas,
    reading: 2 point-on-axis rows, 3 orientation rows, the implicit-PD drive row):
    closed-form driven slider; relative spin about the axis locked with angular
    momentum conserved; transverse impulse on a two-body slider (rigid composite);
  * the 12 warm-start features of a contact, computed by hand from the definitions;
  * the diagonal geometric-stiffness secant (Sec. 8.3, eq. broyden_update and the
    H~ update), against the analytic Hessian of the singular values of a
    tetrahedron's deformation gradient.

All tests here run on the CPU (`-m "not gpu"`)."""
import math
import os

import numpy as np
import pytest

import scene_inputs as si
from oracle import build as obuild
from oracle import oracle as O
from scene_inputs import scenes as S

H = 1.0 / 60.0


# --------------------------------------------------------------------------
# planted mistakes: a variant of the oracle source with one substitution
# --------------------------------------------------------------------------
_SRC = open(obuild.SRC).read()


def mutant(tmp_path, old, new, tag):
    assert _SRC.count(old) == 1, f"mutation site not found once: {old!r}"
    src = tmp_path / f"mut_{tag}.c"
    src.write_text(_SRC.replace(old, new))
    return obuild.build(src=str(src), out=str(tmp_path / f"libmut_{tag}.so"))


def _finalize(d):
    return d.finalize()


# --------------------------------------------------------------------------
# prismatic joints
# --------------------------------------------------------------------------
def _slider_world(x0=0.13, v=(0.4, 0.5, 0.3), w=(1.0, 2.0, 3.0), kp=40.0, kd=0.8, target=0.05, m=1.5):
    """A box (no collision geometry) on a prismatic joint to the world along world x,
    anchor at its centre, driven by implicit PD towards `target`; gravity along -z
    (across the axis).  It starts on the axis with velocity v and spin w."""
    half = np.array([0.05, 0.04, 0.03])
    b = S._nocollide(S._box(m, half, (x0, 0.0, 1.0), v=v, w=w))
    d = S._empty(ground=0, mu=0.0)
    S._set_rigid(d, [b])
    ex, ey = (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)
    S._set_joints(d, [S._prismatic(-1, 0, (0.0, 0.0, 1.0), (0, 0, 0), ex, ex, ey, ey,
                                   drive=(kp, kd, 0.0, 0.0, 0.0, target))])
    return _finalize(d)


def _run_converged(d, lib_path=None, h=H, steps=1):
    env = O.OracleEnv(d, lib_path=lib_path)
    for _ in range(steps):
        st = env.step(h, 80, 80, 1e-12, O.make_params(damping=1.0, line_search=0))
    return env, st


def _check_slider(env, d, h=H):
    """Implicit PD on the axis (reading of the drive: backward Euler, compliance
    1/(kp + kd/h)): v+ = (m v- - h kp (x- - x*)) / (m + h^2 kp + h kd); the point-on-axis
    rows hold the transverse position; the orientation rows remove the spin."""
    s = env.get_state()
    m = d.rigid_mass[0]
    kp, kd, x_star = d.joint_drive[0, 0], d.joint_drive[0, 1], d.joint_drive[0, 5]
    x0, v0 = d.rigid_x[0, 0], d.rigid_v[0, 0]
    v_exp = (m * v0 - h * kp * (x0 - x_star)) / (m + h * h * kp + h * kd)
    assert s["rigid_v"][0, 0] == pytest.approx(v_exp, rel=1e-9, abs=1e-12)
    assert s["rigid_x"][0, 0] == pytest.approx(x0 + h * v_exp, rel=1e-9)
    np.testing.assert_allclose(s["rigid_v"][0, 1:], 0.0, atol=1e-9)
    np.testing.assert_allclose(s["rigid_x"][0, 1:], [0.0, 1.0], atol=1e-10)
    np.testing.assert_allclose(s["rigid_w"][0], 0.0, atol=1e-9)
    np.testing.assert_allclose(np.abs(s["rigid_q"][0]), [1.0, 0.0, 0.0, 0.0], atol=1e-10)


def test_prismatic_driven_slider_closed_form():
    d = _slider_world()
    env, st = _run_converged(d)
    assert st["r_ncp"] < 1e-10
    _check_slider(env, d)


def _spin_pair(wA=(2.0, 0.0, 0.0), wB=(-3.0, 0.0, 0.0), mA=1.0, mB=2.0, gap=0.3):
    """Two cubes (isotropic inertia) joined by a prismatic joint along x through both
    centres, no gravity: a relative spin about the axis only."""
    hA, hB = 0.05, 0.07
    a = S._nocollide(S._box(mA, (hA, hA, hA), (0.0, 0.0, 1.0), w=wA))
    b = S._nocollide(S._box(mB, (hB, hB, hB), (gap, 0.0, 1.0), w=wB))
    d = S._empty(ground=0, mu=0.0, gravity=(0.0, 0.0, 0.0))
    S._set_rigid(d, [a, b])
    ex, ey = (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)
    S._set_joints(d, [S._prismatic(0, 1, (0, 0, 0), (0, 0, 0), ex, ex, ey, ey)])
    return _finalize(d)


def _check_spin_lock(env, d):
    """The orientation rows lock the rotation about the axis too: both bodies end with
    the same spin, and the internal torque conserves angular momentum,
    w+ = (I_A w_A + I_B w_B) / (I_A + I_B) (isotropic inertias, spin about a principal
    axis: no gyroscopic term)."""
    s = env.get_state()
    IA, IB = d.rigid_inertia[0, 0], d.rigid_inertia[1, 0]
    w_exp = (IA * d.rigid_w[0, 0] + IB * d.rigid_w[1, 0]) / (IA + IB)
    for b in (0, 1):
        assert s["rigid_w"][b, 0] == pytest.approx(w_exp, rel=1e-8)
        np.testing.assert_allclose(s["rigid_w"][b, 1:], 0.0, atol=1e-9)
        np.testing.assert_allclose(s["rigid_v"][b], 0.0, atol=1e-9)
    np.testing.assert_allclose(s["rigid_q"][0], s["rigid_q"][1], atol=1e-10)


def test_prismatic_orientation_lock_spin_closed_form():
    d = _spin_pair()
    env, st = _run_converged(d)
    assert st["r_ncp"] < 1e-10
    _check_spin_lock(env, d)


def _transverse_pair(v=1e-4, mA=1.0, mB=2.0, gap=0.3):
    """Two cubes on a prismatic joint along x through both centres, at rest, no
    gravity; B gets a small transverse velocity along y.  The joint then holds the
    pair like one rigid body: total linear momentum m_B v, and the angular momentum
    about the common centre of mass, (m_A m_B / M) gap v, turns the pair about z with
    w = L / (I_A + I_B + (m_A m_B / M) gap^2) (isotropic inertias).  Rotations of
    order h w change the axis between q- and q+, so the step matches this to
    O(h w) relative; v is small enough for 1e-5."""
    hA, hB = 0.05, 0.07
    a = S._nocollide(S._box(mA, (hA, hA, hA), (0.0, 0.0, 1.0)))
    b = S._nocollide(S._box(mB, (hB, hB, hB), (gap, 0.0, 1.0), v=(0.0, v, 0.0)))
    d = S._empty(ground=0, mu=0.0, gravity=(0.0, 0.0, 0.0))
    S._set_rigid(d, [a, b])
    ex, ey = (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)
    S._set_joints(d, [S._prismatic(0, 1, (0, 0, 0), (0, 0, 0), ex, ex, ey, ey)])
    return _finalize(d)


def _check_transverse(env, d):
    s = env.get_state()
    mA, mB = d.rigid_mass
    M = mA + mB
    gap = d.rigid_x[1, 0] - d.rigid_x[0, 0]
    v = d.rigid_v[1, 1]
    mu_red = mA * mB / M
    IA, IB = d.rigid_inertia[0, 0], d.rigid_inertia[1, 0]
    w = mu_red * gap * v / (IA + IB + mu_red * gap * gap)
    V = mB * v / M
    xc = (mA * d.rigid_x[0, 0] + mB * d.rigid_x[1, 0]) / M
    # rigid-body velocities of the composite about its centre of mass
    vA_exp = V + w * (d.rigid_x[0, 0] - xc)
    vB_exp = V + w * (d.rigid_x[1, 0] - xc)
    scale = abs(v)
    assert s["rigid_w"][0, 2] == pytest.approx(w, rel=1e-5)
    assert s["rigid_w"][1, 2] == pytest.approx(w, rel=1e-5)
    assert abs(s["rigid_v"][0, 1] - vA_exp) < 1e-5 * scale
    assert abs(s["rigid_v"][1, 1] - vB_exp) < 1e-5 * scale
    for b in (0, 1):
        assert abs(s["rigid_v"][b, 0]) < 1e-5 * scale and abs(s["rigid_v"][b, 2]) < 1e-5 * scale


def _offset_pair():
    """The same pair with the anchors away from the centres (on the same line), so that
    the arms of the point-on-axis rows matter."""
    d = _transverse_pair()
    d.joint_anchor[0, 0] = [0.2, 0.0, 0.0]
    d.joint_anchor[0, 1] = [-0.1, 0.0, 0.0]
    return d.finalize()


@pytest.mark.parametrize("make", [_transverse_pair, _offset_pair], ids=["centred", "offset"])
def test_prismatic_transverse_impulse_rigid_composite(make):
    d = make()
    env, st = _run_converged(d)
    assert st["r_ncp"] < 1e-10
    _check_transverse(env, d)


# planted mistakes in the prismatic rows: each must break one of the pins above
_PRISMATIC_MUTANTS = [
    # A-side angular part of a point-on-axis row with the wrong sign
    ("rows[k].c[q][3 + i] = txd[i] - rxt[i];", "rows[k].c[q][3 + i] = -(txd[i] - rxt[i]);", "transverse"),
    # the orientation rows built from the wrong pair of frame vectors
    ("*ea[3] = {f.t1, f.t2, f.a}, *eb[3] = {f.s2, f.b, f.s1};",
     "*ea[3] = {f.t1, f.t2, f.a}, *eb[3] = {f.b, f.b, f.s1};", "spin"),
    # the drive row's coordinate with the wrong sign
    ("      c[5] = v3_dot(f.a, d);\n", "      c[5] = -v3_dot(f.a, d);\n", "slider"),
    # the B-side rows of the point-on-axis constraint at the wrong arm
    ("      jrow_add_point(e, &rows[k], B, f.rB, tj[k], 1.0);\n",
     "      jrow_add_point(e, &rows[k], B, f.rA, tj[k], 1.0);\n", "transverse_offset"),
]


@pytest.mark.parametrize("old,new,case", _PRISMATIC_MUTANTS, ids=[m[2] for m in _PRISMATIC_MUTANTS])
def test_prismatic_pins_catch_planted_mistakes(tmp_path, old, new, case):
    lib = mutant(tmp_path, old, new, case)
    checks = {
        "slider": (_slider_world(), _check_slider),
        "spin": (_spin_pair(), _check_spin_lock),
        "transverse": (_transverse_pair(), _check_transverse),
        "transverse_offset": (_offset_pair(), _check_transverse),
    }
    d, check = checks[case]
    env, st = _run_converged(d, lib_path=lib)
    with pytest.raises(AssertionError):
        assert st["r_ncp"] < 1e-10
        check(env, d)


# --------------------------------------------------------------------------
# warm-start features
# --------------------------------------------------------------------------
def _rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _basis(n):
    """Tangent basis of the reading R20: e = the world axis least aligned with n (ties
    by the lowest index), d1 = normalize(n x e), d2 = n x d1."""
    e = np.zeros(3)
    e[int(np.argmin(np.abs(n)))] = 1.0
    d1 = np.cross(n, e)
    d1 /= np.linalg.norm(d1)
    return d1, np.cross(n, d1)


def _feature_scene():
    """Box 0: yawed by 30 degrees, 2 mm above the ground, moving and spinning about z.
    Box 1: tilted by 20 degrees about x, high above the ground.  A tet floats over box
    1: its particle 0 is 1 mm above the centre of box 1's top face, the others far
    above it."""
    b0 = S._box(2.0, (0.1, 0.05, 0.2), (0.0, 0.0, 0.202), q=S.quat_from_axis_angle((0, 0, 1), math.radians(30)),
                v=(0.3, -0.2, -0.5), w=(0.0, 0.0, 1.5))
    q1 = S.quat_from_axis_angle((1, 0, 0), math.radians(20))
    b1 = S._box(3.0, (0.2, 0.2, 0.05), (1.0, 0.0, 0.6), q=q1, v=(0.05, 0.0, -0.1))
    d = S._empty(mu=0.7)
    S._set_rigid(d, [b0, b1])
    R1 = _rot(np.asarray(q1) / np.linalg.norm(q1))
    n = R1[:, 2]
    t1 = R1[:, 0]
    t2 = np.cross(n, t1)
    top = np.array([1.0, 0.0, 0.6]) + 0.05 * n
    p0 = top + 1e-3 * n
    x = np.array([p0, p0 + 0.1 * n + 0.05 * t1, p0 + 0.1 * n - 0.05 * t1, p0 + 0.15 * n + 0.05 * t2])
    S._set_tets(d, x, np.array([[0, 1, 2, 3]], np.int32), 1e5, 0.45, 1000.0,
                v=np.array([[0.1, 0.2, -0.3], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]]))
    d.tet_ids = S._orient_tets(x, d.tet_ids)
    return d.finalize()


def _expected_features(d, prev, h=H):
    """Features of the contacts the scene has, from the definitions: relative velocity
    of the two points under u~ = u- + h M^-1 f (normal, two tangents in the R20
    basis), the signed gap, the previous step's multipliers of the same key (zero if
    none), inverse masses of the two bodies (0 for the ground), mu, n_z, and whether
    the key existed in the previous step."""
    g = np.asarray(d.gravity)
    out = {}
    # box 0 bottom vertices against the ground; key = vertex * n_targets + 0
    n_targets = 1 + d.n_rigid
    R0 = _rot(d.rigid_q[0])
    for v in range(4):  # bits x=1, y=2, z=4: the four with z = -hz
        hx, hy, hz = d.rigid_extent[0]
        loc = np.array([hx if v & 1 else -hx, hy if v & 2 else -hy, -hz])
        arm = R0 @ loc
        pw = d.rigid_x[0] + arm
        # isotropic-free check: spin about the body's principal z axis, no gyroscopic term
        vel = d.rigid_v[0] + h * g + np.cross(d.rigid_w[0], arm)
        n = np.array([0.0, 0.0, 1.0])
        d1, d2 = _basis(n)
        key = v * n_targets + 0
        lam = prev.get(key, np.zeros(3))
        out[key] = np.array([n @ vel, d1 @ vel, d2 @ vel, pw[2], lam[0], lam[1], lam[2],
                             1.0 / d.rigid_mass[0], 0.0, d.mu, n[2], 1.0 if key in prev else 0.0])
    # particle 0 against box 1 (closest point on its top face)
    R1 = _rot(d.rigid_q[1])
    n = R1[:, 2]
    p = d.particle_x[0]
    hz = d.rigid_extent[1, 2]
    b = p - (n @ (p - d.rigid_x[1]) - hz) * n
    vp = d.particle_v[0] + h * g
    vb = d.rigid_v[1] + h * g + np.cross(d.rigid_w[1], b - d.rigid_x[1])
    vr = vp - vb
    d1, d2 = _basis(n)
    # lumped particle mass: rho V_e / 4 from its only tet
    x = d.particle_rest[d.tet_ids[0]]
    Ve = abs(np.linalg.det(np.stack([x[1] - x[0], x[2] - x[0], x[3] - x[0]], axis=1))) / 6.0
    mp = d.tet_material[0, 2] * Ve / 4.0
    key = (8 + 8 + 0) * n_targets + 2  # particle 0 follows the boxes' 16 vertices; target box 1
    lam = prev.get(key, np.zeros(3))
    out[key] = np.array([n @ vr, d1 @ vr, d2 @ vr, n @ (p - b), lam[0], lam[1], lam[2], 1.0 / mp,
                         1.0 / d.rigid_mass[1], d.mu, n[2], 1.0 if key in prev else 0.0])
    return out


def _oracle_features(d, prev, lib_path=None):
    env = O.OracleEnv(d, lib_path=lib_path)
    if prev:
        keys = np.array(sorted(prev), np.int64)
        env.set_prev(keys, np.array([prev[k] for k in keys]), np.zeros(0))
    feat, key = env.contact_features(H, O.make_params())
    return {int(k): f for k, f in zip(key, feat)}


# previous-step multipliers of box 0's vertex 1 on the ground and of the particle contact
PREV = {3: np.array([3.0, 0.5, -0.25]), 50: np.array([0.7, -0.1, 0.05])}


def _check_features(got, exp):
    assert sorted(got) == sorted(exp), (sorted(got), sorted(exp))
    for k in exp:
        np.testing.assert_allclose(got[k], exp[k], rtol=1e-6, atol=1e-7, err_msg=f"key {k}")


def test_features_hand_computed():
    d = _feature_scene()
    prev = dict(PREV)
    exp = _expected_features(d, prev)
    assert 50 in exp, sorted(exp)  # the particle contact carries a previous multiplier
    _check_features(_oracle_features(d, prev), exp)
    # without previous multipliers the history features are zero
    _check_features(_oracle_features(d, {}), _expected_features(d, {}))


_FEATURE_MUTANTS = [
    ("  f[1] = v3_dot(d1, vr);\n  f[2] = v3_dot(d2, vr);\n", "  f[1] = v3_dot(d2, vr);\n  f[2] = v3_dot(d1, vr);\n",
     "tangents_swapped"),
    ("  f[8] = imb;\n", "  f[8] = ima;\n", "inverse_mass_of_wrong_body"),
    ("  f[0] = v3_dot(c->n, vr);\n", "  f[0] = v3_dot(c->n, va);\n", "normal_velocity_not_relative"),
    ("  f[4] = k >= 0 ? e->prev[k].lam[0] : 0.0;\n", "  f[4] = k >= 0 ? e->prev[k].lam[1] : 0.0;\n",
     "previous_multiplier_component"),
]


@pytest.mark.parametrize("old,new,tag", _FEATURE_MUTANTS, ids=[m[2] for m in _FEATURE_MUTANTS])
def test_features_pin_catches_planted_mistakes(tmp_path, old, new, tag):
    lib = mutant(tmp_path, old, new, tag)
    d = _feature_scene()
    with pytest.raises(AssertionError):
        _check_features(_oracle_features(d, dict(PREV), lib_path=lib), _expected_features(d, dict(PREV)))


# --------------------------------------------------------------------------
# geometric-stiffness secant
# --------------------------------------------------------------------------
L_TET = 0.1
SIG = (1.2, 1.1, 0.9)


def _secant_tet(u3=(2e-4, -3e-4, 0.0)):
    """One tet with rest shape L I (vertex 0 at the origin, vertex j at L e_j), deformed
    to F = diag(1.2, 1.1, 0.9) by moving vertices 1..3 along their axes.  Vertices 0-2
    carry 1e8 kg, vertex 3 only its lumped mass and a small initial velocity with x and
    y parts; no gravity, no ground."""
    rest = np.array([[0, 0, 0], [L_TET, 0, 0], [0, L_TET, 0], [0, 0, L_TET]], np.float64)
    x = np.array([[0, 0, 0], [SIG[0] * L_TET, 0, 0], [0, SIG[1] * L_TET, 0], [0, 0, SIG[2] * L_TET]])
    d = S._empty(ground=0, gravity=(0.0, 0.0, 0.0))
    S._set_tets(d, x, np.array([[0, 1, 2, 3]], np.int32), 1e5, 0.45, 1000.0)
    d.particle_rest = rest
    d.particle_mass = np.array([1e8, 1e8, 1e8, 0.0])
    d.particle_v = np.zeros((4, 3))
    d.particle_v[3] = u3
    return d.finalize()


def _secant_record(d, lib_path=None, h=H):
    env = O.OracleEnv(d, lib_path=lib_path)
    env.set_record(1)
    env.step(h, 2, 40, 0.0, O.make_params(geo_stiff=1))
    return env.record()


def _check_secant(rec, d, h=H):
    """At iteration k = 1 from the zero start, vertex 3 moved by x^1 - x^0 = h u^1.  For
    F = diag(s) the forces J^T lambda on vertex 3 have no x or y part, so the secant's
    force change is the x (y) force at x^1, which the second derivative of the singular
    values gives: d^2 s_1 / dF_13^2 = s_1 / (s_1^2 - s_3^2), d^2 s_3 / dF_13^2 =
    s_3 / (s_3^2 - s_1^2) (likewise y with s_2), and F_13 = (x_3 - x_0)_x / L.  Hence
    c_x = h^2 / L^2 (lam_1 s_1 - lam_3 s_3) / (s_1^2 - s_3^2) * du^2 / (du^2 + tau^2),
    with s at x^1, and H~_xx = m - min(0, c_x) (Sec. 8.3).  z: the force change is of
    second order, c_z ~ 0."""
    lam = rec["lam"][:3]
    u1 = rec["u"][9:12]
    assert np.all(rec["uprev"] == 0.0)
    x1 = d.particle_x[3] + h * u1
    s1, s2, s3 = SIG[0], SIG[1], x1[2] / L_TET
    tau = 1e-6
    m3 = d.tet_material[0, 2] * L_TET ** 3 / 6.0 / 4.0
    cx = h * h / L_TET ** 2 * (lam[0] * s1 - lam[2] * s3) / (s1 * s1 - s3 * s3) * u1[0] ** 2 / (u1[0] ** 2 + tau * tau)
    cy = h * h / L_TET ** 2 * (lam[1] * s2 - lam[2] * s3) / (s2 * s2 - s3 * s3) * u1[1] ** 2 / (u1[1] ** 2 + tau * tau)
    assert cx < 0 and cy < 0  # stretched x, y rows against a compressed z row: stiffening
    hd = rec["hdiag"][9:12]
    assert hd[0] == pytest.approx(m3 - cx, rel=1e-4)
    assert hd[1] == pytest.approx(m3 - cy, rel=1e-4)
    assert abs(hd[2] - m3) < 1e-4 * abs(cx)


def test_secant_matches_singular_value_hessian():
    d = _secant_tet()
    rec = _secant_record(d)
    _check_secant(rec, d)


_SECANT_MUTANTS = [
    ("double cj = h * (f[dd] - fhat[dd]) * dU / (dU * dU + TAU_GS * TAU_GS);",
     "double cj = -h * (f[dd] - fhat[dd]) * dU / (dU * dU + TAU_GS * TAU_GS);", "sign"),
    ("for (int r = 0; r < S.nrows; ++r) jrow_scatter(&S.Jprev[r], S.lam[r], fhat);",
     "for (int r = 0; r < S.nrows; ++r) jrow_scatter(&S.J[r], S.lam[r], fhat);", "same_jacobian"),
    ("double cj = h * (f[dd] - fhat[dd]) * dU / (dU * dU + TAU_GS * TAU_GS);",
     "double cj = (f[dd] - fhat[dd]) * dU / (dU * dU + TAU_GS * TAU_GS);", "missing_h"),
    ("double dU = S.u[dd] - S.uprev[dd];",
     "double dU = S.u[particle_dof(e, pi) + (a + 1) % 3] - S.uprev[particle_dof(e, pi) + (a + 1) % 3];",
     "wrong_component"),
]


@pytest.mark.parametrize("old,new,tag", _SECANT_MUTANTS, ids=[m[2] for m in _SECANT_MUTANTS])
def test_secant_pin_catches_planted_mistakes(tmp_path, old, new, tag):
    lib = mutant(tmp_path, old, new, tag)
    d = _secant_tet()
    with pytest.raises(AssertionError):
        _check_secant(_secant_record(d, lib_path=lib), d)


# --------------------------------------------------------------------------
# watchdog switch and the per-iteration record
# --------------------------------------------------------------------------
def test_watchdog_switch_paper_exact_off():
    """Sec. 8.1 names safeguards without using one.  With the switch off (the paper's
    method, default) every iterate is accepted and the step ends on its last iterate;
    with it on, a step whose merit blows up returns its lowest-merit iterate.  Case:
    the stretched sheet without geometric stiffness, where the iterates overshoot."""
    d = si.stretched_sheet()
    p_off = O.make_params(geo_stiff=0)
    p_on = O.make_params(geo_stiff=0, watchdog=1)
    fired = False
    for p, on in [(p_off, False), (p_on, True)]:
        env = O.OracleEnv(d)
        for s in range(8):
            st = env.step(H, 30, 60, 1e-6, p)
            mh = env.merit_history()
            if on and st["watchdog"]:
                fired = True
                assert st["merit"] == pytest.approx(mh.min(), rel=1e-12)
            if not on:
                assert st["watchdog"] == 0
                if not st["nonfinite"]:
                    assert st["merit"] == pytest.approx(mh[-1], rel=1e-12)
    assert fired


def test_eval_iterate_reproduces_the_steps_own_iteration():
    """orc_eval_iterate, given the iterates k-1 and k that a step went through, records
    exactly what that step recorded at iteration k (assembly, secant, Schur system,
    PCR): the per-row parity of the GPU against evaluations at its own iterates is
    parity against the method."""
    for d in [si.batched_env(seed=1003, tets_max=150), si.grasp_scene(seed=0, sphere_cell=0.03)]:
        p = O.make_params()
        recs = []
        for k in (1, 2):
            env = O.OracleEnv(d)
            env.set_record(k)
            env.step(H, 3, 30, 0.0, p)
            recs.append(env.record())
        env = O.OracleEnv(d)
        nc = len(env.contact_features(H, p)[1])
        it = {k: recs[1][k] for k in ["lam", "u", "rx", "rq", "px"]}
        prev = {k: recs[0][k] for k in ["lam", "u", "rx", "rq", "px"]}
        got = env.eval_iterate(H, 30, nc, it, prev=prev, params=p)
        for f in ["err", "cdiag", "P", "b", "Az", "dlam", "g", "hdiag", "alpha", "rn", "rf", "f", "fhat", "active"]:
            np.testing.assert_array_equal(got[f], recs[1][f], err_msg=f)
        # the env's own state is left as it was
        env2 = O.OracleEnv(d)
        for k, v in env2.get_state().items():
            np.testing.assert_array_equal(env.get_state()[k], v)
