"""Pins: fix the FP64 oracle to things other than itself (paper worked examples,
closed forms, textbook special cases, brute force, finite differences).

All tests here run on the CPU (`-m "not gpu"`)."""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

import scene_inputs as si
from oracle import oracle as O
from tests import npref

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")))


def converged(env, h, N=60, M=60, tol=1e-11, **kw):
    return env.step(h, N, M, tol, O.make_params(**kw))


# --------------------------------------------------------------------------- P1
def test_p1_rscaled_min_map_is_linear_one_newton_step():
    """Sec. 7 / Fig. rscalingvis: c = lambda/4 - 1/8 -> lambda = 1/2 in ONE Newton step
    with the r-scaled minimum map (r = h^2 J M^-1 J^T = 1/4) and t = 1, through the whole
    step pipeline: a particle of mass 4h^2 on the ground, z^- + h u~_z = -1/8."""
    g = GOLD["complementarity_preconditioning"]
    h = 0.5
    d = si.particle_on_plane(v=(0.0, 0.0, -0.25), mass=4 * h * h, mu=0.0, gravity=(0, 0, 0))
    env = O.OracleEnv(d)
    st = env.step(h, 1, 10, 0.0, O.make_params(ncp=1, rmode=2, damping=1.0, eps=0.0))
    assert st["n_contacts"] == 1 and st["newton_iters"] == 1
    lam = env.contacts()["lam"][0, 0]
    assert lam == pytest.approx(g["solution"], abs=1e-12)
    # the kinematic consequence: C(lambda) = slope*lambda + offset = 0 at the end
    assert env.get_state()["particle_x"][0, 2] == pytest.approx(0.0, abs=1e-12)


def test_p1_unscaled_min_map_has_kink():
    """With r = 1 the min-map of Fig. rscalingvis has its kink where C = lambda:
    lambda/4 - 1/8 = lambda  ->  lambda = -1/6; on each side it follows one branch."""
    g = GOLD["complementarity_preconditioning"]
    c = lambda l: g["slope"] * l + g["offset"]
    kink = g["offset"] / (1 - g["slope"])
    assert kink == pytest.approx(-1.0 / 6.0)
    for l in [kink - 0.1, kink + 0.1]:
        phi, a, b = O.ncp_min(c(l), l, 1.0)
        assert phi == pytest.approx(min(c(l), l))
        assert (a, b) == ((1.0, 0.0) if c(l) <= l else (0.0, 1.0))


def test_p1_fb_converges_few_steps():
    h = 0.5
    d = si.particle_on_plane(v=(0.0, 0.0, -0.25), mass=4 * h * h, mu=0.0, gravity=(0, 0, 0))
    env = O.OracleEnv(d)
    st = env.step(h, 8, 10, 0.0, O.make_params(ncp=0, rmode=2, damping=1.0, eps=0.0))
    assert env.contacts()["lam"][0, 0] == pytest.approx(0.5, abs=1e-9)


# --------------------------------------------------------------------------- P2
@pytest.mark.parametrize("r", [0.01, 0.3, 1.0, 7.0])
@pytest.mark.parametrize("ncp", [0, 1])
def test_p2_friction_w_at_cone_limit(r, ncp):
    """Fig. friction_functions: |v| = 0.5, lambda_n = 10, mu = 0.5, cone limit 5 N:
    W = |v|/|lambda_f| = 0.1 for every r, and phi_f = v + W lambda_f = 0 at lambda_f = -5."""
    g = GOLD["friction_cone_limit"]
    W = O.friction_w(ncp, g["u0"], g["lambda_n"], g["lambda_f_limit"], g["mu"], r)
    assert W == pytest.approx(g["u0"] / g["lambda_f_limit"], rel=1e-12)
    assert g["u0"] + W * (-g["lambda_f_limit"]) == pytest.approx(0.0, abs=1e-12)


def test_p2_friction_w_inside_cone_sticks_and_outside_penalises():
    # zero slip inside the cone -> W = 0 (sticking), far outside -> large W
    assert O.friction_w(0, 0.0, 10.0, 2.0, 0.5, 1.0) == 0.0
    assert O.friction_w(1, 0.0, 10.0, 2.0, 0.5, 1.0) == 0.0
    assert O.friction_w(0, 0.5, 10.0, 9.0, 0.5, 0.3) > 10 * 0.1


def test_p2_friction_w_outside_cone_closed_form_and_limit():
    """App. A.2 at zero slip outside the cone: s = mu lam_n - |lam_f| < 0 gives
    |v|^{n+1} = 2 r |s| and r |lam_f|^{n+1} = r (2 mu lam_n - |lam_f|), so
    W = 2 r (|lam_f| - mu lam_n) / (2 mu lam_n - |lam_f|), growing without bound as
    |lam_f| -> 2 mu lam_n; beyond, the fixed point asks for no friction force and W is
    infinite (the row's limit drives lam_f to zero)."""
    mu, lam_n = 0.5, 10.0
    for r in [0.3, 1.0, 4.0]:
        for frac in [1.1, 1.5, 1.9, 1.99]:
            lf = frac * mu * lam_n
            W = O.friction_w(0, 0.0, lam_n, lf, mu, r)
            assert W == pytest.approx(2 * r * (lf - mu * lam_n) / (2 * mu * lam_n - lf), rel=1e-12)
        for frac in [2.0, 2.5, 10.0]:
            assert O.friction_w(0, 0.0, lam_n, frac * mu * lam_n, mu, r) == np.inf


def test_p2_friction_fixed_point_is_fb_root():
    """At the fixed point of the iteration (A.2) the FB friction function vanishes:
    psi_FB(|v|, mu lam_n - |lam_f|) = 0 with |v| = W |lam_f|."""
    rng = np.random.default_rng(0)
    for _ in range(50):
        mu, lam_n, r = rng.uniform(0.2, 1), rng.uniform(0.1, 10), rng.uniform(0.01, 5)
        lf = rng.uniform(0.01, 0.99) * mu * lam_n
        v = 0.0
        W = O.friction_w(0, v, lam_n, lf, mu, r)
        assert W == pytest.approx(0.0, abs=1e-15)
        # sliding: |lam_f| = mu lam_n and any |v| -> W = |v|/|lam_f|
        v = rng.uniform(0.01, 3)
        W = O.friction_w(0, v, lam_n, mu * lam_n, mu, r)
        assert W == pytest.approx(v / (mu * lam_n), rel=1e-12)


# --------------------------------------------------------------------------- P3
def test_p3_free_fall_particle():
    h = 1 / 60
    d = si.free_particle()
    env = O.OracleEnv(d)
    converged(env, h)
    x0, v0, g = d.particle_x[0], d.particle_v[0], np.array(d.gravity)
    st = env.get_state()
    np.testing.assert_allclose(st["particle_v"][0], v0 + h * g, atol=1e-12)
    np.testing.assert_allclose(st["particle_x"][0], x0 + h * (v0 + h * g), atol=1e-12)


def test_p3_spinning_rigid_body():
    """Constraint-free rigid body: omega+ = omega- + h I^-1(-omega x I omega) with I at q^-,
    and theta+ is the fixed point of theta+ = normalize(theta- + h/2 [0,omega+] (x) theta+)."""
    h = 1 / 60
    d = si.spinning_box()
    env = O.OracleEnv(d)
    converged(env, h)
    st = env.get_state()
    q0, w0 = d.rigid_q[0] / np.linalg.norm(d.rigid_q[0]), d.rigid_w[0]
    R = npref.quat_rot(q0)
    I = R @ np.diag(d.rigid_inertia[0]) @ R.T
    w_exp = w0 + h * np.linalg.solve(I, -np.cross(w0, I @ w0))
    np.testing.assert_allclose(st["rigid_w"][0], w_exp, atol=1e-12)
    np.testing.assert_allclose(st["rigid_x"][0], d.rigid_x[0] + h * d.rigid_v[0], atol=1e-12)
    q1 = st["rigid_q"][0]
    assert np.linalg.norm(q1) == pytest.approx(1.0, abs=1e-14)
    t = q0 + 0.5 * h * npref.quat_mul(np.r_[0.0, w_exp], q1)
    np.testing.assert_allclose(q1, t / np.linalg.norm(t), atol=1e-12)


def test_p3_quaternion_kinematic_map():
    """Sec. 9 rigid bodies: (1/2) Q(theta) omega equals (1/2)[0, omega] (x) theta."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w = rng.normal(size=3)
        Q = O.quat_kinematic(q)
        np.testing.assert_allclose(Q @ w, npref.quat_mul(np.r_[0.0, w], q), atol=1e-14)


# --------------------------------------------------------------------------- P4
@pytest.mark.parametrize("vt", [0.02, 0.5, 2.0])
def test_p4_particle_sliding_on_plane(vt):
    """Maximal dissipation on a plane: v_t+ = v~_t max(0, 1 - mu g h/|v~_t|), lambda_n = m g."""
    h, mu, m = 1 / 60, 0.5, 1.3
    direction = np.array([0.6, 0.8, 0.0])
    d = si.particle_on_plane(v=tuple(vt * direction), mass=m, mu=mu)
    env = O.OracleEnv(d)
    for ncp in [0, 1]:
        env = O.OracleEnv(d)
        st = converged(env, h, N=80, M=20, ncp=ncp)
        assert st["r_ncp"] < 1e-9
        v = env.get_state()["particle_v"][0]
        g = -d.gravity[2]
        expect = max(0.0, 1 - mu * g * h / vt) * vt
        np.testing.assert_allclose(v[:2], expect * direction[:2], atol=1e-8)
        assert abs(v[2]) < 1e-8
        assert env.contacts()["lam"][0, 0] == pytest.approx(d.particle_mass[0] * g, rel=1e-8)


# --------------------------------------------------------------------------- P5
@pytest.mark.parametrize("theta,mu", [(0.5, 0.3), (0.3, 0.6)])
def test_p5_box_on_incline(theta, mu):
    """Box (4 face contacts) on a static incline: slides with v_k = k h g (sin - mu cos)
    if tan(theta) > mu, else stays at rest; the summed normal force is m g cos(theta)."""
    h, m = 1 / 60, 1.0
    g = 9.81
    d = si.box_on_incline(theta, mu, mass=m)
    env = O.OracleEnv(d)
    for k in range(1, 6):
        st = converged(env, h, N=100, M=40, tol=1e-10)
        assert st["r_ncp"] < 1e-8, st
        v = env.get_state()["rigid_v"][1]
        speed = np.linalg.norm(v)
        lam = env.contacts()["lam"]
        if math.tan(theta) > mu:
            assert speed == pytest.approx(k * h * g * (math.sin(theta) - mu * math.cos(theta)), rel=1e-6)
        else:
            # at rest up to the float32-rounded initial gap closed along the normal
            n = con_normal = env.contacts()["normal"][0]
            assert np.linalg.norm(v - (v @ n) * n) < 1e-9 and speed < 1e-6
        # rel 1e-5: the float32-rounded start leaves a ~1e-8 m gap that the first step closes
        assert lam[:, 0].sum() == pytest.approx(m * g * math.cos(theta), rel=1e-5)


# --------------------------------------------------------------------------- P6
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_p6_frictionless_particles_bruteforce_lcp(seed):
    """Frictionless particles against tilted static planes are exact LCPs in lambda
    (C linear in u): enumerate all active sets and compare with the converged oracle."""
    h = 1 / 60
    d = si.particles_vs_planes_lcp(seed=seed, h=h)
    env = O.OracleEnv(d)
    st = converged(env, h, N=80, M=30, tol=1e-12)
    assert st["r_ncp"] < 1e-10
    con = env.contacts()
    g = np.array(d.gravity)
    nr = d.n_rigid
    for p in range(d.n_particles):
        idx = np.where(con["bodies"][:, 0] == nr + p)[0]
        m = d.particle_mass[p]
        ut = d.particle_v[p] + h * g
        ns, qs = [], []
        for i in idx:
            slab = con["bodies"][i, 1]
            R = npref.quat_rot(d.rigid_q[slab] / np.linalg.norm(d.rigid_q[slab]))
            n_exp = R[:, 2]
            np.testing.assert_allclose(con["normal"][i], n_exp, atol=1e-12)
            b = d.rigid_x[slab] + R @ np.array([0, 0, d.rigid_extent[slab, 2]])
            ns.append(n_exp)
            qs.append(n_exp @ (d.particle_x[p] - b) + h * n_exp @ ut)
        if not ns:
            continue
        N = np.array(ns)
        A = h * h / m * N @ N.T
        lam = npref.lcp_bruteforce(A, np.array(qs))
        np.testing.assert_allclose(con["lam"][idx, 0], lam, atol=1e-8)
        u_exp = ut + h / m * N.T @ lam
        np.testing.assert_allclose(env.get_state()["particle_v"][p], u_exp, atol=1e-9)


# --------------------------------------------------------------------------- P7
def _contact_state(d, st, con, i, h):
    """Independent evaluation of C_n and the relative tangential velocity of contact i."""
    nr = d.n_rigid
    fa, tb = con["bodies"][i]

    def point_and_vel(body, local):
        if body < 0:
            return local, np.zeros(3)
        if body < nr:
            R = npref.quat_rot(st["rigid_q"][body] / np.linalg.norm(st["rigid_q"][body]))
            arm = R @ local
            return st["rigid_x"][body] + arm, st["rigid_v"][body] + np.cross(st["rigid_w"][body], arm)
        p = body - nr
        return st["particle_x"][p], st["particle_v"][p]

    pa, va = point_and_vel(fa, con["a_local"][i])
    pb, vb = point_and_vel(tb, con["b_local"][i])
    n = con["normal"][i]
    Cn = n @ (pa - pb) - con["thickness"][i]
    vr = va - vb
    vt = vr - (n @ vr) * n
    return Cn, vt


@pytest.mark.parametrize("ncp", [0, 1])
def test_p7_ncp_conditions_at_convergence(ncp):
    """Signorini and maximal-dissipation conditions (Sec. 3.3-3.5) hold at a converged step
    of a box thrown sideways onto the ground."""
    h = 1 / 60
    d = si.cube_stack(seed=3, n=1, mu=0.4)
    d.rigid_v[0] = (1.5, 0.4, -0.3)
    d.rigid_w[0] = (0.0, 0.0, 2.0)
    env = O.OracleEnv(d)
    tau = 1e-7
    for _ in range(3):
        st = converged(env, h, N=100, M=60, tol=1e-10, ncp=ncp)
        assert st["r_ncp"] < 1e-8
        con = env.contacts()
        S = env.get_state()
        for i in range(len(con["key"])):
            Cn, vt = _contact_state(d, S, con, i, h)
            ln, lf = con["lam"][i, 0], con["lam"][i, 1:]
            assert Cn >= -tau and ln >= -tau and abs(Cn * ln) <= tau
            assert np.linalg.norm(lf) <= d.mu * ln * (1 + 1e-6) + tau
            if np.linalg.norm(vt) > 1e-5:
                # the contact-basis friction force opposes the slip direction at the limit
                d1, d2 = O.tangent_basis(con["normal"][i])
                fw = lf[0] * d1 + lf[1] * d2
                assert np.linalg.norm(fw) == pytest.approx(d.mu * ln, rel=1e-5, abs=tau)
                assert fw @ vt == pytest.approx(-np.linalg.norm(fw) * np.linalg.norm(vt), rel=1e-5, abs=tau)
            if ln <= tau:
                assert np.linalg.norm(lf) <= tau


# --------------------------------------------------------------------------- P8
def test_p8_momentum_conserved_by_joints_and_drives():
    """Gravity- and contact-free hinged chains with drives: the joint and drive rows are
    internal, so total linear momentum is conserved at convergence."""
    h = 1 / 60
    d = si.batched_env(seed=11, tets_max=0, joints_max=12)
    assert d.n_joints > 0
    d.gravity = (0.0, 0.0, 0.0)
    d.ground = 0
    rng = np.random.default_rng(0)
    d.rigid_v = rng.normal(scale=0.3, size=d.rigid_v.shape)
    d.rigid_w = rng.normal(scale=0.5, size=d.rigid_w.shape)
    d.joint_drive[:, 0] = 3.0
    d.joint_drive[:, 1] = 0.1
    d.joint_drive[:, 2] = 0.4
    d.joint_drive[:, 3] = 1.0
    env = O.OracleEnv(d)
    # only bodies that are not touching anything: ground is off, spread apart -> no contacts
    P0 = (d.rigid_mass[:, None] * d.rigid_v).sum(0)
    for _ in range(5):
        st = converged(env, h, N=60, M=80, tol=1e-11)
        P = (d.rigid_mass[:, None] * env.get_state()["rigid_v"]).sum(0)
        np.testing.assert_allclose(P, P0, atol=1e-8)


def test_p8_pendulum_implicit_pd_closed_form():
    """READING of implicit PD (a soft row under backward Euler): a box hinged at its
    centre about y with no gravity obeys I (w+ - w-)/h = -(kp + kd/h)(th+ - th_eff) with
    th+ = th- + 2 asin(h w+/2) (the fixed point of the normalised quaternion update
    theta+ = normalize(theta- + h/2 [0,w+] (x) theta+) about a fixed axis)."""
    h = 1 / 60
    kp, kd, amp, freq, phase = 5.0, 0.05, 0.3, 0.5, 0.7
    d = si.pendulum_drive(kp=kp, kd=kd, amp=amp, freq=freq, phase=phase)
    env = O.OracleEnv(d)
    Iyy = d.rigid_inertia[0, 1]
    kp, kd, amp, freq, phase = d.joint_drive[0, :5]  # float32-rounded inputs
    th, w = 0.0, 0.0
    for k in range(1, 8):
        st = converged(env, h, N=60, M=30, tol=1e-12)
        tgt = amp * math.sin(2 * math.pi * freq * k * h + phase)
        keff = kp + kd / h
        th_eff = (kp * tgt + kd / h * th) / keff
        f = lambda wp: Iyy * (wp - w) / h + keff * (th + 2 * math.asin(h * wp / 2) - th_eff)
        wp = brentq(f, -100, 100, xtol=1e-15)
        S = env.get_state()
        assert S["rigid_w"][0, 1] == pytest.approx(wp, abs=1e-9)
        th, w = th + 2 * math.asin(h * wp / 2), wp
        q = S["rigid_q"][0]
        assert 2 * math.atan2(q[2], q[0]) == pytest.approx(th, abs=1e-9)


# --------------------------------------------------------------------------- P9
def test_p9_fb_derivatives_finite_difference():
    rng = np.random.default_rng(2)
    eps = 1e-6
    for _ in range(100):
        Cn, lam, r = rng.normal(), rng.normal(), rng.uniform(0.1, 3)
        phi, a, b = O.ncp_fb(Cn, lam, r)
        assert phi == pytest.approx(Cn + r * lam - math.hypot(Cn, r * lam), abs=1e-14)
        da = (O.ncp_fb(Cn + eps, lam, r)[0] - O.ncp_fb(Cn - eps, lam, r)[0]) / (2 * eps)
        db = (O.ncp_fb(Cn, lam + eps, r)[0] - O.ncp_fb(Cn, lam - eps, r)[0]) / (2 * eps)
        assert a == pytest.approx(da, rel=1e-6, abs=1e-8)
        assert b * r == pytest.approx(db, rel=1e-6, abs=1e-8)
    assert O.ncp_fb(0.0, 0.0, 1.0) == (0.0, 0.0, 1.0)  # subgradient choice of Sec. 4.2


def test_p9_neohookean_derivatives_finite_difference():
    C1, D1, al = O.lame(1e5, 0.45)
    rng = np.random.default_rng(3)
    eps = 1e-6
    for _ in range(30):
        s = rng.uniform(0.5, 1.5, 3) * np.array([1, 1, rng.choice([-1, 1])])
        psi, g, H = O.neohookean(s, C1, D1, al)
        J = s.prod()
        assert psi == pytest.approx(C1 * ((s ** 2).sum() - 3) + D1 * (J - al) ** 2, rel=1e-12)
        for i in range(3):
            e = np.zeros(3); e[i] = eps
            gp = (O.neohookean(s + e, C1, D1, al)[0] - O.neohookean(s - e, C1, D1, al)[0]) / (2 * eps)
            assert g[i] == pytest.approx(gp, rel=1e-6)
            Hp = (O.neohookean(s + e, C1, D1, al)[1] - O.neohookean(s - e, C1, D1, al)[1]) / (2 * eps)
            np.testing.assert_allclose(H[:, i], Hp, rtol=1e-6, atol=1e-6 * np.abs(H).max())


def test_p9_signed_svd_and_stretch_derivative():
    """F = U diag(s) V^T with det U = det V = 1 and ds_i/dF = u_i v_i^T."""
    rng = np.random.default_rng(4)
    eps = 1e-7
    for trial in range(30):
        F = np.eye(3) + 0.3 * rng.normal(size=(3, 3))
        if trial % 3 == 0:
            F[:, 0] *= -1  # inverted element
        U, s, V = O.svd3(F)
        np.testing.assert_allclose(U @ np.diag(s) @ V.T, F, atol=1e-12)
        assert np.linalg.det(U) == pytest.approx(1.0) and np.linalg.det(V) == pytest.approx(1.0)
        assert s[0] >= s[1] >= abs(s[2]) - 1e-12
        assert np.sign(s[2]) == np.sign(np.linalg.det(F))
        _, s_np, _ = npref.signed_svd(F)
        np.testing.assert_allclose(s, s_np, atol=1e-10)
        for a in range(3):
            for b in range(3):
                dF = np.zeros((3, 3)); dF[a, b] = eps
                ds = (O.svd3(F + dF)[1] - O.svd3(F - dF)[1]) / (2 * eps)
                np.testing.assert_allclose(ds, U[a, :] * V[b, :], atol=2e-6)


def test_p9_compliance_is_inverse_of_projected_hessian():
    C1, D1, al = O.lame(1e5, 0.45)
    rng = np.random.default_rng(5)
    for _ in range(20):
        H = rng.normal(size=(3, 3)); H = H + H.T
        floor_ = 0.1
        E = O.compliance3(H, floor_)
        w, Q = np.linalg.eigh(H)
        np.testing.assert_allclose(E, Q @ np.diag(1 / np.maximum(w, floor_)) @ Q.T, atol=1e-10)


# --------------------------------------------------------------------------- P10
def test_p10_rest_state_stress_free_and_linear_moduli():
    """READING of the material constants: the rest state is stress free and the rest
    Hessian has the eigenvalues of linear elasticity, 2 mu (twice) and 3 lambda + 2 mu."""
    E, nu = 1e5, 0.45
    mu = E / (2 * (1 + nu))
    la = E * nu / ((1 + nu) * (1 - 2 * nu))
    C1, D1, al = O.lame(E, nu)
    psi, g, H = O.neohookean(np.ones(3), C1, D1, al)
    np.testing.assert_allclose(g, 0.0, atol=1e-9)
    w = np.sort(np.linalg.eigvalsh(H))
    np.testing.assert_allclose(w, [2 * mu, 2 * mu, 3 * la + 2 * mu], rtol=1e-12)


# --------------------------------------------------------------------------- P11
def _fem_energy(x, rest, tets, mats):
    U = 0.0
    for t, (E, nu, rho) in zip(tets, mats):
        Dm = np.stack([rest[t[k]] - rest[t[0]] for k in (1, 2, 3)], axis=1)
        Ds = np.stack([x[t[k]] - x[t[0]] for k in (1, 2, 3)], axis=1)
        F = Ds @ np.linalg.inv(Dm)
        _, s, _ = npref.signed_svd(F)
        mu = E / (2 * (1 + nu)); la = E * nu / ((1 + nu) * (1 - 2 * nu))
        C1, D1, al = mu / 2, (la + mu) / 2, 1 + mu / (la + mu)
        Ve = abs(np.linalg.det(Dm)) / 6
        U += Ve * (C1 * ((s ** 2).sum() - 3) + D1 * (s.prod() - al) ** 2)
    return U


@pytest.mark.parametrize("n_tets,fem_mode", [(1, 0), (5, 0), (5, 1)])
def test_p11_fem_step_is_variational_implicit_euler(n_tets, fem_mode):
    """Sec. 9.1: the generalised-compliance rows reproduce the elastic force, so a
    converged contact-free step satisfies M (u+ - u~) + h grad U(x- + h u+) = 0 with
    U = sum V_e Psi (independent NumPy energy, central differences).  The element is
    deformed with well separated principal stretches; geometric stiffness is on (the
    principal-stretch rows omit the rotational stiffness, Sec. 8.3 restores it).  The
    optimality residual must be at the level of the achieved Newton residual, far below
    the elastic term itself.  Without the rotational stiffness the damped iteration
    converges slowly and erratically (a rounding-level change moves the step at which
    it settles); damping 0.5 settles all three cases within the budget."""
    h = 1 / 60
    F = [[1.15, 0.05, 0.0], [0.0, 1.0, 0.03], [0.02, 0.0, 0.85]]
    d = si.single_tet(perturb=1e-3, seed=n_tets, n_tets=n_tets, deform=F)
    env = O.OracleEnv(d)
    st = converged(env, h, N=300, M=60, tol=1e-10, fem_mode=fem_mode, geo_stiff=1, damping=0.5)
    assert st["r_ncp"] < 1e-4, st
    S = env.get_state()
    x, u = S["particle_x"], S["particle_v"]
    m = np.zeros(d.n_particles)
    for t, (E, nu, rho) in zip(d.tet_ids, d.tet_material):
        Dm = np.stack([d.particle_rest[t[k]] - d.particle_rest[t[0]] for k in (1, 2, 3)], axis=1)
        m[t] += rho * abs(np.linalg.det(Dm)) / 6 / 4
    eps = 1e-7
    grad = np.zeros_like(x)
    for p in range(d.n_particles):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[p, a] += eps; xm[p, a] -= eps
            grad[p, a] = (_fem_energy(xp, d.particle_rest, d.tet_ids, d.tet_material)
                          - _fem_energy(xm, d.particle_rest, d.tet_ids, d.tet_material)) / (2 * eps)
    ut = d.particle_v + h * np.array(d.gravity)
    res = (m[:, None] * (u - ut) + h * grad) / m[:, None]
    elastic = np.abs(h * grad / m[:, None]).max()
    assert elastic > 0.1
    assert np.abs(res).max() < 20 * st["r_ncp"] + 1e-9


# --------------------------------------------------------------------------- P12
def test_p12_pcr_matches_direct_solve_and_is_monotone():
    rng = np.random.default_rng(6)
    for n in [1, 3, 8, 20]:
        B = rng.normal(size=(n, n))
        A = B @ B.T + n * np.eye(n)
        b = rng.normal(size=n)
        P = 1 / np.diag(A)
        x, hist = O.pcr_dense(A, b, P, n)
        # the stop rule ends the iteration once <z, A z> <= 1e-12 of its start, i.e.
        # at a relative residual of about 1e-6
        xd = np.linalg.solve(A, b)
        assert np.linalg.norm(A @ x - b) <= 1e-5 * np.linalg.norm(b)
        np.testing.assert_allclose(x, xd, rtol=1e-4, atol=1e-6 * np.abs(xd).max())
        assert (np.diff(hist) <= 1e-12 * hist[0]).all()


def test_p12_pcr_stops_at_rounding_level():
    """Further iterations after the residual has reached rounding level only amplify
    rounding: with a generous budget the iteration count stays at about n."""
    rng = np.random.default_rng(8)
    n = 5
    B = rng.normal(size=(n, n))
    A = B @ B.T + n * np.eye(n)
    b = rng.normal(size=n)
    P = 1 / np.diag(A)
    x, hist = O.pcr_dense(A, b, P, 200)
    assert len(hist) <= n + 1, len(hist)
    assert np.linalg.norm(A @ x - b) <= 1e-5 * np.linalg.norm(b)


def test_p12_pcr_iterates_minimise_preconditioned_residual_over_krylov_space():
    """CR minimises the residual over the Krylov space (Sec. 8.2): with a left Jacobi
    preconditioner P the k-th iterate minimises sqrt(r^T P r) over span{(PA)^j P b}."""
    rng = np.random.default_rng(7)
    n = 12
    B = rng.normal(size=(n, n))
    A = B @ B.T + 0.5 * np.eye(n)
    b = rng.normal(size=n)
    P = 1 / np.diag(A)
    L = np.sqrt(P)
    for k in range(1, 7):
        x, _ = O.pcr_dense(A, b, P, k)
        K = [P * b]
        for _ in range(k - 1):
            K.append(P * (A @ K[-1]))
        K = np.stack(K, axis=1)
        c, *_ = np.linalg.lstsq(L[:, None] * (A @ K), L * b, rcond=None)
        np.testing.assert_allclose(x, K @ c, rtol=1e-7, atol=1e-9)


# --------------------------------------------------------------------------- P13
def test_p13_solution_invariant_to_r_mode_and_ncp_function():
    """Sec. 7: the converged solution does not depend on r; on a non-redundant problem
    FB and min-map give the same root."""
    h = 1 / 60
    d = si.cube_stack(seed=1, n=1, mu=0.5)
    d.rigid_v[0] = (0.8, -0.2, -0.5)
    results = []
    # identity scaling (rmode 0) is the strategy the paper reports as failing on such
    # sliding contacts (Sec. 11.1); the invariance is checked between the two others.
    for rmode in [1, 2]:
        for ncp in [0, 1]:
            env = O.OracleEnv(d)
            st = converged(env, h, N=200, M=60, tol=1e-11, rmode=rmode, ncp=ncp)
            assert st["r_ncp"] < 1e-9, (rmode, ncp, st)
            S = env.get_state()
            results.append(np.concatenate([S["rigid_x"][0], S["rigid_v"][0], S["rigid_w"][0]]))
    for r in results[1:]:
        np.testing.assert_allclose(r, results[0], atol=1e-8)


def test_p13_rotation_about_vertical_axis_gives_rotated_result():
    """Isotropic friction: rotating a whole scene about z rotates the converged result
    (the tangent basis choice does not matter)."""
    h = 1 / 60
    ang = 0.7
    Rz = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1]])
    qz = np.array([math.cos(ang / 2), 0, 0, math.sin(ang / 2)])
    d0 = si.cube_stack(seed=2, n=1, mu=0.5)
    d0.rigid_v[0] = (0.9, 0.3, -0.2)
    d0.rigid_w[0] = (0.0, 0.0, 1.0)
    d1 = si.cube_stack(seed=2, n=1, mu=0.5)
    d1.rigid_x[0] = Rz @ d0.rigid_x[0]
    d1.rigid_q[0] = npref.quat_mul(qz, d0.rigid_q[0])
    d1.rigid_v[0] = Rz @ d0.rigid_v[0]
    d1.rigid_w[0] = Rz @ d0.rigid_w[0]
    e0, e1 = O.OracleEnv(d0), O.OracleEnv(d1)
    converged(e0, h, N=200, tol=1e-11)
    converged(e1, h, N=200, tol=1e-11)
    s0, s1 = e0.get_state(), e1.get_state()
    # inputs were rounded to float32; compare at that level
    np.testing.assert_allclose(s1["rigid_x"][0], Rz @ s0["rigid_x"][0], atol=1e-6)
    np.testing.assert_allclose(s1["rigid_v"][0], Rz @ s0["rigid_v"][0], atol=1e-5)


# --------------------------------------------------------------------------- misc
def test_contact_keys_sorted_and_unique():
    d = si.tet_block_with_boxes(seed=0, cells=4, n_boxes=4)
    env = O.OracleEnv(d)
    env.step(1 / 60, 2, 10, 0.0)
    k = env.contacts()["key"]
    assert len(k) > 0 and (np.diff(k) > 0).all()


def test_invalid_inputs_rejected():
    d = si.single_tet()
    d.tet_ids[0, 1] = 99
    with pytest.raises(ValueError):
        O.OracleEnv(d)
    d = si.cube_stack(n=1)
    d.rigid_inertia[0, 0] = -1
    with pytest.raises(ValueError):
        O.OracleEnv(d)


def test_deep_penetration_stays_finite():
    d = si.cube_stack(n=1)
    d.rigid_x[0, 2] = 0.0  # 5 cm into the ground
    env = O.OracleEnv(d)
    for _ in range(10):
        st = env.step(1 / 60, 10, 40, 0.0)
        assert not st["nonfinite"]
    assert np.isfinite(env.get_state()["rigid_x"]).all()


def test_set_prev_matches_own_warm_start_bookkeeping():
    """Loading the previous-step multipliers through set_prev reproduces the oracle's
    own warm start (the GPU parity tests feed the GPU's values this way).  set_state
    renormalises quaternions, so the match is to rounding, not bitwise; leaving the
    multipliers out changes the step by far more."""
    d = si.batched_env(seed=1002, tets_max=60)
    op = O.make_params(si.SolverParams(warm=si.WARM_PREV))
    a = O.OracleEnv(d)
    a.step(1 / 60, 3, 20, 0.0, op)
    pre = a.get_state()
    t0 = a.time
    c = a.contacts()
    lj = a.lambdas()[:6 * d.n_joints]
    a.step(1 / 60, 3, 20, 0.0, op)
    b = O.OracleEnv(d)
    b.set_state(pre)
    b.time = t0
    b.set_prev(c["key"], c["lam"], lj)
    b.step(1 / 60, 3, 20, 0.0, op)
    assert len(c["key"]) > 0 and d.n_joints > 0
    cold = O.OracleEnv(d)
    cold.set_state(pre)
    cold.time = t0
    cold.step(1 / 60, 3, 20, 0.0, op)
    ref, got, nop = a.get_state(), b.get_state(), cold.get_state()
    for k in ref:
        np.testing.assert_allclose(got[k], ref[k], rtol=0, atol=1e-7, err_msg=k)
    assert max(np.abs(nop[k] - ref[k]).max() for k in ["rigid_v", "particle_v"]) > 1e-4
    with pytest.raises(ValueError):
        b.set_prev(c["key"][::-1].copy(), c["lam"], lj)  # keys must ascend


def test_warm_start_nonfinite_falls_back_to_plain_start():
    """Recovery rule: a warm-started step whose iterate turns non-finite (here an
    infinite previous normal multiplier) is rerun from the plain start, and then
    equals the plain step from the same state exactly."""
    d = si.cube_stack(seed=0, n=2)
    h = 1 / 60
    a = O.OracleEnv(d)
    a.step(h, 5, 20, 0.0, O.make_params(warm=0))
    pre, t0 = a.get_state(), a.time
    c = a.contacts()
    bad = np.array(c["lam"])
    bad[:, 0] = np.inf
    w = O.OracleEnv(d)
    w.set_state(pre)
    w.time = t0
    w.set_prev(c["key"], bad, np.zeros(0))
    st = w.step(h, 5, 20, 0.0, O.make_params(warm=1))
    assert st["fallback"] == 1 and st["nonfinite"] == 0
    z = O.OracleEnv(d)
    z.set_state(pre)
    z.time = t0
    stz = z.step(h, 5, 20, 0.0, O.make_params(warm=0))
    assert stz["fallback"] == 0
    for k, v in z.get_state().items():
        assert np.array_equal(v, w.get_state()[k]), k
    # the failed attempt stopped at its first residual (no update), so it adds no work
    assert st["newton_iters"] == stz["newton_iters"] and st["cr_iters"] == stz["cr_iters"]


# ------------------------------------------------------------- line search (Sec. 8.1)
@pytest.mark.parametrize("scene", ["lcp", "stack"])
def test_line_search_sufficient_decrease_and_same_solution(scene):
    """Sec. 8.1's back-tracking line search on the L2 merit (frictionless problems):
    every accepted iterate decreases the merit by the sufficient-decrease factor (or
    the step fraction reached its floor 1/64, which decreases it at least by
    1 - 1e-4/64), and the converged state equals the damped iteration's."""
    d = si.particles_vs_planes_lcp(seed=2) if scene == "lcp" else si.cube_stack(seed=3, n=4, mu=0.0)
    h = 1 / 60
    a, b = O.OracleEnv(d), O.OracleEnv(d)
    for s in range(3):
        st = a.step(h, 100, 80, 1e-10, O.make_params(line_search=1, damping=1.0))
        m = a.merit_history()
        assert st["r_ncp"] <= 1e-10 and len(m) >= 2
        assert (m[1:] <= (1 - 1e-4 / 64) * m[:-1]).all(), m
        stb = b.step(h, 200, 80, 1e-10, O.make_params(line_search=0, damping=0.75))
        assert stb["r_ncp"] <= 1e-10
        assert st["newton_iters"] < stb["newton_iters"]
        A, B = a.get_state(), b.get_state()
        for k in ["rigid_v", "particle_v"]:
            if A[k].size:
                np.testing.assert_allclose(A[k], B[k], atol=1e-7, err_msg=k)
        b.set_state(A)
        b.time = a.time


# ------------------------------------------------------------ PCG (solver study, Sec. 8.2)
def test_pcg_matches_direct_solve_and_minimises_energy_over_krylov_space():
    """Preconditioned CG: after n iterations it solves the system; its k-th iterate
    minimises the A-norm of the error over span{(PA)^j P b} (what distinguishes it
    from CR, which minimises the P-norm of the residual)."""
    rng = np.random.default_rng(9)
    for n in [3, 8, 20]:
        B = rng.normal(size=(n, n))
        A = B @ B.T + n * np.eye(n)
        b = rng.normal(size=n)
        P = 1 / np.diag(A)
        x, _ = O.pcg_dense(A, b, P, n)
        assert np.linalg.norm(A @ x - b) <= 1e-5 * np.linalg.norm(b)
    n = 12
    B = rng.normal(size=(n, n))
    A = B @ B.T + 0.5 * np.eye(n)
    b = rng.normal(size=n)
    P = 1 / np.diag(A)
    xs = np.linalg.solve(A, b)
    Lc = np.linalg.cholesky(A)
    for k in range(1, 7):
        x, _ = O.pcg_dense(A, b, P, k)
        K = [P * b]
        for _ in range(k - 1):
            K.append(P * (A @ K[-1]))
        K = np.stack(K, axis=1)
        # min_c |L^T (K c - xs)|  (A-norm of the error)
        c, *_ = np.linalg.lstsq(Lc.T @ K, Lc.T @ xs, rcond=None)
        np.testing.assert_allclose(x, K @ c, rtol=1e-6, atol=1e-8)


def test_pcg_residual_not_monotone_where_pcr_is():
    """The observation behind choosing CR (Sec. 8.2): on an ill-conditioned SPD system
    the preconditioned residual of CG rises between iterations, CR's never does."""
    rng = np.random.default_rng(11)
    found = False
    for trial in range(20):
        n = 30
        Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
        A = Q @ np.diag(np.logspace(0, 5, n)) @ Q.T
        b = rng.normal(size=n)
        P = 1 / np.diag(A)
        _, hg = O.pcg_dense(A, b, P, 25)
        _, hr = O.pcr_dense(A, b, P, 25)
        assert (np.diff(hr) <= 1e-12 * hr[0]).all()
        if (np.diff(hg) > 1e-6 * hg[0]).any():
            found = True
            break
    assert found


# ------------------------------------------------------------------ islands (Sec. 11)
def test_islands_solve_the_same_system():
    """One PCR per island (independent CR scalars) solves the same block-diagonal
    system: steps converged to r_ncp <= 1e-9 agree with those of one PCR over the whole
    env; an env with a single island gives identical steps."""
    h = 1 / 60
    multi = si.batched_env(seed=1005, tets_max=0)  # stacks and chains: several islands
    for d, exact in [(multi, False), (si.cube_stack(seed=1, n=3), True)]:
        a, b = O.OracleEnv(d), O.OracleEnv(d)
        for _ in range(3):
            sa = a.step(h, 100, 400, 1e-9, O.make_params(islands=1))
            sb = b.step(h, 100, 400, 1e-9, O.make_params(islands=0))
            assert sa["r_ncp"] <= 1e-9 and sb["r_ncp"] <= 1e-9
        A, B = a.get_state(), b.get_state()
        for k in A:
            if A[k].size:
                if exact:
                    assert np.array_equal(A[k], B[k]), k
                else:
                    # the rounding-level PCR stop is relative to each island's own start
                    np.testing.assert_allclose(A[k], B[k], atol=1e-6, err_msg=k)


def test_islands_early_exit_keeps_solved_island():
    """Early exit of a solved island (residual mode): two particles resting on the
    ground are two islands.  After a settling step, particle B is thrown down; from the
    previous-step start particle A is solved at the first iterate, so it keeps its start
    velocity and multipliers exactly while B's island iterates to the tolerance.
    Without islands A takes part in every update."""
    h, tol = 1 / 60, 1e-5
    d = si.particle_on_plane(mu=0.5)
    d.particle_x = np.array([[0.1, -0.2, 0.0], [2.0, 0.5, 0.0]])
    d.particle_rest = d.particle_x.copy()
    d.particle_v = np.zeros((2, 3))
    d.particle_mass = np.array([1.0, 1.0])
    d = d.finalize()
    out = {}
    for isl in (1, 0):
        env = O.OracleEnv(d)
        p = O.make_params(si.SolverParams(islands=isl, warm=si.WARM_PREV))
        # settle far below the step's tolerance, so that A starts the next step solved
        assert env.step(h, 50, 40, 1e-10, p)["r_ncp"] <= 1e-10
        S = env.get_state()
        lam0 = env.contacts()["lam"].copy()
        S["particle_v"][1] = [0.3, 0.0, -1.0]
        env.set_state({k: v for k, v in S.items() if k != "time"})
        st = env.step(h, 50, 40, tol, p)
        assert st["r_ncp"] <= tol and st["newton_iters"] >= 2, st
        out[isl] = (S["particle_v"][0].copy(), env.get_state()["particle_v"][0], lam0, env.contacts())
    v0, v1, lam0, con = out[1]
    assert np.array_equal(v0, v1)
    # particle A's contact has the lower key in both steps
    assert np.array_equal(con["lam"][0], lam0[0])
    v0n, v1n, _, _ = out[0]
    assert not np.array_equal(v0n, v1n)
