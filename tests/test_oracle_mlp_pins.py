"""Pins of the oracle's FP64 warm-start MLP (12 -> 64 -> 64 -> 64 -> 3, ReLU)."""
import numpy as np

from oracle import oracle as O

NIN, NH, NOUT = 12, 64, 3


def _offsets():
    sizes = [NH * NIN, NH, NH * NH, NH, NH * NH, NH, NOUT * NH, NOUT]
    return np.cumsum([0] + sizes)


def test_param_count():
    assert O.mlp_num_params() == 9347 == _offsets()[-1]


def test_forward_constructed_weights_route_inputs():
    """Weights built so that y0 = relu(x3 - 0.5), y1 = 2*relu(x7), y2 = -1 + relu(-x0):
    pins the layer order, the row-major [out x in] layout and where ReLU applies."""
    off = _offsets()
    w = np.zeros(off[-1])
    W1 = w[off[0]:off[1]].reshape(NH, NIN); b1 = w[off[1]:off[2]]
    W2 = w[off[2]:off[3]].reshape(NH, NH); W3 = w[off[4]:off[5]].reshape(NH, NH)
    W4 = w[off[6]:off[7]].reshape(NOUT, NH); b4 = w[off[7]:off[8]]
    W1[0, 3] = 1.0; b1[0] = -0.5
    W1[1, 7] = 1.0
    W1[2, 0] = -1.0
    for k in range(3):
        W2[k, k] = 1.0; W3[k, k] = 1.0
    W4[0, 0] = 1.0; W4[1, 1] = 2.0; W4[2, 2] = 1.0; b4[2] = -1.0
    rng = np.random.default_rng(0)
    x = rng.normal(size=(50, NIN))
    y = O.mlp_forward(w, x)
    np.testing.assert_allclose(y[:, 0], np.maximum(x[:, 3] - 0.5, 0), atol=1e-15)
    np.testing.assert_allclose(y[:, 1], 2 * np.maximum(x[:, 7], 0), atol=1e-15)
    np.testing.assert_allclose(y[:, 2], -1 + np.maximum(-x[:, 0], 0), atol=1e-15)


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    w = rng.normal(scale=0.3, size=O.mlp_num_params())
    x = rng.normal(size=(16, NIN))
    t = rng.normal(size=(16, NOUT))
    loss, g = O.mlp_loss_grad(w, x, t)
    y = O.mlp_forward(w, x)
    assert loss == np.mean((y - t) ** 2)  or abs(loss - np.mean((y - t) ** 2)) < 1e-14
    eps = 1e-6
    idx = rng.choice(w.size, size=120, replace=False)
    idx = np.concatenate([idx, _offsets()[:-1]])  # first entry of every block
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += eps; wm[i] -= eps
        fd = (O.mlp_loss_grad(wp, x, t)[0] - O.mlp_loss_grad(wm, x, t)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd))


def _constant_model(ym):
    """A warm-start blob whose network outputs the constant ym for every input: all
    weights zero, unit input and output scales."""
    n = O.mlp_num_params()
    blob = np.zeros(n + 30)
    blob[n + 12:n + 24] = 1.0      # x_std
    blob[n + 24:n + 27] = ym       # y_mean
    blob[n + 27:n + 30] = 1.0      # y_std
    return blob


def test_hybrid_warm_start_keeps_known_contacts_and_predicts_new_ones():
    """Mode 3 takes the previous-step multipliers for every contact whose key existed
    in the previous step and the network's prediction for the others.  With a network
    that outputs the constant (c, 0, 0): known contacts start exactly at their previous
    values, new contacts at (c, 0, 0); mode 2 puts (c, 0, 0) everywhere.  Two special
    cases reduce to other modes: with every key known, a whole step equals the
    previous-step start (mode 1); with no previous step, it equals mode 2."""
    import scene_inputs as si
    d = si.cube_stack(seed=0, n=3)
    h = 1 / 60
    a = O.OracleEnv(d)
    for _ in range(3):
        a.step(h, 20, 40, 0.0, O.make_params(warm=1))
    pre, t0 = a.get_state(), a.time
    c = a.contacts()
    lj = a.lambdas()[:6 * d.n_joints]
    assert len(c["key"]) >= 8 and (c["lam"][:, 0] > 0).any()
    cc = 0.25

    def run(mode, newton=0, drop=0, prev=True):
        e = O.OracleEnv(d)
        e.set_state(pre)
        e.time = t0
        if prev:
            e.set_prev(c["key"][drop:], c["lam"][drop:], lj)
        e.set_mlp(_constant_model([cc, 0.0, 0.0]))
        e.step(h, newton, 40, 0.0, O.make_params(warm=mode))
        return e

    # the first three keys are left out of the previous step: they are new contacts
    got = run(3, drop=3).contacts()
    prev = {int(k): l for k, l in zip(c["key"][3:], c["lam"][3:])}
    n_new = 0
    for k, l in zip(got["key"], got["lam"]):
        if int(k) in prev:
            np.testing.assert_array_equal(l, prev[int(k)])
        else:
            np.testing.assert_allclose(l, [cc, 0.0, 0.0], rtol=0, atol=1e-15)
            n_new += 1
    assert n_new >= 3 and len(got["key"]) > n_new
    l2 = run(2, drop=3).contacts()["lam"]
    np.testing.assert_allclose(l2, np.tile([cc, 0.0, 0.0], (len(l2), 1)), rtol=0, atol=1e-15)
    assert set(int(k) for k in run(3).contacts()["key"]) <= set(int(k) for k in c["key"])  # all known
    for (m1, kw1), (m2, kw2) in [((3, {}), (1, {})), ((3, {"prev": False}), (2, {"prev": False}))]:
        s1, s2 = run(m1, newton=5, **kw1), run(m2, newton=5, **kw2)
        for k, v in s2.get_state().items():
            assert np.array_equal(v, s1.get_state()[k]), (m1, m2, k)
