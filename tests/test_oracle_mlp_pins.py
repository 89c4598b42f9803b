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


# ---- the bf16-rounded backpropagation (the GPU kernels' operand rounding) ----

def _exact_net():
    """A network whose every operand and activation is a small multiple of 1/2 for
    inputs in {0, 1, 2}: sparse +-1 weights, half-integer first-layer biases (so no
    first-layer pre-activation is 0), integer biases elsewhere.  Every value that enters
    a product is then exactly representable in bfloat16, so rounding changes nothing."""
    off = _offsets()
    w = np.zeros(off[-1])
    W1 = w[off[0]:off[1]].reshape(NH, NIN); b1 = w[off[1]:off[2]]
    W2 = w[off[2]:off[3]].reshape(NH, NH); b2 = w[off[3]:off[4]]
    W3 = w[off[4]:off[5]].reshape(NH, NH); b3 = w[off[5]:off[6]]
    W4 = w[off[6]:off[7]].reshape(NOUT, NH); b4 = w[off[7]:off[8]]
    for o in range(NH):
        W1[o, o % NIN] = 1.0
        W1[o, (o + 5) % NIN] = -1.0 if o % 3 == 0 else 1.0
        b1[o] = 0.5 if o % 4 else -2.5
        W2[o, o] = 1.0
        W2[o, (o + 7) % NH] = -1.0 if o % 5 == 0 else 1.0
        b2[o] = 1.0
        W3[o, (o * 3) % NH] = 1.0
        W3[o, (o + 11) % NH] = 1.0 if o % 2 else -1.0
        b3[o] = -1.0 if o % 6 == 0 else 0.0
    for k in range(NOUT):
        W4[k, k] = 1.0
        W4[k, 10 + k] = -1.0
        W4[k, 20 + 3 * k] = 1.0
        b4[k] = float(k)
    x = np.array([[0, 1, 2, 1, 0, 2, 1, 1, 0, 2, 1, 0]], np.float64)
    return off, w, x


def _targets_for_unit_delta(w, x):
    # n = 1: dy = 2 (y - t) / 3, so y - t = 1.5 gives dy = 1 exactly
    return O.mlp_forward(w, x) - 1.5


def test_bf16_backprop_equals_plain_when_every_operand_is_exact():
    """Pins structure (layers, transposes, masks, bias and weight gradients): with
    exactly representable operands the rounded backpropagation is the plain one."""
    off, w, x = _exact_net()
    t = _targets_for_unit_delta(w, x)
    l0, g0 = O.mlp_loss_grad(w, x, t)
    l1, g1 = O.mlp_loss_grad_bf16(w, x, t)
    assert l1 == l0
    assert np.array_equal(g1, g0)
    assert np.count_nonzero(g0[off[0]:off[1]]) > 10  # the gradient reaches layer 1


def test_bf16_backprop_rounds_inputs_and_weights():
    """An input of 1 + 2^-10 and a W2 entry of 1 + 2^-10 are 1 in bfloat16 (8 significant
    bits): the rounded backpropagation equals the plain one at the rounded values and
    differs from the plain one at the given values."""
    off, w, x = _exact_net()
    t = _targets_for_unit_delta(w, x)
    xr = x.copy()
    i = int(np.flatnonzero(x[0] == 1.0)[0])
    x2 = x.copy()
    x2[0, i] = 1.0 + 2.0 ** -10
    w2 = w.copy()
    j = off[2] + 5 * NH + 5  # W2[5, 5] = 1
    assert w[j] == 1.0
    w2[j] = 1.0 + 2.0 ** -10
    l_ref, g_ref = O.mlp_loss_grad(w, xr, t)
    l1, g1 = O.mlp_loss_grad_bf16(w2, x2, t)
    assert l1 == l_ref and np.array_equal(g1, g_ref)
    l_plain, g_plain = O.mlp_loss_grad(w2, x2, t)
    assert not np.array_equal(g_plain, g_ref)


def test_bf16_backprop_rounds_activations_and_deltas():
    """Adding 2^-10 to the first-layer biases makes every positive layer-1 activation a
    half-integer plus 2^-10, which rounds to the half-integer where it enters layer 2
    (the bias gradient and the ReLU mask keep the unrounded value).  A target offset that makes dy =
    1 + 2^-10 rounds dy to 1 in the weight gradient of layer 4 and in the delta sent
    back, but not in the bias gradient b4."""
    off, w, x = _exact_net()
    b1 = slice(off[1], off[2])
    t = _targets_for_unit_delta(w, x)
    wa = w.copy()
    wa[b1] += 2.0 ** -10
    assert (O.mlp_preact_bf16(wa, x)[0, 0] != 0).all()
    l_ref, g_ref = O.mlp_loss_grad(w, x, t)
    la, ga = O.mlp_loss_grad_bf16(wa, x, t)
    assert la == l_ref and np.array_equal(ga, g_ref)
    assert not np.array_equal(O.mlp_loss_grad(wa, x, t)[1], g_ref)
    t2 = O.mlp_forward(w, x) - 1.5 * (1.0 + 2.0 ** -10)
    l2, g2 = O.mlp_loss_grad_bf16(w, x, t2)
    b4 = slice(off[7], off[8])
    np.testing.assert_array_equal(g2[b4], np.full(NOUT, 1.0 + 2.0 ** -10))
    keep = np.ones(off[-1], bool)
    keep[b4] = False
    assert np.array_equal(g2[keep], g_ref[keep])


def test_bf16_backprop_within_bf16_error_of_plain():
    """On random data the rounded gradient stays within the bfloat16 operand error
    (relative 2^-9 per rounding, a few roundings deep) of the plain gradient."""
    rng = np.random.default_rng(3)
    off = _offsets()
    w = rng.normal(scale=0.2, size=off[-1])
    x = rng.normal(size=(300, NIN))
    t = rng.normal(size=(300, NOUT))
    l0, g0 = O.mlp_loss_grad(w, x, t)
    l1, g1 = O.mlp_loss_grad_bf16(w, x, t)
    assert abs(l1 - l0) < 2e-2 * l0
    for a, b in zip(off[:-1], off[1:]):
        assert np.linalg.norm(g1[a:b] - g0[a:b]) < 3e-2 * np.linalg.norm(g0[a:b])
