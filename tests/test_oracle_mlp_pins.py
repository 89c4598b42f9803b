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
