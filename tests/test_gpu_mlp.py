"""BF16-MFMA MLP kernels of the learned warm start against the FP64 oracle MLP.

The GPU rounds weights and activations to bf16 where they enter a product (8-bit
mantissa, relative rounding 2^-9) and accumulates in FP32; the tolerances below are a
few times that rounding, far below the size of a layout or transposition mistake
(which gives O(1) errors)."""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

NP = 9347


def _bf16(a):
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _init_weights(rng):
    w = np.zeros(NP)
    sizes = [(64, 12), (64,), (64, 64), (64,), (64, 64), (64,), (3, 64), (3,)]
    o = 0
    for s in sizes:
        n = int(np.prod(s))
        fan_in = s[1] if len(s) == 2 else 64
        w[o:o + n] = rng.normal(scale=np.sqrt(2.0 / fan_in), size=n) if len(s) == 2 else rng.normal(scale=0.1, size=n)
        o += n
    return w


def _torch():
    import torch
    return torch


def _lib():
    from paper_1907_04587_amd import _lib as L
    return L, L.lib()


def test_forward_matches_oracle():
    torch = _torch()
    L, lib = _lib()
    rng = np.random.default_rng(0)
    w = _init_weights(rng)
    for n in [1, 15, 16, 17, 1000, 4099]:
        x = rng.normal(size=(n, 12))
        wd = torch.tensor(w, dtype=torch.float32, device="cuda")
        xd = torch.tensor(x, dtype=torch.float32, device="cuda")
        yd = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
        st = lib.nsn_mlp_forward(wd.data_ptr(), xd.data_ptr(), yd.data_ptr(), n, None)
        assert st == 0
        torch.cuda.synchronize()
        # oracle on the bf16-rounded weights and inputs (the GPU's operands)
        wr = _bf16(w)
        for off, cnt in [(64 * 12, 64), (64 * 12 + 64 + 4096, 64), (64 * 12 + 64 + 4096 + 64 + 4096, 64),
                         (NP - 3, 3)]:
            wr[off:off + cnt] = w[off:off + cnt]  # biases stay fp32
        yr = O.mlp_forward(wr, _bf16(x))
        y = yd.cpu().numpy()
        scale = np.abs(yr).max() + 1e-6
        assert np.abs(y - yr).max() < 2e-2 * scale, (n, np.abs(y - yr).max(), scale)


def test_loss_gradient_matches_oracle():
    torch = _torch()
    L, lib = _lib()
    rng = np.random.default_rng(1)
    w = _init_weights(rng)
    n = 3000
    x = rng.normal(size=(n, 12))
    t = rng.normal(size=(n, 3))
    wd = torch.tensor(w, dtype=torch.float32, device="cuda")
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    gd = torch.zeros(NP, dtype=torch.float32, device="cuda")
    ld = torch.zeros(1, dtype=torch.float32, device="cuda")
    scratch = torch.zeros(lib.nsn_mlp_scratch_bytes(n) // 4 + 1, dtype=torch.float32, device="cuda")
    st = lib.nsn_mlp_loss_grad(wd.data_ptr(), xd.data_ptr(), td.data_ptr(), n, gd.data_ptr(), ld.data_ptr(),
                               scratch.data_ptr(), None)
    assert st == 0
    torch.cuda.synchronize()
    loss_ref, g_ref = O.mlp_loss_grad(w, x, t)
    g = gd.cpu().numpy().astype(np.float64)
    assert ld.item() == pytest.approx(loss_ref, rel=2e-2)
    cos = g @ g_ref / (np.linalg.norm(g) * np.linalg.norm(g_ref))
    assert cos > 0.999, cos
    assert np.linalg.norm(g - g_ref) < 3e-2 * np.linalg.norm(g_ref)
    # every parameter block individually (a transposed block would fail here)
    offs = [0, 768, 832, 4928, 4992, 9088, 9152, 9344, 9347]
    for a, b in zip(offs[:-1], offs[1:]):
        ga, gr = g[a:b], g_ref[a:b]
        assert np.linalg.norm(ga - gr) < 5e-2 * (np.linalg.norm(gr) + 1e-8), (a, b)


def test_gradient_deterministic():
    torch = _torch()
    L, lib = _lib()
    rng = np.random.default_rng(2)
    w = torch.tensor(_init_weights(rng), dtype=torch.float32, device="cuda")
    x = torch.tensor(rng.normal(size=(5000, 12)), dtype=torch.float32, device="cuda")
    t = torch.tensor(rng.normal(size=(5000, 3)), dtype=torch.float32, device="cuda")
    out = []
    for _ in range(2):
        g = torch.zeros(NP, dtype=torch.float32, device="cuda")
        scratch = torch.zeros(lib.nsn_mlp_scratch_bytes(5000) // 4 + 1, dtype=torch.float32, device="cuda")
        assert lib.nsn_mlp_loss_grad(w.data_ptr(), x.data_ptr(), t.data_ptr(), 5000, g.data_ptr(), None,
                                     scratch.data_ptr(), None) == 0
        torch.cuda.synchronize()
        out.append(g.cpu().numpy())
    assert np.array_equal(out[0], out[1])


def test_adam_update():
    torch = _torch()
    L, lib = _lib()
    rng = np.random.default_rng(3)
    n = 1000
    w0, g0 = rng.normal(size=n), rng.normal(size=n)
    m0, v0 = rng.normal(size=n) * 0.1, rng.uniform(0, 1, size=n)
    w, g = torch.tensor(w0, dtype=torch.float32, device="cuda"), torch.tensor(g0, dtype=torch.float32, device="cuda")
    m, v = torch.tensor(m0, dtype=torch.float32, device="cuda"), torch.tensor(v0, dtype=torch.float32, device="cuda")
    lr, b1, b2, eps, step = 1e-3, 0.9, 0.999, 1e-8, 7
    assert lib.nsn_mlp_adam(w.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), n, C.c_float(lr), C.c_float(b1),
                            C.c_float(b2), C.c_float(eps), step, None) == 0
    torch.cuda.synchronize()
    m1 = b1 * m0 + (1 - b1) * g0
    v1 = b2 * v0 + (1 - b2) * g0 * g0
    w1 = w0 - lr * (m1 / (1 - b1 ** step)) / (np.sqrt(v1 / (1 - b2 ** step)) + eps)
    np.testing.assert_allclose(w.cpu().numpy(), w1, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss():
    from paper_1907_04587_amd.warmstart import train_mlp
    rng = np.random.default_rng(4)
    x = rng.normal(size=(20000, 12)).astype(np.float32)
    t = np.stack([np.maximum(x[:, 0] + 0.5 * x[:, 3], 0), 0.3 * x[:, 1] * x[:, 2], np.tanh(x[:, 5])], 1).astype(np.float32)
    blob, hist = train_mlp(x, t, epochs=15, batch=2048, lr=3e-3, seed=0, log=print)
    assert hist[-1] < 0.25 * hist[0], hist


def _gpu_grad(lib, torch, w, x, t):
    n = x.shape[0]
    wd = torch.tensor(w, dtype=torch.float32, device="cuda")
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    gd = torch.zeros(NP, dtype=torch.float32, device="cuda")
    ld = torch.zeros(1, dtype=torch.float32, device="cuda")
    scratch = torch.zeros(lib.nsn_mlp_scratch_bytes(n) // 4 + 1, dtype=torch.float32, device="cuda")
    assert lib.nsn_mlp_loss_grad(wd.data_ptr(), xd.data_ptr(), td.data_ptr(), n, gd.data_ptr(), ld.data_ptr(),
                                 scratch.data_ptr(), None) == 0
    torch.cuda.synchronize()
    return ld.item(), gd.cpu().numpy().astype(np.float64)


def test_loss_gradient_elementwise_against_bf16_oracle():
    """Every one of the 9347 gradient entries against the oracle's backpropagation with
    the kernels' bf16 operand rounding (sums in FP64).  Samples whose pre-activations
    come within 1e-3 of a ReLU kink in the rounded forward pass are left out: there the
    FP32 and FP64 sums may take different sides of the kink.  Tolerance: 1e-5 of the
    largest entry of the parameter block (FP32 accumulation over the samples and the
    odd one-ulp bf16 rounding flip of an FP32-computed operand; measured about 2e-7)."""
    torch = _torch()
    L, lib = _lib()
    rng = np.random.default_rng(11)
    w = np.asarray(_init_weights(rng), np.float32).astype(np.float64)
    x = rng.normal(size=(4000, 12)).astype(np.float32).astype(np.float64)
    t = rng.normal(size=(4000, 3)).astype(np.float32).astype(np.float64)
    pre = O.mlp_preact_bf16(w, x)
    keep = (np.abs(pre) > 1e-3).all(axis=(1, 2))
    x, t = x[keep], t[keep]
    assert x.shape[0] > 1000, x.shape
    loss, g = _gpu_grad(lib, torch, w, x, t)
    loss_ref, g_ref = O.mlp_loss_grad_bf16(w, x, t)
    assert loss == pytest.approx(loss_ref, rel=1e-5)
    offs = [0, 768, 832, 4928, 4992, 9088, 9152, 9344, 9347]
    names = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]
    for name, a, b in zip(names, offs[:-1], offs[1:]):
        scale = np.abs(g_ref[a:b]).max()
        err = np.abs(g[a:b] - g_ref[a:b]).max()
        print(f"grad {name}: max err {err / scale:.2e} of the block's largest entry", flush=True)
        assert err <= 1e-5 * scale, (name, err, scale)


def _numpy_standardise(x, t, q):
    cols = np.concatenate([x, t], 1).astype(np.float64)
    if q > 0:
        qf = float(np.float32(q))  # the library takes q as a float32 parameter
        lo = np.quantile(cols, qf, axis=0)
        hi = np.quantile(cols, 1 - qf, axis=0)
        cols = np.clip(cols, lo.astype(np.float32), hi.astype(np.float32))
    m, s = cols.mean(0), cols.std(0)
    s = np.where(s > 1e-6, s, 1.0)
    return cols, m, s


def test_training_data_preparation_in_library():
    """nsn_train_warm_start's clipping and z-scoring: the blob's statistics against
    NumPy's quantiles (linear interpolation) and moments of the clipped columns."""
    from paper_1907_04587_amd.warmstart import train_mlp
    rng = np.random.default_rng(5)
    n = 5001
    x = rng.normal(size=(n, 12)).astype(np.float32)
    x[:, 3] *= 50.0
    x[rng.choice(n, 7, replace=False), 2] = 1e4  # outliers the clipping removes
    t = rng.standard_cauchy(size=(n, 3)).astype(np.float32)
    t[:, 2] = 0.5  # a constant column: deviation counts as 1
    for q in [5e-4, 0.0]:
        blob, hist = train_mlp(x, t, epochs=1, batch=1024, lr=1e-3, seed=1, clip_quantile=q)
        _, m, s = _numpy_standardise(x, t, q)
        tail = blob[NP:].astype(np.float64)
        # means to 1e-6 of the column's deviation, deviations to 1e-5 relative
        assert (np.abs(tail[:12] - m[:12]) <= 1e-6 * s[:12] + 1e-5 * np.abs(m[:12])).all(), (q, tail[:12], m[:12])
        assert (np.abs(tail[12:24] - s[:12]) <= 1e-5 * s[:12]).all(), (q, tail[12:24], s[:12])
        assert (np.abs(tail[24:27] - m[12:]) <= 1e-6 * s[12:] + 1e-5 * np.abs(m[12:])).all(), (q, tail[24:27], m[12:])
        assert (np.abs(tail[27:30] - s[12:]) <= 1e-5 * s[12:]).all(), (q, tail[27:30], s[12:])
        assert tail[29] == 1.0


def test_training_step_is_one_adam_update_of_the_library_gradient():
    """One epoch of one full batch from given weights: the result is w minus one Adam
    step (bias-corrected, the first step of the cosine schedule at the full rate) of
    the loss gradient of the standardised data."""
    torch = _torch()
    L, lib = _lib()
    from paper_1907_04587_amd.warmstart import init_params, train_mlp
    rng = np.random.default_rng(6)
    n = 2048
    x = rng.normal(size=(n, 12)).astype(np.float32)
    t = rng.normal(size=(n, 3)).astype(np.float32)
    w0 = init_params(3)
    lr = 1e-3
    blob, hist = train_mlp(x, t, epochs=1, batch=n, lr=lr, seed=2, clip_quantile=0.0, w_init=w0)
    cols, m, s = _numpy_standardise(x, t, 0.0)
    xs = ((cols[:, :12] - m[:12]) / s[:12]).astype(np.float32)
    ts = ((cols[:, 12:] - m[12:]) / s[12:]).astype(np.float32)
    loss, g = _gpu_grad(lib, torch, w0, xs, ts)
    assert hist[0] == pytest.approx(loss, rel=1e-4)
    step = lr * g / (np.abs(g) + 1e-8)
    d = np.abs(blob[:NP] - (w0 - step))
    assert d.max() <= 0.05 * lr, d.max()
    assert (d > 1e-3 * lr).sum() <= 5, (d > 1e-3 * lr).sum()


def test_training_deterministic_and_seeded():
    from paper_1907_04587_amd.warmstart import train_mlp
    rng = np.random.default_rng(7)
    x = rng.normal(size=(3000, 12)).astype(np.float32)
    t = rng.normal(size=(3000, 3)).astype(np.float32)
    a, _ = train_mlp(x, t, epochs=2, batch=512, seed=4)
    b, _ = train_mlp(x, t, epochs=2, batch=512, seed=4)
    c, _ = train_mlp(x, t, epochs=2, batch=512, seed=5)
    assert np.array_equal(a, b)
    assert not np.array_equal(a[:NP], c[:NP])
