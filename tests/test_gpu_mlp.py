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
