"""Learned warm start: dataset generation from the solver's own trajectories and
training of the 12 -> 64 -> 64 -> 64 -> 3 MLP by the library (nsn_train_warm_start: its
BF16-MFMA forward / backward kernels and its Adam kernel, with the data preparation and
the epoch loop in the library too).  Python only marshals the arrays.

Weights blob (float32): 9347 parameters (W1[64x12] b1 W2[64x64] b2 W3[64x64] b3 W4[3x64]
b4) followed by x_mean[12] x_std[12] y_mean[3] y_std[3]."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L

N_PARAMS = 9347
N_IN, N_OUT = 12, 3


def init_params(seed=0):
    """He-initialised parameters drawn on the host (for tests that need known weights;
    nsn_train_warm_start draws its own on the device)."""
    rng = np.random.default_rng(seed)
    w = np.zeros(N_PARAMS, np.float32)
    o = 0
    for shape in [(64, 12), (64,), (64, 64), (64,), (64, 64), (64,), (3, 64), (3,)]:
        n = int(np.prod(shape))
        if len(shape) == 2:  # He initialisation for ReLU layers
            w[o:o + n] = rng.normal(scale=np.sqrt(2.0 / shape[1]), size=n)
        o += n
    return w


def train_mlp(x, t, epochs=20, batch=4096, lr=2e-3, seed=0, clip_quantile=5e-4, w_init=None, log=None,
              device="cuda"):
    """Train on features x [n,12] and targets t [n,3] (raw units) with the library's
    nsn_train_warm_start: quantile clipping, z-scoring, initialisation, shuffling,
    mini-batches and Adam all run on the device.  Returns the weights blob (parameters
    and standardisation) and the per-epoch mean loss (standardised units)."""
    import torch

    lib = L.lib()
    xd = torch.as_tensor(np.ascontiguousarray(x, np.float32)).to(device)
    td = torch.as_tensor(np.ascontiguousarray(t, np.float32)).to(device)
    n = int(xd.shape[0])
    ws_bytes = lib.nsn_train_workspace_bytes(n, int(batch))
    if ws_bytes == 0:
        raise L.NSNError("nsn_train_workspace_bytes: bad sizes or sort query failed")
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
    blob = torch.zeros(N_PARAMS + 2 * N_IN + 2 * N_OUT, dtype=torch.float32, device=device)
    w0 = None if w_init is None else torch.as_tensor(np.ascontiguousarray(w_init, np.float32)).to(device)
    hist = np.zeros(int(epochs), np.float64)
    tp = L.TrainParamsC(epochs=int(epochs), batch=int(batch), lr=float(lr), beta1=0.9, beta2=0.999, adam_eps=1e-8,
                        clip_quantile=float(clip_quantile), seed=int(seed))
    stream = torch.cuda.current_stream().cuda_stream
    L.check(lib.nsn_train_warm_start(xd.data_ptr(), td.data_ptr(), n, C.byref(tp),
                                     w0.data_ptr() if w0 is not None else None, blob.data_ptr(),
                                     hist.ctypes.data_as(L.D), ws.data_ptr(), ws_bytes, C.c_void_p(stream)),
            "nsn_train_warm_start")
    if log:
        for ep, v in enumerate(hist):
            log(f"epoch {ep + 1}/{epochs} loss {v:.5e}")
    return blob.cpu().numpy(), list(hist)


def predict(blob, x, device="cuda"):
    """MLP prediction in raw units on the device (BF16 MFMA kernel)."""
    import torch

    lib = L.lib()
    w = blob[:N_PARAMS]
    xm, xs = blob[N_PARAMS:N_PARAMS + 12], blob[N_PARAMS + 12:N_PARAMS + 24]
    ym, ys = blob[N_PARAMS + 24:N_PARAMS + 27], blob[N_PARAMS + 27:N_PARAMS + 30]
    xd = torch.tensor((x - xm) / xs, dtype=torch.float32, device=device)
    wd = torch.tensor(w, dtype=torch.float32, device=device)
    yd = torch.zeros((x.shape[0], 3), dtype=torch.float32, device=device)
    L.check(lib.nsn_mlp_forward(wd.data_ptr(), xd.data_ptr(), yd.data_ptr(), x.shape[0],
                                C.c_void_p(torch.cuda.current_stream().cuda_stream)), "nsn_mlp_forward")
    return yd.cpu().numpy() * ys + ym


def generate_dataset(envs, steps, h, newton_iters=50, cr_iters=40, tol=1e-6, warmup=5, log=None):
    """Step `envs` (one batched scene) with the plain solver run tight; record for every
    contact the 12 step-start features and the final multipliers (lambda_n, lambda_t1,
    lambda_t2).  Returns (x [n,12], t [n,3])."""
    import scene_inputs as si

    from .scene import Scene

    sc = Scene(envs, si.SolverParams(warm=si.WARM_PREV))
    sc.enable_features(True)
    xs, ts = [], []
    for s in range(warmup + steps):
        sc.step(h, newton_iters, cr_iters, tol)
        if s < warmup:
            continue
        st = sc.stats()
        for e in range(len(envs)):
            if st["nonfinite"][e] or st["fallback"][e]:
                continue  # a step that failed from its start teaches nothing
            f = sc.features(e)
            if len(f) == 0:
                continue
            lam = sc.contacts(e)["lam"][:len(f)]
            ok = np.isfinite(f).all(1) & np.isfinite(lam).all(1)
            xs.append(f[ok])
            ts.append(lam[ok])
        if log and (s + 1) % 20 == 0:
            log(f"dataset step {s + 1}/{warmup + steps}: {sum(len(a) for a in xs)} contacts")
    return np.concatenate(xs), np.concatenate(ts)
