"""Learned warm start: dataset generation from the solver's own trajectories and
training of the 12 -> 64 -> 64 -> 64 -> 3 MLP with the library's BF16-MFMA forward /
backward kernels and its Adam kernel (nsn_mlp_loss_grad, nsn_mlp_adam).  Python only
drives the loop: batching indices, learning-rate schedule, bookkeeping.

Weights blob (float32): 9347 parameters (W1[64x12] b1 W2[64x64] b2 W3[64x64] b3 W4[3x64]
b4) followed by x_mean[12] x_std[12] y_mean[3] y_std[3]."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L

N_PARAMS = 9347
N_IN, N_OUT = 12, 3


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    w = np.zeros(N_PARAMS, np.float32)
    o = 0
    for shape in [(64, 12), (64,), (64, 64), (64,), (64, 64), (64,), (3, 64), (3,)]:
        n = int(np.prod(shape))
        if len(shape) == 2:  # He initialisation for ReLU layers
            w[o:o + n] = rng.normal(scale=np.sqrt(2.0 / shape[1]), size=n)
        o += n
    return w


def standardisation(x, t):
    xm, xs = x.mean(0), x.std(0)
    ym, ys = t.mean(0), t.std(0)
    xs = np.where(xs > 1e-6, xs, 1.0)
    ys = np.where(ys > 1e-6, ys, 1.0)
    return xm.astype(np.float32), xs.astype(np.float32), ym.astype(np.float32), ys.astype(np.float32)


def train_mlp(x, t, epochs=20, batch=4096, lr=2e-3, seed=0, log=None, device="cuda"):
    """Train on features x [n,12] and targets t [n,3] (raw units).  Returns the weights
    blob and the per-epoch mean loss (standardised units)."""
    import torch

    lib = L.lib()
    if not (np.isfinite(x).all() and np.isfinite(t).all()):
        raise ValueError("training data holds non-finite values")
    # steps that diverged leave a few multipliers orders of magnitude above the rest;
    # they would set the target scale, so every column is clipped to its
    # 0.05..99.95 % quantiles (a warm start need not reproduce them)
    x = np.clip(x, *np.quantile(x, [5e-4, 1 - 5e-4], axis=0))
    t = np.clip(t, *np.quantile(t, [5e-4, 1 - 5e-4], axis=0))
    xm, xs, ym, ys = standardisation(x, t)
    xn = torch.tensor((x - xm) / xs, dtype=torch.float32, device=device)
    tn = torch.tensor((t - ym) / ys, dtype=torch.float32, device=device)
    n = xn.shape[0]
    w = torch.tensor(init_params(seed), device=device)
    g = torch.zeros_like(w)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    loss = torch.zeros(1, dtype=torch.float32, device=device)
    scratch = torch.zeros(lib.nsn_mlp_scratch_bytes(batch) // 4 + 1, dtype=torch.float32, device=device)
    stream = torch.cuda.current_stream().cuda_stream
    gen = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(device)
        tot, cnt = 0.0, 0
        lr_ep = lr * 0.5 * (1 + np.cos(np.pi * ep / max(epochs, 1)))  # cosine schedule
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            xb = xn.index_select(0, idx).contiguous()
            tb = tn.index_select(0, idx).contiguous()
            nb = xb.shape[0]
            L.check(lib.nsn_mlp_loss_grad(w.data_ptr(), xb.data_ptr(), tb.data_ptr(), nb, g.data_ptr(),
                                          loss.data_ptr(), scratch.data_ptr(), C.c_void_p(stream)),
                    "nsn_mlp_loss_grad")
            step += 1
            L.check(lib.nsn_mlp_adam(w.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), N_PARAMS,
                                     C.c_float(lr_ep), C.c_float(0.9), C.c_float(0.999), C.c_float(1e-8), step,
                                     C.c_void_p(stream)), "nsn_mlp_adam")
            lv = loss.item()
            if not np.isfinite(lv):
                raise FloatingPointError(f"training loss became non-finite in epoch {ep + 1}")
            tot += lv * nb
            cnt += nb
        hist.append(tot / cnt)
        if log:
            log(f"epoch {ep + 1}/{epochs} loss {hist[-1]:.5e}")
    blob = np.concatenate([w.cpu().numpy(), xm, xs, ym, ys]).astype(np.float32)
    return blob, hist


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
