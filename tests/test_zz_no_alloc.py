"""nsn_mlp_loss_grad_noalloc (the entry point for callers that cannot allocate: its
scratch is a file-scope device array) against nsn_mlp_loss_grad with a caller-given
scratch buffer: the same kernels and reduction order, so the results are identical bit
for bit; two calls in a row, the second with a smaller input; sizes beyond the array
are refused."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NP = 9347


def _case(lib, torch, rng, n):
    w = torch.tensor(rng.normal(scale=0.2, size=NP), dtype=torch.float32, device="cuda")
    x = torch.tensor(rng.normal(size=(n, 12)), dtype=torch.float32, device="cuda")
    t = torch.tensor(rng.normal(size=(n, 3)), dtype=torch.float32, device="cuda")
    g_ref = torch.zeros(NP, dtype=torch.float32, device="cuda")
    l_ref = torch.zeros(1, dtype=torch.float32, device="cuda")
    scratch = torch.zeros(lib.nsn_mlp_scratch_bytes(n) // 4 + 1, dtype=torch.float32, device="cuda")
    assert lib.nsn_mlp_loss_grad(w.data_ptr(), x.data_ptr(), t.data_ptr(), n, g_ref.data_ptr(), l_ref.data_ptr(),
                                 scratch.data_ptr(), None) == 0
    g = torch.full((NP,), float("nan"), dtype=torch.float32, device="cuda")
    l = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    assert lib.nsn_mlp_loss_grad_noalloc(w.data_ptr(), x.data_ptr(), t.data_ptr(), n, g.data_ptr(), l.data_ptr(),
                                         None) == 0, lib.nsn_last_error()
    torch.cuda.synchronize()
    return g_ref.cpu().numpy(), l_ref.item(), g.cpu().numpy(), l.item()


def test_noalloc_matches_scratch_entry_point_twice():
    import torch
    from paper_1907_04587_amd import _lib as L
    lib = L.lib()
    rng = np.random.default_rng(17)
    for n in (70_000, 1_000):  # the second call smaller: fewer workgroups' partials in use
        g_ref, l_ref, g, l = _case(lib, torch, rng, n)
        assert np.array_equal(g, g_ref), (n, np.abs(g - g_ref).max())
        assert l == l_ref
        print(f"n {n}: gradient identical, loss {l:.6e}", flush=True)


def test_noalloc_refuses_and_reports_bad_arguments():
    from paper_1907_04587_amd import _lib as L
    lib = L.lib()
    assert lib.nsn_mlp_noalloc_scratch_bytes() >= lib.nsn_mlp_scratch_bytes(1 << 20)
    assert lib.nsn_mlp_loss_grad_noalloc(None, None, None, 10, None, None, None) == -1
    assert b"bad arguments" in lib.nsn_last_error()
