"""lbm_mlp_backward_static, the backward pass that allocates nothing (its
block partials live in a fixed device array of the library), against
lbm_mlp_backward with a caller workspace: the same kernels in the same fixed
order, so gradient and loss agree bit for bit, on two calls in a row (the
second with a smaller batch, which reads fewer partials than the first left
behind).  A batch above the array's capacity is rejected with LBM_ERANGE."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _inputs(rng, B):
    import torch

    x = np.zeros((B, 32), dtype=np.float16)
    x[:, :27] = rng.uniform(-1.0, 1.0, (B, 27))
    t = rng.standard_normal((B, 4)).astype(np.float32)
    return (torch.tensor(x.view(np.int16), device="cuda"), torch.tensor(t, device="cuda"))


def test_static_backward_matches_workspace_backward():
    import torch

    from paper_2505_01126_amd import lbm

    L = lbm.load_library()
    rng = np.random.default_rng(11)
    w = torch.tensor((rng.standard_normal(lbm.MLP_NPARAM) * 0.2).astype(np.float16).view(np.int16), device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda a: C.c_void_p(a.data_ptr())
    for B in (lbm.MLP_STATIC_MAX_BATCH, 1234):  # the second call reads fewer block partials than the first wrote
        print(f"case static backward B={B}", flush=True)
        x, t = _inputs(rng, B)
        g_ref = torch.zeros(lbm.MLP_NPARAM, dtype=torch.float32, device="cuda")
        l_ref = torch.zeros(1, dtype=torch.float32, device="cuda")
        work = torch.empty(lbm.lbm_mlp_work_bytes(B), dtype=torch.uint8, device="cuda")
        lbm.lbm_mlp_backward(p(w), p(x), p(t), B, p(g_ref), p(l_ref), p(work), work.numel(), stream)
        g = torch.full((lbm.MLP_NPARAM,), float("nan"), dtype=torch.float32, device="cuda")
        l = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        lbm.lbm_mlp_backward_static(p(w), p(x), p(t), B, p(g), p(l), stream)
        torch.cuda.synchronize()
        assert torch.isfinite(g_ref).all() and float(l_ref) > 0.0
        assert torch.equal(g, g_ref), f"B={B}: gradients differ"
        assert torch.equal(l, l_ref), f"B={B}: losses differ"
    # above the fixed capacity: rejected before anything runs
    rc = L.lbm_mlp_backward_static(p(w), p(x), p(t), lbm.MLP_STATIC_MAX_BATCH + 1, p(g), p(l), stream)
    assert rc == lbm.LBM_ERANGE
    assert L.lbm_mlp_backward_static(p(w), p(x), p(t), -1, p(g), p(l), stream) == lbm.LBM_EINVAL
