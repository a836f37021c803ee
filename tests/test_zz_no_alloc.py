"""The no-allocation projection dl_tsk_project_noalloc (GPU): through the C ABI it gives the same
c = V^H w and w - V c as dl_tsk_project, bit for bit, on two calls in a row (the second smaller,
so stale partials from the first would show), maps no device memory, and rejects sizes beyond its
fixed scratch array."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _fields(n, nv, seed):
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    V = torch.randn(nv, n, dtype=torch.complex128, device="cuda", generator=g)
    w = torch.randn(n, dtype=torch.complex128, device="cuda", generator=g)
    return V, w


@pytest.mark.parametrize("subtract", [False, True])
def test_noalloc_projection_equals_allocating_entry_point(gpu_ctx, subtract):
    import torch
    from paper_0901_3163_amd import deflan
    # 16^3 x 32 spinor length with 60 vectors, then a ragged length and 7 vectors
    for n, nv, seed in ((1572864, 60, 1), (3 * 5 * 2 * 4 * 12 + 0, 7, 2)):
        V, w = _fields(n, nv, seed)
        c_ref, w_ref = deflan.dl_tsk_project(gpu_ctx, V, w, subtract=subtract)
        torch.cuda.synchronize()
        c = torch.full((nv,), float("nan"), dtype=torch.complex128, device="cuda")
        w2 = w.clone()
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        deflan.dl_tsk_project_noalloc(gpu_ctx, V, w2, c, subtract=subtract)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0  # no device memory mapped by the call
        assert torch.equal(c, c_ref), (n, nv)
        assert torch.equal(w2, w_ref if subtract else w), (n, nv)
        # against a plain contraction of the same fields (FP64, ordering differs)
        c_np = V.conj().cpu().numpy() @ w.cpu().numpy()
        assert np.max(np.abs(c.cpu().numpy() - c_np)) <= 1e-12 * np.sqrt(n) * np.abs(c_np).max()


def test_noalloc_rejects_sizes_beyond_its_scratch(gpu_ctx):
    import torch
    from paper_0901_3163_amd import deflan
    n, nv = 2048 * 2048, 300  # 2 * 300 * 2048 partials > 2^20
    V = torch.zeros(nv, 16, dtype=torch.complex128, device="cuda")  # only the sizes are read
    w = torch.zeros(16, dtype=torch.complex128, device="cuda")
    c = torch.zeros(nv, dtype=torch.complex128, device="cuda")
    import ctypes as C
    rc = deflan.lib.dl_tsk_project_noalloc(gpu_ctx.h, n, nv, C.c_void_p(V.data_ptr()), C.c_void_p(w.data_ptr()),
                                           C.c_void_p(c.data_ptr()), 0)
    assert rc == deflan.DL_E_INVALID
    assert b"scratch" in deflan.lib.dl_last_error()
