"""The allocation-free backward (rt_lookup_bwd_noalloc) through the C ABI:
the same bits as rt_lookup_bwd with a caller's workspace, call after call on
the library's one scratch array per GPU (a large call, then a smaller one,
then a planned one whose sort is skipped), and a clear refusal of a call whose
workspace would exceed the scratch."""
import ctypes
import math

import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def rt():
    from paper_2301_01719_amd import radtex
    return radtex


def _case(seed, W, H, n, C, N):
    g = torch.Generator().manual_seed(seed)
    tex = torch.rand((H, W, n, n, C), generator=g)
    uv = torch.rand((N, 2), generator=g, dtype=torch.float64) * 3 - 1
    z = torch.rand(N, generator=g, dtype=torch.float64) * 0.95 + 0.05
    phi = torch.rand(N, generator=g, dtype=torch.float64) * 2 * math.pi
    r = torch.sqrt(1 - z * z)
    view = torch.stack([r * torch.cos(phi), r * torch.sin(phi), z], 1)
    tbn = torch.eye(3, dtype=torch.float64).expand(N, 3, 3)
    go = torch.randn((N, C), generator=g)
    return (tex.to(DEV), uv.float().to(DEV), tbn.float().contiguous().to(DEV),
            view.float().to(DEV), go.to(DEV))


def _noalloc(rt, tex, uv, tbn, view, go, mode):
    N, C = uv.shape[0], tex.C
    gt = torch.full((tex.H, tex.W, tex.n, tex.n, C), float("nan"), device=DEV)
    gv = torch.full((N, 3), float("nan"), device=DEV)
    gu = torch.full((N, 2), float("nan"), device=DEV)
    fr = rt._frags(uv, tbn, view)
    st = rt.LIB.rt_lookup_bwd_noalloc(tex.handle, ctypes.byref(fr), rt._ptr(go), rt._ptr(gt),
                                      rt._ptr(gv), rt._ptr(gu), rt.MODES[mode],
                                      rt._stream(tex.device))
    assert st == 0, rt.LIB.rt_last_error()
    return gt, gv, gu


@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_noalloc_backward_is_the_workspace_backward(rt, mode):
    cases = [(64, 64, 16, 4, 400000), (16, 8, 8, 3, 30000)]  # the second smaller
    for k, (W, H, n, C, N) in enumerate(cases):
        tex_d, uv, tbn, view, go = _case(90 + k, W, H, n, C, N)
        tex = rt.Texture(tex_d, W, H, n, C)
        assert rt.bwd_workspace_bytes(tex, N, mode) <= rt.NOALLOC_SCRATCH_BYTES
        gt, gv, gu = _noalloc(rt, tex, uv, tbn, view, go, mode)
        rgt, rgv, rgu = rt.lookup_bwd(tex, uv, tbn, view, go, mode=mode)
        torch.cuda.synchronize()
        assert torch.equal(gt, rgt) and torch.equal(gv, rgv) and torch.equal(gu, rgu), (k, mode)
    # a planned G-buffer: the records come in key order and the sort is skipped
    order, puv, ptbn, pview = rt.plan_fragments(tex, uv, tbn, view, mode=mode)
    pgo = go[order.long()].contiguous()
    gt, gv, gu = _noalloc(rt, tex, puv, ptbn, pview, pgo, mode)
    rgt, rgv, rgu = rt.lookup_bwd(tex, puv, ptbn, pview, pgo, mode=mode)
    torch.cuda.synchronize()
    assert torch.equal(gt, rgt) and torch.equal(gv, rgv) and torch.equal(gu, rgu)


def test_noalloc_backward_refuses_more_than_its_scratch(rt):
    W, H, n, C = 64, 64, 8, 4
    N = 8_000_000  # nearest mode: about 48 bytes of workspace per fragment
    tex = rt.Texture(torch.rand((H, W, n, n, C), device=DEV), W, H, n, C)
    assert rt.bwd_workspace_bytes(tex, N) > rt.NOALLOC_SCRATCH_BYTES
    uv = torch.rand((N, 2), device=DEV)
    tbn = torch.eye(3, device=DEV).expand(N, 3, 3).contiguous()
    view = torch.tensor([0.3, 0.2, 0.9], device=DEV).expand(N, 3).contiguous()
    go = torch.zeros((N, C), device=DEV)
    gt = torch.zeros((H, W, n, n, C), device=DEV)
    fr = rt._frags(uv, tbn, view)
    st = rt.LIB.rt_lookup_bwd_noalloc(tex.handle, ctypes.byref(fr), rt._ptr(go), rt._ptr(gt),
                                      None, None, 0, rt._stream(tex.device))
    assert st == 4  # RT_ERR_WORKSPACE_TOO_SMALL, before anything is enqueued
    assert "scratch" in rt.LIB.rt_last_error().decode()
    torch.cuda.synchronize()
    assert torch.count_nonzero(gt) == 0
    # without the texel gradient no workspace is needed at any size
    gv = torch.empty((N, 3), device=DEV)
    st = rt.LIB.rt_lookup_bwd_noalloc(tex.handle, ctypes.byref(fr), rt._ptr(go), None,
                                      rt._ptr(gv), None, 0, rt._stream(tex.device))
    assert st == 0
    torch.cuda.synchronize()
