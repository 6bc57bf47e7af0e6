"""Differentiable fit of a radiance texture to multi-view target images (the
256x256-bucket, 8x8-sample RGB workload with 16 views of 512x512), through the
library's backward and torch's Adam, with a checkpoint/resume check that relies
on the bitwise determinism of the backward."""
import io

import pytest
import torch

from paper_2301_01719_amd import workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _setup():
    from paper_2301_01719_amd import radtex as rt
    w = wl.WORKLOADS["c4"]
    W, H, n, C = w.W, w.H, w.n, w.C
    gb = w.make_gbuffer(DEV)
    target_tex = wl.smooth_texture(W, H, n, C, seed=40, device=DEV)
    with torch.no_grad():
        target = rt.lookup_fwd(rt.Texture(target_tex, W, H, n, C), gb.uv, gb.tbn, gb.view)
    init = wl.smooth_texture(W, H, n, C, seed=41, device=DEV)
    return rt, w, gb, target, init


def _run(rt, w, gb, target, param, opt, steps, losses):
    n = w.n
    for _ in range(steps):
        opt.zero_grad(set_to_none=True)
        out = rt.lookup(param, gb.uv, gb.tbn, gb.view, n)
        loss = ((out - target) ** 2).mean()
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))


def _state_bytes(param, opt):
    buf = io.BytesIO()
    torch.save({"param": param.detach().clone(), "opt": opt.state_dict()}, buf)
    return buf.getvalue()


def test_fit_converges_and_resumes_bitwise():
    rt, w, gb, target, init = _setup()
    param = torch.nn.Parameter(init.clone())
    opt = torch.optim.Adam([param], lr=0.02)
    losses = []
    _run(rt, w, gb, target, param, opt, 50, losses)
    ckpt = _state_bytes(param, opt)
    _run(rt, w, gb, target, param, opt, 50, losses)
    final = param.detach().clone()
    torch.cuda.synchronize()
    print(f"loss: start {losses[0]:.4e}, step 50 {losses[49]:.4e}, end {losses[-1]:.4e}")
    assert losses[-1] <= 0.01 * losses[0], (losses[0], losses[-1])
    assert losses[99] < losses[50] < losses[10] < losses[0]
    ups = sum(b > a for a, b in zip(losses[10:], losses[11:]))
    assert ups <= 5, losses
    # resume from the step-50 checkpoint: the same 50 steps give the same bits
    st = torch.load(io.BytesIO(ckpt), weights_only=True)
    param2 = torch.nn.Parameter(st["param"].clone())
    opt2 = torch.optim.Adam([param2], lr=0.02)
    opt2.load_state_dict(st["opt"])
    losses2 = []
    _run(rt, w, gb, target, param2, opt2, 50, losses2)
    torch.cuda.synchronize()
    assert torch.equal(param2.detach(), final)
    assert losses2 == losses[50:]


def test_autograd_matches_direct_backward():
    """The autograd wrapper returns the library's backward for the texture,
    the view vectors and the texture coordinates, and nothing for the frame."""
    from paper_2301_01719_amd import radtex as rt
    W, H, n, C, N = 16, 16, 8, 3, 5000
    g = torch.Generator(device="cpu").manual_seed(3)
    tex = torch.rand((H, W, n, n, C), generator=g).to(DEV).requires_grad_(True)
    gbuf = wl.flat_gbuffer(N, seed=9, device=DEV)
    uv = gbuf.uv.clone().requires_grad_(True)
    view = gbuf.view.clone().requires_grad_(True)
    tbn = gbuf.tbn.clone().requires_grad_(True)
    go = torch.randn((N, C), generator=g).to(DEV)
    for mode in ("nearest", "bilinear"):
        out = rt.lookup(tex, uv, tbn, view, n, mode=mode)
        gt, gu, gv, gm = torch.autograd.grad(out, (tex, uv, view, tbn), go, allow_unused=True)
        d_gt, d_gv, d_gu = rt.lookup_bwd(rt.Texture(tex.detach(), W, H, n, C), uv.detach(),
                                         tbn.detach(), view.detach(), go, mode=mode)
        torch.cuda.synchronize()
        assert gm is None
        assert torch.equal(gt, d_gt) and torch.equal(gv, d_gv) and torch.equal(gu, d_gu)
        if mode == "nearest":
            assert torch.all(gu == 0)
