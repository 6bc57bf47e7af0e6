"""The forward with bucket tiles staged in LDS (RT_FWD_STAGE_BUCKETS): the
same bits as the plain forward, in screen order, flat and planned, for every
storage format it takes; the cases it does not take are refused before
anything is enqueued."""
import math

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def rt():
    from paper_2301_01719_amd import radtex
    return radtex


def _case(seed, W, H, n, C, views, height, width):
    g = torch.Generator().manual_seed(seed)
    N = views * height * width
    tex = torch.rand((H, W, n, n, C), generator=g)
    # screen-like UV: each image a smooth patch of the texture, so that
    # neighbouring fragments share buckets as on a rendered view
    yy, xx = torch.meshgrid(torch.arange(height, dtype=torch.float64),
                            torch.arange(width, dtype=torch.float64), indexing="ij")
    uvs = []
    for v in range(views):
        s = 0.3 + 0.4 * torch.rand(1, generator=g, dtype=torch.float64)
        o = torch.rand(2, generator=g, dtype=torch.float64)
        uvs.append(torch.stack([o[0] + s * xx / width, o[1] + s * yy / height], -1).reshape(-1, 2))
    uv = torch.cat(uvs).float()
    z = torch.rand(N, generator=g, dtype=torch.float64) * 0.9 + 0.1
    phi = torch.rand(N, generator=g, dtype=torch.float64) * 2 * math.pi
    r = torch.sqrt(1 - z * z)
    view = torch.stack([r * torch.cos(phi), r * torch.sin(phi), z], 1).float()
    tbn = torch.eye(3).expand(N, 3, 3).contiguous()
    return tex.to(DEV), uv.to(DEV), tbn.to(DEV), view.to(DEV)


@pytest.mark.parametrize("fmt,n,C", [("f32", 8, 4), ("f32", 16, 4), ("f32", 4, 1),
                                     ("bf16", 16, 4), ("bf16", 8, 3), ("fp8", 16, 4),
                                     ("fp8", 4, 1), ("fp8", 8, 2)])
def test_staged_forward_is_the_plain_forward(rt, fmt, n, C):
    W, H, views, height, width = 40, 24, 3, 96, 160
    tex_d, uv, tbn, view = _case(n * 10 + C, W, H, n, C, views, height, width)
    master = rt.Texture(tex_d, W, H, n, C)
    tex = master
    if fmt != "f32":
        codes, scales = rt.quantize(master, fmt)
        tex = rt.Texture(codes, W, H, n, C, fmt, scales)
    image = (views, height, width)
    plain = rt.lookup_fwd(tex, uv, tbn, view, image=image)
    staged = rt.lookup_fwd(tex, uv, tbn, view, image=image, stage_buckets=True)
    flat = rt.lookup_fwd(tex, uv, tbn, view, stage_buckets=True)
    order, puv, ptbn, pview = rt.plan_fragments(master, uv, tbn, view, image=image)
    planned = rt.lookup_fwd(tex, puv, ptbn, pview, stage_buckets=True)
    torch.cuda.synchronize()
    assert torch.equal(staged, plain)
    assert torch.equal(flat, plain)
    assert torch.equal(planned, plain[order.long()])


def test_staged_forward_of_a_ragged_launch(rt):
    """A count that fills no whole workgroup or wavefront."""
    W, H, n, C = 7, 5, 8, 4
    tex_d, uv, tbn, view = _case(3, W, H, n, C, 1, 1, 77)
    tex = rt.Texture(tex_d, W, H, n, C)
    plain = rt.lookup_fwd(tex, uv, tbn, view)
    staged = rt.lookup_fwd(tex, uv, tbn, view, stage_buckets=True)
    torch.cuda.synchronize()
    assert torch.equal(staged, plain)


def test_staged_forward_refuses_what_it_cannot_stage(rt):
    N = 64
    uv = torch.rand((N, 2), device=DEV)
    tbn = torch.eye(3, device=DEV).expand(N, 3, 3).contiguous()
    view = torch.tensor([[0.1, 0.2, 0.9]], device=DEV).expand(N, 3).contiguous()

    def refused(tex, mode="nearest"):
        with pytest.raises(RuntimeError, match="RT_FWD_STAGE_BUCKETS"):
            rt.lookup_fwd(tex, uv, tbn, view, mode=mode, stage_buckets=True)

    refused(rt.Texture(torch.rand((4, 4, 8, 8, 4), device=DEV), 4, 4, 8, 4), mode="bilinear")
    # 32 x 32 x 4 x 4 bytes = 16 KiB is the largest bucket; 64 x 64 x 4 x 4 is not taken
    rt.lookup_fwd(rt.Texture(torch.rand((2, 2, 32, 32, 4), device=DEV), 2, 2, 32, 4), uv, tbn,
                  view, stage_buckets=True)
    refused(rt.Texture(torch.rand((2, 2, 64, 64, 4), device=DEV), 2, 2, 64, 4))
    # 3 x 3 x 1 bytes of FP8 is not a multiple of 16
    t31 = rt.Texture(torch.rand((2, 2, 3, 3, 1), device=DEV), 2, 2, 3, 1)
    c, s = rt.quantize(t31, "fp8")
    refused(rt.Texture(c, 2, 2, 3, 1, "fp8", s))
    # dictionaries
    cb = torch.rand((3, 8, 8, 4), device=DEV)
    refused(rt.DictionaryTexture(cb, torch.zeros((2, 2), dtype=torch.uint8, device=DEV), 2, 2,
                                 8, 4))
    # one-bit textures
    t1 = rt.Texture(torch.rand((2, 2, 8, 8, 1), device=DEV), 2, 2, 8, 1)
    words, _ = rt.quantize(t1, "bit1")
    refused(rt.Texture(words, 2, 2, 8, 1, "bit1"))
    torch.cuda.synchronize()
