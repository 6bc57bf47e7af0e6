"""Flat launches on a texture of at least 1 GiB stage each wavefront's frames
and view vectors through LDS (16-byte loads when the arrays are 16-byte
aligned there, 4-byte loads otherwise); tiled launches and smaller textures
read per lane.  All of these give the same bits: the lookup's output, the
view and uv gradients and the texel gradient of a flat launch equal those of
the same fragments visited in pixel tiles, with the arrays aligned or not and
a last wavefront that is partly empty."""
import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def rt():
    from paper_2301_01719_amd import radtex
    return radtex


@pytest.fixture(scope="module")
def big_texture(rt):
    # 512 x 512 buckets of 16 x 16 RGBA in FP32: 2^30 bytes, the staging threshold
    W = H = 512
    n, C = 16, 4
    g = torch.Generator(device=DEV).manual_seed(5)
    data = torch.rand((H, W, n, n, C), generator=g, device=DEV)
    return rt.Texture(data, W, H, n, C), data


def _fragments(height, width, seed, shift=0):
    """An image of height x width fragments over a patch of the texture; with
    shift > 0 the frame and view arrays start `shift` floats into their
    allocations (4-byte aligned only)."""
    N = height * width
    g = torch.Generator().manual_seed(seed)
    yy, xx = torch.meshgrid(torch.arange(height, dtype=torch.float32),
                            torch.arange(width, dtype=torch.float32), indexing="ij")
    uv = torch.stack([0.1 + 0.5 * xx / width, 0.2 + 0.5 * yy / height], -1).reshape(N, 2)
    view = torch.rand((N, 3), generator=g) * 2 - 1
    view[:, 2] = view[:, 2].abs() + 0.2
    q, _ = torch.linalg.qr(torch.randn((N, 3, 3), generator=g))
    tbn = q.transpose(1, 2).contiguous()
    tb = torch.zeros(N * 9 + shift).to(DEV)
    vb = torch.zeros(N * 3 + shift).to(DEV)
    tb[shift:] = tbn.reshape(-1).to(DEV)
    vb[shift:] = view.reshape(-1).to(DEV)
    return (uv.to(DEV), tb[shift:].view(N, 3, 3), vb[shift:].view(N, 3))


@pytest.mark.parametrize("shift", [0, 1])
@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_staged_frames_give_the_same_bits(rt, big_texture, shift, mode):
    tex, _ = big_texture
    height, width = 301, 517  # 155,617 fragments: the last wavefront is partly empty
    uv, tbn, view = _fragments(height, width, 9, shift)
    if shift:
        assert tbn.data_ptr() % 16 != 0 and view.data_ptr() % 16 != 0
    image = (1, height, width)
    N = height * width
    go = torch.randn((N, 4), generator=torch.Generator().manual_seed(10)).to(DEV)
    flat = rt.lookup_fwd(tex, uv, tbn, view, mode=mode)
    tiled = rt.lookup_fwd(tex, uv, tbn, view, mode=mode, image=image)
    fgt, fgv, fgu = rt.lookup_bwd(tex, uv, tbn, view, go, mode=mode)
    tgt, tgv, tgu = rt.lookup_bwd(tex, uv, tbn, view, go, mode=mode, image=image)
    torch.cuda.synchronize()
    assert torch.equal(flat, tiled)
    assert torch.equal(fgv, tgv) and torch.equal(fgu, tgu)
    assert torch.equal(fgt, tgt)
