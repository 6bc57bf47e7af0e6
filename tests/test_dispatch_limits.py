"""Inputs larger than one dispatch can cover.

A dispatch holds fewer than 2^32 work-items, so the library splits or strides
the elementwise launches that would need more: the quantisers (BF16 and the
1-bit packer past 2^31 values, FP8 past 2^22 buckets, the 1-bit packer of
other n past 2^28 words), the atlas re-layout (2^32 texels and more) and the
zero fill of the level-of-detail backward (a level of 2^32 values), and the
backward's accumulation over groups of buckets (2^28 buckets).  Each test
takes a texture just past the limit, with a ragged end where the format
allows one, and checks the outputs at every cut, at both ends and on a random
sample: the quantisers against the oracle's quantiser on the sampled buckets
(a bucket's codes depend on that bucket's values alone), the re-layout
through lookups against torch's own permutation of the atlas, the backward
against the oracle's on the bucket window its fragments reach.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import EDGE, check_grad_tex, host
from paper_2301_01719_amd import workloads as wl

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

DEV = "cuda:0"


@pytest.fixture(scope="module")
def rt():
    from paper_2301_01719_amd import radtex
    return radtex


@pytest.fixture(autouse=True)
def _release():
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _around(cuts, end, seed, k=4, rand=2048):
    """Indices within k of every cut and of both ends, plus `rand` random ones."""
    idx = set(range(min(k, end))) | set(range(max(0, end - k), end))
    for c in cuts:
        idx.update(range(max(0, c - k), min(end, c + k)))
    idx.update(np.random.default_rng(seed).integers(0, end, rand).tolist())
    return np.array(sorted(idx), np.int64)


def _rows(t, idx):
    """Rows `idx` of a 2-D device tensor, on the host."""
    return host(t[torch.from_numpy(idx).to(DEV)])


def test_bf16_and_fp8_quantisers_past_one_dispatch(rt):
    """65535 x 10923 buckets of one RGB sample: 2,147,516,415 values (past
    2^31, and 3 past a multiple of 4, so the BF16 launch's ragged tail sits in
    its last chunk), 715.8M buckets (171 FP8 chunks of 2^22 buckets)."""
    W, H, n, C = 65535, 10923, 1, 3
    nb = W * H
    total = nb * C
    assert total > 2**31 and total % 4 == 3
    g = torch.Generator(device=DEV).manual_seed(7)
    t = torch.randn((H, W, n, n, C), generator=g, device=DEV)
    tex = rt.Texture(t, W, H, n, C)

    c16, _ = rt.quantize(tex, "bf16")
    torch.cuda.synchronize()
    idx = _around([2**31], total, seed=1, k=16)
    vals = _rows(t.view(-1, 1), idx)
    want, _ = oracle.quantize(vals, len(idx), 1, oracle.FMT_BF16)
    got = _rows(c16.view(-1, 1), idx).view(np.uint16).reshape(-1)
    np.testing.assert_array_equal(got, want)
    del c16

    c8, s8 = rt.quantize(tex, "fp8")
    torch.cuda.synchronize()
    cut = 1 << 22
    bidx = _around(range(cut, nb, cut), nb, seed=2, k=2)
    rows = _rows(t.view(nb, C), bidx)
    oc, osc = oracle.quantize(rows, len(bidx), C, oracle.FMT_FP8_E4M3)
    np.testing.assert_array_equal(_rows(c8.view(nb, C), bidx).reshape(-1), oc)
    np.testing.assert_array_equal(_rows(s8.view(nb, 1), bidx).reshape(-1), osc)


def test_fp8_vector_path_past_one_dispatch(rt):
    """2048 x 2049 buckets of 16 x 16 one-channel samples (whole float4 per
    lane): 2048 buckets past one launch of 2^22; every bucket at its own
    scale."""
    W, H, n, C = 2048, 2049, 16, 1
    nb = W * H
    assert nb > 1 << 22
    g = torch.Generator(device=DEV).manual_seed(11)
    t = torch.randn((H, W, n, n, C), generator=g, device=DEV)
    t *= torch.exp2(torch.randint(-30, 30, (H, W, 1, 1, 1), generator=g, device=DEV).float())
    tex = rt.Texture(t, W, H, n, C)
    c8, s8 = rt.quantize(tex, "fp8")
    torch.cuda.synchronize()
    per = n * n * C
    bidx = _around([1 << 22], nb, seed=3, k=4, rand=512)
    rows = _rows(t.view(nb, per), bidx)
    oc, osc = oracle.quantize(rows, len(bidx), per, oracle.FMT_FP8_E4M3)
    np.testing.assert_array_equal(_rows(c8.view(nb, per), bidx).reshape(-1), oc)
    np.testing.assert_array_equal(_rows(s8.view(nb, 1), bidx).reshape(-1), osc)


@pytest.mark.parametrize("W,H,n,cut", [
    (8192, 4097, 8, 1 << 25),    # n % 8 == 0, flat words: 2^31 samples a launch
    (65536, 4097, 3, 1 << 28),   # one word per bucket: 2^28 words a launch
])
def test_bit_packing_past_one_dispatch(rt, W, H, n, cut):
    nb = W * H
    assert nb > cut
    g = torch.Generator(device=DEV).manual_seed(n)
    t = torch.rand((H, W, n, n, 1), generator=g, device=DEV)
    tex = rt.Texture(t, W, H, n, 1)
    words, _ = rt.quantize(tex, "bit1")
    torch.cuda.synchronize()
    wpb = rt.bit_words(n)
    bidx = _around([cut], nb, seed=4, k=4, rand=1024)
    rows = _rows(t.view(nb, n * n), bidx)
    want = oracle.pack_bits(rows, n)
    got = _rows(words.view(nb, wpb), bidx).view(np.uint32).reshape(-1)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_atlas_relayout_past_one_dispatch(rt, mode):
    """A BF16 atlas of 32768 x 32769 buckets of 2 x 2 samples (4,295,098,368
    texels: the last bucket row lies past 2^32) looks up exactly as the
    bucket-major matrix torch makes from it by a permutation; half of the
    fragments land in the last bucket row."""
    W, H, n, C = 32768, 32769, 2, 1
    assert W * H * n * n > 2**32
    g = torch.Generator(device=DEV).manual_seed(5)
    atlas = torch.randn((H * n, W * n, C), generator=g, device=DEV, dtype=torch.bfloat16)
    bucket = atlas.view(H, n, W, n, C).permute(0, 2, 1, 3, 4).contiguous()
    tex_a = rt.Texture(atlas, W, H, n, C, "bf16", layout="atlas")
    tex_b = rt.Texture(bucket, W, H, n, C, "bf16")
    N = 1 << 16
    gb = wl.flat_gbuffer(N, 6, DEV)
    uv = gb.uv.clone()
    uv[: N // 2, 1] = (H - 1 + uv[: N // 2, 1]) / H
    out_a = rt.lookup_fwd(tex_a, uv, gb.tbn, gb.view, mode)
    out_b = rt.lookup_fwd(tex_b, uv, gb.tbn, gb.view, mode)
    torch.cuda.synchronize()
    assert torch.isfinite(out_b).all()
    assert torch.equal(out_a, out_b)
    tex_a.close()
    tex_b.close()


def test_lod_backward_without_fragments_fills_a_level_of_2_32_values(rt):
    """A chain whose level 0 is 2048 x 2048 buckets of 16 x 16 RGBA (2^32
    values): with no fragment the wanted levels are overwritten with zeros.
    The levels' texels are never read, so they share one buffer."""
    W = H = 2048
    n, C = 16, 4
    L = 12
    buf = torch.empty(W * H * n * n * C, device=DEV)
    chain = []
    for level in range(L):
        w, h = max(W >> level, 1), max(H >> level, 1)
        chain.append(rt.Texture(buf[: w * h * n * n * C].view(h, w, n, n, C), w, h, n, C))
    # leave ones in the memory the caching allocator hands to the gradients
    junk = torch.ones(W * H * n * n * C, device=DEV)
    del junk
    z = torch.empty((0, 1), device=DEV)
    want = [True] + [False] * (L - 2) + [True]
    grads, gv, gu = rt.lookup_lod_bwd(chain, z.new_empty((0, 2)), z.new_empty((0, 9)),
                                      z.new_empty((0, 3)), z.new_empty((0, 4)),
                                      z.new_empty((0, C)), "nearest", want_levels=want)
    torch.cuda.synchronize()
    assert grads[0].numel() == 2**32
    assert int(torch.count_nonzero(grads[0])) == 0
    assert int(torch.count_nonzero(grads[-1])) == 0
    assert all(g is None for g in grads[1:-1])
    for t in chain:
        t.close()


def test_backward_over_2_28_buckets(rt):
    """16384 x 16384 buckets of 2 x 2 one-channel samples: the accumulation's
    groups of 4 buckets would need 2^32 work-items in one dispatch.  The
    fragments fall in the last 64 x 64 buckets (the last groups); the dense
    gradient there matches the oracle's, and every other element of a
    gradient buffer filled with ones beforehand is overwritten with zero."""
    W = H = 16384
    n, C = 2, 1
    N = 1 << 16
    b0 = W - 64
    gb = wl.flat_gbuffer(N, 12, DEV)
    uv = ((b0 + 0.5 + 63 * gb.uv) / W).contiguous()
    g = torch.Generator(device=DEV).manual_seed(13)
    texels = torch.rand((H, W, n, n, C), generator=g, device=DEV)
    tex = rt.Texture(texels, W, H, n, C)
    go = torch.randn((N, C), generator=g, device=DEV)
    uvh, tbnh, viewh = host(uv), host(gb.tbn), host(gb.view)
    _, _, edge = oracle.indices(uvh, tbnh, viewh, W, H, n)
    near = ~((edge[:, 0] >= EDGE) & (edge[:, 1] >= EDGE))
    go[torch.from_numpy(np.nonzero(near)[0]).to(DEV)] = 0.0
    gt = torch.ones((H, W, n, n, C), device=DEV)
    gt, _, _ = rt.lookup_bwd(tex, uv, gb.tbn, gb.view, go, "nearest", want_view=False,
                             want_uv=False, grad_tex=gt)
    torch.cuda.synchronize()
    win = host(gt[b0:, b0:])
    ref = oracle.lookup_bwd(oracle.Tex(np.zeros(W * H * n * n * C, np.float32), W, H, n, C),
                            uvh, tbnh, viewh, host(go), oracle.MODE_NEAREST,
                            window=(b0, b0, 64, 64), want_view=False, want_uv=False)
    check_grad_tex(win, ref, n)
    assert int(torch.count_nonzero(gt)) == int(np.count_nonzero(win))
    tex.close()


def test_backward_sort_past_2_27_records(rt):
    """A bilinear backward of 35.65M fragments (142.6M records) over 1024 x
    1024 buckets of 8 x 8 RGB.  Its 26-bit keys sort in passes of 9, 9 and 8
    bits; the 9-bit passes' histograms hold 512 x 34.8k counts, more block sums
    (4352) than a down-sweep workgroup adds up itself, so their scan takes the
    one-block pass over the sums, and the 8-bit pass (2176 sums) does not.  The
    dense gradient on a 32 x 32 bucket window matches the oracle's (from the
    fragments within one bucket of the window), and the whole gradient sums to
    the upstream gradient's sum (a fragment's bilinear weights sum to 1)."""
    from helpers import away_from_edges
    W = H = 1024
    n, C = 8, 3
    N = 34 * 1024 * 1024
    assert 4 * N > 2**27
    gb = wl.flat_gbuffer(N, 21, DEV)
    g = torch.Generator(device=DEV).manual_seed(22)
    texels = torch.rand((H, W, n, n, C), generator=g, device=DEV)
    tex = rt.Texture(texels, W, H, n, C)
    go = torch.randn((N, C), generator=g, device=DEV)
    bi0, bj0, bw, bh = win = (500, 700, 32, 32)
    idx, _ = rt.debug_indices(tex, gb.uv, gb.tbn, gb.view)
    m = ((idx[:, 0] >= bi0 - 1) & (idx[:, 0] <= bi0 + bw) & (idx[:, 1] >= bj0 - 1)
         & (idx[:, 1] <= bj0 + bh))
    near = torch.nonzero(m).flatten()
    del idx, m
    uvw, tbnw, vw = host(gb.uv[near]), host(gb.tbn[near]), host(gb.view[near])
    keep = away_from_edges(uvw, tbnw, vw, W, H, n, "bilinear")
    go[near[torch.from_numpy(~keep).to(DEV)]] = 0.0
    gt, _, _ = rt.lookup_bwd(tex, gb.uv, gb.tbn, gb.view, go, "bilinear", want_view=False,
                             want_uv=False)
    torch.cuda.synchronize()
    ref = oracle.lookup_bwd(oracle.Tex(host(texels), W, H, n, C), uvw, tbnw, vw,
                            host(go[near]), oracle.MODE_BILINEAR, window=win,
                            want_view=False, want_uv=False)
    assert np.count_nonzero(ref["absg_tex"]) > 1000
    check_grad_tex(host(gt[bj0:bj0 + bh, bi0:bi0 + bw]), ref, n)
    mass = float(torch.sum(gt, dtype=torch.float64))
    want = float(torch.sum(go, dim=0, dtype=torch.float64).sum())
    scale = float(torch.sum(go.abs(), dtype=torch.float64))
    assert abs(mass - want) <= 1e-5 * scale, (mass, want, scale)
    tex.close()


def _mip_windows(W2, H2, w=16):
    """Aligned windows (j0, i0) of w x w buckets of the next level: both
    corners, the middle, and the last buckets."""
    return [(0, 0), (0, W2 - w), (H2 - w, 0), (H2 // 2, W2 // 2), (H2 - w, W2 - w)]


def test_mip_level_past_one_dispatch(rt):
    """16384 x 16384 buckets of one RGBA sample (4 GiB) to the 8192 x 8192
    level: one workgroup of 64 threads per bucket of the next level would be
    2^32 work-items; the capped grid strides.  Windows of the level against the
    oracle's level of the same source window (the mean of a bucket's 2 x 2
    sources depends on those alone)."""
    W = H = 16384
    n, C = 1, 4
    g = torch.Generator(device=DEV).manual_seed(5)
    src = torch.rand((H, W, n, n, C), generator=g, device=DEV)
    tex = rt.Texture(src, W, H, n, C)
    dst = rt.build_mip(tex)
    torch.cuda.synchronize()
    w = 16
    for j0, i0 in _mip_windows(W // 2, H // 2, w):
        s = host(src[2 * j0:2 * j0 + 2 * w, 2 * i0:2 * i0 + 2 * w]).copy()
        want = oracle.build_mips(s, 2 * w, 2 * w, n, C, 2)[1]
        got = host(dst[j0:j0 + w, i0:i0 + w]).astype(np.float64)
        assert np.max(np.abs(got - want)) <= 2.0 ** -22, (j0, i0)
    tex.close()


def test_mip_adjoint_past_one_dispatch(rt):
    """The adjoint of the 4096 x 4096 -> 2048 x 2048 step with one RGBA sample
    per bucket: one 256-thread workgroup per source bucket would be 2^32
    work-items; the capped grid strides.  Windows against the oracle's adjoint
    of the same parent window (each bucket adds its own parent's share)."""
    W = H = 4096
    n, C = 1, 4
    g = torch.Generator(device=DEV).manual_seed(6)
    tex = rt.Texture(torch.zeros((H, W, n, n, C), device=DEV), W, H, n, C)
    gd = torch.randn((H // 2, W // 2, n, n, C), generator=g, device=DEV)
    gs0 = torch.randn((H, W, n, n, C), generator=g, device=DEV)
    gs = rt.build_mip_adjoint(tex, gd, gs0.clone())
    torch.cuda.synchronize()
    w = 16
    for j0, i0 in _mip_windows(W // 2, H // 2, w):
        parent = host(gd[j0:j0 + w, i0:i0 + w]).astype(np.float64)
        base = host(gs0[2 * j0:2 * j0 + 2 * w, 2 * i0:2 * i0 + 2 * w]).astype(np.float64).copy()
        want = oracle.build_mip_adjoint(parent, 2 * w, 2 * w, n, C, grad_src=base)
        got = host(gs[2 * j0:2 * j0 + 2 * w, 2 * i0:2 * i0 + 2 * w]).astype(np.float64)
        # one product by 1/4 (exact) and one binary32 addition per element
        assert np.all(np.abs(got - want) <= 2.0 ** -24 * np.abs(want) + 1e-30), (j0, i0)
    tex.close()
