"""The visit plan (rt_plan_fragments) through the C ABI.

A plan orders a G-buffer by the backward's record key (bucket, then the cell
of the bilinear footprint, ties in fragment order).  What must hold:

* the order is a permutation and the planned G-buffer is the input gathered
  by it; the planned fragments' keys (from the library's own indices) are in
  order, ties in increasing input index;
* a lookup of the planned G-buffer gives, at position k, the bits the lookup
  of the input gives for fragment order[k] (any storage format, both bucket
  modes, the input visited flat or in pixel tiles);
* the backward of the planned G-buffer with the upstream gradient permuted
  the same way gives the same texel gradient bit for bit (its records come
  in key order, so its sort does nothing) and the view and uv gradients of
  fragment order[k] at position k;
* a G-buffer that is almost in plan order (one pair swapped) is still sorted
  and gives the same bits; planning a planned G-buffer returns the identity.
"""
import math

import numpy as np
import pytest
import torch

from paper_2301_01719_amd import workloads as wl

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
    vt = torch.stack([r * torch.cos(phi), r * torch.sin(phi), z], 1)
    q, _ = torch.linalg.qr(torch.randn((N, 3, 3), generator=g, dtype=torch.float64))
    tbn = q.transpose(1, 2).contiguous()
    view = torch.einsum("nkm,nk->nm", tbn, vt)
    return (tex.to(DEV), uv.float().to(DEV), tbn.float().contiguous().to(DEV),
            view.float().contiguous().to(DEV))


def _keys(rt, tex, uv, tbn, view, W, n, mode):
    """The record key of each fragment from the library's indices: bucket
    (nearest, or the first of the bilinear footprint) and the footprint's cell
    (x0 kept at or below n - 2)."""
    idx, _ = rt.debug_indices(tex, uv, tbn, view)
    idx = idx.cpu().numpy().astype(np.int64)
    x0 = np.minimum(idx[:, 2], max(n - 2, 0))
    y0 = np.minimum(idx[:, 3], max(n - 2, 0))
    if mode == "nearest":
        i, j = idx[:, 0], idx[:, 1]
    else:
        u = uv.cpu().numpy().astype(np.float64)
        H = tex.H
        t = u * [W, H]
        p = t - np.floor(t)
        k = np.floor(t).astype(np.int64) - (p < 0.5)
        i, j = k[:, 0] % W, k[:, 1] % H
    return (j * W + i) * (n * n) + y0 * n + x0


@pytest.mark.parametrize("W,H,n,C,N,mode", [(16, 16, 8, 4, 50000, "nearest"),
                                            (16, 16, 8, 4, 50000, "bilinear"),
                                            (5, 3, 3, 1, 777, "nearest"),
                                            (64, 64, 16, 3, 100001, "nearest"),
                                            (2, 2, 2, 2, 1, "nearest")])
def test_plan_is_a_sorting_permutation(rt, W, H, n, C, N, mode):
    tex_d, uv, tbn, view = _case(W + N, W, H, n, C, N)
    tex = rt.Texture(tex_d, W, H, n, C)
    order, puv, ptbn, pview = rt.plan_fragments(tex, uv, tbn, view, mode=mode)
    torch.cuda.synchronize()
    o = order.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(o), np.arange(N))
    ot = order.long()
    assert torch.equal(puv, uv[ot]) and torch.equal(ptbn, tbn[ot]) and torch.equal(pview, view[ot])
    k = _keys(rt, tex, uv, tbn, view, W, n, mode)
    ko = k[o]
    assert np.all(np.diff(ko) >= 0)
    same = np.diff(ko) == 0
    assert np.all(np.diff(o)[same] > 0)  # ties keep the input order
    # planning a planned G-buffer changes nothing
    o2, u2, t2, v2 = rt.plan_fragments(tex, puv, ptbn, pview, mode=mode)
    torch.cuda.synchronize()
    assert torch.equal(o2.long(), torch.arange(N, device=DEV))
    assert torch.equal(u2, puv) and torch.equal(t2, ptbn) and torch.equal(v2, pview)


def test_plan_of_no_fragments(rt):
    tex = rt.Texture(torch.rand((2, 2, 4, 4, 4), device=DEV), 2, 2, 4, 4)
    e = torch.empty((0, 2), device=DEV)
    order, puv, ptbn, pview = rt.plan_fragments(tex, e, torch.empty((0, 3, 3), device=DEV),
                                                torch.empty((0, 3), device=DEV))
    assert order.numel() == 0 and puv.shape == (0, 2)


@pytest.mark.parametrize("fmt", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_planned_lookups_are_the_permuted_lookups(rt, fmt, mode):
    w = wl.WORKLOADS["c4"]
    W, H, n, C = w.W, w.H, w.n, w.C
    tex32 = w.make_texture(DEV)
    gb = w.make_gbuffer(DEV)
    N = gb.count
    master = rt.Texture(tex32, W, H, n, C)
    tex = master
    if fmt != "f32":
        codes, scales = rt.quantize(master, fmt)
        tex = rt.Texture(codes, W, H, n, C, fmt, scales)
    order, puv, ptbn, pview = rt.plan_fragments(tex, gb.uv, gb.tbn, gb.view, mode=mode,
                                                image=gb.image)
    ot = order.long()
    out = rt.lookup_fwd(tex, gb.uv, gb.tbn, gb.view, mode=mode, image=gb.image)
    pout = rt.lookup_fwd(tex, puv, ptbn, pview, mode=mode)
    torch.cuda.synchronize()
    assert torch.equal(pout, out[ot])
    go = wl.grad_out(N, C, seed=w.seed, device=DEV)
    gt, gv, gu = rt.lookup_bwd(tex, gb.uv, gb.tbn, gb.view, go, mode=mode, image=gb.image)
    pgt, pgv, pgu = rt.lookup_bwd(tex, puv, ptbn, pview, go[ot].contiguous(), mode=mode)
    torch.cuda.synchronize()
    _same_texel_gradient(pgt, gt, mode)
    assert torch.equal(pgv, gv[ot]) and torch.equal(pgu, gu[ot])


def _same_texel_gradient(a, b, mode):
    """Nearest mode: the same bits (the records of a key come in input order
    either way).  Bilinear-bucket mode: a fragment's four records are keyed by
    four buckets while the plan orders by the first, so records of one key can
    come in another order and the sums differ by rounding only."""
    if mode == "nearest":
        assert torch.equal(a, b)
    else:
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-6 * float(b.abs().max()))


@pytest.mark.parametrize("N", [1, 2, 3, 5, 1023, 1025])
@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_backward_of_a_few_fragments_planned_and_not(rt, N, mode):
    """A handful of records, in input order and in plan order: the order
    check writes the bucket ranges when the records come in key order (one
    record included), the sort and the range pass otherwise.  A range left
    unwritten would drop records, so the texel gradient must carry the
    upstream gradient's whole mass (each fragment's tap weights sum to one,
    Eq. (5)) both ways, and the two ways agree."""
    W, H, n, C = 6, 5, 8, 4
    tex_d, uv, tbn, view = _case(100 + N, W, H, n, C, N)
    tex = rt.Texture(tex_d, W, H, n, C)
    go = (torch.rand((N, C), generator=torch.Generator().manual_seed(N)) + 0.5).to(DEV)
    gt, gv, gu = rt.lookup_bwd(tex, uv, tbn, view, go, mode=mode)
    order, puv, ptbn, pview = rt.plan_fragments(tex, uv, tbn, view, mode=mode)
    ot = order.long()
    pgt, pgv, pgu = rt.lookup_bwd(tex, puv, ptbn, pview, go[ot].contiguous(), mode=mode)
    torch.cuda.synchronize()
    want = go.double().sum(0).cpu().numpy()
    for g in (gt, pgt):
        t = g.double().reshape(-1, C).sum(0).cpu().numpy()
        np.testing.assert_allclose(t, want, rtol=1e-5)
    _same_texel_gradient(pgt, gt, mode)
    assert torch.equal(pgv, gv[ot]) and torch.equal(pgu, gu[ot])


@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_nearly_planned_fragments_are_still_sorted(rt, mode):
    """One swapped pair breaks the key order: the backward's sort runs and
    the gradients are still the plain ones."""
    W, H, n, C, N = 32, 32, 8, 4, 200000
    tex_d, uv, tbn, view = _case(7, W, H, n, C, N)
    tex = rt.Texture(tex_d, W, H, n, C)
    order, puv, ptbn, pview = rt.plan_fragments(tex, uv, tbn, view, mode=mode)
    go = torch.randn((N, C), generator=torch.Generator().manual_seed(8)).to(DEV)
    gt, gv, gu = rt.lookup_bwd(tex, uv, tbn, view, go, mode=mode)
    k = _keys(rt, tex, puv, ptbn, pview, W, n, mode)
    steps = np.nonzero(np.diff(k) > 0)[0]
    a = int(steps[len(steps) // 3])  # positions a, a + 1 hold different keys
    perm = torch.arange(N, device=DEV)
    perm[a], perm[a + 1] = a + 1, a
    suv, stbn, sview = puv[perm].contiguous(), ptbn[perm].contiguous(), pview[perm].contiguous()
    ot = order.long()[perm]
    sgt, sgv, sgu = rt.lookup_bwd(tex, suv, stbn, sview, go[ot].contiguous(), mode=mode)
    torch.cuda.synchronize()
    _same_texel_gradient(sgt, gt, mode)
    assert torch.equal(sgv, gv[ot]) and torch.equal(sgu, gu[ot])


@pytest.mark.parametrize("where", ["first", "last"])
def test_a_descent_past_one_flag_block_is_found(rt, where):
    """Over 4096 workgroups of 1024 keys the order check's flags are ORed by
    more than one workgroup: one swapped pair in the first or in the last of
    them still sends the backward through its sort (a missed descent would
    split the runs of a key and change the texel gradient)."""
    W, H, n, C, N = 64, 64, 8, 1, 4_400_000  # 4297 flags
    g = torch.Generator().manual_seed(11)
    tex = rt.Texture(torch.rand((H, W, n, n, C), generator=g).to(DEV), W, H, n, C)
    uv = torch.rand((N, 2), generator=g).to(DEV)
    vt = torch.rand((N, 3), generator=g) * 2 - 1
    vt[:, 2] = vt[:, 2].abs() + 0.1
    view = vt.to(DEV)
    tbn = torch.eye(3, device=DEV).expand(N, 3, 3).contiguous()
    order, puv, ptbn, pview = rt.plan_fragments(tex, uv, tbn, view)
    go = torch.randn((N, C), generator=torch.Generator().manual_seed(12)).to(DEV)
    gt, _, _ = rt.lookup_bwd(tex, uv, tbn, view, go, want_view=False, want_uv=False)
    k = _keys(rt, tex, puv, ptbn, pview, W, n, "nearest")
    steps = np.nonzero(np.diff(k) > 0)[0]
    a = int(steps[0] if where == "first" else steps[-1])
    assert (a // 1024 < 4096) == (where == "first")
    perm = torch.arange(N, device=DEV)
    perm[a], perm[a + 1] = a + 1, a
    suv, stbn, sview = puv[perm].contiguous(), ptbn[perm].contiguous(), pview[perm].contiguous()
    ot = order.long()[perm]
    sgt, _, _ = rt.lookup_bwd(tex, suv, stbn, sview, go[ot].contiguous(), want_view=False,
                              want_uv=False)
    torch.cuda.synchronize()
    assert torch.equal(sgt, gt)


def test_plan_validation(rt):
    import ctypes
    tex = rt.Texture(torch.rand((4, 4, 8, 8, 4), device=DEV), 4, 4, 8, 4)
    N = 100
    uv = torch.rand((N, 2), device=DEV)
    tbn = torch.eye(3, device=DEV).expand(N, 3, 3).contiguous()
    view = torch.rand((N, 3), device=DEV)
    fr = rt._frags(uv, tbn, view)
    ws_bytes = rt.plan_workspace_bytes(tex, N)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=DEV)
    o = torch.empty(N, dtype=torch.int32, device=DEV)
    pu, pt, pv = torch.empty_like(uv), torch.empty_like(tbn), torch.empty_like(view)
    call = lambda *a: rt.LIB.rt_plan_fragments(tex.handle, ctypes.byref(fr), *a)
    P = rt._ptr
    assert call(0, None, P(pu), P(pt), P(pv), P(ws), ws_bytes, None) == 1
    assert call(0, P(o), P(uv), P(pt), P(pv), P(ws), ws_bytes, None) == 1  # overlaps the input
    assert "overlap" in rt.LIB.rt_last_error().decode()
    assert call(0, P(o), P(pu), P(pu), P(pv), P(ws), ws_bytes, None) == 1  # overlaps an output
    assert call(0, P(o), P(pu), P(pt), P(pv), P(ws), ws_bytes - 1, None) == 4
    assert call(7, P(o), P(pu), P(pt), P(pv), P(ws), ws_bytes, None) == 1
    assert call(0, P(o), P(pu), P(pt), P(pv), P(ws), ws_bytes, None) == 0
    torch.cuda.synchronize()


@pytest.mark.parametrize("cols,dtype", [(4, torch.float32), (3, torch.float32), (2, torch.float32),
                                        (9, torch.float32), (1, torch.int32)])
def test_plan_permute_gathers_and_scatters_rows(rt, cols, dtype):
    N = 100003
    g = torch.Generator(device=DEV).manual_seed(cols)
    order = torch.randperm(N, generator=g, device=DEV).to(torch.int32)
    src = torch.randn((N, cols), generator=g, device=DEV).to(dtype)
    fwd = rt.plan_permute(order, src)
    assert torch.equal(fwd, src[order.long()])
    back = rt.plan_permute(order, fwd, scatter=True)
    torch.cuda.synchronize()
    assert torch.equal(back, src)
    # an unaligned source takes the 4-byte path
    if cols == 4:
        big = torch.randn(N * 4 + 1, device=DEV)
        s2 = big[1:].view(N, 4)
        assert torch.equal(rt.plan_permute(order, s2), s2[order.long()])


def test_plan_permute_skips_entries_that_are_not_indices(rt):
    """Entries outside 0..count-1 move no row; the others move as usual."""
    N = 5000
    order = torch.arange(N, device=DEV, dtype=torch.int32).flip(0).contiguous()
    bad = torch.tensor([0, 17, N - 1], device=DEV)
    order[bad] = torch.tensor([-1, N, 2 ** 31 - 1], device=DEV, dtype=torch.int32)
    src = torch.randn((N, 4), device=DEV)
    dst = torch.full((N, 4), 7.0, device=DEV)
    rt.plan_permute(order, src, out=dst)
    back = torch.full((N, 4), 7.0, device=DEV)
    rt.plan_permute(order, src, out=back, scatter=True)
    torch.cuda.synchronize()
    ok = torch.ones(N, dtype=torch.bool, device=DEV)
    ok[bad] = False
    o = order.long()
    assert torch.equal(dst[ok], src[o[ok]])
    assert torch.all(dst[~ok] == 7.0)
    assert torch.equal(back[o[ok]], src[ok])
    assert int((back == 7.0).all(1).sum()) == 3


def test_plan_permute_validation(rt):
    order = torch.arange(8, dtype=torch.int32, device=DEV)
    x = torch.zeros((8, 4), device=DEV)
    P = rt._ptr
    assert rt.LIB.rt_plan_permute(P(order), 8, 16, P(x), P(x), 0, None) == 1  # overlap
    assert rt.LIB.rt_plan_permute(P(order), 8, 6, P(x), P(order), 0, None) == 1  # row bytes
    assert rt.LIB.rt_plan_permute(P(order), 8, 16, P(x), None, 0, None) == 1
    assert rt.LIB.rt_plan_permute(P(order), 8, 16, P(x), P(x.clone()), 2, None) == 1
    assert rt.LIB.rt_plan_permute(None, 0, 16, None, None, 0, None) == 0
