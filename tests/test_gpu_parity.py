"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Acceptance: bucket and sample indices bit-exact on fragments at least 1e-6
(normalised) from a cell edge; FP32 forward within 1e-5 absolute; BF16/FP8
forwards within 1e-5 of the oracle run on the oracle's own quantised texture
(whose codes are checked bit-exact against the GPU quantiser's); backward
within 1e-4 relative (grad_tex against the sum of |w g|, grad_view/grad_uv
against the gradient's norm).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from helpers import (EDGE, away_from_edges, bucket_edge_mask, check_fwd, check_grad_tex,
                     check_grad_vec, check_indices, gb_host, host, round_s, round_w)
from paper_2301_01719_amd import workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def rt():
    from paper_2301_01719_amd import radtex
    return radtex


def _sync():
    torch.cuda.synchronize()


def _rand_case(seed, W, H, n, C, N, uv_range=(-2.0, 3.0), zmin=-0.3, frames=True):
    g = torch.Generator().manual_seed(seed)
    tex = torch.rand((H, W, n, n, C), generator=g, dtype=torch.float32)
    uv = (torch.rand((N, 2), generator=g, dtype=torch.float64) * (uv_range[1] - uv_range[0])
          + uv_range[0]).to(torch.float32)
    z = torch.rand(N, generator=g, dtype=torch.float64) * (1 - zmin) + zmin
    phi = torch.rand(N, generator=g, dtype=torch.float64) * 2 * math.pi
    r = torch.sqrt(torch.clamp(1 - z * z, min=0))
    vt = torch.stack([r * torch.cos(phi), r * torch.sin(phi), z], 1)
    if frames:
        q, _ = torch.linalg.qr(torch.randn((N, 3, 3), generator=g, dtype=torch.float64))
        tbn = q.transpose(1, 2).contiguous()  # rows of an orthonormal frame
        view = torch.einsum("nkm,nk->nm", tbn, vt)  # M^T v_t so that M view = v_t
        scale = torch.rand((N, 1), generator=g, dtype=torch.float64) * 2 + 0.25
        view = view * scale
    else:
        tbn = torch.eye(3, dtype=torch.float64).expand(N, 3, 3).contiguous()
        view = vt
    return tex, wl.GBuffer(uv.contiguous(), tbn.to(torch.float32).contiguous(),
                           view.to(torch.float32).contiguous())


def _to_dev(tex, gb):
    return tex.to(DEV).contiguous(), gb.to(DEV)


# ---------------------------------------------------------------------------
# forward, FP32
# ---------------------------------------------------------------------------

def test_c1_full_forward_and_indices(rt):
    w = wl.WORKLOADS["c1"]
    tex_d = w.make_texture(DEV)
    gb_d = w.make_gbuffer(DEV)
    tex = rt.Texture(tex_d, w.W, w.H, w.n, w.C)
    out = rt.lookup_fwd(tex, gb_d.uv, gb_d.tbn, gb_d.view)
    idx, frac = rt.debug_indices(tex, gb_d.uv, gb_d.tbn, gb_d.view)
    _sync()
    uv, tbn, view = gb_host(gb_d)
    excluded = check_indices(host(idx), host(frac), uv, tbn, view, w.W, w.H, w.n)
    assert excluded < 20, excluded
    ref = oracle.lookup_fwd(oracle.Tex(host(tex_d), w.W, w.H, w.n, w.C), uv, tbn, view)
    keep = bucket_edge_mask(uv, tbn, view, w.W, w.H, w.n)
    err = check_fwd(host(out), ref, keep)
    print(f"c1 forward max |err| = {err:.3g}, excluded {excluded} of {len(uv)}")


@pytest.mark.parametrize("W,H,n,C,N", [
    (5, 3, 3, 3, 1), (5, 3, 3, 3, 255), (7, 2, 8, 1, 257), (3, 9, 16, 2, 1000),
    (1, 1, 2, 4, 513), (64, 32, 8, 4, 4097), (2, 2, 1, 4, 300), (4, 4, 32, 3, 777),
    (3, 2, 64, 4, 1500), (2, 3, 48, 3, 999)])
@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_forward_ragged_shapes(rt, W, H, n, C, N, mode):
    tex_c, gb_c = _rand_case(W * 1000 + n * 10 + C + N, W, H, n, C, N)
    tex_d, gb_d = _to_dev(tex_c, gb_c)
    tex = rt.Texture(tex_d, W, H, n, C)
    out = rt.lookup_fwd(tex, gb_d.uv, gb_d.tbn, gb_d.view, mode=mode)
    _sync()
    uv, tbn, view = gb_host(gb_c)
    m = oracle.MODE_NEAREST if mode == "nearest" else oracle.MODE_BILINEAR
    ref = oracle.lookup_fwd(oracle.Tex(tex_c.numpy(), W, H, n, C), uv, tbn, view, mode=m)
    if mode == "nearest":
        keep = bucket_edge_mask(uv, tbn, view, W, H, n)
    else:
        keep = np.ones(N, bool)  # the bilinear-bucket mode is continuous in u, v
    check_fwd(host(out), ref, keep)
    idx, frac = rt.debug_indices(tex, gb_d.uv, gb_d.tbn, gb_d.view)
    _sync()
    check_indices(host(idx), host(frac), uv, tbn, view, W, H, n)


def test_forward_empty(rt):
    tex_d = torch.rand((2, 2, 4, 4, 4), device=DEV)
    tex = rt.Texture(tex_d, 2, 2, 4, 4)
    z2 = torch.empty((0, 2), device=DEV)
    out = rt.lookup_fwd(tex, z2, torch.empty((0, 3, 3), device=DEV), torch.empty((0, 3), device=DEV))
    gt, gv, gu = rt.lookup_bwd(tex, z2, torch.empty((0, 3, 3), device=DEV),
                               torch.empty((0, 3), device=DEV), torch.empty((0, 4), device=DEV))
    _sync()
    assert out.shape == (0, 4)
    assert torch.all(gt == 0)


def test_forward_invariants(rt):
    W, H, n, C, N = 6, 5, 8, 4, 5000
    tex_c, gb_c = _rand_case(3, W, H, n, C, N, frames=False, zmin=0.0)
    tex_d, gb_d = _to_dev(tex_c, gb_c)
    tex = rt.Texture(tex_d, W, H, n, C)
    # normal incidence: the mean of the four centre samples of the bucket
    vn = torch.tensor([0.0, 0.0, 1.0], device=DEV).expand(N, 3).contiguous()
    on = host(rt.lookup_fwd(tex, gb_d.uv, gb_d.tbn, vn))
    idx, _ = rt.debug_indices(tex, gb_d.uv, gb_d.tbn, vn)
    idx = host(idx)
    assert np.all(idx[:, 2] == n // 2 - 1) and np.all(idx[:, 3] == n // 2 - 1)
    T = tex_c.numpy()
    c = n // 2
    centre = T[idx[:, 1], idx[:, 0], c - 1:c + 1, c - 1:c + 1].mean(axis=(1, 2))
    np.testing.assert_allclose(on, centre, atol=2e-7)
    # constant texture: constant image (exactly: the weights sum to 1 in FP32 up to
    # rounding of at most a few ulp)
    tc = rt.Texture(torch.full_like(tex_d, 0.625), W, H, n, C)
    oc = host(rt.lookup_fwd(tc, gb_d.uv, gb_d.tbn, gb_d.view))
    assert np.max(np.abs(oc - 0.625)) <= 4 * np.finfo(np.float32).eps
    # mirror symmetry: mirrored view and texture mirrored inside every bucket
    out = host(rt.lookup_fwd(tex, gb_d.uv, gb_d.tbn, gb_d.view))
    tx = rt.Texture(torch.flip(tex_d, dims=[3]).contiguous(), W, H, n, C)
    vx = (gb_d.view * torch.tensor([-1.0, 1.0, 1.0], device=DEV)).contiguous()
    ox = host(rt.lookup_fwd(tx, gb_d.uv, gb_d.tbn, vx))
    ty = rt.Texture(torch.flip(tex_d, dims=[2]).contiguous(), W, H, n, C)
    vy = (gb_d.view * torch.tensor([1.0, -1.0, 1.0], device=DEV)).contiguous()
    oy = host(rt.lookup_fwd(ty, gb_d.uv, gb_d.tbn, vy))
    uv, tbn, view = gb_host(gb_c)
    _, _, edge = oracle.indices(uv, tbn, view, W, H, n)
    keep = (edge[:, 0] >= EDGE) & (edge[:, 1] >= EDGE)
    assert np.max(np.abs(ox - out)[keep]) <= 1e-6
    assert np.max(np.abs(oy - out)[keep]) <= 1e-6
    # outputs inside the convex hull of their bucket
    b = T[idx[:, 1], idx[:, 0]].reshape(N, -1, C)
    idx2, _ = rt.debug_indices(tex, gb_d.uv, gb_d.tbn, gb_d.view)
    i2 = host(idx2)
    b = T[i2[:, 1], i2[:, 0]].reshape(N, -1, C)
    assert np.all(out >= b.min(axis=1) - 1e-6) and np.all(out <= b.max(axis=1) + 1e-6)


def test_bounds_fuzz(rt):
    """Degenerate coordinates and directions stay inside the texture."""
    W, H, n, C = 3, 5, 8, 4
    specials = [0.0, -0.0, 1.0, np.nextafter(np.float32(1), np.float32(0)),
                -np.float32(1e-45), -1.0, 1e30, -1e30, np.inf, -np.inf, np.nan, 0.5, 2.75, -3.25]
    uvs = np.array([[a, b] for a in specials for b in specials], np.float32)
    views = np.array([[0, 0, 0], [0, 0, -1], [0.3, 0.2, -0.9], [1, 0, 0], [np.nan, 0, 1],
                      [np.inf, 1, 1], [1e-30, 0, 1e-30], [0, 0, 1], [1e30, 1e30, 1e30]],
                     np.float32)
    N = len(uvs) * len(views)
    uv = np.repeat(uvs, len(views), axis=0)
    view = np.tile(views, (len(uvs), 1))
    tbn = np.tile(np.eye(3, dtype=np.float32), (N, 1, 1))
    tex_d = torch.rand((H, W, n, n, C), device=DEV)
    tex = rt.Texture(tex_d, W, H, n, C)
    uv_d, tbn_d, v_d = (torch.from_numpy(a).to(DEV) for a in (uv, tbn, view))
    for mode in ("nearest", "bilinear"):
        out = rt.lookup_fwd(tex, uv_d, tbn_d, v_d, mode=mode)
        gt, gv, gu = rt.lookup_bwd(tex, uv_d, tbn_d, v_d, torch.ones((N, C), device=DEV),
                                   mode=mode)
    idx, frac = rt.debug_indices(tex, uv_d, tbn_d, v_d)
    _sync()
    idx = host(idx)
    assert np.all((idx[:, 0] >= 0) & (idx[:, 0] < W) & (idx[:, 1] >= 0) & (idx[:, 1] < H))
    assert np.all((idx[:, 2] >= 0) & (idx[:, 2] < n) & (idx[:, 3] >= 0) & (idx[:, 3] < n))
    # finite inputs give finite outputs
    fin = np.isfinite(uv).all(1) & np.isfinite(view).all(1) & (np.abs(view).sum(1) > 0)
    o = host(out)
    assert np.all(np.isfinite(o[fin]))
    # on the finite inputs the backward conserves the upstream gradient's mass:
    # each fragment's tap weights sum to one (Eq. (5)), so the texture gradient
    # summed over all texels equals the upstream gradient summed over fragments
    nf = int(fin.sum())
    g = torch.Generator().manual_seed(7)
    g_up = torch.rand((nf, C), generator=g) + 0.5
    sel = torch.from_numpy(np.nonzero(fin)[0]).to(DEV)
    for mode in ("nearest", "bilinear"):
        gt, gv, gu = rt.lookup_bwd(tex, uv_d[sel].contiguous(), tbn_d[sel].contiguous(),
                                   v_d[sel].contiguous(), g_up.to(DEV), mode=mode)
        _sync()
        t = host(gt).astype(np.float64).reshape(-1, C)
        assert np.all(np.isfinite(t)), mode
        np.testing.assert_allclose(t.sum(0), g_up.double().sum(0).numpy(), rtol=1e-5,
                                   err_msg=mode)
        assert np.all(np.isfinite(host(gv))) and np.all(np.isfinite(host(gu))), mode


# ---------------------------------------------------------------------------
# quantiser and the BF16 / FP8 forwards
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("W,H,n,C", [(64, 64, 8, 4), (16, 8, 16, 4), (7, 5, 8, 3), (5, 3, 3, 1),
                                     (3, 2, 64, 4), (2, 2, 40, 3), (5, 3, 16, 4), (7, 3, 16, 2),
                                     (3, 5, 32, 2)])
def test_quantizer_bit_exact(rt, W, H, n, C):
    g = torch.Generator().manual_seed(W * H + n + C)
    t = torch.randn((H, W, n, n, C), generator=g) * torch.exp2(
        torch.randint(-20, 20, (H, W, 1, 1, 1), generator=g).float())
    t[0, 0] = 0.0
    if W * H > 2:
        t[0, 1, 0, 0, 0] = 1e-42  # subnormal amax
    tex = rt.Texture(t.to(DEV), W, H, n, C)
    c16, s16 = rt.quantize(tex, "bf16")
    c8, s8 = rt.quantize(tex, "fp8")
    _sync()
    assert s16 is None
    o16, _ = oracle.quantize(t.numpy(), W * H, n * n * C, oracle.FMT_BF16)
    o8, os8 = oracle.quantize(t.numpy(), W * H, n * n * C, oracle.FMT_FP8_E4M3)
    np.testing.assert_array_equal(host(c16).view(np.uint16).reshape(-1), o16)
    np.testing.assert_array_equal(host(c8).reshape(-1), o8)
    np.testing.assert_array_equal(host(s8).reshape(-1), os8)


@pytest.mark.parametrize("n,C", [(16, 2), (16, 4), (32, 2)])
def test_fp8_bucket_maximum_in_one_half(rt, n, C):
    """Buckets of 512, 1024 and 2048 values are quantised by two wavefronts,
    each over one contiguous half; the bucket's scale must come from the
    larger half whichever half holds it, with NaN ignored and an infinity
    giving scale 1 from either half.  An odd bucket count leaves the last
    workgroup's second bucket empty."""
    per = n * n * C
    nb = 9
    g = torch.Generator().manual_seed(per)
    t = torch.randn((nb, per), generator=g)
    t[0, : per // 2] *= 1000.0           # maximum in the first half
    t[1, per // 2:] *= 1000.0            # maximum in the second half
    t[2, per - 1] = -3.0e4               # a single largest value, last element
    t[3, 0] = float("nan")               # NaN in the first half only
    t[4, per // 2 + 5] = float("nan")    # NaN in the second half only
    t[5, per // 2] = float("inf")        # infinity in the second half
    t[6, 3] = float("-inf")              # infinity in the first half
    t[7] = 0.0                           # all zero: scale 1
    t[8, : per // 2] = 0.0               # first half zero
    tex = rt.Texture(t.to(DEV).view(1, nb, n, n, C), nb, 1, n, C)
    c8, s8 = rt.quantize(tex, "fp8")
    _sync()
    o8, os8 = oracle.quantize(t.numpy(), nb, per, oracle.FMT_FP8_E4M3)
    np.testing.assert_array_equal(host(s8).reshape(-1), os8)
    np.testing.assert_array_equal(host(c8).reshape(-1), o8)
    assert os8[5] == 1.0 and os8[6] == 1.0 and os8[7] == 1.0


def test_e4m3_encode_exhaustive_grid(rt):
    """Every E4M3 value, midpoint and the floats next to the midpoints, through
    one bucket with amax = 448 (inv = 1 exactly)."""
    vals = np.array([oracle.e4m3_to_f64(c) for c in range(0x7F)])
    mids = ((vals[:-1] + vals[1:]) / 2).astype(np.float32)
    pts = np.concatenate([vals.astype(np.float32), mids, np.nextafter(mids, np.float32(0)),
                          np.nextafter(mids, np.float32(1000))])
    pts = np.concatenate([pts, -pts])
    n, C = 8, 4
    per = n * n * C
    nb = (len(pts) + per - 2) // (per - 1)
    buf = np.zeros((nb, per), np.float32)
    flat = np.concatenate([pts, np.zeros(nb * (per - 1) - len(pts), np.float32)])
    buf[:, 1:] = flat.reshape(nb, per - 1)
    buf[:, 0] = 448.0
    tex = rt.Texture(torch.from_numpy(buf).to(DEV), nb, 1, n, C)
    c8, s8 = rt.quantize(tex, "fp8")
    _sync()
    o8, os8 = oracle.quantize(buf, nb, per, oracle.FMT_FP8_E4M3)
    assert np.all(host(s8) == 1.0) and np.all(os8 == 1.0)
    np.testing.assert_array_equal(host(c8).reshape(-1), o8)


@pytest.mark.parametrize("fmt", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("W,H,n,C", [(16, 8, 8, 4), (7, 5, 3, 3), (5, 9, 16, 1), (1, 1, 1, 2)])
def test_atlas_layout_looks_up_as_bucket_major(rt, W, H, n, C, fmt):
    """A texture handed over as an atlas [H n, W n, C] (sample (x, y) of
    bucket (i, j) at row j n + y, column i n + x) looks up exactly as the
    bucket-major matrix torch makes from it by a permutation, in both modes."""
    g = torch.Generator().manual_seed(W * 1000 + H * 100 + n * 10 + C)
    scales = None
    if fmt == "fp8":
        # finite codes only (E4M3 NaN is S.1111.111), random signs
        atlas = (torch.randint(0, 0x7F, (H * n, W * n, C), generator=g)
                 | (torch.randint(0, 2, (H * n, W * n, C), generator=g) << 7)).to(torch.uint8)
        scales = torch.rand((H, W), generator=g).to(DEV)
    else:
        atlas = torch.randn((H * n, W * n, C), generator=g)
        if fmt == "bf16":
            atlas = atlas.to(torch.bfloat16)
    bucket = atlas.reshape(H, n, W, n, C).permute(0, 2, 1, 3, 4).contiguous()
    tex_a = rt.Texture(atlas.to(DEV), W, H, n, C, fmt, scales, layout="atlas")
    tex_b = rt.Texture(bucket.to(DEV), W, H, n, C, fmt, scales)
    gb = wl.flat_gbuffer(4096, W + H + n + C, DEV)
    for mode in ("nearest", "bilinear"):
        out_a = rt.lookup_fwd(tex_a, gb.uv, gb.tbn, gb.view, mode)
        out_b = rt.lookup_fwd(tex_b, gb.uv, gb.tbn, gb.view, mode)
        _sync()
        assert torch.isfinite(out_b).all()
        assert torch.equal(out_a, out_b), mode


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_quantized_forward(rt, fmt, mode):
    W, H, n, C, N = 9, 7, 16, 4, 20000
    tex_c, gb_c = _rand_case(17, W, H, n, C, N)
    tex_d, gb_d = _to_dev(tex_c, gb_c)
    tex = rt.Texture(tex_d, W, H, n, C)
    codes, scales = rt.quantize(tex, fmt)
    qt = rt.Texture(codes, W, H, n, C, fmt, scales)
    out = rt.lookup_fwd(qt, gb_d.uv, gb_d.tbn, gb_d.view, mode=mode)
    out32 = rt.lookup_fwd(tex, gb_d.uv, gb_d.tbn, gb_d.view, mode=mode)
    _sync()
    f = oracle.FMT_BF16 if fmt == "bf16" else oracle.FMT_FP8_E4M3
    ocodes, oscales = oracle.quantize(tex_c.numpy(), W * H, n * n * C, f)
    uv, tbn, view = gb_host(gb_c)
    m = oracle.MODE_NEAREST if mode == "nearest" else oracle.MODE_BILINEAR
    ref = oracle.lookup_fwd(oracle.Tex(ocodes, W, H, n, C, f, oscales), uv, tbn, view, mode=m)
    keep = bucket_edge_mask(uv, tbn, view, W, H, n) if mode == "nearest" else None
    err = check_fwd(host(out), ref, keep)
    e2e = np.abs(host(out) - host(out32))
    print(f"{fmt}/{mode}: max err vs oracle {err:.3g}; vs FP32 storage max {e2e.max():.3g} "
          f"mean {e2e.mean():.3g}")


# ---------------------------------------------------------------------------
# backward
# ---------------------------------------------------------------------------

def _select(gb, keep):
    k = torch.from_numpy(np.nonzero(keep)[0])
    return wl.GBuffer(gb.uv[k].contiguous(), gb.tbn[k].contiguous(), gb.view[k].contiguous())


def _bwd_case(rt, seed, W, H, n, C, N, mode, fmt="f32", uv_range=(-1.0, 2.0), frames=True):
    """Random case with the fragments closer than 1e-6 to a cell edge removed
    (there the two sides may legitimately pick different cells)."""
    tex_c, gb_c = _rand_case(seed, W, H, n, C, N, uv_range=uv_range, frames=frames)
    uv, tbn, view = gb_host(gb_c)
    gb_c = _select(gb_c, away_from_edges(uv, tbn, view, W, H, n, mode))
    N = gb_c.count
    tex_d, gb_d = _to_dev(tex_c, gb_c)
    go = torch.randn((N, C), generator=torch.Generator().manual_seed(seed + 1))
    tex = rt.Texture(tex_d, W, H, n, C)
    otex = oracle.Tex(tex_c.numpy(), W, H, n, C)
    if fmt != "f32":
        codes, scales = rt.quantize(tex, fmt)
        tex = rt.Texture(codes, W, H, n, C, fmt, scales)
        f = oracle.FMT_BF16 if fmt == "bf16" else oracle.FMT_FP8_E4M3
        oc, osc = oracle.quantize(tex_c.numpy(), W * H, n * n * C, f)
        otex = oracle.Tex(oc, W, H, n, C, f, osc)
    gt, gv, gu = rt.lookup_bwd(tex, gb_d.uv, gb_d.tbn, gb_d.view, go.to(DEV), mode=mode)
    _, frac = rt.debug_indices(tex, gb_d.uv, gb_d.tbn, gb_d.view)
    _sync()
    uv, tbn, view = gb_host(gb_c)
    m = oracle.MODE_NEAREST if mode == "nearest" else oracle.MODE_BILINEAR
    ref = oracle.lookup_bwd(otex, uv, tbn, view, go.numpy(), mode=m)
    ref["round_view"], ref["round_uv"] = oracle.lookup_bwd_round(
        otex, uv, tbn, view, go.numpy(), round_s(n), round_w(W, H, uv), mode=m)
    ref["frac_gpu"] = host(frac)
    return (gt, gv, gu), ref, (uv, tbn, view), go.numpy()


def _check_fracs(ref, uv, tbn, view, W, H, n, keep):
    """The GPU's in-bucket fractions within round_s(n) of the oracle's: the
    rounding that the gradients' rounding term assumes."""
    _, fo, _ = oracle.indices(uv, tbn, view, W, H, n)
    d = np.abs(ref["frac_gpu"].astype(np.float64) - fo)[keep]
    assert d.size == 0 or d.max() <= round_s(n), (d.max(), round_s(n))
    return float(d.max()) if d.size else 0.0


def _check_view_uv(ref, gv, gu, go, uv, tbn, view, W, H, n, mode):
    keep = _smooth_mask(uv, tbn, view, W, H, n, mode)
    _check_fracs(ref, uv, tbn, view, W, H, n, keep)
    rv = check_grad_vec(host(gv)[keep], ref["grad_view"][keep], ref["scale_view"][keep],
                        go[keep], ref["round_view"][keep])
    ru = check_grad_vec(host(gu)[keep], ref["grad_uv"][keep], ref["scale_uv"][keep],
                        go[keep], ref["round_uv"][keep])
    return keep, rv, ru


def _smooth_mask(uv, tbn, view, W, H, n, mode):
    _, _, edge = oracle.indices(uv, tbn, view, W, H, n)
    keep = (edge[:, 1] >= 1e-5) & (edge[:, 2] >= 1e-5)
    if mode == "nearest":
        keep &= edge[:, 0] >= EDGE
    else:
        fu = uv.astype(np.float64) - np.floor(uv.astype(np.float64))
        p = fu * [W, H] - 0.5
        keep &= np.all(np.abs(p - np.round(p)) >= 1e-5 * np.array([W, H]), axis=1)
    return keep


@pytest.mark.parametrize("W,H,n,C,N", [(16, 16, 8, 3, 30000), (5, 3, 3, 1, 777),
                                       (64, 64, 16, 4, 50000), (2, 2, 2, 2, 4097),
                                       (6, 5, 64, 1, 20000), (3, 3, 48, 1, 5000)])
@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_backward_vs_oracle(rt, W, H, n, C, N, mode):
    (gt, gv, gu), ref, (uv, tbn, view), go = _bwd_case(rt, W + N + n, W, H, n, C, N, mode)
    rt_tex = check_grad_tex(host(gt), ref, n)
    keep, rv, ru = _check_view_uv(ref, gv, gu, go, uv, tbn, view, W, H, n, mode)
    print(f"{mode} {W}x{H}x{n}x{C} N={N}: grad_tex err/tol {rt_tex:.2e}; grad_view {rv}; "
          f"grad_uv {ru}; {int((~keep).sum())} fragments near kinks")


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_backward_quantized_storage(rt, fmt):
    (gt, gv, gu), ref, (uv, tbn, view), go = _bwd_case(rt, 9, 12, 10, 8, 4, 20000, "nearest",
                                                       fmt=fmt)
    check_grad_tex(host(gt), ref, 8)
    _check_view_uv(ref, gv, gu, go, uv, tbn, view, 12, 10, 8, "nearest")


@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_backward_hot_buckets(rt, mode):
    """Thousands of fragments in a few buckets: the chunked second pass."""
    W, H, n, C, N = 4, 4, 8, 4, 30000
    (gt, gv, gu), ref, (uv, tbn, view), go = _bwd_case(
        rt, 77, W, H, n, C, N, mode, uv_range=(0.30, 0.45))
    check_grad_tex(host(gt), ref, n)
    # a single bucket holding every fragment
    g1 = torch.Generator().manual_seed(5)
    tex_c = torch.rand((H, W, n, n, C), generator=g1)
    Nh = 9000
    uvh = torch.full((Nh, 2), 0.6, dtype=torch.float32)
    _, gbh = _rand_case(6, W, H, n, C, Nh, frames=False)
    gbh = wl.GBuffer(uvh, gbh.tbn, gbh.view)
    gbh = _select(gbh, away_from_edges(*gb_host(gbh), W, H, n, mode))
    uvh = gbh.uv
    Nh = gbh.count
    goh = torch.randn((Nh, C), generator=g1)
    tex = rt.Texture(tex_c.to(DEV), W, H, n, C)
    gt2, _, _ = rt.lookup_bwd(tex, uvh.to(DEV), gbh.tbn.to(DEV), gbh.view.to(DEV), goh.to(DEV),
                              mode=mode, want_view=False, want_uv=False)
    _sync()
    m = oracle.MODE_NEAREST if mode == "nearest" else oracle.MODE_BILINEAR
    r2 = oracle.lookup_bwd(oracle.Tex(tex_c.numpy(), W, H, n, C), uvh.numpy(), host(gbh.tbn),
                           host(gbh.view), goh.numpy(), mode=m, want_view=False, want_uv=False)
    check_grad_tex(host(gt2), r2, n)



def _records_per_bucket(uv, W, H, mode):
    """Records per bucket of the accumulation: one per fragment (nearest) or
    one per fragment and bucket of its bilinear footprint."""
    f = uv.astype(np.float64) - np.floor(uv.astype(np.float64))
    if mode == "nearest":
        i = np.minimum((f[:, 0] * W).astype(np.int64), W - 1)
        j = np.minimum((f[:, 1] * H).astype(np.int64), H - 1)
        return np.bincount(j * W + i, minlength=W * H)
    p = f * [W, H] - 0.5
    i0 = np.floor(p[:, 0]).astype(np.int64)
    j0 = np.floor(p[:, 1]).astype(np.int64)
    b = [((j0 + dj) % H) * W + (i0 + di) % W for dj in (0, 1) for di in (0, 1)]
    return np.bincount(np.concatenate(b), minlength=W * H)


@pytest.mark.parametrize("W,N_uni,clusters", [(16, 2000, ((3, 4, 20000), (10, 11, 600))),
                                              (64, 40000, ((10, 20, 5000), (40, 7, 300)))])
@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_backward_mixed_bucket_sizes(rt, W, N_uni, clusters, mode):
    """Small, big (65..2048 records) and hot buckets in one launch, with more
    and with fewer than 64 records per bucket on average: the accumulation's
    register window then gathers its records from the fragments, or reads
    them from the payload written in sorted order."""
    H, n, C = W, 8, 4
    N = N_uni + sum(c[2] for c in clusters)
    tex_c, gb = _rand_case(81 + W, W, H, n, C, N, uv_range=(0.0, 1.0))
    g = torch.Generator().manual_seed(82 + W)
    uv = gb.uv.clone()
    at = N_uni
    for i, j, cnt in clusters:
        jit = (torch.rand((cnt, 2), generator=g, dtype=torch.float64) - 0.5) * 0.6
        uv[at:at + cnt, 0] = ((i + 0.5 + jit[:, 0]) / W).float()
        uv[at:at + cnt, 1] = ((j + 0.5 + jit[:, 1]) / H).float()
        at += cnt
    gb = wl.GBuffer(uv.contiguous(), gb.tbn, gb.view)
    gb = _select(gb, away_from_edges(*gb_host(gb), W, H, n, mode))
    cnt = _records_per_bucket(host(gb.uv), W, H, mode)
    assert cnt.min() <= 64 and np.any((cnt > 64) & (cnt <= 2048)) and cnt.max() > 2048
    window_path = "payload" if cnt.sum() <= 64 * W * H else "gather"
    assert window_path == ("gather" if W == 16 else "payload")
    go = torch.randn((gb.count, C), generator=torch.Generator().manual_seed(83 + W))
    tex = rt.Texture(tex_c.to(DEV), W, H, n, C)
    gt, gv, gu = rt.lookup_bwd(tex, gb.uv.to(DEV), gb.tbn.to(DEV), gb.view.to(DEV), go.to(DEV),
                               mode=mode)
    _sync()
    u, t, v = gb_host(gb)
    m = oracle.MODE_NEAREST if mode == "nearest" else oracle.MODE_BILINEAR
    otex = oracle.Tex(tex_c.numpy(), W, H, n, C)
    ref = oracle.lookup_bwd(otex, u, t, v, go.numpy(), mode=m)
    check_grad_tex(host(gt), ref, n)
    keep = _smooth_mask(u, t, v, W, H, n, mode)
    rv, ru = oracle.lookup_bwd_round(otex, u, t, v, go.numpy(), round_s(n), round_w(W, H, u),
                                     mode=m)
    check_grad_vec(host(gv)[keep], ref["grad_view"][keep], ref["scale_view"][keep],
                   go.numpy()[keep], rv[keep])
    check_grad_vec(host(gu)[keep], ref["grad_uv"][keep], ref["scale_uv"][keep],
                   go.numpy()[keep], ru[keep])

def test_backward_deterministic(rt):
    W, H, n, C, N = 32, 32, 8, 4, 200000
    tex_c, gb_c = _rand_case(11, W, H, n, C, N, uv_range=(0.0, 0.3))
    tex_d, gb_d = _to_dev(tex_c, gb_c)
    go = torch.randn((N, C), device=DEV)
    tex = rt.Texture(tex_d, W, H, n, C)
    first = rt.lookup_bwd(tex, gb_d.uv, gb_d.tbn, gb_d.view, go)
    base = [host(x).copy() for x in first]
    for rep in range(4):
        # a concurrent load on another stream must not change the result
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            junk = torch.randn((4096, 4096), device=DEV) @ torch.randn((4096, 4096), device=DEV)
        again = rt.lookup_bwd(tex, gb_d.uv, gb_d.tbn, gb_d.view, go)
        _sync()
        for a, b in zip(base, again):
            assert np.array_equal(a.view(np.uint32), host(b).view(np.uint32))
        del junk


def test_backward_identities(rt):
    """Adjoint identity <grad_tex, T> = <g, out> and mass conservation on the GPU
    result alone (exact for a linear map up to rounding)."""
    W, H, n, C, N = 16, 16, 8, 4, 100000
    tex_c, gb_c = _rand_case(12, W, H, n, C, N)
    tex_d, gb_d = _to_dev(tex_c, gb_c)
    go = torch.randn((N, C), device=DEV)
    tex = rt.Texture(tex_d, W, H, n, C)
    out = rt.lookup_fwd(tex, gb_d.uv, gb_d.tbn, gb_d.view)
    gt, gv, _ = rt.lookup_bwd(tex, gb_d.uv, gb_d.tbn, gb_d.view, go)
    _sync()
    lhs = np.sum(host(gt).astype(np.float64) * tex_c.numpy())
    rhs = np.sum(host(go).astype(np.float64) * host(out))
    assert abs(lhs - rhs) <= 1e-5 * np.sum(np.abs(host(go)) * np.abs(host(out)))
    np.testing.assert_allclose(host(gt).astype(np.float64).sum(axis=(0, 1, 2, 3)),
                               host(go).astype(np.float64).sum(0), rtol=1e-5, atol=1e-2)
    # the lookup depends only on the direction of the view vector
    dots = np.abs(np.sum(host(gv) * host(gb_d.view), axis=1))
    assert np.max(dots) <= 1e-3 * max(1.0, np.abs(host(gv)).max())


@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_tiled_fragment_order(rt, mode):
    """The tiling hint (3 views of 37 x 53 pixels: ragged in both directions
    against the 32 x 8 tiles) changes only which thread handles a fragment:
    forwards of every storage format and the whole backward are bit-identical
    to the flat order, and the forward matches the oracle."""
    W, H, n, C = 48, 40, 8, 4
    gb = wl.plane_gbuffer(3, 53, 37, seed=21, device=DEV)
    assert gb.image == (3, 37, 53) and gb.count == 3 * 37 * 53
    tex = wl.iid_texture(W, H, n, C, seed=22, device=DEV)
    master = rt.Texture(tex, W, H, n, C)
    texs = {"f32": (master, oracle.Tex(host(tex), W, H, n, C))}
    for fmt, ofmt in (("bf16", oracle.FMT_BF16), ("fp8", oracle.FMT_FP8_E4M3)):
        c, s = rt.quantize(master, fmt)
        texs[fmt] = (rt.Texture(c, W, H, n, C, fmt, s),
                     oracle.Tex(host(c).view(np.uint16) if fmt == "bf16" else host(c), W, H, n, C,
                                ofmt, None if s is None else host(s)))
    uv, tbn, view = gb_host(gb)
    keep = away_from_edges(uv, tbn, view, W, H, n, mode)
    omode = oracle.MODE_NEAREST if mode == "nearest" else oracle.MODE_BILINEAR
    for fmt, (t, ot) in texs.items():
        flat = rt.lookup_fwd(t, gb.uv, gb.tbn, gb.view, mode)
        tiled = rt.lookup_fwd(t, gb.uv, gb.tbn, gb.view, mode, image=gb.image)
        _sync()
        assert torch.equal(flat, tiled), fmt
        check_fwd(host(tiled), oracle.lookup_fwd(ot, uv, tbn, view, omode), keep)
    go = wl.grad_out(gb.count, C, seed=23, device=DEV)
    a = rt.lookup_bwd(master, gb.uv, gb.tbn, gb.view, go, mode)
    b = rt.lookup_bwd(master, gb.uv, gb.tbn, gb.view, go, mode, image=gb.image)
    _sync()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    with pytest.raises(rt.RadtexError):
        rt.lookup_fwd(master, gb.uv, gb.tbn, gb.view, mode, image=(3, 37, 52))


def test_graph_replay(rt):
    """A captured HIP graph of one whole step (quantise, forward, backward)
    replays bit-identically to the eager step, replay after replay, with the
    program's own eager work and synchronisations in between."""
    W, H, n, C = 32, 24, 8, 4
    gb = wl.plane_gbuffer(2, 61, 29, seed=31, device=DEV)
    tex = wl.smooth_texture(W, H, n, C, seed=32, device=DEV)
    master = rt.Texture(tex, W, H, n, C)
    codes = torch.empty((H, W, n, n, C), dtype=torch.int16, device=DEV)
    tq = rt.Texture(codes, W, H, n, C, "bf16")
    go = wl.grad_out(gb.count, C, seed=33, device=DEV)
    out = torch.empty((gb.count, C), device=DEV)
    gt = torch.empty((H, W, n, n, C), device=DEV)
    ws = torch.empty(rt.bwd_workspace_bytes(tq, gb.count), dtype=torch.uint8, device=DEV)

    def step():
        rt._check(rt.LIB.rt_quantize(master.handle, rt.FORMATS["bf16"], rt._ptr(codes), None,
                                     rt._stream(DEV)))
        rt.lookup_fwd(tq, gb.uv, gb.tbn, gb.view, out=out, image=gb.image)
        return rt.lookup_bwd(tq, gb.uv, gb.tbn, gb.view, go, workspace=ws, grad_tex=gt,
                             image=gb.image)

    _, gv, gu = step()
    _sync()
    ref = [codes.clone(), out.clone(), gt.clone(), gv.clone(), gu.clone()]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        _, gv_g, gu_g = step()
    for r in range(3):
        for t in (codes, out, gt, gv_g, gu_g):
            t.fill_(float("nan") if t.dtype.is_floating_point else -1)  # eager work between
        _sync()
        graph.replay()
        _sync()
        for a, b in zip(ref, (codes, out, gt, gv_g, gu_g)):
            assert torch.equal(a, b), r


@pytest.mark.parametrize("W,H", [(4096, 2), (1, 2048), (1024, 1024)])
def test_bilinear_bucket_weights_keep_their_precision_on_wide_matrices(rt, W, H):
    # the bucket weight a = frac(u) W - 1/2 - floor(...) must not be rounded
    # to the ulp of u W (3e-5 at u W ~ 512): coordinates spread over
    # [-3, 3] against a matrix of up to 4096 buckets per side, with a texture
    # of full contrast between neighbouring buckets
    n, C, N = 2, 1, 20000
    g = torch.Generator().manual_seed(W + H)
    tex_c = (torch.rand((H, W, n, n, C), generator=g) < 0.5).to(torch.float32)
    uv = (torch.rand((N, 2), generator=g, dtype=torch.float64) * 6 - 3).to(torch.float32)
    tbn = torch.eye(3).expand(N, 3, 3).contiguous()
    view = torch.tensor([[0.1, 0.2, 1.0]]).expand(N, 3).contiguous()
    tex_d = tex_c.to(DEV)
    tex = rt.Texture(tex_d, W, H, n, C)
    out = rt.lookup_fwd(tex, uv.to(DEV), tbn.to(DEV), view.to(DEV), mode="bilinear")
    _sync()
    ref = oracle.lookup_fwd(oracle.Tex(tex_c.numpy(), W, H, n, C), uv.numpy(), tbn.numpy(),
                            view.numpy(), mode=oracle.MODE_BILINEAR)
    err = check_fwd(host(out), ref)
    print(f"W={W} H={H}: max |err| {err:.3g}")


def test_backward_refuses_buckets_beyond_its_tiles(rt):
    # n n C above 4096 (n = 64 with two channels) is refused on the host: the
    # accumulation keeps four bucket tiles per workgroup in LDS
    W, H, n, C, N = 2, 2, 64, 2, 100
    tex_c, gb_c = _rand_case(5, W, H, n, C, N)
    tex_d, gb_d = _to_dev(tex_c, gb_c)
    tex = rt.Texture(tex_d, W, H, n, C)
    assert rt.LIB.rt_lookup_bwd_workspace(tex.handle, N, 0) == 0
    with pytest.raises(rt.RadtexError) as e:
        rt.lookup_bwd(tex, gb_d.uv, gb_d.tbn, gb_d.view, torch.ones((N, C), device=DEV))
    assert e.value.status == 2
