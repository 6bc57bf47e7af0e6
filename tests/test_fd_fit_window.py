"""FP64 central finite differences of the backward on the fit workload
(256 x 256 buckets of 8 x 8 RGB samples, 16 views of 512 x 512, upstream
gradients i.i.d. N(0, 1)): every fragment that reads a bucket of the window
[0, 16)^2, every texel of those buckets.

The loss is L = sum_f g_f . out_f over those fragments (those within 1e-6
of a bucket edge left out, where the two sides may pick different buckets).
The differences are taken on the oracle's binary64 forward lookup:

* dL/dtexel: the lookup is linear in the texels, so a central difference of
  step 1/2 is exact up to rounding; one texel position (y, x, c) is moved in
  every window bucket at once (nearest mode: each fragment reads one bucket)
  or in the buckets of one parity class (i mod 2, j mod 2) at once
  (bilinear-bucket mode: a fragment's four buckets have four different
  classes), so each fragment's change belongs to one bucket.
* dL/dview: step 1e-6 on each component of V, on fragments at least 1e-4
  (normalised) from every kink of the mapping (texel lines, clamp bounds, the
  diagonal of Eq. (3), bucket-pair edges).
* dL/duv (bilinear-bucket mode): step 1e-7 on u and v, same fragments.

The oracle's analytic gradients are pinned against these differences on the
CPU; the GPU's (through the C ABI) are compared with the same differences to
the backward's criterion.
"""
import functools

import numpy as np
import pytest
import torch

import oracle
from helpers import check_grad_tex, check_grad_vec, round_s, round_w
from paper_2301_01719_amd import workloads as wl

WIN = 16
H_VIEW, H_UV, H_TEX = 1e-6, 1e-7, 0.5
KINK = 1e-4
MODES = {"nearest": oracle.MODE_NEAREST, "bilinear": oracle.MODE_BILINEAR}


def _buckets_of(uv, W, H, mode):
    """[N, k] bucket columns and rows of each fragment's footprint."""
    u = uv.astype(np.float64)
    f = u - np.floor(u)
    if mode == "nearest":
        i = np.minimum(np.floor(f[:, 0] * W).astype(np.int64), W - 1)
        j = np.minimum(np.floor(f[:, 1] * H).astype(np.int64), H - 1)
        return i[:, None], j[:, None]
    p = f * [W, H] - 0.5
    i0 = np.floor(p[:, 0]).astype(np.int64)
    j0 = np.floor(p[:, 1]).astype(np.int64)
    i = np.stack([i0 % W, (i0 + 1) % W, i0 % W, (i0 + 1) % W], 1)
    j = np.stack([j0 % H, j0 % H, (j0 + 1) % H, (j0 + 1) % H], 1)
    return i, j


@functools.lru_cache(maxsize=None)
def _full():
    w = wl.WORKLOADS["c4"]
    tex = w.make_texture("cpu")
    gb = w.make_gbuffer("cpu")
    go = wl.grad_out(gb.count, w.C, seed=w.seed, device="cpu")
    return w, tex.numpy(), gb, go.numpy()


@functools.lru_cache(maxsize=None)
def _window(mode):
    w, T, gb, go = _full()
    W, H, n, C = w.W, w.H, w.n, w.C
    uv, tbn, view = gb.uv.numpy(), gb.tbn.numpy(), gb.view.numpy()
    bi, bj = _buckets_of(uv, W, H, mode)
    touch = np.any((bi < WIN) & (bj < WIN), axis=1)
    # leave out fragments at a bucket edge (nearest) or a bucket-pair edge
    f = uv.astype(np.float64) - np.floor(uv.astype(np.float64))
    if mode == "nearest":
        e = np.abs(f * [W, H] - np.round(f * [W, H])) / [W, H]
    else:
        p = f * [W, H] - 0.5
        e = np.abs(p - np.round(p)) / [W, H]
    sel = np.nonzero(touch & np.all(e >= 1e-6, axis=1))[0]
    u, t, v, g = uv[sel], tbn[sel], view[sel], go[sel]
    m = MODES[mode]
    # kinks of the mapping for the view and uv differences
    _, _, edge = oracle.indices(u, t, v, W, H, n)
    smooth = (edge[:, 1] >= KINK) & (edge[:, 2] >= KINK) & np.all(e[sel] >= KINK, axis=1)
    U, M, V = u.astype(np.float64), t.astype(np.float64).reshape(-1, 9), v.astype(np.float64)
    g64 = g.astype(np.float64)
    tex32 = oracle.Tex(T, W, H, n, C)
    # dL/dview and dL/duv
    fd_view = np.zeros((len(sel), 3))
    for k in range(3):
        Vp, Vm = V.copy(), V.copy()
        Vp[:, k] += H_VIEW
        Vm[:, k] -= H_VIEW
        op = oracle.lookup_fwd_f64(tex32, U, M, Vp, m)
        om = oracle.lookup_fwd_f64(tex32, U, M, Vm, m)
        fd_view[:, k] = np.sum(g64 * (op - om), axis=1) / (2 * H_VIEW)
    fd_uv = np.zeros((len(sel), 2))
    if mode == "bilinear":
        for k in range(2):
            Up, Um = U.copy(), U.copy()
            Up[:, k] += H_UV
            Um[:, k] -= H_UV
            op = oracle.lookup_fwd_f64(tex32, Up, M, V, m)
            om = oracle.lookup_fwd_f64(tex32, Um, M, V, m)
            fd_uv[:, k] = np.sum(g64 * (op - om), axis=1) / (2 * H_UV)
    # dL/dtexel over the window
    T64 = T.astype(np.float64)
    tex64 = oracle.Tex(T64, W, H, n, C, oracle.FMT_F64)
    assert np.shares_memory(tex64.data, T64)
    fbi, fbj = _buckets_of(u, W, H, mode)
    classes = [(0, 0)] if mode == "nearest" else [(0, 0), (1, 0), (0, 1), (1, 1)]
    fd_tex = np.zeros((WIN, WIN, n, n, C))
    wj, wi = np.mgrid[0:WIN, 0:WIN]
    for ci, cj in classes:
        moved = (wi % 2 == ci) & (wj % 2 == cj) if mode == "bilinear" else np.ones_like(wi, bool)
        mj, mi = wj[moved], wi[moved]
        # the fragment's bucket of this class, if it lies in the window
        if mode == "nearest":
            fi, fj = fbi[:, 0], fbj[:, 0]
        else:
            k = np.argmax((fbi % 2 == ci) & (fbj % 2 == cj), axis=1)
            fi, fj = fbi[np.arange(len(u)), k], fbj[np.arange(len(u)), k]
        inwin = (fi < WIN) & (fj < WIN)
        if mode == "bilinear":
            inwin &= (fi % 2 == ci) & (fj % 2 == cj)
        for y in range(n):
            for x in range(n):
                for c in range(C):
                    T64[mj, mi, y, x, c] += H_TEX
                    op = oracle.lookup_fwd_f64(tex64, U, M, V, m)
                    T64[mj, mi, y, x, c] -= 2 * H_TEX
                    om = oracle.lookup_fwd_f64(tex64, U, M, V, m)
                    T64[mj, mi, y, x, c] += H_TEX
                    dl = g64[:, c] * (op[:, c] - om[:, c]) / (2 * H_TEX)
                    np.add.at(fd_tex[:, :, y, x, c], (fj[inwin], fi[inwin]), dl[inwin])
    assert np.array_equal(T64, T.astype(np.float64))  # restored exactly
    ref = oracle.lookup_bwd(tex32, u, t, v, g, mode=m, window=(0, 0, WIN, WIN))
    rv, ru = oracle.lookup_bwd_round(tex32, u, t, v, g, round_s(n), round_w(W, H, u), mode=m)
    return {"w": w, "T": T, "sel": sel, "uv": u, "tbn": t, "view": v, "g": g, "smooth": smooth,
            "fd_view": fd_view, "fd_uv": fd_uv, "fd_tex": fd_tex, "ref": ref,
            "round_view": rv, "round_uv": ru}


@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_oracle_gradients_match_finite_differences_on_the_fit_window(mode):
    d = _window(mode)
    w, ref, sm = d["w"], d["ref"], d["smooth"]
    n = w.n
    assert len(d["sel"]) > 10000 and sm.sum() > 0.8 * len(d["sel"])
    # every texel of the window
    G, A = ref["grad_tex"], ref["abs_tex"]
    assert np.all(np.abs(G - d["fd_tex"]) <= 1e-12 * np.maximum(A, 1.0))
    # texels no fragment reaches (view directions of the 16 cameras do not
    # cover every sample) have no gradient and no difference
    assert np.count_nonzero(A) > 0.5 * A.size
    assert np.all(d["fd_tex"][A == 0] == 0) and np.all(G[A == 0] == 0)
    sg = np.abs(d["g"].astype(np.float64)).sum(1)
    dv = np.linalg.norm(ref["grad_view"] - d["fd_view"], axis=1)[sm]
    assert np.all(dv <= 1e-6 * np.linalg.norm(d["fd_view"], axis=1)[sm] + 1e-9 * sg[sm])
    du = np.linalg.norm(ref["grad_uv"] - d["fd_uv"], axis=1)[sm]
    if mode == "bilinear":
        assert np.all(du <= 1e-6 * np.linalg.norm(d["fd_uv"], axis=1)[sm] + 1e-9 * w.W * sg[sm])
    else:
        assert np.all(ref["grad_uv"] == 0.0) and np.all(np.abs(d["fd_uv"]) == 0.0)
    # grad_view . view = 0: the lookup depends on the direction of V only
    gv = ref["grad_view"][sm]
    vv = d["view"][sm].astype(np.float64)
    assert np.all(np.abs(np.sum(gv * vv, 1)) <= 1e-9 * np.linalg.norm(gv, axis=1)
                  * np.linalg.norm(vv, axis=1) + 1e-15)


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["nearest", "bilinear"])
def test_gpu_gradients_match_finite_differences_on_the_fit_window(mode):
    from paper_2301_01719_amd import radtex as rt
    d = _window(mode)
    w, ref, sm = d["w"], d["ref"], d["smooth"]
    W, H, n, C = w.W, w.H, w.n, w.C
    dev = "cuda:0"
    tex = rt.Texture(torch.from_numpy(d["T"]).to(dev), W, H, n, C)
    uv, tbn, view = (torch.from_numpy(np.ascontiguousarray(a)).to(dev)
                     for a in (d["uv"], d["tbn"], d["view"]))
    g = torch.from_numpy(d["g"]).to(dev)
    gt, gv, gu = rt.lookup_bwd(tex, uv, tbn, view, g, mode=mode)
    torch.cuda.synchronize()
    Gw = gt[:WIN, :WIN].cpu().numpy()
    r = check_grad_tex(Gw, {"grad_tex": d["fd_tex"], "abs_tex": ref["abs_tex"],
                            "absg_tex": ref["absg_tex"]}, n)
    go = d["g"]
    rv = check_grad_vec(gv.cpu().numpy()[sm], d["fd_view"][sm], ref["scale_view"][sm], go[sm],
                        d["round_view"][sm])
    ru = check_grad_vec(gu.cpu().numpy()[sm], d["fd_uv"][sm], ref["scale_uv"][sm], go[sm],
                        d["round_uv"][sm])
    print(f"{mode}: {len(d['sel'])} fragments ({int(sm.sum())} smooth); grad_tex err/tol "
          f"{r:.3g}; grad_view {rv}; grad_uv {ru}")
    # the same fragments inside the full 16-view launch (the tiled order the
    # bench uses): per-fragment gradients do not depend on the other fragments
    w_, T, gb, gofull = _full()
    texf = rt.Texture(torch.from_numpy(T).to(dev), W, H, n, C)
    gbd = gb.to(dev)
    _, gvf, guf = rt.lookup_bwd(texf, gbd.uv, gbd.tbn, gbd.view, torch.from_numpy(gofull).to(dev),
                                mode=mode, want_tex=False, image=gbd.image)
    torch.cuda.synchronize()
    sel = torch.from_numpy(d["sel"]).to(dev)
    check_grad_vec(gvf[sel].cpu().numpy()[sm], d["fd_view"][sm], ref["scale_view"][sm], go[sm],
                   d["round_view"][sm])
    check_grad_vec(guf[sel].cpu().numpy()[sm], d["fd_uv"][sm], ref["scale_uv"][sm], go[sm],
                   d["round_uv"][sm])
