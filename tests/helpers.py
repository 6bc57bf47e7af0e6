"""Shared helpers of the GPU parity tests: host copies for the oracle and the
acceptance rules (indices exact away from cell edges; forward within 1e-5;
backward within the 1e-4 relative criterion)."""
import numpy as np
import torch

import oracle

EDGE = 1e-6  # fragments closer than this (normalised) to a cell edge are excluded
FWD_TOL = 1e-5
BWD_REL = 1e-4


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def oracle_tex(tex_cpu, W, H, n, C, fmt=oracle.FMT_F32, scales=None):
    return oracle.Tex(tex_cpu, W, H, n, C, fmt, scales)


def gb_host(gb, sel=None):
    uv, tbn, view = host(gb.uv), host(gb.tbn), host(gb.view)
    if sel is not None:
        uv, tbn, view = uv[sel], tbn[sel], view[sel]
    return uv, tbn, view


def check_indices(idx_gpu, frac_gpu, uv, tbn, view, W, H, n):
    """Bit-exact (i, j, x0, y0) on fragments at least EDGE from every cell edge;
    returns the number of excluded fragments."""
    idx_o, frac_o, edge = oracle.indices(uv, tbn, view, W, H, n)
    keep = (edge[:, 0] >= EDGE) & (edge[:, 1] >= EDGE)
    bad = np.nonzero(np.any(idx_gpu[keep] != idx_o[keep], axis=1))[0]
    assert bad.size == 0, (bad[:5], idx_gpu[keep][bad[:5]], idx_o[keep][bad[:5]])
    assert np.all((idx_gpu[:, 0] >= 0) & (idx_gpu[:, 0] < W) & (idx_gpu[:, 1] >= 0)
                  & (idx_gpu[:, 1] < H) & (idx_gpu[:, 2] >= 0) & (idx_gpu[:, 2] < n)
                  & (idx_gpu[:, 3] >= 0) & (idx_gpu[:, 3] < n))
    np.testing.assert_allclose(frac_gpu[keep], frac_o[keep], atol=1e-5)
    return int((~keep).sum())


def bucket_edge_mask(uv, tbn, view, W, H, n):
    _, _, edge = oracle.indices(uv, tbn, view, W, H, n)
    return edge[:, 0] >= EDGE


def check_fwd(out_gpu, out_oracle, keep=None, tol=FWD_TOL):
    d = np.abs(out_gpu.astype(np.float64) - out_oracle)
    if keep is not None:
        d = d[keep]
    assert d.size == 0 or d.max() <= tol, (d.max(), np.unravel_index(np.argmax(d), d.shape))
    return float(d.max()) if d.size else 0.0


def away_from_edges(uv, tbn, view, W, H, n, mode="nearest"):
    """Fragments at least EDGE (normalised) from every cell edge that decides an
    index: bucket edges (nearest mode) or the edges of the bucket pair
    (bilinear-bucket mode), and sample edges with the clamp bounds included."""
    _, _, edge = oracle.indices(uv, tbn, view, W, H, n)
    keep = edge[:, 1] >= EDGE
    if mode == "nearest":
        keep &= edge[:, 0] >= EDGE
    else:
        u = uv.astype(np.float64)
        p = (u - np.floor(u)) * [W, H] - 0.5
        keep &= np.all(np.abs(p - np.round(p)) / [W, H] >= EDGE, axis=1)
    return keep


def weight_tol(n: int) -> float:
    """Absolute error of a binary32 bilinear weight: the sample coordinate
    s = (B + 1) n/2 - 1/2 lies in [0, n-1] and is reached through a few
    roundings of relative size 2^-24, so its error is a few ulp of n."""
    return 8.0 * max(n, 1) * 2.0 ** -24


def check_grad_tex(G_gpu, ref, n, rel=BWD_REL):
    """Per element |G - G*| <= rel * a* + weight_tol(n) * b*: a* = sum |w g| is
    the scale of the accumulated sum, b* = sum |g| over the taps that include
    the element bounds the effect of the rounding of the weights themselves.
    An element no tap includes must be exactly 0."""
    wtol = weight_tol(n)
    G = G_gpu.astype(np.float64)
    G_o, A_o, B_o = ref["grad_tex"], ref["abs_tex"], ref["absg_tex"]
    err = np.abs(G - G_o)
    untouched = B_o == 0
    assert np.all(G[untouched] == 0.0), "gradient written where no fragment contributes"
    bound = rel * A_o + wtol * B_o
    t = ~untouched
    ratio = err[t] / bound[t]
    assert ratio.size == 0 or ratio.max() <= 1.0, (ratio.max(), np.argmax(ratio))
    return float(ratio.max()) if ratio.size else 0.0


# The binary32 sample coordinate s lies in [0, n-1] and is formed by a few
# roundings of relative size 2^-24 of quantities up to n; ROUND_S(n) bounds
# how far it can sit from the exact one (checked against the oracle's
# fractions by the GPU tests), and the oracle's lookup_bwd_round gives how far
# the exact gradient moves when s moves that much.
def round_s(n: int) -> float:
    return 2.0 ** -21 * max(n, 1)


def round_w(W: int, H: int, uv) -> float:
    """Bound on the rounding of the bilinear-bucket fractions a = frac(u) W -
    1/2 in binary32: t = u W is exact for a power-of-two W and the split into
    floor and fraction is exact, leaving one rounding of r + 1/2 (2^-25);
    otherwise u W itself rounds, by up to 2^-24 |u W|."""
    pow2 = lambda x: x > 0 and (x & (x - 1)) == 0
    if pow2(W) and pow2(H):
        return 2.0 ** -24
    u = np.abs(np.asarray(uv, np.float64))
    m = max(1.0, W * float(u[:, 0].max()) if u.size else 0.0,
            H * float(u[:, 1].max()) if u.size else 0.0)
    return 2.0 ** -23 * m


def check_grad_vec(g_gpu, g_o, scale, go=None, rnd=None, rel=BWD_REL, absolute=1e-6):
    """Two bounds per fragment, both enforced:

    * |dg|_2 <= rel * |S|_2, S the oracle's chain rule evaluated with the
      magnitude of every factor (the scale of a binary32 evaluation's
      rounding); where S is 0 the gradient must be exactly 0;
    * with the upstream gradient go given: |dg|_2 <= rel * |g*|_2 +
      absolute * sum_c |go_c| + rnd, where rnd (default 0) is the oracle's
      change of the gradient under the rounding of the sample coordinate
      (lookup_bwd_round with round_s(n)).

    Returns a dict: the worst error / bound of each, the number of fragments
    that exceed rel |g*| + absolute sum |go| alone (those the rounding term
    admits), and the largest plain relative error over fragments whose
    gradient is not tiny."""
    g_gpu = g_gpu.astype(np.float64)
    d = np.linalg.norm(g_gpu - g_o, axis=1)
    sc = np.linalg.norm(scale, axis=1)
    zero = sc == 0
    assert np.all(d[zero] == 0.0), "non-zero gradient where the oracle's scale is 0"
    bound = rel * sc
    bad = np.nonzero((d > bound) & ~zero)[0]
    assert bad.size == 0, (bad[:5], d[bad[:5]], bound[bad[:5]], g_gpu[bad[:5]], g_o[bad[:5]])
    gn = np.linalg.norm(g_o, axis=1)
    big = gn > 1e-3 * (gn.max() if gn.size else 0)
    res = {"magnitude": float(np.max(d[~zero] / bound[~zero])) if np.any(~zero) else 0.0,
           "plain_rel": float(np.max(d[big] / gn[big])) if np.any(big) else 0.0,
           "relative": None, "needs_rounding_term": 0}
    if go is not None:
        base = rel * gn + absolute * np.abs(go.astype(np.float64)).sum(1)
        res["needs_rounding_term"] = int(np.sum(d > base))
        b2 = base + (0.0 if rnd is None else rnd)
        bad = np.nonzero(d > b2)[0]
        assert bad.size == 0, ("relative bound", bad[:5], d[bad[:5]], b2[bad[:5]], gn[bad[:5]])
        res["relative"] = float(np.max(d / np.maximum(b2, 1e-300))) if d.size else 0.0
    return res
