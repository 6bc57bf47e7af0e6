"""A model of the backward's binary32 evaluation (numpy float32 arithmetic,
one rounding per operation, no fused multiply-adds), used only to pin the
error scales of the oracle's backward criterion.

It follows the lookup's steps in binary32: u = M V, the equisolid projection
in the form A = (u_x, u_y) / sqrt(L (L + u_z)) (Eq. (1b)), the square map
(Eq. (3)), the clamped texel coordinate (the Note after Eq. (3)), the
bilinear taps, and then the chain back through them to dL/dview and, in the
bilinear-bucket mode, dL/duv."""
import numpy as np

f = np.float32


def model(T, W, H, n, C, uv, tbn, view, g, mode):
    """(grad_view [N,3], grad_uv [N,2]) as float64 arrays of binary32 values;
    T [H,W,n,n,C] float32, mode 0 nearest, 1 bilinear-bucket."""
    N = uv.shape[0]
    m = tbn.reshape(N, 9).astype(f)
    w = view.astype(f)
    ux = m[:, 0] * w[:, 0] + m[:, 1] * w[:, 1] + m[:, 2] * w[:, 2]
    uy = m[:, 3] * w[:, 0] + m[:, 4] * w[:, 1] + m[:, 5] * w[:, 2]
    uz = m[:, 6] * w[:, 0] + m[:, 7] * w[:, 1] + m[:, 8] * w[:, 2]
    L = np.sqrt(ux * ux + uy * uy + uz * uz)
    q = L * (L + uz)
    k = np.where(q > 0, f(1) / np.sqrt(np.where(q > 0, q, f(1))), f(0)).astype(f)
    ax, ay = ux * k, uy * k
    rho = np.sqrt(ax * ax + ay * ay)
    mx = np.maximum(np.abs(ax), np.abs(ay))
    r = np.where(mx > 0, rho / np.where(mx > 0, mx, f(1)), f(0)).astype(f)
    bx, by = ax * r, ay * r
    hn, top = f(0.5) * f(n), f(n - 1)
    sx = (bx + f(1)) * hn - f(0.5)
    sy = (by + f(1)) * hn - f(0.5)
    clx = ~((sx > 0) & (sx < top))
    cly = ~((sy > 0) & (sy < top))
    sx = np.minimum(np.maximum(sx, f(0)), top)
    sy = np.minimum(np.maximum(sy, f(0)), top)
    hi = max(n - 2, 0)
    x0 = np.minimum(sx.astype(np.int64), hi)
    y0 = np.minimum(sy.astype(np.int64), hi)
    x1 = np.minimum(x0 + 1, n - 1)
    y1 = np.minimum(y0 + 1, n - 1)
    fx = (sx - x0.astype(f)).astype(f)
    fy = (sy - y0.astype(f)).astype(f)
    u = uv.astype(np.float64)
    if mode == 0:
        i = (np.floor(u[:, 0] * W) % W).astype(np.int64)
        j = (np.floor(u[:, 1] * H) % H).astype(np.int64)
        bk = [(j, i)]
        wb = [np.ones(N, f)]
        a = bb = None
    else:
        def pair(x, Wd):
            t = (x.astype(f) * f(Wd)).astype(f)
            ft = np.floor(t)
            rr = (t - ft).astype(f)
            kk = ft.astype(np.int64)
            aa = np.where(rr >= 0.5, rr - f(0.5), rr + f(0.5)).astype(f)
            kk = np.where(rr >= 0.5, kk, kk - 1) % Wd
            return kk, (kk + 1) % Wd, aa
        i0, i1, a = pair(uv[:, 0], W)
        j0, j1, bb = pair(uv[:, 1], H)
        bk = [(j0, i0), (j0, i1), (j1, i0), (j1, i1)]
        wb = [(f(1) - a) * (f(1) - bb), a * (f(1) - bb), (f(1) - a) * bb, a * bb]
    gg = g.astype(f)
    gsx = np.zeros(N, f)
    gsy = np.zeros(N, f)
    taps = []
    for (jj, ii), wk in zip(bk, wb):
        T00 = T[jj, ii, y0, x0].astype(f)
        T01 = T[jj, ii, y0, x1].astype(f)
        T10 = T[jj, ii, y1, x0].astype(f)
        T11 = T[jj, ii, y1, x1].astype(f)
        taps.append((T00, T01, T10, T11))
        gx = np.zeros(N, f)
        gy = np.zeros(N, f)
        for c in range(C):
            gx = gx + gg[:, c] * ((f(1) - fy) * (T01[:, c] - T00[:, c]) + fy * (T11[:, c] - T10[:, c]))
            gy = gy + gg[:, c] * ((f(1) - fx) * (T10[:, c] - T00[:, c]) + fx * (T11[:, c] - T01[:, c]))
        gsx = gsx + wk * gx
        gsy = gsy + wk * gy
    gbx = np.where(clx, f(0), gsx * hn).astype(f)
    gby = np.where(cly, f(0), gsy * hn).astype(f)
    # square vjp
    rho = np.sqrt(ax * ax + ay * ay)
    safe = np.where(rho > 0, rho, f(1))
    xb = np.abs(ax) >= np.abs(ay)
    sgx = np.where(ax >= 0, f(1), f(-1))
    sgy = np.where(ay >= 0, f(1), f(-1))
    axs = np.where(ax != 0, ax, f(1))
    ays = np.where(ay != 0, ay, f(1))
    j00 = np.abs(ax) / safe
    j01 = sgx * ay / safe
    j10 = -sgx * ay * ay * ay / (safe * axs * axs)
    j11 = (ay * ay + safe * safe) / (safe * np.abs(axs))
    gax1 = j00 * gbx + j10 * gby
    gay1 = j01 * gbx + j11 * gby
    k11 = np.abs(ay) / safe
    k10 = sgy * ax / safe
    k01 = -sgy * ax * ax * ax / (safe * ays * ays)
    k00 = (ax * ax + safe * safe) / (safe * np.abs(ays))
    gax2 = k00 * gbx + k10 * gby
    gay2 = k01 * gbx + k11 * gby
    gax = np.where(rho > 0, np.where(xb, gax1, gax2), gbx).astype(f)
    gay = np.where(rho > 0, np.where(xb, gay1, gay2), gby).astype(f)
    ok = (k > 0) & (L > 0)
    sdot = ux * gax + uy * gay
    coef = f(-0.5) * k * k * k * sdot
    Ls = np.where(L > 0, L, f(1))
    t2 = (f(2) * L + uz) / Ls
    gux = np.where(ok, k * gax + coef * ux * t2, f(0))
    guy = np.where(ok, k * gay + coef * uy * t2, f(0))
    guz = np.where(ok, coef * (uz * t2 + L), f(0))
    gv = np.stack([m[:, 0] * gux + m[:, 3] * guy + m[:, 6] * guz,
                   m[:, 1] * gux + m[:, 4] * guy + m[:, 7] * guz,
                   m[:, 2] * gux + m[:, 5] * guy + m[:, 8] * guz], 1)
    guv = np.zeros((N, 2), f)
    if mode == 1:
        wq = [(f(1) - fx) * (f(1) - fy), fx * (f(1) - fy), (f(1) - fx) * fy, fx * fy]
        su = np.zeros(N, f)
        sv = np.zeros(N, f)
        for c in range(C):
            du = np.zeros(N, f)
            dv = np.zeros(N, f)
            for qq in range(4):
                Tk = [taps[kk][qq][:, c] for kk in range(4)]
                du = du + wq[qq] * ((f(1) - bb) * (Tk[1] - Tk[0]) + bb * (Tk[3] - Tk[2]))
                dv = dv + wq[qq] * ((f(1) - a) * (Tk[2] - Tk[0]) + a * (Tk[3] - Tk[1]))
            su = su + gg[:, c] * du
            sv = sv + gg[:, c] * dv
        guv = np.stack([f(W) * su, f(H) * sv], 1)
    return gv.astype(np.float64), guv.astype(np.float64)
