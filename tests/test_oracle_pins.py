"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check is a closed form
stated in the paper, a second formulation the paper gives, a brute-force
search, an invariant of the method, a hand-derived worked example
(tests/golden/worked_examples.txt), or an independent library routine.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.txt")


def _rand_dirs(rng, k, zmin=0.0):
    """Uniform directions on the cap z >= zmin (uniform in z and azimuth)."""
    z = rng.uniform(zmin, 1.0, k)
    phi = rng.uniform(0, 2 * np.pi, k)
    r = np.sqrt(1 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)


def _rand_rot(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


# --------------------------------------------------------------------------
# Eq. (1a)/(1b): equisolid projection
# --------------------------------------------------------------------------

def test_equisolid_radius_closed_form():
    # Sec. 2.1: the projected radius equals sqrt(2) sin(theta/2)
    rng = np.random.default_rng(0)
    I = _rand_dirs(rng, 2000, zmin=-0.999)
    A = oracle.equisolid_tangent(I)
    theta = np.arccos(np.clip(I[:, 2], -1, 1))
    np.testing.assert_allclose(np.linalg.norm(A, axis=1), np.sqrt(2) * np.sin(theta / 2),
                               atol=1e-14)
    # the azimuth is kept: A is parallel to (I_x, I_y)
    cross = A[:, 0] * I[:, 1] - A[:, 1] * I[:, 0]
    assert np.max(np.abs(cross)) < 1e-14
    assert np.all(A[:, 0] * I[:, 0] + A[:, 1] * I[:, 1] >= 0)


def test_equisolid_rim_and_pole():
    # Eq. (1): r = 1 at Omega = 180 deg, i.e. the horizon maps to |A| = 1
    phi = np.linspace(0, 2 * np.pi, 37)
    I = np.stack([np.cos(phi), np.sin(phi), np.zeros_like(phi)], 1)
    A = oracle.equisolid_tangent(I)
    np.testing.assert_allclose(np.linalg.norm(A, axis=1), 1.0, atol=1e-15)
    assert np.all(oracle.equisolid_tangent([0, 0, 1.0]) == 0.0)


def test_equisolid_preserves_area():
    # Sec. 2.1: the projection preserves area, so for directions uniform on
    # the hemisphere |A|^2 (= 1 - cos theta) is uniform on [0, 1].
    from scipy import stats
    rng = np.random.default_rng(1)
    I = _rand_dirs(rng, 20000, zmin=0.0)
    A = oracle.equisolid_tangent(I)
    r2 = np.sum(A * A, axis=1)
    assert stats.kstest(r2, "uniform").pvalue > 1e-3
    # and areas scale by one constant: a cap of half-angle t (solid angle
    # 2 pi (1 - cos t)) maps to a disc of area pi |A|^2 = half that solid
    # angle, for every t (the hemisphere's 2 pi onto the unit disc's pi)
    for t in np.radians([5.0, 30.0, 60.0, 89.0]):
        rad = np.linalg.norm(oracle.equisolid_tangent([np.sin(t), 0, np.cos(t)]))
        assert abs(np.pi * rad ** 2 - 0.5 * 2 * np.pi * (1 - np.cos(t))) < 1e-14


def test_general_normal_form_matches_tangent_form():
    # Eq. (1a) for an arbitrary unit normal N, expressed in a frame (T, B, N),
    # equals Eq. (1b) applied to the incidence moved into that frame.
    rng = np.random.default_rng(2)
    for _ in range(300):
        R = _rand_rot(rng)  # rows T, B, N
        It = _rand_dirs(rng, 1, zmin=-0.9)[0]
        Iw = R.T @ It
        g = oracle.equisolid_general(Iw, R[2])[0]
        A_general = np.array([R[0] @ g, R[1] @ g])
        A_tangent = oracle.equisolid_tangent(It)[0]
        np.testing.assert_allclose(A_general, A_tangent, atol=1e-14)
        # third component of Eq. (1a): sqrt(2) cos(theta/2)
        theta = np.arccos(np.clip(It[2], -1, 1))
        assert abs(R[2] @ g - np.sqrt(2) * np.cos(theta / 2)) < 1e-14


def test_inverse_equisolid_round_trip():
    # Eq. (2c) inverts Eq. (1b) on the whole sphere except -N
    rng = np.random.default_rng(3)
    I = _rand_dirs(rng, 3000, zmin=-0.99)
    A = oracle.equisolid_tangent(I)
    I2 = oracle.inverse_equisolid_tangent(A)
    np.testing.assert_allclose(I2, I, atol=1e-13)
    A2 = rng.uniform(-1, 1, (3000, 2)) * 0.7
    np.testing.assert_allclose(oracle.equisolid_tangent(oracle.inverse_equisolid_tangent(A2)),
                               A2, atol=1e-14)


def test_inverse_general_reduces_to_tangent_form():
    # Eq. (2b) with N = e_z is Eq. (2c)
    rng = np.random.default_rng(4)
    A = rng.uniform(-1, 1, (500, 2)) * 0.7
    Ig = oracle.inverse_equisolid_general(A, np.tile([0.0, 0.0, 1.0], (500, 1)))
    It = oracle.inverse_equisolid_tangent(A)
    np.testing.assert_allclose(Ig, It, atol=1e-14)
    # Eq. (2b) is a reflection: |I| = 1 and I + N is parallel to the half vector
    np.testing.assert_allclose(np.linalg.norm(Ig, axis=1), 1.0, atol=1e-14)


def test_reflection_vector_is_mirror_of_incidence():
    # Eq. (4b): R is the incidence of Eq. (2c) mirrored about the normal
    rng = np.random.default_rng(5)
    A = rng.uniform(-1, 1, (500, 2)) * 0.7
    R = oracle.reflection(A)
    I = oracle.inverse_equisolid_tangent(A)
    np.testing.assert_allclose(R, np.stack([-I[:, 0], -I[:, 1], I[:, 2]], 1), atol=1e-15)
    # and it is the reflection of -I about N = e_z: R = 2 (N . I) N - I ... with
    # the tangential part flipped: R . N = I . N, R_t = -I_t
    np.testing.assert_allclose(R[:, 2], I[:, 2], atol=1e-15)


# --------------------------------------------------------------------------
# Eq. (3)/(4a): disc <-> square
# --------------------------------------------------------------------------

def test_square_map_properties():
    rng = np.random.default_rng(6)
    A = rng.uniform(-1, 1, (5000, 2))
    A = A[np.linalg.norm(A, axis=1) <= 1]
    B = oracle.square(A)
    # |B|_inf = |A|_2 (the disc of radius r goes to the square of half-side r)
    np.testing.assert_allclose(np.max(np.abs(B), axis=1), np.linalg.norm(A, axis=1), atol=1e-15)
    # direction kept
    assert np.max(np.abs(A[:, 0] * B[:, 1] - A[:, 1] * B[:, 0])) < 1e-15
    # Eq. (4a) inverts it, both ways
    np.testing.assert_allclose(oracle.unsquare(B), A, atol=1e-15)
    S = rng.uniform(-1, 1, (3000, 2))
    np.testing.assert_allclose(oracle.square(oracle.unsquare(S)), S, atol=1e-15)
    # on the axes the map is the identity; the unit disc fills [-1,1]^2
    ax = np.array([[0.3, 0.0], [0.0, -0.8], [-1.0, 0.0]])
    np.testing.assert_allclose(oracle.square(ax), ax, atol=0)
    assert np.all(oracle.square([0.0, 0.0]) == 0.0)
    d = 1 / np.sqrt(2)
    np.testing.assert_allclose(oracle.square([d, d])[0], [1.0, 1.0], atol=1e-15)


def test_square_map_d4_equivariance():
    rng = np.random.default_rng(7)
    A = rng.uniform(-1, 1, (1000, 2))
    B = oracle.square(A)
    np.testing.assert_allclose(oracle.square(A[:, ::-1]), B[:, ::-1], atol=1e-15)
    np.testing.assert_allclose(oracle.square(A * [-1, 1]), B * [-1, 1], atol=1e-15)
    np.testing.assert_allclose(oracle.square(A * [1, -1]), B * [1, -1], atol=1e-15)


# --------------------------------------------------------------------------
# bucket-edge clamp and texel coordinate
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 4, 8, 16])
def test_clamp_maps_to_outer_texel_centres(n):
    # The Note after Eq. (3): B clamped to [1/n - 1, 1 - 1/n]; the texel
    # centre reading turns that range into exactly [0, n - 1].
    lo, hi = 1.0 / n - 1.0, 1.0 - 1.0 / n
    s = oracle.texel_coord([[lo, hi], [-1.0, 1.0], [-5.0, 7.0], [0.0, 0.0]], n)
    np.testing.assert_allclose(s[0], [0.0, n - 1.0], atol=1e-12)
    assert np.all(s[1] == [0.0, n - 1.0]) and np.all(s[2] == [0.0, n - 1.0])
    np.testing.assert_allclose(s[3], [(n - 1) / 2.0] * 2, atol=1e-15)
    # sample k's centre in B-space is (2k + 1)/n - 1
    k = np.arange(n)
    Bc = (2 * k + 1.0) / n - 1.0
    sc = oracle.texel_coord(np.stack([Bc, Bc[::-1]], 1), n)
    np.testing.assert_allclose(sc[:, 0], k, atol=1e-12)
    np.testing.assert_allclose(sc[:, 1], k[::-1], atol=1e-12)


def test_worked_examples():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 7
    for r in rows:
        name, n = r[0], int(r[1])
        V = np.array([float(x) for x in r[2:5]])
        exp = np.array([float(x) for x in r[5:11]])
        x0, y0 = int(r[11]), int(r[12])
        fx, fy = float(r[13]), float(r[14])
        got = oracle.map_one(np.eye(3), V, n)
        np.testing.assert_allclose(got, exp, atol=2e-14, err_msg=name)
        uv = np.array([[0.5, 0.5]], np.float32)
        idx, frac, _ = oracle.indices(uv, np.eye(3, dtype=np.float32)[None],
                                      V.astype(np.float32)[None], 4, 4, n)
        assert (idx[0, 2], idx[0, 3]) == (x0, y0), name
        np.testing.assert_allclose(frac[0], [fx, fy], atol=1e-6, err_msg=name)


def test_brute_force_inverse_search():
    # For a direction I, search a fine grid of bucket coordinates B for the one
    # whose inverse-mapped direction (Eq. 4a then Eq. 2c) is closest to I; it
    # must be the B the forward chain (Eq. 1b then Eq. 3) produces.
    rng = np.random.default_rng(8)
    g = np.linspace(-1, 1, 801)
    GX, GY = np.meshgrid(g, g, indexing="xy")
    Bgrid = np.stack([GX.ravel(), GY.ravel()], 1)
    # vectorised inverse (restated only for the grid search)
    rho = np.linalg.norm(Bgrid, axis=1)
    m = np.max(np.abs(Bgrid), axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        Agrid = np.where(rho[:, None] > 0, Bgrid * (m / rho)[:, None], 0.0)
    r2 = np.sum(Agrid ** 2, 1)
    w = np.sqrt(np.maximum(0, 2 - r2))
    Igrid = np.stack([Agrid[:, 0] * w, Agrid[:, 1] * w, 1 - r2], 1)
    # spot check the vectorised inverse against the oracle's Eqs. (4a)/(2c)
    pick = rng.integers(0, len(Bgrid), 50)
    np.testing.assert_allclose(
        oracle.inverse_equisolid_tangent(oracle.unsquare(Bgrid[pick])), Igrid[pick], atol=1e-14)
    for I in _rand_dirs(rng, 40, zmin=0.05):
        B = oracle.square(oracle.equisolid_tangent(I))[0]
        k = np.argmax(Igrid @ I)
        assert np.max(np.abs(Bgrid[k] - B)) <= 2.5 / 800 + 1e-12


# --------------------------------------------------------------------------
# whole lookup: bucket selection, bilinear fetch, invariants
# --------------------------------------------------------------------------

def _tex(rng, W, H, n, C):
    return rng.uniform(0, 1, (H, W, n, n, C)).astype(np.float32)


def test_bucket_index_brute_force():
    # Sec. 2: u,v index the bucket matrix; the bucket of a coordinate is the
    # cell interval [i/W, (i+1)/W) containing frac(u) (UV wrap).
    rng = np.random.default_rng(9)
    for W in (1, 3, 5, 7, 64):
        u = rng.uniform(-3, 3, 4000).astype(np.float32)
        v = rng.uniform(-3, 3, 4000).astype(np.float32)
        uv = np.stack([u, v], 1)
        N = len(u)
        idx, _, edge = oracle.indices(uv, np.tile(np.eye(3, dtype=np.float32), (N, 1, 1)),
                                      np.tile(np.float32([0, 0, 1]), (N, 1)), W, W, 4)
        fu = np.float64(u) - np.floor(np.float64(u))
        for k in range(N):
            cells = [i for i in range(W) if i / W <= fu[k] < (i + 1) / W]
            assert idx[k, 0] == cells[0]
        assert np.all((idx[:, :2] >= 0) & (idx[:, :2] < W))


def test_bilinear_equals_tent_filter_brute_force():
    # out = sum over all n^2 samples of tent(s_x - x) tent(s_y - y) T[y, x],
    # an independent form of the bilinear fetch inside the bucket.
    rng = np.random.default_rng(10)
    W = H = 3
    for n in (2, 3, 5, 8):
        C = 2
        T = _tex(rng, W, H, n, C)
        tex = oracle.Tex(T, W, H, n, C)
        N = 300
        uv = rng.uniform(0, 1, (N, 2)).astype(np.float32)
        V = _rand_dirs(rng, N, zmin=-0.3).astype(np.float32)
        tbn = np.tile(np.eye(3, dtype=np.float32), (N, 1, 1))
        out = oracle.lookup_fwd(tex, uv, tbn, V)
        idx, _, _ = oracle.indices(uv, tbn, V, W, H, n)
        for f in range(N):
            s = oracle.map_one(np.eye(3), V[f].astype(np.float64), n)[4:6]
            xs = np.arange(n)
            wx = np.maximum(0, 1 - np.abs(s[0] - xs))
            wy = np.maximum(0, 1 - np.abs(s[1] - xs))
            bucket = T[idx[f, 1], idx[f, 0]].astype(np.float64)  # [n(y), n(x), C]
            ref = np.einsum("y,x,yxc->c", wy, wx, bucket)
            np.testing.assert_allclose(out[f], ref, atol=1e-14)


def test_lookup_invariants():
    rng = np.random.default_rng(11)
    W, H, n, C = 4, 3, 8, 3
    T = _tex(rng, W, H, n, C)
    tex = oracle.Tex(T, W, H, n, C)
    N = 500
    uv = rng.uniform(-2, 2, (N, 2)).astype(np.float32)
    V = _rand_dirs(rng, N, zmin=0.0).astype(np.float32)
    eye = np.tile(np.eye(3, dtype=np.float32), (N, 1, 1))
    out = oracle.lookup_fwd(tex, uv, eye, V)
    idx, _, _ = oracle.indices(uv, eye, V, W, H, n)
    # normal incidence -> mean of the four centre samples (even n)
    Vn = np.tile(np.float32([0, 0, 1]), (N, 1))
    on = oracle.lookup_fwd(tex, uv, eye, Vn)
    c = n // 2
    for f in range(0, N, 37):
        b = T[idx[f, 1], idx[f, 0]].astype(np.float64)
        np.testing.assert_allclose(on[f], b[c - 1:c + 1, c - 1:c + 1].mean(axis=(0, 1)),
                                   atol=1e-15)
    # constant texture -> constant image
    oc = oracle.lookup_fwd(oracle.Tex(np.full_like(T, 0.375), W, H, n, C), uv, eye, V)
    assert np.all(oc == 0.375)
    # output inside the convex hull of its bucket
    for f in range(N):
        b = T[idx[f, 1], idx[f, 0]].reshape(-1, C)
        assert np.all(out[f] >= b.min(0) - 1e-15) and np.all(out[f] <= b.max(0) + 1e-15)
    # changing every other bucket leaves the output unchanged (no cross-bucket
    # blending, the Note after Eq. (3))
    for f in range(0, N, 50):
        T2 = _tex(rng, W, H, n, C)
        T2[idx[f, 1], idx[f, 0]] = T[idx[f, 1], idx[f, 0]]
        o2 = oracle.lookup_fwd(oracle.Tex(T2, W, H, n, C), uv[f:f + 1], eye[:1], V[f:f + 1])
        np.testing.assert_array_equal(o2[0], out[f])
    # the same lookup with a rotated world: rotating V and the frame together
    R = _rand_rot(rng).astype(np.float64)
    Mrot = np.tile((np.eye(3) @ R.T).astype(np.float32), (N, 1, 1))
    Vrot = (V.astype(np.float64) @ R.T).astype(np.float32)
    orot = oracle.lookup_fwd(tex, uv, Mrot, Vrot)
    assert np.max(np.abs(orot - out)) < 5e-6  # float32 storage of the rotated inputs
    # scale invariance: the view need not be unit (a power of two keeps the
    # float32 direction exact)
    np.testing.assert_allclose(oracle.lookup_fwd(tex, uv, eye, V * 4.0), out, atol=1e-12)
    np.testing.assert_allclose(oracle.lookup_fwd(tex, uv, eye, V * 0.125), out, atol=1e-12)


def test_lookup_mirror_symmetry():
    # mirroring the view in x and the texture inside every bucket in x gives
    # the same output (and likewise y, and the transpose x <-> y)
    rng = np.random.default_rng(12)
    W, H, n, C = 2, 2, 8, 2
    T = _tex(rng, W, H, n, C)
    N = 400
    uv = rng.uniform(0, 1, (N, 2)).astype(np.float32)
    V = _rand_dirs(rng, N, zmin=0.0).astype(np.float32)
    eye = np.tile(np.eye(3, dtype=np.float32), (N, 1, 1))
    out = oracle.lookup_fwd(oracle.Tex(T, W, H, n, C), uv, eye, V)
    Tx = np.ascontiguousarray(T[:, :, :, ::-1, :])
    ox = oracle.lookup_fwd(oracle.Tex(Tx, W, H, n, C), uv, eye, V * np.float32([-1, 1, 1]))
    np.testing.assert_allclose(ox, out, atol=1e-12)
    Ty = np.ascontiguousarray(T[:, :, ::-1, :, :])
    oy = oracle.lookup_fwd(oracle.Tex(Ty, W, H, n, C), uv, eye, V * np.float32([1, -1, 1]))
    np.testing.assert_allclose(oy, out, atol=1e-12)
    Tt = np.ascontiguousarray(np.swapaxes(T, 2, 3))
    ot = oracle.lookup_fwd(oracle.Tex(Tt, W, H, n, C), uv, eye,
                           np.ascontiguousarray(V[:, [1, 0, 2]]))
    np.testing.assert_allclose(ot, out, atol=1e-12)


def test_bilinear_bucket_mode_reduces_to_nearest_at_centres():
    # bilinear-bucket mode sampled at bucket centres equals nearest mode, and
    # is a convex combination of the four neighbouring buckets otherwise
    rng = np.random.default_rng(13)
    W, H, n, C = 4, 8, 4, 3  # powers of two: bucket centres are exact in float32
    T = _tex(rng, W, H, n, C)
    tex = oracle.Tex(T, W, H, n, C)
    N = 60
    ij = np.stack([rng.integers(0, W, N), rng.integers(0, H, N)], 1)
    uv = ((ij + 0.5) / [W, H]).astype(np.float32)
    V = _rand_dirs(rng, N, 0.1).astype(np.float32)
    eye = np.tile(np.eye(3, dtype=np.float32), (N, 1, 1))
    a = oracle.lookup_fwd(tex, uv, eye, V, mode=oracle.MODE_NEAREST)
    b = oracle.lookup_fwd(tex, uv, eye, V, mode=oracle.MODE_BILINEAR)
    np.testing.assert_allclose(a, b, atol=1e-12)
    # halfway between columns i and i+1 (wrapping): average of the two
    uvh = ((ij + [1.0, 0.5]) / [W, H]).astype(np.float32)
    bh = oracle.lookup_fwd(tex, uvh, eye, V, mode=oracle.MODE_BILINEAR)
    nb0 = oracle.lookup_fwd(tex, ((ij + [0.5, 0.5]) / [W, H]).astype(np.float32), eye, V)
    ij1 = ij.copy()
    ij1[:, 0] = (ij1[:, 0] + 1) % W
    nb1 = oracle.lookup_fwd(tex, ((ij1 + [0.5, 0.5]) / [W, H]).astype(np.float32), eye, V)
    np.testing.assert_allclose(bh, 0.5 * (nb0 + nb1), atol=1e-6)


# --------------------------------------------------------------------------
# storage formats and the quantiser
# --------------------------------------------------------------------------

def test_e4m3_decode_matches_torch():
    codes = torch.arange(256, dtype=torch.uint8)
    ref = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    mine = np.array([oracle.e4m3_to_f64(c) for c in range(256)])
    finite = np.isfinite(ref)
    assert np.array_equal(np.isnan(mine), ~finite)
    np.testing.assert_array_equal(mine[finite], ref[finite])
    assert oracle.e4m3_to_f64(0x7E) == 448.0 and oracle.e4m3_to_f64(0x01) == 2.0 ** -9


def _e4m3_test_values():
    # every representable value, every midpoint, and one ulp either side
    vals = np.array([oracle.e4m3_to_f64(c) for c in range(0x7F)], np.float64)
    mids = (vals[:-1] + vals[1:]) / 2
    m32 = mids.astype(np.float32)
    pts = np.concatenate([vals.astype(np.float32), m32, np.nextafter(m32, np.float32(0)),
                          np.nextafter(m32, np.float32(1e9))])
    rng = np.random.default_rng(14)
    pts = np.concatenate([pts, rng.uniform(0, 448, 20000).astype(np.float32),
                          np.exp2(rng.uniform(-14, 8.8, 20000)).astype(np.float32)])
    pts = pts[pts <= 448]
    return np.concatenate([pts, -pts]).astype(np.float32)


def test_e4m3_encode_matches_torch():
    # torch's float8_e4m3fn conversion (round to nearest even) is an
    # independent implementation; inside the finite range the two agree
    x = _e4m3_test_values()
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    lib = oracle._load()
    mine = np.array([lib.orc_f32_to_e4m3_sat(float(v)) for v in x], np.uint8)
    np.testing.assert_array_equal(mine, ref)
    # saturation: beyond 448 (and infinity) the code is +-448, NaN stays NaN
    for v, c in ((449.0, 0x7E), (1e30, 0x7E), (float("inf"), 0x7E), (-500.0, 0xFE)):
        assert oracle.f32_to_e4m3(v) == c
    assert oracle.f32_to_e4m3(float("nan")) & 0x7F == 0x7F


def test_bf16_encode_matches_torch():
    rng = np.random.default_rng(15)
    bits = rng.integers(0, 2 ** 32, 200000, dtype=np.uint64).astype(np.uint32)
    # halfway cases and their neighbours
    half = (rng.integers(0, 2 ** 16, 20000, dtype=np.uint64).astype(np.uint32) << 16) | 0x8000
    bits = np.concatenate([bits, half, half + 1, half - 1])
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    lib = oracle._load()
    mine = np.array([lib.orc_f32_to_bf16_rne(float(v)) for v in x], np.uint16)
    np.testing.assert_array_equal(mine, ref)


def test_quantize_per_bucket_scale():
    rng = np.random.default_rng(16)
    nb, be = 50, 64
    T = (rng.uniform(-1, 1, (nb, be)) * np.exp2(rng.uniform(-12, 6, (nb, 1)))).astype(np.float32)
    T[3] = 0.0  # all-zero bucket: scale 1, codes 0
    codes, scales = oracle.quantize(T, nb, be, oracle.FMT_FP8_E4M3)
    codes = codes.reshape(nb, be)
    amax = np.max(np.abs(T), axis=1)
    for b in range(nb):
        if amax[b] == 0:
            assert scales[b] == 1.0 and np.all(codes[b] == 0)
            continue
        assert scales[b] == np.float32(amax[b]) / np.float32(448.0)
        # the largest magnitude goes to the largest code
        assert np.max(codes[b] & 0x7F) == 0x7E
        dec = np.array([oracle.e4m3_to_f64(c) for c in codes[b]]) * np.float64(scales[b])
        # relative error of E4M3 in the normal range is at most 2^-4; the
        # absolute error below the normal range at most half a subnormal step
        err = np.abs(dec - T[b])
        bound = np.maximum(np.abs(T[b]) * 2.0 ** -4, 2.0 ** -10 * scales[b]) * 1.0001
        assert np.all(err <= bound)
    c16, s16 = oracle.quantize(T, nb, be, oracle.FMT_BF16)
    assert s16 is None
    ref = torch.from_numpy(T.reshape(-1)).to(torch.bfloat16).view(torch.int16).numpy()
    np.testing.assert_array_equal(c16, ref.view(np.uint16))


def test_quantized_lookup_decodes_exactly():
    # the oracle's BF16/FP8 lookup equals its FP32 lookup on the decoded texture
    rng = np.random.default_rng(17)
    W, H, n, C = 3, 3, 8, 4
    T = _tex(rng, W, H, n, C)
    N = 200
    uv = rng.uniform(0, 1, (N, 2)).astype(np.float32)
    V = _rand_dirs(rng, N, 0.05).astype(np.float32)
    eye = np.tile(np.eye(3, dtype=np.float32), (N, 1, 1))
    codes, scales = oracle.quantize(T, W * H, n * n * C, oracle.FMT_FP8_E4M3)
    dec = (np.array([oracle.e4m3_to_f64(c) for c in range(256)])[codes].reshape(W * H, -1)
           * scales[:, None].astype(np.float64))
    o8 = oracle.lookup_fwd(oracle.Tex(codes, W, H, n, C, oracle.FMT_FP8_E4M3, scales), uv, eye, V)
    o64 = oracle.lookup_fwd(oracle.Tex(dec.reshape(-1), W, H, n, C, oracle.FMT_F64), uv, eye, V)
    np.testing.assert_allclose(o8, o64, atol=1e-15)
    c16, _ = oracle.quantize(T, W * H, n * n * C, oracle.FMT_BF16)
    d16 = torch.from_numpy(c16.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    o16 = oracle.lookup_fwd(oracle.Tex(c16, W, H, n, C, oracle.FMT_BF16), uv, eye, V)
    o64b = oracle.lookup_fwd(oracle.Tex(d16, W, H, n, C, oracle.FMT_F64), uv, eye, V)
    np.testing.assert_allclose(o16, o64b, atol=1e-15)


# --------------------------------------------------------------------------
# backward: finite differences and exact identities
# --------------------------------------------------------------------------

def _away_from_kinks(tbn, V, n, margin=2e-3):
    """True when the direction is away from every non-smooth point of the
    lookup: texel lines, clamp bounds, the diagonal |A_x| = |A_y|, A = 0."""
    a = oracle.map_one(tbn, V, n)
    A, B = a[0:2], a[2:4]
    su = (B + 1) * n / 2 - 0.5
    if np.any(np.abs(su - np.round(su)) < margin * n) and True:
        return False
    if abs(abs(A[0]) - abs(A[1])) < margin or np.linalg.norm(A) < margin:
        return False
    return True


def _fd_setup(seed, mode, W=4, H=4, n=8, C=3, N=60):
    rng = np.random.default_rng(seed)
    T = _tex(rng, W, H, n, C)
    tex = oracle.Tex(T, W, H, n, C)
    uv = rng.uniform(-1, 2, (N, 2)).astype(np.float32)
    Vs, Ms = [], []
    while len(Vs) < N:
        R = _rand_rot(rng) if rng.uniform() < 0.5 else np.eye(3)
        Vt = _rand_dirs(rng, 1, zmin=0.02)[0] * rng.uniform(0.5, 2.0)
        M = R.astype(np.float32).astype(np.float64)
        V = (R.T @ Vt).astype(np.float32).astype(np.float64)
        if _away_from_kinks(M.reshape(9), V, n):
            Vs.append(V)
            Ms.append(M)
    return rng, tex, uv, np.array(Ms, np.float32), np.array(Vs, np.float32)


@pytest.mark.parametrize("mode", [oracle.MODE_NEAREST, oracle.MODE_BILINEAR])
def test_grad_view_finite_differences(mode):
    rng, tex, uv, tbn, V = _fd_setup(20 + mode, mode)
    N = len(V)
    g = rng.normal(size=(N, tex.C)).astype(np.float32)
    res = oracle.lookup_bwd(tex, uv, tbn, V, g, mode=mode)
    h = 1e-6
    for f in range(N):
        U = uv[f].astype(np.float64)
        M = tbn[f].astype(np.float64)
        fd = np.zeros(3)
        for k in range(3):
            Vp = V[f].astype(np.float64).copy()
            Vm = Vp.copy()
            Vp[k] += h
            Vm[k] -= h
            op = oracle.lookup_one_f64(tex, U, M, Vp, mode)
            om = oracle.lookup_one_f64(tex, U, M, Vm, mode)
            fd[k] = np.dot(g[f].astype(np.float64), (op - om) / (2 * h))
        gv = res["grad_view"][f]
        assert np.linalg.norm(gv - fd) <= 1e-6 * max(1.0, np.linalg.norm(fd)), (f, gv, fd)
        # the lookup depends on the direction of V only
        assert abs(np.dot(gv, V[f])) <= 1e-9 * max(1.0, np.linalg.norm(gv) * np.linalg.norm(V[f]))


def test_grad_uv_finite_differences_bilinear_bucket_mode():
    rng, tex, uv, tbn, V = _fd_setup(30, oracle.MODE_BILINEAR)
    N = len(V)
    g = rng.normal(size=(N, tex.C)).astype(np.float32)
    res = oracle.lookup_bwd(tex, uv, tbn, V, g, mode=oracle.MODE_BILINEAR)
    h = 1e-7
    checked = 0
    for f in range(N):
        U = uv[f].astype(np.float64)
        p = (U - np.floor(U)) * [tex.W, tex.H] - 0.5
        if np.any(np.abs(p - np.round(p)) < 1e-3):
            continue
        fd = np.zeros(2)
        for k in range(2):
            Up, Um = U.copy(), U.copy()
            Up[k] += h
            Um[k] -= h
            op = oracle.lookup_one_f64(tex, Up, tbn[f], V[f], oracle.MODE_BILINEAR)
            om = oracle.lookup_one_f64(tex, Um, tbn[f], V[f], oracle.MODE_BILINEAR)
            fd[k] = np.dot(g[f].astype(np.float64), (op - om) / (2 * h))
        np.testing.assert_allclose(res["grad_uv"][f], fd, rtol=1e-6, atol=1e-6)
        checked += 1
    assert checked > N // 2
    # nearest mode: piecewise constant in u, v
    res0 = oracle.lookup_bwd(tex, uv, tbn, V, g, mode=oracle.MODE_NEAREST)
    assert np.all(res0["grad_uv"] == 0.0)


@pytest.mark.parametrize("mode", [oracle.MODE_NEAREST, oracle.MODE_BILINEAR])
def test_grad_tex_adjoint_and_conservation(mode):
    # the lookup is linear in the texture, so <grad_tex, T> = <g, out> and a
    # finite difference in one texel is exact up to rounding; every fragment's
    # weights sum to one, so sum over texels of grad_tex = sum of g.
    rng = np.random.default_rng(40 + mode)
    W, H, n, C = 5, 4, 8, 3
    T = _tex(rng, W, H, n, C)
    tex = oracle.Tex(T, W, H, n, C)
    N = 3000
    uv = rng.uniform(-1, 2, (N, 2)).astype(np.float32)
    V = _rand_dirs(rng, N, zmin=-0.2).astype(np.float32)
    tbn = np.tile(np.eye(3, dtype=np.float32), (N, 1, 1))
    g = rng.normal(size=(N, C)).astype(np.float32)
    out = oracle.lookup_fwd(tex, uv, tbn, V, mode=mode)
    res = oracle.lookup_bwd(tex, uv, tbn, V, g, mode=mode)
    G = res["grad_tex"]
    lhs = np.sum(G * T.astype(np.float64))
    rhs = np.sum(g.astype(np.float64) * out)
    assert abs(lhs - rhs) <= 1e-11 * np.sum(np.abs(g) * np.abs(out))
    np.testing.assert_allclose(G.sum(axis=(0, 1, 2, 3)), g.astype(np.float64).sum(0), atol=1e-10)
    assert np.all(res["abs_tex"] >= np.abs(G) - 1e-15)
    if mode == oracle.MODE_NEAREST:
        idx, _, _ = oracle.indices(uv, tbn, V, W, H, n)
        for b in [(0, 0), (2, 3), (4, 1)]:
            sel = (idx[:, 0] == b[0]) & (idx[:, 1] == b[1])
            np.testing.assert_allclose(G[b[1], b[0]].sum(axis=(0, 1)),
                                       g[sel].astype(np.float64).sum(0), atol=1e-11)
    # finite difference in single texels (float64 texture)
    T64 = T.astype(np.float64)
    for _ in range(5):
        j, i, y, x, c = (rng.integers(0, s) for s in (H, W, n, n, C))
        Tp = T64.copy()
        Tp[j, i, y, x, c] += 0.5
        op = oracle.lookup_fwd(oracle.Tex(Tp, W, H, n, C, oracle.FMT_F64), uv, tbn, V, mode=mode)
        fd = np.sum(g.astype(np.float64) * (op - out)) / 0.5
        assert abs(fd - G[j, i, y, x, c]) <= 1e-9 * max(1.0, abs(fd))


def test_grad_tex_window_matches_full():
    rng = np.random.default_rng(50)
    W, H, n, C = 6, 5, 4, 2
    T = _tex(rng, W, H, n, C)
    tex = oracle.Tex(T, W, H, n, C)
    N = 800
    uv = rng.uniform(0, 1, (N, 2)).astype(np.float32)
    V = _rand_dirs(rng, N, 0.0).astype(np.float32)
    tbn = np.tile(np.eye(3, dtype=np.float32), (N, 1, 1))
    g = rng.normal(size=(N, C)).astype(np.float32)
    full = oracle.lookup_bwd(tex, uv, tbn, V, g)["grad_tex"]
    win = oracle.lookup_bwd(tex, uv, tbn, V, g, window=(2, 1, 3, 2))["grad_tex"]
    np.testing.assert_array_equal(win, full[1:3, 2:5])


# --------------------------------------------------------------------------
# The bake (Sec. 2.1 after Eq. (4b)): reflection vectors of the sample
# centres, carried to scene coordinates, sample an analytic environment
# --------------------------------------------------------------------------

_LOBES = np.array([[0.3, -0.2, 1.0, 3.0, 0.8, 0.3, 0.1, 0.5],
                   [1.0, 0.5, 0.4, 2.0, 0.1, 0.6, 0.2, 0.0],
                   [-0.6, 0.9, 0.2, 1.5, 0.3, 0.1, 0.7, 0.9]], np.float32)
_AMBIENT = np.array([0.05, 0.1, 0.02, 0.3], np.float32)


@pytest.mark.parametrize("n", [1, 2, 5, 8, 16])
def test_bake_directions_round_trip_through_the_lookup(n):
    # the incidence of every sample centre maps through Eqs. (1b), (3) and the
    # texel coordinate back onto that sample, and R is its mirror image about
    # the normal by the textbook reflection 2 (N.I) N - I
    inc, refl = oracle.bake_directions(n)
    N = np.array([0.0, 0.0, 1.0])
    for y in range(n):
        for x in range(n):
            s = oracle.map_one(np.eye(3), inc[y, x], n)[4:6]
            np.testing.assert_allclose(s, [x, y], atol=1e-9)
            I = inc[y, x]
            np.testing.assert_allclose(refl[y, x], 2 * np.dot(N, I) * N - I, atol=1e-15)
    np.testing.assert_allclose(np.linalg.norm(refl, axis=2), 1.0, atol=1e-14)
    assert np.all(refl[..., 2] >= 0)


def test_bake_constant_environment_is_constant():
    flat = _LOBES.copy()
    flat[:, 3] = 0.0  # sharpness 0: every lobe is its amplitude everywhere
    t = oracle.bake_environment(3, 2, 7, 4, flat, _AMBIENT)
    want = _AMBIENT.astype(np.float64) + flat[:, 4:8].astype(np.float64).sum(0)
    np.testing.assert_allclose(t, np.broadcast_to(want, t.shape), atol=1e-15)


@pytest.mark.parametrize("n", [6, 7])
def test_bake_lobe_on_the_normal_has_the_bucket_symmetry(n):
    # a lobe around N seen through the identity frame depends only on the
    # polar angle, so the baked bucket has the D4 symmetry of the square map
    lob = np.array([[0, 0, 1, 2.5, 1.0, 0.5, 0.25, 0.125]], np.float32)
    t = oracle.bake_environment(1, 1, n, 4, lob, _AMBIENT)[0, 0]
    np.testing.assert_allclose(t, t[:, ::-1], atol=1e-14)
    np.testing.assert_allclose(t, t[::-1, :], atol=1e-14)
    np.testing.assert_allclose(t, t.transpose(1, 0, 2), atol=1e-14)
    # and it grows toward the centre (the lobe's peak is on the normal)
    r = np.linalg.norm(np.indices((n, n)).transpose(1, 2, 0) - (n - 1) / 2, axis=2)
    order = np.argsort(r, axis=None)
    assert np.all(np.diff(t[..., 0].reshape(-1)[order]) <= 1e-12)


def test_bake_frame_equivariance():
    # sampling along M^T R with a lobe axis mu equals sampling along R with
    # the axis M mu: a frame rotates the scene, not the bucket
    rng = np.random.default_rng(5)
    W, H, n = 3, 2, 6
    frames = np.stack([_rand_rot(rng).T for _ in range(W * H)]).reshape(H, W, 3, 3)
    t = oracle.bake_environment(W, H, n, 4, _LOBES, _AMBIENT, frames=frames.astype(np.float32))
    for j in range(H):
        for i in range(W):
            M = frames[j, i].astype(np.float32).astype(np.float64)
            lob = _LOBES.astype(np.float64).copy()
            ax = lob[:, :3] / np.linalg.norm(lob[:, :3], axis=1, keepdims=True)
            lob[:, :3] = ax @ M.T
            ti = oracle.bake_environment(1, 1, n, 4, lob.astype(np.float32), _AMBIENT)[0, 0]
            np.testing.assert_allclose(t[j, i], ti, atol=2e-6)


def test_bake_centre_sample_sees_the_normal():
    # an odd bucket's centre sample has B = 0, so A = 0 and R = N (Eqs. 4a,
    # 4b): it holds the environment along the frame's normal
    rng = np.random.default_rng(6)
    M = _rand_rot(rng).T.astype(np.float32)
    n = 9
    t = oracle.bake_environment(1, 1, n, 4, _LOBES, _AMBIENT, frames=M.reshape(1, 1, 3, 3))
    Nw = M.astype(np.float64)[2]
    np.testing.assert_allclose(t[0, 0, n // 2, n // 2], oracle.env_eval(_LOBES, _AMBIENT, 4, Nw)[0],
                               atol=1e-14)


def _mirror_error(n, V):
    tex = oracle.bake_environment(1, 1, n, 4, _LOBES, _AMBIENT)
    otex = oracle.Tex(tex, 1, 1, n, 4, oracle.FMT_F64)
    err = []
    for v in V:
        got = oracle.lookup_one_f64(otex, [0.5, 0.5], np.eye(3), v)
        r = 2 * v[2] * np.array([0.0, 0.0, 1.0]) - v  # reflect(-V, N), N = e_z
        err.append(np.max(np.abs(got - oracle.env_eval(_LOBES, _AMBIENT, 4, r)[0])))
    return np.array(err)


def test_baked_mirror_converges_to_the_reflection():
    # a bucket baked from an environment and read back by the lookup gives the
    # mirror reflection env(2 (N.V) N - V) up to the sampling error, which
    # falls as n grows (views of elevation >= 20 degrees stay off the clamp):
    # second order on average (bilinear interpolation of a smooth function),
    # first order at worst (the square map of Eq. (3) is only continuous
    # across the diagonals |B_x| = |B_y|, so the cells there interpolate a kink)
    rng = np.random.default_rng(7)
    V = _rand_dirs(rng, 300, zmin=math.sin(math.radians(20)))
    e = {n: _mirror_error(n, V) for n in (8, 16, 32, 64)}
    mx = [e[n].max() for n in (8, 16, 32, 64)]
    mean = [e[n].mean() for n in (8, 16, 32, 64)]
    for a, b in zip(mx, mx[1:]):
        assert b < 0.6 * a
    for a, b in zip(mean, mean[1:]):
        assert b < 0.35 * a


# --------------------------------------------------------------------------
# Minification: mip chain of bucket matrices and the level of detail
# --------------------------------------------------------------------------

def _levels(W, H):
    return 1 + int(math.log2(max(W, H)))


@pytest.mark.parametrize("W,H", [(8, 4), (1, 8), (16, 16), (2, 1), (4, 32)])
def test_mips_are_block_means_brute_force(W, H):
    rng = np.random.default_rng(W * 7 + H)
    n, C = 3, 2
    t = rng.random((H, W, n, n, C))
    ch = oracle.build_mips(t, W, H, n, C, _levels(W, H))
    for l, lev in enumerate(ch):
        w, h = oracle.level_dims(W, H, l)
        sx, sy = W // w, H // h
        ref = t.reshape(h, sy, w, sx, n, n, C).mean(axis=(1, 3))
        np.testing.assert_allclose(lev, ref, rtol=1e-13, atol=1e-15)
    assert ch[-1].shape[:2] == (1, 1)


def test_lod_closed_forms():
    W, H, L = 64, 32, 7
    for k in range(L):
        assert oracle.lod([2.0 ** k / W, 0, 0, 2.0 ** k / H], W, H, L) == k
    # a rotated square footprint of side s pixels -> rho = s
    for th in (0.3, 1.1, 2.5):
        s = 5.0
        lam = oracle.lod([s * math.cos(th) / W, s * math.sin(th) / H,
                          -s * math.sin(th) / W, s * math.cos(th) / H], W, H, L)
        assert abs(lam - math.log2(s)) < 1e-12
    # anisotropic: the longer axis decides
    assert abs(oracle.lod([3.0 / W, 0, 0, 12.0 / H], W, H, L) - math.log2(12.0)) < 1e-12
    assert oracle.lod([0.25 / W, 0, 0, 0.5 / H], W, H, L) == 0.0      # magnified
    assert oracle.lod([1e6 / W, 0, 0, 1.0 / H], W, H, L) == L - 1     # beyond the chain
    assert oracle.lod([0, 0, 0, 0], W, H, L) == 0.0
    assert oracle.lod([math.nan, 0, 0, 0], W, H, L) == 0.0


def _mip_case(seed, W=16, H=8, n=5, C=3, N=300):
    rng = np.random.default_rng(seed)
    tex = rng.random((H, W, n, n, C)).astype(np.float32)
    uv = rng.uniform(-1.0, 2.0, (N, 2)).astype(np.float32)
    tbn = np.stack([_rand_rot(rng).T for _ in range(N)]).astype(np.float32)
    vt = _rand_dirs(rng, N, zmin=0.1)
    view = np.einsum("fkm,fk->fm", tbn.astype(np.float64), vt).astype(np.float32)
    return tex, uv, tbn, view


def _duv_iso(s, W, H, N):
    return np.tile(np.array([s / W, 0, 0, s / H], np.float32), (N, 1))


@pytest.mark.parametrize("mode", [oracle.MODE_NEAREST, oracle.MODE_BILINEAR])
def test_lod_lookup_reduces_to_the_plain_lookup_when_magnified(mode):
    W, H, n, C = 16, 8, 5, 3
    tex, uv, tbn, view = _mip_case(1)
    ch = oracle.build_mips(tex, W, H, n, C, _levels(W, H))
    got, lam = oracle.lookup_lod(ch, uv, tbn, view, _duv_iso(0.7, W, H, len(uv)), W, H, n, C,
                                 mode)
    assert np.all(lam == 0)
    ref = oracle.lookup_fwd(oracle.Tex(tex, W, H, n, C), uv, tbn, view, mode)
    np.testing.assert_array_equal(got, ref)


def test_lod_lookup_at_integer_levels_is_that_levels_lookup():
    W, H, n, C = 16, 8, 5, 3
    tex, uv, tbn, view = _mip_case(2)
    L = _levels(W, H)
    ch = oracle.build_mips(tex, W, H, n, C, L)
    for k in range(L):
        got, lam = oracle.lookup_lod(ch, uv, tbn, view, _duv_iso(2.0 ** k, W, H, len(uv)),
                                     W, H, n, C)
        assert np.all(lam == k)
        w, h = oracle.level_dims(W, H, k)
        ref = oracle.lookup_fwd(oracle.Tex(ch[k], w, h, n, C, oracle.FMT_F64), uv, tbn, view)
        np.testing.assert_array_equal(got, ref)


def test_lod_lookup_is_continuous_in_lambda():
    W, H, n, C = 16, 8, 5, 3
    tex, uv, tbn, view = _mip_case(3)
    ch = oracle.build_mips(tex, W, H, n, C, _levels(W, H))
    for k in (1, 2, 3):
        at, _ = oracle.lookup_lod(ch, uv, tbn, view, _duv_iso(2.0 ** k, W, H, len(uv)), W, H, n, C)
        for eps in (-1e-5, 1e-5):
            near, lam = oracle.lookup_lod(ch, uv, tbn, view,
                                          _duv_iso(2.0 ** (k + eps), W, H, len(uv)), W, H, n, C)
            assert np.all(np.abs(lam - k) < 2e-5)
            np.testing.assert_allclose(near, at, atol=1e-4)


def test_lod_lookup_of_identical_buckets_ignores_the_level():
    W, H, n, C = 16, 8, 5, 3
    rng = np.random.default_rng(4)
    one = rng.random((n, n, C))
    tex = np.broadcast_to(one, (H, W, n, n, C)).astype(np.float32)
    _, uv, tbn, view = _mip_case(4)
    ch = oracle.build_mips(tex, W, H, n, C, _levels(W, H))
    duv = (rng.uniform(0.1, 30.0, (len(uv), 1)) * np.array([1 / W, 0.3 / H, -0.2 / W, 1 / H])
           ).astype(np.float32)
    got, lam = oracle.lookup_lod(ch, uv, tbn, view, duv, W, H, n, C)
    assert np.any((lam > 0) & (lam != np.floor(lam)))
    ref = oracle.lookup_fwd(oracle.Tex(tex, W, H, n, C), uv, tbn, view)
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_lod_lookup_is_linear_in_the_texture():
    W, H, n, C = 16, 8, 5, 3
    texA, uv, tbn, view = _mip_case(5)
    texB, _, _, _ = _mip_case(6)
    rng = np.random.default_rng(7)
    duv = (rng.uniform(0.5, 20.0, (len(uv), 1)) * np.array([1 / W, 0, 0, 1 / H])).astype(np.float32)
    L = _levels(W, H)
    a, _ = oracle.lookup_lod(oracle.build_mips(texA, W, H, n, C, L), uv, tbn, view, duv, W, H, n, C)
    b, _ = oracle.lookup_lod(oracle.build_mips(texB, W, H, n, C, L), uv, tbn, view, duv, W, H, n, C)
    mix = 0.25 * texA.astype(np.float64) - 1.5 * texB.astype(np.float64)
    m, _ = oracle.lookup_lod(oracle.build_mips(mix, W, H, n, C, L), uv, tbn, view, duv, W, H, n, C)
    np.testing.assert_allclose(m, 0.25 * a - 1.5 * b, atol=1e-12)


def test_level_lookup_is_the_mean_of_plain_lookups_over_its_buckets():
    # the lookup is linear in the buckets and its sample position depends only
    # on the view, so level l at a bucket equals the mean of the level-0
    # lookups over the 2^l x 2^l buckets it covers
    W, H, n, C = 16, 8, 5, 3
    tex, _, tbn, view = _mip_case(8, N=40)
    ch = oracle.build_mips(tex, W, H, n, C, _levels(W, H))
    otex = oracle.Tex(tex, W, H, n, C)
    rng = np.random.default_rng(9)
    for l in (1, 2, 3):
        w, h = oracle.level_dims(W, H, l)
        sx, sy = W // w, H // h
        lvl = oracle.Tex(ch[l], w, h, n, C, oracle.FMT_F64)
        for f in range(len(tbn)):
            i, j = rng.integers(0, w), rng.integers(0, h)
            got = oracle.lookup_fwd(lvl, [[(i + 0.5) / w, (j + 0.5) / h]], tbn[f:f + 1],
                                    view[f:f + 1])[0]
            uvs = np.array([[(i * sx + di + 0.5) / W, (j * sy + dj + 0.5) / H]
                            for dj in range(sy) for di in range(sx)], np.float32)
            base = oracle.lookup_fwd(otex, uvs, np.repeat(tbn[f:f + 1], len(uvs), 0),
                                     np.repeat(view[f:f + 1], len(uvs), 0))
            np.testing.assert_allclose(got, base.mean(0), atol=1e-12)


# --------------------------------------------------------------------------
# Shadowing (Sec. 5, Shadowing): 1-bit storage, the lookup with the light
# direction in place of the incidence, and an analytic occluder bake
# --------------------------------------------------------------------------

def _packbits_reference(x, n):
    """numpy's own bit packer: per bucket the n n flags (x >= 1/2) padded with
    zeros to whole 32-bit words, least significant bit first."""
    nn = n * n
    wpb = (nn + 31) // 32
    flags = (x.reshape(-1, nn) >= 0.5)
    padded = np.zeros((flags.shape[0], wpb * 32), bool)
    padded[:, :nn] = flags
    return np.packbits(padded, axis=1, bitorder="little").view("<u4").reshape(-1)


@pytest.mark.parametrize("n", [1, 3, 5, 8, 16, 31, 32])
def test_pack_bits_matches_numpy_packbits(n):
    rng = np.random.default_rng(n)
    x = rng.uniform(-0.5, 1.5, (3, 4, n, n)).astype(np.float32)
    flat = x.reshape(-1)
    special = np.array([0.5, np.nextafter(np.float32(0.5), np.float32(0)), np.nan, np.inf,
                        -np.inf, -0.0, 1.0, 0.0], np.float32)
    flat[:min(flat.size, special.size)] = special[:flat.size]
    got = oracle.pack_bits(x, n)
    np.testing.assert_array_equal(got, _packbits_reference(x, n))
    # 0.5 is lit, its predecessor and NaN are not
    assert got[0] & 1 == 1
    if n * n > 2:
        assert (got[0] >> 1) & 1 == 0 and (got[0] >> 2) & 1 == 0


@pytest.mark.parametrize("mode", [oracle.MODE_NEAREST, oracle.MODE_BILINEAR])
def test_bit_texture_reads_as_its_zero_one_texture(mode):
    # the 1-bit decode returns exactly the flag, so a 1-bit texture looks up
    # as the binary32 texture of its zeros and ones
    rng = np.random.default_rng(11)
    W, H, n, N = 5, 3, 6, 400
    x = rng.uniform(0, 1, (H, W, n, n)).astype(np.float32)
    zo = (x >= 0.5).astype(np.float32)
    bits = oracle.Tex(oracle.pack_bits(x, n), W, H, n, 1, oracle.FMT_BIT1)
    ref = oracle.Tex(zo, W, H, n, 1)
    uv = rng.uniform(-1, 2, (N, 2)).astype(np.float32)
    tbn = np.stack([_rand_rot(rng) for _ in range(N)]).astype(np.float32)
    view = rng.normal(size=(N, 3)).astype(np.float32)
    np.testing.assert_array_equal(oracle.lookup_fwd(bits, uv, tbn, view, mode),
                                  oracle.lookup_fwd(ref, uv, tbn, view, mode))


def _light_case(seed, W=4, H=3, n=8, C=2, N=200):
    rng = np.random.default_rng(seed)
    tex = oracle.Tex(rng.uniform(0, 1, (H, W, n, n, C)).astype(np.float32), W, H, n, C)
    uv = rng.uniform(-1, 2, (N, 2)).astype(np.float32)
    tbn = np.stack([_rand_rot(rng) for _ in range(N)]).astype(np.float32)
    return rng, tex, uv, tbn


@pytest.mark.parametrize("mode", [oracle.MODE_NEAREST, oracle.MODE_BILINEAR])
def test_one_light_sample_is_the_view_lookup(mode):
    # one directional sample: the lookup of Sec. 2.1 with that direction as
    # the incidence; a point light whose sample sits at pos + V (dyadic
    # values, so the difference is exact in binary32) gives the lookup of V
    rng, tex, uv, tbn = _light_case(12)
    N = uv.shape[0]
    L = np.array([[0.3, -0.2, 0.9]], np.float32)
    np.testing.assert_allclose(
        oracle.lookup_light(tex, uv, tbn, L, oracle.LIGHT_DIRECTIONAL, mode=mode),
        oracle.lookup_fwd(tex, uv, tbn, np.repeat(L, N, 0), mode), atol=1e-15)
    V = (rng.integers(-64, 65, (N, 3)) / 64.0).astype(np.float32)
    V[np.all(V == 0, axis=1)] = [0, 0, 1]
    Q = np.array([[1.5, -2.25, 3.0]], np.float32)
    pos = (Q - V).astype(np.float32)
    assert np.array_equal(Q - pos, V)
    np.testing.assert_allclose(
        oracle.lookup_light(tex, uv, tbn, Q, oracle.LIGHT_POINT, pos=pos, mode=mode),
        oracle.lookup_fwd(tex, uv, tbn, V, mode), atol=1e-15)


@pytest.mark.parametrize("n", [3, 8, 16])
def test_light_toward_a_sample_reads_that_samples_bit(n):
    # a light along the scene direction M^T I(x, y) of sample (x, y) (I from
    # Eqs. (4a), (2c)) is mapped onto that sample's centre, so a 1-bit texture
    # returns the sample's flag; a point light reaches it from any distance
    # along that direction, and the opposite direction does not
    rng = np.random.default_rng(13 + n)
    x = rng.uniform(0, 1, (1, 1, n, n)).astype(np.float32)
    tex = oracle.Tex(oracle.pack_bits(x, n), 1, 1, n, 1, oracle.FMT_BIT1)
    inc, _ = oracle.bake_directions(n)
    M = _rand_rot(rng).T
    uv = np.array([[0.25, 0.75]], np.float32)
    tbn = M.astype(np.float32)[None]
    P = np.array([[0.5, -1.0, 2.0]], np.float32)
    flips = 0
    for y in range(n):
        for xx in range(n):
            d = (tbn[0].astype(np.float64).T @ inc[y, xx]).astype(np.float32)[None]
            want = float(x[0, 0, y, xx] >= 0.5)
            got = oracle.lookup_light(tex, uv, tbn, d, oracle.LIGHT_DIRECTIONAL)[0, 0]
            assert abs(got - want) <= 1e-5, (y, xx, got, want)
            Q = (P.astype(np.float64) + 3.0 * d).astype(np.float32)
            got = oracle.lookup_light(tex, uv, tbn, Q, oracle.LIGHT_POINT, pos=P)[0, 0]
            assert abs(got - want) <= 1e-5, (y, xx, got, want)
            away = oracle.lookup_light(tex, uv, tbn, -d, oracle.LIGHT_DIRECTIONAL)[0, 0]
            flips += abs(away - want) > 1e-3
    if n >= 8:
        assert flips > 0  # the light's sign matters


def test_area_light_is_the_mean_of_its_samples():
    # directions aimed at three lit samples and one dark sample read 3/4; at
    # one lit and two dark, 1/3; the order of the samples does not matter
    n = 8
    x = np.zeros((1, 1, n, n), np.float32)
    x[0, 0, 2, 3] = x[0, 0, 5, 5] = x[0, 0, 6, 1] = 1.0
    tex = oracle.Tex(oracle.pack_bits(x, n), 1, 1, n, 1, oracle.FMT_BIT1)
    inc, _ = oracle.bake_directions(n)
    uv = np.array([[0.5, 0.5]], np.float32)
    tbn = np.eye(3, dtype=np.float32)[None]
    d = lambda y, xx: inc[y, xx].astype(np.float32)
    L1 = np.stack([d(2, 3), d(5, 5), d(6, 1), d(4, 4)])
    assert abs(oracle.lookup_light(tex, uv, tbn, L1)[0, 0] - 0.75) <= 1e-6
    L2 = np.stack([d(0, 0), d(6, 1), d(7, 7)])
    assert abs(oracle.lookup_light(tex, uv, tbn, L2)[0, 0] - 1 / 3) <= 1e-6
    assert abs(oracle.lookup_light(tex, uv, tbn, L2[::-1].copy())[0, 0] - 1 / 3) <= 1e-6


def _cone_hits(o, d, c, r):
    """Whether the ray o + t d (t > 0, d unit) meets the ball (c, r), by the
    cone the ball subtends at o: the origin is inside, or the angle between d
    and c - o is at most asin(r / |c - o|).  Also the angular margin."""
    oc = c - o
    l = np.linalg.norm(oc)
    if l <= r:
        return True, np.inf
    ang = math.acos(max(-1.0, min(1.0, float(np.dot(d, oc) / l))))
    half = math.asin(r / l)
    return ang <= half, abs(ang - half)


def test_shadow_bake_agrees_with_the_subtended_cone():
    rng = np.random.default_rng(14)
    W, H, n, K = 3, 2, 9, 4
    origins = rng.uniform(-1, 1, (H, W, 3)).astype(np.float32)
    spheres = np.concatenate([rng.uniform(-2, 2, (K, 3)), rng.uniform(0.3, 1.2, (K, 1))],
                             1).astype(np.float32)
    frames = np.stack([_rand_rot(rng).T for _ in range(W * H)]).reshape(H, W, 3, 3)
    frames = frames.astype(np.float32)
    words, margin = oracle.bake_shadow(W, H, n, origins, spheres, frames=frames)
    inc, _ = oracle.bake_directions(n)
    wpb = oracle.words_per_bucket(n)
    checked = lit = 0
    for j in range(H):
        for i in range(W):
            M = frames[j, i].astype(np.float64)
            o = origins[j, i].astype(np.float64)
            for y in range(n):
                for x in range(n):
                    d = M.T @ inc[y, x]
                    d /= np.linalg.norm(d)
                    hits = [_cone_hits(o, d, s[:3].astype(np.float64), float(s[3]))
                            for s in spheres]
                    if min(h[1] for h in hits) < 1e-9:
                        continue
                    k = y * n + x
                    bit = (words[(j * W + i) * wpb + k // 32] >> (k % 32)) & 1
                    assert bit == (not any(h[0] for h in hits)), (i, j, x, y)
                    checked += 1
                    lit += bit
    assert checked > 0.95 * W * H * n * n and 0 < lit < checked
    # padding bits past n n stay clear
    assert np.all(words.reshape(-1, wpb)[:, -1] >> ((n * n) % 32) == 0)


def test_shadow_bake_frame_equivariance():
    # baking with the frame M around the origin o equals baking with the
    # identity frame after carrying each ball's centre to o + M (c - o): the
    # frame turns the scene into the bucket's texture space, where the light
    # lookup (u = M L) reads it
    rng = np.random.default_rng(15)
    n = 12
    o = np.array([0.25, -0.5, 0.125], np.float32)
    M = _rand_rot(rng).T
    balls = np.array([[0.5, 0.2, 1.5, 0.6], [-1.0, 0.5, 0.8, 0.4], [0.3, -1.2, 0.9, 0.5]])
    w1, m1 = oracle.bake_shadow(1, 1, n, o.reshape(1, 1, 3), balls.astype(np.float32),
                                frames=M.astype(np.float32).reshape(1, 1, 3, 3))
    Mf = M.astype(np.float32).astype(np.float64)
    moved = balls.copy()
    moved[:, :3] = o + (balls[:, :3] - o) @ Mf.T
    w2, m2 = oracle.bake_shadow(1, 1, n, o.reshape(1, 1, 3), moved.astype(np.float32))
    keep = (np.minimum(m1, m2) > 1e-5).reshape(-1)
    k = np.arange(n * n)
    b1 = (w1[k // 32] >> (k % 32)) & 1
    b2 = (w2[k // 32] >> (k % 32)) & 1
    assert keep.sum() > 0.9 * n * n
    np.testing.assert_array_equal(b1[keep], b2[keep])
    assert 0 < b1.sum() < n * n


def test_shadow_of_a_ball_over_the_normal_is_a_cap():
    # a ball of radius r centred at height h over the origin shades exactly
    # the directions within asin(r / h) of the normal: with h = 2, r = 1 the
    # samples whose incidence has I_z > cos 30 degrees
    n = 15
    words, _ = oracle.bake_shadow(1, 1, n, np.zeros((1, 1, 3), np.float32),
                                  np.array([[0, 0, 2, 1]], np.float32))
    inc, _ = oracle.bake_directions(n)
    for y in range(n):
        for x in range(n):
            cz = inc[y, x, 2]
            if abs(cz - math.cos(math.radians(30))) < 1e-9:
                continue
            k = y * n + x
            assert ((words[k // 32] >> (k % 32)) & 1) == (cz < math.cos(math.radians(30)))
    c = n // 2 * n + n // 2
    assert (words[c // 32] >> (c % 32)) & 1 == 0  # the centre sample looks up the normal


def _sun_samples(axis, alpha, k):
    """k directions uniform in solid angle over the cap of half-angle alpha
    around the unit axis, on a golden-angle spiral (every sample at its own
    polar angle, so no ring of samples sits on an occluder's outline)."""
    i = np.arange(k) + 0.5
    cz = 1 - i / k * (1 - math.cos(alpha))
    phi = i * math.pi * (3 - math.sqrt(5))
    sz = np.sqrt(1 - cz * cz)
    loc = np.stack([sz * np.cos(phi), sz * np.sin(phi), cz], -1)
    a = np.asarray(axis, np.float64) / np.linalg.norm(axis)
    t = np.cross(a, [1.0, 0, 0]) if abs(a[0]) < 0.9 else np.cross(a, [0, 1.0, 0])
    t /= np.linalg.norm(t)
    b = np.cross(a, t)
    return loc @ np.stack([t, b, a])


def test_area_shadow_converges_to_the_exact_penumbra():
    # a sun of angular radius 25 degrees, tilted 20 degrees off the normal,
    # partly hidden by the ball of the previous test.  Per sun sample the
    # lookup departs from the exact visibility only within one cell of the
    # occluder's outline, so the mean per-sample error falls as 1/n; the
    # area light's value (the mean over the samples) is off by at most half
    # the measure of that band.  A sun centred on the occluder approaches the
    # closed-form cap fraction (cos theta_o - cos alpha) / (1 - cos alpha).
    c = np.array([0.0, 0.0, 2.0])
    sun = _sun_samples([math.sin(math.radians(20)), 0.0, math.cos(math.radians(20))],
                       math.radians(25), 2048)
    exact = np.array([not _cone_hits(np.zeros(3), s, c, 1.0)[0] for s in sun], np.float64)
    uv = np.array([[0.5, 0.5]], np.float32)
    eye = np.eye(3, dtype=np.float32)[None]
    sun32 = sun.astype(np.float32)
    per_sample, area = [], []
    for n in (8, 16, 32, 64):
        words, _ = oracle.bake_shadow(1, 1, n, np.zeros((1, 1, 3), np.float32),
                                      np.array([[0, 0, 2, 1]], np.float32))
        tex = oracle.Tex(words, 1, 1, n, 1, oracle.FMT_BIT1)
        each = oracle.lookup_fwd(tex, np.repeat(uv, len(sun), 0), np.repeat(eye, len(sun), 0),
                                 sun32)[:, 0]
        got = oracle.lookup_light(tex, uv, eye, sun32)[0, 0]
        assert abs(got - each.mean()) < 1e-12
        per_sample.append(np.abs(each - exact).mean())
        area.append(abs(got - exact.mean()))
    assert 0.2 < exact.mean() < 0.8
    for a, b in zip(per_sample, per_sample[1:]):
        assert b < 0.7 * a, per_sample
    assert area[-1] <= per_sample[-1] + 1e-12 and area[-1] < 0.03, area
    centred = _sun_samples([0, 0, 1.0], math.radians(40), 4096)
    words, _ = oracle.bake_shadow(1, 1, 64, np.zeros((1, 1, 3), np.float32),
                                  np.array([[0, 0, 2, 1]], np.float32))
    got = oracle.lookup_light(oracle.Tex(words, 1, 1, 64, 1, oracle.FMT_BIT1), uv, eye,
                              centred.astype(np.float32))
    cap = ((math.cos(math.radians(30)) - math.cos(math.radians(40)))
           / (1 - math.cos(math.radians(40))))
    assert abs(got[0, 0] - cap) < 0.03, (got[0, 0], cap)


# --------------------------------------------------------------------------
# Bucket dictionary: "simple compression" of repetitive buckets (Sec. 1,
# Sec. 2) as a codebook of bucket entries, an index map and per-bucket gains;
# the codebook built by Lloyd's k-means steps
# --------------------------------------------------------------------------

def _dict_case(seed, W=5, H=4, n=6, C=3, K=7, N=500):
    rng = np.random.default_rng(seed)
    cb = rng.uniform(0, 1, (K, n, n, C)).astype(np.float32)
    index = rng.integers(0, K, (H, W)).astype(np.int32)
    gains = rng.uniform(0.5, 2.0, (H, W)).astype(np.float32)
    uv = rng.uniform(-1, 2, (N, 2)).astype(np.float32)
    tbn = np.stack([_rand_rot(rng) for _ in range(N)]).astype(np.float32)
    view = rng.normal(size=(N, 3)).astype(np.float32)
    return cb, index, gains, uv, tbn, view


@pytest.mark.parametrize("mode", [oracle.MODE_NEAREST, oracle.MODE_BILINEAR])
@pytest.mark.parametrize("with_gains", [False, True])
def test_dictionary_lookup_is_the_lookup_of_the_decoded_matrix(mode, with_gains):
    # decoded bucket b = gain(b) * codebook[index(b)], formed here by numpy's
    # fancy indexing; the dictionary lookup reads exactly that matrix
    W, H, n, C, K = 5, 4, 6, 3, 7
    cb, index, gains, uv, tbn, view = _dict_case(31)
    g = gains if with_gains else None
    dec = cb.astype(np.float64)[index]
    if with_gains:
        dec = dec * gains.astype(np.float64)[:, :, None, None, None]
    want = oracle.lookup_fwd(oracle.Tex(dec, W, H, n, C, oracle.FMT_F64), uv, tbn, view, mode)
    got = oracle.lookup_fwd_dict(cb, K, index, g, W, H, n, C, uv, tbn, view, mode=mode)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)


def test_dictionary_with_bf16_entries_and_the_identity_map():
    # an identity index map without gains is the plain texture; BF16 entries
    # decode exactly (the bits of the upper half of a binary32)
    W, H, n, C = 4, 3, 5, 2
    rng = np.random.default_rng(32)
    tex = rng.uniform(0, 1, (H, W, n, n, C)).astype(np.float32)
    uv = rng.uniform(0, 1, (300, 2)).astype(np.float32)
    tbn = np.stack([_rand_rot(rng) for _ in range(300)]).astype(np.float32)
    view = rng.normal(size=(300, 3)).astype(np.float32)
    ident = np.arange(W * H, dtype=np.int32).reshape(H, W)
    for mode in (oracle.MODE_NEAREST, oracle.MODE_BILINEAR):
        np.testing.assert_array_equal(
            oracle.lookup_fwd_dict(tex.reshape(W * H, n, n, C), W * H, ident, None, W, H, n, C,
                                   uv, tbn, view, mode=mode),
            oracle.lookup_fwd(oracle.Tex(tex, W, H, n, C), uv, tbn, view, mode))
    codes = (tex.view(np.uint32) >> 16).astype(np.uint16)
    trunc = (codes.astype(np.uint32) << 16).view(np.float32)
    np.testing.assert_array_equal(
        oracle.lookup_fwd_dict(codes.reshape(W * H, n, n, C), W * H, ident, None, W, H, n, C, uv,
                               tbn, view, fmt=oracle.FMT_BF16),
        oracle.lookup_fwd(oracle.Tex(trunc, W, H, n, C), uv, tbn, view))


def test_vq_assignment_is_scipys_nearest_neighbour():
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(33)
    X = rng.normal(size=(400, 48)).astype(np.float32)
    cb = rng.normal(size=(37, 48)).astype(np.float32)
    cb[5] = cb[20]  # an exact duplicate entry: ties go to the smaller index
    a, d = oracle.vq_assign(X, cb)
    full = cdist(X.astype(np.float64), cb.astype(np.float64), "sqeuclidean")
    np.testing.assert_array_equal(a, np.argmin(full, axis=1))
    np.testing.assert_allclose(d, full.min(axis=1), rtol=1e-12)
    assert not np.any(a == 20)
    # a row equal to an entry is assigned to it at distance 0
    a2, d2 = oracle.vq_assign(cb[[3, 9]], cb)
    np.testing.assert_array_equal(a2, [3, 9])
    assert np.all(d2 == 0)


def test_vq_update_is_the_mean_of_each_cluster():
    rng = np.random.default_rng(34)
    X = rng.normal(size=(300, 20)).astype(np.float32)
    K = 9
    a = rng.integers(0, K - 2, 300).astype(np.int32)  # entries 7 and 8 stay empty
    prev = rng.normal(size=(K, 20)).astype(np.float32)
    out, cnt = oracle.vq_update(X, a, prev)
    np.testing.assert_array_equal(cnt, np.bincount(a, minlength=K))
    for k in range(K):
        if cnt[k]:
            np.testing.assert_allclose(out[k], X[a == k].astype(np.float64).mean(0), rtol=1e-13,
                                       atol=1e-15)
        else:
            np.testing.assert_array_equal(out[k], prev[k].astype(np.float64))


def test_lloyd_never_increases_the_distortion_and_recovers_separated_clusters():
    # the k-means invariant: an assignment step then an update step cannot
    # raise the sum of squared distances; on repetitive buckets (noisy copies
    # of a few prototypes) one step from one member of each group finds them
    rng = np.random.default_rng(35)
    X = rng.normal(size=(600, 16)).astype(np.float32)
    cb = X[rng.choice(600, 12, replace=False)].copy()
    prev = np.inf
    for _ in range(6):
        a, d = oracle.vq_assign(X, cb)
        assert d.sum() <= prev * (1 + 1e-12)
        prev = d.sum()
        cb = oracle.vq_update(X, a, cb)[0].astype(np.float32)
    protos = rng.uniform(0, 1, (8, 32)).astype(np.float32)
    labels = rng.integers(0, 8, 2000)
    Y = (protos[labels] + rng.normal(0, 0.01, (2000, 32))).astype(np.float32)
    init = np.stack([Y[np.nonzero(labels == k)[0][0]] for k in range(8)])
    a, _ = oracle.vq_assign(Y, init)
    np.testing.assert_array_equal(a, labels)
    new, cnt = oracle.vq_update(Y, a, init)
    np.testing.assert_array_equal(cnt, np.bincount(labels, minlength=8))
    assert np.abs(new - protos).max() < 0.003


# --------------------------------------------------------------------------
# Backward of the level-of-detail lookup and the adjoint of the mip chain
# --------------------------------------------------------------------------

def _lod_bwd_case(seed, mode, W=8, H=4, n=5, C=3, N=200):
    tex, uv, tbn, view = _mip_case(seed, W, H, n, C, N)
    rng = np.random.default_rng(seed + 1)
    L = _levels(W, H)
    chain = oracle.build_mips(tex, W, H, n, C, L)
    # footprints from 0.3 to 12 buckets: every level and the clamp are used
    s = np.exp(rng.uniform(np.log(0.3), np.log(12.0), N))
    duv = np.stack([s / W, s * rng.uniform(-0.3, 0.3, N) / H, s * rng.uniform(-0.3, 0.3, N) / W,
                    s / H], 1).astype(np.float32)
    g = rng.normal(size=(N, C)).astype(np.float32)
    return chain, uv, tbn, view, duv, g


@pytest.mark.parametrize("mode", [oracle.MODE_NEAREST, oracle.MODE_BILINEAR])
def test_lod_backward_is_the_adjoint_of_the_lod_lookup(mode):
    # the trilinear lookup is linear in the chain's texels, so for any
    # perturbation of every level sum_f g_f . out_f(delta) = <grad_chain, delta>
    W, H, n, C = 8, 4, 5, 3
    chain, uv, tbn, view, duv, g = _lod_bwd_case(40 + mode, mode)
    grads, _, _ = oracle.lookup_lod_bwd(chain, uv, tbn, view, duv, g, W, H, n, C, mode=mode)
    rng = np.random.default_rng(41)
    delta = [rng.normal(size=np.asarray(c).shape) for c in chain]
    out, _ = oracle.lookup_lod(delta, uv, tbn, view, duv, W, H, n, C, mode=mode)
    lhs = float(np.sum(g.astype(np.float64) * out))
    rhs = float(sum(np.sum(a * b) for a, b in zip(grads, delta)))
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))
    assert all(np.any(gr != 0) for gr in grads[:3])  # several levels are reached


def test_lod_backward_of_one_level_is_the_plain_backward():
    W, H, n, C = 8, 4, 5, 3
    chain, uv, tbn, view, duv, g = _lod_bwd_case(42, oracle.MODE_BILINEAR)
    grads, gv, gu = oracle.lookup_lod_bwd(chain[:1], uv, tbn, view, duv, g, W, H, n, C,
                                          mode=oracle.MODE_BILINEAR)
    ref = oracle.lookup_bwd(oracle.Tex(chain[0], W, H, n, C, oracle.FMT_F64), uv, tbn, view, g,
                            mode=oracle.MODE_BILINEAR)
    np.testing.assert_allclose(grads[0], ref["grad_tex"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(gv, ref["grad_view"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(gu, ref["grad_uv"], rtol=0, atol=1e-13)


@pytest.mark.parametrize("mode", [oracle.MODE_NEAREST, oracle.MODE_BILINEAR])
def test_lod_backward_view_and_uv_finite_differences(mode):
    W, H, n, C = 8, 4, 5, 3
    chain, uv, tbn, view, duv, g = _lod_bwd_case(44 + mode, mode, N=80)
    _, gv, gu = oracle.lookup_lod_bwd(chain, uv, tbn, view, duv, g, W, H, n, C, mode=mode)
    checked = 0
    for f in range(len(uv)):
        if not _away_from_kinks(tbn[f].astype(np.float64).reshape(9), view[f].astype(np.float64), n):
            continue
        U = uv[f].astype(np.float64)
        p = (U - np.floor(U)) * [W, H] - 0.5
        fd_v, fd_u = np.zeros(3), np.zeros(2)
        for k in range(3):
            # central differences with a step the float32 inputs represent
            # exactly in size (the actual step is taken from the rounded values)
            h = 2e-4
            Vp, Vm = view[f].astype(np.float64).copy(), view[f].astype(np.float64).copy()
            Vp[k] += h
            Vm[k] -= h
            Vp32, Vm32 = Vp.astype(np.float32), Vm.astype(np.float32)
            op, _ = oracle.lookup_lod(chain, uv[f:f + 1], tbn[f:f + 1], Vp32[None],
                                      duv[f:f + 1], W, H, n, C, mode=mode)
            om, _ = oracle.lookup_lod(chain, uv[f:f + 1], tbn[f:f + 1], Vm32[None],
                                      duv[f:f + 1], W, H, n, C, mode=mode)
            step = float(Vp32[k]) - float(Vm32[k])
            fd_v[k] = np.dot(g[f].astype(np.float64), (op[0] - om[0]) / step)
        assert np.linalg.norm(gv[f] - fd_v) <= 2e-4 * max(1.0, np.linalg.norm(fd_v)), (f, gv[f], fd_v)
        if mode == oracle.MODE_BILINEAR and np.all(np.abs(p - np.round(p)) > 2e-2):
            for k in range(2):
                h = 2e-3 / max(W, H)
                Up, Um = U.copy(), U.copy()
                Up[k] += h
                Um[k] -= h
                op, _ = oracle.lookup_lod(chain, Up.astype(np.float32)[None], tbn[f:f + 1],
                                          view[f:f + 1], duv[f:f + 1], W, H, n, C, mode=mode)
                om, _ = oracle.lookup_lod(chain, Um.astype(np.float32)[None], tbn[f:f + 1],
                                          view[f:f + 1], duv[f:f + 1], W, H, n, C, mode=mode)
                step = float(np.float32(Up[k])) - float(np.float32(Um[k]))
                fd_u[k] = np.dot(g[f].astype(np.float64), (op[0] - om[0]) / step)
            assert np.linalg.norm(gu[f] - fd_u) <= 1e-3 * max(1.0, np.linalg.norm(fd_u)), (f, gu[f], fd_u)
        if mode == oracle.MODE_NEAREST:
            assert np.all(gu[f] == 0)
        checked += 1
    assert checked > 20


@pytest.mark.parametrize("W,H", [(8, 4), (1, 8), (4, 1), (2, 2)])
def test_mip_adjoint_identity(W, H):
    # the adjoint of the 2 x 2 (or 2) block mean: <A^T G, X> = <G, A X>
    n, C = 3, 2
    rng = np.random.default_rng(W * 10 + H)
    X = rng.normal(size=(H, W, n, n, C))
    nxt = oracle.build_mips(X, W, H, n, C, 2)[1]
    G = rng.normal(size=nxt.shape)
    AtG = oracle.build_mip_adjoint(G, W, H, n, C)
    assert abs(np.sum(AtG * X) - np.sum(G * nxt)) <= 1e-12 * np.sum(np.abs(G * nxt))
    # adding into an existing gradient
    base = rng.normal(size=X.shape)
    acc = oracle.build_mip_adjoint(G, W, H, n, C, grad_src=base.copy())
    np.testing.assert_allclose(acc - base, AtG, atol=1e-14)


# --------------------------------------------------------------------------
# the error scales of the backward's criterion: the magnitude chain S
# (scale_view, scale_uv) and the rounding term (lookup_bwd_round)
# --------------------------------------------------------------------------

def _scale_case(seed, W, H, n, C, N, frames=True):
    rng = np.random.default_rng(seed)
    T = _tex(rng, W, H, n, C)
    uv = rng.uniform(-1, 2, (N, 2)).astype(np.float32)
    d = _rand_dirs(rng, N, zmin=0.05) * rng.uniform(0.5, 2.0, (N, 1))
    if frames:
        R = np.array([_rand_rot(rng) for _ in range(N)])
        tbn = R.astype(np.float32)
        view = np.einsum("nkm,nk->nm", R, d).astype(np.float32)  # M view = d
    else:
        tbn = np.tile(np.eye(3, dtype=np.float32), (N, 1, 1))
        view = d.astype(np.float32)
    g = rng.normal(size=(N, C)).astype(np.float32)
    return T, uv, tbn, view, g


def _smooth(uv, tbn, view, W, H, n, mode, margin=1e-5):
    _, _, edge = oracle.indices(uv, tbn, view, W, H, n)
    keep = (edge[:, 0] >= margin) & (edge[:, 1] >= margin) & (edge[:, 2] >= margin)
    if mode == oracle.MODE_BILINEAR:
        f = uv.astype(np.float64) - np.floor(uv.astype(np.float64))
        p = f * [W, H] - 0.5
        keep &= np.all(np.abs(p - np.round(p)) >= margin * np.array([W, H]), axis=1)
    return keep


@pytest.mark.parametrize("mode", [oracle.MODE_NEAREST, oracle.MODE_BILINEAR])
def test_magnitude_scale_bounds_the_gradient(mode):
    # S takes every factor and term of the chain by its magnitude, so by the
    # triangle inequality it bounds each component of the gradient
    W, H, n, C = 6, 5, 8, 3
    T, uv, tbn, view, g = _scale_case(60 + mode, W, H, n, C, 3000)
    r = oracle.lookup_bwd(oracle.Tex(T, W, H, n, C), uv, tbn, view, g, mode=mode,
                          want_tex=False)
    assert np.all(np.abs(r["grad_view"]) <= r["scale_view"] * (1 + 1e-12))
    assert np.all(np.abs(r["grad_uv"]) <= r["scale_uv"] * (1 + 1e-12))
    assert np.all(r["scale_view"] >= 0) and np.any(r["scale_view"] > 0)
    if mode == oracle.MODE_BILINEAR:
        assert np.any(r["scale_uv"] > 0)
    else:
        assert np.all(r["scale_uv"] == 0)


def test_magnitude_scale_equals_the_gradient_without_cancellation():
    # normal incidence in the identity frame: A = 0, Eq. (3)'s Jacobian is the
    # identity, Eq. (1b)'s is sqrt(2)/2 on the tangent axes, and no term of the
    # chain has a sign of its own; with each channel's texel slope and upstream
    # gradient of one sign along an axis, nothing cancels and S = |g*|
    n, C = 8, 3
    bx = np.array([0.1, -0.2, 0.05])
    by = np.array([-0.05, 0.1, -0.02])
    y, x = np.mgrid[0:n, 0:n]
    T = (0.5 + bx * x[..., None] + by * y[..., None]).astype(np.float32)[None, None]
    tex = oracle.Tex(T, 1, 1, n, C)
    uv = np.array([[0.3, 0.6]], np.float32)
    tbn = np.eye(3, dtype=np.float32)[None]
    view = np.array([[0, 0, 1.0]], np.float32)
    for g in ([1.0, -2.0, 0.5], [-1.0, 2.0, -0.5]):
        g = np.array([g], np.float32)
        r = oracle.lookup_bwd(tex, uv, tbn, view, g, want_tex=False)
        np.testing.assert_allclose(r["scale_view"], np.abs(r["grad_view"]), rtol=1e-14,
                                   atol=1e-16)
        # and the closed form: (sqrt2/2)(n/2) sum_c g_c (slope_x, slope_y), 0
        want = np.sqrt(2) / 2 * n / 2 * np.array([np.dot(g[0], bx), np.dot(g[0], by), 0.0])
        np.testing.assert_allclose(r["grad_view"][0], want, rtol=1e-6, atol=1e-12)
    # the uv scale: bucket column i0 = 0 holds zeros and column 1 holds positive
    # texels, so dL/du = W ((1 - b) L1 + b L3) with nothing subtracted
    W, H = 2, 2
    rng = np.random.default_rng(61)
    T = rng.uniform(0.1, 1.0, (H, W, n, n, C)).astype(np.float32)
    T[:, 0] = 0.0
    tex = oracle.Tex(T, W, H, n, C)
    N = 200
    uv = np.stack([rng.uniform(0.26, 0.74, N), rng.uniform(0, 1, N)], 1).astype(np.float32)
    view = _rand_dirs(rng, N, zmin=0.2).astype(np.float32)
    tbn = np.tile(np.eye(3, dtype=np.float32), (N, 1, 1))
    g = rng.uniform(0.1, 1.0, (N, C)).astype(np.float32)
    r = oracle.lookup_bwd(tex, uv, tbn, view, g, mode=oracle.MODE_BILINEAR, want_tex=False)
    assert np.all(r["grad_uv"][:, 0] > 0)
    np.testing.assert_allclose(r["scale_uv"][:, 0], r["grad_uv"][:, 0], rtol=1e-13)


@pytest.mark.parametrize("W,H,n,C,mode,frames", [
    (6, 5, 8, 3, oracle.MODE_NEAREST, True), (6, 5, 8, 3, oracle.MODE_BILINEAR, True),
    (8, 8, 16, 4, oracle.MODE_NEAREST, True), (8, 8, 16, 4, oracle.MODE_BILINEAR, False),
    (4, 4, 64, 1, oracle.MODE_BILINEAR, True)])
def test_error_scales_bound_a_binary32_evaluation(W, H, n, C, mode, frames):
    # an independent binary32 evaluation of the lookup and its chain (numpy
    # float32, one rounding per operation) differs from the oracle's gradient
    # by at most 2^-20 S plus the rounding term: S covers the rounding of the
    # chain's own arithmetic and the rounding term that of the quantities the
    # taps are weighted with.  A scale missing a factor or a term would let
    # some fragment exceed it.
    from binary32_model import model
    from helpers import round_s, round_w
    T, uv, tbn, view, g = _scale_case(70 + n + mode, W, H, n, C, 20000, frames)
    tex = oracle.Tex(T, W, H, n, C)
    r = oracle.lookup_bwd(tex, uv, tbn, view, g, mode=mode, want_tex=False)
    rv, ru = oracle.lookup_bwd_round(tex, uv, tbn, view, g, round_s(n), round_w(W, H, uv),
                                     mode=mode)
    keep = _smooth(uv, tbn, view, W, H, n, mode)
    gv, gu = model(T, W, H, n, C, uv, tbn, view, g, mode)
    for mine, ref, S, rnd in ((gv, r["grad_view"], r["scale_view"], rv),
                              (gu, r["grad_uv"], r["scale_uv"], ru)):
        err = np.linalg.norm(mine - ref, axis=1)[keep]
        bound = 2.0 ** -20 * np.linalg.norm(S, axis=1)[keep] + rnd[keep]
        assert np.all(err <= bound), (np.max(err / np.maximum(bound, 1e-300)))
        # and the reading of "1e-4 relative": 1e-4 |g*| + 1e-6 sum |go| + the rounding term
        gn = np.linalg.norm(ref, axis=1)[keep]
        assert np.all(err <= 1e-4 * gn + 1e-6 * np.abs(g[keep]).sum(1) + rnd[keep])
    if n == 64:
        # at n = 64 the rounding of s (up to 2^-24 n) outweighs the chain's
        # own: without the rounding term some fragments exceed 2^-20 S, so
        # the term is needed, not decoration
        err = np.linalg.norm(gv - r["grad_view"], axis=1)[keep]
        assert np.any(err > 2.0 ** -20 * np.linalg.norm(r["scale_view"], axis=1)[keep])


@pytest.mark.parametrize("mode", [oracle.MODE_NEAREST, oracle.MODE_BILINEAR])
def test_rounding_term_vanishes_on_untwisted_buckets(mode):
    # buckets whose texels are affine in (x, y) with one slope for all buckets:
    # dL/ds is then the same wherever s sits in its cell, and the buckets'
    # differences do not depend on s either, so moving s (or a, b: the
    # gradient is linear in them, with the same slopes) changes nothing that
    # the rounding term measures -- except a, b for dL/dview, which weigh
    # equal slopes and so also change nothing
    W, H, n, C = 4, 4, 8, 2
    rng = np.random.default_rng(80)
    y, x = np.mgrid[0:n, 0:n]
    sl = np.array([[0.03, -0.02], [0.01, 0.04]])  # [axis][channel]
    off = rng.uniform(0, 0.5, (H, W, 1, 1, C))
    T = off + sl[0] * x[..., None] + sl[1] * y[..., None]  # binary64: exactly affine
    tex = oracle.Tex(T, W, H, n, C, oracle.FMT_F64)
    T2, uv, tbn, view, g = _scale_case(81, W, H, n, C, 500)
    keep = _smooth(uv, tbn, view, W, H, n, mode)
    rv, ru = oracle.lookup_bwd_round(tex, uv, tbn, view, g, 1e-3, 1e-3, mode=mode)
    r = oracle.lookup_bwd(tex, uv, tbn, view, g, mode=mode, want_tex=False)
    gscale = np.linalg.norm(r["scale_view"], axis=1)[keep]
    assert np.all(rv[keep] <= 1e-12 * gscale + 1e-15)
    if mode == oracle.MODE_NEAREST:
        assert np.all(ru == 0)
    # a random (twisted) texture moves the gradient by an amount linear in the move
    tex2 = oracle.Tex(T2, W, H, n, C)
    a1, b1 = oracle.lookup_bwd_round(tex2, uv, tbn, view, g, 1e-4, 0.0, mode=mode)
    a2, b2 = oracle.lookup_bwd_round(tex2, uv, tbn, view, g, 2e-4, 0.0, mode=mode)
    live = keep & (a1 > 1e-9)  # both axes clamped: no view gradient to move
    assert live.sum() > 0.5 * keep.sum()
    np.testing.assert_allclose(a2[live], 2 * a1[live], rtol=1e-3)


def test_rounding_term_is_the_gradient_at_the_moved_coordinate():
    # brute force through the ordinary backward: replacing a fragment's four
    # taps by its cell's bilinear patch shifted by (sx, sy) delta (corner values
    # of the extended patch, binary64 texture) makes the plain backward return
    # the gradient at s + (sx, sy) delta with every other factor unchanged; the
    # largest change over the four shifts is the rounding term
    n, C = 8, 3
    rng = np.random.default_rng(82)
    T = rng.uniform(0, 1, (1, 1, n, n, C))
    delta = 1e-3
    _, uv, tbn, view, g = _scale_case(83, 1, 1, n, C, 40)
    idx, frac, edge = oracle.indices(uv, tbn, view, 1, 1, n)
    checked = 0
    for f in range(len(uv)):
        x0, y0 = idx[f, 2], idx[f, 3]
        if edge[f, 1] < 1e-3 or edge[f, 2] < 1e-3 or x0 >= n - 1 or y0 >= n - 1:
            continue
        one = (uv[f:f + 1], tbn[f:f + 1], view[f:f + 1], g[f:f + 1])
        base = oracle.lookup_bwd(oracle.Tex(T, 1, 1, n, C, oracle.FMT_F64), *one,
                                 want_tex=False)["grad_view"][0]
        c = T[0, 0, y0:y0 + 2, x0:x0 + 2]  # [dy, dx, C]

        def patch(u, v):
            return (1 - v) * ((1 - u) * c[0, 0] + u * c[0, 1]) + v * ((1 - u) * c[1, 0] + u * c[1, 1])
        worst = 0.0
        for sy in (-1, 1):
            for sx in (-1, 1):
                Tm = T.copy()
                du, dv = sx * delta, sy * delta
                Tm[0, 0, y0, x0] = patch(du, dv)
                Tm[0, 0, y0, x0 + 1] = patch(1 + du, dv)
                Tm[0, 0, y0 + 1, x0] = patch(du, 1 + dv)
                Tm[0, 0, y0 + 1, x0 + 1] = patch(1 + du, 1 + dv)
                moved = oracle.lookup_bwd(oracle.Tex(Tm, 1, 1, n, C, oracle.FMT_F64), *one,
                                          want_tex=False)["grad_view"][0]
                worst = max(worst, np.linalg.norm(moved - base))
        rv, _ = oracle.lookup_bwd_round(oracle.Tex(T, 1, 1, n, C, oracle.FMT_F64), *one, delta)
        assert abs(rv[0] - worst) <= 1e-9 * max(worst, 1e-12), (f, rv[0], worst)
        checked += 1
    assert checked >= 20
    # the bucket fractions: moving u, v by delta_w / W, delta_w / H moves a, b
    # by delta_w and nothing else (dyadic coordinates keep the moves exact)
    W, H = 4, 4
    T = rng.uniform(0, 1, (H, W, n, n, C)).astype(np.float32)
    tex = oracle.Tex(T, W, H, n, C)
    dw = 2.0 ** -10
    _, _, tbn, view, g = _scale_case(84, W, H, n, C, 30)
    uv = (np.round(rng.uniform(0.1, 0.9, (30, 2)) * 2 ** 16) / 2 ** 16).astype(np.float32)
    for f in range(len(uv)):
        one = lambda u: (u[None].astype(np.float32), tbn[f:f + 1], view[f:f + 1], g[f:f + 1])
        base = oracle.lookup_bwd(tex, *one(uv[f]), mode=oracle.MODE_BILINEAR, want_tex=False)
        worst_v = worst_u = 0.0
        for sb in (-1, 1):
            for sa in (-1, 1):
                u2 = uv[f].astype(np.float64) + [sa * dw / W, sb * dw / H]
                m = oracle.lookup_bwd(tex, *one(u2), mode=oracle.MODE_BILINEAR, want_tex=False)
                worst_v = max(worst_v, np.linalg.norm(m["grad_view"][0] - base["grad_view"][0]))
                worst_u = max(worst_u, np.linalg.norm(m["grad_uv"][0] - base["grad_uv"][0]))
        rv, ru = oracle.lookup_bwd_round(tex, *one(uv[f]), 0.0, dw, mode=oracle.MODE_BILINEAR)
        assert abs(rv[0] - worst_v) <= 1e-9 * max(worst_v, 1e-12)
        assert abs(ru[0] - worst_u) <= 1e-9 * max(worst_u, 1e-12)
