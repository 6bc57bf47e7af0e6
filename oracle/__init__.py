"""ctypes front-end of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  It never imports the HIP library and the HIP library never
imports it.  All arrays are numpy; float32 inputs are widened exactly to
binary64 inside the C code.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

FMT_F32, FMT_BF16, FMT_FP8_E4M3, FMT_F64, FMT_BIT1 = 0, 1, 2, 3, 4
LIGHT_DIRECTIONAL, LIGHT_POINT = 0, 1
MODE_NEAREST, MODE_BILINEAR = 0, 1

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, d = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.orc_num_threads.restype = i32
    lib.orc_set_num_threads.argtypes = [i32]
    lib.orc_bf16_to_f64.argtypes = [ctypes.c_uint16]
    lib.orc_bf16_to_f64.restype = d
    lib.orc_e4m3_to_f64.argtypes = [ctypes.c_uint8]
    lib.orc_e4m3_to_f64.restype = d
    lib.orc_f32_to_bf16_rne.argtypes = [ctypes.c_float]
    lib.orc_f32_to_bf16_rne.restype = ctypes.c_uint16
    lib.orc_f32_to_e4m3_sat.argtypes = [ctypes.c_float]
    lib.orc_f32_to_e4m3_sat.restype = ctypes.c_uint8
    lib.orc_quantize.argtypes = [P, i64, i64, i32, P, P]
    for name in ("orc_equisolid_tangent", "orc_square", "orc_unsquare",
                 "orc_inverse_equisolid_tangent", "orc_reflection"):
        getattr(lib, name).argtypes = [P, P]
    lib.orc_equisolid_general.argtypes = [P, P, P]
    lib.orc_inverse_equisolid_general.argtypes = [P, P, P]
    lib.orc_texel_coord.argtypes = [P, i32, P]
    lib.orc_lookup_fwd.argtypes = [i64, P, P, P, i32, i32, i32, i32, i32, P, P, i32, P]
    lib.orc_lookup_one_f64.argtypes = [P, P, P, i32, i32, i32, i32, i32, P, P, i32, P]
    lib.orc_lookup_fwd_f64.argtypes = [i64, P, P, P, i32, i32, i32, i32, i32, P, P, i32, P]
    lib.orc_lookup_bwd_round.argtypes = [i64, P, P, P, P, i32, i32, i32, i32, i32, P, P, i32, d,
                                         d, P, P]
    lib.orc_indices.argtypes = [i64, P, P, P, i32, i32, i32, P, P, P]
    lib.orc_map_one.argtypes = [P, P, i32, P]
    lib.orc_lookup_bwd.argtypes = [i64, P, P, P, P, i32, i32, i32, i32, i32, P, P, i32,
                                   P, P, P, i32, i32, i32, i32, P, P, P, P]
    lib.orc_bake_directions.argtypes = [i32, P, P]
    lib.orc_bake_environment.argtypes = [i32, i32, i32, i32, P, P, i32, P, i32, i32, i32, i32, P]
    lib.orc_env_eval.argtypes = [P, i32, P, i32, P, P]
    lib.orc_build_mip.argtypes = [i32, i32, i32, i32, P, P]
    lib.orc_lod.argtypes = [P, i32, i32, i32]
    lib.orc_lod.restype = d
    lib.orc_lookup_lod.argtypes = [i64, P, P, P, P, i32, i32, i32, i32, i32, P, i32, P, P]
    lib.orc_lookup_lod_bwd.argtypes = [i64, P, P, P, P, P, i32, i32, i32, i32, i32, P, i32, P,
                                       P, P, P, P, P, P]
    lib.orc_build_mip_adjoint.argtypes = [i32, i32, i32, i32, P, P]
    lib.orc_pack_bits.argtypes = [P, i64, i32, P]
    lib.orc_lookup_light.argtypes = [i64, P, P, P, i32, i32, P, i32, i32, i32, i32, i32, P, P,
                                     i32, P]
    lib.orc_bake_shadow.argtypes = [i32, i32, i32, P, P, P, i32, P, P]
    lib.orc_lookup_fwd_dict.argtypes = [i64, P, P, P, i32, i32, i32, i32, i32, P, i32, P, P, i32,
                                        P]
    lib.orc_vq_assign.argtypes = [i64, i32, P, i32, P, P, P]
    lib.orc_vq_update.argtypes = [i64, i32, P, P, i32, P, P, P]
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(k: int) -> None:
    """Threads of the oracle's parallel loops from here on."""
    _load().orc_set_num_threads(int(k))


# --- scalar conversions ----------------------------------------------------

def bf16_to_f64(code: int) -> float:
    return _load().orc_bf16_to_f64(int(code))


def e4m3_to_f64(code: int) -> float:
    return _load().orc_e4m3_to_f64(int(code))


def f32_to_bf16(x: float) -> int:
    return int(_load().orc_f32_to_bf16_rne(float(np.float32(x))))


def f32_to_e4m3(x: float) -> int:
    return int(_load().orc_f32_to_e4m3_sat(float(np.float32(x))))


def quantize(tex_f32: np.ndarray, n_buckets: int, bucket_elems: int, fmt: int):
    """Per-bucket quantiser.  Returns (codes, scales-or-None)."""
    t = _c(tex_f32, np.float32).reshape(-1)
    assert t.size == n_buckets * bucket_elems
    if fmt == FMT_BF16:
        codes = np.empty(t.size, np.uint16)
        _load().orc_quantize(_p(t), n_buckets, bucket_elems, fmt, _p(codes), None)
        return codes, None
    codes = np.empty(t.size, np.uint8)
    scales = np.empty(n_buckets, np.float32)
    _load().orc_quantize(_p(t), n_buckets, bucket_elems, fmt, _p(codes), _p(scales))
    return codes, scales


# --- mapping pieces (binary64) ---------------------------------------------

def _vec_call(fn, inp, in_len, out_len):
    a = _c(inp, np.float64).reshape(-1, in_len)
    out = np.empty((a.shape[0], out_len), np.float64)
    for k in range(a.shape[0]):
        fn(_p(a[k]), _p(out[k]))
    return out


def equisolid_tangent(I):
    return _vec_call(_load().orc_equisolid_tangent, I, 3, 2)


def square(A):
    return _vec_call(_load().orc_square, A, 2, 2)


def unsquare(B):
    return _vec_call(_load().orc_unsquare, B, 2, 2)


def inverse_equisolid_tangent(A):
    return _vec_call(_load().orc_inverse_equisolid_tangent, A, 2, 3)


def reflection(A):
    return _vec_call(_load().orc_reflection, A, 2, 3)


def equisolid_general(I, N):
    I = _c(I, np.float64).reshape(-1, 3)
    N = _c(N, np.float64).reshape(-1, 3)
    out = np.empty((I.shape[0], 3))
    for k in range(I.shape[0]):
        _load().orc_equisolid_general(_p(I[k]), _p(N[k]), _p(out[k]))
    return out


def inverse_equisolid_general(A, N):
    A = _c(A, np.float64).reshape(-1, 2)
    N = _c(N, np.float64).reshape(-1, 3)
    out = np.empty((A.shape[0], 3))
    for k in range(A.shape[0]):
        _load().orc_inverse_equisolid_general(_p(A[k]), _p(N[k]), _p(out[k]))
    return out


def texel_coord(B, n):
    B = _c(B, np.float64).reshape(-1, 2)
    out = np.empty((B.shape[0], 2))
    for k in range(B.shape[0]):
        _load().orc_texel_coord(_p(B[k]), int(n), _p(out[k]))
    return out


def map_one(M, V, n):
    """(A_x, A_y, B_x, B_y, s_x, s_y) for frame M (9) and view V (3)."""
    M = _c(M, np.float64).reshape(9)
    V = _c(V, np.float64).reshape(3)
    out = np.empty(6)
    _load().orc_map_one(_p(M), _p(V), int(n), _p(out))
    return out


# --- whole lookups -----------------------------------------------------------

class Tex:
    """Texture description for the oracle (host arrays, bucket-major)."""

    def __init__(self, data, W, H, n, C, fmt=FMT_F32, scales=None):
        dt = {FMT_F32: np.float32, FMT_BF16: np.uint16, FMT_FP8_E4M3: np.uint8,
              FMT_F64: np.float64, FMT_BIT1: np.uint32}[fmt]
        self.data = _c(data, dt).reshape(-1)
        if fmt == FMT_BIT1:
            assert C == 1 and self.data.size == W * H * words_per_bucket(n), (self.data.size, n)
        else:
            assert self.data.size == W * H * n * n * C, (self.data.size, W, H, n, C)
        self.W, self.H, self.n, self.C, self.fmt = int(W), int(H), int(n), int(C), fmt
        self.scales = None if scales is None else _c(scales, np.float32).reshape(-1)
        if fmt == FMT_FP8_E4M3:
            assert self.scales is not None and self.scales.size == W * H

    def args(self):
        return (self.W, self.H, self.n, self.C, self.fmt, _p(self.data), _p(self.scales))


def _frags(uv, tbn, view):
    uv = _c(uv, np.float32).reshape(-1, 2)
    tbn = _c(tbn, np.float32).reshape(-1, 9)
    view = _c(view, np.float32).reshape(-1, 3)
    assert uv.shape[0] == tbn.shape[0] == view.shape[0]
    return uv, tbn, view


def lookup_fwd(tex: Tex, uv, tbn, view, mode=MODE_NEAREST):
    uv, tbn, view = _frags(uv, tbn, view)
    N = uv.shape[0]
    out = np.empty((N, tex.C), np.float64)
    _load().orc_lookup_fwd(N, _p(uv), _p(tbn), _p(view), *tex.args(), int(mode), _p(out))
    return out


def lookup_one_f64(tex: Tex, U, M, V, mode=MODE_NEAREST):
    U = _c(U, np.float64).reshape(2)
    M = _c(M, np.float64).reshape(9)
    V = _c(V, np.float64).reshape(3)
    out = np.empty(tex.C, np.float64)
    _load().orc_lookup_one_f64(_p(U), _p(M), _p(V), *tex.args(), int(mode), _p(out))
    return out


def lookup_fwd_f64(tex: Tex, U, M, V, mode=MODE_NEAREST):
    """Forward lookup of N fragments whose u,v [N,2], frames [N,3,3] and view
    vectors [N,3] are binary64 (finite differences); out [N,C] float64."""
    U = _c(U, np.float64).reshape(-1, 2)
    M = _c(M, np.float64).reshape(-1, 9)
    V = _c(V, np.float64).reshape(-1, 3)
    N = U.shape[0]
    assert M.shape[0] == N and V.shape[0] == N
    out = np.empty((N, tex.C), np.float64)
    _load().orc_lookup_fwd_f64(N, _p(U), _p(M), _p(V), *tex.args(), int(mode), _p(out))
    return out


def indices(uv, tbn, view, W, H, n):
    """Returns idx [N,4] int32 (i, j, x0, y0), frac [N,2] and edge [N,3]:
    distances to the nearest bucket edge, sample edge (clamp bounds included)
    and to the diagonal |A_x| = |A_y|."""
    uv, tbn, view = _frags(uv, tbn, view)
    N = uv.shape[0]
    idx = np.empty((N, 4), np.int32)
    frac = np.empty((N, 2), np.float64)
    edge = np.empty((N, 3), np.float64)
    _load().orc_indices(N, _p(uv), _p(tbn), _p(view), int(W), int(H), int(n), _p(idx),
                        _p(frac), _p(edge))
    return idx, frac, edge


def lookup_bwd(tex: Tex, uv, tbn, view, g, mode=MODE_NEAREST, want_tex=True, window=None,
               want_view=True, want_uv=True, want_abs=True):
    """Analytic backward in binary64.

    window = (bi0, bj0, bw, bh) restricts grad_tex to that bucket rectangle
    (default: the whole matrix).  Returns dict with grad_tex [bh,bw,n,n,C],
    abs_tex (sum of |w g|), absg_tex (sum of |g| over the taps touching the
    element; both left out with want_abs=False), grad_view [N,3], grad_uv
    [N,2], and scale_view / scale_uv (the chain rule evaluated with
    magnitudes); entries are None when not asked.
    """
    uv, tbn, view = _frags(uv, tbn, view)
    g = _c(g, np.float32).reshape(-1, tex.C)
    N = uv.shape[0]
    assert g.shape[0] == N
    if window is None:
        window = (0, 0, tex.W, tex.H)
    bi0, bj0, bw, bh = (int(x) for x in window)
    gt = at = ag = gv = gu = sv = su = None
    if want_tex:
        gt = np.empty((bh, bw, tex.n, tex.n, tex.C), np.float64)
        if want_abs:
            at = np.empty_like(gt)
            ag = np.empty_like(gt)
    if want_view:
        gv = np.empty((N, 3), np.float64)
        sv = np.empty((N, 3), np.float64)
    if want_uv:
        gu = np.empty((N, 2), np.float64)
        su = np.empty((N, 2), np.float64)
    _load().orc_lookup_bwd(N, _p(uv), _p(tbn), _p(view), _p(g), *tex.args(), int(mode),
                           _p(gt), _p(at), _p(ag), bi0, bj0, bw, bh, _p(gv), _p(gu), _p(sv),
                           _p(su))
    return {"grad_tex": gt, "abs_tex": at, "absg_tex": ag, "grad_view": gv, "grad_uv": gu,
            "scale_view": sv, "scale_uv": su}


def lookup_bwd_round(tex: Tex, uv, tbn, view, g, delta_s, delta_w=0.0, mode=MODE_NEAREST):
    """Per fragment, how far the exact view and uv gradients move when the
    sample coordinate s moves by +-delta_s along each axis and (bilinear-bucket
    mode) the bucket fractions a, b by +-delta_w, everything else held: the
    largest 2-norm change over the sign patterns.  This is the part of a
    binary32 gradient's error that the rounding of those quantities alone
    causes.  Returns (round_view [N], round_uv [N]) float64."""
    uv, tbn, view = _frags(uv, tbn, view)
    g = _c(g, np.float32).reshape(-1, tex.C)
    N = uv.shape[0]
    assert g.shape[0] == N
    rv = np.empty(N, np.float64)
    ru = np.empty(N, np.float64)
    _load().orc_lookup_bwd_round(N, _p(uv), _p(tbn), _p(view), _p(g), *tex.args(), int(mode),
                                 float(delta_s), float(delta_w), _p(rv), _p(ru))
    return rv, ru


# --- the bake ----------------------------------------------------------------

def bake_directions(n):
    """(inc, refl) [n, n, 3] float64: per sample centre of a bucket, the
    incidence I (Eqs. (4a), (2c)) and the reflection vector R (Eqs. (4a),
    (4b)) in orthogonal texture space; [y, x] indexing."""
    inc = np.empty((n, n, 3), np.float64)
    refl = np.empty((n, n, 3), np.float64)
    _load().orc_bake_directions(int(n), _p(inc), _p(refl))
    return inc, refl


def _lobes(lobes, ambient):
    lobes = _c(lobes, np.float32).reshape(-1, 8)
    ambient = _c(ambient, np.float32).reshape(4)
    return lobes, ambient


def bake_environment(W, H, n, C, lobes, ambient, frames=None, window=None):
    """Baked texels [bh, bw, n, n, C] float64 of the bucket window (default:
    all): env(normalize(M^T R)) per sample centre.  lobes [K, 8] float32 (axis
    xyz, sharpness, amplitude per channel 0..3), ambient [4]; frames [H, W, 3,
    3] float32 rows T, B, N, or None for the identity."""
    lobes, ambient = _lobes(lobes, ambient)
    if frames is not None:
        frames = _c(frames, np.float32).reshape(H * W * 9)
    bi0, bj0, bw, bh = window if window is not None else (0, 0, W, H)
    out = np.empty((bh, bw, n, n, C), np.float64)
    _load().orc_bake_environment(int(W), int(H), int(n), int(C), _p(frames), _p(lobes),
                                 lobes.shape[0], _p(ambient), int(bi0), int(bj0), int(bw),
                                 int(bh), _p(out))
    return out


def env_eval(lobes, ambient, C, d):
    """env_c at directions d [..., 3] (normalised inside): [..., C] float64."""
    lobes, ambient = _lobes(lobes, ambient)
    d = _c(d, np.float64).reshape(-1, 3)
    out = np.empty((d.shape[0], C), np.float64)
    for r in range(d.shape[0]):
        _load().orc_env_eval(_p(lobes), lobes.shape[0], _p(ambient), int(C),
                             _p(d[r]), _p(out[r]))
    return out


# --- minification: mip chain and level-of-detail lookup ----------------------

def level_dims(W, H, l):
    return max(1, W >> l), max(1, H >> l)


def build_mips(tex, W, H, n, C, levels):
    """The mip chain [level 0 (as float64), level 1, ...] of a bucket-major
    texture [H, W, n, n, C] (W, H powers of two)."""
    cur = np.ascontiguousarray(np.asarray(tex, np.float64).reshape(H, W, n, n, C))
    out = [cur]
    for l in range(1, levels):
        w, h = level_dims(W, H, l - 1)
        w2, h2 = level_dims(W, H, l)
        nxt = np.empty((h2, w2, n, n, C), np.float64)
        _load().orc_build_mip(w, h, int(n), int(C), _p(cur), _p(nxt))
        out.append(nxt)
        cur = nxt
    return out


def lod(duv, W, H, levels):
    duv = _c(duv, np.float64).reshape(4)
    return float(_load().orc_lod(_p(duv), int(W), int(H), int(levels)))


def lookup_lod(chain, uv, tbn, view, duv, W, H, n, C, mode=MODE_NEAREST):
    """Trilinear lookup over the mip chain (list of float64 levels).  Returns
    (out [N, C] float64, lambda [N])."""
    uv, tbn, view = _frags(uv, tbn, view)
    duv = _c(duv, np.float32).reshape(-1, 4)
    N = uv.shape[0]
    assert duv.shape[0] == N
    flat = np.ascontiguousarray(np.concatenate([np.asarray(c, np.float64).reshape(-1)
                                                for c in chain]))
    out = np.empty((N, C), np.float64)
    lam = np.empty(N, np.float64)
    _load().orc_lookup_lod(N, _p(uv), _p(tbn), _p(view), _p(duv), int(W), int(H), int(n),
                           int(C), len(chain), _p(flat), int(mode), _p(out), _p(lam))
    return out, lam


def lookup_lod_bwd(chain, uv, tbn, view, duv, g, W, H, n, C, mode=MODE_NEAREST, full=False):
    """Backward of the trilinear lookup over the mip chain (list of float64
    levels) for upstream g [N, C] float32: (list of per-level gradients,
    grad_view [N, 3], grad_uv [N, 2]), all float64.  With full=True a dict
    that also holds the per-level magnitude sums abs / absg (as in
    lookup_bwd) and scale_view / scale_uv."""
    uv, tbn, view = _frags(uv, tbn, view)
    duv = _c(duv, np.float32).reshape(-1, 4)
    g = _c(g, np.float32).reshape(-1, C)
    N = uv.shape[0]
    flat = np.ascontiguousarray(np.concatenate([np.asarray(c, np.float64).reshape(-1)
                                                for c in chain]))
    gchain, achain, bchain = (np.empty_like(flat) for _ in range(3))
    gv, sv = np.empty((N, 3), np.float64), np.empty((N, 3), np.float64)
    gu, su = np.empty((N, 2), np.float64), np.empty((N, 2), np.float64)
    _load().orc_lookup_lod_bwd(N, _p(uv), _p(tbn), _p(view), _p(duv), _p(g), int(W), int(H),
                               int(n), int(C), len(chain), _p(flat), int(mode), _p(gchain),
                               _p(achain), _p(bchain), _p(gv), _p(gu), _p(sv), _p(su))

    def split(a):
        out, off = [], 0
        for c in chain:
            k = np.asarray(c).size
            out.append(a[off:off + k].reshape(np.asarray(c).shape))
            off += k
        return out
    if full:
        return {"grad": split(gchain), "abs": split(achain), "absg": split(bchain),
                "grad_view": gv, "grad_uv": gu, "scale_view": sv, "scale_uv": su}
    return split(gchain), gv, gu


def build_mip_adjoint(grad_dst, W, H, n, C, grad_src=None):
    """Adds the adjoint of one chain level (level W x H -> the next) applied to
    grad_dst into grad_src (zeros if None); returns grad_src (float64)."""
    gd = _c(grad_dst, np.float64)
    gs = np.zeros((H, W, n, n, C), np.float64) if grad_src is None else grad_src
    assert gs.dtype == np.float64 and gs.flags.c_contiguous
    _load().orc_build_mip_adjoint(int(W), int(H), int(n), int(C), _p(gd), _p(gs))
    return gs


# --- shadowing: 1-bit textures and the light-direction lookup -------------------

def words_per_bucket(n):
    """32-bit words of one bucket of the 1-bit storage: ceil(n n / 32)."""
    return (int(n) * int(n) + 31) // 32


def pack_bits(tex, n):
    """1-bit storage of a one-channel texture [..., n, n] (or [..., n, n, 1])
    float32: per bucket, sample k = y n + x is bit k % 32 of word k / 32, set
    iff the value is >= 1/2; returns uint32 words [buckets * ceil(n n/32)]."""
    t = _c(tex, np.float32).reshape(-1)
    nn = int(n) * int(n)
    assert t.size % nn == 0
    nb = t.size // nn
    out = np.empty(nb * words_per_bucket(n), np.uint32)
    _load().orc_pack_bits(_p(t), nb, nn, _p(out))
    return out


def lookup_light(tex: Tex, uv, tbn, vec, kind=LIGHT_DIRECTIONAL, pos=None, mode=MODE_NEAREST):
    """Mean over the light samples of the lookup taken with the direction
    toward the light: vec [S, 3] float32 holds directions (directional light)
    or sample points (point light; L = vec[s] - pos[f], pos [N, 3] float32).
    Returns [N, C] float64."""
    uv = _c(uv, np.float32).reshape(-1, 2)
    tbn = _c(tbn, np.float32).reshape(-1, 9)
    vec = _c(vec, np.float32).reshape(-1, 3)
    N = uv.shape[0]
    if kind == LIGHT_POINT:
        pos = _c(pos, np.float32).reshape(-1, 3)
        assert pos.shape[0] == N
    else:
        pos = None
    out = np.empty((N, tex.C), np.float64)
    _load().orc_lookup_light(N, _p(uv), _p(tbn), _p(pos), int(kind), vec.shape[0], _p(vec),
                             *tex.args(), int(mode), _p(out))
    return out


def bake_shadow(W, H, n, origins, spheres, frames=None):
    """1-bit shadow texture of analytic occluders: (words [H W ceil(n n/32)]
    uint32, margin [H, W, n, n] float64).  origins [H, W, 3] float32 scene
    points of the buckets, spheres [K, 4] float32 (centre, radius), frames
    [H, W, 3, 3] float32 rows T, B, N or None (identity)."""
    origins = _c(origins, np.float32).reshape(H * W * 3)
    spheres = _c(spheres, np.float32).reshape(-1, 4)
    if frames is not None:
        frames = _c(frames, np.float32).reshape(H * W * 9)
    words = np.empty(W * H * words_per_bucket(n), np.uint32)
    margin = np.empty((H, W, n, n), np.float64)
    _load().orc_bake_shadow(int(W), int(H), int(n), _p(origins), _p(frames), _p(spheres),
                            spheres.shape[0], _p(words), _p(margin))
    return words, margin


# --- bucket dictionary: codebook + index map (+ gains), and Lloyd's steps ---------

def lookup_fwd_dict(codebook, K, index, gains, W, H, n, C, uv, tbn, view, fmt=FMT_F32,
                    mode=MODE_NEAREST):
    """Lookup on a dictionary texture: bucket b decodes to gains[b] (1 if
    gains is None) times codebook entry index[b]; codebook [K, n, n, C] in
    FMT_F32 (float32) or FMT_BF16 (uint16 codes)."""
    dt = {FMT_F32: np.float32, FMT_BF16: np.uint16}[fmt]
    cb = _c(codebook, dt).reshape(-1)
    assert cb.size == K * n * n * C
    idx = _c(index, np.int32).reshape(-1)
    assert idx.size == W * H and idx.min() >= 0 and idx.max() < K
    g = None if gains is None else _c(gains, np.float32).reshape(-1)
    uv, tbn, view = _frags(uv, tbn, view)
    N = uv.shape[0]
    out = np.empty((N, C), np.float64)
    _load().orc_lookup_fwd_dict(N, _p(uv), _p(tbn), _p(view), int(W), int(H), int(n), int(C),
                                int(fmt), _p(cb), int(K), _p(idx), _p(g), int(mode), _p(out))
    return out


def vq_assign(X, codebook):
    """Nearest entry of every row of X [M, D] float32 among codebook [K, D]
    float32 (squared distance in binary64, ties to the smallest index):
    (assign [M] int32, dist [M] float64)."""
    X = _c(X, np.float32)
    cb = _c(codebook, np.float32)
    M, D = X.shape
    K = cb.shape[0]
    assert cb.shape[1] == D
    a = np.empty(M, np.int32)
    d = np.empty(M, np.float64)
    _load().orc_vq_assign(M, D, _p(X), K, _p(cb), _p(a), _p(d))
    return a, d


def vq_update(X, assign, codebook):
    """Lloyd update: (entries [K, D] float64 = mean of the assigned rows, or
    the previous entry when none is assigned; counts [K] int64)."""
    X = _c(X, np.float32)
    cb = _c(codebook, np.float32)
    a = _c(assign, np.int32)
    M, D = X.shape
    K = cb.shape[0]
    out = np.empty((K, D), np.float64)
    cnt = np.empty(K, np.int64)
    _load().orc_vq_update(M, D, _p(X), _p(a), K, _p(cb), _p(out), _p(cnt))
    return out, cnt
