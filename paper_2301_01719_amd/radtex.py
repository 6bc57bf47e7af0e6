"""ctypes binding of libradtex.so (include/radtex.h) with torch tensors for
device memory and streams.

Only argument marshalling happens here: every step of the lookup, the
quantiser and the backward runs in the library's HIP kernels.  If the
library has not been built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libradtex.so")

RT_OK = 0
RT_FMT_F32, RT_FMT_BF16, RT_FMT_FP8_E4M3, RT_FMT_BIT1 = 0, 1, 2, 3
RT_LAYOUT_BUCKET_MAJOR, RT_LAYOUT_ATLAS = 0, 1
RT_BUCKET_NEAREST, RT_BUCKET_BILINEAR = 0, 1
RT_FWD_STAGE_BUCKETS = 2
RT_LIGHT_DIRECTIONAL, RT_LIGHT_POINT = 0, 1
RT_MAX_LIGHT_SAMPLES = 64

FORMATS = {"f32": RT_FMT_F32, "bf16": RT_FMT_BF16, "fp8": RT_FMT_FP8_E4M3, "bit1": RT_FMT_BIT1}
MODES = {"nearest": RT_BUCKET_NEAREST, "bilinear": RT_BUCKET_BILINEAR}
LIGHTS = {"directional": RT_LIGHT_DIRECTIONAL, "point": RT_LIGHT_POINT}
_CODE_DTYPE = {RT_FMT_F32: torch.float32, RT_FMT_BF16: torch.int16, RT_FMT_FP8_E4M3: torch.uint8,
               RT_FMT_BIT1: torch.int32}


def bit_words(n: int) -> int:
    """32-bit words per bucket of a 1-bit texture: ceil(n n / 32)."""
    return (int(n) * int(n) + 31) // 32

EXPORTS = ("rt_create_texture", "rt_destroy_texture", "rt_quantize", "rt_lookup_fwd",
           "rt_lookup_bwd_workspace", "rt_lookup_bwd", "rt_debug_indices", "rt_last_error",
           "rt_status_string", "rt_version", "rt_profile_enable", "rt_profile_reset",
           "rt_profile_kernel_count", "rt_profile_kernel_name", "rt_profile_read",
           "rt_bake_directions", "rt_bake_environment", "rt_build_mip", "rt_lookup_fwd_lod",
           "rt_lookup_light", "rt_bake_shadow", "rt_create_dictionary_texture",
           "rt_vq_assign", "rt_vq_update_workspace", "rt_vq_update",
           "rt_lookup_lod_bwd_workspace", "rt_lookup_lod_bwd", "rt_build_mip_adjoint",
           "rt_plan_workspace", "rt_plan_fragments", "rt_plan_permute",
           "rt_lookup_bwd_noalloc")


class RadtexError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class TextureDesc(ctypes.Structure):
    _fields_ = [("buckets_w", ctypes.c_int32), ("buckets_h", ctypes.c_int32),
                ("n", ctypes.c_int32), ("channels", ctypes.c_int32),
                ("format", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("data", ctypes.c_void_p), ("scales", ctypes.c_void_p)]


class DictionaryDesc(ctypes.Structure):
    _fields_ = [("buckets_w", ctypes.c_int32), ("buckets_h", ctypes.c_int32),
                ("n", ctypes.c_int32), ("channels", ctypes.c_int32),
                ("entries", ctypes.c_int32), ("format", ctypes.c_int32),
                ("index_bytes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("codebook", ctypes.c_void_p), ("index", ctypes.c_void_p),
                ("gains", ctypes.c_void_p)]


class EnvLobe(ctypes.Structure):
    _fields_ = [("axis", ctypes.c_float * 3), ("sharpness", ctypes.c_float),
                ("amplitude", ctypes.c_float * 4)]


class Light(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("samples", ctypes.c_int32),
                ("vec", (ctypes.c_float * 3) * RT_MAX_LIGHT_SAMPLES)]


class Fragments(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("views", ctypes.c_int32),
                ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("uv", ctypes.c_void_p), ("tbn", ctypes.c_void_p), ("view", ctypes.c_void_p)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2301_01719_amd/build.py "
                          "(the lookup has no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                            ctypes.c_size_t)
    sig = {
        "rt_create_texture": ([ctypes.POINTER(TextureDesc), P, ctypes.POINTER(P)], i32),
        "rt_destroy_texture": ([P], i32),
        "rt_quantize": ([P, i32, P, P, P], i32),
        "rt_lookup_fwd": ([P, ctypes.POINTER(Fragments), P, u32, P], i32),
        "rt_lookup_bwd_workspace": ([P, i64, u32], sz),
        "rt_lookup_bwd": ([P, ctypes.POINTER(Fragments), P, P, P, P, P, sz, u32, P], i32),
        "rt_debug_indices": ([P, ctypes.POINTER(Fragments), P, P, P], i32),
        "rt_plan_workspace": ([P, i64, u32], sz),
        "rt_plan_permute": ([P, i64, i32, P, P, u32, P], i32),
        "rt_lookup_bwd_noalloc": ([P, ctypes.POINTER(Fragments), P, P, P, P, u32, P], i32),
        "rt_plan_fragments": ([P, ctypes.POINTER(Fragments), u32, P, P, P, P, P, sz, P], i32),
        "rt_last_error": ([], ctypes.c_char_p),
        "rt_status_string": ([i32], ctypes.c_char_p),
        "rt_version": ([], i32),
        "rt_profile_enable": ([i32], i32),
        "rt_profile_reset": ([], i32),
        "rt_profile_kernel_count": ([], i32),
        "rt_profile_kernel_name": ([i32], ctypes.c_char_p),
        "rt_profile_read": ([i32, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)], i32),
        "rt_bake_directions": ([i32, P, P, P], i32),
        "rt_build_mip": ([P, P, P], i32),
        "rt_lookup_fwd_lod": ([ctypes.POINTER(P), i32, ctypes.POINTER(Fragments), P, P, u32, P],
                              i32),
        "rt_bake_environment": ([i32, i32, i32, i32, P, ctypes.POINTER(EnvLobe), i32,
                                 ctypes.POINTER(ctypes.c_float), P, P], i32),
        "rt_lookup_light": ([P, ctypes.POINTER(Fragments), P, ctypes.POINTER(Light), P, u32, P],
                            i32),
        "rt_bake_shadow": ([i32, i32, i32, P, P, ctypes.POINTER(ctypes.c_float), i32, P, P], i32),
        "rt_create_dictionary_texture": ([ctypes.POINTER(DictionaryDesc), ctypes.POINTER(P)], i32),
        "rt_vq_assign": ([P, i64, i32, P, i32, P, P, P], i32),
        "rt_vq_update_workspace": ([i64, i32, i32], sz),
        "rt_vq_update": ([P, i64, i32, P, i32, P, P, P, sz, P], i32),
        "rt_lookup_lod_bwd_workspace": ([ctypes.POINTER(P), i32, i64, u32], sz),
        "rt_lookup_lod_bwd": ([ctypes.POINTER(P), i32, ctypes.POINTER(Fragments), P, P,
                               ctypes.POINTER(P), P, P, P, sz, u32, P], i32),
        "rt_build_mip_adjoint": ([P, P, P, P], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


LIB = _load()


def _check(status: int):
    if status != RT_OK:
        msg = LIB.rt_last_error().decode()
        raise RadtexError(status, msg)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need_gpu(t: torch.Tensor, name: str, dtype=None):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (the lookup runs only on the GPU)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")


class Texture:
    """A radiance texture: a W x H matrix of n x n buckets with C channels.

    The handle borrows `data` (bucket-major [H, W, n, n, C]) and `scales`
    (FP8 only, [H, W]); both tensors are kept referenced by this object.
    With layout="atlas" the data is [H*n, W*n, C] and the library keeps a
    bucket-major copy.
    """

    def __init__(self, data: torch.Tensor, W: int, H: int, n: int, C: int, fmt="f32",
                 scales: Optional[torch.Tensor] = None, layout: str = "bucket"):
        self.fmt = FORMATS[fmt] if isinstance(fmt, str) else int(fmt)
        _need_gpu(data, "texture data")
        if scales is not None:
            _need_gpu(scales, "scales", torch.float32)
        self.data, self.scales = data, scales
        self.W, self.H, self.n, self.C = int(W), int(H), int(n), int(C)
        if self.fmt == RT_FMT_BIT1:
            want = W * H * bit_words(n) * 4
        else:
            want = W * H * n * n * C * [4, 2, 1][self.fmt]
        if data.numel() * data.element_size() != want:
            raise ValueError("texture data size does not match the matrix in this format")
        desc = TextureDesc(self.W, self.H, self.n, self.C, self.fmt,
                           RT_LAYOUT_ATLAS if layout == "atlas" else RT_LAYOUT_BUCKET_MAJOR,
                           data.data_ptr(), None if scales is None else scales.data_ptr())
        h = ctypes.c_void_p()
        _check(LIB.rt_create_texture(ctypes.byref(desc), _stream(data.device), ctypes.byref(h)))
        self.handle = h
        self.device = data.device

    def close(self):
        if getattr(self, "handle", None):
            LIB.rt_destroy_texture(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def bucket_elems(self) -> int:
        return self.n * self.n * self.C


class DictionaryTexture(Texture):
    """A bucket dictionary (rt_create_dictionary_texture): bucket (i, j)
    decodes to gains[j, i] (1 without gains) times codebook[index[j, i]].
    codebook [K, n, n, C] float32 or bf16 codes (int16), index [H, W] uint8,
    int16 (read as unsigned 16-bit) or int32, gains [H, W] float32 or None.
    All tensors stay referenced by this object."""

    def __init__(self, codebook: torch.Tensor, index: torch.Tensor, W: int, H: int, n: int,
                 C: int, fmt="f32", gains: Optional[torch.Tensor] = None):
        self.fmt = FORMATS[fmt] if isinstance(fmt, str) else int(fmt)
        _need_gpu(codebook, "codebook")
        _need_gpu(index, "index")
        if gains is not None:
            _need_gpu(gains, "gains", torch.float32)
        K = codebook.shape[0]
        self.data, self.scales, self.index, self.gains = codebook, None, index, gains
        self.W, self.H, self.n, self.C, self.K = int(W), int(H), int(n), int(C), int(K)
        ib = index.element_size()
        desc = DictionaryDesc(self.W, self.H, self.n, self.C, self.K, self.fmt, ib, 0,
                              codebook.data_ptr(), index.data_ptr(),
                              None if gains is None else gains.data_ptr())
        h = ctypes.c_void_p()
        _check(LIB.rt_create_dictionary_texture(ctypes.byref(desc), ctypes.byref(h)))
        self.handle = h
        self.device = codebook.device


def vq_assign(x: torch.Tensor, codebook: torch.Tensor, want_dist: bool = False):
    """Nearest codebook row of every row of x [M, D] (rt_vq_assign): returns
    assign [M] int32 and, if asked, the squared distances [M] float32."""
    _need_gpu(x, "x", torch.float32)
    _need_gpu(codebook, "codebook", torch.float32)
    M, D = x.shape
    K = codebook.shape[0]
    assign = torch.empty(M, dtype=torch.int32, device=x.device)
    dist = torch.empty(M, dtype=torch.float32, device=x.device) if want_dist else None
    _check(LIB.rt_vq_assign(_ptr(x), M, D, _ptr(codebook), K, _ptr(assign), _ptr(dist),
                            _stream(x.device)))
    return (assign, dist) if want_dist else assign


def vq_update(x: torch.Tensor, assign: torch.Tensor, codebook: torch.Tensor, workspace=None):
    """Lloyd update of codebook [K, D] in place (rt_vq_update); returns the
    counts [K] int32."""
    _need_gpu(x, "x", torch.float32)
    _need_gpu(assign, "assign", torch.int32)
    _need_gpu(codebook, "codebook", torch.float32)
    M, D = x.shape
    K = codebook.shape[0]
    need = LIB.rt_vq_update_workspace(M, D, K)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    counts = torch.empty(K, dtype=torch.int32, device=x.device)
    _check(LIB.rt_vq_update(_ptr(x), M, D, _ptr(assign), K, _ptr(codebook), _ptr(counts),
                            _ptr(workspace), workspace.numel(), _stream(x.device)))
    return counts


def _frags(uv, tbn, view, image=None) -> Fragments:
    """image = (views, height, width): the fragments are that many row-major
    images (a tiling hint, checked by the library); None: a flat list.  view
    may be None where the entry point does not read it."""
    N = uv.shape[0]
    for t, name, shape in ((uv, "uv", (N, 2)), (tbn, "tbn", (N, 3, 3)), (view, "view", (N, 3))):
        if t is None and name == "view":
            continue
        _need_gpu(t, name, torch.float32)
        if tuple(t.shape) != shape and not (name == "tbn" and tuple(t.shape) == (N, 9)):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")
    v, h, w = image if image is not None else (0, 0, 0)
    return Fragments(N, v, h, w, uv.data_ptr(), tbn.data_ptr(),
                     None if view is None else view.data_ptr())


def quantize(tex: Texture, fmt: str):
    """Per-bucket quantiser: returns (codes, scales); scales is None for BF16
    and 1-bit ("bit1": int32 words [H, W, ceil(n n/32)] of a one-channel
    texture)."""
    f = FORMATS[fmt]
    shape = (tex.H, tex.W, tex.n, tex.n, tex.C)
    if f == RT_FMT_BIT1:
        shape = (tex.H, tex.W, bit_words(tex.n))
    codes = torch.empty(shape, dtype=_CODE_DTYPE[f], device=tex.device)
    scales = (torch.empty((tex.H, tex.W), dtype=torch.float32, device=tex.device)
              if f == RT_FMT_FP8_E4M3 else None)
    _check(LIB.rt_quantize(tex.handle, f, _ptr(codes), _ptr(scales), _stream(tex.device)))
    return codes, scales


def lookup_fwd(tex: Texture, uv, tbn, view, mode: str = "nearest", out=None, image=None,
               stage_buckets: bool = False):
    """rt_lookup_fwd; stage_buckets adds RT_FWD_STAGE_BUCKETS (nearest mode)."""
    fr = _frags(uv, tbn, view, image)
    if out is None:
        out = torch.empty((fr.count, tex.C), dtype=torch.float32, device=tex.device)
    else:
        _need_gpu(out, "out", torch.float32)
    flags = MODES[mode] | (RT_FWD_STAGE_BUCKETS if stage_buckets else 0)
    _check(LIB.rt_lookup_fwd(tex.handle, ctypes.byref(fr), _ptr(out), flags,
                             _stream(tex.device)))
    return out


def bwd_workspace_bytes(tex: Texture, count: int, mode: str = "nearest") -> int:
    return int(LIB.rt_lookup_bwd_workspace(tex.handle, int(count), MODES[mode]))


def lookup_bwd(tex: Texture, uv, tbn, view, grad_out, mode: str = "nearest", want_tex=True,
               want_view=True, want_uv=True, workspace: Optional[torch.Tensor] = None,
               grad_tex: Optional[torch.Tensor] = None, image=None):
    """Returns (grad_tex [H,W,n,n,C] f32, grad_view [N,3], grad_uv [N,2]); None where
    not requested."""
    fr = _frags(uv, tbn, view, image)
    _need_gpu(grad_out, "grad_out", torch.float32)
    dev = tex.device
    N = fr.count
    gt = gv = gu = None
    if want_tex:
        gt = grad_tex if grad_tex is not None else torch.empty(
            (tex.H, tex.W, tex.n, tex.n, tex.C), dtype=torch.float32, device=dev)
    if want_view:
        gv = torch.empty((N, 3), dtype=torch.float32, device=dev)
    if want_uv:
        gu = torch.empty((N, 2), dtype=torch.float32, device=dev)
    ws_bytes = 0
    if want_tex:
        ws_bytes = bwd_workspace_bytes(tex, N, mode)
        if workspace is None or workspace.numel() < ws_bytes:
            workspace = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dev)
    _check(LIB.rt_lookup_bwd(tex.handle, ctypes.byref(fr), _ptr(grad_out), _ptr(gt), _ptr(gv),
                             _ptr(gu), _ptr(workspace) if want_tex else None,
                             ws_bytes if want_tex else 0, MODES[mode], _stream(dev)))
    return gt, gv, gu


def plan_workspace_bytes(tex: Texture, count: int, mode: str = "nearest") -> int:
    return int(LIB.rt_plan_workspace(tex.handle, int(count), MODES[mode]))


def plan_fragments(tex: Texture, uv, tbn, view, mode: str = "nearest", image=None,
                   workspace: Optional[torch.Tensor] = None, out=None):
    """Visit plan (rt_plan_fragments): returns (order [N] int32, uv, tbn, view)
    with the G-buffer in plan order; planned fragment k is the caller's
    fragment order[k].  out = (order, uv, tbn, view) preallocated, or None."""
    fr = _frags(uv, tbn, view, image)
    dev = tex.device
    N = fr.count
    if out is None:
        out = (torch.empty(N, dtype=torch.int32, device=dev),
               torch.empty((N, 2), dtype=torch.float32, device=dev),
               torch.empty((N, 3, 3), dtype=torch.float32, device=dev),
               torch.empty((N, 3), dtype=torch.float32, device=dev))
    order, puv, ptbn, pview = out
    ws_bytes = plan_workspace_bytes(tex, N, mode)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dev)
    _check(LIB.rt_plan_fragments(tex.handle, ctypes.byref(fr), MODES[mode], _ptr(order),
                                 _ptr(puv), _ptr(ptbn), _ptr(pview), _ptr(workspace),
                                 ws_bytes, _stream(dev)))
    return order, puv, ptbn, pview


def plan_permute(order: torch.Tensor, src: torch.Tensor, out=None, scatter: bool = False):
    """Rows of a per-fragment array moved by a plan's order (rt_plan_permute):
    out[k] = src[order[k]] (into plan order), or with scatter=True
    out[order[k]] = src[k] (back to the caller's order)."""
    _need_gpu(order, "order", torch.int32)
    _need_gpu(src, "src")
    N = order.numel()
    if src.shape[0] != N:
        raise ValueError("src must have one row per fragment")
    if out is None:
        out = torch.empty_like(src)
    row = src[0].numel() * src.element_size() if N else 4
    _check(LIB.rt_plan_permute(_ptr(order), N, row, _ptr(src), _ptr(out), 1 if scatter else 0,
                               _stream(src.device)))
    return out


NOALLOC_SCRATCH_BYTES = 256 << 20


def lookup_bwd_noalloc(tex: Texture, uv, tbn, view, grad_out, grad_tex, grad_view, grad_uv,
                       mode: str = "nearest", image=None):
    """rt_lookup_bwd_noalloc: the backward into caller-allocated outputs (any of
    them None to skip it), with the library's scratch as the workspace; the
    call allocates nothing."""
    fr = _frags(uv, tbn, view, image)
    _need_gpu(grad_out, "grad_out", torch.float32)
    _check(LIB.rt_lookup_bwd_noalloc(tex.handle, ctypes.byref(fr), _ptr(grad_out),
                                     _ptr(grad_tex), _ptr(grad_view), _ptr(grad_uv),
                                     MODES[mode], _stream(tex.device)))


def debug_indices(tex: Texture, uv, tbn, view, image=None):
    fr = _frags(uv, tbn, view, image)
    idx = torch.empty((fr.count, 4), dtype=torch.int32, device=tex.device)
    frac = torch.empty((fr.count, 2), dtype=torch.float32, device=tex.device)
    _check(LIB.rt_debug_indices(tex.handle, ctypes.byref(fr), _ptr(idx), _ptr(frac),
                                _stream(tex.device)))
    return idx, frac


def build_mip(tex: Texture, out=None):
    """The next level of the mip chain of an FP32 texture: [max(1, H/2),
    max(1, W/2), n, n, C], each bucket the texel-wise mean of the 2 x 2 (or 2)
    buckets it covers."""
    W2, H2 = max(1, tex.W // 2), max(1, tex.H // 2)
    if out is None:
        out = torch.empty((H2, W2, tex.n, tex.n, tex.C), dtype=torch.float32, device=tex.device)
    else:
        _need_gpu(out, "out", torch.float32)
    _check(LIB.rt_build_mip(tex.handle, _ptr(out), _stream(tex.device)))
    return out


def build_mips(tex: Texture, levels: Optional[int] = None):
    """The whole chain as Texture handles [level 0 (tex), level 1, ...]; levels
    defaults to 1 + log2(max(W, H))."""
    full = 1 + max(tex.W, tex.H).bit_length() - 1
    levels = full if levels is None else levels
    chain = [tex]
    for _ in range(1, levels):
        prev = chain[-1]
        data = build_mip(prev)
        chain.append(Texture(data, max(1, prev.W // 2), max(1, prev.H // 2), prev.n, prev.C))
    return chain


def lookup_lod_bwd_workspace(levels, count: int, mode: str = "nearest") -> int:
    """Bytes of workspace rt_lookup_lod_bwd needs for `count` fragments."""
    handles = (ctypes.c_void_p * len(levels))(*[t.handle for t in levels])
    return int(LIB.rt_lookup_lod_bwd_workspace(handles, len(levels), count, MODES[mode]))


def lookup_lod_bwd(levels, uv, tbn, view, duv, grad_out, mode: str = "nearest",
                   want_levels=True, want_view=True, want_uv=True, workspace=None, image=None):
    """Backward of lookup_fwd_lod (rt_lookup_lod_bwd): returns (per-level
    texel gradients (None where not wanted), grad_view, grad_uv)."""
    fr = _frags(uv, tbn, view, image)
    _need_gpu(duv, "duv", torch.float32)
    _need_gpu(grad_out, "grad_out", torch.float32)
    t0 = levels[0]
    dev = t0.device
    L = len(levels)
    handles = (ctypes.c_void_p * L)(*[t.handle for t in levels])
    if isinstance(want_levels, bool):
        want_levels = [want_levels] * L
    grads = [torch.empty((t.H, t.W, t.n, t.n, t.C), dtype=torch.float32, device=dev)
             if want_levels[l] else None for l, t in enumerate(levels)]
    gptr = (ctypes.c_void_p * L)(*[None if g is None else g.data_ptr() for g in grads])
    gv = torch.empty((fr.count, 3), dtype=torch.float32, device=dev) if want_view else None
    gu = torch.empty((fr.count, 2), dtype=torch.float32, device=dev) if want_uv else None
    need = lookup_lod_bwd_workspace(levels, fr.count, mode)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(LIB.rt_lookup_lod_bwd(handles, L, ctypes.byref(fr), _ptr(duv), _ptr(grad_out), gptr,
                                 _ptr(gv), _ptr(gu), _ptr(workspace), workspace.numel(),
                                 MODES[mode], _stream(dev)))
    return grads, gv, gu


def build_mip_adjoint(src: Texture, grad_dst: torch.Tensor, grad_src: torch.Tensor):
    """grad_src (level of src's shape) += the adjoint of build_mip applied to
    grad_dst (the next level's gradient); returns grad_src."""
    _need_gpu(grad_dst, "grad_dst", torch.float32)
    _need_gpu(grad_src, "grad_src", torch.float32)
    _check(LIB.rt_build_mip_adjoint(src.handle, _ptr(grad_dst), _ptr(grad_src),
                                    _stream(src.device)))
    return grad_src


def lookup_fwd_lod(levels, uv, tbn, view, duv, mode: str = "nearest", out=None, image=None):
    """Lookup over a mip chain (list of Texture, level 0 first) with the level
    of detail from duv [N, 4] = (du/dx, dv/dx, du/dy, dv/dy) per fragment."""
    fr = _frags(uv, tbn, view, image)
    _need_gpu(duv, "duv", torch.float32)
    if tuple(duv.shape) != (fr.count, 4):
        raise ValueError(f"duv has shape {tuple(duv.shape)}, expected {(fr.count, 4)}")
    t0 = levels[0]
    if out is None:
        out = torch.empty((fr.count, t0.C), dtype=torch.float32, device=t0.device)
    else:
        _need_gpu(out, "out", torch.float32)
    handles = (ctypes.c_void_p * len(levels))(*[t.handle for t in levels])
    _check(LIB.rt_lookup_fwd_lod(handles, len(levels), ctypes.byref(fr), _ptr(duv), _ptr(out),
                                 MODES[mode], _stream(t0.device)))
    return out


def bake_directions(n: int, device="cuda:0"):
    """(inc, refl) float32 [n, n, 3]: per sample centre of a bucket, the
    incidence I (Eqs. 4a, 2c) and the reflection vector R (Eqs. 4a, 4b) in
    orthogonal texture space."""
    inc = torch.empty((n, n, 3), dtype=torch.float32, device=device)
    refl = torch.empty((n, n, 3), dtype=torch.float32, device=device)
    _check(LIB.rt_bake_directions(int(n), _ptr(inc), _ptr(refl), _stream(inc.device)))
    return inc, refl


def _lobe_array(lobes):
    """lobes: a sequence of (axis xyz, sharpness, amplitudes[<=4]) or an [K, 8]
    array (axis xyz, sharpness, amplitude per channel)."""
    rows = [list(map(float, r)) for r in lobes]
    arr = (EnvLobe * max(len(rows), 1))()
    for k, r in enumerate(rows):
        if len(r) != 8:
            raise ValueError("a lobe is 8 numbers: axis x, y, z, sharpness, 4 amplitudes")
        arr[k].axis[:] = r[0:3]
        arr[k].sharpness = r[3]
        arr[k].amplitude[:] = r[4:8]
    return arr, len(rows)


def bake_environment(W: int, H: int, n: int, C: int, lobes, ambient, frames=None, out=None,
                     device="cuda:0"):
    """Bake a W x H matrix of n x n buckets (FP32 [H, W, n, n, C]) from the
    analytic environment ambient + spherical Gaussian lobes, sampled along each
    sample's reflection vector carried to scene coordinates by the bucket's
    frame (frames [H, W, 3, 3] rows T, B, N, or None: identity)."""
    if out is None:
        out = torch.empty((H, W, n, n, C), dtype=torch.float32, device=device)
    else:
        _need_gpu(out, "out", torch.float32)
    if frames is not None:
        _need_gpu(frames, "frames", torch.float32)
        if frames.numel() != H * W * 9:
            raise ValueError("frames must hold H * W frames of 3 x 3")
    arr, K = _lobe_array(lobes)
    amb = (ctypes.c_float * 4)(*[float(a) for a in ambient])
    _check(LIB.rt_bake_environment(int(W), int(H), int(n), int(C), _ptr(frames), arr, K, amb,
                                   _ptr(out), _stream(out.device)))
    return out


# --- shadowing: 1-bit textures read with the light direction -------------------

def make_light(vecs, kind: str = "directional") -> Light:
    """A light of S = len(vecs) samples (S <= 64): directions toward the light
    ("directional") or points of the light ("point"), scene space."""
    import numpy as np
    v = np.asarray(vecs, dtype=np.float32).reshape(-1, 3)
    if not 1 <= v.shape[0] <= RT_MAX_LIGHT_SAMPLES:
        raise ValueError(f"a light has 1..{RT_MAX_LIGHT_SAMPLES} samples, got {v.shape[0]}")
    L = Light()
    L.kind = LIGHTS[kind]
    L.samples = v.shape[0]
    for s in range(v.shape[0]):
        for k in range(3):
            L.vec[s][k] = float(v[s, k])
    return L


def lookup_light(tex: Texture, uv, tbn, light: Light, pos=None, mode: str = "nearest",
                 out=None, image=None):
    """Mean over the light's samples of the lookup with the direction toward
    the light in place of the view vector (rt_lookup_light); pos [N, 3] is the
    fragments' scene positions, read for point lights."""
    fr = _frags(uv, tbn, None, image)
    if pos is not None:
        _need_gpu(pos, "pos", torch.float32)
        if tuple(pos.shape) != (fr.count, 3):
            raise ValueError(f"pos has shape {tuple(pos.shape)}, expected {(fr.count, 3)}")
    if out is None:
        out = torch.empty((fr.count, tex.C), dtype=torch.float32, device=tex.device)
    else:
        _need_gpu(out, "out", torch.float32)
    _check(LIB.rt_lookup_light(tex.handle, ctypes.byref(fr), _ptr(pos), ctypes.byref(light),
                               _ptr(out), MODES[mode], _stream(tex.device)))
    return out


def bake_shadow(W: int, H: int, n: int, origins, balls, frames=None, out=None):
    """1-bit shadow texture (int32 words [H, W, ceil(n n/32)]) of the balls
    [K, 4] (centre, radius; host values) seen from the buckets' scene points
    origins [H, W, 3] with frames [H, W, 3, 3] (None: identity)."""
    import numpy as np
    _need_gpu(origins, "origins", torch.float32)
    dev = origins.device
    b = np.ascontiguousarray(np.asarray(balls, dtype=np.float32).reshape(-1, 4))
    if frames is not None:
        _need_gpu(frames, "frames", torch.float32)
    if out is None:
        out = torch.empty((H, W, bit_words(n)), dtype=torch.int32, device=dev)
    else:
        _need_gpu(out, "out", torch.int32)
    _check(LIB.rt_bake_shadow(int(W), int(H), int(n), _ptr(origins), _ptr(frames),
                              b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), b.shape[0],
                              _ptr(out), _stream(dev)))
    return out


class _LookupFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, texels, uv, view, tbn, shape, mode, scales, fmt, image):
        W, H, n, C = shape
        tex = Texture(texels, W, H, n, C, fmt, scales)
        out = lookup_fwd(tex, uv, tbn, view, mode, image=image)
        ctx.save_for_backward(texels, uv, view, tbn, scales if scales is not None else uv)
        ctx.shape, ctx.mode, ctx.fmt, ctx.has_scales = shape, mode, fmt, scales is not None
        ctx.image = image
        return out

    @staticmethod
    def backward(ctx, grad_out):
        texels, uv, view, tbn, scales = ctx.saved_tensors
        W, H, n, C = ctx.shape
        tex = Texture(texels, W, H, n, C, ctx.fmt, scales if ctx.has_scales else None)
        need_tex, need_uv, need_view = ctx.needs_input_grad[0], ctx.needs_input_grad[1], \
            ctx.needs_input_grad[2]
        gt, gv, gu = lookup_bwd(tex, uv, tbn, view, grad_out.contiguous(), ctx.mode,
                                want_tex=need_tex, want_view=need_view, want_uv=need_uv,
                                image=ctx.image)
        return gt, gu, gv, None, None, None, None, None, None


def lookup(texels: torch.Tensor, uv, tbn, view, n: int, mode: str = "nearest", fmt="f32",
           scales: Optional[torch.Tensor] = None, image=None):
    """Differentiable lookup.  texels: bucket-major [H, W, n, n, C]; gradients
    flow to texels (dense, deterministic), uv and view; none to tbn.  image =
    (views, height, width) is the optional tiling hint of the fragments."""
    H, W = texels.shape[0], texels.shape[1]
    C = texels.shape[-1]
    return _LookupFn.apply(texels, uv, view, tbn, (W, H, n, C), mode, scales, fmt, image)


# --- kernel timer -------------------------------------------------------------

def profile_enable(on: bool = True):
    _check(LIB.rt_profile_enable(1 if on else 0))


def profile_reset():
    _check(LIB.rt_profile_reset())


def profile_read() -> dict:
    """{kernel name: (launches, total ms)} for kernels launched since the reset."""
    res = {}
    for k in range(LIB.rt_profile_kernel_count()):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(LIB.rt_profile_read(k, ctypes.byref(n), ctypes.byref(ms)))
        if n.value:
            res[LIB.rt_profile_kernel_name(k).decode()] = (n.value, ms.value)
    return res
