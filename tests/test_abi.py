"""The C ABI of libradtex.so, without a GPU: the library loads, exports every
function include/radtex.h declares, and rejects bad arguments on the host
before anything is enqueued (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "radtex.h")
LIB = os.path.join(ROOT, "paper_2301_01719_amd", "libradtex.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def rt():
    if not os.path.exists(LIB):
        pytest.fail("libradtex.so is not built (run __graft_entry__.build())")
    from paper_2301_01719_amd import radtex
    return radtex


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("rt_create_texture", "rt_destroy_texture", "rt_quantize", "rt_lookup_fwd",
                     "rt_lookup_bwd", "rt_lookup_bwd_workspace", "rt_debug_indices",
                     "rt_last_error", "rt_plan_workspace", "rt_plan_fragments"):
        assert required in names


def test_library_exports_every_declared_symbol(rt):
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(rt.EXPORTS) <= set(_declared())


def test_version_and_status_strings(rt):
    assert rt.LIB.rt_version() == 201
    assert rt.LIB.rt_status_string(0) == b"RT_OK"
    assert rt.LIB.rt_status_string(4) == b"RT_ERR_WORKSPACE_TOO_SMALL"
    assert rt.LIB.rt_profile_kernel_count() >= 10
    assert rt.LIB.rt_profile_kernel_name(0) == b"k_lookup_fwd"


def _fr(rt, count, uv, tbn, view, image=(0, 0, 0)):
    v, h, w = image
    return rt.Fragments(count=count, views=v, height=h, width=w, uv=uv, tbn=tbn, view=view)


def _desc(rt, **kw):
    d = dict(buckets_w=4, buckets_h=4, n=8, channels=4, format=0, layout=0, data=0x10000,
             scales=None)
    d.update(kw)
    return rt.TextureDesc(**d)


@pytest.mark.parametrize("kw,status,text", [
    (dict(buckets_w=0), 1, "bucket matrix"),
    (dict(buckets_h=-3), 1, "bucket matrix"),
    (dict(buckets_w=70000), 2, "exceeds"),
    (dict(n=0), 1, "angular resolution"),
    (dict(n=65), 2, "exceeds 64"),
    (dict(channels=5), 1, "channels"),
    (dict(channels=0), 1, "channels"),
    (dict(format=7), 1, "format"),
    (dict(layout=2), 1, "layout"),
    (dict(data=None), 1, "data is NULL"),
    (dict(data=0x10004), 1, "16-byte"),
    (dict(format=2), 1, "scales"),
    (dict(format=2, scales=0x20002), 1, "4-byte"),
    (dict(format=1, scales=0x20000), 1, "must be NULL"),
])
def test_create_texture_validation(rt, kw, status, text):
    h = ctypes.c_void_p()
    st = rt.LIB.rt_create_texture(ctypes.byref(_desc(rt, **kw)), None, ctypes.byref(h))
    assert st == status
    assert text in rt.LIB.rt_last_error().decode()
    assert not h.value


def test_null_arguments(rt):
    h = ctypes.c_void_p()
    assert rt.LIB.rt_create_texture(None, None, ctypes.byref(h)) == 1
    assert rt.LIB.rt_create_texture(ctypes.byref(_desc(rt)), None, None) == 1
    fr = _fr(rt, 10, 0x1000, 0x2000, 0x3000)
    assert rt.LIB.rt_lookup_fwd(None, ctypes.byref(fr), 0x4000, 0, None) == 1
    assert "texture handle" in rt.LIB.rt_last_error().decode()
    assert rt.LIB.rt_quantize(None, 1, 0x1000, None, None) == 1
    assert rt.LIB.rt_debug_indices(None, ctypes.byref(fr), 0x1000, 0x2000, None) == 1
    assert rt.LIB.rt_lookup_bwd(None, ctypes.byref(fr), 0x1000, 0x2000, None, None, 0x3000, 1 << 20,
                                0, None) == 1
    assert rt.LIB.rt_lookup_bwd_workspace(None, 10, 0) == 0
    assert rt.LIB.rt_plan_fragments(None, ctypes.byref(fr), 0, 0x1000, 0x2000, 0x3000, 0x4000,
                                    0x5000, 1 << 20, None) == 1
    assert "texture handle" in rt.LIB.rt_last_error().decode()
    assert rt.LIB.rt_plan_workspace(None, 10, 0) == 0
    assert rt.LIB.rt_destroy_texture(None) == 0


def test_no_device_or_texture_handle(rt):
    """Without a GPU a valid description is refused with RT_ERR_NO_DEVICE; with
    one, the handle (host metadata only: the data pointer is never touched for
    bucket-major layout) is used to exercise the remaining validation."""
    h = ctypes.c_void_p()
    st = rt.LIB.rt_create_texture(ctypes.byref(_desc(rt)), None, ctypes.byref(h))
    if st == 5:
        assert "no HIP device" in rt.LIB.rt_last_error().decode()
        return
    assert st == 0 and h.value
    try:
        L = rt.LIB
        good = _fr(rt, 10, 0x1000, 0x2000, 0x3000)
        # fragments
        for fr, text in ((_fr(rt, -1, 0x1000, 0x2000, 0x3000), "< 0"),
                         (_fr(rt, 10, None, 0x2000, 0x3000), "non-NULL"),
                         (_fr(rt, 10, 0x1004, 0x2000, 0x3000), "8-byte"),
                         (_fr(rt, 10, 0x1000, 0x2001, 0x3000), "4-byte"),
                         (_fr(rt, 1 << 31, 0x1000, 0x2000, 0x3000), "2^31"),
                         (_fr(rt, 10, 0x1000, 0x2000, 0x3000, (1, 2, 0)), "all three"),
                         (_fr(rt, 10, 0x1000, 0x2000, 0x3000, (1, -2, 5)), "all three"),
                         (_fr(rt, 10, 0x1000, 0x2000, 0x3000, (1, 2, 6)), "does not match")):
            st = L.rt_lookup_fwd(h, ctypes.byref(fr), 0x4000, 0, None)
            assert st in (1, 2) and text in L.rt_last_error().decode()
        assert L.rt_lookup_fwd(h, ctypes.byref(good), None, 0, None) == 1
        assert L.rt_lookup_fwd(h, ctypes.byref(good), 0x4008, 0, None) == 1  # C=4 needs 16 B
        assert L.rt_lookup_fwd(h, ctypes.byref(good), 0x4000, 7, None) == 1  # flags
        # quantiser
        assert L.rt_quantize(h, 0, 0x4000, None, None) == 1
        assert L.rt_quantize(h, 2, 0x4000, None, None) == 1
        assert L.rt_quantize(h, 1, 0x4000, 0x5000, None) == 1
        assert L.rt_quantize(h, 1, 0x4004, None, None) == 1
        # backward: workspace size and checks
        need = L.rt_lookup_bwd_workspace(h, 10, 0)
        assert need > 0 and need % 256 == 0
        # four records per fragment in the bilinear-bucket mode (once the
        # records, not the fixed counters, dominate the size)
        assert L.rt_lookup_bwd_workspace(h, 10000, 1) > L.rt_lookup_bwd_workspace(h, 10000, 0)
        st = L.rt_lookup_bwd(h, ctypes.byref(good), 0x6000, 0x7000, None, None, 0x8000, need - 1,
                             0, None)
        assert st == 4 and "needed" in L.rt_last_error().decode()
        st = L.rt_lookup_bwd(h, ctypes.byref(good), 0x6000, 0x7000, None, None, 0x8010, need, 0,
                             None)
        assert st == 1 and "256-byte" in L.rt_last_error().decode()
        st = L.rt_lookup_bwd(h, ctypes.byref(good), None, 0x7000, None, None, 0x8000, need, 0,
                             None)
        assert st == 1 and "grad_out" in L.rt_last_error().decode()
        st = L.rt_lookup_bwd(h, ctypes.byref(good), 0x6000, 0x7004, None, None, 0x8000, need, 0,
                             None)
        assert st == 1 and "grad_tex" in L.rt_last_error().decode()
        # nothing requested: OK without launching anything
        assert L.rt_lookup_bwd(h, ctypes.byref(good), 0x6000, None, None, None, None, 0, 0,
                               None) == 0
        assert L.rt_debug_indices(h, ctypes.byref(good), 0x1004, 0x2000, None) == 1
    finally:
        L.rt_destroy_texture(h)


def test_backward_limits_are_reported(rt):
    """The sort key W*H*n*n must fit 32 bits: the workspace query returns 0 and
    the backward RT_ERR_UNSUPPORTED, decided on the host."""
    h = ctypes.c_void_p()
    d = _desc(rt, buckets_w=65536, buckets_h=65536, n=32)
    st = rt.LIB.rt_create_texture(ctypes.byref(d), None, ctypes.byref(h))
    if st == 5:
        pytest.skip("no device: handle creation refused before the limit check")
    assert st == 0
    try:
        assert rt.LIB.rt_lookup_bwd_workspace(h, 10, 0) == 0
        fr = _fr(rt, 10, 0x1000, 0x2000, 0x3000)
        st = rt.LIB.rt_lookup_bwd(h, ctypes.byref(fr), 0x6000, 0x7000, None, None, 0x8000,
                                  1 << 30, 0, None)
        assert st == 2
    finally:
        rt.LIB.rt_destroy_texture(h)


def test_product_path_refuses_cpu_tensors(rt):
    import torch
    with pytest.raises(ValueError, match="GPU tensor"):
        rt.Texture(torch.zeros(4 * 4 * 8 * 8 * 4), 4, 4, 8, 4)


def test_bake_validation(rt):
    """The bake entries reject bad arguments on the host; the placeholder
    pointers are never dereferenced because every call here fails before a
    launch (the one well-formed call runs only where no device is visible)."""
    import math
    import torch
    L = rt.LIB
    amb = (ctypes.c_float * 4)(0.1, 0.2, 0.3, 0.4)

    def call(W=4, H=3, n=8, C=4, frames=None, lobes=((0, 0, 1, 2, 1, 1, 1, 1),), nlobes=None,
             ambient=amb, texels=0x10000):
        arr, K = rt._lobe_array(lobes)
        return L.rt_bake_environment(W, H, n, C, frames, arr, K if nlobes is None else nlobes,
                                     ambient, texels, None)

    for kw, status, text in (
            (dict(W=0), 1, "bucket matrix"), (dict(H=70000), 2, "exceeds"),
            (dict(n=0), 1, "angular resolution"), (dict(n=65), 2, "exceeds 64"),
            (dict(C=0), 1, "channels"), (dict(C=5), 1, "channels"),
            (dict(nlobes=17), 2, "exceeds 16"), (dict(nlobes=-1), 1, "< 0"),
            (dict(ambient=None), 1, "ambient"), (dict(texels=None), 1, "texels is NULL"),
            (dict(texels=0x10004), 1, "16-byte"), (dict(C=2, texels=0x10004), 1, "8-byte"),
            (dict(frames=0x2002), 1, "frames"),
            (dict(lobes=((0, 0, 0, 2, 1, 1, 1, 1),)), 1, "axis"),
            (dict(lobes=((0, 0, 1, -1, 1, 1, 1, 1),)), 1, "sharpness"),
            (dict(lobes=((0, 0, 1, math.inf, 1, 1, 1, 1),)), 1, "sharpness"),
            (dict(lobes=((0, 0, 1, 1, 1, math.nan, 1, 1),)), 1, "amplitude")):
        assert call(**kw) == status, kw
        assert text in L.rt_last_error().decode(), (kw, L.rt_last_error())
    assert L.rt_bake_directions(0, 0x1000, 0x2000, None) == 1
    assert L.rt_bake_directions(65, 0x1000, 0x2000, None) == 2
    assert L.rt_bake_directions(8, 0x1002, None, None) == 1
    assert L.rt_bake_directions(8, None, None, None) == 0  # nothing asked, nothing launched
    if not torch.cuda.is_available():
        assert call() == 5 and "no HIP device" in L.rt_last_error().decode()


def test_mip_entries_reject_bad_arguments(rt):
    L = rt.LIB
    assert L.rt_build_mip(None, 0x1000, None) == 1
    assert "texture handle" in L.rt_last_error().decode()
    fr = _fr(rt, 10, 0x1000, 0x2000, 0x3000)
    assert L.rt_lookup_fwd_lod(None, 1, ctypes.byref(fr), 0x4000, 0x5000, 0, None) == 1
    lv = (ctypes.c_void_p * 2)(None, None)
    assert L.rt_lookup_fwd_lod(lv, 0, ctypes.byref(fr), 0x4000, 0x5000, 0, None) == 1
    assert L.rt_lookup_fwd_lod(lv, 18, ctypes.byref(fr), 0x4000, 0x5000, 0, None) == 2
    assert L.rt_lookup_fwd_lod(lv, 2, ctypes.byref(fr), 0x4000, 0x5000, 0, None) == 1
    assert "level 0 is NULL" in L.rt_last_error().decode()


def test_lod_backward_entries_reject_bad_arguments(rt):
    """Host checks of the level-of-detail backward and the chain adjoint, made
    before any device work."""
    L = rt.LIB
    fr = _fr(rt, 10, 0x1000, 0x2000, 0x3000)
    gl = (ctypes.c_void_p * 2)(None, None)

    def bwd(levels, nlevels, duv=0x4000, grad_out=0x5000, grads=gl):
        return L.rt_lookup_lod_bwd(levels, nlevels, ctypes.byref(fr), duv, grad_out, grads,
                                   None, None, None, 0, 0, None)

    assert bwd(None, 1) == 1 and "levels is NULL" in L.rt_last_error().decode()
    lv = (ctypes.c_void_p * 2)(None, None)
    assert bwd(lv, 0) == 1 and "< 1" in L.rt_last_error().decode()
    assert bwd(lv, 18) == 2 and "exceeds" in L.rt_last_error().decode()
    assert bwd(lv, 2) == 1 and "level 0 is NULL" in L.rt_last_error().decode()
    # the workspace query answers 0 for arguments it cannot plan
    assert L.rt_lookup_lod_bwd_workspace(None, 1, 10, 0) == 0
    assert L.rt_lookup_lod_bwd_workspace(lv, 0, 10, 0) == 0
    assert L.rt_lookup_lod_bwd_workspace(lv, 2, 10, 0) == 0
    assert L.rt_lookup_lod_bwd_workspace(lv, 1, -1, 0) == 0
    assert L.rt_build_mip_adjoint(None, 0x1000, 0x2000, None) == 1
    assert "texture handle" in L.rt_last_error().decode()


def test_one_bit_texture_descriptors(rt):
    """1-bit textures: one channel, bucket-major, no scales (host checks made
    before the device is looked for)."""
    L = rt.LIB
    h = ctypes.c_void_p()
    for kw, status, text in ((dict(format=3, channels=4), 1, "one channel"),
                             (dict(format=3, channels=1, layout=1), 2, "bucket-major"),
                             (dict(format=3, channels=1, scales=0x2000), 1, "scales"),
                             (dict(format=4, channels=1), 1, "unknown format")):
        d = _desc(rt, **kw)
        assert L.rt_create_texture(ctypes.byref(d), None, ctypes.byref(h)) == status, kw
        assert text in L.rt_last_error().decode(), (kw, L.rt_last_error())


def test_shadow_bake_validation(rt):
    import math
    import torch
    L = rt.LIB

    def call(W=4, H=3, n=8, origins=0x1000, frames=None, balls=((0, 0, 2, 1),), nballs=None,
             words=0x3000):
        import numpy as np
        b = np.ascontiguousarray(np.asarray(balls, np.float32).reshape(-1, 4))
        ptr = b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if b.size else None
        return L.rt_bake_shadow(W, H, n, origins, frames, ptr,
                                b.shape[0] if nballs is None else nballs, words, None)

    for kw, status, text in (
            (dict(W=0), 1, "bucket matrix"), (dict(H=70000), 2, "exceeds"),
            (dict(n=0), 1, "angular resolution"), (dict(n=65), 2, "exceeds 64"),
            (dict(nballs=65), 2, "exceeds 64"), (dict(nballs=-1), 1, "< 0"),
            (dict(balls=(), nballs=2), 1, "balls is NULL"),
            (dict(origins=None), 1, "origins"), (dict(words=None), 1, "words"),
            (dict(origins=0x1002), 1, "aligned"), (dict(frames=0x2001), 1, "aligned"),
            (dict(words=0x3002), 1, "aligned"),
            (dict(balls=((0, 0, 2, 0),)), 1, "radius"), (dict(balls=((0, 0, 2, -1),)), 1, "radius"),
            (dict(balls=((0, math.nan, 2, 1),)), 1, "finite"),
            (dict(balls=((0, 0, math.inf, 1),)), 1, "finite")):
        assert call(**kw) == status, kw
        assert text in L.rt_last_error().decode(), (kw, L.rt_last_error())
    if not torch.cuda.is_available():
        assert call() == 5 and "no HIP device" in L.rt_last_error().decode()
        assert call(balls=(), nballs=0) == 5


def test_light_lookup_needs_a_texture_and_a_light(rt):
    L = rt.LIB
    fr = _fr(rt, 10, 0x1000, 0x2000, None)
    light = rt.make_light([(0, 0, 1)])
    assert L.rt_lookup_light(None, ctypes.byref(fr), None, ctypes.byref(light), 0x4000, 0,
                             None) == 1
    assert "texture handle" in L.rt_last_error().decode()
    with pytest.raises(ValueError, match="1..64"):
        rt.make_light([(0, 0, 1)] * 65)
    with pytest.raises(KeyError):
        rt.make_light([(0, 0, 1)], kind="spot")


def test_light_lookup_validation_with_a_handle(rt):
    """Checks that need a texture handle (skipped where no device is visible)."""
    import math
    L = rt.LIB
    h = ctypes.c_void_p()
    d = _desc(rt, format=3, channels=1)
    st = L.rt_create_texture(ctypes.byref(d), None, ctypes.byref(h))
    if st == 5:
        pytest.skip("no device: handle creation refused before the light checks")
    assert st == 0
    try:
        good = _fr(rt, 10, 0x1000, 0x2000, None)
        lt = rt.make_light([(0, 0, 1), (0.1, 0, 1)])

        def call(fr=good, pos=None, light=lt, out=0x4000, flags=0):
            return L.rt_lookup_light(h, ctypes.byref(fr), pos,
                                     None if light is None else ctypes.byref(light), out, flags,
                                     None)
        assert call(light=None) == 1 and "light is NULL" in L.rt_last_error().decode()
        bad = rt.make_light([(0, 0, 1)])
        bad.kind = 7
        assert call(light=bad) == 1 and "kind" in L.rt_last_error().decode()
        bad = rt.make_light([(0, 0, 1)])
        bad.samples = 0
        assert call(light=bad) == 1 and "samples" in L.rt_last_error().decode()
        bad.samples = 65
        assert call(light=bad) == 1 and "samples" in L.rt_last_error().decode()
        bad = rt.make_light([(0, 0, math.nan)])
        assert call(light=bad) == 1 and "finite" in L.rt_last_error().decode()
        pl = rt.make_light([(0, 0, 3)], kind="point")
        assert call(light=pl) == 1 and "positions" in L.rt_last_error().decode()
        assert call(light=pl, pos=0x5002) == 1 and "pos" in L.rt_last_error().decode()
        assert call(out=None) == 1 and "out is NULL" in L.rt_last_error().decode()
        assert call(flags=2) == 1 and "flags" in L.rt_last_error().decode()
        nouv = _fr(rt, 10, None, 0x2000, None)
        assert call(fr=nouv) == 1 and "uv and tbn" in L.rt_last_error().decode()
        # the backward and the level-of-detail lookup refuse 1-bit textures
        fr3 = _fr(rt, 10, 0x1000, 0x2000, 0x3000)
        assert L.rt_lookup_bwd(h, ctypes.byref(fr3), 0x6000, 0x7000, None, None, 0x8000,
                               1 << 30, 0, None) == 2
        lv = (ctypes.c_void_p * 1)(h)
        assert L.rt_lookup_fwd_lod(lv, 1, ctypes.byref(fr3), 0x4000, 0x5000, 0, None) == 2
        assert L.rt_build_mip(h, 0x1000, None) == 2
    finally:
        L.rt_destroy_texture(h)


def test_dictionary_and_encoder_validation(rt):
    """Host checks of the dictionary texture and of Lloyd's steps."""
    L = rt.LIB
    h = ctypes.c_void_p()

    def desc(**kw):
        d = dict(buckets_w=4, buckets_h=4, n=8, channels=4, entries=16, format=0, index_bytes=1,
                 reserved=0, codebook=0x10000, index=0x20000, gains=None)
        d.update(kw)
        return rt.DictionaryDesc(**d)
    for kw, status, text in ((dict(buckets_w=0), 1, "bucket matrix"),
                             (dict(n=65), 2, "exceeds 64"), (dict(channels=5), 1, "channels"),
                             (dict(format=2), 2, "F32 or BF16"), (dict(format=3), 2, "F32 or BF16"),
                             (dict(index_bytes=3), 1, "index_bytes"), (dict(entries=0), 1, "entries"),
                             (dict(entries=257), 1, "do not fit"),
                             (dict(index_bytes=2, entries=65537), 1, "do not fit"),
                             (dict(codebook=None), 1, "non-NULL"), (dict(index=None), 1, "non-NULL"),
                             (dict(codebook=0x10008), 1, "16-byte"),
                             (dict(index_bytes=4, index=0x20002), 1, "4-byte"),
                             (dict(gains=0x30002), 1, "gains")):
        d = desc(**kw)
        assert L.rt_create_dictionary_texture(ctypes.byref(d), ctypes.byref(h)) == status, kw
        assert text in L.rt_last_error().decode(), (kw, L.rt_last_error())
    assert L.rt_create_dictionary_texture(None, ctypes.byref(h)) == 1
    # assignment
    A = L.rt_vq_assign
    assert A(0x1000, -1, 8, 0x2000, 4, 0x3000, None, None) == 1
    assert A(0x1000, 1 << 31, 8, 0x2000, 4, 0x3000, None, None) == 2
    assert A(0x1000, 10, 0, 0x2000, 4, 0x3000, None, None) == 1
    assert A(0x1000, 10, 8, 0x2000, 0, 0x3000, None, None) == 1
    assert A(0x1000, 10, 8, 0x2000, 65537, 0x3000, None, None) == 2
    assert A(None, 0, 8, None, 4, None, None, None) == 0  # nothing to assign
    assert A(None, 10, 8, 0x2000, 4, 0x3000, None, None) == 1
    assert A(0x1008, 10, 8, 0x2000, 4, 0x3000, None, None) == 1
    assert "16-byte" in L.rt_last_error().decode()
    assert A(0x1000, 10, 8, 0x2000, 4, 0x3002, None, None) == 1
    assert A(0x1000, 10, 8, 0x2000, 4, 0x3000, 0x4001, None) == 1
    # update
    assert L.rt_vq_update_workspace(1000, 16, 4096) > 0
    assert L.rt_vq_update_workspace(1000, 16, 4097) == 0
    assert L.rt_vq_update_workspace(0, 16, 4) == 0
    Up = L.rt_vq_update
    need = L.rt_vq_update_workspace(1000, 16, 8)
    assert Up(0x1000, 0, 16, 0x2000, 8, 0x3000, None, 0x10000, need, None) == 1
    assert Up(0x1000, 1000, 16, 0x2000, 5000, 0x3000, None, 0x10000, need, None) == 2
    assert Up(None, 1000, 16, 0x2000, 8, 0x3000, None, 0x10000, need, None) == 1
    assert Up(0x1000, 1000, 16, 0x2000, 8, 0x3000, None, None, need, None) == 1
    assert Up(0x1000, 1000, 16, 0x2000, 8, 0x3000, None, 0x10080, need, None) == 1
    assert Up(0x1000, 1000, 16, 0x2000, 8, 0x3000, None, 0x10000, need - 1, None) == 4
    assert Up(0x1000, 1000, 16, 0x2000, 8, 0x3000, 0x5002, 0x10000, need, None) == 1
