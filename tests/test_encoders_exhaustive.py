"""Every binary32 bit pattern through the GPU quantiser's encoders, checked
code for code against the oracle's encoders written from the format
definitions (round to nearest even to BF16; round to nearest even to OCP
E4M3 with saturation to +-448, NaN kept as NaN).

The patterns go through rt_quantize itself, in chunks of 2^28.  BF16 has no
scale, so a chunk is a texture whose values are the patterns.  E4M3 divides
by a per-bucket scale; a bucket whose largest magnitude is not finite has
scale and inverse scale one, so every bucket starts with +inf and holds the
patterns in its other slots: the encoder then sees each pattern unchanged
(x * 1 = x in binary32).  Buckets of 16 x 16 RGBA values take the paired
quantiser, which encodes buckets with finite values and inverse scale by the
hardware conversion: there every bucket starts with 448 (inverse scale one)
and the other slots run through every finite magnitude up to 448, both
signs, the only values that path is given."""
import numpy as np
import pytest
import torch

import oracle
from helpers import host

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# a chunk: 128 x 128 buckets of 64 x 64 texels, 4 channels (2^28 values)
W = H = 128
N, C = 64, 4
ELEMS = N * N * C
BUCKETS = W * H


@pytest.fixture(scope="module")
def rt():
    from paper_2301_01719_amd import radtex
    return radtex


def _patterns(start, count):
    assert 0 <= start and start + count <= 1 << 32
    return (np.arange(count, dtype=np.uint32) + np.uint32(start)).view(np.float32)


def test_bf16_encoder_all_binary32(rt):
    total = 1 << 32
    per = BUCKETS * ELEMS
    for start in range(0, total, per):
        x = _patterns(start, per)
        tex = rt.Texture(torch.from_numpy(x).to(DEV).view(H, W, N, N, C), W, H, N, C)
        codes, _ = rt.quantize(tex, "bf16")
        torch.cuda.synchronize()
        got = host(codes).view(np.uint16).reshape(-1)
        want, _ = oracle.quantize(x, BUCKETS, ELEMS, oracle.FMT_BF16)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (f"BF16: {bad.size} codes differ from 0x{start:08x} on, first "
                               f"pattern 0x{start + int(bad[0]):08x}: gpu 0x{int(got[bad[0]]):04x}"
                               f" oracle 0x{int(want[bad[0]]):04x}")
        del tex, codes


def _e4m3_chunks(rt, ranges, first, n, c):
    """Quantise every pattern of the [lo, hi) ranges, in buckets of n x n x c
    values whose slot 0 holds `first`, through rt_quantize; compare code for
    code with the oracle.  Returns the number of patterns compared."""
    elems = n * n * c
    side = int(np.sqrt((1 << 28) // elems))
    buckets = side * side
    per = buckets * (elems - 1)
    pats = np.concatenate([np.arange(lo, hi, dtype=np.uint32) for lo, hi in ranges]) \
        if sum(hi - lo for lo, hi in ranges) <= per else None
    total = sum(hi - lo for lo, hi in ranges)
    done = 0
    while done < total:
        count = min(per, total - done)
        if pats is not None:
            chunk = pats[done:done + count]
        else:
            parts, skip, need = [], done, count
            for lo, hi in ranges:
                span = hi - lo
                if skip >= span:
                    skip -= span
                    continue
                take = min(span - skip, need)
                parts.append(np.arange(lo + skip, lo + skip + take, dtype=np.uint32))
                need -= take
                skip = 0
                if need == 0:
                    break
            chunk = np.concatenate(parts)
        x = np.zeros((buckets, elems), np.float32)
        x[:, 0] = first
        x[:, 1:].reshape(-1)[:count] = chunk.view(np.float32)
        flat = x.reshape(-1)
        tex = rt.Texture(torch.from_numpy(flat).to(DEV).view(side, side, n, n, c), side, side, n, c)
        codes, scales = rt.quantize(tex, "fp8")
        torch.cuda.synchronize()
        got = host(codes).reshape(buckets, elems)
        gs = host(scales).reshape(-1)
        want, ws = oracle.quantize(flat, buckets, elems, oracle.FMT_FP8_E4M3)
        want = want.reshape(buckets, elems)
        assert np.all(gs == 1.0) and np.all(ws == 1.0)
        assert np.all(got[:, 0] == want[:, 0]) and np.all(got[:, 0] == 0x7E)
        g1 = got[:, 1:].reshape(-1)[:count]
        w1 = want[:, 1:].reshape(-1)[:count]
        bad = np.nonzero(g1 != w1)[0]
        assert bad.size == 0, (f"E4M3 ({n}x{n}x{c}): {bad.size} codes differ, first pattern "
                               f"0x{int(chunk[bad[0]]):08x}: gpu 0x{int(g1[bad[0]]):02x} oracle "
                               f"0x{int(w1[bad[0]]):02x}")
        del tex, codes, scales
        done += count
    return done


@pytest.mark.parametrize("n,c", [(N, C), (16, 4)])
def test_e4m3_encoder_all_binary32(rt, n, c):
    # slot 0 holds +inf: scale and inverse scale one, the software encoder
    assert _e4m3_chunks(rt, [(0, 1 << 32)], np.inf, n, c) == 1 << 32


def test_e4m3_hardware_path_every_finite_value_up_to_448(rt):
    # slot 0 holds 448: the largest magnitude, inverse scale one; every
    # finite value of magnitude at most 448 (0x43E00000), both signs
    top = 0x43E00000 + 1
    ranges = [(0, top), (0x80000000, 0x80000000 + top)]
    assert _e4m3_chunks(rt, ranges, 448.0, 16, 4) == 2 * top


def test_e4m3_hardware_path_scaled_maximum_above_448(rt):
    """A largest magnitude m for which m * (448 / m) rounds above 448 in
    binary32 (to 448 (1 + 2^-23)): the code is still 448's."""
    g = np.random.default_rng(7)
    m = (g.random(1 << 22, dtype=np.float32) + np.float32(1)) * \
        np.exp2(g.integers(-30, 30, 1 << 22)).astype(np.float32)
    inv = np.float32(448) / m
    over = m[(m * inv) > np.float32(448)]
    assert over.size > 1000
    over = over[:4096]
    n, c = 16, 4
    elems = n * n * c
    x = (np.random.default_rng(8).random((over.size, elems), dtype=np.float32) - 0.5) * over[:, None]
    x[:, 5] = over
    x[: over.size // 2, 5] = -over[: over.size // 2]
    tex = rt.Texture(torch.from_numpy(x.reshape(-1)).to(DEV).view(1, over.size, n, n, c),
                     over.size, 1, n, c)
    codes, scales = rt.quantize(tex, "fp8")
    torch.cuda.synchronize()
    want, ws = oracle.quantize(x.reshape(-1), over.size, elems, oracle.FMT_FP8_E4M3)
    np.testing.assert_array_equal(host(scales).reshape(-1), ws)
    np.testing.assert_array_equal(host(codes).reshape(-1), want)
    got = host(codes).reshape(over.size, elems)[:, 5]
    assert np.all((got & 0x7F) == 0x7E)
