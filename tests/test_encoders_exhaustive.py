"""Every binary32 bit pattern through the GPU quantiser's encoders, checked
code for code against the oracle's encoders written from the format
definitions (round to nearest even to BF16; round to nearest even to OCP
E4M3 with saturation to +-448, NaN kept as NaN).

The patterns go through rt_quantize itself, in chunks of 2^28.  BF16 has no
scale, so a chunk is a texture whose values are the patterns.  E4M3 divides
by a per-bucket scale; a bucket whose largest magnitude is not finite has
scale and inverse scale one, so every bucket starts with +inf and holds the
patterns in its other slots: the encoder then sees each pattern unchanged
(x * 1 = x in binary32)."""
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


def test_e4m3_encoder_all_binary32(rt):
    total = 1 << 32
    per = BUCKETS * (ELEMS - 1)  # slot 0 of each bucket holds +inf
    for start in range(0, total, per):
        count = min(per, total - start)
        x = np.zeros((BUCKETS, ELEMS), np.float32)
        x[:, 0] = np.inf
        x[:, 1:].reshape(-1)[:count] = _patterns(start, count)
        flat = x.reshape(-1)
        tex = rt.Texture(torch.from_numpy(flat).to(DEV).view(H, W, N, N, C), W, H, N, C)
        codes, scales = rt.quantize(tex, "fp8")
        torch.cuda.synchronize()
        got = host(codes).reshape(BUCKETS, ELEMS)
        gs = host(scales).reshape(-1)
        want, ws = oracle.quantize(flat, BUCKETS, ELEMS, oracle.FMT_FP8_E4M3)
        want = want.reshape(BUCKETS, ELEMS)
        assert np.all(gs == 1.0) and np.all(ws == 1.0)
        assert np.all(got[:, 0] == 0x7E)  # +inf saturates to +448
        g1 = got[:, 1:].reshape(-1)[:count]
        w1 = want[:, 1:].reshape(-1)[:count]
        bad = np.nonzero(g1 != w1)[0]
        assert bad.size == 0, (f"E4M3: {bad.size} codes differ from 0x{start:08x} on, first "
                               f"pattern 0x{start + int(bad[0]):08x}: gpu 0x{int(g1[bad[0]]):02x}"
                               f" oracle 0x{int(w1[bad[0]]):02x}")
        del tex, codes, scales
