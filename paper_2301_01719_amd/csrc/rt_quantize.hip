// rt_quantize.hip -- per-bucket BF16 / FP8-E4M3 quantiser, the 1-bit packer
// of shadow textures, and the atlas -> bucket-major re-layout, for gfx950.
//
// All are HBM streams.  BF16 is elementwise (float4 in, 4 x bf16 out).  FP8
// runs one or two wavefronts per bucket: the bucket's amax is reduced across
// the wave with cross-lane max (and between the two waves through LDS), then
// every lane encodes its values with the bucket's inverse scale.  Encodes are written from the formats' definitions with
// integer arithmetic (round to nearest even, E4M3 saturating to +-448).
#include <algorithm>

#include "rt_device.hpp"
#include "rt_kernels.hpp"

namespace rt {

// binary32 -> bfloat16 bits, round to nearest even; NaN stays (quiet) NaN.
__device__ __forceinline__ uint32_t f32_to_bf16_bits(float x) {
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7FFFFFFFu) > 0x7F800000u) return (b >> 16) | 0x40u;
    return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}

// binary32 -> OCP E4M3 (bias 7, max 448, S.1111.111 = NaN), round to nearest
// even, saturating: magnitudes >= 448 and infinities give 448.
__device__ __forceinline__ uint32_t f32_to_e4m3_bits(float y) {
    uint32_t b = __float_as_uint(y);
    uint32_t sign = (b >> 24) & 0x80u;
    uint32_t a = b & 0x7FFFFFFFu;
    if (a > 0x7F800000u) return sign | 0x7Fu;   // NaN
    if (a >= 0x43E00000u) return sign | 0x7Eu;  // >= 448
    if (a < 0x3C800000u) {                       // below 2^-6: multiples of 2^-9
        float t = __uint_as_float(a) * 512.0f;   // exact
        return sign | (uint32_t)rintf(t);        // 0..8 (8 is the first normal)
    }
    // keep 3 mantissa bits, round to nearest even on the 20 dropped bits; a
    // carry moves into the exponent field, which is the right result
    uint32_t r = a + 0x7FFFFu + ((a >> 20) & 1u);
    return sign | ((r >> 20) - (120u << 3));
}

// Codes of v * inv, byte k from component k, by the software encoder.
__device__ __forceinline__ uint32_t e4m3_pack4(f4v v, float inv) {
    return f32_to_e4m3_bits(v.x * inv) | (f32_to_e4m3_bits(v.y * inv) << 8) |
           (f32_to_e4m3_bits(v.z * inv) << 16) | (f32_to_e4m3_bits(v.w * inv) << 24);
}

// The same by the hardware conversion (v_cvt_pk_fp8_f32, two values per
// instruction).  It rounds to nearest even as the software encoder does but
// does not saturate (magnitudes from 464 up and infinities become NaN) and
// writes 0xFF for every NaN; on every other binary32 input its code is the
// software encoder's.  So it serves buckets whose values and inverse scale
// are finite, where every scaled value is at most 448 (1 + 2^-23) in
// magnitude.
__device__ __forceinline__ uint32_t e4m3_pack4_hw(f4v v, float inv) {
    const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(v.x * inv, v.y * inv, 0, false);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v.z * inv, v.w * inv, lo, true);
}

// Elementwise: each thread converts QB_UNROLL float4 (loads issued together),
// streamed with non-temporal loads and stores.
constexpr int QB_UNROLL = 2;

template <int QB_UNROLL>
__global__ __launch_bounds__(256) void k_quant_bf16(const float* __restrict__ src,
                                                    uint16_t* __restrict__ dst, int64_t total) {
    const int64_t quads = total / 4;
    const int64_t base =
        (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * (256 * QB_UNROLL) + threadIdx.x;
    f4v v[QB_UNROLL];
#pragma unroll
    for (int k = 0; k < QB_UNROLL; k++) {
        const int64_t q = base + k * 256;
        if (q < quads) v[k] = __builtin_nontemporal_load((const f4v*)src + q);
    }
#pragma unroll
    for (int k = 0; k < QB_UNROLL; k++) {
        const int64_t q = base + k * 256;
        if (q < quads) {
            u2v o;
            o.x = f32_to_bf16_bits(v[k].x) | (f32_to_bf16_bits(v[k].y) << 16);
            o.y = f32_to_bf16_bits(v[k].z) | (f32_to_bf16_bits(v[k].w) << 16);
            __builtin_nontemporal_store(o, (u2v*)dst + q);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < (total & 3)) {
        const int64_t e = quads * 4 + threadIdx.x;
        dst[e] = (uint16_t)f32_to_bf16_bits(src[e]);
    }
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Shapes of the FP8 quantiser.  QF8_PAIR (buckets of 512, 1024 or 2048
// values, HALF = values / 512): a 128-thread workgroup per bucket, each of its
// two wavefronts streaming one contiguous half of the bucket's float4s (2 KiB
// of a 16x16 RGBA bucket), the halves' maxima meeting in LDS; a bucket whose
// values and inverse scale are finite is encoded by the hardware conversion,
// any other by the software encoder.  With the encode that cheap, streaming 2 KiB per
// wavefront moves this 4:1 read/write mix faster than 4 KiB.  QF8_WAVE: one
// wavefront per bucket, whole float4s per lane.  QF8_SCALAR: one wavefront
// per bucket, one element per lane and step (any element count).  The
// bucket's largest magnitude is an exact maximum and both encoders give the
// same codes where they are used, so the codes and scales do not depend on
// the shape.
constexpr int QF8_SCALAR = 0, QF8_WAVE = 1, QF8_PAIR = 2;

template <int SHAPE, int HALF>
__global__ __launch_bounds__(SHAPE == QF8_PAIR ? 128 : 256) void k_quant_fp8(
    const float* __restrict__ src, uint8_t* __restrict__ dst, float* __restrict__ scales,
    int64_t n_buckets, int elems) {
    const int lane = threadIdx.x & 63;
    if constexpr (SHAPE == QF8_PAIR) {
        // elems = 512 * HALF: HALF float4 per lane in each half; the
        // workgroup's two wavefronts share its bucket
        __shared__ float part[2];
        __shared__ uint32_t odd[2];
        const int w = threadIdx.x >> 6;
        const int64_t b = (int64_t)xcd_block_id(blockIdx.x, gridDim.x);
        const bool live = b < n_buckets;
        const int64_t first = (int64_t)w * HALF * 64;  // float4 index of the half
        const f4v* s = (const f4v*)(src + (live ? b : 0) * elems) + first;
        f4v cache[HALF > 0 ? HALF : 1];
        float amax = 0.f;
        float nonfinite = 0.f;  // NaN once a NaN or an infinity is seen
        if (live) {
            // all loads issued before the first use
#pragma unroll
            for (int k = 0; k < HALF; k++) cache[k] = __builtin_nontemporal_load(s + k * 64 + lane);
#pragma unroll
            for (int k = 0; k < HALF; k++) {
                amax = fmaxf(amax, fmaxf(fmaxf(fabsf(cache[k].x), fabsf(cache[k].y)),
                                         fmaxf(fabsf(cache[k].z), fabsf(cache[k].w))));
                nonfinite += (cache[k].x * 0.f + cache[k].y * 0.f) +
                             (cache[k].z * 0.f + cache[k].w * 0.f);
            }
        }
        amax = wave_max(amax);
        const bool any_odd = __ballot(nonfinite != nonfinite) != 0ull;
        if (lane == 0) {
            part[w] = amax;
            odd[w] = any_odd ? 1u : 0u;
        }
        __syncthreads();
        if (!live) return;
        amax = fmaxf(part[0], part[1]);
        float inv = 1.f, scale = 1.f;
        if (amax > 0.f && amax <= 3.402823466e38f) {
            inv = 448.0f / amax;
            scale = amax / 448.0f;
        }
        // finite values and a finite inverse scale (a largest magnitude below
        // about 1.3e-36 overflows it): every scaled value is finite and at
        // most 448 (1 + 2^-23) in magnitude
        const bool finite = (odd[0] | odd[1]) == 0u && inv <= 3.402823466e38f;
        uint32_t* d = (uint32_t*)(dst + b * elems) + first;
        if (finite) {
#pragma unroll
            for (int k = 0; k < HALF; k++)
                __builtin_nontemporal_store(e4m3_pack4_hw(cache[k], inv), d + k * 64 + lane);
        } else {
#pragma unroll
            for (int k = 0; k < HALF; k++)
                __builtin_nontemporal_store(e4m3_pack4(cache[k], inv), d + k * 64 + lane);
        }
        if (w == 0 && lane == 0) scales[b] = scale;
        return;
    }
    const int64_t b =
        (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (b >= n_buckets) return;
    const float* s = src + b * elems;
    uint8_t* d = dst + b * elems;
    float amax = 0.f;
    if constexpr (SHAPE == QF8_WAVE) {
        const int per_lane = elems / 256;  // float4 per lane
        float4 cache[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (k < per_lane) {
                const f4v t = __builtin_nontemporal_load((const f4v*)s + k * 64 + lane);
                cache[k] = make_float4(t.x, t.y, t.z, t.w);
                amax = fmaxf(amax, fmaxf(fmaxf(fabsf(cache[k].x), fabsf(cache[k].y)),
                                         fmaxf(fabsf(cache[k].z), fabsf(cache[k].w))));
            }
        }
        for (int k = 4; k < per_lane; k++) {
            float4 v = ((const float4*)s)[k * 64 + lane];
            amax = fmaxf(amax, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
        amax = wave_max(amax);
        float inv = 1.f, scale = 1.f;
        if (amax > 0.f && amax <= 3.402823466e38f) {
            inv = 448.0f / amax;
            scale = amax / 448.0f;
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (k < per_lane) {
                float4 v = cache[k];
                uint32_t w = f32_to_e4m3_bits(v.x * inv) | (f32_to_e4m3_bits(v.y * inv) << 8) |
                             (f32_to_e4m3_bits(v.z * inv) << 16) | (f32_to_e4m3_bits(v.w * inv) << 24);
                __builtin_nontemporal_store(w, (uint32_t*)d + k * 64 + lane);
            }
        }
        for (int k = 4; k < per_lane; k++) {
            float4 v = ((const float4*)s)[k * 64 + lane];
            uint32_t w = f32_to_e4m3_bits(v.x * inv) | (f32_to_e4m3_bits(v.y * inv) << 8) |
                         (f32_to_e4m3_bits(v.z * inv) << 16) | (f32_to_e4m3_bits(v.w * inv) << 24);
            ((uint32_t*)d)[k * 64 + lane] = w;
        }
        if (lane == 0) scales[b] = scale;
    } else {
        for (int e = lane; e < elems; e += 64) amax = fmaxf(amax, fabsf(s[e]));
        amax = wave_max(amax);
        float inv = 1.f, scale = 1.f;
        if (amax > 0.f && amax <= 3.402823466e38f) {
            inv = 448.0f / amax;
            scale = amax / 448.0f;
        }
        for (int e = lane; e < elems; e += 64) d[e] = (uint8_t)f32_to_e4m3_bits(s[e] * inv);
        if (lane == 0) scales[b] = scale;
    }
}

// 1-bit packer (Sec. 5, Shadowing: a 1-bit texture holds occlusion): each
// sample becomes the bit (x >= 1/2).  When n is a multiple of 8 a bucket is
// a whole number of words and the bits of the texture are one flat array:
// each lane reads a float4 (four consecutive samples) and eight neighbouring
// lanes OR their nibbles into one word.
template <int U>
__global__ __launch_bounds__(256) void k_pack_bits_flat(const float* __restrict__ src,
                                                        uint32_t* __restrict__ words,
                                                        int64_t quads) {
    const int64_t base = (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * (256 * U) + threadIdx.x;
    f4v v[U];
#pragma unroll
    for (int k = 0; k < U; k++) {
        const int64_t q = base + k * 256;
        if (q < quads) v[k] = __builtin_nontemporal_load((const f4v*)src + q);
    }
#pragma unroll
    for (int k = 0; k < U; k++) {
        const int64_t q = base + k * 256;
        uint32_t nib = 0;
        if (q < quads)
            nib = (v[k].x >= 0.5f ? 1u : 0u) | (v[k].y >= 0.5f ? 2u : 0u) |
                  (v[k].z >= 0.5f ? 4u : 0u) | (v[k].w >= 0.5f ? 8u : 0u);
        uint32_t w = nib << (4 * (threadIdx.x & 7));
        w |= __shfl_xor(w, 1, 64);
        w |= __shfl_xor(w, 2, 64);
        w |= __shfl_xor(w, 4, 64);
        if (q < quads && (threadIdx.x & 7) == 0) words[q >> 3] = w;
    }
}

// Any n: one lane per word, reading the (up to) 32 samples it holds.
__global__ __launch_bounds__(256) void k_pack_bits_words(const float* __restrict__ src,
                                                         uint32_t* __restrict__ words,
                                                         int64_t total_words, int nn, int wpb) {
    const int64_t g = (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (g >= total_words) return;
    const int64_t b = g / wpb;
    const int k0 = (int)(g - b * wpb) * 32;
    const int k1 = min(k0 + 32, nn);
    const float* p = src + b * nn;
    uint32_t w = 0;
    for (int k = k0; k < k1; k++) w |= (p[k] >= 0.5f ? 1u : 0u) << (k - k0);
    words[g] = w;
}

// A dispatch holds fewer than 2^32 work-items, so a texture that would need
// more is quantised in chunks of at most MAX_LAUNCH_BLOCKS workgroups, each a
// launch over its own slice (cut at a bucket, or for the elementwise kernels at
// a whole group of float4).  Every workload up to 2^31 FP32 values (BF16) or
// 2^22 buckets (FP8) is one launch.
constexpr int64_t MAX_LAUNCH_BLOCKS = int64_t(1) << 20;

hipError_t launch_quantize(const TexView& t, int dst_fmt, void* codes, float* scales,
                           hipStream_t s) {
    const int64_t nb = (int64_t)t.W * t.H;
    const int elems = t.n * t.n * t.C;
    const float* src = (const float*)t.data;
    if (dst_fmt == FMT_BIT1) {
        prof_begin(K_PACK_BITS, s);
        if (t.n % 8 == 0) {
            // a chunk is a whole number of words: 8 float4 per word
            constexpr int U = 2;
            const int64_t quads = nb * elems / 4;
            const int64_t chunk = MAX_LAUNCH_BLOCKS * 256 * U;
            for (int64_t q0 = 0; q0 < quads; q0 += chunk) {
                const int64_t q = std::min(chunk, quads - q0);
                hipLaunchKernelGGL(k_pack_bits_flat<U>, dim3((uint32_t)((q + 256 * U - 1) / (256 * U))),
                                   dim3(256), 0, s, src + q0 * 4, (uint32_t*)codes + q0 / 8, q);
            }
        } else {
            const int wpb = bit_words(t.n);
            const int64_t chunk_b = MAX_LAUNCH_BLOCKS * 256 / wpb;
            for (int64_t b0 = 0; b0 < nb; b0 += chunk_b) {
                const int64_t words = std::min(chunk_b, nb - b0) * wpb;
                hipLaunchKernelGGL(k_pack_bits_words, dim3((uint32_t)((words + 255) / 256)),
                                   dim3(256), 0, s, src + b0 * elems,
                                   (uint32_t*)codes + b0 * wpb, words, elems, wpb);
            }
        }
        prof_end(K_PACK_BITS, s);
        return hipGetLastError();
    }
    if (dst_fmt == FMT_BF16) {
        // only the last chunk holds the (total mod 4) tail elements
        const int64_t total = nb * elems;
        const int64_t quads = total / 4;
        const int64_t chunk = MAX_LAUNCH_BLOCKS * 256 * QB_UNROLL;
        prof_begin(K_QUANT_BF16, s);
        int64_t q0 = 0;
        do {
            const int64_t q = std::min(chunk, quads - q0);
            const bool last = q0 + q == quads;
            const int64_t count = last ? total - q0 * 4 : q * 4;
            const uint32_t blocks =
                (uint32_t)((q + 256 * QB_UNROLL - 1) / (256 * QB_UNROLL)) + (q == 0 ? 1 : 0);
            hipLaunchKernelGGL(k_quant_bf16<QB_UNROLL>, dim3(blocks), dim3(256), 0, s,
                               src + q0 * 4, (uint16_t*)codes + q0 * 4, count);
            q0 += q;
        } while (q0 < quads);
        prof_end(K_QUANT_BF16, s);
        return hipGetLastError();
    }
    // at most 2^22 buckets per launch: 2^22 workgroups of 128 work-items in
    // the paired shape (2^29 work-items), 2^20 of 256 in the others
    const int64_t chunk_b = MAX_LAUNCH_BLOCKS * 4;
    prof_begin(K_QUANT_FP8, s);
    for (int64_t b0 = 0; b0 < nb; b0 += chunk_b) {
        const int64_t b = std::min(chunk_b, nb - b0);
        const float* bs = src + b0 * elems;
        uint8_t* bd = (uint8_t*)codes + b0 * elems;
        const dim3 pairs((uint32_t)b), quads((uint32_t)((b + 3) / 4));
        if (elems == 512)
            hipLaunchKernelGGL((k_quant_fp8<QF8_PAIR, 1>), pairs, dim3(128), 0, s, bs, bd,
                               scales + b0, b, elems);
        else if (elems == 1024)
            hipLaunchKernelGGL((k_quant_fp8<QF8_PAIR, 2>), pairs, dim3(128), 0, s, bs, bd,
                               scales + b0, b, elems);
        else if (elems == 2048)
            hipLaunchKernelGGL((k_quant_fp8<QF8_PAIR, 4>), pairs, dim3(128), 0, s, bs, bd,
                               scales + b0, b, elems);
        else if (elems % 256 == 0)
            hipLaunchKernelGGL((k_quant_fp8<QF8_WAVE, 0>), quads, dim3(256), 0, s, bs, bd,
                               scales + b0, b, elems);
        else
            hipLaunchKernelGGL((k_quant_fp8<QF8_SCALAR, 0>), quads, dim3(256), 0, s, bs, bd,
                               scales + b0, b, elems);
    }
    prof_end(K_QUANT_FP8, s);
    return hipGetLastError();
}

// Atlas [H*n][W*n][C] -> bucket-major [H][W][n][n][C]; a lane per texel
// (grid-stride), elements of `eb` bytes (4, 2 or 1).
template <typename E>
__global__ __launch_bounds__(256) void k_atlas_to_buckets(const E* __restrict__ src,
                                                          E* __restrict__ dst, int W, int H,
                                                          int n, int C) {
    const int64_t total = (int64_t)W * H * n * n;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t texel = (int64_t)blockIdx.x * 256 + threadIdx.x; texel < total; texel += stride) {
        const int x = (int)(texel % n);
        const int y = (int)((texel / n) % n);
        const int64_t b = texel / ((int64_t)n * n);
        const int i = (int)(b % W), j = (int)(b / W);
        const int64_t row = (int64_t)j * n + y, col = (int64_t)i * n + x;
        const int64_t s = (row * ((int64_t)W * n) + col) * C;
        for (int c = 0; c < C; c++) dst[texel * C + c] = src[s + c];
    }
}

hipError_t launch_atlas_to_buckets(const void* atlas, void* dst, int W, int H, int n, int C,
                                   int elem_bytes, hipStream_t s) {
    // grid-stride: a texture can hold 2^32 texels or more, more than one
    // dispatch may have work-items
    const int64_t total = (int64_t)W * H * n * n;
    const uint32_t blocks = (uint32_t)std::min<int64_t>((total + 255) / 256, 1 << 20);
    prof_begin(K_ATLAS_RELAYOUT, s);
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_atlas_to_buckets<uint32_t>, dim3(blocks), dim3(256), 0, s,
                           (const uint32_t*)atlas, (uint32_t*)dst, W, H, n, C);
    else if (elem_bytes == 2)
        hipLaunchKernelGGL(k_atlas_to_buckets<uint16_t>, dim3(blocks), dim3(256), 0, s,
                           (const uint16_t*)atlas, (uint16_t*)dst, W, H, n, C);
    else
        hipLaunchKernelGGL(k_atlas_to_buckets<uint8_t>, dim3(blocks), dim3(256), 0, s,
                           (const uint8_t*)atlas, (uint8_t*)dst, W, H, n, C);
    prof_end(K_ATLAS_RELAYOUT, s);
    return hipGetLastError();
}

}  // namespace rt
