// rt_mip.hip -- one level of the mip chain of bucket matrices for gfx950.
//
// The synthesised W x H texture of Sec. 2 takes one sample per bucket and the
// lookup is linear in the buckets, so minifying it by 2 x 2 pixels is the
// lookup in the texel-wise mean of 2 x 2 buckets.  Level l+1 has
// max(1, W/2) x max(1, H/2) buckets (W, H powers of two; a side of 1 is not
// halved); its bucket (i, j) is the mean of the 4 (or 2) buckets it covers.
// A stream: each lane reads four texels of each source bucket and writes
// four texels of the destination, so the bound is HBM bandwidth.
#include <algorithm>

#include "rt_device.hpp"
#include "rt_kernels.hpp"

namespace rt {

// One workgroup per bucket of the next level (its position worked out once):
// the threads stream the bucket's float4s, each the mean of the 2 x 2 (or 2)
// source buckets' float4s at the same offset, summed as ((a + b) + (c + d)).
// At most MIP_GRID workgroups stride over the buckets, so a launch stays
// within one dispatch however many buckets the level has.
constexpr int64_t MIP_GRID = int64_t(1) << 20;

__global__ __launch_bounds__(256) void k_build_mip(const float* __restrict__ src,
                                                   float* __restrict__ dst, int W, int H,
                                                   int per) {
    const int W2 = W > 1 ? W / 2 : 1, H2 = H > 1 ? H / 2 : 1;
    const int64_t nb2 = (int64_t)W2 * H2;
    const int sx = W > 1 ? 2 : 1, sy = H > 1 ? 2 : 1;
    const int q4 = per / 4;  // per (n n C) is a multiple of 4 on this path
    const float inv = 1.f / (float)(sx * sy);
    for (int64_t b = blockIdx.x; b < nb2; b += gridDim.x) {
        const int j = (int)(b / W2), i = (int)(b - (int64_t)j * W2);
        const f4v* s0 = (const f4v*)(src + ((int64_t)(j * sy) * W + i * sx) * per);
        const f4v* s1 = (const f4v*)((const float*)s0 + (int64_t)W * per);
        f4v* d = (f4v*)(dst + b * per);
        for (int q = threadIdx.x; q < q4; q += blockDim.x) {
            f4v acc = s0[q];
            if (sx == 2) acc += s0[q4 + q];
            if (sy == 2) {
                f4v lo = s1[q];
                if (sx == 2) lo += s1[q4 + q];
                acc += lo;
            }
            d[q] = acc * inv;
        }
    }
}

// texel counts that are not a multiple of 4
__global__ __launch_bounds__(256) void k_build_mip_scalar(const float* __restrict__ src,
                                                          float* __restrict__ dst, int W, int H,
                                                          int per) {
    const int W2 = W > 1 ? W / 2 : 1, H2 = H > 1 ? H / 2 : 1;
    const int sx = W > 1 ? 2 : 1, sy = H > 1 ? 2 : 1;
    const int64_t total = (int64_t)W2 * H2 * per;
    const float inv = 1.f / (float)(sx * sy);
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t e = (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * 256 + threadIdx.x; e < total;
         e += stride) {
        const int64_t b = e / per;
        const int r = (int)(e - b * per);
        const int i = (int)(b % W2), j = (int)(b / W2);
        const int64_t s0 = ((int64_t)(j * sy) * W + i * sx) * per + r;
        float acc = src[s0];
        if (sx == 2) acc += src[s0 + per];
        if (sy == 2) {
            float lo = src[s0 + (int64_t)W * per];
            if (sx == 2) lo += src[s0 + (int64_t)W * per + per];
            acc += lo;
        }
        dst[e] = acc * inv;
    }
}

hipError_t launch_build_mip(const TexView& src, float* dst, hipStream_t s) {
    const int W2 = src.W > 1 ? src.W / 2 : 1, H2 = src.H > 1 ? src.H / 2 : 1;
    const int per = src.n * src.n * src.C;
    const int64_t work = (int64_t)W2 * H2 * ((per % 4 == 0) ? per / 4 : per);
    const uint32_t blocks = (uint32_t)std::min<int64_t>((work + 255) / 256, 256 * 64);
    prof_begin(K_BUILD_MIP, s);
    if (per % 4 == 0) {
        // one workgroup per bucket of the next level (at most MIP_GRID of them,
        // striding); as many threads as the bucket has float4s (rounded up to
        // whole wavefronts, at most 256)
        const int64_t nb2 = (int64_t)W2 * H2;
        const uint32_t gx = (uint32_t)std::min<int64_t>(nb2, MIP_GRID);
        const int threads = std::min(256, ((per / 4 + 63) / 64) * 64);
        hipLaunchKernelGGL(k_build_mip, dim3(gx), dim3(threads), 0, s,
                           (const float*)src.data, dst, src.W, src.H, per);
    } else
        hipLaunchKernelGGL(k_build_mip_scalar, dim3(blocks), dim3(256), 0, s,
                           (const float*)src.data, dst, src.W, src.H, per);
    prof_end(K_BUILD_MIP, s);
    return hipGetLastError();
}

}  // namespace rt
