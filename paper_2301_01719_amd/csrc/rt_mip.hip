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

__global__ __launch_bounds__(256) void k_build_mip(const float* __restrict__ src,
                                                   float* __restrict__ dst, int W, int H,
                                                   int per) {
    const int W2 = W > 1 ? W / 2 : 1, H2 = H > 1 ? H / 2 : 1;
    const int sx = W > 1 ? 2 : 1, sy = H > 1 ? 2 : 1;
    const int q4 = per / 4;  // per (n n C) is a multiple of 4 on this path
    const int64_t groups = (int64_t)W2 * H2 * q4;
    const float inv = 1.f / (float)(sx * sy);
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t g = (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * 256 + threadIdx.x; g < groups;
         g += stride) {
        const int64_t b = g / q4;
        const int r = (int)(g - b * q4) * 4;
        const int i = (int)(b % W2), j = (int)(b / W2);
        const int64_t s0 = ((int64_t)(j * sy) * W + i * sx) * per + r;
        f4v acc = *(const f4v*)(src + s0);
        if (sx == 2) acc += *(const f4v*)(src + s0 + per);
        if (sy == 2) {
            f4v lo = *(const f4v*)(src + s0 + (int64_t)W * per);
            if (sx == 2) lo += *(const f4v*)(src + s0 + (int64_t)W * per + per);
            acc += lo;
        }
        *(f4v*)(dst + b * per + r) = acc * inv;
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
    if (per % 4 == 0)
        hipLaunchKernelGGL(k_build_mip, dim3(blocks), dim3(256), 0, s, (const float*)src.data, dst,
                           src.W, src.H, per);
    else
        hipLaunchKernelGGL(k_build_mip_scalar, dim3(blocks), dim3(256), 0, s,
                           (const float*)src.data, dst, src.W, src.H, per);
    prof_end(K_BUILD_MIP, s);
    return hipGetLastError();
}

}  // namespace rt
