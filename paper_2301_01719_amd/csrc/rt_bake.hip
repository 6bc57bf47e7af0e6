// rt_bake.hip -- the write side of the method for gfx950: the reflection
// vector of every sample centre (Eqs. 4a, 4b) and the bake of a radiance
// texture from an analytic environment sampled along it (Sec. 2.1: ray-traced
// data is sampled onto the texture along R).
//
// One lane per texel, grid-stride over the whole texture.  Per lane: the
// reflection vector R of its sample (the sample centre B, A from Eq. (4a), R
// from Eq. (4b), formed once per workgroup), the scene direction
// d = normalize(M^T R) with the bucket's frame M = [T;B;N], and per channel
// ambient + sum_k a_k exp(lambda_k (mu_k . d - 1)).  The texture is written
// once, so the bound is HBM bandwidth on the writes.
#include <algorithm>

#include "rt_device.hpp"
#include "rt_kernels.hpp"

namespace rt {

// Eq. (4a) then Eq. (4b) at the centre of sample (x, y) of an n x n bucket:
// B = ((2x+1)/n - 1, (2y+1)/n - 1); A = max(|B_x|, |B_y|) / |B| B (A = 0 at
// B = 0); R = (-A_x w, -A_y w, 1 - |A|^2), w = sqrt(2 - |A|^2).  Also the
// incidence I of Eq. (2c), R mirrored about the normal.
__device__ __forceinline__ void sample_directions(int x, int y, int n, float R[3], float I[3]) {
    const float bx = (float)(2 * x + 1) / (float)n - 1.f;
    const float by = (float)(2 * y + 1) / (float)n - 1.f;
    const float rho = sqrtf(bx * bx + by * by);
    const float m = fmaxf(fabsf(bx), fabsf(by));
    float ax = 0.f, ay = 0.f;
    if (rho > 0.f) {
        const float f = m / rho;
        ax = f * bx;
        ay = f * by;
    }
    const float r2 = ax * ax + ay * ay;
    const float w = sqrtf(fmaxf(0.f, 2.f - r2));
    R[0] = -ax * w;
    R[1] = -ay * w;
    R[2] = 1.f - r2;
    I[0] = ax * w;
    I[1] = ay * w;
    I[2] = 1.f - r2;
}

__global__ __launch_bounds__(256) void k_bake_directions(int n, float* __restrict__ inc,
                                                         float* __restrict__ refl) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n * n) return;
    const int y = t / n, x = t - y * n;
    float R[3], I[3];
    sample_directions(x, y, n, R, I);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        if (inc) inc[t * 3 + k] = I[k];
        if (refl) refl[t * 3 + k] = R[k];
    }
}

// The reflection vectors of the n x n samples are the same in every bucket:
// each workgroup forms them once in LDS, beside the environment's lobes.  The grid-stride loop steps the
// (bucket, sample) pair of its texel incrementally, with no division per
// texel.  Each lobe arrives as (lambda log2e mu, -lambda log2e), so its value
// is the hardware exp2 of one fused dot product.
template <int C>
__global__ __launch_bounds__(256) void k_bake_env(int64_t nbuckets, int n,
                                                  const float* __restrict__ frames, EnvParams env,
                                                  float* __restrict__ texels) {
    __shared__ float Rt[3 * 32 * 32];
    __shared__ float4 lob[2 * MAX_LOBES];
    const int nn = n * n;
    const int nl = env.lobes;
    if (threadIdx.x < 2 * nl) {
        const float* L = env.lobe[threadIdx.x >> 1] + 4 * (threadIdx.x & 1);
        lob[threadIdx.x] = make_float4(L[0], L[1], L[2], L[3]);
    }
    for (int q = threadIdx.x; q < nn; q += 256) {
        const int y = q / n, x = q - y * n;
        float R[3], I[3];
        sample_directions(x, y, n, R, I);
        Rt[3 * q + 0] = R[0];
        Rt[3 * q + 1] = R[1];
        Rt[3 * q + 2] = R[2];
    }
    __syncthreads();
    const int64_t total = nbuckets * nn;
    const int64_t start = (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t b = start / nn;
    int s = (int)(start - b * nn);
    const int64_t db = stride / nn;
    const int ds = (int)(stride - db * nn);
    // U consecutive texels of the lane's grid-stride sequence share each read
    // of a lobe's parameters
    constexpr int U = 4;
    for (int64_t t0 = start; t0 < total; t0 += U * stride) {
        float d[U][3], v[U][4];
        int64_t tt[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            tt[u] = t0 + u * stride;
            const float r0 = Rt[3 * s + 0], r1 = Rt[3 * s + 1], r2 = Rt[3 * s + 2];
            if (frames && tt[u] < total) {
                const float* M = frames + b * 9;
#pragma unroll
                for (int k = 0; k < 3; k++) d[u][k] = M[k] * r0 + M[3 + k] * r1 + M[6 + k] * r2;
            } else {
                d[u][0] = r0;
                d[u][1] = r1;
                d[u][2] = r2;
            }
            // d is a unit vector up to rounding (R is, frames are rotations): the
            // hardware reciprocal square root only removes that residue
            const float inv = rsqrtf(d[u][0] * d[u][0] + d[u][1] * d[u][1] + d[u][2] * d[u][2]);
            d[u][0] *= inv;
            d[u][1] *= inv;
            d[u][2] *= inv;
#pragma unroll
            for (int c = 0; c < 4; c++) v[u][c] = env.ambient[c];
            s += ds;
            b += db;
            if (s >= nn) {
                s -= nn;
                b += 1;
            }
        }
        for (int k = 0; k < nl; k++) {
            const float4 ax = lob[2 * k], am = lob[2 * k + 1];
#pragma unroll
            for (int u = 0; u < U; u++) {
                // lambda (mu . d - 1) in base 2: (lambda log2e mu) . d - lambda log2e
                const float e = __builtin_amdgcn_exp2f(
                    fmaf(ax.x, d[u][0], fmaf(ax.y, d[u][1], fmaf(ax.z, d[u][2], ax.w))));
                v[u][0] += am.x * e;
                if constexpr (C > 1) v[u][1] += am.y * e;
                if constexpr (C > 2) v[u][2] += am.z * e;
                if constexpr (C > 3) v[u][3] += am.w * e;
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t t = tt[u];
            if (t >= total) break;
            if constexpr (C == 4) {
                ((float4*)texels)[t] = make_float4(v[u][0], v[u][1], v[u][2], v[u][3]);
            } else if constexpr (C == 2) {
                ((float2*)texels)[t] = make_float2(v[u][0], v[u][1]);
            } else {
#pragma unroll
                for (int c = 0; c < C; c++) texels[t * C + c] = v[u][c];
            }
        }
    }
}

hipError_t launch_bake_directions(int n, float* inc, float* refl, hipStream_t s) {
    const uint32_t blocks = (uint32_t)((n * n + 255) / 256);
    prof_begin(K_BAKE_DIRECTIONS, s);
    hipLaunchKernelGGL(k_bake_directions, dim3(blocks), dim3(256), 0, s, n, inc, refl);
    prof_end(K_BAKE_DIRECTIONS, s);
    return hipGetLastError();
}

hipError_t launch_bake_env(int W, int H, int n, int C, const float* frames, const EnvParams& env,
                           float* texels, hipStream_t s) {
    const int64_t total = (int64_t)W * H * n * n;
    if (total == 0) return hipSuccess;
    // 16 workgroups per CU: each lane then covers many texels, so the per-
    // workgroup table of sample directions is formed once for all of them
    const uint32_t blocks = (uint32_t)std::min<int64_t>((total + 255) / 256, 256 * 16);
    prof_begin(K_BAKE_ENV, s);
    switch (C) {
    case 1: hipLaunchKernelGGL((k_bake_env<1>), dim3(blocks), dim3(256), 0, s, (int64_t)W * H, n, frames, env, texels); break;
    case 2: hipLaunchKernelGGL((k_bake_env<2>), dim3(blocks), dim3(256), 0, s, (int64_t)W * H, n, frames, env, texels); break;
    case 3: hipLaunchKernelGGL((k_bake_env<3>), dim3(blocks), dim3(256), 0, s, (int64_t)W * H, n, frames, env, texels); break;
    default: hipLaunchKernelGGL((k_bake_env<4>), dim3(blocks), dim3(256), 0, s, (int64_t)W * H, n, frames, env, texels); break;
    }
    prof_end(K_BAKE_ENV, s);
    return hipGetLastError();
}

}  // namespace rt
