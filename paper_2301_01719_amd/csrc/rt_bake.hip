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
//
// The shadow bake (Sec. 5, Shadowing) fills a 1-bit texture: the sample's
// bit says whether the ray from the bucket's scene point along the sample's
// incidence direction (the direction that the light lookup maps onto it)
// escapes a set of balls that stand in for the ray-traced occluders.
#include <algorithm>

#include "rt_device.hpp"
#include "rt_kernels.hpp"

namespace rt {

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
// LDS of the bake kernels: 3 n n floats of sample directions, then (16-byte
// aligned) the kernel's float4 tables.
__host__ __device__ __forceinline__ int bake_dir_floats(int n) { return (3 * n * n + 3) & ~3; }

template <int C>
__global__ __launch_bounds__(256) void k_bake_env(int64_t nbuckets, int n,
                                                  const float* __restrict__ frames, EnvParams env,
                                                  float* __restrict__ texels) {
    extern __shared__ float smem[];
    float* Rt = smem;
    float4* lob = (float4*)(smem + bake_dir_floats(n));  // 2 MAX_LOBES entries
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

// Shadow bake: one wavefront per bucket at a time, one lane per sample.  The
// incidence directions of the n x n samples sit in LDS.  Per bucket, lane q
// first forms ball q's offset from the bucket's origin o, e = c - o (into the
// wave's LDS slots), and whether o lies inside it (then every sample of the
// bucket is shaded).  Each lane then turns its direction into the scene
// frame (d = M^T I, normalised) and tests every ball: the ray o + t d
// (t > 0) meets ball (c, r) iff t* = d . e > 0 and |e - t* d| <= r.  The
// distance is formed from the vector e - t* d rather than as |e|^2 - t*^2,
// which cancels when the ray points at the centre.  A wave ballot packs 64
// samples into two words; samples past n n give 0, which clears the padding
// bits of the last word.
__global__ __launch_bounds__(256) void k_bake_shadow(int64_t nbuckets, int n,
                                                     const float* __restrict__ origins,
                                                     const float* __restrict__ frames,
                                                     Occluders occ, uint32_t* __restrict__ words) {
    extern __shared__ float smem[];
    float* It = smem;
    float4* ball = (float4*)(smem + bake_dir_floats(n));  // MAX_OCCLUDERS entries
    float4* relw = ball + MAX_OCCLUDERS;                   // per wave: (e, r^2) of each ball
    const int nn = n * n;
    if (threadIdx.x < occ.count)
        ball[threadIdx.x] = make_float4(occ.ball[threadIdx.x][0], occ.ball[threadIdx.x][1],
                                        occ.ball[threadIdx.x][2], occ.ball[threadIdx.x][3]);
    for (int q = threadIdx.x; q < nn; q += 256) {
        const int y = q / n, x = q - y * n;
        float R[3], I[3];
        sample_directions(x, y, n, R, I);
        It[3 * q + 0] = I[0];
        It[3 * q + 1] = I[1];
        It[3 * q + 2] = I[2];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int nballs = occ.count;
    const int wpb = bit_words(n);
    const int chunks = (nn + 63) >> 6;
    const int64_t waves = (int64_t)gridDim.x * 4;
    const int64_t first = (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * 4 + wv;
    for (int64_t b = first; b < nbuckets; b += waves) {
        float M[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
        if (frames) {
#pragma unroll
            for (int k = 0; k < 9; k++) M[k] = frames[b * 9 + k];
        }
        const float ox = origins[b * 3 + 0], oy = origins[b * 3 + 1], oz = origins[b * 3 + 2];
        bool inside = false;
        if (lane < nballs) {
            const float4 bl = ball[lane];
            const float ex = bl.x - ox, ey = bl.y - oy, ez = bl.z - oz;
            const float r2 = bl.w * bl.w;
            relw[wv * MAX_OCCLUDERS + lane] = make_float4(ex, ey, ez, r2);
            inside = ex * ex + ey * ey + ez * ez <= r2;
        }
        const bool blocked = __ballot(inside) != 0;
        wave_lds_sync();
        for (int c = 0; c < chunks; c++) {
            const int k = c * 64 + lane;
            bool lit = false;
            if (k < nn && !blocked) {
                const float i0 = It[3 * k + 0], i1 = It[3 * k + 1], i2 = It[3 * k + 2];
                float dx = M[0] * i0 + M[3] * i1 + M[6] * i2;
                float dy = M[1] * i0 + M[4] * i1 + M[7] * i2;
                float dz = M[2] * i0 + M[5] * i1 + M[8] * i2;
                const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
                dx *= inv;
                dy *= inv;
                dz *= inv;
                bool hit = false;
                for (int q = 0; q < nballs; q++) {
                    const float4 e = relw[wv * MAX_OCCLUDERS + q];
                    const float ts = dx * e.x + dy * e.y + dz * e.z;
                    const float hx = e.x - ts * dx, hy = e.y - ts * dy, hz = e.z - ts * dz;
                    hit |= ts > 0.f && hx * hx + hy * hy + hz * hz <= e.w;
                }
                lit = !hit;
            }
            const uint64_t bits = __ballot(lit);
            const int w = 2 * c + lane;
            if (lane < 2 && w < wpb)
                words[b * wpb + w] = lane == 0 ? (uint32_t)bits : (uint32_t)(bits >> 32);
        }
        wave_lds_sync();  // the next bucket rewrites this wave's ball terms
    }
}

hipError_t launch_bake_shadow(int W, int H, int n, const float* origins, const float* frames,
                              const Occluders& occ, uint32_t* words, hipStream_t s) {
    const int64_t nb = (int64_t)W * H;
    if (nb == 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)std::min<int64_t>((nb + 3) / 4, 256 * 16);
    prof_begin(K_BAKE_SHADOW, s);
    const size_t shm = (size_t)(bake_dir_floats(n) + 4 * MAX_OCCLUDERS * 5) * 4;
    hipLaunchKernelGGL(k_bake_shadow, dim3(blocks), dim3(256), shm, s, nb, n, origins, frames, occ,
                       words);
    prof_end(K_BAKE_SHADOW, s);
    return hipGetLastError();
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
    const size_t shm = (size_t)(bake_dir_floats(n) + 4 * 2 * MAX_LOBES) * 4;
    prof_begin(K_BAKE_ENV, s);
    switch (C) {
    case 1: hipLaunchKernelGGL((k_bake_env<1>), dim3(blocks), dim3(256), shm, s, (int64_t)W * H, n, frames, env, texels); break;
    case 2: hipLaunchKernelGGL((k_bake_env<2>), dim3(blocks), dim3(256), shm, s, (int64_t)W * H, n, frames, env, texels); break;
    case 3: hipLaunchKernelGGL((k_bake_env<3>), dim3(blocks), dim3(256), shm, s, (int64_t)W * H, n, frames, env, texels); break;
    default: hipLaunchKernelGGL((k_bake_env<4>), dim3(blocks), dim3(256), shm, s, (int64_t)W * H, n, frames, env, texels); break;
    }
    prof_end(K_BAKE_ENV, s);
    return hipGetLastError();
}

}  // namespace rt
