// rt_lookup.hip -- forward radiance-bucket lookup for gfx950, on one bucket
// matrix or, with a level of detail, on a mip chain of them.
//
// One lane per fragment.  Per lane: the 56-byte G-buffer record (uv, frame,
// view) is read, the incidence is mapped to the in-bucket sample coordinate
// (Eq. 1b, Eq. 3, the clamp after Eq. 3), the bucket is selected from (u, v)
// (Sec. 2) and four taps of C channels are read from the bucket-major
// texture and blended bilinearly.  The path is a gather: no contraction, so
// no MFMA; the bound is HBM bandwidth (the G-buffer stream dominates).
//
// The light lookup (shadowing) takes the direction toward the light in place
// of the view vector and averages the lookups over an area light's samples;
// on a 1-bit texture each tap is one bit of the bucket's words.
#include "rt_device.hpp"
#include "rt_kernels.hpp"

namespace rt {

// The four taps around footprint p of the bucket whose first texel is at
// `bucket` (global memory or a copy in LDS), blended and added to acc with
// factor f.
template <int FMT, int C>
__device__ __forceinline__ void blend_taps(const void* bucket, int n, const Foot& p, float f,
                                           float acc[4]) {
    F4 t00 = load_texel<FMT, C>(bucket, p.y0 * n + p.x0);
    F4 t01 = load_texel<FMT, C>(bucket, p.y0 * n + p.x1);
    F4 t10 = load_texel<FMT, C>(bucket, p.y1 * n + p.x0);
    F4 t11 = load_texel<FMT, C>(bucket, p.y1 * n + p.x1);
    float w00 = (1.f - p.fx) * (1.f - p.fy), w01 = p.fx * (1.f - p.fy);
    float w10 = (1.f - p.fx) * p.fy, w11 = p.fx * p.fy;
#pragma unroll
    for (int c = 0; c < C; c++) {
        float v = w00 * t00.v[c] + w01 * t01.v[c] + w10 * t10.v[c] + w11 * t11.v[c];
        acc[c] += f * v;
    }
}

// The four taps of bucket b around footprint p, blended and added to acc
// with weight wgt.  DICT: b is read through the dictionary (its entry in the
// codebook, times its gain).
template <int FMT, int C, bool DICT = false>
__device__ __forceinline__ void bucket_bilerp(const TexView& t, int64_t b, const Foot& p,
                                              float wgt, float acc[4]) {
    const int n = t.n;
    if constexpr (DICT) {
        if (t.gains) wgt *= t.gains[b];
        b = dict_entry(t, b);
    }
    if constexpr (FMT == FMT_BIT1) {
        const uint32_t* w = (const uint32_t*)t.data + b * bit_words(n);
        const int k00 = p.y0 * n + p.x0, k01 = p.y0 * n + p.x1;
        const int k10 = p.y1 * n + p.x0, k11 = p.y1 * n + p.x1;
        const float t00 = (float)((w[k00 >> 5] >> (k00 & 31)) & 1u);
        const float t01 = (float)((w[k01 >> 5] >> (k01 & 31)) & 1u);
        const float t10 = (float)((w[k10 >> 5] >> (k10 & 31)) & 1u);
        const float t11 = (float)((w[k11 >> 5] >> (k11 & 31)) & 1u);
        const float v = (1.f - p.fx) * (1.f - p.fy) * t00 + p.fx * (1.f - p.fy) * t01 +
                        (1.f - p.fx) * p.fy * t10 + p.fx * p.fy * t11;
        acc[0] += wgt * v;
        return;
    }
    const unsigned char* bucket =
        (const unsigned char*)t.data + b * (int64_t)(n * n) * C * storage_bytes<FMT>();
    blend_taps<FMT, C>(bucket, n, p, wgt * bucket_factor<FMT>(t.scales, b), acc);
}

// The lookup's output is written once and not read back by the library: it
// is stored non-temporally (past the caches the G-buffer and the taps use).
template <int C>
__device__ __forceinline__ void store_out(float* __restrict__ out, int64_t f, const float acc[4]) {
    if constexpr (C == 4) {
        const f4v v = {acc[0], acc[1], acc[2], acc[3]};
        __builtin_nontemporal_store(v, (f4v*)out + f);
    } else {
#pragma unroll
        for (int c = 0; c < C; c++) __builtin_nontemporal_store(acc[c], out + f * C + c);
    }
}

template <int FMT, int C, int MODE, bool DICT>
__global__ __launch_bounds__(256) void k_lookup_fwd(TexView t, const float* __restrict__ uv,
                                                    const float* __restrict__ tbn,
                                                    const float* __restrict__ view,
                                                    float* __restrict__ out, FragMap m) {
    __shared__ FragStage stage;
    const int64_t f = frag_of(m, blockIdx.x, gridDim.x, threadIdx.x);
    Frag g = load_frag_block(uv, tbn, view, m, f, stage);
    if (f < 0) return;
    Dir d = map_direction(g.m, g.w, t.n);
    Foot p = footprint(d.sx, d.sy, t.n);
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if constexpr (MODE == MODE_NEAREST) {
        int i = bucket_of(g.u, t.W), j = bucket_of(g.v, t.H);
        bucket_bilerp<FMT, C, DICT>(t, (int64_t)j * t.W + i, p, 1.0f, acc);
    } else {
        int i0, i1, j0, j1;
        float a, bb;
        bucket_pair(g.u, t.W, i0, i1, a);
        bucket_pair(g.v, t.H, j0, j1, bb);
        bucket_bilerp<FMT, C, DICT>(t, (int64_t)j0 * t.W + i0, p, (1.f - a) * (1.f - bb), acc);
        bucket_bilerp<FMT, C, DICT>(t, (int64_t)j0 * t.W + i1, p, a * (1.f - bb), acc);
        bucket_bilerp<FMT, C, DICT>(t, (int64_t)j1 * t.W + i0, p, (1.f - a) * bb, acc);
        bucket_bilerp<FMT, C, DICT>(t, (int64_t)j1 * t.W + i1, p, a * bb, acc);
    }
    store_out<C>(out, f, acc);
}

// The forward with bucket tiles staged in LDS (nearest buckets, plain
// textures): per wavefront, the bucket of the first fragment still to serve
// is found with a ballot, every lane whose fragment lies in that bucket joins
// the group, the wavefront copies the whole bucket into its LDS tile with
// 16-byte loads, and the group blends its taps from LDS; repeated until every
// fragment is served.  The blend is blend_taps on the copy, so the results
// are those of k_lookup_fwd bit for bit.  It pays only where a wavefront's
// fragments share few buckets and read much of each.
template <int FMT, int C>
__global__ __launch_bounds__(256) void k_lookup_fwd_staged(TexView t, const float* __restrict__ uv,
                                                           const float* __restrict__ tbn,
                                                           const float* __restrict__ view,
                                                           float* __restrict__ out, FragMap m) {
    extern __shared__ uint4 tiles[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int bucket_bytes = t.n * t.n * C * storage_bytes<FMT>();  // a multiple of 16
    uint4* mine = tiles + w * (bucket_bytes / 16);
    const int64_t f = frag_of(m, blockIdx.x, gridDim.x, threadIdx.x);
    const bool live = f >= 0;
    Foot p{};
    int64_t b = -1;
    if (live) {
        const Frag g = load_frag(uv, tbn, view, f);
        const Dir d = map_direction(g.m, g.w, t.n);
        p = footprint(d.sx, d.sy, t.n);
        b = (int64_t)bucket_of(g.v, t.H) * t.W + bucket_of(g.u, t.W);
    }
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    uint64_t todo = __ballot(live);
    while (todo != 0ull) {
        const int leader = __builtin_ctzll(todo);
        const uint32_t lo = __builtin_amdgcn_readfirstlane(__shfl((uint32_t)b, leader, 64));
        const uint32_t hi =
            __builtin_amdgcn_readfirstlane(__shfl((uint32_t)((uint64_t)b >> 32), leader, 64));
        const int64_t bk = (int64_t)(((uint64_t)hi << 32) | lo);
        const uint64_t grp = __ballot(live && b == bk);
        const uint4* src = (const uint4*)((const unsigned char*)t.data + bk * bucket_bytes);
        for (int q = lane; q < bucket_bytes / 16; q += 64) mine[q] = src[q];
        wave_lds_sync();
        if ((grp >> lane) & 1ull)
            blend_taps<FMT, C>(mine, t.n, p, 1.0f * bucket_factor<FMT>(t.scales, bk), acc);
        wave_lds_sync();
        todo &= ~grp;
    }
    if (live) store_out<C>(out, f, acc);
}

__global__ __launch_bounds__(256) void k_debug_indices(TexView t, const float* __restrict__ uv,
                                                       const float* __restrict__ tbn,
                                                       const float* __restrict__ view,
                                                       int32_t* __restrict__ idx,
                                                       float* __restrict__ frac, FragMap m) {
    const int64_t f = frag_of(m, blockIdx.x, gridDim.x, threadIdx.x);
    if (f < 0) return;
    Frag g = load_frag(uv, tbn, view, f);
    Dir d = map_direction(g.m, g.w, t.n);
    int x0 = (int)d.sx, y0 = (int)d.sy;
    ((int4*)idx)[f] = make_int4(bucket_of(g.u, t.W), bucket_of(g.v, t.H), x0, y0);
    ((float2*)frac)[f] = make_float2(d.sx - (float)x0, d.sy - (float)y0);
}

// Storage of level l of a chain, selected with compile-time indices so that
// the per-lane choice stays in registers.
__device__ __forceinline__ void level_storage(const LevelSet& ls, int l, const void*& data,
                                              const float*& scales) {
    data = ls.data[0];
    scales = ls.scales[0];
#pragma unroll
    for (int k = 1; k < MAX_LEVELS; k++) {
        if (l == k) {
            data = ls.data[k];
            scales = ls.scales[k];
        }
    }
}

// The forward's bucket footprint and in-bucket bilinear blend, on level l.
template <int FMT, int C, int MODE>
__device__ __forceinline__ void level_lookup(const LevelSet& ls, int l, const Frag& g,
                                             const Foot& p, float acc[4]) {
    TexView t{};
    level_storage(ls, l, t.data, t.scales);
    t.W = max(ls.W >> l, 1);
    t.H = max(ls.H >> l, 1);
    t.n = ls.n;
    t.C = ls.C;
    if constexpr (MODE == MODE_NEAREST) {
        const int i = bucket_of(g.u, t.W), j = bucket_of(g.v, t.H);
        bucket_bilerp<FMT, C>(t, (int64_t)j * t.W + i, p, 1.0f, acc);
    } else {
        int i0, i1, j0, j1;
        float a, bb;
        bucket_pair(g.u, t.W, i0, i1, a);
        bucket_pair(g.v, t.H, j0, j1, bb);
        bucket_bilerp<FMT, C>(t, (int64_t)j0 * t.W + i0, p, (1.f - a) * (1.f - bb), acc);
        bucket_bilerp<FMT, C>(t, (int64_t)j0 * t.W + i1, p, a * (1.f - bb), acc);
        bucket_bilerp<FMT, C>(t, (int64_t)j1 * t.W + i0, p, (1.f - a) * bb, acc);
        bucket_bilerp<FMT, C>(t, (int64_t)j1 * t.W + i1, p, a * bb, acc);
    }
}

// Lookup over a mip chain of bucket matrices: the level of detail is
// lambda = log2 rho, rho the larger of the pixel's two UV footprints in
// buckets of level 0 (duv = du/dx, dv/dx, du/dy, dv/dy), clamped to the
// chain; the lookups on levels floor(lambda) and floor(lambda) + 1 are
// blended with weights 1 - t and t, t = lambda - floor(lambda).
template <int FMT, int C, int MODE>
__global__ __launch_bounds__(256) void k_lookup_lod(LevelSet ls, const float* __restrict__ uv,
                                                    const float* __restrict__ tbn,
                                                    const float* __restrict__ view,
                                                    const float* __restrict__ duv,
                                                    float* __restrict__ out, FragMap m) {
    const int64_t f = frag_of(m, blockIdx.x, gridDim.x, threadIdx.x);
    if (f < 0) return;
    const Frag g = load_frag(uv, tbn, view, f);
    int l0;
    float t;
    lod_split(((const float4*)duv)[f], ls.W, ls.H, ls.levels, l0, t);
    const Dir dd = map_direction(g.m, g.w, ls.n);
    const Foot p = footprint(dd.sx, dd.sy, ls.n);
    float a[4] = {0.f, 0.f, 0.f, 0.f}, b[4] = {0.f, 0.f, 0.f, 0.f};
    level_lookup<FMT, C, MODE>(ls, l0, g, p, a);
    if (t > 0.f) {
        level_lookup<FMT, C, MODE>(ls, l0 + 1, g, p, b);
#pragma unroll
        for (int c = 0; c < C; c++) a[c] = (1.f - t) * a[c] + t * b[c];
    }
    store_out<C>(out, f, a);
}

template <int FMT, int MODE, bool DICT = false>
static hipError_t launch_fwd_c(const TexView& t, const float* uv, const float* tbn,
                               const float* view, float* out, const FragMap& m, hipStream_t s) {
    const uint32_t blocks = fragmap_blocks(m);
    switch (t.C) {
    case 1: hipLaunchKernelGGL((k_lookup_fwd<FMT, 1, MODE, DICT>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, view, out, m); break;
    case 2: hipLaunchKernelGGL((k_lookup_fwd<FMT, 2, MODE, DICT>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, view, out, m); break;
    case 3: hipLaunchKernelGGL((k_lookup_fwd<FMT, 3, MODE, DICT>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, view, out, m); break;
    default: hipLaunchKernelGGL((k_lookup_fwd<FMT, 4, MODE, DICT>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, view, out, m); break;
    }
    return hipGetLastError();
}

template <int FMT>
static hipError_t launch_fwd_staged_c(const TexView& t, const float* uv, const float* tbn,
                                      const float* view, float* out, const FragMap& m,
                                      hipStream_t s) {
    const uint32_t blocks = fragmap_blocks(m);
    const size_t shm = (size_t)4 * t.n * t.n * t.C * storage_bytes<FMT>();
    switch (t.C) {
    case 1: hipLaunchKernelGGL((k_lookup_fwd_staged<FMT, 1>), dim3(blocks), dim3(256), shm, s, t, uv, tbn, view, out, m); break;
    case 2: hipLaunchKernelGGL((k_lookup_fwd_staged<FMT, 2>), dim3(blocks), dim3(256), shm, s, t, uv, tbn, view, out, m); break;
    case 3: hipLaunchKernelGGL((k_lookup_fwd_staged<FMT, 3>), dim3(blocks), dim3(256), shm, s, t, uv, tbn, view, out, m); break;
    default: hipLaunchKernelGGL((k_lookup_fwd_staged<FMT, 4>), dim3(blocks), dim3(256), shm, s, t, uv, tbn, view, out, m); break;
    }
    return hipGetLastError();
}

bool lookup_staged_supported(const TexView& t, int fmt) {
    if (t.index || (fmt != FMT_F32 && fmt != FMT_BF16 && fmt != FMT_FP8)) return false;
    const int64_t bytes = (int64_t)t.n * t.n * t.C * (fmt == FMT_F32 ? 4 : fmt == FMT_BF16 ? 2 : 1);
    return bytes % 16 == 0 && bytes <= STAGED_BUCKET_BYTES;
}

hipError_t launch_lookup_fwd_staged(const TexView& t, int fmt, const float* uv, const float* tbn,
                                    const float* view, float* out, const FragMap& m,
                                    hipStream_t s) {
    if (m.N <= 0) return hipSuccess;
    hipError_t e;
    prof_begin(K_LOOKUP_FWD, s);
    if (fmt == FMT_F32) e = launch_fwd_staged_c<FMT_F32>(t, uv, tbn, view, out, m, s);
    else if (fmt == FMT_BF16) e = launch_fwd_staged_c<FMT_BF16>(t, uv, tbn, view, out, m, s);
    else e = launch_fwd_staged_c<FMT_FP8>(t, uv, tbn, view, out, m, s);
    prof_end(K_LOOKUP_FWD, s);
    return e;
}

hipError_t launch_lookup_fwd(const TexView& t, int fmt, int mode, const float* uv,
                             const float* tbn, const float* view, float* out, const FragMap& frags,
                             hipStream_t s) {
    if (frags.N <= 0) return hipSuccess;
    const FragMap m = with_frame_staging(frags, t, fmt);
    hipError_t e;
    prof_begin(K_LOOKUP_FWD, s);
    const uint32_t blocks = fragmap_blocks(m);
    if (t.index) {  // a bucket dictionary (F32 or BF16 codebook)
        if (mode == MODE_NEAREST) {
            if (fmt == FMT_F32) e = launch_fwd_c<FMT_F32, MODE_NEAREST, true>(t, uv, tbn, view, out, m, s);
            else e = launch_fwd_c<FMT_BF16, MODE_NEAREST, true>(t, uv, tbn, view, out, m, s);
        } else {
            if (fmt == FMT_F32) e = launch_fwd_c<FMT_F32, MODE_BILINEAR, true>(t, uv, tbn, view, out, m, s);
            else e = launch_fwd_c<FMT_BF16, MODE_BILINEAR, true>(t, uv, tbn, view, out, m, s);
        }
    } else if (fmt == FMT_BIT1) {
        if (mode == MODE_NEAREST)
            hipLaunchKernelGGL((k_lookup_fwd<FMT_BIT1, 1, MODE_NEAREST, false>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, view, out, m);
        else
            hipLaunchKernelGGL((k_lookup_fwd<FMT_BIT1, 1, MODE_BILINEAR, false>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, view, out, m);
        e = hipGetLastError();
    } else if (mode == MODE_NEAREST) {
        if (fmt == FMT_F32) e = launch_fwd_c<FMT_F32, MODE_NEAREST>(t, uv, tbn, view, out, m, s);
        else if (fmt == FMT_BF16) e = launch_fwd_c<FMT_BF16, MODE_NEAREST>(t, uv, tbn, view, out, m, s);
        else e = launch_fwd_c<FMT_FP8, MODE_NEAREST>(t, uv, tbn, view, out, m, s);
    } else {
        if (fmt == FMT_F32) e = launch_fwd_c<FMT_F32, MODE_BILINEAR>(t, uv, tbn, view, out, m, s);
        else if (fmt == FMT_BF16) e = launch_fwd_c<FMT_BF16, MODE_BILINEAR>(t, uv, tbn, view, out, m, s);
        else e = launch_fwd_c<FMT_FP8, MODE_BILINEAR>(t, uv, tbn, view, out, m, s);
    }
    prof_end(K_LOOKUP_FWD, s);
    return e;
}

template <int FMT, int MODE>
static void launch_lod_c(const LevelSet& ls, const float* uv, const float* tbn, const float* view,
                         const float* duv, float* out, const FragMap& m, hipStream_t s) {
    const uint32_t blocks = fragmap_blocks(m);
    switch (ls.C) {
    case 1: hipLaunchKernelGGL((k_lookup_lod<FMT, 1, MODE>), dim3(blocks), dim3(256), 0, s, ls, uv, tbn, view, duv, out, m); break;
    case 2: hipLaunchKernelGGL((k_lookup_lod<FMT, 2, MODE>), dim3(blocks), dim3(256), 0, s, ls, uv, tbn, view, duv, out, m); break;
    case 3: hipLaunchKernelGGL((k_lookup_lod<FMT, 3, MODE>), dim3(blocks), dim3(256), 0, s, ls, uv, tbn, view, duv, out, m); break;
    default: hipLaunchKernelGGL((k_lookup_lod<FMT, 4, MODE>), dim3(blocks), dim3(256), 0, s, ls, uv, tbn, view, duv, out, m); break;
    }
}

hipError_t launch_lookup_lod(const LevelSet& ls, int fmt, int mode, const float* uv,
                             const float* tbn, const float* view, const float* duv, float* out,
                             const FragMap& m, hipStream_t s) {
    if (m.N <= 0) return hipSuccess;
    prof_begin(K_LOOKUP_LOD, s);
    if (mode == MODE_NEAREST) {
        if (fmt == FMT_F32) launch_lod_c<FMT_F32, MODE_NEAREST>(ls, uv, tbn, view, duv, out, m, s);
        else if (fmt == FMT_BF16) launch_lod_c<FMT_BF16, MODE_NEAREST>(ls, uv, tbn, view, duv, out, m, s);
        else launch_lod_c<FMT_FP8, MODE_NEAREST>(ls, uv, tbn, view, duv, out, m, s);
    } else {
        if (fmt == FMT_F32) launch_lod_c<FMT_F32, MODE_BILINEAR>(ls, uv, tbn, view, duv, out, m, s);
        else if (fmt == FMT_BF16) launch_lod_c<FMT_BF16, MODE_BILINEAR>(ls, uv, tbn, view, duv, out, m, s);
        else launch_lod_c<FMT_FP8, MODE_BILINEAR>(ls, uv, tbn, view, duv, out, m, s);
    }
    prof_end(K_LOOKUP_LOD, s);
    return hipGetLastError();
}

hipError_t launch_debug_indices(const TexView& t, const float* uv, const float* tbn,
                                const float* view, int32_t* idx, float* frac, const FragMap& m,
                                hipStream_t s) {
    if (m.N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_debug_indices, dim3(fragmap_blocks(m)), dim3(256), 0, s, t, uv, tbn,
                       view, idx, frac, m);
    return hipGetLastError();
}

// In-bucket sample coordinate of a light direction for the light lookup:
// the steps of map_direction (u = M L, Eq. 1b in the k = 1/sqrt(|u| (|u| +
// u_z)) form, Eq. 3, the clamp) with the hardware square root, reciprocal
// square root and reciprocal (about 1 ulp each) in place of the correctly
// rounded ones.  Eq. 3's factor |A|_2 / |A|_inf is taken from u directly (k
// cancels).  The coordinate moves by a few ulp of n, far below the bilinear
// weights' tolerance, and an area light evaluates this once per sample, so
// the light lookup is bound by this arithmetic rather than by memory.
__device__ __forceinline__ void light_coord(const float M[9], const float L[3], int n, float& sx,
                                            float& sy) {
    const float ux = M[0] * L[0] + M[1] * L[1] + M[2] * L[2];
    const float uy = M[3] * L[0] + M[4] * L[1] + M[5] * L[2];
    const float uz = M[6] * L[0] + M[7] * L[1] + M[8] * L[2];
    const float rho2 = ux * ux + uy * uy;
    const float len = __builtin_amdgcn_sqrtf(rho2 + uz * uz);
    const float q = len * (len + uz);
    const float k = q > 0.f ? __builtin_amdgcn_rsqf(q) : 0.f;  // q = 0: u = -|u| N or 0
    const float mx = fmaxf(fabsf(ux), fabsf(uy));
    const float r = mx > 0.f ? __builtin_amdgcn_sqrtf(rho2) * __builtin_amdgcn_rcpf(mx) : 0.f;
    const float kr = k * r;
    const float half_n = 0.5f * (float)n;
    const float top = (float)(n - 1);
    sx = fminf(fmaxf((ux * kr + 1.0f) * half_n - 0.5f, 0.f), top);  // NaN -> 0
    sy = fminf(fmaxf((uy * kr + 1.0f) * half_n - 0.5f, 0.f), top);
}

// Light lookup: the bucket footprint depends on (u, v) only, so it is formed
// once per fragment; each light sample then maps its own direction and adds
// its bilinear taps.  The direction toward the light is the sample's vector
// (directional light) or the sample point minus the fragment's position
// (point light).  The samples live in the kernel's argument block and are
// read with scalar loads (every lane of a wave reads the same sample).
//
// CACHE (1-bit textures of n <= 16, several samples): the words of the
// fragment's buckets (at most 8 each) are copied once into LDS, word-major
// ([word][lane], so that lanes reading different words still hit distinct
// banks), and every tap of every sample is one LDS read instead of a global
// gather.  Each lane reads only its own column: no barrier is needed.
template <int FMT, int C, int MODE, bool CACHE, bool DICT>
__global__ __launch_bounds__(256) void k_lookup_light(TexView t, const float* __restrict__ uv,
                                                      const float* __restrict__ tbn,
                                                      const float* __restrict__ pos,
                                                      LightParams lp, float* __restrict__ out,
                                                      FragMap m) {
    constexpr int NB = MODE == MODE_NEAREST ? 1 : 4;
    __shared__ uint32_t cache[CACHE ? 8 * NB : 1][256];
    const int64_t f = frag_of(m, blockIdx.x, gridDim.x, threadIdx.x);
    if (f < 0) return;
    const float2 q = ((const float2*)uv)[f];
    float M[9];
#pragma unroll
    for (int k = 0; k < 9; k++) M[k] = tbn[f * 9 + k];
    float P[3] = {0.f, 0.f, 0.f};
    if (lp.kind == LIGHT_POINT) {
#pragma unroll
        for (int k = 0; k < 3; k++) P[k] = pos[f * 3 + k];
    }
    int64_t bk[NB];
    float bw[NB];
    if constexpr (MODE == MODE_NEAREST) {
        bk[0] = (int64_t)bucket_of(q.y, t.H) * t.W + bucket_of(q.x, t.W);
        bw[0] = 1.f;
    } else {
        int i0, i1, j0, j1;
        float a, bb;
        bucket_pair(q.x, t.W, i0, i1, a);
        bucket_pair(q.y, t.H, j0, j1, bb);
        bk[0] = (int64_t)j0 * t.W + i0;
        bk[1] = (int64_t)j0 * t.W + i1;
        bk[2] = (int64_t)j1 * t.W + i0;
        bk[3] = (int64_t)j1 * t.W + i1;
        bw[0] = (1.f - a) * (1.f - bb);
        bw[1] = a * (1.f - bb);
        bw[2] = (1.f - a) * bb;
        bw[3] = a * bb;
    }
    const int n = t.n;
    if constexpr (CACHE) {
        const int wpb = bit_words(n);
#pragma unroll
        for (int r = 0; r < NB; r++) {
            const uint32_t* src = (const uint32_t*)t.data + bk[r] * wpb;
#pragma unroll
            for (int w = 0; w < 8; w++) cache[r * 8 + w][threadIdx.x] = w < wpb ? src[w] : 0u;
        }
    }
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < lp.samples; s++) {
        float L[3];
#pragma unroll
        for (int k = 0; k < 3; k++) L[k] = lp.vec[s][k] - P[k];
        float sx, sy;
        light_coord(M, L, n, sx, sy);
        const Foot p = footprint(sx, sy, n);
        if constexpr (CACHE) {
            const int k00 = p.y0 * n + p.x0, k01 = p.y0 * n + p.x1;
            const int k10 = p.y1 * n + p.x0, k11 = p.y1 * n + p.x1;
            const float w00 = (1.f - p.fx) * (1.f - p.fy), w01 = p.fx * (1.f - p.fy);
            const float w10 = (1.f - p.fx) * p.fy, w11 = p.fx * p.fy;
#pragma unroll
            for (int r = 0; r < NB; r++) {
                const uint32_t* col = &cache[r * 8][threadIdx.x];
                const float t00 = (float)((col[(k00 >> 5) * 256] >> (k00 & 31)) & 1u);
                const float t01 = (float)((col[(k01 >> 5) * 256] >> (k01 & 31)) & 1u);
                const float t10 = (float)((col[(k10 >> 5) * 256] >> (k10 & 31)) & 1u);
                const float t11 = (float)((col[(k11 >> 5) * 256] >> (k11 & 31)) & 1u);
                acc[0] += bw[r] * (w00 * t00 + w01 * t01 + w10 * t10 + w11 * t11);
            }
        } else {
#pragma unroll
            for (int r = 0; r < NB; r++) bucket_bilerp<FMT, C, DICT>(t, bk[r], p, bw[r], acc);
        }
    }
#pragma unroll
    for (int c = 0; c < C; c++) acc[c] *= lp.inv_samples;
    store_out<C>(out, f, acc);
}

template <int FMT, int MODE, bool DICT = false>
static void launch_light_c(const TexView& t, const float* uv, const float* tbn, const float* pos,
                           const LightParams& lp, float* out, const FragMap& m, hipStream_t s) {
    const uint32_t blocks = fragmap_blocks(m);
    switch (t.C) {
    case 1: hipLaunchKernelGGL((k_lookup_light<FMT, 1, MODE, false, DICT>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, pos, lp, out, m); break;
    case 2: hipLaunchKernelGGL((k_lookup_light<FMT, 2, MODE, false, DICT>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, pos, lp, out, m); break;
    case 3: hipLaunchKernelGGL((k_lookup_light<FMT, 3, MODE, false, DICT>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, pos, lp, out, m); break;
    default: hipLaunchKernelGGL((k_lookup_light<FMT, 4, MODE, false, DICT>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, pos, lp, out, m); break;
    }
}

hipError_t launch_lookup_light(const TexView& t, int fmt, int mode, const float* uv,
                               const float* tbn, const float* pos, const LightParams& lp,
                               float* out, const FragMap& m, hipStream_t s) {
    if (m.N <= 0) return hipSuccess;
    prof_begin(K_LOOKUP_LIGHT, s);
    const uint32_t blocks = fragmap_blocks(m);
    if (fmt == FMT_BIT1) {
        // the LDS copy of the buckets pays off once several samples read them
        const bool cache = t.n <= 16 && lp.samples >= 4;
        if (mode == MODE_NEAREST) {
            if (cache) hipLaunchKernelGGL((k_lookup_light<FMT_BIT1, 1, MODE_NEAREST, true, false>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, pos, lp, out, m);
            else hipLaunchKernelGGL((k_lookup_light<FMT_BIT1, 1, MODE_NEAREST, false, false>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, pos, lp, out, m);
        } else {
            if (cache) hipLaunchKernelGGL((k_lookup_light<FMT_BIT1, 1, MODE_BILINEAR, true, false>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, pos, lp, out, m);
            else hipLaunchKernelGGL((k_lookup_light<FMT_BIT1, 1, MODE_BILINEAR, false, false>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, pos, lp, out, m);
        }
    } else if (t.index) {  // a bucket dictionary (F32 or BF16 codebook)
        if (mode == MODE_NEAREST) {
            if (fmt == FMT_F32) launch_light_c<FMT_F32, MODE_NEAREST, true>(t, uv, tbn, pos, lp, out, m, s);
            else launch_light_c<FMT_BF16, MODE_NEAREST, true>(t, uv, tbn, pos, lp, out, m, s);
        } else {
            if (fmt == FMT_F32) launch_light_c<FMT_F32, MODE_BILINEAR, true>(t, uv, tbn, pos, lp, out, m, s);
            else launch_light_c<FMT_BF16, MODE_BILINEAR, true>(t, uv, tbn, pos, lp, out, m, s);
        }
    } else if (mode == MODE_NEAREST) {
        if (fmt == FMT_F32) launch_light_c<FMT_F32, MODE_NEAREST>(t, uv, tbn, pos, lp, out, m, s);
        else if (fmt == FMT_BF16) launch_light_c<FMT_BF16, MODE_NEAREST>(t, uv, tbn, pos, lp, out, m, s);
        else launch_light_c<FMT_FP8, MODE_NEAREST>(t, uv, tbn, pos, lp, out, m, s);
    } else {
        if (fmt == FMT_F32) launch_light_c<FMT_F32, MODE_BILINEAR>(t, uv, tbn, pos, lp, out, m, s);
        else if (fmt == FMT_BF16) launch_light_c<FMT_BF16, MODE_BILINEAR>(t, uv, tbn, pos, lp, out, m, s);
        else launch_light_c<FMT_FP8, MODE_BILINEAR>(t, uv, tbn, pos, lp, out, m, s);
    }
    prof_end(K_LOOKUP_LIGHT, s);
    return hipGetLastError();
}

}  // namespace rt
