// rt_device.hpp -- device-side building blocks shared by the gfx950 kernels of
// the radiance-bucket lookup: the incidence -> bucket mapping in binary32,
// texel loads and decodes for the storage formats, the sample directions of
// the bake, and launch helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rt {

constexpr int FMT_F32 = 0;
constexpr int FMT_BF16 = 1;
constexpr int FMT_FP8 = 2;
constexpr int FMT_BIT1 = 3;  // one bit per sample, one channel

// 32-bit words per bucket of the 1-bit storage: sample k = y n + x is bit
// k % 32 of word k / 32 of its bucket; the bits past n n are zero.
__host__ __device__ __forceinline__ int bit_words(int n) { return (n * n + 31) >> 5; }

constexpr int MODE_NEAREST = 0;
constexpr int MODE_BILINEAR = 1;

// Native vector types (for non-temporal loads and stores).
typedef float f4v __attribute__((ext_vector_type(4)));
typedef uint32_t u2v __attribute__((ext_vector_type(2)));

// Texture as seen by a kernel: bucket-major [H][W][n][n][C].  A bucket
// dictionary keeps `entries` buckets in data (its codebook) and an index map
// [H][W] (1, 2 or 4 bytes per bucket) naming each bucket's entry, with an
// optional gain per bucket.
struct TexView {
    const void* data;     // FMT_BIT1: uint32 words, bit_words(n) per bucket
    const float* scales;  // [H][W], FP8 only
    int W, H, n, C;
    const void* index;    // dictionary: entry of each bucket, or nullptr
    const float* gains;   // dictionary: gain of each bucket, or nullptr (1)
    int index_bytes;      // 1, 2 or 4
    int entries;          // dictionary: codebook entries K
};

// Entry of bucket b of a dictionary; numbers past the codebook read its last
// entry (the index map is caller data that the host cannot check).
__device__ __forceinline__ int64_t dict_entry(const TexView& t, int64_t b) {
    uint32_t e;
    if (t.index_bytes == 1) e = ((const uint8_t*)t.index)[b];
    else if (t.index_bytes == 2) e = ((const uint16_t*)t.index)[b];
    else e = ((const uint32_t*)t.index)[b];
    return (int64_t)min(e, (uint32_t)(t.entries - 1));
}

// A mip chain: level l has max(1, W >> l) x max(1, H >> l) buckets of the
// same n, C and format; only the storage pointers differ per level.
constexpr int MAX_LEVELS = 17;
struct LevelSet {
    const void* data[MAX_LEVELS];
    const float* scales[MAX_LEVELS];
    int levels;
    int W, H, n, C;  // level 0
};

// ---------------------------------------------------------------------------
// Launch geometry: gfx950 places consecutive workgroups of a launch on its 8
// XCDs round-robin.  Renumbering the workgroups so that each XCD receives a
// contiguous range of the logical index space keeps neighbouring fragments
// (which land in the same buckets) on the same L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xcd_block_id(uint32_t bid, uint32_t nblocks) {
    constexpr uint32_t XCDS = 8;
    uint32_t xcd = bid % XCDS;
    uint32_t q = nblocks / XCDS, r = nblocks % XCDS;
    uint32_t before = xcd * q + (xcd < r ? xcd : r);
    return before + bid / XCDS;
}

// ---------------------------------------------------------------------------
// Decodes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// E4M3 byte -> binary32 value divided by 2^8.  The byte's exponent and
// mantissa fields are placed in the corresponding fields of a binary16 (whose
// exponent bias is 8 larger), which represents e4m3 * 2^-8 exactly for every
// finite code, subnormals included; the 2^8 is folded into the bucket scale.
__device__ __forceinline__ float e4m3_div256(uint32_t byte) {
    uint32_t h = ((byte & 0x80u) << 8) | ((byte & 0x7Fu) << 7);
    return (float)__builtin_bit_cast(_Float16, (unsigned short)h);
}

struct F4 {
    float v[4];
};

// Load the C channels of texel `t` (index in texels, bucket-major) as
// binary32.  For FP8 the values are e4m3/256; the caller multiplies by
// 256 * scale once per bucket.
template <int FMT, int C>
__device__ __forceinline__ F4 load_texel(const void* __restrict__ data, int64_t t) {
    F4 r;
#pragma unroll
    for (int c = 0; c < 4; c++) r.v[c] = 0.f;
    if constexpr (FMT == FMT_F32) {
        const float* p = (const float*)data;
        if constexpr (C == 4) {
            float4 q = ((const float4*)p)[t];
            r.v[0] = q.x; r.v[1] = q.y; r.v[2] = q.z; r.v[3] = q.w;
        } else if constexpr (C == 2) {
            float2 q = ((const float2*)p)[t];
            r.v[0] = q.x; r.v[1] = q.y;
        } else {
#pragma unroll
            for (int c = 0; c < C; c++) r.v[c] = p[t * C + c];
        }
    } else if constexpr (FMT == FMT_BF16) {
        const uint16_t* p = (const uint16_t*)data;
        if constexpr (C == 4) {
            uint2 q = ((const uint2*)p)[t];
            r.v[0] = bf16_lo(q.x); r.v[1] = bf16_hi(q.x);
            r.v[2] = bf16_lo(q.y); r.v[3] = bf16_hi(q.y);
        } else if constexpr (C == 2) {
            uint32_t q = ((const uint32_t*)p)[t];
            r.v[0] = bf16_lo(q); r.v[1] = bf16_hi(q);
        } else {
#pragma unroll
            for (int c = 0; c < C; c++) r.v[c] = bf16_lo((uint32_t)p[t * C + c]);
        }
    } else {
        const uint8_t* p = (const uint8_t*)data;
        if constexpr (C == 4) {
            uint32_t q = ((const uint32_t*)p)[t];
#pragma unroll
            for (int c = 0; c < 4; c++) r.v[c] = e4m3_div256((q >> (8 * c)) & 0xFFu);
        } else if constexpr (C == 2) {
            uint32_t q = ((const uint16_t*)p)[t];
            r.v[0] = e4m3_div256(q & 0xFFu); r.v[1] = e4m3_div256(q >> 8);
        } else {
#pragma unroll
            for (int c = 0; c < C; c++) r.v[c] = e4m3_div256((uint32_t)p[t * C + c]);
        }
    }
    return r;
}

// Bytes of one stored sample value (channel) in format FMT (not RT_FMT_BIT1).
template <int FMT>
__host__ __device__ constexpr int storage_bytes() {
    return FMT == FMT_F32 ? 4 : FMT == FMT_BF16 ? 2 : 1;
}

// Orders a wavefront's LDS accesses before and after it (the wavefront owns
// the memory, so no workgroup barrier is needed).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Factor applied to a bucket's decoded samples: 1, or 256 * scale for FP8.
template <int FMT>
__device__ __forceinline__ float bucket_factor(const float* __restrict__ scales, int64_t b) {
    if constexpr (FMT == FMT_FP8) return 256.0f * scales[b];
    else return 1.0f;
}

// ---------------------------------------------------------------------------
// Fragment inputs.
// ---------------------------------------------------------------------------

// Which fragment a thread handles.  Flat: workgroup b, thread t -> 256 b + t.
// Tiled (the caller's images of height x width pixels): workgroup b is one
// TILE_X x TILE_Y pixel tile, tiles row-major within an image and images in
// order, so the fragments of one workgroup are neighbouring pixels and
// neighbouring workgroups are neighbouring tiles.  Either way the workgroup
// index is first renumbered with xcd_block_id.
constexpr int TILE_X = 32, TILE_Y = 8;
static_assert(TILE_X * TILE_Y == 256, "one tile per 256-thread workgroup");

struct FragMap {
    int64_t N;
    int32_t width, height;     // 0: flat
    int32_t tiles_x, tiles_y;  // tiles per row and per column of an image
    int32_t stage;             // flat launches: stage the frames in LDS
};

inline FragMap make_fragmap(int64_t N, int32_t views, int32_t height, int32_t width) {
    FragMap m{N, 0, 0, 0, 0, 0};
    if (views > 0 && height > 0 && width > 0) {
        m.width = width;
        m.height = height;
        m.tiles_x = (width + TILE_X - 1) / TILE_X;
        m.tiles_y = (height + TILE_Y - 1) / TILE_Y;
    }
    return m;
}

// Flat launches of the lookup and of its per-fragment backward stage their
// fragments' frames and view vectors through LDS (load_frag_block) when the
// texture is larger than the caches.  Then the taps come from HBM and the
// launch is bound by its memory instructions, which the 16-byte staging
// loads reduce; on a texture the caches hold the launch is bound by issue,
// and the staging's LDS traffic costs more than it saves.
constexpr int64_t STAGE_FRAMES_MIN_TEXTURE_BYTES = int64_t(1) << 30;

inline FragMap with_frame_staging(FragMap m, const TexView& t, int fmt) {
    int64_t bytes = 0;
    if (!t.index) {
        const int64_t buckets = (int64_t)t.W * t.H;
        if (fmt == FMT_BIT1) bytes = buckets * bit_words(t.n) * 4;
        else bytes = buckets * t.n * t.n * t.C * (fmt == FMT_F32 ? 4 : fmt == FMT_BF16 ? 2 : 1);
    }
    m.stage = m.width == 0 && bytes >= STAGE_FRAMES_MIN_TEXTURE_BYTES ? 1 : 0;
    return m;
}

// workgroups of a launch over all fragments
inline uint32_t fragmap_blocks(const FragMap& m) {
    if (m.width == 0) return (uint32_t)((m.N + 255) / 256);
    const int64_t views = m.N / ((int64_t)m.width * m.height);
    return (uint32_t)(views * m.tiles_x * m.tiles_y);
}

// fragment of thread `tid` in workgroup `bid`, or -1 past the end / outside
// the image
__device__ __forceinline__ int64_t frag_of(const FragMap& m, uint32_t bid, uint32_t nblocks,
                                           int tid) {
    const uint32_t b = xcd_block_id(bid, nblocks);
    if (m.width == 0) {
        const int64_t f = (int64_t)b * 256 + tid;
        return f < m.N ? f : -1;
    }
    const uint32_t per_view = (uint32_t)(m.tiles_x * m.tiles_y);
    const uint32_t v = b / per_view, r = b - v * per_view;
    const uint32_t ty = r / (uint32_t)m.tiles_x, tx = r - ty * (uint32_t)m.tiles_x;
    const int x = (int)tx * TILE_X + (tid % TILE_X), y = (int)ty * TILE_Y + (tid / TILE_X);
    if (x >= m.width || y >= m.height) return -1;
    return ((int64_t)v * m.height + y) * m.width + x;
}

struct Frag {
    float u, v;
    float m[9];
    float w[3];
};

__device__ __forceinline__ Frag load_frag(const float* __restrict__ uv, const float* __restrict__ tbn,
                                          const float* __restrict__ view, int64_t f) {
    Frag r;
    float2 t = ((const float2*)uv)[f];
    r.u = t.x;
    r.v = t.y;
#pragma unroll
    for (int k = 0; k < 9; k++) r.m[k] = tbn[f * 9 + k];
#pragma unroll
    for (int k = 0; k < 3; k++) r.w[k] = view[f * 3 + k];
    return r;
}

// The frames and view vectors of a flat launch's wavefront (64 consecutive
// fragments) staged in LDS.  A fragment's 36 + 12 bytes do not fall on a
// lane's 16-byte vector, but the wavefront's 2304 + 768 bytes do: they are
// read with 16-byte loads when both arrays are 16-byte aligned there, else
// with 4-byte loads, and every lane then takes its own record from LDS (a
// stride of 9 or 3 words: no bank conflicts).  Each wavefront stages its own
// records, so no workgroup barrier couples the wavefronts.  Tiled launches
// read per lane.
struct FragStage {
    float tbn[256 * 9];
    float view[256 * 3];
};

// Returns the record of fragment f (f >= 0); every lane of a wavefront must
// reach it together.
__device__ __forceinline__ Frag load_frag_block(const float* __restrict__ uv,
                                                const float* __restrict__ tbn,
                                                const float* __restrict__ view, const FragMap& m,
                                                int64_t f, FragStage& s) {
    if (m.width != 0 || !m.stage) return f >= 0 ? load_frag(uv, tbn, view, f) : Frag{};
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t f0 = (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * 256 + w * 64;
    const int nf = (int)(m.N - f0 < 64 ? (m.N - f0 > 0 ? m.N - f0 : 0) : 64);
    const float* bt = tbn + f0 * 9;
    const float* bv = view + f0 * 3;
    float* st = s.tbn + w * 64 * 9;
    float* sv = s.view + w * 64 * 3;
    if (nf == 64 && ((((uintptr_t)bt) | ((uintptr_t)bv)) & 15) == 0) {
        for (int q = lane; q < 144; q += 64) ((f4v*)st)[q] = ((const f4v*)bt)[q];
        if (lane < 48) ((f4v*)sv)[lane] = ((const f4v*)bv)[lane];
    } else {
        for (int q = lane; q < nf * 9; q += 64) st[q] = bt[q];
        for (int q = lane; q < nf * 3; q += 64) sv[q] = bv[q];
    }
    wave_lds_sync();
    Frag r{};
    if (f >= 0) {
        const float2 t = ((const float2*)uv)[f];
        r.u = t.x;
        r.v = t.y;
#pragma unroll
        for (int k = 0; k < 9; k++) r.m[k] = st[lane * 9 + k];
#pragma unroll
        for (int k = 0; k < 3; k++) r.w[k] = sv[lane * 3 + k];
    }
    return r;
}

// ---------------------------------------------------------------------------
// Incidence -> in-bucket sample coordinate, binary32.
//
//   u = M V (rows T, B, N), L = |u|
//   Eq. (1b) with I = u / L:  A = sqrt(2) (I_x, I_y) / |(I_x, I_y, I_z + 1)|.
//   For unit I, |(I_x, I_y, I_z + 1)|^2 = 2 (1 + I_z), so A = (u_x, u_y) k with
//   k = 1 / sqrt(L (L + u_z)); this form avoids normalising u first.
//   Eq. (3): B = (|A|_2 / max(|A_x|, |A_y|)) A, B = 0 at A = 0.
//   Clamp (Note after Eq. 3) and texel centres: s = clamp((B + 1) n/2 - 1/2, 0, n-1).
// ---------------------------------------------------------------------------
struct Dir {
    float sx, sy;        // clamped sample coordinates
    bool clx, cly;       // axis at or beyond its clamp bound
    float ax, ay;        // A
    float ux, uy, uz, L; // tangent-space incidence before normalisation
    float k;             // 1 / sqrt(L (L + u_z))
};

// The mapping is evaluated with one rounding per operation (no fused
// multiply-adds), so that every kernel that maps a fragment -- the lookups,
// the backward, the visit plan -- computes the same sample coordinate and the
// same footprint for it, whatever the surrounding code lets the compiler fuse.
__device__ __forceinline__ Dir map_direction(const float m[9], const float w[3], int n) {
#pragma clang fp contract(off)
    Dir d;
    d.ux = m[0] * w[0] + m[1] * w[1] + m[2] * w[2];
    d.uy = m[3] * w[0] + m[4] * w[1] + m[5] * w[2];
    d.uz = m[6] * w[0] + m[7] * w[1] + m[8] * w[2];
    d.L = sqrtf(d.ux * d.ux + d.uy * d.uy + d.uz * d.uz);
    float q = d.L * (d.L + d.uz);
    d.k = q > 0.f ? 1.0f / sqrtf(q) : 0.f;  // q = 0: I = -N (or u = 0): A = 0
    d.ax = d.ux * d.k;
    d.ay = d.uy * d.k;
    float rho = sqrtf(d.ax * d.ax + d.ay * d.ay);
    float mx = fmaxf(fabsf(d.ax), fabsf(d.ay));
    float r = mx > 0.f ? rho / mx : 0.f;
    float bx = d.ax * r, by = d.ay * r;
    float half_n = 0.5f * (float)n;
    float top = (float)(n - 1);
    float sx = (bx + 1.0f) * half_n - 0.5f;
    float sy = (by + 1.0f) * half_n - 0.5f;
    d.clx = !(sx > 0.f && sx < top);
    d.cly = !(sy > 0.f && sy < top);
    d.sx = fminf(fmaxf(sx, 0.f), top);  // NaN -> 0
    d.sy = fminf(fmaxf(sy, 0.f), top);
    return d;
}

// Bilinear footprint inside a bucket.  The first sample is kept at or below
// n-2 so that the second is always x0+1 (at s = n-1 the weight of the first is
// then exactly 0); for n = 1 both are sample 0.
struct Foot {
    int x0, y0, x1, y1;
    float fx, fy;
};

__device__ __forceinline__ Foot footprint(float sx, float sy, int n) {
#pragma clang fp contract(off)
    Foot p;
    int hi = n >= 2 ? n - 2 : 0;
    p.x0 = min((int)sx, hi);
    p.y0 = min((int)sy, hi);
    p.x1 = min(p.x0 + 1, n - 1);
    p.y1 = min(p.y0 + 1, n - 1);
    p.fx = sx - (float)p.x0;
    p.fy = sy - (float)p.y0;
    if (n == 1) { p.fx = 0.f; p.fy = 0.f; }
    return p;
}

// Bucket column (or row) of a texture coordinate: floor(frac(u) W) with the UV
// plane repeating.  It is evaluated as floor(u W) mod W, which is the same
// integer, because u W is exact for a power-of-two W whereas frac(u) = u + 1
// of a small negative u is not representable in binary32.  Non-finite and
// huge coordinates (where binary32 has no fraction left) select bucket 0.
__device__ __forceinline__ int bucket_of(float u, int W) {
    const float fq = floorf(u * (float)W);
    if (!(fabsf(fq) < 1073741824.0f)) return 0;
    const int i = (int)fq % W;
    return i < 0 ? i + W : i;
}

// Bilinear-bucket footprint in UV: p = frac(u) W - 1/2, columns floor(p) and
// floor(p)+1 (wrapping), weight a = p - floor(p).  Evaluated from t = u W
// (exact for a power-of-two W) split into floor(t) and r = t - floor(t)
// (exact, except for -1/2 < t < 0 where it rounds by at most 2^-25); then
// a = r - 1/2 (exact) or r + 1/2 (rounded by at most 2^-25).  The weight is
// thus within 2^-24 however large u W is, whereas forming u W - 1/2 first
// would round it to the ulp of u W.  Non-finite and huge coordinates behave
// as u = 0.
__device__ __forceinline__ void bucket_pair(float u, int W, int& i0, int& i1, float& a) {
    const float t = u * (float)W;
    const float ft = floorf(t);
    if (!(fabsf(ft) < 1073741824.0f)) {
        i0 = W - 1;
        i1 = 0;
        a = 0.5f;
        return;
    }
    const float r = t - ft;
    int k = (int)ft;
    if (r >= 0.5f) {
        a = r - 0.5f;
    } else {
        a = r + 0.5f;
        k -= 1;
    }
    k %= W;
    i0 = k < 0 ? k + W : k;
    i1 = i0 + 1 == W ? 0 : i0 + 1;
}

// Level of detail of a fragment from its UV screen derivatives d = (du/dx,
// dv/dx, du/dy, dv/dy): rho = the larger pixel footprint in buckets of level 0
// (W x H), lambda = log2 rho clamped to [0, levels - 1] (0 when rho is 0 or
// not finite); the lookup blends levels l0 = floor(lambda) and l0 + 1 with
// weights 1 - t and t (t = 0 on the last level).
__device__ __forceinline__ void lod_split(const float4 d, int W, int H, int levels, int& l0,
                                          float& t) {
    const float ax = d.x * (float)W, ay = d.y * (float)H;
    const float bx = d.z * (float)W, by = d.w * (float)H;
    const float rho = fmaxf(sqrtf(ax * ax + ay * ay), sqrtf(bx * bx + by * by));
    float lambda = 0.f;
    if (rho > 0.f && rho <= 3.0e38f) lambda = fminf(fmaxf(log2f(rho), 0.f), (float)(levels - 1));
    l0 = (int)floorf(lambda);
    t = lambda - (float)l0;
    if (l0 >= levels - 1) {
        l0 = levels - 1;
        t = 0.f;
    }
}

// ---------------------------------------------------------------------------
// Sample centres of a bucket as directions (the write side: Eqs. 4a, 4b, 2c).
// At sample (x, y) of an n x n bucket: B = ((2x+1)/n - 1, (2y+1)/n - 1);
// A = max(|B_x|, |B_y|) / |B| B (A = 0 at B = 0); the reflection vector
// R = (-A_x w, -A_y w, 1 - |A|^2), w = sqrt(2 - |A|^2), and the incidence
// I = (A_x w, A_y w, 1 - |A|^2) that the lookup maps onto the sample (R
// mirrored about the normal).
// ---------------------------------------------------------------------------
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

}  // namespace rt
