// rt_backward.hip -- deterministic backward of the radiance-bucket lookup for
// gfx950.
//
//   1. k_bwd_fragment   one lane per fragment: recompute the mapping, write
//                       dL/dview (chain through the bilinear weights, the
//                       clamp, Eq. 3, Eq. 1b and the normalisation) and
//                       dL/duv, and emit one record per (fragment, bucket):
//                       key = bucket << cell_bits | (y0 n + x0).
//   2. radix sort       stable LSD sort of (key, record) by digits of up to
//                       10 bits (9 for large inputs): per-tile digit
//                       histograms, one exclusive scan over (digit, tile),
//                       stable in-tile ranking with wave ballots.  Equal keys
//                       keep record order, so the sorted sequence depends only
//                       on the inputs.
//   3. k_bucket_ranges  [start, end) of every bucket in the sorted records.
//      k_payload        (buckets of at most 64 records on average) the
//                       fractions and weighted upstream gradient of the
//                       records of buckets with at most 64 records, written in
//                       sorted order.
//   4. k_segacc         eight buckets per wavefront (pass 1): the records of a
//                       bucket with at most 64 are held in a register window
//                       (read from the payload, or gathered from the
//                       fragments) and reduced per cell by a segmented scan
//                       across lanes with a fixed shape; the four cell sums are
//                       added to the texels of the cell in four ordered phases
//                       in LDS, and the n x n x C tile is written once.
//                       Untouched buckets get zeros.  Buckets with 65..PIECE
//                       records go to k_segacc_big (rounds of 64 with a
//                       carry), more to pass 2.
//   5. k_segacc_hot /   pass 2: hot buckets are cut at fixed chunk boundaries of
//      k_combine_hot    the sorted records; each chunk's part is reduced as in
//                       pass 1 into a partial tile, and the partials are summed
//                       in chunk order.
// No float atomics are used, and every summation order is a function of the
// sorted records alone, so the gradient is bitwise reproducible.
#include <algorithm>

#include "rt_device.hpp"
#include "rt_kernels.hpp"

namespace rt {

constexpr int SORT_THREADS = 256;
constexpr int SORT_IPT = 16;
constexpr int SORT_TILE = SORT_THREADS * SORT_IPT;  // 4096
constexpr int SCAN_TILE = 4096;
constexpr int64_t SCAN_FUSED_BLOCKS = 4096;

// ---------------------------------------------------------------------------
// 1. per-fragment backward
// ---------------------------------------------------------------------------

// dL/dA from dL/dB through Eq. (3).  On the branch |A_x| >= |A_y|,
// B = (rho sgn A_x, rho A_y / |A_x|); the other branch mirrors it; at A = 0
// the map's limit along the axes (identity) is used.
__device__ __forceinline__ void square_vjp(float ax, float ay, float gbx, float gby, float& gax,
                                           float& gay) {
    float rho = sqrtf(ax * ax + ay * ay);
    if (!(rho > 0.f)) {
        gax = gbx;
        gay = gby;
        return;
    }
    if (fabsf(ax) >= fabsf(ay)) {
        float sx = ax >= 0.f ? 1.f : -1.f;
        float j00 = fabsf(ax) / rho, j01 = sx * ay / rho;
        float j10 = -sx * ay * ay * ay / (rho * ax * ax);
        float j11 = (ay * ay + rho * rho) / (rho * fabsf(ax));
        gax = j00 * gbx + j10 * gby;
        gay = j01 * gbx + j11 * gby;
    } else {
        float sy = ay >= 0.f ? 1.f : -1.f;
        float j11 = fabsf(ay) / rho, j10 = sy * ax / rho;
        float j01 = -sy * ax * ax * ax / (rho * ay * ay);
        float j00 = (ax * ax + rho * rho) / (rho * fabsf(ay));
        gax = j00 * gbx + j10 * gby;
        gay = j01 * gbx + j11 * gby;
    }
}

// Per-bucket part of the per-fragment backward: dL/ds (x, y) and sum_c g_c * value.
template <int FMT, int C>
__device__ __forceinline__ void bucket_grads(const TexView& t, int64_t b, const Foot& p,
                                             const float go[4], float& dsx, float& dsy,
                                             float& lval) {
    const int n = t.n;
    const int64_t base = b * (int64_t)(n * n);
    F4 t00 = load_texel<FMT, C>(t.data, base + p.y0 * n + p.x0);
    F4 t01 = load_texel<FMT, C>(t.data, base + p.y0 * n + p.x1);
    F4 t10 = load_texel<FMT, C>(t.data, base + p.y1 * n + p.x0);
    F4 t11 = load_texel<FMT, C>(t.data, base + p.y1 * n + p.x1);
    float f = bucket_factor<FMT>(t.scales, b);
    float gx = 0.f, gy = 0.f, lv = 0.f;
    float w00 = (1.f - p.fx) * (1.f - p.fy), w01 = p.fx * (1.f - p.fy);
    float w10 = (1.f - p.fx) * p.fy, w11 = p.fx * p.fy;
#pragma unroll
    for (int c = 0; c < C; c++) {
        gx += go[c] * ((1.f - p.fy) * (t01.v[c] - t00.v[c]) + p.fy * (t11.v[c] - t10.v[c]));
        gy += go[c] * ((1.f - p.fx) * (t10.v[c] - t00.v[c]) + p.fx * (t11.v[c] - t01.v[c]));
        lv += go[c] * (w00 * t00.v[c] + w01 * t01.v[c] + w10 * t10.v[c] + w11 * t11.v[c]);
    }
    dsx = f * gx;
    dsy = f * gy;
    lval = f * lv;
}

// Bilinear-bucket mode: the slopes dL/ds of the four buckets (weighted by
// their bucket weights wb, as bucket_grads forms them) and dL/du, dL/dv.  The
// uv derivatives are formed from the differences of corresponding taps of
// neighbouring buckets, each tap times its bucket's factor, so their rounding
// follows the size of those differences rather than of the texel values:
//   dL/du = W sum_c g_c sum_taps w_tap [(1 - b)(T(i1,j0) - T(i0,j0)) + b (T(i1,j1) - T(i0,j1))]
//   dL/dv = H sum_c g_c sum_taps w_tap [(1 - a)(T(i0,j1) - T(i0,j0)) + a (T(i1,j1) - T(i1,j0))]
// with the buckets ordered (i0,j0), (i1,j0), (i0,j1), (i1,j1).
template <int FMT, int C>
__device__ __forceinline__ void pair_grads(const TexView& t, const int64_t bk[4], const float wb[4],
                                           float a, float bb, const Foot& p, const float go[4],
                                           bool want_uv, float& gsx, float& gsy, float& gu,
                                           float& gv) {
    const int n = t.n;
    float T[4][4][4];  // [bucket][tap 00, 01, 10, 11][channel], times the bucket factor
    gsx = 0.f;
    gsy = 0.f;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int64_t base = bk[k] * (int64_t)(n * n);
        const F4 t00 = load_texel<FMT, C>(t.data, base + p.y0 * n + p.x0);
        const F4 t01 = load_texel<FMT, C>(t.data, base + p.y0 * n + p.x1);
        const F4 t10 = load_texel<FMT, C>(t.data, base + p.y1 * n + p.x0);
        const F4 t11 = load_texel<FMT, C>(t.data, base + p.y1 * n + p.x1);
        const float f = bucket_factor<FMT>(t.scales, bk[k]);
        float gx = 0.f, gy = 0.f;
#pragma unroll
        for (int c = 0; c < C; c++) {
            gx += go[c] * ((1.f - p.fy) * (t01.v[c] - t00.v[c]) + p.fy * (t11.v[c] - t10.v[c]));
            gy += go[c] * ((1.f - p.fx) * (t10.v[c] - t00.v[c]) + p.fx * (t11.v[c] - t01.v[c]));
            T[k][0][c] = f * t00.v[c];
            T[k][1][c] = f * t01.v[c];
            T[k][2][c] = f * t10.v[c];
            T[k][3][c] = f * t11.v[c];
        }
        gsx += wb[k] * (f * gx);
        gsy += wb[k] * (f * gy);
    }
    gu = 0.f;
    gv = 0.f;
    if (!want_uv) return;
    const float w[4] = {(1.f - p.fx) * (1.f - p.fy), p.fx * (1.f - p.fy), (1.f - p.fx) * p.fy,
                        p.fx * p.fy};
    float su = 0.f, sv = 0.f;
#pragma unroll
    for (int c = 0; c < C; c++) {
        float du = 0.f, dv = 0.f;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            du += w[q] * ((1.f - bb) * (T[1][q][c] - T[0][q][c]) + bb * (T[3][q][c] - T[2][q][c]));
            dv += w[q] * ((1.f - a) * (T[2][q][c] - T[0][q][c]) + a * (T[3][q][c] - T[1][q][c]));
        }
        su += go[c] * du;
        sv += go[c] * dv;
    }
    gu = (float)t.W * su;
    gv = (float)t.H * sv;
}

// The per-fragment outputs (view and uv gradients, and in nearest mode the
// sort keys and fractions) are stored non-temporally: they are written once
// and read back, if at all, by later passes over millions of records.
__device__ __forceinline__ void nt_store2(float* p, float a, float b) {
    __builtin_nontemporal_store(a, p);
    __builtin_nontemporal_store(b, p + 1);
}

template <int FMT, int C, int MODE>
__global__ __launch_bounds__(256) void k_bwd_fragment(
    TexView t, const float* __restrict__ uv, const float* __restrict__ tbn,
    const float* __restrict__ view, const float* __restrict__ grad_out,
    float* __restrict__ grad_view, float* __restrict__ grad_uv, uint32_t* __restrict__ keys,
    float* __restrict__ wrec, FragMap m, int cell_bits, uint32_t sentinel) {
    __shared__ FragStage stage;
    const int64_t f = frag_of(m, blockIdx.x, gridDim.x, threadIdx.x);
    const int n = t.n;
    float go[4] = {0.f, 0.f, 0.f, 0.f};
    bool zero = true;
    if (f >= 0) {
#pragma unroll
        for (int c = 0; c < C; c++) {
            go[c] = grad_out[f * C + c];
            zero = zero && go[c] == 0.f;
        }
    }
    Frag g;
    if (sentinel == 0u) {
        // every fragment contributes: its frame comes from the wavefront's
        // staged block (every lane takes part in staging it)
        g = load_frag_block(uv, tbn, view, m, f, stage);
        if (f < 0) return;
    } else if (f < 0) {
        return;
    } else if (zero) {
        // sparse plan: no contribution, no records; its gradients are 0
        if (grad_view) {
            grad_view[f * 3 + 0] = 0.f;
            grad_view[f * 3 + 1] = 0.f;
            grad_view[f * 3 + 2] = 0.f;
        }
        if (grad_uv) nt_store2(grad_uv + 2 * f, 0.f, 0.f);
        if (keys) {
            if constexpr (MODE == MODE_NEAREST) keys[f] = sentinel;
            else ((uint4*)keys)[f] = make_uint4(sentinel, sentinel, sentinel, sentinel);
        }
        return;
    } else {
        g = load_frag(uv, tbn, view, f);
    }
    Dir d = map_direction(g.m, g.w, n);
    Foot p = footprint(d.sx, d.sy, n);
    const uint32_t cell = (uint32_t)(p.y0 * n + p.x0);

    float gsx = 0.f, gsy = 0.f;
    if constexpr (MODE == MODE_NEAREST) {
        int i = bucket_of(g.u, t.W), j = bucket_of(g.v, t.H);
        int64_t b = (int64_t)j * t.W + i;
        float lv;
        if (grad_view) bucket_grads<FMT, C>(t, b, p, go, gsx, gsy, lv);
        if (grad_uv) nt_store2(grad_uv + 2 * f, 0.f, 0.f);
        if (keys) {
            __builtin_nontemporal_store(((uint32_t)b << cell_bits) | cell, keys + f);
            nt_store2(wrec + 2 * f, p.fx, p.fy);
        }
    } else {
        int i0, i1, j0, j1;
        float a, bb;
        bucket_pair(g.u, t.W, i0, i1, a);
        bucket_pair(g.v, t.H, j0, j1, bb);
        const int64_t bk[4] = {(int64_t)j0 * t.W + i0, (int64_t)j0 * t.W + i1,
                               (int64_t)j1 * t.W + i0, (int64_t)j1 * t.W + i1};
        const float wb[4] = {(1.f - a) * (1.f - bb), a * (1.f - bb), (1.f - a) * bb, a * bb};
        if (grad_view || grad_uv) {
            float gu, gv;
            pair_grads<FMT, C>(t, bk, wb, a, bb, p, go, grad_uv != nullptr, gsx, gsy, gu, gv);
            if (grad_uv) nt_store2(grad_uv + 2 * f, gu, gv);
        }
        if (keys) {
#pragma unroll
            for (int k = 0; k < 4; k++) keys[4 * f + k] = ((uint32_t)bk[k] << cell_bits) | cell;
            ((float4*)wrec)[f] = make_float4(p.fx, p.fy, a, bb);
        }
    }

    if (grad_view) {
        // dL/dB = (n/2) dL/ds on unclamped axes
        float gbx = d.clx ? 0.f : gsx * (0.5f * (float)n);
        float gby = d.cly ? 0.f : gsy * (0.5f * (float)n);
        float gax, gay;
        square_vjp(d.ax, d.ay, gbx, gby, gax, gay);
        // A = (u_x, u_y) k, k = (L (L + u_z))^(-1/2):
        // dk/du = -k^3/2 * [(u / L)(2L + u_z) + L e_z]
        float gux = 0.f, guy = 0.f, guz = 0.f;
        if (d.k > 0.f && d.L > 0.f) {
            float sdot = d.ux * gax + d.uy * gay;
            float coef = -0.5f * d.k * d.k * d.k * sdot;
            float t2 = (2.f * d.L + d.uz) / d.L;
            gux = d.k * gax + coef * d.ux * t2;
            guy = d.k * gay + coef * d.uy * t2;
            guz = coef * (d.uz * t2 + d.L);
        }
        // dL/dV = M^T dL/du
        __builtin_nontemporal_store(g.m[0] * gux + g.m[3] * guy + g.m[6] * guz, grad_view + f * 3 + 0);
        __builtin_nontemporal_store(g.m[1] * gux + g.m[4] * guy + g.m[7] * guz, grad_view + f * 3 + 1);
        __builtin_nontemporal_store(g.m[2] * gux + g.m[5] * guy + g.m[8] * guz, grad_view + f * 3 + 2);
    }
}

// Level-of-detail backward, per fragment (the lookup blends levels l0 and
// l0 + 1 with weights 1 - t and t; the level of detail is not
// differentiated).  The mapping is formed once; each of the fragment's two
// units u = 2f + s (level l0 + s) gets the upstream gradient times its weight,
// its records in the chain's bucket numbering (start[l] + the level's bucket)
// and the level's view and uv gradients, computed as in k_bwd_fragment and
// summed over the units in level order.  A unit without weight or past the
// last level makes no records (sentinel keys).  Units on a level whose
// gradient is not wanted still make theirs (only the stores are skipped), so
// the sorted positions, and with them the summation order of every written
// level, do not depend on which levels are asked for.
struct LevelStarts {
    int64_t v[MAX_LEVELS + 1];
};

template <int FMT, int C, int MODE>
__global__ __launch_bounds__(256) void k_lod_bwd_fragment(
    LevelSet ls, const float* __restrict__ uv, const float* __restrict__ tbn,
    const float* __restrict__ view, const float* __restrict__ duv,
    const float* __restrict__ grad_out, LevelStarts start,
    float* __restrict__ grad_view, float* __restrict__ grad_uv, uint32_t* __restrict__ keys,
    float* __restrict__ wrec, float* __restrict__ gl, FragMap m, int cell_bits,
    uint32_t sentinel) {
    const int64_t f = frag_of(m, blockIdx.x, gridDim.x, threadIdx.x);
    if (f < 0) return;
    const int n = ls.n;
    float g[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < C; c++) g[c] = grad_out[f * C + c];
    int l0;
    float tt;
    lod_split(((const float4*)duv)[f], ls.W, ls.H, ls.levels, l0, tt);
    const Frag fr = load_frag(uv, tbn, view, f);
    const Dir d = map_direction(fr.m, fr.w, n);
    const Foot p = footprint(d.sx, d.sy, n);
    const uint32_t cell = (uint32_t)(p.y0 * n + p.x0);
    float vx = 0.f, vy = 0.f, vz = 0.f, su = 0.f, sv = 0.f;
    for (int sl = 0; sl < 2; sl++) {
        const int l = l0 + sl;
        const int64_t u = 2 * f + sl;
        const float w = sl == 0 ? 1.f - tt : tt;
        float go[4] = {0.f, 0.f, 0.f, 0.f};
        bool zero = true;
#pragma unroll
        for (int c = 0; c < C; c++) {
            go[c] = w * g[c];
            zero = zero && go[c] == 0.f;
        }
        const bool live = l < ls.levels && !zero;
        const bool rec = live && keys != nullptr;
        if (!rec && keys) {
            if constexpr (MODE == MODE_NEAREST) keys[u] = sentinel;
            else ((uint4*)keys)[u] = make_uint4(sentinel, sentinel, sentinel, sentinel);
        }
        if (!live) continue;
        TexView t{};
        t.data = ls.data[0];
        t.scales = ls.scales[0];
#pragma unroll
        for (int k = 1; k < MAX_LEVELS; k++) {
            if (l == k) {
                t.data = ls.data[k];
                t.scales = ls.scales[k];
            }
        }
        t.W = max(ls.W >> l, 1);
        t.H = max(ls.H >> l, 1);
        t.n = n;
        t.C = C;
        if (rec) {
#pragma unroll
            for (int c = 0; c < C; c++) gl[u * C + c] = go[c];
        }
        const int64_t b0 = start.v[0];
        int64_t off = b0;
#pragma unroll
        for (int k = 1; k < MAX_LEVELS; k++)
            if (l == k) off = start.v[k];
        float gsx = 0.f, gsy = 0.f;
        if constexpr (MODE == MODE_NEAREST) {
            const int i = bucket_of(fr.u, t.W), j = bucket_of(fr.v, t.H);
            const int64_t b = (int64_t)j * t.W + i;
            float lv;
            if (grad_view) bucket_grads<FMT, C>(t, b, p, go, gsx, gsy, lv);
            if (rec) {
                keys[u] = ((uint32_t)(off + b) << cell_bits) | cell;
                ((float2*)wrec)[u] = make_float2(p.fx, p.fy);
            }
        } else {
            int i0, i1, j0, j1;
            float a, bb;
            bucket_pair(fr.u, t.W, i0, i1, a);
            bucket_pair(fr.v, t.H, j0, j1, bb);
            const int64_t bk[4] = {(int64_t)j0 * t.W + i0, (int64_t)j0 * t.W + i1,
                                   (int64_t)j1 * t.W + i0, (int64_t)j1 * t.W + i1};
            const float wb[4] = {(1.f - a) * (1.f - bb), a * (1.f - bb), (1.f - a) * bb, a * bb};
            if (grad_view || grad_uv) {
                float gu, gv;
                pair_grads<FMT, C>(t, bk, wb, a, bb, p, go, grad_uv != nullptr, gsx, gsy, gu, gv);
                su += gu;
                sv += gv;
            }
            if (rec) {
#pragma unroll
                for (int k = 0; k < 4; k++)
                    keys[4 * u + k] = ((uint32_t)(off + bk[k]) << cell_bits) | cell;
                ((float4*)wrec)[u] = make_float4(p.fx, p.fy, a, bb);
            }
        }
        if (grad_view) {
            // as in k_bwd_fragment: dL/dB = (n/2) dL/ds on unclamped axes
            float gbx = d.clx ? 0.f : gsx * (0.5f * (float)n);
            float gby = d.cly ? 0.f : gsy * (0.5f * (float)n);
            float gax, gay;
            square_vjp(d.ax, d.ay, gbx, gby, gax, gay);
            float gux = 0.f, guy = 0.f, guz = 0.f;
            if (d.k > 0.f && d.L > 0.f) {
                float sdot = d.ux * gax + d.uy * gay;
                float coef = -0.5f * d.k * d.k * d.k * sdot;
                float t2 = (2.f * d.L + d.uz) / d.L;
                gux = d.k * gax + coef * d.ux * t2;
                guy = d.k * gay + coef * d.uy * t2;
                guz = coef * (d.uz * t2 + d.L);
            }
            vx += fr.m[0] * gux + fr.m[3] * guy + fr.m[6] * guz;
            vy += fr.m[1] * gux + fr.m[4] * guy + fr.m[7] * guz;
            vz += fr.m[2] * gux + fr.m[5] * guy + fr.m[8] * guz;
        }
    }
    if (grad_view) {
        grad_view[f * 3 + 0] = vx;
        grad_view[f * 3 + 1] = vy;
        grad_view[f * 3 + 2] = vz;
    }
    if (grad_uv) ((float2*)grad_uv)[f] = make_float2(su, sv);
}

// ---------------------------------------------------------------------------
// 2. stable LSD radix sort of (key, record index), 8-bit digits
// ---------------------------------------------------------------------------

// Records made in key order already (fragments visited in the order of a
// visit plan): k_keys_in_order leaves 0 in the disorder word, every launch of
// the sort then returns at once, and the later passes read the keys where the
// per-fragment pass wrote them, each record's position being its number.  A
// stable sort of keys in order is the identity, so the results are the same
// bits either way.
__device__ __forceinline__ bool sort_skipped(const uint32_t* __restrict__ disorder) {
    return disorder != nullptr && __builtin_amdgcn_readfirstlane(*disorder) == 0u;
}

// Whether any key is smaller than the one before it, in two launches.  The
// first writes one flag per workgroup of 1024 keys (four per thread with one
// 16-byte load -- the key buffer is padded to 256 bytes -- and the keys
// around them), the second ORs the flags into *disorder (cleared before) with
// one atomic per 4096 flags.  On unsorted keys nearly every wave finds a
// descent, and atomics of every wave on one address would serialise.
//
// With `range` the first launch also writes the [start, end) of every bucket
// as k_bucket_ranges forms them, from each workgroup whose 1024 keys (and
// the key before them) are in order: when all are, the sort and
// k_bucket_ranges return at once and these are the ranges; when some are not,
// k_bucket_ranges writes both ends of every bucket the sorted keys hold (the
// same buckets these keys hold) after the sort, and buckets without keys keep
// the zeros filled in before.  Unsorted keys make nearly every record a
// boundary, so workgroups with a descent write nothing.
__global__ __launch_bounds__(256) void k_keys_in_order(const uint32_t* __restrict__ keys, int64_t R,
                                                       uint32_t* __restrict__ flags, int cell_bits,
                                                       int64_t nb, int2* __restrict__ range) {
    __shared__ uint32_t wave_down[4];
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    bool down = false;
    uint32_t k[6] = {0u, 0u, 0u, 0u, 0u, 0u};
    if (i0 < R) {
        const uint4 q = *(const uint4*)(keys + i0);
        k[0] = keys[i0 > 0 ? i0 - 1 : 0];
        k[1] = q.x;
        k[2] = q.y;
        k[3] = q.z;
        k[4] = q.w;
        k[5] = keys[i0 + 4 < R ? i0 + 4 : R - 1];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t i = i0 + u;
            if (i > 0 && i < R && k[u + 1] < k[u]) down = true;
        }
    }
    const uint64_t m = __ballot(down);
    if ((threadIdx.x & 63) == 0) wave_down[threadIdx.x >> 6] = m != 0ull ? 1u : 0u;
    __syncthreads();
    const uint32_t any = wave_down[0] | wave_down[1] | wave_down[2] | wave_down[3];
    if (threadIdx.x == 0) flags[blockIdx.x] = any;
    if (range && any == 0u && i0 < R) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t i = i0 + u;
            if (i >= R) break;
            const uint32_t bu = k[u + 1] >> cell_bits;
            if (bu >= nb) continue;  // records of a sparse plan without a bucket
            if (i == 0 || (k[u] >> cell_bits) != bu) range[bu].x = (int)i;
            if (i == R - 1 || (k[u + 2] >> cell_bits) != bu) range[bu].y = (int)(i + 1);
        }
    }
}

__global__ __launch_bounds__(256) void k_flags_any(const uint32_t* __restrict__ flags,
                                                   int64_t nflags,
                                                   uint32_t* __restrict__ disorder) {
    const int64_t f0 = (int64_t)blockIdx.x * 4096 + threadIdx.x;
    uint32_t any = 0u;
#pragma unroll
    for (int u = 0; u < 16; u++) {
        const int64_t f = f0 + 256 * u;
        if (f < nflags) any |= flags[f];
    }
    if (__syncthreads_or((int)any) && threadIdx.x == 0) atomicOr(disorder, 1u);
}

// Digit counts of one tile of SORT_TILE keys: hist[d * tiles + tile].  Tiles
// are renumbered so that each XCD takes a contiguous range: the counts of
// neighbouring tiles share cache lines of the digit-major table, and so the
// strided 4-byte stores of one XCD's tiles combine in its L2.
template <int D>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                             int64_t R, int shift,
                                                             uint32_t* __restrict__ hist,
                                                             int64_t tiles,
                                                             const uint32_t* __restrict__ skip) {
    constexpr int B = 1 << D;
    __shared__ uint32_t cnt[B];
    if (sort_skipped(skip)) return;
    const int t = threadIdx.x;
    for (int d = t; d < B; d += SORT_THREADS) cnt[d] = 0;
    __syncthreads();
    const int64_t tile = xcd_block_id(blockIdx.x, gridDim.x);
    const int64_t base = tile * SORT_TILE;
    uint32_t k[SORT_IPT];
#pragma unroll
    for (int r = 0; r < SORT_IPT; r++) {
        const int64_t i = base + r * SORT_THREADS + t;
        k[r] = i < R ? keys[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < SORT_IPT; r++) {
        const int64_t i = base + r * SORT_THREADS + t;
        if (i < R) atomicAdd(&cnt[(k[r] >> shift) & (B - 1)], 1u);
    }
    __syncthreads();
    for (int d = t; d < B; d += SORT_THREADS) hist[(int64_t)d * tiles + tile] = cnt[d];
}

// x from the lane `o` below in the wavefront, for a power of two o < 64;
// lanes under `o` receive 0 or some lane's x, which their callers mask.
// Offsets 1 and 2 take one or two DPP wavefront shifts (wave_shr:1) on the
// vector ALU instead of a trip through the LDS crossbar (ds_bpermute); the
// value is the same either way, so the segmented scans below add in the same
// order.  A lane without a source lane reads 0 (bound_ctrl), which lets the
// compiler fold the last shift into the addition that uses it
// (v_add_f32_dpp).
__device__ __forceinline__ int dpp_shr1(int x) {
    return __builtin_amdgcn_mov_dpp(x, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ int lanes_up(int x, int o) {
    if (o == 1) return dpp_shr1(x);
    if (o == 2) return dpp_shr1(dpp_shr1(x));
    return __shfl_up(x, o, 64);
}
__device__ __forceinline__ uint32_t lanes_up(uint32_t x, int o) {
    return (uint32_t)lanes_up((int)x, o);
}
__device__ __forceinline__ float lanes_up(float x, int o) {
    return __int_as_float(lanes_up(__float_as_int(x), o));
}
// x from the lane one above (lane 63 receives 0, which its callers mask): one
// DPP wavefront shift (wave_shl:1)
__device__ __forceinline__ int lane_above(int x) {
    return __builtin_amdgcn_mov_dpp(x, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t lane_above(uint32_t x) { return (uint32_t)lane_above((int)x); }

// exclusive prefix of v over the 256 threads of the block; *total receives the sum
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t* wsum, uint32_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        uint32_t s = wsum[k];
        if (k < w) before += s;
        all += s;
    }
    __syncthreads();
    if (total) *total = all;
    return before + x - v;
}

// device-wide exclusive scan: per-block sums, a one-block scan of the sums,
// then per-block scans offset by the scanned sums; up to SCAN_FUSED_BLOCKS
// blocks (every sort of up to 2^27 records) the per-block scans add up the sums
// before them themselves, one launch fewer.  Each thread owns 16
// consecutive counts, read (and written) as four 16-byte vectors when all 16
// lie inside the array and the pointers are 16-byte aligned.
__device__ __forceinline__ void load16(const uint32_t* __restrict__ in, int64_t base, int64_t L,
                                       bool vec, uint32_t v[16]) {
    if (vec && base + 16 <= L) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint4 q = ((const uint4*)(in + base))[k];
            v[4 * k] = q.x;
            v[4 * k + 1] = q.y;
            v[4 * k + 2] = q.z;
            v[4 * k + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++) v[k] = (base + k < L) ? in[base + k] : 0u;
    }
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t L,
                                                     uint32_t* __restrict__ part,
                                                     const uint32_t* __restrict__ skip) {
    __shared__ uint32_t wsum[4];
    if (sort_skipped(skip)) return;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * 16;
    const bool vec = ((uintptr_t)in & 15) == 0;
    uint32_t v[16], s = 0;
    load16(in, base, L, vec, v);
#pragma unroll
    for (int k = 0; k < 16; k++) s += v[k];
    uint32_t total;
    block_exclusive(s, wsum, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_scan_top(uint32_t* __restrict__ part, int64_t P,
                                                  const uint32_t* __restrict__ skip) {
    __shared__ uint32_t wsum[4];
    if (sort_skipped(skip)) return;
    uint32_t carry = 0;
    for (int64_t base = 0; base < P; base += 256 * 16) {
        const int64_t b = base + threadIdx.x * 16;
        uint32_t v[16], s = 0;
#pragma unroll
        for (int k = 0; k < 16; k++) {
            v[k] = (b + k < P) ? part[b + k] : 0u;
            s += v[k];
        }
        uint32_t total;
        uint32_t run = carry + block_exclusive(s, wsum, &total);
#pragma unroll
        for (int k = 0; k < 16; k++) {
            if (b + k < P) part[b + k] = run;
            run += v[k];
        }
        carry += total;
    }
}

// SCANNED: part holds the scanned block sums (k_scan_top ran); otherwise it
// holds the plain sums and the block adds up those of the blocks before it
// (at most SCAN_FUSED_BLOCKS of them, so at most 16 loads per thread).
template <bool SCANNED>
__global__ __launch_bounds__(256) void k_scan_down(const uint32_t* __restrict__ in, int64_t L,
                                                   const uint32_t* __restrict__ part,
                                                   uint32_t* __restrict__ out,
                                                   const uint32_t* __restrict__ skip) {
    __shared__ uint32_t wsum[4];
    if (sort_skipped(skip)) return;
    uint32_t offset;
    if constexpr (SCANNED) {
        offset = part[blockIdx.x];
    } else {
        uint32_t ps = 0;
        for (uint32_t j = threadIdx.x; j < blockIdx.x; j += 256) ps += part[j];
        block_exclusive(ps, wsum, &offset);
    }
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * 16;
    const bool vec = (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
    uint32_t v[16], s = 0;
    load16(in, base, L, vec, v);
#pragma unroll
    for (int k = 0; k < 16; k++) s += v[k];
    uint32_t run = offset + block_exclusive(s, wsum, nullptr);
    uint32_t o[16];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        o[k] = run;
        run += v[k];
    }
    if (vec && base + 16 <= L) {
#pragma unroll
        for (int k = 0; k < 4; k++)
            ((uint4*)(out + base))[k] = make_uint4(o[4 * k], o[4 * k + 1], o[4 * k + 2], o[4 * k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++)
            if (base + k < L) out[base + k] = o[k];
    }
}

// Stable scatter of one radix pass.  Wave w ranks the contiguous quarter
// [w SORT_TILE/4, (w+1) SORT_TILE/4) of the tile in 16 rounds of 64 records:
// lanes holding the same digit are found with one ballot per digit bit, a
// record's rank is the number of such lanes below it plus the wave's running
// count of that digit (kept in LDS by the digit's lowest lane).  The tile's
// order within a digit is therefore wave, round, lane: index order.  The tile
// is ordered in LDS, then written so that each digit's run is contiguous in
// memory.  Tiles are renumbered per XCD as in the histogram: a digit's runs
// from neighbouring tiles are adjacent in the output, so their partial-line
// stores meet in one L2.
template <int D>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, int64_t R, int shift,
    const uint32_t* __restrict__ hoff, int64_t tiles, const uint32_t* __restrict__ skip) {
    constexpr int B = 1 << D;
    constexpr int DPT = B / SORT_THREADS;  // digits per thread in the digit phase
    constexpr int QUARTER = SORT_TILE / 4;
    __shared__ uint32_t skeys[SORT_TILE];
    __shared__ uint32_t svals[SORT_TILE];
    __shared__ uint32_t wcnt[4][B];  // running counts, then exclusive prefixes over waves
    __shared__ uint32_t dstart[B], goff[B];
    __shared__ uint32_t wsum[4];
    if (sort_skipped(skip)) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t tile = xcd_block_id(blockIdx.x, gridDim.x);
    const int64_t base = tile * SORT_TILE;
    for (int d = t; d < B; d += SORT_THREADS) {
        wcnt[0][d] = wcnt[1][d] = wcnt[2][d] = wcnt[3][d] = 0;
        goff[d] = hoff[(int64_t)d * tiles + tile];
    }
    uint32_t k[SORT_IPT], v[SORT_IPT], loc[SORT_IPT];
    const int64_t wbase = base + w * QUARTER;
#pragma unroll
    for (int r = 0; r < SORT_IPT; r++) {
        const int64_t i = wbase + r * 64 + lane;
        k[r] = 0u;
        v[r] = 0u;
        if (i < R) {
            k[r] = keys_in[i];
            v[r] = vals_in ? vals_in[i] : (uint32_t)i;
        }
    }
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < SORT_IPT; r++) {
        const int64_t i = wbase + r * 64 + lane;
        const bool valid = i < R;
        const uint32_t dg = (k[r] >> shift) & (B - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < D; bit++) {
            const bool on = (dg >> bit) & 1u;
            const uint64_t m = __ballot(on);
            peers &= on ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        const uint32_t before = valid ? wcnt[w][dg] : 0u;
        loc[r] = before + rank;
        wave_lds_sync();
        if (valid && rank == 0) wcnt[w][dg] = before + (uint32_t)__popcll(peers);
        wave_lds_sync();
    }
    __syncthreads();
    // digits: prefixes over the waves, and the tile's exclusive scan over digits
    uint32_t tot[DPT], mine = 0;
#pragma unroll
    for (int j = 0; j < DPT; j++) {
        const int d = t * DPT + j;
        const uint32_t c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d], c3 = wcnt[3][d];
        wcnt[0][d] = 0;
        wcnt[1][d] = c0;
        wcnt[2][d] = c0 + c1;
        wcnt[3][d] = c0 + c1 + c2;
        tot[j] = c0 + c1 + c2 + c3;
        mine += tot[j];
    }
    uint32_t run = block_exclusive(mine, wsum, nullptr);
#pragma unroll
    for (int j = 0; j < DPT; j++) {
        dstart[t * DPT + j] = run;
        run += tot[j];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SORT_IPT; r++) {
        const int64_t i = wbase + r * 64 + lane;
        if (i < R) {
            const uint32_t dg = (k[r] >> shift) & (B - 1);
            const uint32_t pos = dstart[dg] + wcnt[w][dg] + loc[r];
            skeys[pos] = k[r];
            svals[pos] = v[r];
        }
    }
    __syncthreads();
    const int64_t nvalid = (R - base) < SORT_TILE ? (R - base) : SORT_TILE;
#pragma unroll
    for (int r = 0; r < SORT_IPT; r++) {
        const int p = r * SORT_THREADS + t;
        if (p < nvalid) {
            const uint32_t kk = skeys[p];
            const uint32_t dg = (kk >> shift) & (B - 1);
            const uint32_t dst = goff[dg] + ((uint32_t)p - dstart[dg]);
            keys_out[dst] = kk;
            vals_out[dst] = svals[p];
        }
    }
}

// ---------------------------------------------------------------------------
// 3. bucket ranges in the sorted records
// ---------------------------------------------------------------------------

// Grid-stride fill (the bucket ranges of 2^31 buckets are 2^32 words).
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Four sorted keys per thread (one 16-byte load; the key buffer is padded to
// 256 bytes, so the load of a partial last group stays inside it) and the
// two neighbours, loaded unconditionally from clamped positions.
__global__ __launch_bounds__(256) void k_bucket_ranges(const uint32_t* __restrict__ skeys,
                                                       int64_t R, int cell_bits, int64_t nb,
                                                       int2* __restrict__ range,
                                                       const uint32_t* __restrict__ disorder) {
    // records made in key order: the order check wrote the ranges
    if (sort_skipped(disorder)) return;
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (i0 >= R) return;
    const uint4 q = *(const uint4*)(skeys + i0);
    const uint32_t prev = skeys[i0 > 0 ? i0 - 1 : 0];
    const uint32_t next = skeys[i0 + 4 < R ? i0 + 4 : R - 1];
    const uint32_t b[6] = {prev >> cell_bits, q.x >> cell_bits, q.y >> cell_bits,
                           q.z >> cell_bits, q.w >> cell_bits, next >> cell_bits};
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int64_t i = i0 + u;
        if (i >= R) break;
        const uint32_t bu = b[u + 1];
        if (bu >= nb) continue;  // records of a sparse plan without a bucket (sorted last)
        if (i == 0 || b[u] != bu) range[bu].x = (int)i;
        if (i == R - 1 || b[u + 2] != bu) range[bu].y = (int)(i + 1);
    }
}

// One sorted record's payload (records of buckets with more than 64 records
// are skipped: their passes gather).
template <int C, int MODE>
__device__ __forceinline__ void payload_record(const uint32_t* __restrict__ skeys,
                                               const uint32_t* __restrict__ svals,
                                               const float* __restrict__ wrec,
                                               const float* __restrict__ grad_out,
                                               const int2* __restrict__ range, int64_t i,
                                               int cell_bits, int64_t nb,
                                               float* __restrict__ payf,
                                               float* __restrict__ payg) {
    const uint32_t b = skeys[i] >> cell_bits;
    if (b >= nb) return;
    const int2 r = range[b];
    if (r.y - r.x > 64) return;
    const uint32_t rec = svals[i];
    float fx, fy, wb = 1.f;
    int64_t frag;
    if constexpr (MODE == MODE_NEAREST) {
        frag = rec;
        const float2 w2 = ((const float2*)wrec)[frag];
        fx = w2.x;
        fy = w2.y;
    } else {
        frag = rec >> 2;
        const int k = rec & 3;
        const float4 w4 = ((const float4*)wrec)[frag];
        fx = w4.x;
        fy = w4.y;
        const float aa = w4.z, bb = w4.w;
        wb = (k == 0) ? (1.f - aa) * (1.f - bb)
                      : (k == 1) ? aa * (1.f - bb) : (k == 2) ? (1.f - aa) * bb : aa * bb;
    }
    ((float2*)payf)[i] = make_float2(fx, fy);
    if constexpr (C == 4) {
        const float4 g = ((const float4*)grad_out)[frag];
        ((float4*)payg)[i] = make_float4(g.x * wb, g.y * wb, g.z * wb, g.w * wb);
    } else if constexpr (C == 2) {
        const float2 g = ((const float2*)grad_out)[frag];
        ((float2*)payg)[i] = make_float2(g.x * wb, g.y * wb);
    } else {
#pragma unroll
        for (int c = 0; c < C; c++) payg[i * C + c] = grad_out[frag * C + c] * wb;
    }
}

// The payload of the sorted records of buckets with at most 64 records (the
// ones the first accumulation pass serves from its register window), in
// sorted order: the fractions (fx, fy) and the upstream gradient times the
// bucket weight (1 in nearest mode).  That pass then reads its records
// contiguously instead of gathering them from the fragments; the passes for
// bigger buckets, whose records share cache lines, keep gathering.  Records
// past the last bucket (sparse plans) are skipped.  Workgroups are renumbered
// per XCD (neighbouring records gather from neighbouring fragments); a
// workgroup takes PAYLOAD_PER_THREAD x 256 consecutive records, a thread every
// 256th of them with its loads issued together, which also keeps the launch
// small when the records came in key order and there is nothing to do.
template <int C, int MODE>
__global__ __launch_bounds__(256) void k_payload(const uint32_t* __restrict__ skeys,
                                                 const uint32_t* __restrict__ svals,
                                                 const float* __restrict__ wrec,
                                                 const float* __restrict__ grad_out,
                                                 const int2* __restrict__ range, int64_t R,
                                                 int cell_bits, int64_t nb,
                                                 float* __restrict__ payf,
                                                 float* __restrict__ payg,
                                                 const uint32_t* __restrict__ disorder) {
    // records in key order are read where they were made: no payload
    if (sort_skipped(disorder)) return;
    const int64_t base =
        (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * (256 * PAYLOAD_PER_THREAD) + threadIdx.x;
#pragma unroll
    for (int k = 0; k < PAYLOAD_PER_THREAD; k++) {
        const int64_t i = base + 256 * k;
        if (i < R)
            payload_record<C, MODE>(skeys, svals, wrec, grad_out, range, i, cell_bits, nb, payf,
                                    payg);
    }
}

// ---------------------------------------------------------------------------
// 4./5. segmented reduction of a bucket's records into its gradient tile
// ---------------------------------------------------------------------------

// Upstream gradient of sorted record i from the payload (bucket weight
// already applied).
template <int C>
__device__ __forceinline__ void load_payg(const float* __restrict__ payg, int64_t i, float g[C]) {
    if constexpr (C == 4) {
        const float4 q = ((const float4*)payg)[i];
        g[0] = q.x;
        g[1] = q.y;
        g[2] = q.z;
        g[3] = q.w;
    } else if constexpr (C == 2) {
        const float2 q = ((const float2*)payg)[i];
        g[0] = q.x;
        g[1] = q.y;
    } else {
#pragma unroll
        for (int c = 0; c < C; c++) g[c] = payg[i * C + c];
    }
}

// One round of up to 64 sorted records of one bucket, one record per lane
// (lanes without a record carry a cell no record has).  The four tap
// contributions are summed per cell by an inclusive segmented scan across
// lanes with a fixed shape.  `ends_here` tells whether a lane's cell ends in
// this round; a cell that ends adds its four sums to its four texels in four
// phases, so no two lanes touch one texel at once.
template <int C>
__device__ __forceinline__ void accumulate_tails(int cell, const float v[4 * C], bool tail, int n,
                                                 float* tile);

template <int C>
__device__ __forceinline__ void accumulate_round(int cell, float v[4 * C], bool valid,
                                                 bool next_same, int n, float* tile) {
    const int lane = threadIdx.x & 63;
    constexpr int F = 4 * C;
    // a run of equal cells is contiguous, so once no lane has a partner at
    // distance o every run is at most o long and the scan is complete
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int oc = lanes_up(cell, o);
        const bool same = lane >= o && oc == cell;
        if (__ballot(same) == 0ull) break;
#pragma unroll
        for (int q = 0; q < F; q++) {
            const float ov = lanes_up(v[q], o);
            if (same) v[q] += ov;
        }
    }
    const bool tail = valid && !next_same;
    accumulate_tails<C>(cell, v, tail, n, tile);
}

template <int C>
__device__ __forceinline__ void accumulate_tails(int cell, const float v[4 * C], bool tail, int n,
                                                 float* tile) {
    if (__ballot(tail) == 0ull) return;
    int y0 = 0, x0 = 0, x1 = 0, y1 = 0;
    if (tail) {
        y0 = cell / n;
        x0 = cell - y0 * n;
        x1 = min(x0 + 1, n - 1);
        y1 = min(y0 + 1, n - 1);
    }
    wave_lds_sync();
    if (tail) {
#pragma unroll
        for (int c = 0; c < C; c++) tile[(y0 * n + x0) * C + c] += v[0 * C + c];
    }
    wave_lds_sync();
    if (tail) {
#pragma unroll
        for (int c = 0; c < C; c++) tile[(y0 * n + x1) * C + c] += v[1 * C + c];
    }
    wave_lds_sync();
    if (tail) {
#pragma unroll
        for (int c = 0; c < C; c++) tile[(y1 * n + x0) * C + c] += v[2 * C + c];
    }
    wave_lds_sync();
    if (tail) {
#pragma unroll
        for (int c = 0; c < C; c++) tile[(y1 * n + x1) * C + c] += v[3 * C + c];
    }
    wave_lds_sync();
}

// A sorted record as loaded: its key, its bilinear fractions and its upstream
// gradient times the bucket weight (1 in nearest mode).
template <int C>
struct RawRec {
    uint32_t key;
    float fx, fy;
    float g[C];
};

template <int C, int MODE>
__device__ __forceinline__ void load_raw(const uint32_t* __restrict__ skeys,
                                         const uint32_t* __restrict__ svals,
                                         const float* __restrict__ wrec,
                                         const float* __restrict__ grad_out, int64_t i,
                                         RawRec<C>& r) {
    r.key = skeys[i];
    const uint32_t rec = svals ? svals[i] : (uint32_t)i;
    float wb = 1.f;
    int64_t frag;
    if constexpr (MODE == MODE_NEAREST) {
        frag = rec;
        const float2 w2 = ((const float2*)wrec)[frag];
        r.fx = w2.x;
        r.fy = w2.y;
    } else {
        frag = rec >> 2;
        const int k = rec & 3;
        const float4 w4 = ((const float4*)wrec)[frag];
        r.fx = w4.x;
        r.fy = w4.y;
        const float aa = w4.z, bb = w4.w;
        wb = (k == 0) ? (1.f - aa) * (1.f - bb)
                      : (k == 1) ? aa * (1.f - bb) : (k == 2) ? (1.f - aa) * bb : aa * bb;
    }
#pragma unroll
    for (int c = 0; c < C; c++) r.g[c] = grad_out[frag * C + c] * wb;
}

// The four tap contributions of a loaded record: v = (w00, w01, w10, w11) x g.
template <int C>
__device__ __forceinline__ void expand_raw(const RawRec<C>& r, float v[4 * C]) {
    const float w00 = (1.f - r.fx) * (1.f - r.fy), w01 = r.fx * (1.f - r.fy);
    const float w10 = (1.f - r.fx) * r.fy, w11 = r.fx * r.fy;
#pragma unroll
    for (int c = 0; c < C; c++) {
        const float gc = r.g[c];
        v[0 * C + c] = w00 * gc;
        v[1 * C + c] = w01 * gc;
        v[2 * C + c] = w10 * gc;
        v[3 * C + c] = w11 * gc;
    }
}

// Reduce sorted records [a, e) (all of one bucket) into the wave's LDS tile
// (zeroed by the caller), in rounds of 64 records.  A cell that runs past a
// round carries its partial sum into the next round's first lane.  Each
// round's records are loaded while the round before is summed.
template <int C, int MODE>
__device__ __forceinline__ void reduce_records(const uint32_t* __restrict__ skeys,
                                               const uint32_t* __restrict__ svals,
                                               const float* __restrict__ wrec,
                                               const float* __restrict__ grad_out, int64_t a,
                                               int64_t e, int n, uint32_t cell_mask,
                                               float* tile) {
    const int lane = threadIdx.x & 63;
    constexpr int F = 4 * C;
    float carry[F];
#pragma unroll
    for (int q = 0; q < F; q++) carry[q] = 0.f;
    int carry_cell = -1;
    RawRec<C> cur{}, nxt{};
    if (a + lane < e) load_raw<C, MODE>(skeys, svals, wrec, grad_out, a + lane, cur);
    for (int64_t base = a; base < e; base += 64) {
        const int64_t i = base + lane;
        const bool valid = i < e;
        if (i + 64 < e) load_raw<C, MODE>(skeys, svals, wrec, grad_out, i + 64, nxt);
        int cell = -2 - lane;  // distinct from every real cell and from each other
        float v[F];
#pragma unroll
        for (int q = 0; q < F; q++) v[q] = 0.f;
        if (valid) {
            cell = (int)(cur.key & cell_mask);
            expand_raw<C>(cur, v);
        }
        if (lane == 0 && cell == carry_cell) {
#pragma unroll
            for (int q = 0; q < F; q++) v[q] = carry[q] + v[q];
        }
        const int next_cell = lane_above(cell);
        bool next_same = valid && lane < 63 && i + 1 < e && next_cell == cell;
        bool spills = false;
        // record i + 1 of lane 63 is the next round's first
        const uint32_t key_after = __shfl(nxt.key, 0, 64);
        if (valid && lane == 63 && i + 1 < e) spills = (int)(key_after & cell_mask) == cell;
        // the scan runs before the carry is taken from lane 63
        accumulate_round<C>(cell, v, valid, next_same || spills, n, tile);
        if (__ballot(spills) != 0ull) {
#pragma unroll
            for (int q = 0; q < F; q++) carry[q] = __shfl(v[q], 63, 64);
            carry_cell = __shfl(cell, 63, 64);
        } else {
            carry_cell = -1;
        }
        cur = nxt;
    }
}

// A window of up to 64 consecutive sorted records held in registers, one per
// lane (cell, bilinear fractions and weighted upstream gradient), so that the
// small buckets of a group are served without further global loads.
template <int C>
struct RecWindow {
    int64_t start, end;  // records [start, end) are held; lane l holds start + l
    int cell;
    uint32_t key;
    float fx, fy;
    float g[C];
};

// payf == nullptr: the records are gathered from the fragments (svals, wrec,
// grad_out); otherwise they are read from the sorted payload (payf, payg).
template <int C, int MODE>
__device__ __forceinline__ void load_window(const uint32_t* __restrict__ skeys,
                                            const uint32_t* __restrict__ svals,
                                            const float* __restrict__ wrec,
                                            const float* __restrict__ grad_out,
                                            const float* __restrict__ payf,
                                            const float* __restrict__ payg, int64_t start,
                                            int64_t R, uint32_t cell_mask, RecWindow<C>& w) {
    const int lane = threadIdx.x & 63;
    w.start = start;
    w.end = (start + 64 < R) ? start + 64 : R;
    w.cell = -2 - lane;
    w.key = 0u;
    w.fx = w.fy = 0.f;
#pragma unroll
    for (int c = 0; c < C; c++) w.g[c] = 0.f;
    const int64_t i = start + lane;
    if (i < w.end) {
        w.key = skeys[i];
        w.cell = (int)(w.key & cell_mask);
        if (payf) {
            const float2 f2 = ((const float2*)payf)[i];
            w.fx = f2.x;
            w.fy = f2.y;
            load_payg<C>(payg, i, w.g);
        } else {
            const uint32_t rec = svals ? svals[i] : (uint32_t)i;
            float wb = 1.f;
            int64_t frag;
            if constexpr (MODE == MODE_NEAREST) {
                frag = rec;
                const float2 w2 = ((const float2*)wrec)[frag];
                w.fx = w2.x;
                w.fy = w2.y;
            } else {
                frag = rec >> 2;
                const int k = rec & 3;
                const float4 w4 = ((const float4*)wrec)[frag];
                w.fx = w4.x;
                w.fy = w4.y;
                const float aa = w4.z, bb = w4.w;
                wb = (k == 0) ? (1.f - aa) * (1.f - bb)
                              : (k == 1) ? aa * (1.f - bb) : (k == 2) ? (1.f - aa) * bb : aa * bb;
            }
#pragma unroll
            for (int c = 0; c < C; c++) w.g[c] = grad_out[frag * C + c] * wb;
        }
    }
}

// Segmented sums over the whole window, segments being runs of one sort key
// (bucket and cell): each run's last lane ends with its run's sum, formed by
// the same lanes and additions as a per-bucket scan would form it.
template <int C>
__device__ __forceinline__ void scan_window(const RecWindow<C>& w, float v[4 * C], bool& tail) {
    const int lane = threadIdx.x & 63;
    const int64_t i = w.start + lane;
    const bool valid = i < w.end;
    const float w00 = (1.f - w.fx) * (1.f - w.fy), w01 = w.fx * (1.f - w.fy);
    const float w10 = (1.f - w.fx) * w.fy, w11 = w.fx * w.fy;
#pragma unroll
    for (int c = 0; c < C; c++) {
        const float gc = valid ? w.g[c] : 0.f;
        v[0 * C + c] = w00 * gc;
        v[1 * C + c] = w01 * gc;
        v[2 * C + c] = w10 * gc;
        v[3 * C + c] = w11 * gc;
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t ok = lanes_up(w.key, o);
        const bool same = valid && lane >= o && ok == w.key;
        if (__ballot(same) == 0ull) break;
#pragma unroll
        for (int q = 0; q < 4 * C; q++) {
            const float ov = lanes_up(v[q], o);
            if (same) v[q] += ov;
        }
    }
    const uint32_t nk = lane_above(w.key);
    tail = valid && (lane == 63 || i + 1 >= w.end || nk != w.key);
}

__device__ __forceinline__ void tile_zero(float* tile, int te) {
    const int lane = threadIdx.x & 63;
    if ((te & 3) == 0) {
        const f4v z = {0.f, 0.f, 0.f, 0.f};
        for (int q = lane; q < te / 4; q += 64) ((f4v*)tile)[q] = z;
    } else {
        for (int q = lane; q < te; q += 64) tile[q] = 0.f;
    }
    wave_lds_sync();
}

// The dense gradient is written once and not read back by this library, so
// its stores are non-temporal (streamed past the caches).
__device__ __forceinline__ void tile_store(const float* tile, float* __restrict__ dst, int te) {
    const int lane = threadIdx.x & 63;
    wave_lds_sync();
    if ((te & 255) == 0) {
        for (int q = lane; q < te / 4; q += 64)
            __builtin_nontemporal_store(((const f4v*)tile)[q], (f4v*)dst + q);
    } else {
        for (int q = lane; q < te; q += 64) __builtin_nontemporal_store(tile[q], dst + q);
    }
    wave_lds_sync();
}

// Destination of the tile of bucket b (wave-uniform), or nullptr when the
// bucket's level is not written.  The level index is wave-uniform, so the
// table is read from the kernel arguments with scalar loads, one level at a
// time (a single level for the plain backward: no loop at all).
__device__ __forceinline__ float* tile_dst(const TileOut& o, int64_t b, int te) {
    const int64_t bu = (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
    int l = 0;
#pragma unroll 1
    for (int k = 1; k < o.levels; k++)
        if (bu >= o.start[k]) l = k;
    l = __builtin_amdgcn_readfirstlane(l);
    float* g = o.grad[l];
    return g ? g + (bu - o.start[l]) * (int64_t)te : nullptr;
}

__device__ __forceinline__ void zero_store(float* __restrict__ dst, int te) {
    const int lane = threadIdx.x & 63;
    if ((te & 255) == 0) {
        const f4v z = {0.f, 0.f, 0.f, 0.f};
        for (int q = lane; q < te / 4; q += 64) __builtin_nontemporal_store(z, (f4v*)dst + q);
    } else {
        for (int q = lane; q < te; q += 64) __builtin_nontemporal_store(0.f, dst + q);
    }
}

// pass 1: each wavefront owns G consecutive buckets (their ranges come in one
// coalesced load) and writes their tiles one after the other, so the stores
// of untouched buckets are issued back to back; four wavefronts per
// workgroup.  G = SEG_GROUP (8), or 4 when the records are read from the
// sorted payload (shorter groups spread the buckets over more wavefronts once
// the window loads are cheap).  k_segacc writes the untouched buckets and those with at most 64
// records (served from one register window) and lists those with 65..PIECE
// records for k_segacc_big (rounds of 64 with a carry).  Splitting keeps the
// register footprint of the common case small.  The list is split over
// BIG_LISTS counters, one atomic per group, so that workloads where most
// buckets are big do not serialise on one address: runs of BIG_RUN groups
// take the lists in turn (group g appends to list (g / BIG_RUN) mod
// BIG_LISTS), which keeps neighbouring buckets on one XCD in k_segacc_big.
// The order inside a list does not matter, each bucket is reduced alone.
template <int C, int MODE, int G>
__global__ __launch_bounds__(256) void k_segacc(const uint32_t* __restrict__ skeys,
                                                const uint32_t* __restrict__ svals,
                                                const float* __restrict__ wrec,
                                                const float* __restrict__ grad_out,
                                                const float* __restrict__ payf,
                                                const float* __restrict__ payg,
                                                const int2* __restrict__ range,
                                                const TileOut out, int64_t nbuckets,
                                                int64_t R, int n, uint32_t cell_mask,
                                                uint32_t* __restrict__ big_count,
                                                uint32_t* __restrict__ big_list,
                                                int64_t big_cap,
                                                const uint32_t* __restrict__ keys_made,
                                                const uint32_t* __restrict__ disorder) {
    if (sort_skipped(disorder)) {
        skeys = keys_made;
        svals = nullptr;
        payf = nullptr;
    }
    extern __shared__ float lds[];
    const int te = n * n * C;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float* tile = lds + w * te;
    const int64_t ngroups = (nbuckets + G - 1) / G;
    for (int64_t grp = (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * 4 + w; grp < ngroups;
         grp += (int64_t)gridDim.x * 4) {
        const int64_t b0 = grp * G;
        int2 rl = make_int2(0, 0);
        if (lane < G && b0 + lane < nbuckets) rl = range[b0 + lane];
        const int nb = (int)((nbuckets - b0) < G ? (nbuckets - b0) : G);
        // list the group's buckets with 65..PIECE records (more go to pass 2)
        const int cl = rl.y - rl.x;
        const bool big = cl > 64 && cl <= PIECE;
        const uint64_t bm = __ballot(big);
        // a bucket for pass 2: raise the flag that lets its kernels run
        if (__ballot(cl > PIECE) != 0ull && lane == 0) atomicOr(big_count + HOT_FLAG, 1u);
        if (bm != 0ull) {
            const int64_t list = (grp / BIG_RUN) % BIG_LISTS;
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(big_count + list * BIG_STRIDE, (uint32_t)__popcll(bm));
            base = __shfl(base, 0, 64);
            if (big) {
                const uint32_t below = (uint32_t)__popcll(bm & ((1ull << lane) - 1ull));
                big_list[list * big_cap + base + below] = (uint32_t)(b0 + lane);
            }
        }
        RecWindow<C> win;
        win.start = win.end = -1;
        float v[4 * C];
        bool tail = false;
        for (int k = 0; k < nb; k++) {
            // wave-uniform bucket range (scalar registers, scalar loop control)
            const int rx = __builtin_amdgcn_readfirstlane(__shfl(rl.x, k, 64));
            const int ry = __builtin_amdgcn_readfirstlane(__shfl(rl.y, k, 64));
            float* dst = tile_dst(out, b0 + k, te);
            const int cnt = ry - rx;
            if (cnt <= 0) {
                if (dst) zero_store(dst, te);
                continue;
            }
            if (cnt > 64 || !dst) continue;  // listed above, or hot; or not written
            if (!(rx >= win.start && ry <= win.end)) {
                load_window<C, MODE>(skeys, svals, wrec, grad_out, payf, payg, rx, R, cell_mask,
                                     win);
                scan_window<C>(win, v, tail);
            }
            tile_zero(tile, te);
            const int64_t i = win.start + lane;
            accumulate_tails<C>(win.cell, v, tail && i >= rx && i < ry, n, tile);
            tile_store(tile, dst, te);
        }
    }
}

// Buckets with 65..PIECE records, listed by k_segacc: workgroup x serves list
// x mod BIG_LISTS, one wavefront per listed bucket, rounds of 64 records with a
// carry.
template <int C, int MODE>
__global__ __launch_bounds__(256) void k_segacc_big(const uint32_t* __restrict__ skeys,
                                                    const uint32_t* __restrict__ svals,
                                                    const float* __restrict__ wrec,
                                                    const float* __restrict__ grad_out,
                                                    const int2* __restrict__ range,
                                                    const TileOut out, int n,
                                                    uint32_t cell_mask,
                                                    const uint32_t* __restrict__ big_count,
                                                    const uint32_t* __restrict__ big_list,
                                                    int64_t big_cap,
                                                    const uint32_t* __restrict__ keys_made,
                                                    const uint32_t* __restrict__ disorder) {
    if (sort_skipped(disorder)) {
        skeys = keys_made;
        svals = nullptr;
    }
    extern __shared__ float lds[];
    const int te = n * n * C;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float* tile = lds + w * te;
    const uint32_t list = blockIdx.x % BIG_LISTS;
    const uint32_t part = blockIdx.x / BIG_LISTS, parts = gridDim.x / BIG_LISTS;
    const uint32_t count = __builtin_amdgcn_readfirstlane(big_count[list * BIG_STRIDE]);
    const uint32_t* entries = big_list + list * big_cap;
    const uint32_t stride = parts * 4;
    // the next listed bucket and its range are read while this one is summed
    uint32_t e = part * 4 + w;
    uint32_t b_next = 0;
    int2 r_next = make_int2(0, 0);
    if (e < count) {
        b_next = __builtin_amdgcn_readfirstlane(entries[e]);
        r_next = range[b_next];
    }
    for (; e < count; e += stride) {
        const uint32_t b = b_next;
        const int rx = __builtin_amdgcn_readfirstlane(r_next.x);
        const int ry = __builtin_amdgcn_readfirstlane(r_next.y);
        if (e + stride < count) {
            b_next = __builtin_amdgcn_readfirstlane(entries[e + stride]);
            r_next = range[b_next];
        }
        float* dst = tile_dst(out, b, te);
        if (!dst) continue;
        tile_zero(tile, te);
        reduce_records<C, MODE>(skeys, svals, wrec, grad_out, rx, ry, n, cell_mask, tile);
        tile_store(tile, dst, te);
    }
}

// pass 2a: one wavefront per fixed chunk of PIECE sorted records; a hot bucket
// overlapping the chunk (only the chunk's first or last bucket can be hot)
// gets a partial tile, slot 0 for the first bucket and slot 1 for the last.
template <int C, int MODE>
__global__ __launch_bounds__(64) void k_segacc_hot(const uint32_t* __restrict__ skeys,
                                                   const uint32_t* __restrict__ svals,
                                                   const float* __restrict__ wrec,
                                                   const float* __restrict__ grad_out,
                                                   const int2* __restrict__ range,
                                                   float* __restrict__ part, int64_t R, int n,
                                                   int cell_bits, int64_t nb,
                                                   const uint32_t* __restrict__ keys_made,
                                                   const uint32_t* __restrict__ disorder,
                                                   const uint32_t* __restrict__ hot) {
    if (__builtin_amdgcn_readfirstlane(hot[0]) == 0u) return;  // no bucket for pass 2
    if (sort_skipped(disorder)) {
        skeys = keys_made;
        svals = nullptr;
    }
    extern __shared__ float lds[];
    const int te = n * n * C;
    const uint32_t cell_mask = (cell_bits >= 32) ? 0xFFFFFFFFu : ((1u << cell_bits) - 1u);
    const int64_t k = blockIdx.x;
    const int64_t c0 = k * PIECE;
    const int64_t c1 = (c0 + PIECE < R) ? c0 + PIECE : R;
    const uint32_t bf = skeys[c0] >> cell_bits;
    const uint32_t bl = skeys[c1 - 1] >> cell_bits;
    for (int slot = 0; slot < 2; slot++) {
        const uint32_t b = slot == 0 ? bf : bl;
        if (slot == 1 && bl == bf) break;
        if (b >= nb) break;  // the records past the last bucket (sparse plans)
        const int2 r = range[b];
        if ((int64_t)r.y - r.x <= PIECE) continue;
        const int64_t a = r.x > c0 ? r.x : c0;
        const int64_t e = r.y < c1 ? r.y : c1;
        tile_zero(lds, te);
        reduce_records<C, MODE>(skeys, svals, wrec, grad_out, a, e, n, cell_mask, lds);
        tile_store(lds, part + (k * 2 + slot) * (int64_t)te, te);
        wave_lds_sync();
    }
}

// pass 2b: the chunk in which a hot bucket starts sums its partial tiles in
// chunk order and writes the bucket's tile.
__global__ __launch_bounds__(64) void k_combine_hot(const uint32_t* __restrict__ skeys,
                                                    const int2* __restrict__ range,
                                                    const float* __restrict__ part,
                                                    const TileOut out, int64_t R,
                                                    int te, int cell_bits, int64_t nb,
                                                    const uint32_t* __restrict__ keys_made,
                                                    const uint32_t* __restrict__ disorder,
                                                    const uint32_t* __restrict__ hot) {
    if (__builtin_amdgcn_readfirstlane(hot[0]) == 0u) return;  // no bucket for pass 2
    if (sort_skipped(disorder)) skeys = keys_made;
    const int lane = threadIdx.x;
    const int64_t k = blockIdx.x;
    const int64_t c0 = k * PIECE;
    const int64_t c1 = (c0 + PIECE < R) ? c0 + PIECE : R;
    const uint32_t bf = skeys[c0] >> cell_bits;
    const uint32_t bl = skeys[c1 - 1] >> cell_bits;
    for (int slot = 0; slot < 2; slot++) {
        const uint32_t b = slot == 0 ? bf : bl;
        if (slot == 1 && bl == bf) break;
        if (b >= nb) break;  // the records past the last bucket (sparse plans)
        const int2 r = range[b];
        if ((int64_t)r.y - r.x <= PIECE) continue;
        if ((int64_t)r.x / PIECE != k) continue;  // combined by the chunk it starts in
        const int64_t k0 = (int64_t)r.x / PIECE, k1 = ((int64_t)r.y - 1) / PIECE;
        float* dst = tile_dst(out, b, te);
        if (!dst) continue;
        for (int q0 = 0; q0 < te; q0 += 64 * 8) {
            float acc[8];
#pragma unroll
            for (int u = 0; u < 8; u++) acc[u] = 0.f;
            for (int64_t kc = k0; kc <= k1; kc++) {
                const int s = ((skeys[kc * PIECE] >> cell_bits) == b) ? 0 : 1;
                const float* src = part + (kc * 2 + s) * (int64_t)te;
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int q = q0 + u * 64 + lane;
                    if (q < te) acc[u] += src[q];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int q = q0 + u * 64 + lane;
                if (q < te) dst[q] = acc[u];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// planning and launch sequence
// ---------------------------------------------------------------------------

static int ceil_log2(uint64_t x) {
    int b = 0;
    while ((1ull << b) < x) b++;
    return b;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool plan_backward(int W, int H, int n, int C, int64_t N, int mode, BwdPlan* p, bool sparse) {
    // the accumulation holds four bucket tiles per workgroup in LDS (64 KiB)
    if ((int64_t)n * n * C > 4096) return false;
    const int64_t nb = (int64_t)W * H;
    // a sparse plan keeps the all-ones key free for records without a bucket
    const int bucket_bits = ceil_log2((uint64_t)nb + (sparse ? 1 : 0));
    const int cell_bits = ceil_log2((uint64_t)n * n);
    if (bucket_bits + cell_bits > 32) return false;
    const int64_t R = mode == MODE_NEAREST ? N : 4 * N;
    if (R >= (1ll << 31)) return false;
    p->records = R;
    p->key_bits = bucket_bits + cell_bits;
    p->cell_bits = cell_bits;
    p->buckets = nb;
    p->sentinel = !sparse ? 0u
                  : (p->key_bits >= 32 ? 0xFFFFFFFFu : (uint32_t)((1ull << p->key_bits) - 1));
    // as few passes as digits of at most 10 bits allow (9 bits beyond 4M
    // records, where the histograms, their scan and the scatter's LDS, which
    // grow as 2^D, cost more than a pass saves), the bits spread evenly
    const int kb = std::max(1, p->key_bits);
    const int maxd = R <= (1ll << 22) ? 10 : 9;
    p->passes = (kb + maxd - 1) / maxd;
    int at = 0, widest = 0;
    for (int q = 0; q < 4; q++) {
        const int bits = q < p->passes ? kb / p->passes + (q < kb % p->passes ? 1 : 0) : 0;
        p->digit_bits[q] = bits;
        p->digit_shift[q] = at;
        at += bits;
        widest = std::max(widest, bits);
    }
    p->bins = 1 << std::max(8, widest);
    p->tiles = (R + SORT_TILE - 1) / SORT_TILE;
    p->scan_len = (int64_t)p->bins * p->tiles;
    p->scan_blocks = (p->scan_len + SCAN_TILE - 1) / SCAN_TILE;
    p->chunks = (R + PIECE - 1) / PIECE;
    p->tile_elems = (int64_t)n * n * C;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += align256(bytes);
        return at;
    };
    // the sort's buffers and the disorder word first: a visit plan's
    // workspace is this prefix
    p->off_keys0 = take((size_t)R * 4);
    p->off_keys1 = take((size_t)R * 4);
    p->off_vals0 = take((size_t)R * 4);
    p->off_vals1 = take((size_t)R * 4);
    p->off_hist = take((size_t)p->scan_len * 4);
    p->off_hoff = take((size_t)p->scan_len * 4);
    p->off_scanp = take((size_t)(p->scan_blocks + 1) * 4);
    // the disorder word, then one order flag per 1024 records
    p->off_disorder = take((size_t)(ORDER_FLAGS_AT + (R + 1023) / 1024) * 4);
    p->sort_total = o;
    p->off_wrec = take((size_t)N * (mode == MODE_NEAREST ? 8 : 16));
    p->off_payf = take((size_t)R * 8);
    p->off_payg = take((size_t)R * 4 * C);
    // big-bucket lists: list l receives the runs r of BIG_RUN groups with
    // r mod BIG_LISTS = l, at most ceil(ngroups / (BIG_RUN BIG_LISTS)) runs of
    // BIG_RUN * SEG_GROUP buckets, and no list exceeds the R/65 buckets that
    // can hold more than 64 records
    const int64_t ngroups = (nb + SEG_GROUP - 1) / SEG_GROUP;
    const int64_t runs_per_list = (ngroups + BIG_RUN * BIG_LISTS - 1) / (BIG_RUN * BIG_LISTS);
    const int64_t per_list = runs_per_list * BIG_RUN * SEG_GROUP;
    p->big_cap = std::max<int64_t>(1, std::min<int64_t>(per_list, R / 65));
    p->off_range = take((size_t)BIG_LISTS * BIG_STRIDE * 4 + (size_t)nb * 8);
    p->off_biglist = take((size_t)BIG_LISTS * p->big_cap * 4);
    p->off_part = take((size_t)p->chunks * 2 * p->tile_elems * 4);
    p->total = o;
    return true;
}

template <int FMT, int MODE>
static void launch_bwd_fragment_c(const TexView& t, const float* uv, const float* tbn,
                                  const float* view, const float* go, float* gview, float* guv,
                                  uint32_t* keys, float* wrec, const FragMap& m, int cell_bits,
                                  uint32_t sentinel, hipStream_t s) {
    const uint32_t blocks = fragmap_blocks(m);
    switch (t.C) {
    case 1: hipLaunchKernelGGL((k_bwd_fragment<FMT, 1, MODE>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, view, go, gview, guv, keys, wrec, m, cell_bits, sentinel); break;
    case 2: hipLaunchKernelGGL((k_bwd_fragment<FMT, 2, MODE>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, view, go, gview, guv, keys, wrec, m, cell_bits, sentinel); break;
    case 3: hipLaunchKernelGGL((k_bwd_fragment<FMT, 3, MODE>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, view, go, gview, guv, keys, wrec, m, cell_bits, sentinel); break;
    default: hipLaunchKernelGGL((k_bwd_fragment<FMT, 4, MODE>), dim3(blocks), dim3(256), 0, s, t, uv, tbn, view, go, gview, guv, keys, wrec, m, cell_bits, sentinel); break;
    }
}

template <int MODE, int G>
static void launch_segacc_c(int C, dim3 grid, size_t shm, hipStream_t s, const uint32_t* sk,
                            const uint32_t* sv, const float* wrec, const float* go,
                            const float* pf, const float* pg,
                            const int2* range, const TileOut& gt, int64_t nb, int64_t R, int n,
                            uint32_t mask, uint32_t* bc, uint32_t* bl, int64_t cap,
                            const uint32_t* km, const uint32_t* dis) {
    switch (C) {
    case 1: hipLaunchKernelGGL((k_segacc<1, MODE, G>), grid, dim3(256), shm, s, sk, sv, wrec, go, pf, pg, range, gt, nb, R, n, mask, bc, bl, cap, km, dis); break;
    case 2: hipLaunchKernelGGL((k_segacc<2, MODE, G>), grid, dim3(256), shm, s, sk, sv, wrec, go, pf, pg, range, gt, nb, R, n, mask, bc, bl, cap, km, dis); break;
    case 3: hipLaunchKernelGGL((k_segacc<3, MODE, G>), grid, dim3(256), shm, s, sk, sv, wrec, go, pf, pg, range, gt, nb, R, n, mask, bc, bl, cap, km, dis); break;
    default: hipLaunchKernelGGL((k_segacc<4, MODE, G>), grid, dim3(256), shm, s, sk, sv, wrec, go, pf, pg, range, gt, nb, R, n, mask, bc, bl, cap, km, dis); break;
    }
}

template <int MODE>
static void launch_segacc_big_c(int C, dim3 grid, size_t shm, hipStream_t s, const uint32_t* sk,
                                const uint32_t* sv, const float* wrec, const float* go,
                                const int2* range, const TileOut& gt, int n, uint32_t mask,
                                const uint32_t* bc, const uint32_t* bl, int64_t cap,
                                const uint32_t* km, const uint32_t* dis) {
    switch (C) {
    case 1: hipLaunchKernelGGL((k_segacc_big<1, MODE>), grid, dim3(256), shm, s, sk, sv, wrec, go, range, gt, n, mask, bc, bl, cap, km, dis); break;
    case 2: hipLaunchKernelGGL((k_segacc_big<2, MODE>), grid, dim3(256), shm, s, sk, sv, wrec, go, range, gt, n, mask, bc, bl, cap, km, dis); break;
    case 3: hipLaunchKernelGGL((k_segacc_big<3, MODE>), grid, dim3(256), shm, s, sk, sv, wrec, go, range, gt, n, mask, bc, bl, cap, km, dis); break;
    default: hipLaunchKernelGGL((k_segacc_big<4, MODE>), grid, dim3(256), shm, s, sk, sv, wrec, go, range, gt, n, mask, bc, bl, cap, km, dis); break;
    }
}

template <int MODE>
static void launch_segacc_hot_c(int C, dim3 grid, size_t shm, hipStream_t s, const uint32_t* sk,
                                const uint32_t* sv, const float* wrec, const float* go,
                                const int2* range, float* part, int64_t R, int n, int cb,
                                int64_t nb, const uint32_t* km, const uint32_t* dis,
                                const uint32_t* hot) {
    switch (C) {
    case 1: hipLaunchKernelGGL((k_segacc_hot<1, MODE>), grid, dim3(64), shm, s, sk, sv, wrec, go, range, part, R, n, cb, nb, km, dis, hot); break;
    case 2: hipLaunchKernelGGL((k_segacc_hot<2, MODE>), grid, dim3(64), shm, s, sk, sv, wrec, go, range, part, R, n, cb, nb, km, dis, hot); break;
    case 3: hipLaunchKernelGGL((k_segacc_hot<3, MODE>), grid, dim3(64), shm, s, sk, sv, wrec, go, range, part, R, n, cb, nb, km, dis, hot); break;
    default: hipLaunchKernelGGL((k_segacc_hot<4, MODE>), grid, dim3(64), shm, s, sk, sv, wrec, go, range, part, R, n, cb, nb, km, dis, hot); break;
    }
}

template <int MODE>
static void launch_payload_c(int C, dim3 grid, hipStream_t s, const uint32_t* sk,
                             const uint32_t* sv, const float* wrec, const float* go,
                             const int2* range, int64_t R, int cb, int64_t nb, float* pf,
                             float* pg, const uint32_t* dis) {
    switch (C) {
    case 1: hipLaunchKernelGGL((k_payload<1, MODE>), grid, dim3(256), 0, s, sk, sv, wrec, go, range, R, cb, nb, pf, pg, dis); break;
    case 2: hipLaunchKernelGGL((k_payload<2, MODE>), grid, dim3(256), 0, s, sk, sv, wrec, go, range, R, cb, nb, pf, pg, dis); break;
    case 3: hipLaunchKernelGGL((k_payload<3, MODE>), grid, dim3(256), 0, s, sk, sv, wrec, go, range, R, cb, nb, pf, pg, dis); break;
    default: hipLaunchKernelGGL((k_payload<4, MODE>), grid, dim3(256), 0, s, sk, sv, wrec, go, range, R, cb, nb, pf, pg, dis); break;
    }
}

static void launch_fill(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return;
    prof_begin(K_FILL, s);
    const uint32_t blocks = (uint32_t)std::min<int64_t>((n + 255) / 256, int64_t(1) << 20);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, n, v);
    prof_end(K_FILL, s);
}

static void launch_scan(const uint32_t* in, uint32_t* out, uint32_t* part, int64_t L,
                        int64_t blocks, hipStream_t s, const uint32_t* skip = nullptr) {
    prof_begin(K_SCAN, s);
    hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)blocks), dim3(256), 0, s, in, L, part, skip);
    if (blocks <= SCAN_FUSED_BLOCKS) {
        hipLaunchKernelGGL(k_scan_down<false>, dim3((uint32_t)blocks), dim3(256), 0, s, in, L,
                           part, out, skip);
    } else {
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, part, blocks, skip);
        hipLaunchKernelGGL(k_scan_down<true>, dim3((uint32_t)blocks), dim3(256), 0, s, in, L,
                           part, out, skip);
    }
    prof_end(K_SCAN, s);
}

hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, uint32_t* part, int64_t L,
                                 hipStream_t s) {
    if (L <= 0) return hipSuccess;
    launch_scan(in, out, part, L, (L + SCAN_TILE - 1) / SCAN_TILE, s);
    return hipGetLastError();
}

hipError_t launch_backward(const TexView& t, int fmt, int mode, const float* uv,
                           const float* tbn, const float* view, const float* grad_out,
                           float* grad_tex, float* grad_view, float* grad_uv,
                           const FragMap& frags, const BwdPlan& plan, void* ws, hipStream_t s) {
    const FragMap m = with_frame_staging(frags, t, fmt);
    const int64_t N = m.N;
    char* wsb = (char*)ws;
    uint32_t* keys0 = (uint32_t*)(wsb + plan.off_keys0);
    float* wrec = (float*)(wsb + plan.off_wrec);
    const bool want_tex = grad_tex != nullptr;

    // 1. per fragment
    if (N > 0 && (want_tex || grad_view || grad_uv)) {
        prof_begin(K_BWD_FRAGMENT, s);
        uint32_t* kp = want_tex ? keys0 : nullptr;
        if (mode == MODE_NEAREST) {
            if (fmt == FMT_F32) launch_bwd_fragment_c<FMT_F32, MODE_NEAREST>(t, uv, tbn, view, grad_out, grad_view, grad_uv, kp, wrec, m, plan.cell_bits, plan.sentinel, s);
            else if (fmt == FMT_BF16) launch_bwd_fragment_c<FMT_BF16, MODE_NEAREST>(t, uv, tbn, view, grad_out, grad_view, grad_uv, kp, wrec, m, plan.cell_bits, plan.sentinel, s);
            else launch_bwd_fragment_c<FMT_FP8, MODE_NEAREST>(t, uv, tbn, view, grad_out, grad_view, grad_uv, kp, wrec, m, plan.cell_bits, plan.sentinel, s);
        } else {
            if (fmt == FMT_F32) launch_bwd_fragment_c<FMT_F32, MODE_BILINEAR>(t, uv, tbn, view, grad_out, grad_view, grad_uv, kp, wrec, m, plan.cell_bits, plan.sentinel, s);
            else if (fmt == FMT_BF16) launch_bwd_fragment_c<FMT_BF16, MODE_BILINEAR>(t, uv, tbn, view, grad_out, grad_view, grad_uv, kp, wrec, m, plan.cell_bits, plan.sentinel, s);
            else launch_bwd_fragment_c<FMT_FP8, MODE_BILINEAR>(t, uv, tbn, view, grad_out, grad_view, grad_uv, kp, wrec, m, plan.cell_bits, plan.sentinel, s);
        }
        prof_end(K_BWD_FRAGMENT, s);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!want_tex) return hipSuccess;

    TileOut out{};
    out.levels = 1;
    out.start[0] = 0;
    out.start[1] = (int64_t)t.W * t.H;
    out.grad[0] = grad_tex;
    return launch_accumulate(t.n, t.C, mode, grad_out, out, plan, ws, s);
}

// The stable sort of the R records' keys in keys0 (record numbers implied by
// position).  The sorted keys and their record numbers end in *skeys, *svals.
// disorder: NULL, or the device word k_keys_in_order wrote: when it holds 0
// every launch returns at once (the keys are already in order).
void launch_sort_records(const BwdPlan& plan, void* ws, const uint32_t* disorder, hipStream_t s,
                         const uint32_t** skeys_out, const uint32_t** svals_out) {
    char* wsb = (char*)ws;
    uint32_t* keys0 = (uint32_t*)(wsb + plan.off_keys0);
    uint32_t* keys1 = (uint32_t*)(wsb + plan.off_keys1);
    uint32_t* vals0 = (uint32_t*)(wsb + plan.off_vals0);
    uint32_t* vals1 = (uint32_t*)(wsb + plan.off_vals1);
    uint32_t* hist = (uint32_t*)(wsb + plan.off_hist);
    uint32_t* hoff = (uint32_t*)(wsb + plan.off_hoff);
    uint32_t* scanp = (uint32_t*)(wsb + plan.off_scanp);
    const int64_t R = plan.records;
    const uint32_t* kin = keys0;
    const uint32_t* vin = nullptr;
    for (int pass = 0; pass < plan.passes; pass++) {
        uint32_t* kout = (pass & 1) ? keys0 : keys1;
        uint32_t* vout = (pass & 1) ? vals0 : vals1;
        const int shift = plan.digit_shift[pass];
        const int D = std::max(8, plan.digit_bits[pass]);
        const int64_t len = ((int64_t)1 << D) * plan.tiles;
        const dim3 grid((uint32_t)plan.tiles), block(SORT_THREADS);
        prof_begin(K_RADIX_HIST, s);
        if (D == 8) hipLaunchKernelGGL(k_radix_hist<8>, grid, block, 0, s, kin, R, shift, hist, plan.tiles, disorder);
        else if (D == 9) hipLaunchKernelGGL(k_radix_hist<9>, grid, block, 0, s, kin, R, shift, hist, plan.tiles, disorder);
        else hipLaunchKernelGGL(k_radix_hist<10>, grid, block, 0, s, kin, R, shift, hist, plan.tiles, disorder);
        prof_end(K_RADIX_HIST, s);
        launch_scan(hist, hoff, scanp, len, (len + SCAN_TILE - 1) / SCAN_TILE, s, disorder);
        prof_begin(K_RADIX_SCATTER, s);
        if (D == 8) hipLaunchKernelGGL(k_radix_scatter<8>, grid, block, 0, s, kin, vin, kout, vout, R, shift, hoff, plan.tiles, disorder);
        else if (D == 9) hipLaunchKernelGGL(k_radix_scatter<9>, grid, block, 0, s, kin, vin, kout, vout, R, shift, hoff, plan.tiles, disorder);
        else hipLaunchKernelGGL(k_radix_scatter<10>, grid, block, 0, s, kin, vin, kout, vout, R, shift, hoff, plan.tiles, disorder);
        prof_end(K_RADIX_SCATTER, s);
        kin = kout;
        vin = vout;
    }
    *skeys_out = kin;
    *svals_out = vin;
}

// Whether the R keys in keys0 are in order: the workspace's disorder word
// is cleared, then set by any descent.  With `range` (zero-filled before) the
// check also writes the bucket ranges the keys give if they are in order.
static uint32_t* launch_order_check(const BwdPlan& plan, void* ws, int2* range, hipStream_t s) {
    char* wsb = (char*)ws;
    const uint32_t* keys0 = (const uint32_t*)(wsb + plan.off_keys0);
    uint32_t* disorder = (uint32_t*)(wsb + plan.off_disorder);
    const int64_t R = plan.records;
    uint32_t* flags = disorder + ORDER_FLAGS_AT;
    launch_fill(disorder, 1, 0u, s);
    if (R > 0) {
        const int64_t nflags = (R + 1023) / 1024;
        prof_begin(K_ORDER_CHECK, s);
        hipLaunchKernelGGL(k_keys_in_order, dim3((uint32_t)nflags), dim3(256), 0, s, keys0, R,
                           flags, plan.cell_bits, plan.buckets, range);
        hipLaunchKernelGGL(k_flags_any, dim3((uint32_t)((nflags + 4095) / 4096)), dim3(256), 0, s,
                           flags, nflags, disorder);
        prof_end(K_ORDER_CHECK, s);
    }
    return disorder;
}

hipError_t launch_accumulate(int n, int C, int mode, const float* grad_out, const TileOut& out,
                             const BwdPlan& plan, void* ws, hipStream_t s) {
    char* wsb = (char*)ws;
    uint32_t* keys0 = (uint32_t*)(wsb + plan.off_keys0);
    float* wrec = (float*)(wsb + plan.off_wrec);
    float* payf = (float*)(wsb + plan.off_payf);
    float* payg = (float*)(wsb + plan.off_payg);
    uint32_t* big_count = (uint32_t*)(wsb + plan.off_range);  // BIG_LISTS counters
    int2* range = (int2*)(big_count + BIG_LISTS * BIG_STRIDE);
    uint32_t* big_list = (uint32_t*)(wsb + plan.off_biglist);
    float* part = (float*)(wsb + plan.off_part);
    const int64_t R = plan.records;

    // 2. sort, skipped on the device when the records were made in key order
    // (the order check then also writes the bucket ranges)
    const int64_t nb = plan.buckets;
    launch_fill(big_count, BIG_LISTS * BIG_STRIDE + nb * 2, 0u, s);  // counters and ranges
    const uint32_t* skeys = keys0;
    const uint32_t* svals = nullptr;
    const uint32_t* dis = nullptr;
    if (R > 0) {
        dis = launch_order_check(plan, ws, range, s);
        launch_sort_records(plan, ws, dis, s, &skeys, &svals);
    }

    // 3. ranges of sorted records (returns at once when the sort did)
    if (R > 0) {
        prof_begin(K_BUCKET_RANGES, s);
        hipLaunchKernelGGL(k_bucket_ranges, dim3((uint32_t)((R + 1023) / 1024)), dim3(256), 0, s,
                           skeys, R, plan.cell_bits, nb, range, dis);
        prof_end(K_BUCKET_RANGES, s);
    }

    // 4. the records' payload in sorted order (when buckets hold 64 records or
    // fewer on average: most records then go through the register window;
    // not written when the records came in order), then pass 1 over buckets
    const bool pay = R > 0 && R <= 64 * nb;
    if (pay) {
        const int64_t per_block = 256 * PAYLOAD_PER_THREAD;
        const dim3 gp((uint32_t)((R + per_block - 1) / per_block));
        prof_begin(K_PAYLOAD, s);
        if (mode == MODE_NEAREST) launch_payload_c<MODE_NEAREST>(C, gp, s, skeys, svals, wrec, grad_out, range, R, plan.cell_bits, nb, payf, payg, dis);
        else launch_payload_c<MODE_BILINEAR>(C, gp, s, skeys, svals, wrec, grad_out, range, R, plan.cell_bits, nb, payf, payg, dis);
        prof_end(K_PAYLOAD, s);
    }
    const int te = (int)plan.tile_elems;
    const uint32_t cell_mask = plan.cell_bits >= 32 ? 0xFFFFFFFFu : ((1u << plan.cell_bits) - 1u);
    // the big-bucket lists' capacity (planned for SEG_GROUP) also holds the
    // lists of groups of 4: ceil(2x) <= 2 ceil(x) runs of half the buckets
    const int G = pay ? 4 : SEG_GROUP;
    const int64_t groups = (nb + G - 1) / G;
    // the workgroups stride over the groups, so at most 2^20 of them keep the
    // launch within one dispatch (2^28 buckets and more at small n)
    const dim3 g1((uint32_t)std::min<int64_t>((groups + 3) / 4, int64_t(1) << 20));
    const float* pf = pay ? payf : nullptr;
    prof_begin(K_SEGACC, s);
    if (mode == MODE_NEAREST) {
        if (pay) launch_segacc_c<MODE_NEAREST, 4>(C, g1, (size_t)4 * te * 4, s, skeys, svals, wrec, grad_out, pf, payg, range, out, nb, R, n, cell_mask, big_count, big_list, plan.big_cap, keys0, dis);
        else launch_segacc_c<MODE_NEAREST, SEG_GROUP>(C, g1, (size_t)4 * te * 4, s, skeys, svals, wrec, grad_out, pf, payg, range, out, nb, R, n, cell_mask, big_count, big_list, plan.big_cap, keys0, dis);
    } else {
        if (pay) launch_segacc_c<MODE_BILINEAR, 4>(C, g1, (size_t)4 * te * 4, s, skeys, svals, wrec, grad_out, pf, payg, range, out, nb, R, n, cell_mask, big_count, big_list, plan.big_cap, keys0, dis);
        else launch_segacc_c<MODE_BILINEAR, SEG_GROUP>(C, g1, (size_t)4 * te * 4, s, skeys, svals, wrec, grad_out, pf, payg, range, out, nb, R, n, cell_mask, big_count, big_list, plan.big_cap, keys0, dis);
    }
    prof_end(K_SEGACC, s);
    if (R > 64) {
        // BIG_LISTS x parts workgroups, four wavefronts each; parts grows with
        // the number of buckets that can be big
        const int64_t parts = std::min<int64_t>(std::max<int64_t>(
            1, (R / 65 + 4 * BIG_LISTS - 1) / (4 * BIG_LISTS)), 64);
        const dim3 g2((uint32_t)(BIG_LISTS * parts));
        prof_begin(K_SEGACC_BIG, s);
        if (mode == MODE_NEAREST)
            launch_segacc_big_c<MODE_NEAREST>(C, g2, (size_t)4 * te * 4, s, skeys, svals, wrec, grad_out, range, out, n, cell_mask, big_count, big_list, plan.big_cap, keys0, dis);
        else
            launch_segacc_big_c<MODE_BILINEAR>(C, g2, (size_t)4 * te * 4, s, skeys, svals, wrec, grad_out, range, out, n, cell_mask, big_count, big_list, plan.big_cap, keys0, dis);
        prof_end(K_SEGACC_BIG, s);
    }

    // 5. pass 2 for buckets with more than PIECE records
    if (R > PIECE) {
        const dim3 g2((uint32_t)plan.chunks);
        prof_begin(K_SEGACC_HOT, s);
        if (mode == MODE_NEAREST)
            launch_segacc_hot_c<MODE_NEAREST>(C, g2, (size_t)te * 4, s, skeys, svals, wrec, grad_out, range, part, R, n, plan.cell_bits, nb, keys0, dis, big_count + HOT_FLAG);
        else
            launch_segacc_hot_c<MODE_BILINEAR>(C, g2, (size_t)te * 4, s, skeys, svals, wrec, grad_out, range, part, R, n, plan.cell_bits, nb, keys0, dis, big_count + HOT_FLAG);
        prof_end(K_SEGACC_HOT, s);
        prof_begin(K_COMBINE_HOT, s);
        hipLaunchKernelGGL(k_combine_hot, g2, dim3(64), 0, s, skeys, range, part, out, R, te,
                           plan.cell_bits, nb, keys0, dis, big_count + HOT_FLAG);
        prof_end(K_COMBINE_HOT, s);
    }
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// visit plan
// ---------------------------------------------------------------------------

// The record key of each fragment as k_bwd_fragment makes it in the nearest
// mode (bucket << cell_bits | cell of its footprint); in the bilinear-bucket
// mode the key of its first bucket (i0, j0) with its cell.
template <int MODE>
__global__ __launch_bounds__(256) void k_plan_keys(int W, int H, int n,
                                                   const float* __restrict__ uv,
                                                   const float* __restrict__ tbn,
                                                   const float* __restrict__ view,
                                                   uint32_t* __restrict__ keys, FragMap m,
                                                   int cell_bits) {
    const int64_t f = frag_of(m, blockIdx.x, gridDim.x, threadIdx.x);
    if (f < 0) return;
    const Frag g = load_frag(uv, tbn, view, f);
    const Dir d = map_direction(g.m, g.w, n);
    const Foot p = footprint(d.sx, d.sy, n);
    int64_t b;
    if constexpr (MODE == MODE_NEAREST) {
        const int i = bucket_of(g.u, W), j = bucket_of(g.v, H);
        b = (int64_t)j * W + i;
    } else {
        int i0, i1, j0, j1;
        float a, bb;
        bucket_pair(g.u, W, i0, i1, a);
        bucket_pair(g.v, H, j0, j1, bb);
        b = (int64_t)j0 * W + i0;
    }
    keys[f] = ((uint32_t)b << cell_bits) | (uint32_t)(p.y0 * n + p.x0);
}

// Planned fragment k is the caller's fragment svals[k] (k itself when the
// keys came in order): its index and its 56-byte record are copied.
__global__ __launch_bounds__(256) void k_plan_gather(const uint32_t* __restrict__ svals,
                                                     int64_t N, const float* __restrict__ uv,
                                                     const float* __restrict__ tbn,
                                                     const float* __restrict__ view,
                                                     int32_t* __restrict__ order,
                                                     float* __restrict__ uv_out,
                                                     float* __restrict__ tbn_out,
                                                     float* __restrict__ view_out,
                                                     const uint32_t* __restrict__ disorder) {
    if (sort_skipped(disorder)) svals = nullptr;
    const int64_t k = (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (k >= N) return;
    const int64_t f = svals ? (int64_t)svals[k] : k;
    order[k] = (int32_t)f;
    ((float2*)uv_out)[k] = ((const float2*)uv)[f];
#pragma unroll
    for (int q = 0; q < 9; q++) tbn_out[k * 9 + q] = tbn[f * 9 + q];
#pragma unroll
    for (int q = 0; q < 3; q++) view_out[k * 3 + q] = view[f * 3 + q];
}

// Rows of a per-fragment array moved by a plan's order: gather (dst[k] =
// src[order[k]], into plan order) or scatter (dst[order[k]] = src[k], back to
// the caller's order).  Rows of `row` 4-byte words; 16-byte accesses when the
// row is a whole number of them and both arrays are 16-byte aligned.
template <bool VEC>
__global__ __launch_bounds__(256) void k_permute_rows(const int32_t* __restrict__ order,
                                                      int64_t N, int row,
                                                      const uint32_t* __restrict__ src,
                                                      uint32_t* __restrict__ dst, int scatter) {
    const int64_t k = (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (k >= N) return;
    const int64_t o = order[k];
    if (o < 0 || o >= N) return;  // not an index of the array: no row moves
    const int64_t from = scatter ? k : o, to = scatter ? o : k;
    if constexpr (VEC) {
        const int q = row / 4;
        const uint4* s4 = (const uint4*)src + from * q;
        uint4* d4 = (uint4*)dst + to * q;
        for (int i = 0; i < q; i++) d4[i] = s4[i];
    } else {
        for (int i = 0; i < row; i++) dst[to * row + i] = src[from * row + i];
    }
}

hipError_t launch_permute_rows(const int32_t* order, int64_t N, int row_words, const void* src,
                               void* dst, bool scatter, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const bool vec = row_words % 4 == 0 && ((uintptr_t)src % 16) == 0 && ((uintptr_t)dst % 16) == 0;
    const dim3 grid((uint32_t)((N + 255) / 256));
    prof_begin(K_PERMUTE, s);
    if (vec)
        hipLaunchKernelGGL(k_permute_rows<true>, grid, dim3(256), 0, s, order, N, row_words,
                           (const uint32_t*)src, (uint32_t*)dst, (int)scatter);
    else
        hipLaunchKernelGGL(k_permute_rows<false>, grid, dim3(256), 0, s, order, N, row_words,
                           (const uint32_t*)src, (uint32_t*)dst, (int)scatter);
    prof_end(K_PERMUTE, s);
    return hipGetLastError();
}

hipError_t launch_plan(const TexView& t, int mode, const float* uv, const float* tbn,
                       const float* view, const FragMap& m, const BwdPlan& plan, void* ws,
                       int32_t* order, float* uv_out, float* tbn_out, float* view_out,
                       hipStream_t s) {
    const int64_t N = m.N;
    if (N <= 0) return hipSuccess;
    uint32_t* keys0 = (uint32_t*)((char*)ws + plan.off_keys0);
    prof_begin(K_PLAN_KEYS, s);
    if (mode == MODE_NEAREST)
        hipLaunchKernelGGL(k_plan_keys<MODE_NEAREST>, dim3(fragmap_blocks(m)), dim3(256), 0, s,
                           t.W, t.H, t.n, uv, tbn, view, keys0, m, plan.cell_bits);
    else
        hipLaunchKernelGGL(k_plan_keys<MODE_BILINEAR>, dim3(fragmap_blocks(m)), dim3(256), 0, s,
                           t.W, t.H, t.n, uv, tbn, view, keys0, m, plan.cell_bits);
    prof_end(K_PLAN_KEYS, s);
    const uint32_t* dis = launch_order_check(plan, ws, nullptr, s);
    const uint32_t *skeys = nullptr, *svals = nullptr;
    launch_sort_records(plan, ws, dis, s, &skeys, &svals);
    prof_begin(K_PLAN_GATHER, s);
    hipLaunchKernelGGL(k_plan_gather, dim3((uint32_t)((N + 255) / 256)), dim3(256), 0, s, svals,
                       N, uv, tbn, view, order, uv_out, tbn_out, view_out, dis);
    prof_end(K_PLAN_GATHER, s);
    return hipGetLastError();
}

template <int FMT, int MODE>
static void launch_lod_frag_c(int C, dim3 grid, hipStream_t s, const LevelSet& ls,
                              const float* uv, const float* tbn, const float* view,
                              const float* duv, const float* go, const LevelStarts& st, float* gview, float* guv, uint32_t* keys,
                              float* wrec, float* gl, const FragMap& m, int cb, uint32_t sent) {
    switch (C) {
    case 1: hipLaunchKernelGGL((k_lod_bwd_fragment<FMT, 1, MODE>), grid, dim3(256), 0, s, ls, uv, tbn, view, duv, go, st, gview, guv, keys, wrec, gl, m, cb, sent); break;
    case 2: hipLaunchKernelGGL((k_lod_bwd_fragment<FMT, 2, MODE>), grid, dim3(256), 0, s, ls, uv, tbn, view, duv, go, st, gview, guv, keys, wrec, gl, m, cb, sent); break;
    case 3: hipLaunchKernelGGL((k_lod_bwd_fragment<FMT, 3, MODE>), grid, dim3(256), 0, s, ls, uv, tbn, view, duv, go, st, gview, guv, keys, wrec, gl, m, cb, sent); break;
    default: hipLaunchKernelGGL((k_lod_bwd_fragment<FMT, 4, MODE>), grid, dim3(256), 0, s, ls, uv, tbn, view, duv, go, st, gview, guv, keys, wrec, gl, m, cb, sent); break;
    }
}

hipError_t launch_lod_bwd_fragment(const LevelSet& ls, int fmt, int mode, const float* uv,
                                   const float* tbn, const float* view, const float* duv,
                                   const float* grad_out, const int64_t* start, float* grad_view, float* grad_uv,
                                   uint32_t* keys, float* wrec, float* gl, const FragMap& m,
                                   int cell_bits, uint32_t sentinel, hipStream_t s) {
    LevelStarts st{};
    for (int l = 0; l <= ls.levels && l <= MAX_LEVELS; l++) st.v[l] = start[l];
    const dim3 grid(fragmap_blocks(m));
    const int C = ls.C;
    prof_begin(K_LOD_BWD_FRAGMENT, s);
    if (mode == MODE_NEAREST) {
        if (fmt == FMT_F32) launch_lod_frag_c<FMT_F32, MODE_NEAREST>(C, grid, s, ls, uv, tbn, view, duv, grad_out, st, grad_view, grad_uv, keys, wrec, gl, m, cell_bits, sentinel);
        else if (fmt == FMT_BF16) launch_lod_frag_c<FMT_BF16, MODE_NEAREST>(C, grid, s, ls, uv, tbn, view, duv, grad_out, st, grad_view, grad_uv, keys, wrec, gl, m, cell_bits, sentinel);
        else launch_lod_frag_c<FMT_FP8, MODE_NEAREST>(C, grid, s, ls, uv, tbn, view, duv, grad_out, st, grad_view, grad_uv, keys, wrec, gl, m, cell_bits, sentinel);
    } else {
        if (fmt == FMT_F32) launch_lod_frag_c<FMT_F32, MODE_BILINEAR>(C, grid, s, ls, uv, tbn, view, duv, grad_out, st, grad_view, grad_uv, keys, wrec, gl, m, cell_bits, sentinel);
        else if (fmt == FMT_BF16) launch_lod_frag_c<FMT_BF16, MODE_BILINEAR>(C, grid, s, ls, uv, tbn, view, duv, grad_out, st, grad_view, grad_uv, keys, wrec, gl, m, cell_bits, sentinel);
        else launch_lod_frag_c<FMT_FP8, MODE_BILINEAR>(C, grid, s, ls, uv, tbn, view, duv, grad_out, st, grad_view, grad_uv, keys, wrec, gl, m, cell_bits, sentinel);
    }
    prof_end(K_LOD_BWD_FRAGMENT, s);
    return hipGetLastError();
}

}  // namespace rt
