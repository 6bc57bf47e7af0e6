// rt_lod_backward.hip -- backward of the level-of-detail lookup over a mip
// chain, and the adjoint of one chain step, for gfx950.
//
// The trilinear lookup blends the lookups on levels l0 and l0 + 1 with
// weights 1 - t and t (the level of detail comes from the UV screen
// derivatives and is not differentiated).  So the gradient of level l's
// texels is the plain backward on level l with each fragment's upstream
// gradient scaled by its weight on that level, and the view and uv gradients
// are the sums over the levels of the plain backward's.  All levels are done
// in one pass: the chain's buckets are numbered one level after the other,
// every fragment makes records on the (at most two) levels it blends, and one
// sort and one accumulation (the plain backward's) write every level's tiles.
// The view and uv gradients are summed over the fragment's levels in level
// order in registers, so the result is bitwise reproducible.
//
// Chain adjoint: level l+1's bucket is the mean of the 2 x 2 (or 2) buckets of
// level l it covers, so each of those receives the parent's gradient divided
// by their number (one workgroup per bucket of level l: no two threads write
// one element).
#include <algorithm>

#include "rt_device.hpp"
#include "rt_kernels.hpp"

namespace rt {

// Grid-stride zero fill: a level can hold 2^32 elements or more, more than one
// dispatch may have work-items.
__global__ __launch_bounds__(256) void k_fill_f32(float* __restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = 0.f;
}

static uint32_t blocks_of(int64_t n) { return (uint32_t)std::min<int64_t>((n + 255) / 256, 65536); }

hipError_t launch_lookup_lod_bwd(const LevelSet& ls, int fmt, int mode, const float* uv,
                                 const float* tbn, const float* view, const float* duv,
                                 const float* grad_out, float* const* grad_levels,
                                 float* grad_view, float* grad_uv, const FragMap& m,
                                 const BwdPlan& plan, const LodBwdLayout& lay, void* ws,
                                 hipStream_t s) {
    const int64_t N = m.N;
    const int64_t te = (int64_t)ls.n * ls.n * ls.C;
    TileOut out{};
    out.levels = ls.levels;
    uint32_t want = 0;
    int64_t at = 0;
    for (int l = 0; l < ls.levels; l++) {
        out.start[l] = at;
        out.grad[l] = grad_levels[l];
        if (grad_levels[l]) want |= 1u << l;
        at += (int64_t)std::max(ls.W >> l, 1) * std::max(ls.H >> l, 1);
    }
    out.start[ls.levels] = at;
    if (N <= 0) {
        // no fragment: every level's gradient is zero
        for (int l = 0; l < ls.levels; l++) {
            if (!grad_levels[l]) continue;
            const int64_t e = (out.start[l + 1] - out.start[l]) * te;
            hipLaunchKernelGGL(k_fill_f32, dim3(blocks_of(e)), dim3(256), 0, s, grad_levels[l], e);
        }
        return hipGetLastError();
    }
    char* base = (char*)ws;
    char* bws = base + lay.off_bwd;
    float* gl = (float*)(base + lay.off_gl);
    uint32_t* keys = want ? (uint32_t*)(bws + plan.off_keys0) : nullptr;
    float* wrec = (float*)(bws + plan.off_wrec);
    hipError_t e = launch_lod_bwd_fragment(ls, fmt, mode, uv, tbn, view, duv, grad_out,
                                           out.start, grad_view, grad_uv, keys, wrec, gl, m,
                                           plan.cell_bits, plan.sentinel, s);
    if (e != hipSuccess || !want) return e;
    return launch_accumulate(ls.n, ls.C, mode, gl, out, plan, bws, s);
}

// grad_src (level l, W x H buckets of E values) += adjoint of the chain step
// applied to grad_dst (level l+1).  One workgroup per bucket of level l, so
// the parent's position is worked out once per bucket; the bucket's E values
// and its parent's are streamed with 16-byte accesses when both buffers allow.
// Each element adds its parent's value times 1/2 or 1/4 (an exact product).
template <bool VEC>
__global__ __launch_bounds__(256) void k_mip_adjoint(const float* __restrict__ grad_dst,
                                                     float* __restrict__ grad_src, int W, int H,
                                                     int E) {
    const int64_t nb = (int64_t)W * H;
    const int fx = W > 1 ? 2 : 1, fy = H > 1 ? 2 : 1;
    const int W2 = W > 1 ? W / 2 : 1;
    const float s = 1.0f / (float)(fx * fy);
    // at most ADJ_GRID workgroups stride over the buckets (one dispatch)
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const int j = (int)(b / W), i = (int)(b - (int64_t)j * W);
        const int64_t parent = (int64_t)(j / fy) * W2 + i / fx;
        const float* __restrict__ src = grad_dst + parent * E;
        float* __restrict__ dst = grad_src + b * E;
        if constexpr (VEC) {
            const float4* s4 = (const float4*)src;
            float4* d4 = (float4*)dst;
            for (int q = threadIdx.x; q < E / 4; q += 256) {
                const float4 p = s4[q];
                float4 d = d4[q];
                d.x += p.x * s;
                d.y += p.y * s;
                d.z += p.z * s;
                d.w += p.w * s;
                d4[q] = d;
            }
        } else {
            for (int q = threadIdx.x; q < E; q += 256) dst[q] += src[q] * s;
        }
    }
}

hipError_t launch_mip_adjoint(const TexView& src, const float* grad_dst, float* grad_src,
                              hipStream_t s) {
    const int E = src.n * src.n * src.C;
    const int64_t nb = (int64_t)src.W * src.H;
    // one workgroup per bucket, at most 2^20 of them striding over the rest
    const uint32_t gx = (uint32_t)std::min<int64_t>(nb, int64_t(1) << 20);
    const bool vec = (E % 4) == 0 && ((uintptr_t)grad_dst % 16) == 0 &&
                     ((uintptr_t)grad_src % 16) == 0;
    prof_begin(K_MIP_ADJOINT, s);
    if (vec)
        hipLaunchKernelGGL(k_mip_adjoint<true>, dim3(gx), dim3(256), 0, s, grad_dst, grad_src,
                           src.W, src.H, E);
    else
        hipLaunchKernelGGL(k_mip_adjoint<false>, dim3(gx), dim3(256), 0, s, grad_dst,
                           grad_src, src.W, src.H, E);
    prof_end(K_MIP_ADJOINT, s);
    return hipGetLastError();
}

}  // namespace rt
