/*
 * radtex.h -- C ABI of the MI355X (gfx950) radiance-bucket lookup library
 * (libradtex.so).
 *
 * Method: "Radiance Textures for Rasterizing Ray-Traced Data" (Fober, 2023,
 * arXiv 2301.01719).  A radiance texture is a W x H matrix of "buckets"; each
 * bucket is an n x n discrete map of the hemisphere (Sec. 2).  A fragment's
 * texture coordinate (u, v) selects the bucket and its incidence (view)
 * vector, moved into the orthogonal texture space of the surface, selects the
 * position inside the bucket through the equisolid projection (Eq. 1b) and
 * the disc-to-square map (Eq. 3); the position is clamped half a sample away
 * from the bucket edge (the Note after Eq. 3) and a bilinear fetch is taken
 * from the bucket's samples.
 *
 * Conventions used by every entry point
 *   - All array pointers are DEVICE pointers (HIP global memory) that the
 *     caller allocates and owns.  The library never frees them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     work is enqueued asynchronously on it; no entry point synchronises the
 *     host with the device, except rt_profile_read.
 *   - Every entry point returns an rt_status and never throws or aborts.
 *     Arguments are validated on the host before anything is enqueued; on a
 *     non-OK status no output has been touched.  rt_last_error() returns a
 *     thread-local message describing the last non-OK status.  Faults of
 *     already-enqueued kernels surface at the caller's next synchronisation.
 *   - All GPU arithmetic is binary32.
 *
 * Layouts
 *   texture, bucket-major   [H][W][n][n][C]: bucket (column i, row j) holds
 *                           n rows y of n samples x of C channels, contiguous.
 *                           Bucket axes: x follows the tangent T (+u), y the
 *                           bitangent B (+v); row j = 0 is first in memory.
 *   texture, atlas          [H*n][W*n][C]: the paper's arrangement of buckets
 *                           "in place of the texture's pixels" (Sec. 2); it is
 *                           re-laid into bucket-major by rt_create_texture.
 *   fragments               uv [N][2], tbn [N][3][3] (rows T, B, N of the
 *                           world-to-tangent frame, row-major), view [N][3]
 *                           (from the surface toward the eye; need not be unit).
 *   outputs                 out / grad_out [N][C]; grad_view [N][3];
 *                           grad_uv [N][2]; grad_tex bucket-major float32.
 *
 * Alignment: texture data and grad_tex 16 bytes; scales 4; uv and grad_uv 8;
 * out and grad_out 16 (C = 4), 8 (C = 2) or 4 (C = 1, 3); tbn, view and
 * grad_view 4; workspace 256.
 */
#ifndef RADTEX_H
#define RADTEX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT_VERSION 201

typedef enum {
    RT_OK = 0,
    RT_ERR_INVALID_ARG = 1,        /* NULL / misaligned pointer, bad size or enum   */
    RT_ERR_UNSUPPORTED = 2,        /* valid request outside the supported range     */
    RT_ERR_OUT_OF_MEMORY = 3,      /* device allocation failed (atlas copy only)    */
    RT_ERR_WORKSPACE_TOO_SMALL = 4,
    RT_ERR_NO_DEVICE = 5,          /* no HIP device is visible                      */
    RT_ERR_HIP = 6                 /* a HIP runtime call or kernel launch failed    */
} rt_status;

typedef enum {
    RT_FMT_F32 = 0,       /* binary32 texels                                        */
    RT_FMT_BF16 = 1,      /* bfloat16 texels (round-to-nearest-even), no scale      */
    RT_FMT_FP8_E4M3 = 2,  /* OCP E4M3 ("FN": bias 7, max 448, no inf) texels, times */
                          /* one binary32 scale per bucket                          */
    RT_FMT_BIT1 = 3       /* one bit per sample, one channel, bucket-major only: the */
                          /* 1-bit texture of Sec. 5 (Shadowing).  Bucket b holds    */
                          /* ceil(n*n/32) uint32 words; sample k = y*n + x is bit    */
                          /* k % 32 of word k / 32; the bits past n*n are zero.  A  */
                          /* tap reads 0.0 or 1.0, so a bilinear fetch blends flags. */
} rt_format;

typedef enum {
    RT_LAYOUT_BUCKET_MAJOR = 0,
    RT_LAYOUT_ATLAS = 1
} rt_layout;

/* lookup flags */
enum {
    RT_BUCKET_NEAREST = 0,   /* one bucket per fragment: the paper's "single sample
                                per bucket" synthesis (Sec. 2)                    */
    RT_BUCKET_BILINEAR = 1,  /* the synthesised W x H output sampled bilinearly in
                                UV: four buckets around frac(u)W - 1/2, wrapping   */
    RT_FWD_STAGE_BUCKETS = 2 /* rt_lookup_fwd only, with RT_BUCKET_NEAREST: each
                                wavefront groups its fragments by bucket with
                                ballots and copies each bucket whole into LDS,
                                where the group reads its taps; the same results
                                bit for bit.  Plain F32 / BF16 / FP8 textures
                                whose bucket (n*n*C samples) is a multiple of 16
                                bytes and at most 16 KiB.                         */
};

/* Limits: 1 <= W, H <= 65536; 1 <= n <= 64; 1 <= C <= 4.  The backward
 * additionally needs W*H*n*n <= 2^32 (its sort key), n*n*C <= 4096 (its
 * bucket tiles in LDS: n = 64 with one channel, n = 32 with four), and the
 * number of records (N, or 4N in the bilinear-bucket mode) below 2^31. */

typedef struct {
    int32_t buckets_w;      /* W: bucket-matrix width  (paper's w, Sec. 2)        */
    int32_t buckets_h;      /* H: bucket-matrix height (paper's h, Sec. 2)        */
    int32_t n;              /* angular resolution: each bucket is n x n samples   */
    int32_t channels;       /* C, 1..4                                            */
    int32_t format;         /* rt_format                                          */
    int32_t layout;         /* rt_layout                                          */
    const void* data;       /* texels in `format` and `layout`                    */
    const float* scales;    /* [H][W] per-bucket scale: required for FP8 (decoded */
                            /* value = e4m3(code) * scale), must be NULL otherwise */
} rt_texture_desc;

/* Fragments of a G-buffer: for every visible pixel its texture coordinates
 * u,v and its incidence (view) vector, with the tangent frame that moves the
 * vector into orthogonal texture space (Sec. 2 and 2.1).
 * views/height/width are an optional tiling hint.  When all three are positive
 * the N = views * height * width fragments are `views` images of height x
 * width pixels, view-major and row-major, and the kernels visit them in
 * 32 x 8 pixel tiles, which keeps the texture fetches of neighbouring pixels
 * together in the caches; all three 0 means a flat list.  The hint changes
 * only the order of the visits, never a result.  Any other combination, or a
 * product that differs from count, is RT_ERR_INVALID_ARG. */
typedef struct {
    int64_t count;          /* N fragments (0 allowed)                            */
    int32_t views;          /* tiling hint: images, or 0                          */
    int32_t height;         /* tiling hint: rows per image, or 0                  */
    int32_t width;          /* tiling hint: pixels per row, or 0                  */
    const float* uv;        /* [N][2] texture coordinates; wrap (repeat)          */
    const float* tbn;       /* [N][3][3] rows T, B, N                              */
    const float* view;      /* [N][3] surface -> eye                               */
} rt_fragments;

typedef struct rt_texture rt_texture;   /* opaque handle (host metadata)          */

/* Wrap a radiance texture (Sec. 2: the bucket matrix of n x n hemispherical
 * maps).  For RT_LAYOUT_BUCKET_MAJOR the handle BORROWS desc->data and
 * desc->scales: the caller keeps them alive and unmodified while work that
 * reads them is in flight, and no device memory is allocated.  For
 * RT_LAYOUT_ATLAS the handle allocates a bucket-major copy on the current
 * device and enqueues the re-layout on `stream` (RT_ERR_OUT_OF_MEMORY if the
 * allocation fails); the handle owns that copy.
 * Errors: RT_ERR_INVALID_ARG (NULL pointers, sizes, enum values, alignment,
 * scales present/absent against the format), RT_ERR_UNSUPPORTED (limits),
 * RT_ERR_NO_DEVICE, RT_ERR_HIP. */
rt_status rt_create_texture(const rt_texture_desc* desc, void* stream, rt_texture** out);

/* A bucket dictionary: the compression of repetitive buckets ("highly
 * repetitive ... simple compression", Sec. 1 and Sec. 2) as a codebook of K
 * bucket entries, an index map naming each bucket's entry, and optionally a
 * gain per bucket.  Decoded bucket b = gains[b] * codebook[index[b]]; every
 * lookup reads that decoded matrix (a two-level gather). */
typedef struct {
    int32_t buckets_w;      /* W                                                  */
    int32_t buckets_h;      /* H                                                  */
    int32_t n;              /* angular resolution                                 */
    int32_t channels;       /* C, 1..4                                            */
    int32_t entries;        /* K >= 1 (<= 256 for 1-byte, <= 65536 for 2-byte   */
                            /* entry numbers)                                     */
    int32_t format;         /* codebook storage: RT_FMT_F32 or RT_FMT_BF16        */
    int32_t index_bytes;    /* 1, 2 or 4: unsigned entry numbers                  */
    int32_t reserved;       /* 0                                                  */
    const void* codebook;   /* [K][n][n][C] in `format`, 16-byte aligned          */
    const void* index;      /* [H][W] entry numbers; a number >= K reads entry    */
                            /* K-1 (device data is not checked on the host)       */
    const float* gains;     /* [H][W] per-bucket factor, or NULL (1)              */
} rt_dictionary_desc;

/* Wrap a bucket dictionary.  The handle BORROWS codebook, index and gains
 * (device memory the caller keeps alive).  It is accepted by rt_lookup_fwd,
 * rt_lookup_light and rt_debug_indices; rt_lookup_bwd, rt_quantize,
 * rt_build_mip and rt_lookup_fwd_lod refuse it.
 * Errors: RT_ERR_INVALID_ARG (NULL pointers, sizes, index_bytes, entries that
 * do not fit the entry numbers, alignment), RT_ERR_UNSUPPORTED (limits, a
 * format other than F32 or BF16), RT_ERR_NO_DEVICE. */
rt_status rt_create_dictionary_texture(const rt_dictionary_desc* desc, rt_texture** out);

/* Release a handle (and its owned copy, after a device synchronisation when
 * it owns one).  NULL is accepted. */
rt_status rt_destroy_texture(rt_texture* tex);

/* Per-bucket quantiser (the storage-footprint lever named in the abstract:
 * buckets "compress" well).  src must be an RT_FMT_F32 texture.
 *   RT_FMT_BF16      dst_codes: uint16 [H][W][n][n][C], round-to-nearest-even;
 *                    dst_scales must be NULL.
 *   RT_FMT_FP8_E4M3  per bucket: amax = max |x| (binary32); if amax is 0 or not
 *                    finite, scale = 1 and inv = 1, else inv = 448 / amax and
 *                    scale = amax / 448 (binary32, correctly rounded); codes =
 *                    E4M3 round-to-nearest-even of x * inv with saturation to
 *                    +-448 (NaN stays NaN).  dst_codes: uint8 [H][W][n][n][C];
 *                    dst_scales: float [H][W].
 *   RT_FMT_BIT1      src with C = 1: each sample becomes the bit (x >= 0.5), NaN
 *                    giving 0, in the layout of RT_FMT_BIT1.  dst_codes: uint32
 *                    [H][W][ceil(n*n/32)], 4-byte aligned, every word
 *                    OVERWRITTEN; dst_scales must be NULL.
 * Errors: RT_ERR_INVALID_ARG (NULL/misaligned outputs, src not F32, bad dst,
 * C != 1 for RT_FMT_BIT1). */
rt_status rt_quantize(const rt_texture* src, int32_t dst_format, void* dst_codes,
                      float* dst_scales, void* stream);

/* Forward lookup (Sec. 2 and 2.1): for every fragment f and channel c,
 *   M = tbn[f], I = M view / |M view|         (tangent-space incidence)
 *   A = sqrt(2) (I_x, I_y) / |(I_x, I_y, I_z + 1)|          (Eq. 1b)
 *   B = (|A|_2 / |A|_inf) A, B = 0 at A = 0                 (Eq. 3)
 *   B clamped to [1/n - 1, 1 - 1/n]^2                       (Note after Eq. 3)
 *   s = (B + 1) n / 2 - 1/2 in [0, n-1]^2  (sample centres at integers)
 *   bucket i = floor(frac(u) W), j = floor(frac(v) H)       (Sec. 2; nearest)
 *   out[f][c] = bilinear fetch at s inside bucket (i, j), decoded to binary32.
 * flags: RT_BUCKET_NEAREST or RT_BUCKET_BILINEAR, optionally with
 * RT_FWD_STAGE_BUCKETS (see the flags).  out: float [N][C].
 * Any storage format, RT_FMT_BIT1 included (its taps read 0 or 1).
 * Non-finite inputs give unspecified values but never out-of-bounds reads.
 * Errors: RT_ERR_INVALID_ARG (NULL/misaligned pointers, N < 0, bad flags),
 * RT_ERR_UNSUPPORTED (RT_FWD_STAGE_BUCKETS with the bilinear-bucket mode, a
 * dictionary or 1-bit texture, or a bucket it cannot stage). */
rt_status rt_lookup_fwd(const rt_texture* tex, const rt_fragments* frags, float* out,
                        uint32_t flags, void* stream);

/* Bytes of device workspace rt_lookup_bwd needs for `count` fragments (0 when
 * the arguments are invalid). */
size_t rt_lookup_bwd_workspace(const rt_texture* tex, int64_t count, uint32_t flags);

/* Backward of rt_lookup_fwd (an addition to the paper, which has no
 * derivatives) for upstream gradients grad_out [N][C]:
 *   grad_tex   float [H][W][n][n][C], dL/d(decoded texel); every element is
 *              OVERWRITTEN (untouched buckets get 0).  Computed by a stable
 *              bucket sort of the fragments' taps followed by a two-pass
 *              segmented reduction with a fixed summation order: the result is
 *              bitwise reproducible run to run and uses no float atomics.
 *              For BF16/FP8 textures it is the gradient w.r.t. the decoded
 *              values (straight-through).  NULL skips it.
 *   grad_view  float [N][3], dL/d(view).  NULL skips it.
 *   grad_uv    float [N][2], dL/d(u,v): 0 in nearest mode (the lookup is
 *              piecewise constant in u, v); the bilinear-bucket weights'
 *              derivative in RT_BUCKET_BILINEAR mode.  NULL skips it.
 * At the non-smooth points (texel lines, clamp bounds, the diagonal
 * |A_x| = |A_y|, A = 0, bucket edges) one-sided values are returned: an axis
 * clamped at (or beyond) its bound contributes no view gradient.
 * workspace: device memory of at least rt_lookup_bwd_workspace() bytes,
 * 256-byte aligned, owned by the caller, not used by concurrent calls.
 * Errors: RT_ERR_INVALID_ARG, RT_ERR_WORKSPACE_TOO_SMALL, RT_ERR_UNSUPPORTED
 * (sort key, bucket size or record count beyond the limits above, an
 * RT_FMT_BIT1 texture, a dictionary). */
rt_status rt_lookup_bwd(const rt_texture* tex, const rt_fragments* frags,
                        const float* grad_out, float* grad_tex, float* grad_view,
                        float* grad_uv, void* workspace, size_t workspace_bytes,
                        uint32_t flags, void* stream);

/* Allocation-free backward, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops that forbid allocation): the
 * same computation, arguments and results as rt_lookup_bwd, with the
 * workspace taken from a scratch array the library holds in device memory,
 * RT_NOALLOC_SCRATCH_BYTES (256 MiB) per GPU, kept until the process ends.
 * The call allocates nothing itself (with the kernel timer of rt_profile_*
 * enabled it records no events for this call).  Every call on a GPU shares
 * that GPU's scratch: calls that overlap in time on one GPU (other streams,
 * other threads) race and give undefined results; calls ordered on one
 * stream are safe (each clears what it needs).
 * Errors: as rt_lookup_bwd, and RT_ERR_WORKSPACE_TOO_SMALL when
 * rt_lookup_bwd_workspace() for these arguments exceeds
 * RT_NOALLOC_SCRATCH_BYTES (about five million nearest-mode fragments of
 * four channels), RT_ERR_HIP when the scratch's address cannot be found. */
#define RT_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
rt_status rt_lookup_bwd_noalloc(const rt_texture* tex, const rt_fragments* frags,
                                const float* grad_out, float* grad_tex, float* grad_view,
                                float* grad_uv, uint32_t flags, void* stream);

/* --- Visit plan ------------------------------------------------------------
 * The lookup is a gather (Sec. 2: the bucket is chosen by u, v and the sample
 * inside it by the view direction), so the order in which fragments are
 * visited decides how often a bucket's lines are fetched.  A visit plan
 * reorders a G-buffer by the backward's record key -- bucket (j W + i), then
 * cell (y0 n + x0) of the bilinear footprint, ties in the caller's fragment
 * order -- so that fragments reading the same bucket are visited together
 * (and, in nearest mode, the backward finds its records already sorted and
 * skips its sort; the results are the same bits either way).  It depends on
 * u, v, the frame and the view vector only, not on the texels: one plan
 * serves every step of a fit whose G-buffer stays fixed.
 *
 * Every per-fragment array of a planned lookup is in plan order: out and
 * grad_out of planned fragment k belong to the caller's fragment order[k].
 * A caller that keeps its own per-fragment data (targets, weights) permutes
 * it once with order. */

/* Bytes of device workspace rt_plan_fragments needs (0 when the arguments are
 * invalid). */
size_t rt_plan_workspace(const rt_texture* tex, int64_t count, uint32_t flags);

/* Plan the fragments of `frags` against the geometry (W, H, n) of `tex`
 * (its texels are not read).  flags: RT_BUCKET_NEAREST keys by the nearest
 * bucket; RT_BUCKET_BILINEAR by the first bucket (i0, j0) of the bilinear
 * footprint.
 *   order     DEVICE int32 [N], written: order[k] is the caller's index of
 *             planned fragment k (a permutation of 0..N-1).
 *   uv_out    DEVICE float [N][2], tbn_out [N][3][3], view_out [N][3],
 *             written: the planned G-buffer (fragment order[k] of the input at
 *             position k), for rt_lookup_fwd / rt_lookup_bwd without a tiling
 *             hint.  None of the four may overlap the input or each other.
 * The tiling hint of `frags` only decides which thread reads which fragment.
 * workspace: at least rt_plan_workspace() bytes, 256-byte aligned, owned by
 * the caller, not used by concurrent calls.  Asynchronous on `stream`.
 * Errors: RT_ERR_INVALID_ARG (NULL, alignment: order, tbn_out, view_out 4 B,
 * uv_out 8 B; overlapping arrays), RT_ERR_WORKSPACE_TOO_SMALL,
 * RT_ERR_UNSUPPORTED (W H n n beyond 2^32, count >= 2^31). */
rt_status rt_plan_fragments(const rt_texture* tex, const rt_fragments* frags, uint32_t flags,
                            int32_t* order, float* uv_out, float* tbn_out, float* view_out,
                            void* workspace, size_t workspace_bytes, void* stream);

/* Moves the rows of a per-fragment array by a plan's order: with
 * RT_PLAN_GATHER dst[k] = src[order[k]] (the caller's data into plan order:
 * targets, weights, an upstream gradient), with RT_PLAN_SCATTER
 * dst[order[k]] = src[k] (plan-order results back to the caller's order).
 * order: DEVICE int32 [count], a permutation of 0..count-1 (as written by
 * rt_plan_fragments); an entry outside 0..count-1 moves no row (its
 * destination row keeps its contents), and a repeated entry leaves which of
 * its rows a scatter keeps unspecified.  src, dst: DEVICE
 * arrays of count rows of row_bytes bytes (a multiple of 4, at most 4096),
 * 4-byte aligned (16-byte rows and alignment take 16-byte accesses), not
 * overlapping.  Asynchronous on `stream`.
 * Errors: RT_ERR_INVALID_ARG (NULL, alignment, sizes, overlap). */
enum { RT_PLAN_GATHER = 0, RT_PLAN_SCATTER = 1 };
rt_status rt_plan_permute(const int32_t* order, int64_t count, int32_t row_bytes,
                          const void* src, void* dst, uint32_t direction, void* stream);

/* Per-fragment indices of the nearest-bucket lookup, for exact checks:
 * idx int32 [N][4] = (i, j, x0, y0) with x0 = floor(s_x) in [0, n-1], and
 * frac float [N][2] = (s_x - x0, s_y - y0).  Same arithmetic as the lookup. */
rt_status rt_debug_indices(const rt_texture* tex, const rt_fragments* frags, int32_t* idx,
                           float* frac, void* stream);

/* --- Minification across the bucket matrix ---------------------------------
 * Sec. 2: taking one sample per bucket synthesises an ordinary W x H texture,
 * and the lookup is linear in the buckets (the sample position depends only
 * on the view), so minifying that texture by 2 x 2 pixels is the lookup in
 * the texel-wise mean of 2 x 2 buckets: a mip chain of bucket matrices. */

/* One level of the chain: dst = the level below src, a matrix of
 * max(1, W/2) x max(1, H/2) buckets whose bucket (i, j) is the texel-wise mean
 * of the 4 buckets (2i..2i+1, 2j..2j+1) of src (2 once a side of src is 1).
 * src: an FP32 bucket-major texture with W, H powers of two, not both 1.
 * dst: DEVICE float [max(1,H/2)][max(1,W/2)][n][n][C], 16-byte aligned,
 * every element OVERWRITTEN.  The mean of four FP32 values is formed as
 * ((a + b) + (c + d)) / 4.
 * Errors: RT_ERR_INVALID_ARG (NULL, alignment, sizes that are not powers of
 * two, a 1 x 1 source), RT_ERR_UNSUPPORTED (a format other than FP32). */
rt_status rt_build_mip(const rt_texture* src, float* dst, void* stream);

/* Lookup over a mip chain: levels[l] (l < nlevels) is a texture of
 * max(1, W >> l) x max(1, H >> l) buckets of level 0's n, channels and format
 * (W, H powers of two when nlevels > 1; nlevels <= 1 + log2(max(W, H)), at
 * most 17).  Per fragment, from duv[f] = (du/dx, dv/dx, du/dy, dv/dy), the
 * texture-coordinate derivatives across one pixel:
 *   rho    = max(|(du/dx W, dv/dx H)|, |(du/dy W, dv/dy H)|),
 *   lambda = log2 rho clamped to [0, nlevels - 1] (0 if rho is 0 or not
 *            finite),
 *   out    = (1 - t) L(floor(lambda)) + t L(floor(lambda) + 1),
 *            t = lambda - floor(lambda) (one level when t = 0),
 * with L(l) the lookup of rt_lookup_fwd on level l (flags as there).
 * duv: DEVICE float [N][4], 16-byte aligned; out as for rt_lookup_fwd.
 * Errors: RT_ERR_INVALID_ARG (NULL levels, a level of the wrong size, n,
 * channels or format, sizes that are not powers of two, duv/out NULL or
 * misaligned, bad fragments or flags), RT_ERR_UNSUPPORTED (nlevels > 17, an
 * RT_FMT_BIT1 chain). */
rt_status rt_lookup_fwd_lod(const rt_texture* const* levels, int32_t nlevels,
                            const rt_fragments* frags, const float* duv, float* out,
                            uint32_t flags, void* stream);

/* Bytes of device workspace rt_lookup_lod_bwd needs for `count` fragments
 * (0 when the arguments are invalid). */
size_t rt_lookup_lod_bwd_workspace(const rt_texture* const* levels, int32_t nlevels,
                                   int64_t count, uint32_t flags);

/* Backward of rt_lookup_fwd_lod for upstream gradients grad_out [N][C] (an
 * addition to the paper, like rt_lookup_bwd).  The level of detail is taken
 * as given (not differentiated): with each fragment's weights 1 - t on level
 * l0 and t on l0 + 1,
 *   grad_levels[l]  float [H_l][W_l][n][n][C], dL/d(level l's decoded texels):
 *                   rt_lookup_bwd's gradient on level l with every fragment's
 *                   upstream gradient times its weight on l; every element
 *                   OVERWRITTEN; a NULL entry skips that level;
 *   grad_view       float [N][3], the sum over the levels of rt_lookup_bwd's
 *                   view gradients (NULL skips it);
 *   grad_uv         float [N][2], likewise (0 in nearest mode).
 * Bitwise reproducible (a fixed summation order per bucket; the view and uv
 * gradients summed over the levels in level order), and a level's bits do
 * not depend on which other levels are requested.  To reach level 0 of
 * a chain built by rt_build_mip, fold each level's gradient down with
 * rt_build_mip_adjoint.  grad_levels: HOST array of nlevels DEVICE pointers
 * (16-byte aligned); duv as for rt_lookup_fwd_lod; workspace: DEVICE, at
 * least rt_lookup_lod_bwd_workspace() bytes, 256-byte aligned.
 * All levels are done in one pass: one sort key numbers the buckets of every
 * level, so the chain's buckets plus one must fit in 32 - ceil(log2(n*n))
 * bits (a level 0 of up to 4096 x 2048 buckets at n = 16).
 * Errors: as rt_lookup_fwd_lod and rt_lookup_bwd (RT_ERR_UNSUPPORTED for a
 * level beyond the backward's limits). */
rt_status rt_lookup_lod_bwd(const rt_texture* const* levels, int32_t nlevels,
                            const rt_fragments* frags, const float* duv, const float* grad_out,
                            float* const* grad_levels, float* grad_view, float* grad_uv,
                            void* workspace, size_t workspace_bytes, uint32_t flags,
                            void* stream);

/* Adjoint of rt_build_mip: src is the source level (its W x H, n, C; W and H
 * powers of two, not both 1); every bucket (i, j) of it receives
 * grad_dst[j / 2][i / 2] (for a side of 1: that coordinate itself) divided by
 * the number of buckets its parent averages (4, or 2 once a side is 1),
 * ADDED to grad_src.  grad_dst: DEVICE float [max(1,H/2)][max(1,W/2)][n][n][C];
 * grad_src: DEVICE float [H][W][n][n][C]; both 4-byte aligned.
 * Errors: RT_ERR_INVALID_ARG (NULL, alignment, sizes). */
rt_status rt_build_mip_adjoint(const rt_texture* src, const float* grad_dst, float* grad_src,
                               void* stream);

/* --- The bake: the write side of the method --------------------------------
 * Sec. 2.1 (after Eq. (4b)): ray-traced data is sampled onto the radiance
 * texture along the equisolid reflection vector R of every sample.  Here an
 * analytic environment stands in for the ray-traced radiance. */

/* Directions of the n x n sample centres of a bucket in orthogonal texture
 * space (N = e_z).  The centre of sample (x, y) is
 * B = ((2x+1)/n - 1, (2y+1)/n - 1); A follows from Eq. (4a); refl[y][x] is
 * the reflection vector of Eq. (4b) and inc[y][x] the incidence of Eq. (2c)
 * (its mirror image about N, the view direction the lookup maps onto that
 * sample).  inc, refl: DEVICE float [n][n][3], 4-byte aligned, either NULL.
 * Errors: RT_ERR_INVALID_ARG (n < 1, alignment), RT_ERR_UNSUPPORTED (n > 64),
 * RT_ERR_NO_DEVICE. */
rt_status rt_bake_directions(int32_t n, float* inc, float* refl, void* stream);

/* One spherical Gaussian lobe of the analytic environment. */
typedef struct {
    float axis[3];          /* direction in scene coordinates (normalised here)   */
    float sharpness;        /* lambda >= 0                                         */
    float amplitude[4];     /* per channel                                         */
} rt_env_lobe;

/* Bake a W x H matrix of n x n buckets with C channels, FP32 bucket-major:
 *   texels[j][i][y][x][c] = ambient[c]
 *       + sum_k amplitude_k[c] exp(sharpness_k (axis_k . d - 1)),
 *   d = normalize(M_ji^T R(x, y)),
 * R(x, y) as in rt_bake_directions and M_ji = frames[j][i] (rows T, B, N,
 * world -> tangent as in the lookup), so d is R in scene coordinates; a
 * mirror texture baked this way renders env(reflect(-V, N)) through
 * rt_lookup_fwd.  frames: DEVICE float [H][W][3][3], 4-byte aligned, or NULL
 * for the identity frame of every bucket.  lobes: HOST array of nlobes
 * (0..16), read during the call; ambient: HOST float[4].  texels: DEVICE
 * float [H][W][n][n][C], aligned to 16 (C = 4), 8 (C = 2) or 4 bytes,
 * every element OVERWRITTEN.
 * Errors: RT_ERR_INVALID_ARG (sizes, NULL pointers, alignment, a zero or
 * non-finite axis, negative or non-finite sharpness, non-finite amplitude or
 * ambient), RT_ERR_UNSUPPORTED (W or H > 65536, n > 64, nlobes > 16),
 * RT_ERR_NO_DEVICE, RT_ERR_HIP (launch). */
rt_status rt_bake_environment(int32_t W, int32_t H, int32_t n, int32_t C, const float* frames,
                              const rt_env_lobe* lobes, int32_t nlobes, const float* ambient,
                              float* texels, void* stream);

/* --- Shadowing (Sec. 5, Shadowing) -----------------------------------------
 * A 1-bit radiance texture holds the occlusion of static geometry: a sample's
 * bit says whether light from the sample's direction reaches the bucket's
 * surface point.  It is read with the direction toward the light in place of
 * the incidence vector, for directional and point lights, and an area light
 * is several light samples whose lookups are averaged (a soft shadow). */

enum {
    RT_LIGHT_DIRECTIONAL = 0,   /* vec[s]: direction toward the light (scene space) */
    RT_LIGHT_POINT = 1          /* vec[s]: a point of the light (scene space)        */
};
#define RT_MAX_LIGHT_SAMPLES 64

typedef struct {
    int32_t kind;                          /* RT_LIGHT_DIRECTIONAL or RT_LIGHT_POINT */
    int32_t samples;                       /* S, 1..RT_MAX_LIGHT_SAMPLES             */
    float vec[RT_MAX_LIGHT_SAMPLES][3];    /* the first S are used; need not be unit */
} rt_light;

/* Light lookup: for every fragment f and channel c,
 *   L_s    = vec[s]            (RT_LIGHT_DIRECTIONAL)
 *          = vec[s] - pos[f]   (RT_LIGHT_POINT, binary32 difference)
 *   out[f][c] = (1/S) sum_s lookup(tex, uv[f], tbn[f], L_s)[c],
 * where lookup is rt_lookup_fwd's computation with L_s in the place of the
 * view vector (flags as there).  With an RT_FMT_BIT1 texture out is the lit
 * fraction of the light's samples; any other format gives the light-indexed
 * radiance.  A light below the surface's horizon is not treated specially
 * (its direction is clamped onto the bucket edge as any vector is): the
 * cosine factor of the shading belongs to the caller.
 * frags: uv and tbn as for rt_lookup_fwd; frags->view is not read (may be
 * NULL).  pos: DEVICE float [N][3], 4-byte aligned, read for point lights
 * only (may be NULL otherwise).  light: HOST, read during the call.  out:
 * DEVICE float [N][C], aligned as for rt_lookup_fwd.
 * Errors: RT_ERR_INVALID_ARG (NULL/misaligned pointers, bad fragments, flags,
 * light kind or sample count, non-finite light vectors, pos NULL for a point
 * light). */
rt_status rt_lookup_light(const rt_texture* tex, const rt_fragments* frags, const float* pos,
                          const rt_light* light, float* out, uint32_t flags, void* stream);

/* Bake of a 1-bit shadow texture from analytic occluders, standing in for the
 * ray-traced visibility: bucket (i, j) sits at the scene point origins[j][i]
 * with frame M_ji = frames[j][i] (rows T, B, N as in the lookup; NULL: the
 * identity), and sample (x, y) gets bit 1 (lit) iff the ray from the origin
 * along d = normalize(M_ji^T I(x, y)) meets none of the balls, I(x, y) being
 * the incidence of rt_bake_directions (the direction the light lookup maps
 * onto that sample).  The ray o + t d, t > 0, meets ball (c, r) iff
 * |c - o| <= r, or t* = d . (c - o) > 0 and |c - o - t* d| <= r.
 * origins: DEVICE float [H][W][3]; frames: DEVICE float [H][W][3][3] or NULL;
 * both 4-byte aligned.  balls: HOST float [nballs][4] (centre x, y, z,
 * radius > 0), nballs 0..64, read during the call.  words: DEVICE uint32
 * [H][W][ceil(n*n/32)] in the layout of RT_FMT_BIT1, 4-byte aligned, every
 * word OVERWRITTEN.
 * Errors: RT_ERR_INVALID_ARG (sizes, NULL pointers, alignment, non-finite
 * balls, radius <= 0), RT_ERR_UNSUPPORTED (W or H > 65536, n > 64,
 * nballs > 64), RT_ERR_NO_DEVICE, RT_ERR_HIP (launch). */
rt_status rt_bake_shadow(int32_t W, int32_t H, int32_t n, const float* origins,
                         const float* frames, const float* balls, int32_t nballs,
                         uint32_t* words, void* stream);

/* --- Building a bucket dictionary: Lloyd's k-means steps --------------------
 * The rows are buckets as vectors of D = n*n*C values (a bucket-major FP32
 * texture is such a [W*H][D] matrix as it stands). */

/* Assignment: assign[b] = argmin_k |x_b - c_k|^2 over the K codebook rows,
 * evaluated as |c_k|^2 - 2 x_b . c_k with the products on the matrix cores in
 * binary32 (ties to the smaller k; near-ties within binary32 rounding may go
 * either way); dist[b] (if not NULL) = |x_b - c_assign|^2 >= 0.
 * x: DEVICE float [M][D], codebook: DEVICE float [K][D], both 16-byte
 * aligned; assign: DEVICE int32 [M]; dist: DEVICE float [M] or NULL.
 * Errors: RT_ERR_INVALID_ARG (NULL, alignment, M < 0, D < 1, K < 1),
 * RT_ERR_UNSUPPORTED (M >= 2^31, K > 65536). */
rt_status rt_vq_assign(const float* x, int64_t M, int32_t D, const float* codebook, int32_t K,
                       int32_t* assign, float* dist, void* stream);

/* Bytes of device workspace rt_vq_update needs (0 when the sizes are
 * outside its limits). */
size_t rt_vq_update_workspace(int64_t M, int32_t D, int32_t K);

/* Update: every codebook row k with at least one assigned row becomes the
 * mean of its rows (binary32 sums in a fixed order: the rows of an entry in
 * increasing b, in pieces of 64 whose sums are added in order), so the result
 * is bitwise reproducible; rows with no assigned row are left unchanged.
 * counts[k] (if not NULL) = rows assigned to k.  An entry number outside
 * [0, K) counts as the nearest valid one.
 * x: DEVICE float [M][D]; assign: DEVICE int32 [M]; codebook: DEVICE float
 * [K][D], updated in place; counts: DEVICE int32 [K] or NULL; all 4-byte
 * aligned.  workspace: DEVICE, rt_vq_update_workspace bytes, 256-byte
 * aligned, caller-owned, not shared by concurrent calls.
 * Errors: RT_ERR_INVALID_ARG (NULL, alignment, M < 1, D < 1, K < 1),
 * RT_ERR_WORKSPACE_TOO_SMALL, RT_ERR_UNSUPPORTED (K > 4096, M >= 2^31). */
rt_status rt_vq_update(const float* x, int64_t M, int32_t D, const int32_t* assign, int32_t K,
                       float* codebook, int32_t* counts, void* workspace,
                       size_t workspace_bytes, void* stream);

/* Thread-local description of the last non-OK status ("" if none). */
const char* rt_last_error(void);
const char* rt_status_string(rt_status status);
int32_t rt_version(void);

/* Kernel timing.  While enabled, every kernel the library enqueues is
 * bracketed by a pair of HIP events recorded on the same stream.
 * rt_profile_read synchronises on the recorded events and returns, for
 * kernel id k in [0, rt_profile_kernel_count()), the number of launches and
 * their summed duration in milliseconds since the last reset. */
rt_status rt_profile_enable(int32_t enabled);
rt_status rt_profile_reset(void);
int32_t rt_profile_kernel_count(void);
const char* rt_profile_kernel_name(int32_t kernel);
rt_status rt_profile_read(int32_t kernel, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* RADTEX_H */
