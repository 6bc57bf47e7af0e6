// rt_kernels.hpp -- host-side launchers of the gfx950 kernels (internal to
// libradtex.so; the public interface is include/radtex.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rt {

struct TexView;
struct FragMap;
struct LevelSet;

// Kernel ids for the event-based timing of rt_profile_*.
enum KernelId {
    K_LOOKUP_FWD = 0,
    K_DEBUG_INDICES,
    K_QUANT_BF16,
    K_QUANT_FP8,
    K_ATLAS_RELAYOUT,
    K_BWD_FRAGMENT,
    K_FILL,
    K_RADIX_HIST,
    K_SCAN,
    K_RADIX_SCATTER,
    K_BUCKET_RANGES,
    K_SEGACC,
    K_SEGACC_HOT,
    K_COMBINE_HOT,
    K_SEGACC_BIG,
    K_BAKE_DIRECTIONS,
    K_BAKE_ENV,
    K_BUILD_MIP,
    K_LOOKUP_LOD,
    K_PACK_BITS,
    K_LOOKUP_LIGHT,
    K_BAKE_SHADOW,
    K_VQ_ASSIGN,
    K_VQ_HIST,
    K_VQ_SCATTER,
    K_VQ_PIECES,
    K_VQ_COMBINE,
    K_LOD_BWD_FRAGMENT,
    K_MIP_ADJOINT,
    K_PAYLOAD,
    K_ORDER_CHECK,
    K_PLAN_KEYS,
    K_PLAN_GATHER,
    K_PERMUTE,
    K_COUNT
};
const char* kernel_name(int id);
void prof_begin(int id, hipStream_t s);
void prof_end(int id, hipStream_t s);

hipError_t launch_lookup_fwd(const TexView& t, int fmt, int mode, const float* uv,
                             const float* tbn, const float* view, float* out, const FragMap& m,
                             hipStream_t s);
// The forward with bucket tiles staged in LDS (nearest buckets): supported
// for plain F32 / BF16 / FP8 textures whose bucket is a multiple of 16 bytes
// and at most STAGED_BUCKET_BYTES (four wavefronts' tiles per workgroup).
constexpr int STAGED_BUCKET_BYTES = 16384;
bool lookup_staged_supported(const TexView& t, int fmt);
hipError_t launch_lookup_fwd_staged(const TexView& t, int fmt, const float* uv, const float* tbn,
                                    const float* view, float* out, const FragMap& m,
                                    hipStream_t s);
hipError_t launch_debug_indices(const TexView& t, const float* uv, const float* tbn,
                                const float* view, int32_t* idx, float* frac, const FragMap& m,
                                hipStream_t s);
hipError_t launch_quantize(const TexView& src, int dst_fmt, void* codes, float* scales,
                           hipStream_t s);
hipError_t launch_build_mip(const TexView& src, float* dst, hipStream_t s);
hipError_t launch_lookup_lod(const LevelSet& ls, int fmt, int mode, const float* uv,
                             const float* tbn, const float* view, const float* duv, float* out,
                             const FragMap& m, hipStream_t s);
// Light lookup (shadowing with a 1-bit texture, or any radiance texture
// indexed by the light direction): per fragment the mean over the light's
// samples of the lookup taken with the direction toward the light.
constexpr int MAX_LIGHT_SAMPLES = 64;
constexpr int LIGHT_DIRECTIONAL = 0, LIGHT_POINT = 1;
struct LightParams {
    int kind;           // LIGHT_DIRECTIONAL: vec = directions; LIGHT_POINT: sample points
    int samples;        // 1..MAX_LIGHT_SAMPLES
    float inv_samples;  // 1 / samples
    float vec[MAX_LIGHT_SAMPLES][3];
};
hipError_t launch_lookup_light(const TexView& t, int fmt, int mode, const float* uv,
                               const float* tbn, const float* pos, const LightParams& lp,
                               float* out, const FragMap& m, hipStream_t s);
hipError_t launch_atlas_to_buckets(const void* atlas, void* dst, int W, int H, int n, int C,
                                   int elem_bytes, hipStream_t s);

// Bake: the analytic environment, lobe axes normalised on the host.
constexpr int MAX_LOBES = 16;
struct EnvParams {
    int lobes;
    float ambient[4];
    // per lobe: lambda log2(e) times the unit axis (x, y, z), -lambda log2(e),
    // amplitude per channel; the lobe's value at d is exp2(first three . d + 4th)
    float lobe[MAX_LOBES][8];
};
hipError_t launch_bake_directions(int n, float* inc, float* refl, hipStream_t s);

// Shadow bake: balls (centre x, y, z, radius) as the occluders.
constexpr int MAX_OCCLUDERS = 64;
struct Occluders {
    int count;
    float ball[MAX_OCCLUDERS][4];
};
hipError_t launch_bake_shadow(int W, int H, int n, const float* origins, const float* frames,
                              const Occluders& occ, uint32_t* words, hipStream_t s);
hipError_t launch_bake_env(int W, int H, int n, int C, const float* frames, const EnvParams& env,
                           float* texels, hipStream_t s);

// Backward.
struct BwdPlan {
    int64_t records;      // N (nearest) or 4N (bilinear-bucket)
    int key_bits;         // bucket bits + cell bits
    int cell_bits;
    int passes;           // radix passes, digits of at most 10 (9) bits
    int digit_bits[4];    // bits of each pass's digit (balanced)
    int digit_shift[4];   // position of each pass's digit in the key
    int bins;             // 2^D of the widest pass's kernel (D = 8, 9 or 10)
    int64_t tiles;        // radix tiles
    int64_t scan_len;     // bins * tiles
    int64_t scan_blocks;  // partial sums of the scan
    int64_t chunks;       // fixed chunks of the sorted records (hot buckets)
    int64_t tile_elems;   // n*n*C
    int64_t big_cap;      // entries per big-bucket list (one list per counter)
    int64_t buckets;      // W * H
    uint32_t sentinel;    // sparse plans: the key of a fragment whose upstream
                          // gradient is zero (past every bucket); 0 otherwise
    // workspace offsets (bytes); the sort's buffers and the disorder word
    // come first and end at sort_total
    size_t off_keys0, off_keys1, off_vals0, off_vals1, off_hist, off_hoff, off_scanp,
        off_disorder, sort_total, off_wrec, off_payf, off_payg, off_range, off_biglist,
        off_part, total;
};
constexpr int PIECE = 2048;  // records per chunk; buckets with more are "hot"
constexpr int SEG_GROUP = 8;  // buckets per wavefront in the first accumulation pass
constexpr int BIG_LISTS = 64; // big-bucket lists, each with its own counter
constexpr int BIG_STRIDE = 64;  // u32 between two counters (256 bytes)
constexpr int HOT_FLAG = 1;     // u32 after counter 0: set when a bucket needs pass 2
constexpr int PAYLOAD_PER_THREAD = 4;  // sorted records per thread in the payload launch
constexpr int ORDER_FLAGS_AT = 64;  // u32 after the disorder word where the order flags start
constexpr int BIG_RUN = 64;     // consecutive groups that append to one list
// sparse: fragments whose upstream gradient is all zero make no records (their
// keys sort past every bucket and are skipped), at the price of one key bit.
bool plan_backward(int W, int H, int n, int C, int64_t N, int mode, BwdPlan* p,
                   bool sparse = false);

// Where the accumulation writes the tile of bucket b: the buckets of one
// gradient, or those of the levels of a chain numbered one level after the
// other (level l holds buckets [start[l], start[l + 1]) and writes them to
// grad[l]; a NULL level is not written).
struct TileOut {
    int levels;
    int64_t start[MAX_LEVELS + 1];
    float* grad[MAX_LEVELS];
};

// Steps after the per-fragment kernel: sort the records, find the bucket
// ranges, write the sorted payload, accumulate the tiles into `out`.
// grad_out: the upstream gradient of the records' fragments (units).
hipError_t launch_accumulate(int n, int C, int mode, const float* grad_out, const TileOut& out,
                             const BwdPlan& plan, void* ws, hipStream_t s);

// Backward of the level-of-detail lookup in one pass: every fragment makes
// records on the (one or two) levels it blends, in the chain's bucket
// numbering, as two units 2f and 2f + 1 (levels l0 and l0 + 1) whose upstream
// gradient is the fragment's times the level's weight; one sort and one
// accumulation serve all levels.  Workspace: the backward's for 2N units, then
// the units' weighted gradient [2N][C].
struct LodBwdLayout {
    size_t off_bwd, off_gl, total;
};
hipError_t launch_lookup_lod_bwd(const LevelSet& ls, int fmt, int mode, const float* uv,
                                 const float* tbn, const float* view, const float* duv,
                                 const float* grad_out, float* const* grad_levels,
                                 float* grad_view, float* grad_uv, const FragMap& m,
                                 const BwdPlan& plan, const LodBwdLayout& lay, void* ws,
                                 hipStream_t s);
hipError_t launch_lod_bwd_fragment(const LevelSet& ls, int fmt, int mode, const float* uv,
                                   const float* tbn, const float* view, const float* duv,
                                   const float* grad_out, const int64_t* start,
                                   float* grad_view, float* grad_uv,
                                   uint32_t* keys, float* wrec, float* gl, const FragMap& m,
                                   int cell_bits, uint32_t sentinel, hipStream_t s);
hipError_t launch_mip_adjoint(const TexView& src, const float* grad_dst, float* grad_src,
                              hipStream_t s);

// Device-wide exclusive scan of L uint32 values (the backward's three-kernel
// scan); part holds ceil(L / 4096) + 1 words.
hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, uint32_t* part, int64_t L,
                                 hipStream_t s);

// Bucket dictionary: Lloyd's assignment (MFMA) and update steps.
constexpr int VQ_MAX_UPDATE_ENTRIES = 4096;  // entries the update's LDS counters hold
constexpr int VQ_CHUNK = 4096;               // rows per chunk of the update's counting sort
constexpr int VQ_PIECE = 64;                 // rows summed by one workgroup of the update
struct VqPlan {
    int64_t M;
    int D, K;
    int64_t chunks, hist_len, pieces_max;
    size_t off_hist, off_offs, off_part, off_sorted, off_ptab, off_pstart, off_ppart, off_sums,
        total;
};
bool plan_vq_update(int64_t M, int D, int K, VqPlan* p);
hipError_t launch_vq_assign(const float* x, int64_t M, int D, const float* codebook, int K,
                            int32_t* assign, float* dist, hipStream_t s);
hipError_t launch_vq_update(const float* x, const int32_t* assign, float* codebook,
                            int32_t* counts, const VqPlan& plan, void* ws, hipStream_t s);

// The stable sort of a plan's records (keys in the workspace's keys0); with
// disorder non-NULL its launches return at once when that device word is 0.
void launch_sort_records(const BwdPlan& plan, void* ws, const uint32_t* disorder, hipStream_t s,
                         const uint32_t** skeys, const uint32_t** svals);

// Visit plan: the fragments ordered by their nearest-mode record key (or the
// key of their first bucket in the bilinear-bucket mode), stable in the
// fragment index; writes order[k] (the caller's index of planned fragment k)
// and the planned G-buffer.  plan: plan_backward(W, H, n, 1, N, MODE_NEAREST);
// the workspace needs plan.sort_total bytes.
hipError_t launch_plan(const TexView& t, int mode, const float* uv, const float* tbn,
                       const float* view, const FragMap& m, const BwdPlan& plan, void* ws,
                       int32_t* order, float* uv_out, float* tbn_out, float* view_out,
                       hipStream_t s);

// The allocation-free backward's scratch: a file-scope device array of
// NOALLOC_SCRATCH_BYTES per GPU; *out receives the current device's address
// of it (looked up once per device).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(256) << 20;
hipError_t noalloc_scratch(void** out);

// While alive, the kernel timer records nothing on this thread (it would
// create events).
struct ProfileSuspend {
    ProfileSuspend();
    ~ProfileSuspend();
};

// Rows of row_words 4-byte words moved by a plan's order: dst[k] =
// src[order[k]] (gather) or dst[order[k]] = src[k] (scatter).
hipError_t launch_permute_rows(const int32_t* order, int64_t N, int row_words, const void* src,
                               void* dst, bool scatter, hipStream_t s);

hipError_t launch_backward(const TexView& t, int fmt, int mode, const float* uv,
                           const float* tbn, const float* view, const float* grad_out,
                           float* grad_tex, float* grad_view, float* grad_uv, const FragMap& m,
                           const BwdPlan& plan, void* ws, hipStream_t s);

}  // namespace rt
