// rt_dictionary.hip -- building a bucket dictionary on gfx950: Lloyd's
// assignment step as an FP32 matrix-core contraction with an argmin epilogue,
// and a deterministic update step (counting sort of the rows by entry, then
// fixed-order sums).
//
// The dictionary is the compression of repetitive buckets (Sec. 1 and
// Sec. 2): each bucket, a vector of D = n n C values, is replaced by the
// nearest of K codebook entries.  Assignment: e(b) = argmin_k |x_b - c_k|^2
// = argmin_k (|c_k|^2 - 2 x_b . c_k), so the work is the M x K x D product of
// the buckets with the codebook: a dense contraction, on MFMA.
#include <algorithm>

#include "rt_device.hpp"
#include "rt_kernels.hpp"

namespace rt {

typedef float v4f __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Assignment.  A workgroup (4 waves) owns VQ_BM = 64 rows and sweeps the
// codebook in chunks of VQ_BN = 256 entries, staging VQ_BK = 32 columns of
// the rows and of the chunk's entries in LDS (k-major, padded so that the
// operand reads of a wave hit distinct banks).  Wave w computes the 64 x 64
// block of dot products of all rows with entries 64w .. 64w+63 of the chunk
// as 4 x 4 tiles of v_mfma_f32_16x16x4_f32:
//   A operand (16 x 4): lane l holds A[l % 16][l / 16] = x[row][k]
//   B operand (4 x 16): lane l holds B[l / 16][l % 16] = c[entry][k]
//   result (16 x 16):   lane l holds D[4 (l / 16) + i][l % 16], i = 0..3
// (the layout was checked on the device against a host product).  Thread t
// also accumulates |c|^2 of entry t of the chunk from the staged values.
// Epilogue: per row the smallest |c|^2 - 2 x . c over the chunk (ties to the
// smaller entry), reduced across the 16 lanes that share a row, then across
// the 4 waves, then against the previous chunks.
// ---------------------------------------------------------------------------
constexpr int VQ_BM = 64, VQ_BN = 256, VQ_BK = 32;

__device__ __forceinline__ bool vq_better(float v, int k, float bv, int bk) {
    return v < bv || (v == bv && k < bk);
}

__global__ __launch_bounds__(256) void k_vq_assign(const float* __restrict__ X, int64_t M, int D,
                                                   const float* __restrict__ Cb, int K,
                                                   int32_t* __restrict__ assign,
                                                   float* __restrict__ dist) {
    __shared__ float Xs[VQ_BK][VQ_BM + 1];
    __shared__ float Cs[VQ_BK][VQ_BN + 1];
    __shared__ float cn[VQ_BN];
    __shared__ float xn[VQ_BM];
    __shared__ float red_v[4][VQ_BM];
    __shared__ int red_k[4][VQ_BM];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int64_t r0 = (int64_t)xcd_block_id(blockIdx.x, gridDim.x) * VQ_BM;
    const bool vec = (D % 8) == 0;  // rows and entries 32-byte aligned: vector loads
    float best_v = INFINITY;
    int best_k = 0;
    // staging roles: row tr = tid / 4 takes 8 columns starting at tk = 8 (tid % 4)
    const int tr = tid >> 2, tk = (tid & 3) * 8;
    const int64_t xrow = r0 + tr;
    float xsq = 0.f;
    for (int e0 = 0; e0 < K; e0 += VQ_BN) {
        v4f acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++) acc[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
        const int ent = e0 + tid;  // entry whose column this thread stages
        float csq = 0.f;
        for (int k0 = 0; k0 < D; k0 += VQ_BK) {
            __syncthreads();  // the previous stage's operands have been read
            float xv[8];
            if (vec && xrow < M && k0 + tk < D) {
                const float4* src = (const float4*)(X + xrow * D + k0 + tk);
                const float4 p = src[0], q = src[1];
                xv[0] = p.x; xv[1] = p.y; xv[2] = p.z; xv[3] = p.w;
                xv[4] = q.x; xv[5] = q.y; xv[6] = q.z; xv[7] = q.w;
            } else {
#pragma unroll
                for (int j = 0; j < 8; j++)
                    xv[j] = (xrow < M && k0 + tk + j < D) ? X[xrow * D + k0 + tk + j] : 0.f;
            }
#pragma unroll
            for (int j = 0; j < 8; j++) {
                Xs[tk + j][tr] = xv[j];
                if (e0 == 0) xsq += xv[j] * xv[j];
            }
            if (ent < K) {
                const float* src = Cb + (int64_t)ent * D + k0;
                if (vec && k0 + VQ_BK <= D) {
#pragma unroll
                    for (int j = 0; j < VQ_BK; j += 4) {
                        const float4 p = *(const float4*)(src + j);
                        Cs[j][tid] = p.x; Cs[j + 1][tid] = p.y;
                        Cs[j + 2][tid] = p.z; Cs[j + 3][tid] = p.w;
                        csq += p.x * p.x + p.y * p.y + p.z * p.z + p.w * p.w;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < VQ_BK; j++) {
                        const float v = k0 + j < D ? src[j] : 0.f;
                        Cs[j][tid] = v;
                        csq += v * v;
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < VQ_BK; j++) Cs[j][tid] = 0.f;
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < VQ_BK / 4; s++) {
                const int kk = 4 * s + (lane >> 4);
                float av[4], bv[4];
#pragma unroll
                for (int a = 0; a < 4; a++) av[a] = Xs[kk][16 * a + (lane & 15)];
#pragma unroll
                for (int b = 0; b < 4; b++) bv[b] = Cs[kk][64 * w + 16 * b + (lane & 15)];
#pragma unroll
                for (int a = 0; a < 4; a++)
#pragma unroll
                    for (int b = 0; b < 4; b++)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b],
                                                                         0, 0, 0);
            }
        }
        cn[tid] = csq;
        if (e0 == 0) {
            // |x|^2 of row tr from its four stagers
            float t = xsq;
            t += __shfl_xor(t, 1, 64);
            t += __shfl_xor(t, 2, 64);
            if ((tid & 3) == 0) xn[tr] = t;
        }
        __syncthreads();
        // per row: the best entry of this wave's 64 columns
#pragma unroll
        for (int a = 0; a < 4; a++) {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                float bvv = INFINITY;
                int bkk = 0x7FFFFFFF;
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    const int col = 64 * w + 16 * b + (lane & 15);
                    const int e = e0 + col;
                    const float v = e < K ? cn[col] - 2.f * acc[a][b][i] : INFINITY;
                    if (vq_better(v, e, bvv, bkk)) { bvv = v; bkk = e; }
                }
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) {
                    const float ov = __shfl_xor(bvv, o, 64);
                    const int ok = __shfl_xor(bkk, o, 64);
                    if (vq_better(ov, ok, bvv, bkk)) { bvv = ov; bkk = ok; }
                }
                if ((lane & 15) == 0) {
                    const int row = 16 * a + 4 * (lane >> 4) + i;
                    red_v[w][row] = bvv;
                    red_k[w][row] = bkk;
                }
            }
        }
        __syncthreads();
        if (tid < VQ_BM) {
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (vq_better(red_v[q][tid], red_k[q][tid], best_v, best_k)) {
                    best_v = red_v[q][tid];
                    best_k = red_k[q][tid];
                }
        }
    }
    if (tid < VQ_BM && r0 + tid < M) {
        assign[r0 + tid] = best_k;
        if (dist) dist[r0 + tid] = fmaxf(best_v + xn[tid], 0.f);
    }
}

hipError_t launch_vq_assign(const float* x, int64_t M, int D, const float* codebook, int K,
                            int32_t* assign, float* dist, hipStream_t s) {
    if (M <= 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)((M + VQ_BM - 1) / VQ_BM);
    prof_begin(K_VQ_ASSIGN, s);
    hipLaunchKernelGGL(k_vq_assign, dim3(blocks), dim3(256), 0, s, x, M, D, codebook, K, assign,
                       dist);
    prof_end(K_VQ_ASSIGN, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Update: entry k becomes the mean of the rows assigned to it, summed in a
// fixed order, so the result is bitwise reproducible (no float atomics).
//   1. per chunk of VQ_CHUNK rows, the count of each entry (LDS counters);
//      counts laid out entry-major, hist[k][chunk];
//   2. exclusive scan of hist: where each (entry, chunk) run starts in the
//      rows sorted by entry;
//   3. stable scatter of the row ids, chunk by chunk in rounds of 256 rows
//      (a row's rank among the round's rows of its entry is counted from
//      LDS), so each entry's rows end up in increasing order;
//   4. each entry's rows are cut into pieces of VQ_PIECE; one workgroup sums a
//      piece's rows in order; then one workgroup per entry sums its pieces in
//      order and divides by the count (an entry with no row keeps its value).
// Entry numbers past K - 1 are read as K - 1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int vq_entry(const int32_t* assign, int64_t r, int K) {
    const int e = assign[r];
    return e < 0 ? 0 : (e >= K ? K - 1 : e);
}

__global__ __launch_bounds__(256) void k_vq_hist(const int32_t* __restrict__ assign, int64_t M,
                                                 int K, int64_t chunks,
                                                 uint32_t* __restrict__ hist) {
    __shared__ uint32_t cnt[VQ_MAX_UPDATE_ENTRIES];
    const int64_t c = blockIdx.x;
    for (int k = threadIdx.x; k < K; k += 256) cnt[k] = 0;
    __syncthreads();
    const int64_t r0 = c * VQ_CHUNK;
    const int64_t r1 = std::min<int64_t>(r0 + VQ_CHUNK, M);
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) atomicAdd(&cnt[vq_entry(assign, r, K)], 1u);
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += 256) hist[(int64_t)k * chunks + c] = cnt[k];
}

__global__ __launch_bounds__(256) void k_vq_scatter(const int32_t* __restrict__ assign, int64_t M,
                                                    int K, int64_t chunks,
                                                    const uint32_t* __restrict__ offs,
                                                    uint32_t* __restrict__ sorted) {
    __shared__ uint32_t base[VQ_MAX_UPDATE_ENTRIES];
    __shared__ int keys[256];
    const int64_t c = blockIdx.x;
    for (int k = threadIdx.x; k < K; k += 256) base[k] = offs[(int64_t)k * chunks + c];
    const int64_t r0 = c * VQ_CHUNK;
    const int64_t r1 = std::min<int64_t>(r0 + VQ_CHUNK, M);
    for (int64_t rb = r0; rb < r1; rb += 256) {
        const int64_t r = rb + threadIdx.x;
        const int k = r < r1 ? vq_entry(assign, r, K) : -1;
        __syncthreads();  // base is current, keys free
        keys[threadIdx.x] = k;
        __syncthreads();
        int rank = 0, after = 0;
        if (k >= 0) {
            for (int q = 0; q < 256; q++) {
                const int kq = keys[q];
                rank += (q < (int)threadIdx.x && kq == k) ? 1 : 0;
                after += (q > (int)threadIdx.x && kq == k) ? 1 : 0;
            }
            sorted[base[k] + rank] = (uint32_t)r;
        }
        __syncthreads();  // every thread has read base
        if (k >= 0 && after == 0) base[k] += (uint32_t)(rank + 1);
    }
}

// pieces of each entry: ptab[k] = ceil(count_k / VQ_PIECE); count_k from the
// scanned offsets (the scan's value past the last element is the total M)
__global__ __launch_bounds__(256) void k_vq_piece_table(const uint32_t* __restrict__ offs, int K,
                                                        int64_t chunks, int64_t M,
                                                        uint32_t* __restrict__ ptab) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= K) return;
    const uint32_t start = offs[(int64_t)k * chunks];
    const uint32_t end = k + 1 < K ? offs[(int64_t)(k + 1) * chunks] : (uint32_t)M;
    ptab[k] = (end - start + VQ_PIECE - 1) / VQ_PIECE;
}

// one workgroup per piece: sum its rows in order (columns over the threads)
__global__ __launch_bounds__(256) void k_vq_piece_sum(const float* __restrict__ X, int64_t M,
                                                      int D, int K, int64_t chunks,
                                                      const uint32_t* __restrict__ offs,
                                                      const uint32_t* __restrict__ pstart,
                                                      const uint32_t* __restrict__ ptab,
                                                      const uint32_t* __restrict__ sorted,
                                                      float* __restrict__ psum) {
    const uint32_t q = blockIdx.x;
    const uint32_t total = pstart[K - 1] + ptab[K - 1];
    if (q >= total) return;
    // the entry holding piece q: the last k with pstart[k] <= q
    int lo = 0, hi = K - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pstart[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    const int k = lo;
    const uint32_t start = offs[(int64_t)k * chunks];
    const uint32_t end = k + 1 < K ? offs[(int64_t)(k + 1) * chunks] : (uint32_t)M;
    const uint32_t m0 = start + (q - pstart[k]) * VQ_PIECE;
    const uint32_t m1 = std::min<uint32_t>(m0 + VQ_PIECE, end);
    for (int d = threadIdx.x; d < D; d += 256) {
        // eight rows' loads in flight at a time; the sum still runs in order
        float acc = 0.f;
        uint32_t m = m0;
        for (; m + 8 <= m1; m += 8) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; j++) v[j] = X[(int64_t)sorted[m + j] * D + d];
#pragma unroll
            for (int j = 0; j < 8; j++) acc += v[j];
        }
        for (; m < m1; m++) acc += X[(int64_t)sorted[m] * D + d];
        psum[(int64_t)q * D + d] = acc;
    }
}

// one workgroup per (entry, 256 columns): the entry's pieces in order, then
// the mean; eight pieces' loads in flight at a time
__global__ __launch_bounds__(256) void k_vq_combine(int64_t M, int D, int K, int64_t chunks,
                                                    const uint32_t* __restrict__ offs,
                                                    const uint32_t* __restrict__ pstart,
                                                    const uint32_t* __restrict__ ptab,
                                                    const float* __restrict__ psum,
                                                    float* __restrict__ Cb,
                                                    int32_t* __restrict__ counts) {
    const int k = blockIdx.x;
    const int d = blockIdx.y * 256 + threadIdx.x;
    const uint32_t start = offs[(int64_t)k * chunks];
    const uint32_t end = k + 1 < K ? offs[(int64_t)(k + 1) * chunks] : (uint32_t)M;
    const uint32_t cnt = end - start;
    if (blockIdx.y == 0 && threadIdx.x == 0 && counts) counts[k] = (int32_t)cnt;
    if (cnt == 0 || d >= D) return;
    const float* src = psum + (int64_t)pstart[k] * D + d;
    const uint32_t np = ptab[k];
    float acc = 0.f;
    uint32_t p = 0;
    for (; p + 8 <= np; p += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; j++) v[j] = src[(int64_t)(p + j) * D];
#pragma unroll
        for (int j = 0; j < 8; j++) acc += v[j];
    }
    for (; p < np; p++) acc += src[(int64_t)p * D];
    Cb[(int64_t)k * D + d] = acc * (1.0f / (float)cnt);
}

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

bool plan_vq_update(int64_t M, int D, int K, VqPlan* p) {
    if (M < 1 || D < 1 || K < 1 || K > VQ_MAX_UPDATE_ENTRIES || M >= (1ll << 31)) return false;
    p->M = M;
    p->D = D;
    p->K = K;
    p->chunks = (M + VQ_CHUNK - 1) / VQ_CHUNK;
    p->hist_len = (int64_t)K * p->chunks;
    p->pieces_max = (M + VQ_PIECE - 1) / VQ_PIECE + K;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += a256(bytes);
        return o;
    };
    p->off_hist = take((size_t)p->hist_len * 4);
    p->off_offs = take((size_t)p->hist_len * 4);
    p->off_part = take((size_t)((p->hist_len + 4095) / 4096 + 1) * 4);
    p->off_sorted = take((size_t)M * 4);
    p->off_ptab = take((size_t)K * 4);
    p->off_pstart = take((size_t)K * 4);
    p->off_ppart = take((size_t)((K + 4095) / 4096 + 1) * 4);
    p->off_sums = take((size_t)p->pieces_max * D * 4);
    p->total = off;
    return true;
}

hipError_t launch_vq_update(const float* x, const int32_t* assign, float* codebook,
                            int32_t* counts, const VqPlan& p, void* ws, hipStream_t s) {
    char* base = (char*)ws;
    uint32_t* hist = (uint32_t*)(base + p.off_hist);
    uint32_t* offs = (uint32_t*)(base + p.off_offs);
    uint32_t* part = (uint32_t*)(base + p.off_part);
    uint32_t* sorted = (uint32_t*)(base + p.off_sorted);
    uint32_t* ptab = (uint32_t*)(base + p.off_ptab);
    uint32_t* pstart = (uint32_t*)(base + p.off_pstart);
    uint32_t* ppart = (uint32_t*)(base + p.off_ppart);
    float* psum = (float*)(base + p.off_sums);
    prof_begin(K_VQ_HIST, s);
    hipLaunchKernelGGL(k_vq_hist, dim3((uint32_t)p.chunks), dim3(256), 0, s, assign, p.M, p.K,
                       p.chunks, hist);
    prof_end(K_VQ_HIST, s);
    hipError_t e = launch_exclusive_scan(hist, offs, part, p.hist_len, s);
    if (e != hipSuccess) return e;
    prof_begin(K_VQ_SCATTER, s);
    hipLaunchKernelGGL(k_vq_scatter, dim3((uint32_t)p.chunks), dim3(256), 0, s, assign, p.M, p.K,
                       p.chunks, (const uint32_t*)offs, sorted);
    hipLaunchKernelGGL(k_vq_piece_table, dim3((uint32_t)((p.K + 255) / 256)), dim3(256), 0, s,
                       (const uint32_t*)offs, p.K, p.chunks, p.M, ptab);
    prof_end(K_VQ_SCATTER, s);
    e = launch_exclusive_scan(ptab, pstart, ppart, p.K, s);
    if (e != hipSuccess) return e;
    prof_begin(K_VQ_PIECES, s);
    hipLaunchKernelGGL(k_vq_piece_sum, dim3((uint32_t)p.pieces_max), dim3(256), 0, s, x, p.M, p.D,
                       p.K, p.chunks, (const uint32_t*)offs, (const uint32_t*)pstart,
                       (const uint32_t*)ptab, (const uint32_t*)sorted, psum);
    prof_end(K_VQ_PIECES, s);
    prof_begin(K_VQ_COMBINE, s);
    hipLaunchKernelGGL(k_vq_combine, dim3((uint32_t)p.K, (uint32_t)((p.D + 255) / 256)), dim3(256), 0, s, p.M, p.D, p.K,
                       p.chunks, (const uint32_t*)offs, (const uint32_t*)pstart,
                       (const uint32_t*)ptab, (const float*)psum, codebook, counts);
    prof_end(K_VQ_COMBINE, s);
    return hipGetLastError();
}

}  // namespace rt
