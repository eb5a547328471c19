// Device-wide exclusive prefix sum of u32 words (reduce, scan the tile sums,
// scan tiles again and add; one block for short arrays), plus a fill kernel.
#include "internal.h"

namespace sfcnl {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 4;
constexpr int kTile = kThreads * kItems;

// Exclusive scan of one value per thread over a 256-thread block.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_waves, uint32_t *total) {
    const int lane = sfc_lane();
    const int w = threadIdx.x / kWave;
    uint32_t inc = sfc_incl_scan(v);
    if (lane == kWave - 1) s_waves[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kThreads / kWave; k++) {
        uint32_t t = s_waves[k];
        if (k < w) before += t;
        all += t;
    }
    __syncthreads();
    if (total) *total = all;
    return before + inc - v;
}

__global__ __launch_bounds__(kThreads) void k_reduce(const uint32_t *__restrict__ in, int64_t n,
                                                     uint32_t *__restrict__ sums) {
    __shared__ uint32_t s_w[kThreads / kWave];
    int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kItems; k++) {
        int64_t i = base + k * kThreads + threadIdx.x;
        if (i < n) acc += in[i];
    }
    uint32_t tot;
    block_excl_scan(acc, s_w, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_top(uint32_t *__restrict__ sums, int64_t nb, uint32_t *total) {
    __shared__ uint32_t s_w[1024 / kWave];
    const int t = threadIdx.x;
    int64_t per = (nb + 1023) / 1024;
    int64_t b0 = t * per, b1 = b0 + per < nb ? b0 + per : nb;
    uint32_t acc = 0;
    for (int64_t b = b0; b < b1; b++) acc += sums[b];
    // block scan over 1024 threads (16 waves)
    const int lane = sfc_lane(), w = t / kWave;
    uint32_t inc = sfc_incl_scan(acc);
    if (lane == kWave - 1) s_w[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int k = 0; k < 1024 / kWave; k++) {
        uint32_t v = s_w[k];
        if (k < w) before += v;
        all += v;
    }
    uint32_t run = before + inc - acc;
    for (int64_t b = b0; b < b1; b++) {
        uint32_t v = sums[b];
        sums[b] = run;
        run += v;
    }
    if (t == 0 && total) *total = all;
}

__global__ __launch_bounds__(kThreads) void k_down(const uint32_t *in, uint32_t *out, int64_t n,
                                                   const uint32_t *__restrict__ sums) {
    __shared__ uint32_t s_w[kThreads / kWave];
    int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kItems; k++) {
        v[k] = (base + k < n) ? in[base + k] : 0u;
        acc += v[k];
    }
    uint32_t run = block_excl_scan(acc, s_w, nullptr) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kItems; k++) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

// The whole scan in one block for short arrays, in chunks of 32768 words
// staged through LDS: a coalesced load of the chunk, then thread t scans the
// contiguous run [32 t, 32 t + 32) (one padding word after every 32 keeps
// those runs on distinct banks), then a coalesced store; a carry joins the
// chunks (in == out works). With d_count the length is min(*d_count, n).
constexpr int kSmallThreads = 1024;
constexpr int kSmallPer = 32;
constexpr int64_t kSmallChunk = (int64_t)kSmallThreads * kSmallPer;
constexpr int64_t kSmallScan = 4 * kSmallChunk;  // longest static scan done by one block

__device__ __forceinline__ int small_slot(int i) { return i + (i >> 5); }

__global__ __launch_bounds__(kSmallThreads) void k_scan_small(const uint32_t *in, uint32_t *out, int64_t n,
                                                              const uint32_t *d_count, uint32_t *total) {
    __shared__ uint32_t s_v[kSmallChunk + kSmallChunk / kSmallPer];
    __shared__ uint32_t s_w[kSmallThreads / kWave];
    const int t = threadIdx.x;
    if (d_count) {
        const int64_t c = *d_count;
        n = c < n ? c : n;
    }
    const int lane = sfc_lane(), w = t / kWave;
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < n; c0 += kSmallChunk) {
        const int m = (int)(n - c0 < kSmallChunk ? n - c0 : kSmallChunk);
        // unconditional loads from a clamped index (m >= 1), eight in flight
        // together (more would spill); the select happens afterwards
#pragma unroll 1
        for (int g = 0; g < kSmallPer && g * kSmallThreads < m; g += 8) {
            uint32_t ld[8];
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const int i = (g + k) * kSmallThreads + t;
                ld[k] = in[c0 + (i < m ? i : m - 1)];
            }
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const int i = (g + k) * kSmallThreads + t;
                s_v[small_slot(i)] = i < m ? ld[k] : 0u;
            }
        }
        // groups past the end hold zeros
#pragma unroll 1
        for (int g = ((m + 8 * kSmallThreads - 1) / (8 * kSmallThreads)) * 8; g < kSmallPer; g += 8) {
#pragma unroll
            for (int k = 0; k < 8; k++) s_v[small_slot((g + k) * kSmallThreads + t)] = 0u;
        }
        __syncthreads();
        uint32_t acc = 0;
        const int b0 = t * kSmallPer;
#pragma unroll
        for (int k = 0; k < kSmallPer; k++) acc += s_v[small_slot(b0 + k)];
        const uint32_t inc = sfc_incl_scan(acc);
        if (lane == kWave - 1) s_w[w] = inc;
        __syncthreads();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int k = 0; k < kSmallThreads / kWave; k++) {
            const uint32_t v = s_w[k];
            if (k < w) before += v;
            all += v;
        }
        uint32_t run = carry + before + inc - acc;
#pragma unroll
        for (int k = 0; k < kSmallPer; k++) {
            const int q = small_slot(b0 + k);
            const uint32_t v = s_v[q];
            s_v[q] = run;
            run += v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSmallPer; k++) {
            const int i = k * kSmallThreads + t;
            if (i < m) out[c0 + i] = s_v[small_slot(i)];
        }
        carry += all;
        __syncthreads();  // the next chunk overwrites s_v and s_w
    }
    if (t == 0 && total) *total = carry;
}

// Fills of n words, four per thread: 16-byte stores where the array is
// 16-byte aligned (the host checks), the last ragged words one at a time.
__device__ __forceinline__ void fill4(uint32_t *p, int64_t n, int64_t i, uint32_t v, bool vec) {
    if (vec && i + 4 <= n) {
        *reinterpret_cast<uint4 *>(p + i) = make_uint4(v, v, v, v);
    } else {
        for (int64_t k = i; k < i + 4 && k < n; k++) p[k] = v;
    }
}

__global__ void k_fill(uint32_t *p, int64_t n, uint32_t v, bool vec) {
    const int64_t i = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) fill4(p, n, i, v, vec);
}

// Two arrays of n words at once (q may be null).
__global__ void k_fill2(uint32_t *p, uint32_t *q, int64_t n, uint32_t v, bool vec) {
    const int64_t i = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) {
        fill4(p, n, i, v, vec);
        if (q) fill4(q, n, i, v, vec);
    }
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) { return align_up((size_t)(blocks_for(n, kTile) + 1) * 4, 256); }

int scan_u32(sfcnl_ctx ctx, const uint32_t *in, uint32_t *out, int64_t n, uint32_t *d_total, void *tmp) {
    if (n <= 0) {
        if (d_total) return fill_u32(ctx, d_total, 1, 0);
        return SFCNL_OK;
    }
    if (n <= kSmallScan) {
        k_scan_small<<<1, kSmallThreads, 0, ctx->stream>>>(in, out, n, nullptr, d_total);
        SFCNL_LAUNCHED(ctx);
        return SFCNL_OK;
    }
    unsigned nb = blocks_for(n, kTile);
    uint32_t *sums = reinterpret_cast<uint32_t *>(tmp);
    // k_down reads its tile before writing, so in == out is allowed
    k_reduce<<<nb, kThreads, 0, ctx->stream>>>(in, n, sums);
    SFCNL_LAUNCHED(ctx);
    k_top<<<1, 1024, 0, ctx->stream>>>(sums, nb, d_total);
    SFCNL_LAUNCHED(ctx);
    k_down<<<nb, kThreads, 0, ctx->stream>>>(in, out, n, sums);
    SFCNL_LAUNCHED(ctx);
    return SFCNL_OK;
}

int scan_u32_dyn(sfcnl_ctx ctx, const uint32_t *in, uint32_t *out, const uint32_t *d_count, int64_t cap) {
    if (cap <= 0) return SFCNL_OK;
    k_scan_small<<<1, kSmallThreads, 0, ctx->stream>>>(in, out, cap, d_count, nullptr);
    SFCNL_LAUNCHED(ctx);
    return SFCNL_OK;
}

int fill_u32(sfcnl_ctx ctx, uint32_t *p, int64_t n, uint32_t v) {
    if (n <= 0) return SFCNL_OK;
    k_fill<<<blocks_for((n + 3) / 4, 256), 256, 0, ctx->stream>>>(p, n, v, ((uintptr_t)p & 15u) == 0);
    SFCNL_LAUNCHED(ctx);
    return SFCNL_OK;
}

int fill2_u32(sfcnl_ctx ctx, uint32_t *p, uint32_t *q, int64_t n, uint32_t v) {
    if (n <= 0) return SFCNL_OK;
    k_fill2<<<blocks_for((n + 3) / 4, 256), 256, 0, ctx->stream>>>(p, q, n, v, (((uintptr_t)p | (uintptr_t)q) & 15u) == 0);
    SFCNL_LAUNCHED(ctx);
    return SFCNL_OK;
}

}  // namespace sfcnl
