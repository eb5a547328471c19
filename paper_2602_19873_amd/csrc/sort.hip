// SFC order of the particles (Sec. II-A): 63-bit Hilbert keys, a stable LSD
// radix sort of (key, index), and the gather of particle fields.
#include <mutex>

#include "hilbert_table.h"
#include "internal.h"

namespace sfcnl {
namespace {

// ---------------------------------------------------------------------------
// Hilbert keys
// ---------------------------------------------------------------------------

// The key tables (hilbert_table.h) in device memory; each block that makes
// keys copies them into LDS, where the lanes' lookups land at random.
__device__ const hilbert::Tables kHilbertTables = hilbert::kTables;
constexpr int kHilbertWords = (int)(sizeof(hilbert::Tables) / 4);  // 16-bit entries, two per word

// Cooperative copy of the key tables into LDS (the caller synchronises).
__device__ __forceinline__ void hilbert_tables_to_lds(uint32_t *s_tab) {
    const uint32_t *g = reinterpret_cast<const uint32_t *>(&kHilbertTables);
    for (int i = (int)threadIdx.x; i < kHilbertWords; i += (int)blockDim.x) s_tab[i] = g[i];
}

// Hilbert key of a 21-bit cell (a0, a1, a2) from the tables in LDS: the top
// level from the start state, then the levels two at a time (11 lookups);
// digit k (axis 0 in its top bit) lands at key bits 3k .. 3k + 2.
__device__ __forceinline__ uint64_t hilbert_key(uint32_t a0, uint32_t a1, uint32_t a2, const uint32_t *s_tab) {
    const hilbert::Tables &T = *reinterpret_cast<const hilbert::Tables *>(s_tab);
    uint32_t e = T.start[((a0 >> 20) & 1u) << 2 | ((a1 >> 20) & 1u) << 1 | ((a2 >> 20) & 1u)];
    uint64_t key = e & 7u;
    uint32_t st = e >> 3;
#pragma unroll
    for (int k = 18; k >= 0; k -= 2) {
        const uint32_t o = __builtin_amdgcn_ubfe(a0, k, 2) << 4 | __builtin_amdgcn_ubfe(a1, k, 2) << 2 |
                           __builtin_amdgcn_ubfe(a2, k, 2);
        e = T.pair[st << 6 | o];
        key = key << 6 | (e & 63u);
        st = e >> 6;
    }
    return key;
}

__device__ __forceinline__ uint32_t quantise(float x, float lo, float s) {
    float t = x - lo;
    t = t * s;
    if (!(t > 0.0f)) return 0u;
    if (t >= 2097151.0f) return 2097151u;
    return (uint32_t)t;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits, 8 passes. Per pass: tile histograms,
// a scan over tiles per digit, and a scatter that ranks each tile stably in
// LDS before writing runs of equal digits out contiguously.
// ---------------------------------------------------------------------------

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;
constexpr int kWavesPerBlock = kThreads / kWave;
constexpr int kRadix = 256;
constexpr int kPasses = 8;

// System of input particle i: the last s with off[s] <= i (off has nsys + 1
// entries, off[0] = 0).
__device__ __forceinline__ uint32_t system_of(uint32_t i, const uint32_t *__restrict__ off, int nsys) {
    int lo = 0, hi = nsys;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return (uint32_t)lo;
}

// Digit of an element: 8 bits of its key, or (batched systems) 8 bits of the
// system its original index belongs to.
struct DigitOf {
    int shift;
    const uint32_t *sys_off;  // null: key digit
    int nsys;
    __device__ __forceinline__ uint32_t operator()(uint64_t key, uint32_t val) const {
        if (sys_off) return (system_of(val, sys_off, nsys) >> shift) & 255u;
        return (uint32_t)(key >> shift) & 255u;
    }
};

__global__ __launch_bounds__(kThreads) void k_hist(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                                                   int64_t n, DigitOf dg, uint32_t ntiles,
                                                   uint32_t *__restrict__ hist) {
    __shared__ uint32_t s_h[kRadix];
    const int t = threadIdx.x;
    s_h[t] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kTile;
    // unconditional loads from a clamped index, all in flight together
    uint32_t d[kItems];
    if (dg.sys_off) {
        uint32_t v[kItems];
#pragma unroll
        for (int k = 0; k < kItems; k++) {
            const int64_t i = base + k * kThreads + t;
            v[k] = vals[i < n ? i : n - 1];
        }
#pragma unroll
        for (int k = 0; k < kItems; k++) d[k] = dg(0ull, v[k]);
    } else {
        uint64_t kk[kItems];
#pragma unroll
        for (int k = 0; k < kItems; k++) {
            const int64_t i = base + k * kThreads + t;
            kk[k] = keys[i < n ? i : n - 1];
        }
#pragma unroll
        for (int k = 0; k < kItems; k++) d[k] = dg(kk[k], 0u);
    }
#pragma unroll
    for (int k = 0; k < kItems; k++)
        if (base + k * kThreads + t < n) atomicAdd(&s_h[d[k]], 1u);
    __syncthreads();
    hist[(size_t)t * ntiles + blockIdx.x] = s_h[t];
}

// One block per digit: exclusive scan of hist[d][0..ntiles) in place.
__global__ __launch_bounds__(kThreads) void k_digit_scan(uint32_t *__restrict__ hist, uint32_t ntiles,
                                                         uint32_t *__restrict__ digit_tot) {
    __shared__ uint32_t s_w[kWavesPerBlock];
    uint32_t *row = hist + (size_t)blockIdx.x * ntiles;
    const int t = threadIdx.x, lane = sfc_lane(), w = t / kWave;
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < ntiles; c0 += kThreads * 4) {
        uint32_t v[4], acc = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            uint32_t i = c0 + t * 4 + k;
            v[k] = i < ntiles ? row[i] : 0u;
            acc += v[k];
        }
        uint32_t inc = sfc_incl_scan(acc);
        if (lane == kWave - 1) s_w[w] = inc;
        __syncthreads();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int k = 0; k < kWavesPerBlock; k++) {
            if (k < w) before += s_w[k];
            all += s_w[k];
        }
        __syncthreads();
        uint32_t run = carry + before + inc - acc;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            uint32_t i = c0 + t * 4 + k;
            if (i < ntiles) row[i] = run;
            run += v[k];
        }
        carry += all;
    }
    if (t == 0) digit_tot[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kThreads) void k_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                      uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                      int64_t n, DigitOf dg, uint32_t ntiles,
                                                      const uint32_t *__restrict__ hist,
                                                      const uint32_t *__restrict__ digit_tot) {
    __shared__ uint64_t s_keys[kTile];
    __shared__ uint32_t s_vals[kTile];
    __shared__ uint32_t s_cnt[kWavesPerBlock][kRadix];
    __shared__ uint32_t s_gbase[kRadix];
    __shared__ uint32_t s_w[2][kWavesPerBlock];

    const int t = threadIdx.x, lane = sfc_lane(), w = t / kWave;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int tile_n = (int)((n - base) < kTile ? (n - base) : kTile);

#pragma unroll
    for (int k = 0; k < kWavesPerBlock; k++) s_cnt[k][t] = 0;
    __syncthreads();

    uint64_t key[kItems];
    uint32_t val[kItems], lrank[kItems];
    const uint64_t lt = sfc_lt_mask();
    // unconditional loads from a clamped index (tile_n >= 1), all in flight
    // together
#pragma unroll
    for (int k = 0; k < kItems; k++) {
        const int li = w * (kItems * kWave) + k * kWave + lane;  // striped: wave, item, lane
        const int lc = li < tile_n ? li : tile_n - 1;
        key[k] = kin[base + lc];
        val[k] = vin[base + lc];
    }
#pragma unroll
    for (int k = 0; k < kItems; k++) {
        int li = w * (kItems * kWave) + k * kWave + lane;  // striped: wave, item, lane
        bool valid = li < tile_n;
        uint32_t d = valid ? dg(key[k], val[k]) : 0u;
        uint64_t m = sfc_ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            bool bit = (d >> b) & 1u;
            uint64_t bb = sfc_ballot(valid && bit);
            m &= bit ? bb : ~bb;
        }
        uint32_t r = (uint32_t)sfc_popc(m & lt);
        uint32_t before = valid ? s_cnt[w][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        lrank[k] = before + r;
        if (valid && r == 0) s_cnt[w][d] = before + (uint32_t)sfc_popc(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // per digit t: prefix over waves, then the tile-local start of digit t
    uint32_t c[kWavesPerBlock], tot = 0;
#pragma unroll
    for (int k = 0; k < kWavesPerBlock; k++) {
        c[k] = s_cnt[k][t];
        tot += c[k];
    }
    uint32_t dt = digit_tot[t];
    uint32_t inc_tile = sfc_incl_scan(tot);
    uint32_t inc_glob = sfc_incl_scan(dt);
    if (lane == kWave - 1) {
        s_w[0][w] = inc_tile;
        s_w[1][w] = inc_glob;
    }
    __syncthreads();
    uint32_t tile_start = inc_tile - tot, glob_start = inc_glob - dt;
    for (int k = 0; k < w; k++) {
        tile_start += s_w[0][k];
        glob_start += s_w[1][k];
    }
    uint32_t run = tile_start;
#pragma unroll
    for (int k = 0; k < kWavesPerBlock; k++) {
        s_cnt[k][t] = run;
        run += c[k];
    }
    s_gbase[t] = glob_start + hist[(size_t)t * ntiles + blockIdx.x] - tile_start;
    __syncthreads();

#pragma unroll
    for (int k = 0; k < kItems; k++) {
        int li = w * (kItems * kWave) + k * kWave + lane;
        if (li < tile_n) {
            uint32_t d = dg(key[k], val[k]);
            uint32_t lp = s_cnt[w][d] + lrank[k];
            s_keys[lp] = key[k];
            s_vals[lp] = val[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; k++) {
        int lp = k * kThreads + t;
        if (lp < tile_n) {
            uint64_t kk = s_keys[lp];
            uint32_t vv = s_vals[lp];
            uint32_t d = dg(kk, vv);
            uint32_t gp = s_gbase[d] + (uint32_t)lp;
            kout[gp] = kk;
            vout[gp] = vv;
        }
    }
}

// ---------------------------------------------------------------------------
// Sort of one system. Three stable counting passes order the particles by the
// top 24 key bits (digit bits 39..46, 47..54, 55..62; the keys kernel also
// builds the first pass's tile histograms), which leaves runs of equal 24-bit
// prefixes in input order -- mostly single particles, as a prefix is a cell
// of octree level 8. One more kernel then sorts every longer run by the whole
// key, stably: block b takes the runs that begin in particles [b T, b T + T)
// (the last of them may extend past that range). The result is the stable
// order by the full key, as eight 8-bit passes would give, in ten launches
// instead of twenty-five. A run too long for LDS is sorted by one block in
// passes through global memory.
// ---------------------------------------------------------------------------

constexpr int kPreShift = 39;      // the runs share key bits 39..62
constexpr int kLocTile = 2048;     // run starts handled per block
constexpr int kLocCap = 2048;      // longest range sorted in LDS
constexpr int kLocItems = kLocCap / kThreads;  // 8 per thread
constexpr int kRankRun = 64;       // runs up to this length are placed by counting

__device__ __forceinline__ uint64_t key_prefix(uint64_t k) { return k >> kPreShift; }

// Keys and indices as k_keys, plus the tile histograms of key bits 39..46
// (a tile of kTile particles per block of 1024 threads, two each).
constexpr int kKeysThreads = 1024;
constexpr int kKeysItems = kTile / kKeysThreads;

__global__ __launch_bounds__(kKeysThreads) void k_keys_hist(int64_t n, const float *__restrict__ x,
                                                            const float *__restrict__ y, const float *__restrict__ z,
                                                            float lox, float sx, float loy, float sy, float loz,
                                                            float sz, uint64_t *__restrict__ keys,
                                                            uint32_t *__restrict__ idx, uint32_t ntiles,
                                                            uint32_t *__restrict__ hist, uint32_t *status) {
    __shared__ uint32_t s_h[kRadix];
    __shared__ uint32_t s_tab[kHilbertWords];
    const int t = threadIdx.x;
    if (t < kRadix) s_h[t] = 0;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    float px[kKeysItems], py[kKeysItems], pz[kKeysItems];
#pragma unroll
    for (int k = 0; k < kKeysItems; k++) {
        const int64_t i = base + k * kKeysThreads + t;
        const int64_t ic = i < n ? i : n - 1;
        px[k] = x[ic];
        py[k] = y[ic];
        pz[k] = z[ic];
    }
    hilbert_tables_to_lds(s_tab);
    __syncthreads();
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kKeysItems; k++) {
        const int64_t i = base + k * kKeysThreads + t;
        if (i < n) {
            if (!(isfinite(px[k]) && isfinite(py[k]) && isfinite(pz[k]))) bad = true;
            const uint64_t key =
                hilbert_key(quantise(px[k], lox, sx), quantise(py[k], loy, sy), quantise(pz[k], loz, sz), s_tab);
            keys[i] = key;
            idx[i] = (uint32_t)i;
            atomicAdd(&s_h[(uint32_t)(key >> kPreShift) & 255u], 1u);
        }
    }
    if (bad) atomicOr(&status[kStInputErr], 1u);
    __syncthreads();
    if (t < kRadix) hist[(size_t)t * ntiles + blockIdx.x] = s_h[t];
}

// Stable LSD sort of m <= kLocCap (key, value) pairs held in LDS by bits
// [0, hb] of the key, 8 bits per pass, with the 256 threads of the block.
// Element e sits in wave e / 1024, step e / 64 % 16, lane e % 64, so ranking
// the steps in order and the waves in order keeps equal digits in place.
__device__ __forceinline__ void lds_radix(uint64_t *sk, uint32_t *sv, int m, int hb, uint32_t (*s_cnt)[kRadix], uint32_t *s_w) {
    const int t = threadIdx.x, lane = sfc_lane(), w = t / kWave;
    const uint64_t lt = sfc_lt_mask();
    for (int lo = 0; lo <= hb; lo += 8) {
#pragma unroll
        for (int k = 0; k < kWavesPerBlock; k++) s_cnt[k][t] = 0;
        uint64_t key[kLocItems];
        uint32_t val[kLocItems], lrank[kLocItems];
#pragma unroll
        for (int k = 0; k < kLocItems; k++) {
            const int e = w * (kLocItems * kWave) + k * kWave + lane;
            const int ec = e < m ? e : m - 1;
            key[k] = sk[ec];
            val[k] = sv[ec];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kLocItems; k++) {
            const int e = w * (kLocItems * kWave) + k * kWave + lane;
            const bool valid = e < m;
            const uint32_t d = (uint32_t)(key[k] >> lo) & 255u;
            uint64_t mm = sfc_ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; b++) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = sfc_ballot(valid && bit);
                mm &= bit ? bb : ~bb;
            }
            const uint32_t r = (uint32_t)sfc_popc(mm & lt);
            const uint32_t before = valid ? s_cnt[w][d] : 0u;
            __builtin_amdgcn_wave_barrier();
            lrank[k] = before + r;
            if (valid && r == 0) s_cnt[w][d] = before + (uint32_t)sfc_popc(mm);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        // digit t: its start over the block, then each wave's start inside it
        uint32_t c[kWavesPerBlock], tot = 0;
#pragma unroll
        for (int k = 0; k < kWavesPerBlock; k++) {
            c[k] = s_cnt[k][t];
            tot += c[k];
        }
        const uint32_t inc = sfc_incl_scan(tot);
        if (lane == kWave - 1) s_w[w] = inc;
        __syncthreads();
        uint32_t run = inc - tot;
        for (int k = 0; k < w; k++) run += s_w[k];
#pragma unroll
        for (int k = 0; k < kWavesPerBlock; k++) {
            s_cnt[k][t] = run;
            run += c[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kLocItems; k++) {
            const int e = w * (kLocItems * kWave) + k * kWave + lane;
            if (e < m) {
                const uint32_t d = (uint32_t)(key[k] >> lo) & 255u;
                const uint32_t q = s_cnt[w][d] + lrank[k];
                sk[q] = key[k];
                sv[q] = val[k];
            }
        }
        __syncthreads();
    }
}

// Highest bit in which the keys of [r0, r1) differ (-1 if all are equal),
// over the whole block (s_or: one LDS word pair).
__device__ __forceinline__ int range_diff_bit(const uint64_t *__restrict__ keys, int64_t r0, int64_t r1, unsigned long long *s_or) {
    const uint64_t k0 = keys[r0];
    uint64_t acc = 0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kThreads) acc |= keys[i] ^ k0;
    if (threadIdx.x == 0) *s_or = 0ull;
    __syncthreads();
    if (acc) atomicOr(s_or, (unsigned long long)acc);
    __syncthreads();
    const uint64_t all = *s_or;
    __syncthreads();
    return all ? 63 - __clzll((long long)all) : -1;
}

// Sorts [r0, r1) (whole runs, at most kLocCap pairs) by the full key in LDS.
// Runs of up to kRankRun pairs (the common case) are placed by counting:
// each pair finds its run in LDS and its place in it from the smaller keys
// and the equal keys before it (which keeps equal keys in input order), and
// only pairs of runs longer than one are written; all reads come from LDS,
// so those global writes race with nothing. A range holding a longer run is
// sorted by the LDS radix passes instead.
__device__ __forceinline__ void sort_range_lds(uint64_t *__restrict__ keys, uint32_t *__restrict__ vals, int64_t r0,
                                               int64_t r1, uint64_t *sk, uint32_t *sv, uint32_t (*s_cnt)[kRadix],
                                               uint32_t *s_w, unsigned long long *s_or) {
    const int m = (int)(r1 - r0);
    if (m < 2) return;
    const int t = threadIdx.x;
    {
        // unconditional loads from a clamped index, all in flight together
        uint64_t lk[kLocItems];
        uint32_t lv[kLocItems];
#pragma unroll
        for (int k = 0; k < kLocItems; k++) {
            const int e = k * kThreads + t;
            const int ec = e < m ? e : m - 1;
            lk[k] = keys[r0 + ec];
            lv[k] = vals[r0 + ec];
        }
#pragma unroll
        for (int k = 0; k < kLocItems; k++) {
            const int e = k * kThreads + t;
            if (e < m) {
                sk[e] = lk[k];
                sv[e] = lv[k];
            }
        }
    }
    __syncthreads();
    int ra[kLocItems], rb[kLocItems];
    bool longrun = false;
#pragma unroll
    for (int k = 0; k < kLocItems; k++) {
        const int e = k * kThreads + t;
        int a = e, b = e + 1;
        if (e < m) {
            const uint64_t p = key_prefix(sk[e]);
            while (a > 0 && e - a < kRankRun && key_prefix(sk[a - 1]) == p) a--;
            while (b < m && b - e <= kRankRun && key_prefix(sk[b]) == p) b++;
        }
        ra[k] = a;
        rb[k] = b;
        if (b - a > kRankRun) longrun = true;
    }
    if (__syncthreads_or(longrun)) {
        const int hb = range_diff_bit(keys, r0, r1, s_or);
        if (hb < 0) return;  // equal keys: input order is already the order
        lds_radix(sk, sv, m, hb, s_cnt, s_w);
        for (int e = t; e < m; e += kThreads) {
            keys[r0 + e] = sk[e];
            vals[r0 + e] = sv[e];
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < kLocItems; k++) {
        const int e = k * kThreads + t;
        const int a = ra[k], b = rb[k];
        if (e >= m || b - a == 1) continue;  // a run of one stays where it is
        const uint64_t key = sk[e];
        int r = 0;
        for (int q = a; q < b; q++) {
            const uint64_t kq = sk[q];
            r += (kq < key || (kq == key && q < e)) ? 1 : 0;
        }
        keys[r0 + a + r] = key;
        vals[r0 + a + r] = sv[e];
    }
}

// Sorts one long run [r0, r1) (equal prefixes, so bits below 47 decide) by one
// block in stable 8-bit passes through global memory, ping-ponging with the
// same range of (tk, tv); tiles of kLocCap pairs are ranked in LDS in order.
__device__ __forceinline__ void sort_range_stream(uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                  uint64_t *__restrict__ tk, uint32_t *__restrict__ tv, int64_t r0, int64_t r1,
                                  uint32_t (*s_cnt)[kRadix], uint32_t *s_w, uint32_t *s_run,
                                  unsigned long long *s_or) {
    const int t = threadIdx.x, lane = sfc_lane(), w = t / kWave;
    const uint64_t lt = sfc_lt_mask();
    const int hb = range_diff_bit(keys, r0, r1, s_or);
    if (hb < 0) return;
    uint64_t *ka = keys, *kb = tk;
    uint32_t *va = vals, *vb = tv;
    int npass = 0;
    for (int lo = 0; lo <= hb; lo += 8, npass++) {
        // digit totals over the run, then running starts
        s_run[t] = 0;
        __syncthreads();
        for (int64_t i = r0 + t; i < r1; i += kThreads) atomicAdd(&s_run[(uint32_t)(ka[i] >> lo) & 255u], 1u);
        __syncthreads();
        {
            const uint32_t v = s_run[t];
            const uint32_t inc = sfc_incl_scan(v);
            if (lane == kWave - 1) s_w[w] = inc;
            __syncthreads();
            uint32_t ex = inc - v;
            for (int k = 0; k < w; k++) ex += s_w[k];
            __syncthreads();
            s_run[t] = ex;
        }
        for (int64_t c0 = r0; c0 < r1; c0 += kLocCap) {
            const int m = (int)(r1 - c0 < kLocCap ? r1 - c0 : kLocCap);
#pragma unroll
            for (int k = 0; k < kWavesPerBlock; k++) s_cnt[k][t] = 0;
            __syncthreads();
            uint64_t key[kLocItems];
            uint32_t val[kLocItems], lrank[kLocItems];
#pragma unroll
            for (int k = 0; k < kLocItems; k++) {
                const int e = w * (kLocItems * kWave) + k * kWave + lane;
                const int ec = e < m ? e : m - 1;
                key[k] = ka[c0 + ec];
                val[k] = va[c0 + ec];
            }
#pragma unroll
            for (int k = 0; k < kLocItems; k++) {
                const int e = w * (kLocItems * kWave) + k * kWave + lane;
                const bool valid = e < m;
                const uint32_t d = (uint32_t)(key[k] >> lo) & 255u;
                uint64_t mm = sfc_ballot(valid);
#pragma unroll
                for (int b = 0; b < 8; b++) {
                    const bool bit = (d >> b) & 1u;
                    const uint64_t bb = sfc_ballot(valid && bit);
                    mm &= bit ? bb : ~bb;
                }
                const uint32_t r = (uint32_t)sfc_popc(mm & lt);
                const uint32_t before = valid ? s_cnt[w][d] : 0u;
                __builtin_amdgcn_wave_barrier();
                lrank[k] = before + r;
                if (valid && r == 0) s_cnt[w][d] = before + (uint32_t)sfc_popc(mm);
                __builtin_amdgcn_wave_barrier();
            }
            __syncthreads();
            // digit t: the running start, then each wave's start inside the tile
            uint32_t c[kWavesPerBlock], tot = 0;
#pragma unroll
            for (int k = 0; k < kWavesPerBlock; k++) {
                c[k] = s_cnt[k][t];
                tot += c[k];
            }
            uint32_t run = s_run[t];
#pragma unroll
            for (int k = 0; k < kWavesPerBlock; k++) {
                s_cnt[k][t] = run;
                run += c[k];
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kLocItems; k++) {
                const int e = w * (kLocItems * kWave) + k * kWave + lane;
                if (e < m) {
                    const uint32_t d = (uint32_t)(key[k] >> lo) & 255u;
                    const int64_t q = r0 + s_cnt[w][d] + lrank[k];
                    kb[q] = key[k];
                    vb[q] = val[k];
                }
            }
            __syncthreads();
            s_run[t] += tot;
            __syncthreads();
        }
        uint64_t *tk2 = ka;
        ka = kb;
        kb = tk2;
        uint32_t *tv2 = va;
        va = vb;
        vb = tv2;
        // the next pass reads what this one wrote (other threads' stores):
        // a device-scope fence, so that no stale line of the vector cache
        // serves those reads
        __threadfence();
        __syncthreads();
    }
    if (npass & 1) {  // the result is in the temporary range: copy it back
        for (int64_t i = r0 + t; i < r1; i += kThreads) {
            keys[i] = tk[i];
            vals[i] = tv[i];
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_local_sort(uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                         uint64_t *__restrict__ tk, uint32_t *__restrict__ tv,
                                                         int64_t n) {
    __shared__ uint64_t sk[kLocCap];
    __shared__ uint32_t sv[kLocCap];
    __shared__ uint32_t s_cnt[kWavesPerBlock][kRadix];
    __shared__ uint32_t s_run[kRadix];
    __shared__ uint32_t s_w[kWavesPerBlock];
    __shared__ unsigned long long s_or;
    __shared__ uint32_t s_first, s_last, s_end;
    const int t = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * kLocTile;
    if (b0 >= n) return;
    const int64_t b1 = b0 + kLocTile < n ? b0 + kLocTile : n;
    if (t == 0) {
        s_first = 0xFFFFFFFFu;
        s_last = 0u;
        s_end = (uint32_t)b1;
    }
    __syncthreads();
    // the runs that begin in [b0, b1): the first and the last of them (keys
    // and their predecessors loaded unconditionally from clamped indices, all
    // in flight together; one LDS atomic per wave)
    {
        uint64_t kc[kLocTile / kThreads], kp[kLocTile / kThreads];
#pragma unroll
        for (int k = 0; k < kLocTile / kThreads; k++) {
            const int64_t i = b0 + k * kThreads + t;
            const int64_t ic = i < b1 ? i : b1 - 1;
            kc[k] = keys[ic];
            kp[k] = keys[ic > 0 ? ic - 1 : 0];
        }
        uint32_t first = 0xFFFFFFFFu, last = 0u;
#pragma unroll
        for (int k = 0; k < kLocTile / kThreads; k++) {
            const int64_t i = b0 + k * kThreads + t;
            const bool start = i < b1 && (i == 0 || key_prefix(kc[k]) != key_prefix(kp[k]));
            const uint64_t bal = sfc_ballot(start);
            if (bal) {
                const int64_t wbase = b0 + k * kThreads + (t & ~(kWave - 1));
                first = min(first, (uint32_t)(wbase + __ffsll((long long)bal) - 1));
                last = max(last, (uint32_t)(wbase + 63 - __clzll((long long)bal)));
            }
        }
        if (sfc_lane() == 0) {
            if (first != 0xFFFFFFFFu) atomicMin(&s_first, first);
            atomicMax(&s_last, last);
        }
    }
    // the last run ends at the first key past b1 - 1 with a larger prefix:
    // the first wave looks 64 keys at a time (runs are short but for
    // clustered inputs)
    if (t < kWave && b1 < n) {
        const uint64_t p = key_prefix(keys[b1 - 1]);
        for (int64_t c0 = b1; c0 < n; c0 += kWave) {
            const int64_t i = c0 + t;
            const uint64_t diff = sfc_ballot(i < n && key_prefix(keys[i < n ? i : n - 1]) != p);
            if (diff) {
                if (t == 0) s_end = (uint32_t)(c0 + __ffsll((long long)diff) - 1);
                break;
            }
            if (c0 + kWave >= n && t == 0) s_end = (uint32_t)n;
        }
    }
    __syncthreads();
    if (s_first == 0xFFFFFFFFu) return;  // inside a run that began in an earlier block
    const int64_t r0 = s_first, rl = s_last, r1 = s_end;
    if (r1 - r0 <= kLocCap) {
        sort_range_lds(keys, vals, r0, r1, sk, sv, s_cnt, s_w, &s_or);
        return;
    }
    // too long for LDS: the runs before the last one (fewer than kLocTile
    // pairs), then the last run alone
    sort_range_lds(keys, vals, r0, rl, sk, sv, s_cnt, s_w, &s_or);
    __syncthreads();
    if (r1 - rl <= kLocCap)
        sort_range_lds(keys, vals, rl, r1, sk, sv, s_cnt, s_w, &s_or);
    else
        sort_range_stream(keys, vals, tk, tv, rl, r1, s_cnt, s_w, s_run, &s_or);
}

struct GatherArgs {
    const float *in[8];
    float *out[8];
    int nf;
};

// out[f][i] = in[f][perm[i]] for i < n_out, perm[i] < n_in; with `pad`, the
// index 0xFFFFFFFF marks a padding slot that gets NaN.
__global__ __launch_bounds__(256) void k_gather(int64_t n_out, int64_t n_in, const uint32_t *__restrict__ perm,
                                                GatherArgs a, bool pad, uint32_t *status) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    uint32_t p = perm[i];
    if (pad && p == 0xFFFFFFFFu) {
#pragma unroll
        for (int f = 0; f < 8; f++)
            if (f < a.nf) a.out[f][i] = __builtin_nanf("");
        return;
    }
    if (p >= (uint64_t)n_in) {  // not a permutation of [0, n): report, never read outside
        atomicOr(&status[kStInputErr], 4u);
        p = 0;
    }
#pragma unroll
    for (int f = 0; f < 8; f++)
        if (f < a.nf) a.out[f][i] = a.in[f][p];
}

// Staged gather: up to four fields packed into 16-byte records in input order
// (coalesced), then one random 16-byte read per particle instead of one per
// field.
struct Pack4 {
    const float *in[4];
    float *out[4];
    int nf;
};

__global__ __launch_bounds__(256) void k_pack4(int64_t n, Pack4 a, float4 *__restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float4 r;
    r.x = a.in[0][i];
    r.y = a.nf > 1 ? a.in[1][i] : 0.0f;
    r.z = a.nf > 2 ? a.in[2][i] : 0.0f;
    r.w = a.nf > 3 ? a.in[3][i] : 0.0f;
    rec[i] = r;
}

__global__ __launch_bounds__(256) void k_gather4(int64_t n, const uint32_t *__restrict__ perm,
                                                 const float4 *__restrict__ rec, Pack4 a, uint32_t *status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t p = perm[i];
    if (p >= (uint64_t)n) {  // not a permutation of [0, n): report, never read outside
        atomicOr(&status[kStInputErr], 4u);
        p = 0;
    }
    const float4 r = rec[p];
    a.out[0][i] = r.x;
    if (a.nf > 1) a.out[1][i] = r.y;
    if (a.nf > 2) a.out[2][i] = r.z;
    if (a.nf > 3) a.out[3][i] = r.w;
}

// Keys of batched systems: particle i of the concatenated input uses its own
// system's box.
__global__ __launch_bounds__(256) void k_batch_keys(int64_t n, const float *__restrict__ x,
                                                    const float *__restrict__ y, const float *__restrict__ z,
                                                    const uint32_t *__restrict__ in_off, int nsys,
                                                    const float *__restrict__ lo, const float *__restrict__ sc,
                                                    uint64_t *__restrict__ keys, uint32_t *__restrict__ idx,
                                                    uint32_t *status) {
    __shared__ uint32_t s_tab[kHilbertWords];
    hilbert_tables_to_lds(s_tab);
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t sy = system_of((uint32_t)i, in_off, nsys);
    float px = x[i], py = y[i], pz = z[i];
    if (!(isfinite(px) && isfinite(py) && isfinite(pz))) atomicOr(&status[kStInputErr], 1u);
    keys[i] = hilbert_key(quantise(px, lo[3 * sy], sc[3 * sy]), quantise(py, lo[3 * sy + 1], sc[3 * sy + 1]),
                          quantise(pz, lo[3 * sy + 2], sc[3 * sy + 2]), s_tab);
    idx[i] = (uint32_t)i;
}

// Spreads the (system, key)-sorted input into the padded layout: slot q of
// system s holds its (q - pbase[s])-th particle, or padding (key all ones,
// index 0xFFFFFFFF).
__global__ __launch_bounds__(256) void k_batch_pad(int64_t n_pad, const uint64_t *__restrict__ ks,
                                                   const uint32_t *__restrict__ vs, SegTable seg,
                                                   const uint32_t *__restrict__ in_off, uint64_t *__restrict__ keys,
                                                   uint32_t *__restrict__ perm) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_pad) return;
    const int sy = seg.sc_sys[q / kScSize];
    const uint32_t local = (uint32_t)q - seg.pbase[sy];
    if (local < seg.count[sy]) {
        keys[q] = ks[in_off[sy] + local];
        perm[q] = vs[in_off[sy] + local];
    } else {
        keys[q] = ~0ull;
        perm[q] = 0xFFFFFFFFu;
    }
}

struct SortWs {
    uint64_t *ktmp;
    uint32_t *vtmp;
    uint32_t *hist;
    uint32_t *dtot;
};

size_t carve_sort(Carver &cv, SortWs &s, int64_t n) {
    uint32_t ntiles = blocks_for(n, kTile);
    s.ktmp = cv.take<uint64_t>((size_t)n);
    s.vtmp = cv.take<uint32_t>((size_t)n);
    s.hist = cv.take<uint32_t>((size_t)kRadix * ntiles);
    s.dtot = cv.take<uint32_t>(kRadix);
    return cv.used;
}

// One stable counting pass: (ka, va) -> (kb, vb) by the digit dg.
int radix_pass(sfcnl_ctx ctx, const SortWs &s, const uint64_t *ka, const uint32_t *va, uint64_t *kb, uint32_t *vb,
               int64_t n, DigitOf dg) {
    hipStream_t st = ctx->stream;
    const uint32_t ntiles = blocks_for(n, kTile);
    k_hist<<<ntiles, kThreads, 0, st>>>(ka, va, n, dg, ntiles, s.hist);
    SFCNL_LAUNCHED(ctx);
    k_digit_scan<<<kRadix, kThreads, 0, st>>>(s.hist, ntiles, s.dtot);
    SFCNL_LAUNCHED(ctx);
    k_scatter<<<ntiles, kThreads, 0, st>>>(ka, va, kb, vb, n, dg, ntiles, s.hist, s.dtot);
    SFCNL_LAUNCHED(ctx);
    return SFCNL_OK;
}

float box_scale(float lo, float hi) { return (float)(2097152.0 / ((double)hi - (double)lo)); }

}  // namespace
}  // namespace sfcnl

using namespace sfcnl;

extern "C" int sfc_sort_workspace(int64_t n, size_t *ws_bytes) {
    if (n < 0 || !ws_bytes) return SFCNL_E_ARG;
    Carver cv{nullptr, 0};
    SortWs s;
    *ws_bytes = align_up(carve_sort(cv, s, n), 256) + 256;
    return SFCNL_OK;
}

namespace sfcnl {
namespace {

// Keys and the radix passes over a workspace already checked to be large
// enough (sfc_sort_workspace(n) bytes at d_ws).
int sort_impl(sfcnl_ctx ctx, int64_t n, const float *d_x, const float *d_y, const float *d_z, const float *h_box,
              uint64_t *d_keys_out, uint32_t *d_perm_out, void *d_ws) {
    Carver cv{reinterpret_cast<char *>(d_ws), 0};
    SortWs s;
    carve_sort(cv, s, n);

    hipStream_t st = ctx->stream;
    const uint32_t ntiles = blocks_for(n, kTile);
    // keys (into the temporary buffers) with the first pass's tile histograms
    prof_mark(ctx, kStageKeys, false);
    k_keys_hist<<<ntiles, kKeysThreads, 0, st>>>(n, d_x, d_y, d_z, h_box[0], box_scale(h_box[0], h_box[1]), h_box[2],
                                                 box_scale(h_box[2], h_box[3]), h_box[4], box_scale(h_box[4], h_box[5]),
                                                 s.ktmp, s.vtmp, ntiles, s.hist, ctx->d_status);
    SFCNL_LAUNCHED(ctx);
    prof_mark(ctx, kStageKeys, true);
    prof_mark(ctx, kStageSort, false);
    // stable passes on key bits 39..46, 47..54, 55..62 (the last into the outputs)
    const DigitOf d0{kPreShift, nullptr, 0}, d1{kPreShift + 8, nullptr, 0}, d2{kPreShift + 16, nullptr, 0};
    k_digit_scan<<<kRadix, kThreads, 0, st>>>(s.hist, ntiles, s.dtot);
    SFCNL_LAUNCHED(ctx);
    k_scatter<<<ntiles, kThreads, 0, st>>>(s.ktmp, s.vtmp, d_keys_out, d_perm_out, n, d0, ntiles, s.hist, s.dtot);
    SFCNL_LAUNCHED(ctx);
    int rc = radix_pass(ctx, s, d_keys_out, d_perm_out, s.ktmp, s.vtmp, n, d1);
    if (rc) return rc;
    rc = radix_pass(ctx, s, s.ktmp, s.vtmp, d_keys_out, d_perm_out, n, d2);
    if (rc) return rc;
    // every run of equal 24-bit prefixes by the full key
    k_local_sort<<<blocks_for(n, kLocTile), kThreads, 0, st>>>(d_keys_out, d_perm_out, s.ktmp, s.vtmp, n);
    SFCNL_LAUNCHED(ctx);
    prof_mark(ctx, kStageSort, true);
    return SFCNL_OK;
}

int sort_args(sfcnl_ctx ctx, const char *fn, int64_t n, const float *d_x, const float *d_y, const float *d_z,
              const float *h_box, uint64_t *d_keys_out, uint32_t *d_perm_out) {
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "%s: n=%lld out of range", fn, (long long)n);
    if (n == 0) return SFCNL_OK;
    if (!d_x || !d_y || !d_z || !h_box || !d_keys_out || !d_perm_out)
        return set_err(ctx, SFCNL_E_ARG, "%s: null pointer", fn);
    for (int a = 0; a < 3; a++)
        if (!(h_box[2 * a + 1] > h_box[2 * a]) || !__builtin_isfinite(h_box[2 * a]) || !__builtin_isfinite(h_box[2 * a + 1]))
            return set_err(ctx, SFCNL_E_ARG, "%s: box axis %d empty or not finite", fn, a);
    return SFCNL_OK;
}

// Workspace of sfc_sort_noalloc: the sort workspace at the largest n it
// accepts (the carve's sizes with its 256-byte alignment), in a fixed array.
constexpr size_t ws_bound(int64_t n) {
    const size_t ntiles = (size_t)((n + kTile - 1) / kTile);
    return 256 + align_up((size_t)n * 8, 256) + align_up((size_t)n * 4, 256) + align_up(kRadix * ntiles * 4, 256) +
           align_up(kRadix * 4, 256) + 256;
}
constexpr size_t kScratchBytes = ws_bound(SFCNL_SORT_NOALLOC_MAX_N);
static __device__ __align__(256) char scratch[kScratchBytes];

// Device address of `scratch` per device ordinal (each GPU holds its own copy
// of the array); looked up once per device, with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

}  // namespace
}  // namespace sfcnl

int sfcnl::sort_scratch_setup(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return SFCNL_E_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SFCNL_E_HIP;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return SFCNL_OK;
}

extern "C" int sfc_sort(sfcnl_ctx ctx, int64_t n, const float *d_x, const float *d_y, const float *d_z,
                        const float *h_box, uint64_t *d_keys_out, uint32_t *d_perm_out, void *d_ws,
                        size_t ws_bytes) {
    if (!ctx) return SFCNL_E_ARG;
    int rc = sort_args(ctx, "sfc_sort", n, d_x, d_y, d_z, h_box, d_keys_out, d_perm_out);
    if (rc || n == 0) return rc;
    if (!d_ws) return set_err(ctx, SFCNL_E_ARG, "sfc_sort: null workspace");
    size_t need;
    sfc_sort_workspace(n, &need);
    if (ws_bytes < need)
        return set_err(ctx, SFCNL_E_ARG, "sfc_sort: workspace %zu bytes < %zu needed", ws_bytes, need);
    return sort_impl(ctx, n, d_x, d_y, d_z, h_box, d_keys_out, d_perm_out, d_ws);
}

extern "C" int sfc_sort_noalloc(sfcnl_ctx ctx, int64_t n, const float *d_x, const float *d_y, const float *d_z,
                                const float *h_box, uint64_t *d_keys_out, uint32_t *d_perm_out) {
    if (!ctx) return SFCNL_E_ARG;
    if (n > SFCNL_SORT_NOALLOC_MAX_N)
        return set_err(ctx, SFCNL_E_ARG, "sfc_sort_noalloc: n=%lld above the maximum %d of its fixed scratch",
                       (long long)n, SFCNL_SORT_NOALLOC_MAX_N);
    int rc = sort_args(ctx, "sfc_sort_noalloc", n, d_x, d_y, d_z, h_box, d_keys_out, d_perm_out);
    if (rc || n == 0) return rc;
    if (!ctx->d_sort_scratch) return set_err(ctx, SFCNL_E_HIP, "sfc_sort_noalloc: scratch array not located");
    size_t need;
    sfc_sort_workspace(n, &need);
    if (need > kScratchBytes)  // cannot happen for n within the maximum
        return set_err(ctx, SFCNL_E_ARG, "sfc_sort_noalloc: needs %zu bytes > %zu", need, kScratchBytes);
    return sort_impl(ctx, n, d_x, d_y, d_z, h_box, d_keys_out, d_perm_out, ctx->d_sort_scratch);
}

extern "C" int sfc_gather(sfcnl_ctx ctx, int64_t n, const uint32_t *d_perm, int nfields, const float *const *h_in,
                          float *const *h_out) {
    if (!ctx) return SFCNL_E_ARG;
    if (n < 0 || n >= (int64_t(1) << 31) || nfields < 1 || nfields > 8 || !h_in || !h_out)
        return set_err(ctx, SFCNL_E_ARG, "sfc_gather: bad arguments");
    if (n == 0) return SFCNL_OK;
    if (!d_perm) return set_err(ctx, SFCNL_E_ARG, "sfc_gather: null perm");
    GatherArgs a{};
    a.nf = nfields;
    for (int f = 0; f < nfields; f++) {
        if (!h_in[f] || !h_out[f]) return set_err(ctx, SFCNL_E_ARG, "sfc_gather: null field %d", f);
        a.in[f] = h_in[f];
        a.out[f] = h_out[f];
    }
    prof_mark(ctx, kStageGather, false);
    k_gather<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, n, d_perm, a, false, ctx->d_status);
    SFCNL_LAUNCHED(ctx);
    prof_mark(ctx, kStageGather, true);
    return SFCNL_OK;
}

extern "C" int sfc_gather_workspace(int64_t n, size_t *ws_bytes) {
    if (n < 0 || !ws_bytes) return SFCNL_E_ARG;
    *ws_bytes = align_up((size_t)n * sizeof(float4), 256) + 256;
    return SFCNL_OK;
}

extern "C" int sfc_gather_ws(sfcnl_ctx ctx, int64_t n, const uint32_t *d_perm, int nfields, const float *const *h_in,
                             float *const *h_out, void *d_ws, size_t ws_bytes) {
    if (!ctx) return SFCNL_E_ARG;
    if (n < 0 || n >= (int64_t(1) << 31) || nfields < 1 || nfields > 8 || !h_in || !h_out)
        return set_err(ctx, SFCNL_E_ARG, "sfc_gather_ws: bad arguments");
    if (n == 0) return SFCNL_OK;
    if (!d_perm || !d_ws) return set_err(ctx, SFCNL_E_ARG, "sfc_gather_ws: null perm or workspace");
    size_t need;
    sfc_gather_workspace(n, &need);
    if (ws_bytes < need)
        return set_err(ctx, SFCNL_E_ARG, "sfc_gather_ws: workspace %zu bytes < %zu needed", ws_bytes, need);
    for (int f = 0; f < nfields; f++)
        if (!h_in[f] || !h_out[f]) return set_err(ctx, SFCNL_E_ARG, "sfc_gather_ws: null field %d", f);
    // records start at the first 256-byte boundary of the workspace (the
    // size includes that slack)
    float4 *rec = reinterpret_cast<float4 *>(align_up(reinterpret_cast<uintptr_t>(d_ws), 256));
    hipStream_t st = ctx->stream;
    const unsigned g = blocks_for(n, 256);
    prof_mark(ctx, kStageGather, false);
    for (int f0 = 0; f0 < nfields; f0 += 4) {
        const int nf = nfields - f0 < 4 ? nfields - f0 : 4;
        if (nf == 1) {  // a single field gains nothing from staging
            GatherArgs a{};
            a.nf = 1;
            a.in[0] = h_in[f0];
            a.out[0] = h_out[f0];
            k_gather<<<g, 256, 0, st>>>(n, n, d_perm, a, false, ctx->d_status);
            SFCNL_LAUNCHED(ctx);
            continue;
        }
        Pack4 a{};
        a.nf = nf;
        for (int f = 0; f < nf; f++) {
            a.in[f] = h_in[f0 + f];
            a.out[f] = h_out[f0 + f];
        }
        k_pack4<<<g, 256, 0, st>>>(n, a, rec);
        SFCNL_LAUNCHED(ctx);
        k_gather4<<<g, 256, 0, st>>>(n, d_perm, rec, a, ctx->d_status);
        SFCNL_LAUNCHED(ctx);
    }
    prof_mark(ctx, kStageGather, true);
    return SFCNL_OK;
}

// ---------------------------------------------------------------------------
// Batched systems: keys in each system's own box, a stable sort by (system,
// key) -- the key passes, then one or two passes on the system of the
// original index -- and the spread into the padded layout.
// ---------------------------------------------------------------------------

namespace {

struct BatchSortWs {
    SortWs s;
    uint64_t *k2;
    uint32_t *v2;
};

size_t carve_batch_sort(Carver &cv, BatchSortWs &w, int64_t n_in) {
    carve_sort(cv, w.s, n_in);
    w.k2 = cv.take<uint64_t>((size_t)n_in);
    w.v2 = cv.take<uint32_t>((size_t)n_in);
    return cv.used;
}

}  // namespace

extern "C" int sfcnl_batch_sort_workspace(sfcnl_batch b, size_t *ws_bytes) {
    if (!b || !ws_bytes) return SFCNL_E_ARG;
    Carver cv{nullptr, 0};
    BatchSortWs w;
    *ws_bytes = align_up(carve_batch_sort(cv, w, b->n_in), 256) + 256;
    return SFCNL_OK;
}

extern "C" int sfcnl_batch_sort(sfcnl_ctx ctx, sfcnl_batch b, const float *d_x, const float *d_y, const float *d_z,
                                uint64_t *d_keys_out, uint32_t *d_perm_out, void *d_ws, size_t ws_bytes) {
    if (!ctx) return SFCNL_E_ARG;
    if (!b) return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_sort: null batch");
    if (b->device != ctx->device) return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_sort: batch on another device");
    if (b->n_pad == 0) return SFCNL_OK;
    if (!d_keys_out || !d_perm_out || ((!d_x || !d_y || !d_z || !d_ws) && b->n_in))
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_sort: null pointer");
    size_t need;
    sfcnl_batch_sort_workspace(b, &need);
    if (ws_bytes < need)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_sort: workspace %zu bytes < %zu needed", ws_bytes, need);
    const int64_t n = b->n_in;
    const SegTable seg = seg_of(b);
    hipStream_t st = ctx->stream;
    if (n == 0) {  // only padding
        k_batch_pad<<<blocks_for(b->n_pad, 256), 256, 0, st>>>(b->n_pad, nullptr, nullptr, seg, b->d_in_off,
                                                               d_keys_out, d_perm_out);
        SFCNL_LAUNCHED(ctx);
        return SFCNL_OK;
    }
    Carver cv{reinterpret_cast<char *>(d_ws), 0};
    BatchSortWs w;
    carve_batch_sort(cv, w, n);
    prof_mark(ctx, kStageKeys, false);
    k_batch_keys<<<blocks_for(n, 256), 256, 0, st>>>(n, d_x, d_y, d_z, b->d_in_off, b->nsys, b->d_lo, b->d_scale,
                                                     w.k2, w.v2, ctx->d_status);
    SFCNL_LAUNCHED(ctx);
    prof_mark(ctx, kStageKeys, true);
    prof_mark(ctx, kStageSort, false);
    uint64_t *ka = w.k2, *kb = w.s.ktmp;
    uint32_t *va = w.v2, *vb = w.s.vtmp;
    const int sys_passes = b->nsys <= 1 ? 0 : (b->nsys <= 256 ? 1 : 2);
    for (int pass = 0; pass < kPasses + sys_passes; pass++) {
        const DigitOf dg = pass < kPasses ? DigitOf{8 * pass, nullptr, 0}
                                          : DigitOf{8 * (pass - kPasses), b->d_in_off, b->nsys};
        int rc = radix_pass(ctx, w.s, ka, va, kb, vb, n, dg);
        if (rc) return rc;
        uint64_t *tk = ka;
        ka = kb;
        kb = tk;
        uint32_t *tv = va;
        va = vb;
        vb = tv;
    }
    k_batch_pad<<<blocks_for(b->n_pad, 256), 256, 0, st>>>(b->n_pad, ka, va, seg, b->d_in_off, d_keys_out,
                                                           d_perm_out);
    SFCNL_LAUNCHED(ctx);
    prof_mark(ctx, kStageSort, true);
    return SFCNL_OK;
}

extern "C" int sfcnl_batch_gather(sfcnl_ctx ctx, sfcnl_batch b, const uint32_t *d_perm, int nfields,
                                  const float *const *h_in, float *const *h_out) {
    if (!ctx) return SFCNL_E_ARG;
    if (!b || nfields < 1 || nfields > 8 || !h_in || !h_out)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_gather: bad arguments");
    if (b->n_pad == 0) return SFCNL_OK;
    if (!d_perm) return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_gather: null perm");
    GatherArgs a{};
    a.nf = nfields;
    for (int f = 0; f < nfields; f++) {
        if ((!h_in[f] && b->n_in) || !h_out[f]) return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_gather: null field %d", f);
        a.in[f] = h_in[f];
        a.out[f] = h_out[f];
    }
    prof_mark(ctx, kStageGather, false);
    k_gather<<<blocks_for(b->n_pad, 256), 256, 0, ctx->stream>>>(b->n_pad, b->n_in, d_perm, a, true, ctx->d_status);
    SFCNL_LAUNCHED(ctx);
    prof_mark(ctx, kStageGather, true);
    return SFCNL_OK;
}
