// Clusters, octree traversal and compressed list encoding (Sec. II-A, II-B,
// II-C).
//
// One wavefront builds the list of one super-cluster (64 particles = 8
// i-clusters of 8).
//
// Traversal: depth-first from the root with an LDS stack; at an internal node
// 64 lanes test up to 8 children against 8 boxes of the super-cluster and
// push the survivors in reverse key order, so leaves come out in key order
// and the list is sorted without a sort (Sec. II-A). At a leaf, 64 lanes test
// the i-cluster boxes against the boxes of the leaf's candidate j-clusters;
// each candidate with a nonempty i-cluster mask joins an LDS queue. Once 64
// are queued (and at the end) the queue is drained in order, the
// j-particles of a batch of queued candidates arriving with one load per
// field while the previous batch's tests run. For cluster size 8 the exact
// tests are lane-parallel over the batch's (candidate, i-cluster) tiles: a
// group of 8 lanes takes one tile and steps through its 8 j-particles (see
// drain_lanes); sizes 4 and 16 give each tile one 64-lane step. Box tests
// are conservative under FP32 rounding (rounding is monotone), so they
// never drop a pair the exact test keeps; the masks are exact.
//
// The list is staged in 64-entry chunks with its encoded size computed on the
// fly (a super-cluster's first chunk is its own, later ones come from 64
// striped counters), a prefix sum places the super-clusters in order, and a
// second kernel writes masks and nibble segments.
#include <cstring>
#include <type_traits>
#include <utility>

#include "internal.h"

namespace sfcnl {
namespace {

// Lambdas of the traversal kernel are always inlined: a lambda left as a call
// takes the kernel's argument block by reference, which then lives in
// scratch memory, and every pointer from it is loaded through scratch.
#define SFC_INLINE __attribute__((always_inline))

// One wavefront (one super-cluster) per block for the traversal and the
// encoder: a block's resources are released only when its slowest wave ends,
// and super-clusters differ in work; measured 10 % faster than four.
constexpr int kWavesPerBlock = 1;
constexpr int kStackCap = 160;  // 1 + 7 * 21 pushes at most
constexpr int kSegCap = 80;     // words of one 64-value segment: 2 + (64 + 512 + 7) / 8
constexpr int kQueueCap = 96;   // queued candidates: drained at 64, one box step adds at most 16
constexpr uint32_t kUnstaged = 0xFFFFFFFFu;  // sc_nj of a list that found no staging room

__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned g) {
    // blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous
    // range of super-clusters so neighbouring ones share its L2
    const unsigned per = g / 8, rem = g % 8, x = b % 8, i = b / 8;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Boxes carry .w of lo = largest radius inside. True if some particle pair
// across the two boxes could satisfy d2 < max(h_i, h_j)^2.
template <bool kPbc>
__device__ __forceinline__ bool boxes_near_p(float4 alo, float4 ahi, float4 blo, float4 bhi, const Period &per) {
    float gx = axis_gap<kPbc>(blo.x - ahi.x, alo.x - bhi.x, per.L[0]);
    float gy = axis_gap<kPbc>(blo.y - ahi.y, alo.y - bhi.y, per.L[1]);
    float gz = axis_gap<kPbc>(blo.z - ahi.z, alo.z - bhi.z, per.L[2]);
    float gxx = gx * gx;
    float d2 = __builtin_fmaf(gz, gz, __builtin_fmaf(gy, gy, gxx));
    float ra = alo.w * alo.w, rb = blo.w * blo.w;
    return d2 < fmaxf(ra, rb);
}
// per is wave-uniform: super-clusters that need no wrapping take the open test
template <bool kPbc = false>
__device__ __forceinline__ bool boxes_near(float4 alo, float4 ahi, float4 blo, float4 bhi, const Period &per = Period{}) {
    if (kPbc && per.on()) return boxes_near_p<true>(alo, ahi, blo, bhi, per);
    return boxes_near_p<false>(alo, ahi, blo, bhi, per);
}

// Position for absent particles: any distance to it overflows to +inf.
constexpr float kFar = 3.0e38f;

// OR of the eight bytes of a ballot: bit k set iff some lane k + 8c is set.
__device__ __forceinline__ uint32_t byte_or(uint64_t b) {
    b |= b >> 32;
    b |= b >> 16;
    b |= b >> 8;
    return (uint32_t)(b & 0xFFu);
}

__device__ __forceinline__ uint32_t nibbles_of(uint32_t v) { return (32u - (uint32_t)__clz((int)v) + 3u) >> 2; }

// ---------------------------------------------------------------------------
// Clusters: bounding boxes and radius maxima, input checks.
// ---------------------------------------------------------------------------
template <int CS, bool kVec>
__global__ __launch_bounds__(256) void k_cluster_bbox(int64_t n, const float *__restrict__ x,
                                                      const float *__restrict__ y, const float *__restrict__ z,
                                                      const float *__restrict__ h, float4 *__restrict__ bbox,
                                                      uint32_t *status, SegTable seg) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (n + CS - 1) / CS) return;
    // batched systems: particles from pend on are padding (NaN, ignored by
    // fminf / fmaxf and never checked)
    int64_t pend = n;
    if (seg.on()) {
        const int sy = seg.sc_sys[c * CS / kScSize];
        pend = (int64_t)seg.pbase[sy] + seg.count[sy];
    }
    // a whole cluster of 16-byte-aligned fields comes as CS / 4 float4 loads
    // per field (one request per 16 bytes instead of one per 4); the last,
    // partial cluster or unaligned fields read each particle from a clamped
    // index; all loads are in flight together
    float px[CS], py[CS], pz[CS], ph[CS];
    if (kVec && c * CS + CS <= n) {
        const float4 *x4 = reinterpret_cast<const float4 *>(x) + c * (CS / 4);
        const float4 *y4 = reinterpret_cast<const float4 *>(y) + c * (CS / 4);
        const float4 *z4 = reinterpret_cast<const float4 *>(z) + c * (CS / 4);
        const float4 *h4 = reinterpret_cast<const float4 *>(h) + c * (CS / 4);
#pragma unroll
        for (int q = 0; q < CS / 4; q++) {
            const float4 vx = x4[q], vy = y4[q], vz = z4[q], vh = h4[q];
            px[4 * q] = vx.x, px[4 * q + 1] = vx.y, px[4 * q + 2] = vx.z, px[4 * q + 3] = vx.w;
            py[4 * q] = vy.x, py[4 * q + 1] = vy.y, py[4 * q + 2] = vy.z, py[4 * q + 3] = vy.w;
            pz[4 * q] = vz.x, pz[4 * q + 1] = vz.y, pz[4 * q + 2] = vz.z, pz[4 * q + 3] = vz.w;
            ph[4 * q] = vh.x, ph[4 * q + 1] = vh.y, ph[4 * q + 2] = vh.z, ph[4 * q + 3] = vh.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < CS; k++) {
            const int64_t p = c * CS + k;
            const int64_t q = p < n ? p : n - 1;
            px[k] = x[q];
            py[k] = y[q];
            pz[k] = z[q];
            ph[k] = h[q];
        }
    }
    float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
    float4 hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
    uint32_t bad = 0;
#pragma unroll
    for (int k = 0; k < CS; k++) {
        const int64_t p = c * CS + k;
        if (p < n) {
            const bool pad = p >= pend;
            if (!pad && !(isfinite(px[k]) && isfinite(py[k]) && isfinite(pz[k]))) bad |= 1u;
            if (!pad && !(isfinite(ph[k]) && ph[k] > 0.0f)) bad |= 2u;
            lo.x = fminf(lo.x, px[k]);
            lo.y = fminf(lo.y, py[k]);
            lo.z = fminf(lo.z, pz[k]);
            lo.w = fmaxf(lo.w, ph[k]);
            hi.x = fmaxf(hi.x, px[k]);
            hi.y = fmaxf(hi.y, py[k]);
            hi.z = fmaxf(hi.z, pz[k]);
        }
    }
    bbox[2 * c] = lo;
    bbox[2 * c + 1] = hi;
    if (bad) atomicOr(&status[kStInputErr], bad);
}

// ---------------------------------------------------------------------------
// Traversal
// ---------------------------------------------------------------------------
struct TravArgs {
    int64_t n;
    uint32_t nsc, nclu;
    int compress;
    const float *x, *y, *z, *h;
    const float4 *bbox;
    const float4 *cs_box;  // octree child slots (slot 0 = root)
    const uint4 *cs_rec;
    uint32_t nslots;       // capacity of the slot arrays
    SegTable seg;          // batched systems (empty for one system)
    Period per;            // periodic axes (used by the kPbc kernels)
    const uint32_t *active;  // nullable: super-clusters with active[s] == 0 get an empty list
    // nullable: a counting list for the flagged particles only (own radius):
    // pairs d2 < h_i^2 for i with p_active[i] != 0; node, cluster and j radii
    // are ignored, so the octree's boxes need no refit when only radii change
    const uint8_t *p_active;
    const uint32_t *gate;  // nullable: every list empty when *gate <= gate_max
    uint32_t gate_max;
    // staging: 64-entry chunks; chunk s is super-cluster s's first, longer
    // lists continue in chunks nsc + id taken from the stripe counters
    // (take_chunk); chunk_next links a list's chunks in order
    uint32_t *list_j;
    uint16_t *list_m;
    uint32_t *chunk_next;
    uint32_t nshared;      // shared chunks (ids 0 .. nshared - 1)
    uint32_t *chunk_ctr;   // the stripe counters that hand them out; word 1 of each line holds the stripe's longest list (zeroed before the build)
    uint32_t *sc_nj, *sc_words;
    uint32_t *status;
};

// Lane roles of a super-cluster's wavefront for cluster size CS (64 / CS
// i-clusters per super-cluster).
//
// Box tests: lane l pairs the box of i-cluster l % (64 / CS) with candidate
// slot l / (64 / CS), so one ballot holds in consecutive groups of 64 / CS
// bits the i-cluster mask of each candidate slot (8 slots of 8 bits for CS = 8,
// 4 of 16 for CS = 4, 16 of 4 for CS = 16). Node tests pair child l / 8 with
// the box of super-cluster particles [8g, 8g + 8), g = l % 8 (for CS = 16 the
// box of the i-cluster holding them).
//
// Exact tests (one step is 64 particle pairs):
//   CS = 8:  lane (il, jl) = (lane / 8, lane % 8); register k holds i-particle
//            8k + il (i-cluster k); one step is one 8x8 cluster pair.
//   CS = 4:  lane (q, il, jl) = (lane / 16, lane / 4 % 4, lane % 4); register
//            k holds i-particle 16k + lane / 4 (i-cluster 4k + q); one step is
//            four 4x4 pairs (i-clusters 4k .. 4k + 3 against one j-cluster).
//   CS = 16: lane (il, jq) = (lane / 4, lane % 4); register k holds
//            i-particle 16k + il (i-cluster k); a 16x16 pair takes four steps
//            (j-particles 4t + jq).
template <int CS>
struct Shape {
    static constexpr int kNsub = kScSize / CS;        // i-clusters per super-cluster
    static constexpr int kNreg = CS == 8 ? 8 : 4;     // i-particles per lane
    static constexpr int kNj = CS == 16 ? 4 : 1;      // j-particles per lane and candidate
    static constexpr int kMaskBytes = kNsub > 8 ? 2 : 1;
    static constexpr int kSlots = kWave / kNsub;      // candidate j-clusters per box step
    static constexpr uint32_t kFull = (1u << kNsub) - 1u;
    __device__ static int ipart(int k, int lane) { return CS == 8 ? 8 * k + (lane >> 3) : 16 * k + (lane >> 2); }
    __device__ static int jpart(int t, int lane) { return CS == 8 ? (lane & 7) : (CS == 4 ? (lane & 3) : 4 * t + (lane & 3)); }
};

__device__ __forceinline__ void box_union(float4 &lo, float4 &hi, float4 blo, float4 bhi) {
    lo.x = fminf(lo.x, blo.x);
    lo.y = fminf(lo.y, blo.y);
    lo.z = fminf(lo.z, blo.z);
    lo.w = fmaxf(lo.w, blo.w);
    hi.x = fmaxf(hi.x, bhi.x);
    hi.y = fmaxf(hi.y, bhi.y);
    hi.z = fmaxf(hi.z, bhi.z);
}

constexpr uint32_t kNoChunk = 0xFFFFFFFFu;

// A shared staging chunk for super-cluster s: from stripe s % kChunkStripes,
// else from the next stripes while one is used up; kNoChunk once all are
// (every one of the nshared ids is taken). Called by one lane.
__device__ uint32_t take_chunk(uint32_t *ctr, uint32_t nshared, uint32_t s) {
    for (uint32_t t = 0; t < (uint32_t)kChunkStripes; t++) {
        const uint32_t k = (s + t) % kChunkStripes;
        if (k >= nshared) continue;  // an empty stripe
        const uint32_t cap = (nshared - k + kChunkStripes - 1) / kChunkStripes;
        const uint32_t i = atomicAdd(&ctr[k * kStripeWords], 1u);
        if (i < cap) return k + kChunkStripes * i;
    }
    return kNoChunk;
}

// Bit k of the result: byte k of b is nonzero.
__device__ __forceinline__ uint32_t nonzero_bytes(uint64_t b) {
    b |= b >> 4;
    b |= b >> 2;
    b |= b >> 1;
    b &= 0x0101010101010101ull;
    return (uint32_t)((b * 0x0102040810204080ull) >> 56);
}

// f(std::integral_constant<int, i>{}) for i = 0 .. N - 1
template <int N, typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

// v of lane P of the quad (DPP quad_perm broadcast). With all rows and banks
// enabled and bound_ctrl set, the compiler folds the move into the consuming
// instruction's first operand, so the broadcast costs no instruction.
template <int P>
__device__ __forceinline__ float quad_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), P * 0x55, 0xF, 0xF, true));
}

// max of two squared radii (both >= +0): the integer order of their bit
// patterns is their order, and the integer max needs no canonicalisation
__device__ __forceinline__ float max_sq(float u, float v) {
    return __int_as_float(max(__float_as_int(u), __float_as_int(v)));
}

// Five waves per SIMD (at most 96 VGPRs).
template <int CS, bool kHalf, bool kPbc>
__global__ __launch_bounds__(kWave * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_traverse(TravArgs a) {
    using S = Shape<CS>;
    constexpr int kNsub = S::kNsub, kNreg = S::kNreg, kNj = S::kNj, kSlots = S::kSlots;
    __shared__ uint4 s_stack[kWavesPerBlock][kStackCap];
    __shared__ uint2 s_queue[kWavesPerBlock][kQueueCap];
    const int lane = sfc_lane();
    const int w = threadIdx.x / kWave;
    // wave-uniform: keep the super-cluster index (and all derived from it) scalar
    const uint32_t s = (uint32_t)__builtin_amdgcn_readfirstlane((int)(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + w));
    if (s >= a.nsc) return;
    if ((a.active && !a.active[s]) || (a.gate && *a.gate <= a.gate_max)) {  // no list for this super-cluster
        if (sfc_lane() == 0) {
            a.sc_nj[s] = 0;
            a.sc_words[s] = 0;
        }
        return;
    }
    const int64_t n = a.n;
    const bool gather = a.p_active != nullptr;
    // i particles; absent ones are put far away so that no test accepts them.
    // Cluster size 8 keeps them in LDS for its lane-parallel tiles (lane l
    // loads particle l; particle 8c + l' sits at 9c + l', a padding slot after
    // each cluster keeps the clusters on distinct banks), the other sizes in
    // the registers of their tile lanes.
    constexpr bool kLaneTiles = CS == 8;
    __shared__ float4 s_ip[kWavesPerBlock][kLaneTiles ? 72 : 1];
    float ix[kNreg], iy[kNreg], iz[kNreg], ih2[kNreg];
    float lh2 = 0.0f;  // cluster size 8: the squared radius of particle lane
    bool big = false;  // a radius reaches half a period
    if constexpr (kLaneTiles) {
        const int64_t i = (int64_t)s * kScSize + lane;
        const bool v = i < n;
        float hh = v ? a.h[i] : 0.0f;
        if (kPbc) big = !(hh < a.per.hmin);
        if (gather && v && !a.p_active[i]) hh = 0.0f;  // counting list: flagged particles only
        lh2 = hh * hh;
        s_ip[w][9 * (lane >> 3) + (lane & 7)] = make_float4(v ? a.x[i] : kFar, v ? a.y[i] : kFar, v ? a.z[i] : kFar, lh2);
    } else {
#pragma unroll
        for (int k = 0; k < kNreg; k++) {
            const int64_t i = (int64_t)s * kScSize + S::ipart(k, lane);
            const bool v = i < n;
            ix[k] = v ? a.x[i] : kFar;
            iy[k] = v ? a.y[i] : kFar;
            iz[k] = v ? a.z[i] : kFar;
            float hh = v ? a.h[i] : 0.0f;
            if (kPbc) big = big || !(hh < a.per.hmin);
            if (gather && v && !a.p_active[i]) hh = 0.0f;  // counting list: flagged particles only
            ih2[k] = hh * hh;
        }
    }
    if (kPbc && sfc_ballot(big) && lane == 0) atomicOr(&a.status[kStInputErr], 8u);
    const uint32_t own_c0 = s * kNsub;  // first i-cluster of this super-cluster
    const uint32_t own_p0 = s * kScSize;  // and its first particle

    constexpr bool half = kHalf;
    const float4 empty_lo = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
    const float4 empty_hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
    // box tests: the box of i-cluster lane % kNsub
    float4 ilo, ihi;
    {
        const uint32_t ic = own_c0 + (uint32_t)(lane & (kNsub - 1));
        const bool v = ic < a.nclu;
        ilo = v ? a.bbox[2 * (size_t)ic] : empty_lo;
        ihi = v ? a.bbox[2 * (size_t)ic + 1] : empty_hi;
    }
    // node tests: the box of super-cluster particles [8g, 8g + 8), g = lane % 8
    // (for CS = 16 the box of their i-cluster)
    float4 glo, ghi;
    if (CS == 8) {
        glo = ilo;
        ghi = ihi;
    } else {
        const int g = lane & 7;
        const uint32_t c0 = own_c0 + (CS == 4 ? 2 * g : (g >> 1));
        const bool v0 = c0 < a.nclu;
        glo = v0 ? a.bbox[2 * (size_t)c0] : empty_lo;
        ghi = v0 ? a.bbox[2 * (size_t)c0 + 1] : empty_hi;
        if (CS == 4 && c0 + 1 < a.nclu) box_union(glo, ghi, a.bbox[2 * (size_t)c0 + 2], a.bbox[2 * (size_t)c0 + 3]);
    }

    if (gather) {
        // radii of the boxes: the largest flagged radius inside, from the i
        // registers (a radius 0 box passes no test)
        __shared__ float s_hmax[kWavesPerBlock][kScSize];
        float *hm = s_hmax[w];
        if constexpr (kLaneTiles) {
            hm[lane] = __builtin_sqrtf(lh2);
        } else {
#pragma unroll
            for (int k = 0; k < kNreg; k++) {
                if ((lane & 3) == 0) hm[S::ipart(k, lane)] = __builtin_sqrtf(ih2[k]);
            }
        }
        wave_sync();
        auto rmax = [&](int p0, int cnt) SFC_INLINE {
            float r = 0.0f;
            for (int q = 0; q < cnt; q++) r = fmaxf(r, hm[p0 + q]);
            return r;
        };
        ilo.w = rmax((lane & (kNsub - 1)) * CS, CS);
        if (CS == 8)
            glo.w = ilo.w;
        else if (CS == 4)
            glo.w = rmax(8 * (lane & 7), 8);
        else
            glo.w = rmax(16 * ((lane & 7) >> 1), 16);
        wave_sync();
    }

    // Periodic axes: a pair can take an image one period away only if the
    // super-cluster lies within the largest search radius R of the far face
    // of the particles' span (a direct difference above L - R). Otherwise
    // every minimum image is the direct one and the super-cluster runs the
    // open-boundary tests; the margin on R keeps the decision on the safe side
    // of FP32 rounding, so no accepted pair changes.
    bool wraps = false;
    IBox sbox;  // the super-cluster's box (positions), for the batches' own decision
    if (kPbc) {
        float slo[3] = {glo.x, glo.y, glo.z}, shi[3] = {ghi.x, ghi.y, ghi.z};
        float r = glo.w;  // full build: replaced by the largest radius of all
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
#pragma unroll
            for (int t = 0; t < 3; t++) {
                slo[t] = fminf(slo[t], __shfl_xor(slo[t], d, 64));
                shi[t] = fmaxf(shi[t], __shfl_xor(shi[t], d, 64));
            }
            r = fmaxf(r, __shfl_xor(r, d, 64));
        }
        const float4 rlo = a.cs_box[0], rhi = a.cs_box[1];  // root box: the particles' span
        if (!gather) r = fmaxf(r, rlo.w);  // pairs use max(h_i, h_j)
        const float plo[3] = {rlo.x, rlo.y, rlo.z}, phi[3] = {rhi.x, rhi.y, rhi.z};
        bool w_lane = false;
#pragma unroll
        for (int t = 0; t < 3; t++) {
            if (a.per.L[t] < INFINITY) {
                const float reach = a.per.L[t] - 1.0001f * r - 1e-5f * a.per.L[t];
                w_lane = w_lane || !(phi[t] - slo[t] <= reach) || !(shi[t] - plo[t] <= reach);
            }
        }
        wraps = sfc_ballot(w_lane) != 0;
#pragma unroll
        for (int t = 0; t < 3; t++) {  // wave-uniform: scalar registers
            sbox.lo[t] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, slo[t])));
            sbox.hi[t] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, shi[t])));
        }
    }
    const Period per = wraps ? a.per : Period{};
    // minimum images of a pair's components on periodic axes
    auto wrap = [&](float &dx, float &dy, float &dz) SFC_INLINE {
        if (wraps) wave_min_image(dx, dy, dz, a.per);
    };

    // stack of node records {first, end, child count (0 = leaf), first child
    // slot}; a node is pushed only after its box passed the test
    uint4 *stack = s_stack[w];
    uint2 *queue = s_queue[w];
    int sp = 0;
    // the tree of this super-cluster's system; list entries are cluster
    // indices relative to the system's first cluster
    uint32_t jbase = 0;
    if (a.seg.on()) {
        const int sy = a.seg.sc_sys[s];
        jbase = a.seg.pbase[sy] / CS;
        if (lane == 0) stack[0] = a.seg.roots[sy];
    } else {
        if (lane == 0) stack[0] = a.cs_rec[0];  // root
    }
    sp = 1;
    wave_sync();

    int64_t last = -1;  // highest j-cluster already tested
    uint32_t nj = 0, prevj = 0xFFFFFFFFu, seg_words = 0;
    // entries collect in lane (index % 64) of ej / em and leave 64 at a time
    // into the next staging chunk: one coalesced store each, and the
    // compressed size of the 64-entry segment (first difference from the
    // previous segment's last index; difference 1: no nibble, up to 9: one,
    // else one plus its hex digits)
    uint32_t ej = 0, em = 0;
    uint32_t chunk = s;        // chunk being filled
    bool staged = true;        // false once the shared chunks ran out
    auto flush = [&](uint32_t cnt) SFC_INLINE {
        if (nj > cnt) {  // beyond the first chunk: take a shared one
            uint32_t id = kNoChunk;
            if (lane == 0 && staged) id = take_chunk(a.chunk_ctr, a.nshared, s);
            id = (uint32_t)__builtin_amdgcn_readfirstlane((int)id);
            if (id != kNoChunk) {
                if (lane == 0) a.chunk_next[chunk] = a.nsc + id;
                chunk = a.nsc + id;
            } else {
                if (lane == 0) atomicAdd(&a.status[kStChunks], 1u);  // a request left unserved (sizes the retry)
                staged = false;
            }
        }
        if (staged && (uint32_t)lane < cnt) {
            a.list_j[(size_t)chunk * kWave + lane] = ej;
            a.list_m[(size_t)chunk * kWave + lane] = (uint16_t)em;
        }
        const uint32_t up = __shfl_up(ej, 1, 64);
        const uint32_t v = ej - (lane == 0 ? prevj : up);
        const uint32_t nib = (uint32_t)lane < cnt ? (v == 1u ? 0u : (v <= 9u ? 1u : 1u + nibbles_of(v))) : 0u;
        const uint32_t tot = sfc_readlane(sfc_incl_scan(nib), kWave - 1);
        seg_words += 2u + (tot + 7u) / 8u;
        prevj = sfc_readlane(ej, (int)cnt - 1);
    };

    // Exact tests of the queued candidates, in queue order. Lane (q, p) =
    // (lane / CS, lane % CS) loads particle p of candidate b + q, so one load
    // per field brings the j-particles of kBatch = 64 / CS candidates, and the
    // next batch loads while the current one's tiles run; each tile's lanes
    // then take their j-particle from lane q CS + p with ds_bpermute (a lane
    // exchange, no memory access). Absent particles (past n) are put far away
    // with a zero radius; counting lists use the i radius only (a zero j
    // radius makes max(h_i^2, h_j^2) = h_i^2).
    constexpr int kBatch = kWave / CS;
    uint32_t qn = 0;
    // The loads read a clamped index unconditionally, so they stay in flight
    // while the current batch's tiles run (a load behind a branch, or one
    // whose value is used at once, ends with a wait); validity and the squared
    // radius apply when the batch is used (drains run with qn >= 1).
    struct JLoad {
        float x, y, z, h;
        bool v;
    };
    auto load_batch = [&](uint32_t b0, JLoad &f) SFC_INLINE {
        const uint32_t e = b0 + (uint32_t)(lane / CS);
        const uint32_t cj = queue[e < qn ? e : qn - 1u].x;
        const int64_t p = (int64_t)cj * CS + (lane & (CS - 1));
        const int64_t pc = p < n ? p : n - 1;
        f.v = e < qn && p < n;
        f.x = a.x[pc];
        f.y = a.y[pc];
        f.z = a.z[pc];
        f.h = a.h[pc];
    };
    auto batch_vals = [&](const JLoad &f) SFC_INLINE {
        const float hh = f.v && !gather ? f.h : 0.0f;
        return make_float4(f.v ? f.x : kFar, f.v ? f.y : kFar, f.v ? f.z : kFar, hh * hh);
    };
    auto lane_f = [](int src, float v) SFC_INLINE {  // v of lane src (ds_bpermute takes a byte address)
        return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
    };

    // Cluster sizes 4 and 16: one step tests the 64 particle pairs of one
    // tile (CS = 4: four), the queued candidates one after another.
    auto drain_regs = [&]() SFC_INLINE {
        wave_sync();
        JLoad f;
        load_batch(0, f);
        for (uint32_t b0 = 0; b0 < qn; b0 += kBatch) {
            const float4 c = batch_vals(f);
            const float cx = c.x, cy = c.y, cz = c.z, ch2 = c.w;
            if (b0 + kBatch < qn) load_batch(b0 + kBatch, f);
            const uint32_t bn = qn - b0 < (uint32_t)kBatch ? qn - b0 : (uint32_t)kBatch;
            for (uint32_t q = 0; q < bn; q++) {
            const uint2 qe = queue[b0 + q];
            const uint32_t cjv = (uint32_t)__builtin_amdgcn_readfirstlane((int)qe.x);
            const uint32_t cmask = (uint32_t)__builtin_amdgcn_readfirstlane((int)qe.y);
            float xj[kNj], yj[kNj], zj[kNj], hj2[kNj];
#pragma unroll
            for (int t = 0; t < kNj; t++) {
                const int src = (int)q * CS + S::jpart(t, lane);
                xj[t] = lane_f(src, cx);
                yj[t] = lane_f(src, cy);
                zj[t] = lane_f(src, cz);
                hj2[t] = lane_f(src, ch2);
            }
            // the j-cluster is one of our own i-clusters: exclude i == j
            // (full list) or keep only j > i (half list)
            const int self_c = (cjv >= own_c0 && cjv < own_c0 + kNsub) ? (int)(cjv - own_c0) : -1;
            auto keep = [&](int ci, int ipos, int jpos) SFC_INLINE {
                return half ? (ci < self_c || (ci == self_c && jpos > ipos)) : (ci != self_c || jpos != ipos);
            };
            uint32_t mask = 0;
            if constexpr (CS == 4) {
                const int jl = lane & 3, il = (lane >> 2) & 3, q = lane >> 4;
#pragma unroll
                for (int k = 0; k < kNreg; k++) {
                    if ((cmask >> (4 * k)) & 0xFu) {
                        float dx = xj[0] - ix[k];
                        float dy = yj[0] - iy[k];
                        float dz = zj[0] - iz[k];
                        if (kPbc) wrap(dx, dy, dz);
                        const float dxx = dx * dx;
                        const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
                        bool pr = d2 < max_sq(ih2[k], hj2[0]);
                        if (self_c >= 0) pr = pr && keep(4 * k + q, il, jl);
                        const uint64_t b = sfc_ballot(pr);
                        const uint32_t g = (uint32_t)((b & 0xFFFFull) != 0) |
                                           ((uint32_t)(((b >> 16) & 0xFFFFull) != 0) << 1) |
                                           ((uint32_t)(((b >> 32) & 0xFFFFull) != 0) << 2) |
                                           ((uint32_t)((b >> 48) != 0) << 3);
                        mask |= g << (4 * k);
                    }
                }
            } else {
                const int jq = lane & 3, il = lane >> 2;
#pragma unroll
                for (int c = 0; c < kNreg; c++) {
                    if ((cmask >> c) & 1u) {
                        bool pr = false;
#pragma unroll
                        for (int t = 0; t < 4; t++) {
                            float dx = xj[t] - ix[c];
                            float dy = yj[t] - iy[c];
                            float dz = zj[t] - iz[c];
                            if (kPbc) wrap(dx, dy, dz);
                            const float dxx = dx * dx;
                            const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
                            bool p = d2 < max_sq(ih2[c], hj2[t]);
                            if (self_c >= 0) {
                                if (half)
                                    p = p && (c < self_c || (c == self_c && 4 * t + jq > il));
                                else if (c == self_c)
                                    p = p && 4 * t + jq != il;
                            }
                            pr = pr || p;
                        }
                        if (sfc_ballot(pr)) mask |= 1u << c;
                    }
                }
            }
            if (mask) {
                const bool mine = lane == (int)(nj & (kWave - 1));
                ej = mine ? cjv - jbase : ej;
                em = mine ? mask : em;
                if ((++nj & (kWave - 1)) == 0) flush(kWave);
            }
            }
        }
        qn = 0;
        wave_sync();
    };

    // Cluster size 8: lane-parallel tiles. A batch is 8 queued candidates;
    // bit 8q + c of W says that the box test kept i-cluster c for candidate
    // q. W's set bits, numbered in order, are the batch's tiles, and a round
    // hands tiles 8r .. 8r + 7 to the eight groups of 8 lanes: lane (g, l)
    // takes i-particle l of its tile's i-cluster and steps through the 8
    // j-particles of its candidate, one pair per step, so one step tests one
    // pair of each of 8 tiles. A tile passes if a lane of its group saw a
    // pair; the results go back to W's bit positions (R), whose bytes are the
    // candidates' masks. The j-particles of the batch wait in LDS (candidate
    // q's particle p at 9q + p).
    __shared__ float4 s_jp[kWavesPerBlock][kLaneTiles ? 72 : 1];
    // tile t of the batch: byte offsets of its i-cluster in s_ip (bits 0-10),
    // of its candidate's own i-cluster if it is one of ours, else 8 clusters
    // (bits 11-21), and of its candidate in s_jp (bits 22-31)
    __shared__ uint32_t s_tile[kWavesPerBlock][kLaneTiles ? 64 : 1];
    __shared__ uint2 s_ent[kWavesPerBlock][kLaneTiles ? 8 : 1];
    __shared__ uint64_t s_hits[kWavesPerBlock][kLaneTiles ? 8 : 1];
    if constexpr (kLaneTiles) s_tile[w][lane] = 0u;  // entries past a batch's tiles stay valid offsets
    auto drain_lanes = [&]() SFC_INLINE {
        wave_sync();
        constexpr uint32_t kRow = 9 * sizeof(float4);  // one cluster's stride in s_ip and s_jp
        constexpr uint64_t kBytes = 0x0101010101010101ull;
        const int g = lane >> 3, l = lane & 7;
        const char *ipb = reinterpret_cast<const char *>(s_ip[w]) + l * sizeof(float4);
        const char *jpb = reinterpret_cast<const char *>(s_jp[w]);
        JLoad f;
        load_batch(0, f);
        for (uint32_t b0 = 0; b0 < qn; b0 += kBatch) {
            const float4 jv = batch_vals(f);
            s_jp[w][9 * g + l] = jv;
            // a wrapping super-cluster still skips the minimum images for a
            // batch whose j-particles all lie within half a period of both
            // ends of its box on every periodic axis (far_from_box)
            bool bwrap = false;
            if constexpr (kPbc) bwrap = wraps && sfc_ballot(b0 + (uint32_t)g < qn && far_from_box(jv, sbox, a.per)) != 0;
            if (b0 + kBatch < qn) load_batch(b0 + kBatch, f);
            // lane (g, l): candidate b0 + g against i-cluster l
            const uint32_t e = b0 + (uint32_t)g;
            const bool ev = e < qn;
            const uint2 qe = queue[ev ? e : b0];
            const uint32_t rel = qe.x - own_c0;  // below 8: the candidate is our own i-cluster rel
            const bool bit = ev && ((qe.y >> l) & 1u);
            const uint64_t W = sfc_ballot(bit);
            const bool mixed = sfc_ballot(ev && rel < 8u) != 0;  // a candidate of the batch is ours
            const int T = sfc_popc(W);
            const uint32_t k = __builtin_amdgcn_mbcnt_hi((uint32_t)(W >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)W, 0u));
            if (bit) s_tile[w][k] = kRow * (uint32_t)l | (kRow * (rel < 8u ? rel : 8u)) << 11 | (kRow * (uint32_t)g) << 22;
            wave_sync();
            // s_hits[r]: round r's ballot (byte g: group g, i.e. tile 8r + g,
            // saw a pair); bytes of tiles past T are never read
            for (int r = 0; 8 * r < T; r++) {
                const uint32_t tv = s_tile[w][8 * r + g];  // tiles past T: stale valid offsets, results unread
                const uint32_t ioff = tv & 0x7FFu, soff = (tv >> 11) & 0x7FFu;
                const float4 ip = *reinterpret_cast<const float4 *>(ipb + ioff);
                // lane (g, l) holds j-particles l % 4 and 4 + l % 4 of its
                // candidate; step p takes particle p from lane p % 4 of the
                // quad (a DPP operand, no LDS traffic)
                const float4 *jb = reinterpret_cast<const float4 *>(jpb + (tv >> 22));
                const float4 ja = jb[l & 3], jz = jb[4 + (l & 3)];
                // the round's tests; batches that can wrap take the minimum
                // images (one wave-uniform choice per round keeps the 8 steps
                // free of branches)
                auto tests = [&](auto wrapc) SFC_INLINE {
                    constexpr bool kW = decltype(wrapc)::value;
                    uint64_t t = 0;
                    if (!mixed) {
                        static_for<CS>([&](auto pc) {
                            constexpr int p = decltype(pc)::value;
                            const float4 &jq = p < 4 ? ja : jz;
                            float dx = quad_bcast<p & 3>(jq.x) - ip.x;
                            float dy = quad_bcast<p & 3>(jq.y) - ip.y;
                            float dz = quad_bcast<p & 3>(jq.z) - ip.z;
                            if constexpr (kW) wave_min_image(dx, dy, dz, a.per);
                            const float dxx = dx * dx;
                            const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
                            t |= sfc_ballot(d2 < max_sq(quad_bcast<p & 3>(jq.w), ip.w));
                        });
                    } else {
                        // pairs within our own super-cluster: i = 8c + l and
                        // j = 8c' + p; the half list keeps j > i (c < c', or
                        // c = c' and l < p), the full list all but i = j
                        const uint64_t below = sfc_ballot(ioff < soff), same = sfc_ballot(ioff == soff);
                        static_for<CS>([&](auto pc) {
                            constexpr int p = decltype(pc)::value;
                            const float4 &jq = p < 4 ? ja : jz;
                            float dx = quad_bcast<p & 3>(jq.x) - ip.x;
                            float dy = quad_bcast<p & 3>(jq.y) - ip.y;
                            float dz = quad_bcast<p & 3>(jq.z) - ip.z;
                            if constexpr (kW) wave_min_image(dx, dy, dz, a.per);
                            const float dxx = dx * dx;
                            const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
                            const uint64_t keep = half ? below | (same & (((1ull << p) - 1ull) * kBytes)) : ~(same & ((1ull << p) * kBytes));
                            t |= sfc_ballot(d2 < max_sq(quad_bcast<p & 3>(jq.w), ip.w)) & keep;
                        });
                    }
                    return t;
                };
                uint64_t acc;
                if constexpr (kPbc) {
                    if (bwrap)
                        acc = tests(std::true_type{});
                    else
                        acc = tests(std::false_type{});
                } else {
                    acc = tests(std::false_type{});
                }
                if (lane == 0) s_hits[w][r] = acc;
            }
            wave_sync();
            // W's bit of rank k: tile k, byte k % 8 of round k / 8
            const uint32_t hw = reinterpret_cast<const uint32_t *>(s_hits[w])[(k >> 2) & 15u];
            const uint64_t R = sfc_ballot(bit && ((hw >> (8 * (k & 3u))) & 0xFFu) != 0u);
            // candidate g's mask is byte g of R; the nonempty ones join the
            // list in queue order (lane (nj + rank) % 64 of ej / em)
            const uint32_t mq = lane < kBatch ? (uint32_t)(R >> ((8 * lane) & 63)) & 0xFFu : 0u;
            const uint64_t ne = sfc_ballot(mq != 0u);
            if (ne) {
                const uint32_t cnt = (uint32_t)sfc_popc(ne);
                if (mq) {
                    const uint32_t rk = __builtin_amdgcn_mbcnt_lo((uint32_t)ne, 0u);
                    s_ent[w][rk] = make_uint2(queue[b0 + lane].x - jbase, mq);
                }
                wave_sync();
                const uint32_t base = nj & (kWave - 1);
                const uint32_t first = cnt < kWave - base ? cnt : kWave - base;
                const uint32_t d = (uint32_t)lane - base;
                if (d < first) {
                    const uint2 v = s_ent[w][d];
                    ej = v.x;
                    em = v.y;
                }
                nj += first;
                if ((nj & (kWave - 1)) == 0) flush(kWave);
                if (cnt > first) {
                    if ((uint32_t)lane < cnt - first) {
                        const uint2 v = s_ent[w][first + lane];
                        ej = v.x;
                        em = v.y;
                    }
                    nj += cnt - first;
                }
                wave_sync();  // the next batch rewrites s_ent
            }
        }
        qn = 0;
        wave_sync();
    };

    auto drain = [&]() SFC_INLINE {
        if constexpr (kLaneTiles)
            drain_lanes();
        else
            drain_regs();
    };

    const uint64_t lt = sfc_lt_mask();
    while (sp > 0) {
        sp--;
        const uint4 rv = stack[sp];
        const uint32_t nfirst = (uint32_t)__builtin_amdgcn_readfirstlane((int)rv.x);
        const uint32_t nend = (uint32_t)__builtin_amdgcn_readfirstlane((int)rv.y);
        const uint32_t nchild = (uint32_t)__builtin_amdgcn_readfirstlane((int)rv.z);
        const uint32_t cslot = (uint32_t)__builtin_amdgcn_readfirstlane((int)rv.w);
        if (nend > (uint64_t)n || nfirst >= nend || cslot + nchild > a.nslots) {  // only on a broken tree
            if (lane == 0) atomicOr(&a.status[kStTree], 16u);
            break;
        }
        if (nchild == 0) {
            int64_t c0 = nfirst / CS;
            const int64_t c1 = (nend - 1) / CS;
            if (c0 <= last) c0 = last + 1;
            if (half && c0 < (int64_t)own_c0) c0 = own_c0;  // j-clusters wholly before i: no j > i
            // candidate clusters cb .. cb + kSlots - 1: lane l tests i-cluster
            // l % kNsub against the box of candidate cb + l / kNsub; the
            // survivors (nonempty i-cluster masks) join the queue in order
            for (int64_t cb = c0; cb <= c1; cb += kSlots) {
                // unconditional loads from a clamped index (cluster indices
                // fit 32 bits); the slots past c1 (repeats of c1) are left
                // out of the ballot (one vector compare: a scalar mask took
                // ten scalar instructions per step)
                const uint32_t cjc = min((uint32_t)cb + (uint32_t)(lane / kNsub), (uint32_t)c1);
                const float4 l = a.bbox[2 * (size_t)cjc], u = a.bbox[2 * (size_t)cjc + 1];
                const float4 blo = make_float4(l.x, l.y, l.z, gather ? 0.0f : l.w);  // own radius only when counting
                const int64_t nv = (c1 - cb + 1) * kNsub;  // lanes holding candidates cb .. c1
                const uint64_t bal = sfc_ballot(boxes_near<kPbc>(ilo, ihi, blo, u, per) && lane < nv);
                if (bal) {
                    const int sl = lane < kSlots ? lane : 0;
                    const uint32_t cm = lane < kSlots ? (uint32_t)(bal >> (sl * kNsub)) & S::kFull : 0u;
                    const uint64_t sv = sfc_ballot(cm != 0u);
                    if (cm) queue[qn + (uint32_t)sfc_popc(sv & lt)] = make_uint2((uint32_t)cb + (uint32_t)lane, cm);
                    qn += (uint32_t)sfc_popc(sv);
                    if (qn >= (uint32_t)kWave) drain();
                }
            }
            if (c1 > last) last = c1;
        } else {
            // lane (ch, g): child ch = lane / 8 of the node against group g's box
            const int ch = lane >> 3;
            const bool act = ch < (int)nchild;
            // unconditional loads from a clamped slot (an internal node has
            // at least one child), then the select
            const uint32_t slot = cslot + (uint32_t)(act ? ch : 0);
            const float4 l = a.cs_box[2 * (size_t)slot];
            const float4 hi = a.cs_box[2 * (size_t)slot + 1];
            const uint4 crec = a.cs_rec[slot];
            const float4 lo = make_float4(l.x, l.y, l.z, gather ? 0.0f : l.w);  // own radius only when counting
            // a half list never needs a node that ends before the super-cluster
            const bool hit = act && boxes_near<kPbc>(glo, ghi, lo, hi, per) && (!half || crec.y > own_p0);
            const uint32_t keep = nonzero_bytes(sfc_ballot(hit));
            const int cnt = __popc(keep);
            if (sp + cnt > kStackCap) {  // cannot happen in a valid octree (depth <= 21)
                if (lane == 0) atomicOr(&a.status[kStTree], 8u);
                break;
            }
            if ((lane & 7) == 0 && ((keep >> ch) & 1u)) {
                const int r = __popc(keep & ((1u << ch) - 1u));
                stack[sp + cnt - 1 - r] = crec;  // first child on top
            }
            sp += cnt;
            wave_sync();
        }
    }
    if (qn) drain();
    if (nj & (kWave - 1)) flush(nj & (kWave - 1));
    if (lane == 0) {
        const uint32_t mwords = (nj * S::kMaskBytes + 3u) / 4u;
        a.sc_nj[s] = staged ? nj : kUnstaged;
        a.sc_words[s] = staged ? mwords + (a.compress ? seg_words : nj) : 0u;
        atomicMax(&a.chunk_ctr[(s % kChunkStripes) * kStripeWords + 1], nj);  // longest list, per stripe
        if (!staged) atomicOr(&a.status[kStScratch], 1u);
    }
}

// ---------------------------------------------------------------------------
// Encoder: masks, then raw indices or 64-wide nibble segments.
// ---------------------------------------------------------------------------
struct EncArgs {
    uint32_t nsc;
    int compress;
    int mask_bytes;  // 2 for 16 i-clusters per super-cluster, else 1
    const uint32_t *list_j;  // staging chunks (see TravArgs)
    const uint16_t *list_m;
    const uint32_t *chunk_next;
    const uint32_t *sc_nj, *sc_off;  // sc_off has nsc + 1 entries
    uint32_t *sc_info;
    uint32_t *pool;
    uint64_t pool_words;
    const uint32_t *chunk_ctr;  // the traversal's stripe counters
    uint32_t nshared;
    uint32_t *status;
};

__global__ __launch_bounds__(kWave * kWavesPerBlock) void k_encode(EncArgs a) {
    __shared__ uint32_t s_seg[kWavesPerBlock][kSegCap];
    const int lane = sfc_lane();
    const int w = threadIdx.x / kWave;
    // wave-uniform: keep the super-cluster index (and all derived from it) scalar
    const uint32_t s = (uint32_t)__builtin_amdgcn_readfirstlane((int)(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + w));
    // the pool total (the scan's last entry) into the status block, the
    // shared staging chunks taken added to the requests left unserved (a
    // stripe counter runs past its share when a request probes it full), and
    // the longest list over the stripes' maxima
    if (blockIdx.x == 0 && w == 0) {
        uint32_t taken = 0, longest = 0;
        if ((uint32_t)lane < (uint32_t)kChunkStripes) {
            longest = a.chunk_ctr[lane * kStripeWords + 1];
            if ((uint32_t)lane < a.nshared) {
                const uint32_t cap = (a.nshared - lane + kChunkStripes - 1) / kChunkStripes;
                taken = min(a.chunk_ctr[lane * kStripeWords], cap);
            }
        }
        const uint32_t tot = sfc_readlane(sfc_incl_scan(taken), kWave - 1);
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) longest = max(longest, (uint32_t)__shfl_xor((int)longest, d, kWave));
        if (lane == 0) {
            a.status[kStTotalLo] = a.sc_off[a.nsc];
            a.status[kStChunks] += tot;
            a.status[kStMaxNj] = max(a.status[kStMaxNj], longest);
        }
    }
    if (s >= a.nsc) return;
    const uint32_t nj = a.sc_nj[s];
    const uint32_t off = a.sc_off[s];
    const uint32_t words = a.sc_off[s + 1] - off;
    // a list that could not be staged or stored is recorded as empty (the
    // status block reports it), so that a pass launched regardless never
    // reads past the pool
    const bool fits = nj != kUnstaged && (uint64_t)off + words <= a.pool_words;
    if (lane == 0) {
        a.sc_info[2 * s] = off;
        a.sc_info[2 * s + 1] = fits ? nj : 0u;
        if (nj != kUnstaged && !fits) atomicOr(&a.status[kStPoolOverflow], 1u);
    }
    if (!fits) return;
    const uint32_t mwords = (nj * (uint32_t)a.mask_bytes + 3u) / 4u;
    uint32_t *mout = a.pool + off;
    uint32_t *out = mout + mwords;
    uint32_t *seg = s_seg[w];
    const uint64_t lt = sfc_lt_mask();
    uint32_t prevj = 0xFFFFFFFFu;
    uint32_t chunk = s;
    for (uint32_t b0 = 0; b0 < nj; b0 += kWave) {
        const uint32_t cnt = nj - b0 < (uint32_t)kWave ? nj - b0 : (uint32_t)kWave;
        const bool valid = (uint32_t)lane < cnt;
        // every lane of a 64-entry chunk is inside the staging arrays: the
        // loads go out unconditionally, the select follows
        const uint32_t jl = a.list_j[(size_t)chunk * kWave + lane];
        const uint32_t ml = (uint32_t)a.list_m[(size_t)chunk * kWave + lane];
        const uint32_t j = valid ? jl : 0u;
        const uint32_t m = valid ? ml : 0u;
        if (b0 + kWave < nj) chunk = a.chunk_next[chunk];
        // masks of this block: 4 (or 2) consecutive entries per word
        if (a.mask_bytes == 1) {
            uint32_t v = m << (8 * (lane & 3));
            v |= __shfl_xor(v, 1, 64);
            v |= __shfl_xor(v, 2, 64);
            if ((lane & 3) == 0 && (uint32_t)lane < cnt) mout[b0 / 4 + lane / 4] = v;
        } else {
            uint32_t v = m << (16 * (lane & 1));
            v |= __shfl_xor(v, 1, 64);
            if ((lane & 1) == 0 && (uint32_t)lane < cnt) mout[b0 / 2 + lane / 2] = v;
        }
        if (!a.compress) {
            if (valid) out[b0 + lane] = j;
            continue;
        }
        uint32_t jprev = __shfl_up(j, 1, 64);
        if (lane == 0) jprev = prevj;
        const uint32_t v = j - jprev;
        const bool nonone = valid && v != 1u;
        const uint64_t mk = sfc_ballot(nonone);
        const bool small = v <= 9u;
        const uint32_t nn = nibbles_of(v);
        const uint32_t ndata = (nonone && !small) ? nn : 0u;
        const uint32_t info = small ? v + 6u : nn - 1u;
        const uint32_t ninfo = (uint32_t)sfc_popc(mk);
        const uint32_t ipos = (uint32_t)sfc_popc(mk & lt);
        const uint32_t incl = sfc_incl_scan(ndata);
        const uint32_t dpos = ninfo + incl - ndata;
        const uint32_t total_nib = ninfo + sfc_readlane(incl, kWave - 1);
        const uint32_t segw = 2u + (total_nib + 7u) / 8u;
        for (uint32_t q = lane; q < segw; q += kWave) seg[q] = 0u;
        wave_sync();
        if (lane == 0) {
            seg[0] = (uint32_t)mk;
            seg[1] = (uint32_t)(mk >> 32);
        }
        if (nonone) {
            atomicOr(&seg[2 + ipos / 8], info << (4 * (ipos % 8)));
            for (uint32_t d = 0; d < ndata; d++) {
                const uint32_t nib = (v >> (4 * (ndata - 1 - d))) & 0xFu;
                const uint32_t t = dpos + d;
                atomicOr(&seg[2 + t / 8], nib << (4 * (t % 8)));
            }
        }
        wave_sync();
        for (uint32_t q = lane; q < segw; q += kWave) out[q] = seg[q];
        wave_sync();
        out += segw;
        prevj = sfc_readlane(j, (int)cnt - 1);
    }
}

struct NlistWs {
    Octree tree;
    uint32_t nchunks;     // staging chunks: nsc first ones, then the shared ones
    uint32_t *list_j;
    uint16_t *list_m;
    uint32_t *chunk_next;
    uint32_t *sc_nj, *sc_words, *sc_off;
    uint32_t *sc_active;  // per super-cluster counts / flags for restricted rebuilds (h-iteration)
    uint32_t *sc_scan;    // their prefix sum (nsc + 1)
    uint8_t *p_active;    // per particle flags for restricted rebuilds
    void *scan_tmp;
    uint32_t *plist;      // the flagged particles, compacted
};

// Staging chunks per super-cluster (on average): max_j_per_sc rounded up to
// whole 64-entry chunks.
inline int64_t staging_chunks(int max_j_per_sc) { return ((int64_t)max_j_per_sc + kWave - 1) / kWave; }

void carve_nlist(Carver &cv, NlistWs &ws, int64_t n, const sfcnl_nlist_opts &o, int nsys = 1) {
    const uint32_t nsc = (uint32_t)((n + kScSize - 1) / kScSize);
    octree_carve(cv, ws.tree, n, o.leaf_bucket, nsys, o.cluster_size);
    ws.nchunks = nsc * (uint32_t)staging_chunks(o.max_j_per_sc);
    ws.list_j = cv.take<uint32_t>((size_t)ws.nchunks * kWave);
    ws.list_m = cv.take<uint16_t>((size_t)ws.nchunks * kWave);
    ws.chunk_next = cv.take<uint32_t>(ws.nchunks);
    ws.sc_nj = cv.take<uint32_t>(nsc);
    ws.sc_words = cv.take<uint32_t>(nsc);
    ws.sc_off = cv.take<uint32_t>((size_t)nsc + 1);
    ws.sc_active = cv.take<uint32_t>(nsc);
    ws.sc_scan = cv.take<uint32_t>((size_t)nsc + 1);
    ws.p_active = cv.take<uint8_t>((size_t)n);
    ws.scan_tmp = cv.take<char>(scan_tmp_bytes(nsc));
    ws.plist = cv.take<uint32_t>((size_t)n);
}

template <bool kPbc>
void launch_traverse(int cs, int half, unsigned gb, hipStream_t st, const TravArgs &ta) {
    if (cs == 4) {
        if (half) k_traverse<4, true, kPbc><<<gb, kWave * kWavesPerBlock, 0, st>>>(ta); else k_traverse<4, false, kPbc><<<gb, kWave * kWavesPerBlock, 0, st>>>(ta);
    } else if (cs == 16) {
        if (half) k_traverse<16, true, kPbc><<<gb, kWave * kWavesPerBlock, 0, st>>>(ta); else k_traverse<16, false, kPbc><<<gb, kWave * kWavesPerBlock, 0, st>>>(ta);
    } else {
        if (half) k_traverse<8, true, kPbc><<<gb, kWave * kWavesPerBlock, 0, st>>>(ta); else k_traverse<8, false, kPbc><<<gb, kWave * kWavesPerBlock, 0, st>>>(ta);
    }
}

// Periodic axes: the particles must span less than one period (the root box
// of the octree holds the exact extent).
__global__ void k_check_span(const float4 *__restrict__ root_box, Period per, uint32_t *status) {
    const float4 lo = root_box[0], hi = root_box[1];
    const bool bad = !(hi.x - lo.x < per.L[0]) || !(hi.y - lo.y < per.L[1]) || !(hi.z - lo.z < per.L[2]);
    if (bad) atomicOr(&status[kStInputErr], 8u);
}

int check_opts(sfcnl_ctx ctx, const sfcnl_nlist_opts *o) {
    if (!o) return set_err(ctx, SFCNL_E_ARG, "null options");
    if (o->cluster_size != 4 && o->cluster_size != 8 && o->cluster_size != 16)
        return set_err(ctx, SFCNL_E_ARG, "cluster_size %d not supported (4, 8, 16)", o->cluster_size);
    if (o->compress != 0 && o->compress != 1) return set_err(ctx, SFCNL_E_ARG, "compress must be 0 or 1");
    if (o->half != 0 && o->half != 1) return set_err(ctx, SFCNL_E_ARG, "half must be 0 or 1");
    if (o->leaf_bucket < 8 || o->leaf_bucket > 256)
        return set_err(ctx, SFCNL_E_ARG, "leaf_bucket %d outside [8, 256]", o->leaf_bucket);
    if (o->max_j_per_sc < 1) return set_err(ctx, SFCNL_E_ARG, "max_j_per_sc must be positive");
    if (!period_ok(o->period)) return set_err(ctx, SFCNL_E_ARG, "period must be 3 finite values >= 0");
    return SFCNL_OK;
}

}  // namespace
}  // namespace sfcnl

using namespace sfcnl;

int sfcnl::clusters_impl(sfcnl_ctx ctx, int64_t n, const float *x, const float *y, const float *z, const float *h,
                         int cs, float *bbox, const SegTable &seg) {
    if (n == 0) return SFCNL_OK;
    const int64_t nclu = (n + cs - 1) / cs;
    prof_mark(ctx, kStageClusters, false);
    float4 *b4 = reinterpret_cast<float4 *>(bbox);
    const unsigned g = blocks_for(nclu, 256);
    const bool vec = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y) |
                       reinterpret_cast<uintptr_t>(z) | reinterpret_cast<uintptr_t>(h)) & 15u) == 0;
    hipStream_t st = ctx->stream;
    if (cs == 4) {
        if (vec) k_cluster_bbox<4, true><<<g, 256, 0, st>>>(n, x, y, z, h, b4, ctx->d_status, seg);
        else k_cluster_bbox<4, false><<<g, 256, 0, st>>>(n, x, y, z, h, b4, ctx->d_status, seg);
    } else if (cs == 16) {
        if (vec) k_cluster_bbox<16, true><<<g, 256, 0, st>>>(n, x, y, z, h, b4, ctx->d_status, seg);
        else k_cluster_bbox<16, false><<<g, 256, 0, st>>>(n, x, y, z, h, b4, ctx->d_status, seg);
    } else {
        if (vec) k_cluster_bbox<8, true><<<g, 256, 0, st>>>(n, x, y, z, h, b4, ctx->d_status, seg);
        else k_cluster_bbox<8, false><<<g, 256, 0, st>>>(n, x, y, z, h, b4, ctx->d_status, seg);
    }
    SFCNL_LAUNCHED(ctx);
    prof_mark(ctx, kStageClusters, true);
    return SFCNL_OK;
}

extern "C" int build_clusters(sfcnl_ctx ctx, int64_t n, const float *d_x, const float *d_y, const float *d_z,
                              const float *d_h, int cluster_size, float *d_bbox_out) {
    if (!ctx) return SFCNL_E_ARG;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "build_clusters: n out of range");
    if (cluster_size != 4 && cluster_size != 8 && cluster_size != 16)
        return set_err(ctx, SFCNL_E_ARG, "build_clusters: cluster_size %d not supported (4, 8, 16)", cluster_size);
    if (n == 0) return SFCNL_OK;
    if (!d_x || !d_y || !d_z || !d_h || !d_bbox_out) return set_err(ctx, SFCNL_E_ARG, "build_clusters: null pointer");
    return clusters_impl(ctx, n, d_x, d_y, d_z, d_h, cluster_size, d_bbox_out, SegTable{});
}

size_t sfcnl::nlist_ws_bytes(int64_t n, const sfcnl_nlist_opts &o, int nsys) {
    Carver cv{nullptr, 0};
    NlistWs ws;
    carve_nlist(cv, ws, n, o, nsys);
    return align_up(cv.used, 256) + 256;
}

extern "C" int build_nlist_workspace(int64_t n, const sfcnl_nlist_opts *opts, size_t *ws_bytes) {
    if (n < 0 || !ws_bytes || !opts || check_opts(nullptr, opts)) return SFCNL_E_ARG;
    *ws_bytes = nlist_ws_bytes(n, *opts, 1);
    return SFCNL_OK;
}

int sfcnl::read_status(sfcnl_ctx ctx) {
    SFCNL_HIP(ctx, hipMemcpyAsync(ctx->h_status, ctx->d_status, kStWords * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                  ctx->stream));
    SFCNL_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return SFCNL_OK;
}

sfcnl::ActiveWs sfcnl::nlist_ws_active(void *d_ws, int64_t n, const sfcnl_nlist_opts &o, int nsys) {
    Carver cv{reinterpret_cast<char *>(d_ws), 0};
    NlistWs ws;
    carve_nlist(cv, ws, n, o, nsys);
    return ActiveWs{ws.sc_active, ws.sc_scan, ws.p_active, ws.scan_tmp, ws.plist, ws.tree.cs_box, ws.tree.cs_rec,
                    ws.tree.node_cap};
}

int sfcnl::nlist_build_impl(sfcnl_ctx ctx, int64_t n, const uint64_t *d_keys, const float *d_x, const float *d_y,
                            const float *d_z, const float *d_h, const float *d_bbox, const sfcnl_nlist_opts &o,
                            void *d_ws, size_t ws_bytes, uint32_t *d_sc_info, uint32_t *d_pool, size_t pool_bytes,
                            const SegTable &seg, bool readback, size_t *h_used_bytes, int64_t *h_max_nj,
                            const uint32_t *active, const uint8_t *p_active, bool reuse_tree, const uint32_t *gate,
                            uint32_t gate_max) {
    if ((active || p_active) && o.half)
        return set_err(ctx, SFCNL_E_ARG, "build_nlist: a restricted rebuild needs the full list");
    const Period per = make_period(o.period);
    if (per.on() && seg.on()) return set_err(ctx, SFCNL_E_ARG, "batched lists take open boundaries only");
    const int nsys = seg.on() ? seg.nsys : 1;
    Carver cv{reinterpret_cast<char *>(d_ws), 0};
    NlistWs ws;
    carve_nlist(cv, ws, n, o, nsys);
    if (cv.used > ws_bytes) return set_err(ctx, SFCNL_E_ARG, "build_nlist: workspace %zu < %zu bytes", ws_bytes, cv.used);
    const uint32_t nsc = (uint32_t)((n + kScSize - 1) / kScSize);
    const int cs = o.cluster_size;
    const uint32_t nclu = (uint32_t)((n + cs - 1) / cs);
    hipStream_t st = ctx->stream;

    // the status words and stripe counters start at zero: cleared by the
    // octree's first launch, or by a fill when the tree is reused
    uint32_t *const st_clear = ctx->d_status + kStPoolOverflow;
    const int st_nclear = kStatusAlloc - kStPoolOverflow;
    int rc = SFCNL_OK;
    if (reuse_tree) {  // the tree of the previous build (same keys and bucket) serves
        rc = fill_u32(ctx, st_clear, st_nclear, 0);
        if (rc) return rc;
    } else {
        prof_mark(ctx, kStageOctree, false);
        rc = octree_build(ctx, ws.tree, d_keys, d_x, d_y, d_z, d_h, reinterpret_cast<const float4 *>(d_bbox), seg,
                          st_clear, st_nclear);
        if (rc) return rc;
        if (per.on()) {
            k_check_span<<<1, 1, 0, st>>>(ws.tree.cs_box, per, ctx->d_status);
            SFCNL_LAUNCHED(ctx);
        }
        prof_mark(ctx, kStageOctree, true);
    }

    TravArgs ta;
    ta.n = n;
    ta.nsc = nsc;
    ta.nclu = nclu;
    ta.compress = o.compress;
    ta.x = d_x;
    ta.y = d_y;
    ta.z = d_z;
    ta.h = d_h;
    ta.bbox = reinterpret_cast<const float4 *>(d_bbox);
    ta.cs_box = ws.tree.cs_box;
    ta.cs_rec = ws.tree.cs_rec;
    ta.nslots = ws.tree.node_cap;
    ta.seg = seg;
    ta.per = per;
    ta.active = active;
    ta.p_active = p_active;
    ta.gate = gate;
    ta.gate_max = gate_max;
    ta.list_j = ws.list_j;
    ta.list_m = ws.list_m;
    ta.chunk_next = ws.chunk_next;
    ta.nshared = ws.nchunks - nsc;
    ta.chunk_ctr = ctx->d_status + kStWords;
    ta.sc_nj = ws.sc_nj;
    ta.sc_words = ws.sc_words;
    ta.status = ctx->d_status;
    const unsigned gb = blocks_for(nsc, kWavesPerBlock);
    prof_mark(ctx, kStageTraverse, false);
    if (per.on())
        launch_traverse<true>(cs, o.half, gb, st, ta);
    else
        launch_traverse<false>(cs, o.half, gb, st, ta);
    SFCNL_LAUNCHED(ctx);
    prof_mark(ctx, kStageTraverse, true);
    prof_mark(ctx, kStageEncode, false);
    rc = scan_u32(ctx, ws.sc_words, ws.sc_off, nsc, ws.sc_off + nsc, ws.scan_tmp);
    if (rc) return rc;

    EncArgs ea;
    ea.nsc = nsc;
    ea.compress = o.compress;
    ea.mask_bytes = cs == 4 ? 2 : 1;
    ea.list_j = ws.list_j;
    ea.list_m = ws.list_m;
    ea.chunk_next = ws.chunk_next;
    ea.sc_nj = ws.sc_nj;
    ea.sc_off = ws.sc_off;
    ea.sc_info = d_sc_info;
    ea.pool = d_pool;
    ea.pool_words = pool_bytes / 4;
    ea.chunk_ctr = ctx->d_status + kStWords;
    ea.nshared = ws.nchunks - nsc;
    ea.status = ctx->d_status;
    k_encode<<<gb, kWave * kWavesPerBlock, 0, st>>>(ea);
    SFCNL_LAUNCHED(ctx);
    prof_mark(ctx, kStageEncode, true);
    if (!readback) return SFCNL_OK;

    rc = read_status(ctx);
    if (rc) return rc;
    return nlist_status(ctx, ctx->h_status, pool_bytes, o.max_j_per_sc, nsc, h_used_bytes, h_max_nj);
}

// Sizes and errors of a build from its copied status block.
int sfcnl::nlist_status(sfcnl_ctx ctx, const uint32_t *hs, size_t pool_bytes, int max_j_per_sc, uint32_t nsc,
                        size_t *h_used_bytes, int64_t *h_max_nj) {
    int rc;
    *h_used_bytes = (size_t)hs[kStTotalLo] * 4;
    *h_max_nj = hs[kStMaxNj];
    if (hs[kStInputErr]) {
        uint32_t e = hs[kStInputErr];
        rc = fill_u32(ctx, ctx->d_status + kStInputErr, 1, 0);
        if (rc) return rc;
        return set_err(ctx, SFCNL_E_INPUT,
                       "input error flags 0x%x (1: non-finite position, 2: bad radius, 4: bad permutation, "
                       "8: positions span a period or a radius reaches half of it)", e);
    }
    if (hs[kStTree]) return set_err(ctx, SFCNL_E_HIP, "internal error: octree invariant broken (0x%x)", hs[kStTree]);
    if (hs[kStScratch]) {
        *h_max_nj = staging_fit(hs, nsc);
        return set_err(ctx, SFCNL_E_CAPACITY, "staging list of max_j_per_sc %d too small: %lld holds the lists",
                       max_j_per_sc, (long long)*h_max_nj);
    }
    if (hs[kStPoolOverflow])
        return set_err(ctx, SFCNL_E_CAPACITY, "pool of %zu bytes < %zu needed", pool_bytes, *h_used_bytes);
    return SFCNL_OK;
}

extern "C" int build_nlist(sfcnl_ctx ctx, int64_t n, const uint64_t *d_keys, const float *d_x, const float *d_y,
                           const float *d_z, const float *d_h, const float *d_bbox, const sfcnl_nlist_opts *opts,
                           void *d_ws, size_t ws_bytes, uint32_t *d_sc_info, uint32_t *d_pool, size_t pool_bytes,
                           size_t *h_used_bytes, int64_t *h_max_nj) {
    if (!ctx) return SFCNL_E_ARG;
    int rc = check_opts(ctx, opts);
    if (rc) return rc;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "build_nlist: n out of range");
    if (!h_used_bytes || !h_max_nj) return set_err(ctx, SFCNL_E_ARG, "build_nlist: null result pointer");
    *h_used_bytes = 0;
    *h_max_nj = 0;
    if (n == 0) return SFCNL_OK;
    if (!d_keys || !d_x || !d_y || !d_z || !d_h || !d_bbox || !d_ws || !d_sc_info || (!d_pool && pool_bytes))
        return set_err(ctx, SFCNL_E_ARG, "build_nlist: null pointer");
    return nlist_build_impl(ctx, n, d_keys, d_x, d_y, d_z, d_h, d_bbox, *opts, d_ws, ws_bytes, d_sc_info, d_pool,
                            pool_bytes, SegTable{}, true, h_used_bytes, h_max_nj);
}

// The async build's status to the host: word k (zero when `zero`) with the
// build's number in the high half, as one 64-bit store (single-copy atomic),
// so the host knows each word's build without a fence between the stores.
// One wave.
__global__ void k_post_status(const uint32_t *__restrict__ status, uint64_t *out, uint32_t seq, int zero) {
    const int t = threadIdx.x;
    if (t < kStWords) {
        const uint32_t v = zero ? 0u : status[t];
        __hip_atomic_store(out + t, ((uint64_t)seq << 32) | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// The async build's bookkeeping: the status block posted behind the work
// (a kernel instead of a copy and an event, whose barrier would stall the
// stream), numbered so that the result call knows it when it arrives.
static int mark_pending(sfcnl_ctx ctx, int64_t n, const sfcnl_nlist_opts *opts, size_t pool_bytes) {
    ctx->pend_seq = ctx->pend_seq + 1u ? ctx->pend_seq + 1u : 1u;  // 0: nothing posted yet
    k_post_status<<<1, kWave, 0, ctx->stream>>>(ctx->d_status, ctx->d_pend, ctx->pend_seq, n > 0 ? 0 : 1);
    SFCNL_LAUNCHED(ctx);
    ctx->pend = 1;
    ctx->pend_pool_bytes = pool_bytes;
    ctx->pend_max_j = opts->max_j_per_sc;
    ctx->pend_nsc = (uint32_t)((n + kScSize - 1) / kScSize);
    return SFCNL_OK;
}

extern "C" int build_nlist_async(sfcnl_ctx ctx, int64_t n, const uint64_t *d_keys, const float *d_x,
                                 const float *d_y, const float *d_z, const float *d_h, const float *d_bbox,
                                 const sfcnl_nlist_opts *opts, void *d_ws, size_t ws_bytes, uint32_t *d_sc_info,
                                 uint32_t *d_pool, size_t pool_bytes) {
    if (!ctx) return SFCNL_E_ARG;
    ctx->pend = 0;
    int rc = check_opts(ctx, opts);
    if (rc) return rc;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "build_nlist_async: n out of range");
    if (n > 0 && (!d_keys || !d_x || !d_y || !d_z || !d_h || !d_bbox || !d_ws || !d_sc_info || (!d_pool && pool_bytes)))
        return set_err(ctx, SFCNL_E_ARG, "build_nlist_async: null pointer");
    if (n > 0) {
        size_t used;
        int64_t maxnj;
        rc = nlist_build_impl(ctx, n, d_keys, d_x, d_y, d_z, d_h, d_bbox, *opts, d_ws, ws_bytes, d_sc_info, d_pool,
                              pool_bytes, SegTable{}, false, &used, &maxnj);
        if (rc) return rc;
    }
    return mark_pending(ctx, n, opts, pool_bytes);
}

extern "C" int build_nlist_result(sfcnl_ctx ctx, size_t *h_used_bytes, int64_t *h_max_nj) {
    if (!ctx) return SFCNL_E_ARG;
    if (!h_used_bytes || !h_max_nj) return set_err(ctx, SFCNL_E_ARG, "build_nlist_result: null result pointer");
    *h_used_bytes = 0;
    *h_max_nj = 0;
    if (!ctx->pend) return set_err(ctx, SFCNL_E_ARG, "build_nlist_result: no build_nlist_async pending");
    ctx->pend = 0;
    // wait until every status word carries the build's number; every 256
    // rounds the stream's state is asked: an error ends the wait, and an idle
    // stream means the post has run (its stores are visible by then)
    const uint32_t seq = ctx->pend_seq;
    uint32_t hs[kStWords];
    for (uint32_t spin = 1;; spin++) {
        int have = 0;
        for (int k = 0; k < kStWords; k++) {
            const uint64_t v = __atomic_load_n(&ctx->h_pend[k], __ATOMIC_ACQUIRE);
            hs[k] = (uint32_t)v;
            have += (uint32_t)(v >> 32) == seq;
        }
        if (have == kStWords) break;
        if (spin % 256u) continue;
        const hipError_t e = hipStreamQuery(ctx->stream);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return set_err(ctx, SFCNL_E_HIP, "build_nlist_result: %s", hipGetErrorString(e));
        for (int k = 0; k < kStWords; k++) {
            const uint64_t v = __atomic_load_n(&ctx->h_pend[k], __ATOMIC_ACQUIRE);
            if ((uint32_t)(v >> 32) != seq)
                return set_err(ctx, SFCNL_E_HIP, "build_nlist_result: the stream is idle but the build's status did not arrive");
            hs[k] = (uint32_t)v;
        }
        break;
    }
    return nlist_status(ctx, hs, ctx->pend_pool_bytes, ctx->pend_max_j, ctx->pend_nsc, h_used_bytes, h_max_nj);
}
