// Internal declarations of the sfcnl GPU library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>

#include "sfcnl.h"

namespace sfcnl {

constexpr int kWave = 64;
constexpr int kScSize = SFCNL_SC_SIZE;   // particles per super-cluster
constexpr int kCs = 8;                   // default particles per cluster
constexpr int kMaxBoxLevels = 12;        // 8^12 clusters > 2^31 particles

// Status block words (device, mirrored into pinned host memory).
enum StatusWord : int {
    kStInputErr = 0,     // bit 0: non-finite coordinate, bit 1: bad radius, bit 3: period violated
    kStPoolOverflow = 1, // set if the pool is too small
    kStMaxNj = 2,        // largest list length (atomicMax)
    kStTotalLo = 3,      // total pool words (exclusive scan total)
    kStScratch = 4,      // set if a list found no staging room
    kStTree = 5,         // octree invariant broken (internal error)
    kStUnconverged = 6,  // h iteration: particles that moved this round
    kStChunks = 7,       // shared staging chunks the lists asked for (taken, plus requests left unserved)
    kStWords = 16
};

// Shared staging chunks are handed out by kChunkStripes counters that follow
// the status words in the same allocation, each on its own 128-byte line:
// stripe k gives out ids k, k + kChunkStripes, k + 2 kChunkStripes, ..., so
// that the super-clusters' requests spread over many addresses instead of
// queueing on one. Word 1 of a stripe's line holds the longest list among
// the super-clusters s with s % kChunkStripes = k.
constexpr int kChunkStripes = 64;
constexpr int kStripeWords = 32;
constexpr int kStatusAlloc = kStWords + kChunkStripes * kStripeWords;  // words of the device status allocation

}  // namespace sfcnl

struct sfcnl_ctx_s {
    int device;
    hipStream_t stream;
    uint32_t *d_status;
    uint32_t *h_status;
    char err[512];
    // build_nlist_async: the status block written behind the build by a
    // one-wave kernel into coherent pinned memory (d_pend is its device
    // view), each word as one 64-bit store with the build's number pend_seq
    // in the high half; and what the result call needs for its messages
    uint64_t *h_pend;
    uint64_t *d_pend;
    uint32_t pend_seq;
    int pend;
    size_t pend_pool_bytes;
    int pend_max_j;
    uint32_t pend_nsc;
    // waves (super-clusters) per block of the density passes (1, 2 or 4)
    int pass_waves;
    // device address of sfc_sort_noalloc's scratch array on this device
    void *d_sort_scratch;
    // stage timing (sfcnl_profile_begin / _end), for the stages in prof_mask
    int prof_slots;
    uint32_t prof_mask;
    int prof_used[SFCNL_NSTAGE];
    hipEvent_t *prof_ev[SFCNL_NSTAGE];  // 2 * prof_slots events per stage
};

namespace sfcnl {

int set_err(sfcnl_ctx ctx, int code, const char *fmt, ...);

#define SFCNL_HIP(ctx, call)                                                                   \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::sfcnl::set_err(ctx, SFCNL_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define SFCNL_LAUNCHED(ctx) SFCNL_HIP(ctx, hipGetLastError())

enum Stage : int { kStageKeys = 0, kStageSort, kStageGather, kStageClusters, kStageOctree, kStageTraverse,
                   kStageEncode, kStagePass };

// Brackets one stage of a call with events when profiling is on.
inline void prof_mark(sfcnl_ctx ctx, int stage, bool end) {
    if (!ctx->prof_slots || !((ctx->prof_mask >> stage) & 1u)) return;
    int k = ctx->prof_used[stage];
    if (k >= ctx->prof_slots) return;
    (void)hipEventRecord(ctx->prof_ev[stage][2 * k + (end ? 1 : 0)], ctx->stream);
    if (end) ctx->prof_used[stage] = k + 1;
}

inline unsigned blocks_for(int64_t n, int per_block) { return (unsigned)((n + per_block - 1) / per_block); }

constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Carves aligned sub-buffers out of a caller workspace.
struct Carver {
    char *base;
    size_t used;
    template <class T>
    T *take(size_t count) {
        used = align_up(used, 256);
        T *p = reinterpret_cast<T *>(base ? base + used : nullptr);
        used += count * sizeof(T);
        return p;
    }
};

// ---- device-wide exclusive scan of u32 (scan.hip) ----
size_t scan_tmp_bytes(int64_t n);
// out[i] = sum_{k<i} in[i]; *d_total = sum (may be null). in and out may alias.
int scan_u32(sfcnl_ctx ctx, const uint32_t *in, uint32_t *out, int64_t n, uint32_t *d_total, void *tmp);
// The same over the first min(*d_count, cap) words, the count known only on
// the device (one block; the scan ends at that count, later words untouched).
int scan_u32_dyn(sfcnl_ctx ctx, const uint32_t *in, uint32_t *out, const uint32_t *d_count, int64_t cap);
// Fills n u32 words with a value (a kernel, so it can sit inside a captured graph).
int fill_u32(sfcnl_ctx ctx, uint32_t *p, int64_t n, uint32_t v);
// The same over two arrays of n words in one launch (q may be null).
int fill2_u32(sfcnl_ctx ctx, uint32_t *p, uint32_t *q, int64_t n, uint32_t v);

// ---- batched systems ----
// Several independent systems laid out one after another from padded bases
// that are multiples of 64 particles (padding particles are NaN). All pointers
// are device pointers; a default-constructed table means one system.
struct SegTable {
    int nsys = 0;
    const uint16_t *sc_sys = nullptr;  // per super-cluster: its system
    const uint32_t *pbase = nullptr;   // nsys + 1 padded particle bases
    const uint32_t *count = nullptr;   // nsys real particle counts
    const float *edge = nullptr;       // nsys key-box edges (features)
    uint4 *roots = nullptr;            // nsys root records, written by the octree build
    __host__ __device__ bool on() const { return sc_sys != nullptr; }
};

// Periodic axes (Sec. II-A: periodic boundaries without shift vectors, the
// periodic distance of a pair computed whenever it is needed). L[a] is the
// period of axis a, +inf for an open axis, hL[a] = f32(L[a] / 2). A component
// difference d becomes its minimum image: d - L if d > L/2, d + L if d < -L/2
// (with L = +inf it stays d). Positions must lie within one period and radii
// below hmin, the smallest half period, so one image is the only candidate.
struct Period {
    float L[3] = {INFINITY, INFINITY, INFINITY};
    float hL[3] = {INFINITY, INFINITY, INFINITY};
    float hmin = INFINITY;
    __host__ __device__ bool on() const { return hmin < INFINITY; }
};
// period: 3 lengths (0 = open axis) or nullptr (all open); the caller has
// checked them (finite, >= 0)
Period make_period(const float *period);
bool period_ok(const float *period);

// d - L for d > L/2 and d + L for d < -L/2, as one subtraction of L with d's
// sign (the same FP32 operation either way).
__device__ __forceinline__ float min_image(float d, float L, float hL) {
    return fabsf(d) > hL ? d - copysignf(L, d) : d;
}

// Box of particle positions (a wave's i-particles, or a super-cluster in the
// traversal); absent particles, placed far away, make it huge.
struct IBox {
    float lo[3] = {0.0f, 0.0f, 0.0f}, hi[3] = {0.0f, 0.0f, 0.0f};
};
// True if the difference of j and some point of the box exceeds half a
// period on a periodic axis. FP32 subtraction is monotonic, so when it is
// false every pair of j with a particle inside the box has |fl(x_j - x_i)| at
// most half a period on every axis: its minimum image is the difference
// itself, and a batch of such j-particles can skip the wrap.
__device__ __forceinline__ bool far_from_box(float4 j, const IBox &b, const Period &p) {
    return fmaxf(fabsf(j.x - b.lo[0]), fabsf(j.x - b.hi[0])) > p.hL[0] ||
           fmaxf(fabsf(j.y - b.lo[1]), fabsf(j.y - b.hi[1])) > p.hL[1] ||
           fmaxf(fabsf(j.z - b.lo[2]), fabsf(j.z - b.hi[2])) > p.hL[2];
}

}  // namespace sfcnl

// A batch of independent systems (batch.hip). Input particles are the
// systems concatenated (system s at in_off[s]); the padded layout puts system
// s at pbase[s], a multiple of 64, followed by NaN padding up to pbase[s+1].
struct sfcnl_batch_s {
    int device;
    int nsys;
    int64_t n_in, n_pad;
    int64_t *h_in_off;   // nsys + 1
    int64_t *h_pbase;    // nsys + 1
    float *h_box;        // 6 per system
    // device tables
    uint16_t *d_sc_sys;      // n_pad / 64
    uint32_t *d_pbase;       // nsys + 1
    uint32_t *d_count;       // nsys
    uint32_t *d_in_off;      // nsys + 1
    float *d_edge;           // nsys: largest box side
    float *d_lo, *d_scale;   // 3 per system: key quantisation
    uint4 *d_roots;          // nsys
    uint32_t *d_sys_moved;   // nsys: particles moved in the last round
    uint32_t *h_sys_moved;   // pinned mirrors, one slot per round of a replay (kGraphRounds x nsys)
    uint32_t *h_rstat;       // pinned status blocks, one per round of a replay (kGraphRounds x kStWords)
    hipStream_t stream;      // capture stream (default priority)
    hipEvent_t ev_in, ev_out;
};

namespace sfcnl {

// Rounds of the batched h-iteration captured into one graph replay (the host
// reads their status blocks after the replay).
constexpr int kGraphRounds = 4;

inline SegTable seg_of(const sfcnl_batch_s *b) {
    SegTable t;
    t.nsys = b->nsys;
    t.sc_sys = b->d_sc_sys;
    t.pbase = b->d_pbase;
    t.count = b->d_count;
    t.edge = b->d_edge;
    t.roots = b->d_roots;
    return t;
}

// ---- pieces of build_nlist (octree.hip, traverse.hip) ----
struct Octree {
    int64_t n;
    int bucket;
    int cs;             // cluster size of the boxes the node boxes are built from
    uint32_t node_cap;  // capacity of the per-node and child-slot arrays
    // per particle
    int8_t *cdig;      // common 3-bit digits with the previous key (-1 for particle 0)
    int8_t *lleaf;     // octree level of the leaf holding p
    uint32_t *node_at; // index of the first node starting at particle p (leaf starts)
    uint32_t *blk;     // node counts per block of 256 particles, then their prefix sum
    // per node (capacity: a proven upper bound on the node count)
    uint32_t *nfirst, *nend, *nesc;
    uint8_t *nlevel, *nleaf, *nnchild;
    uint32_t *parent;  // parent node (roots: never read)
    uint8_t *pidx;     // index among the parent's children
    uint32_t *cbase;   // child counts, then their prefix sum: first child slot of each node, minus one
    float4 *cs_box;    // child slots: box of the child (2 per slot)
    uint4 *cs_rec;     // child slots: {first, end, child count, first child slot}
    // box hierarchy above the cluster boxes (groups of 8, 64, ... clusters)
    float4 *boxlvl[kMaxBoxLevels];
    int nboxlvl;
    uint32_t *d_nnodes;
    void *scan_tmp;
};

void octree_carve(Carver &cv, Octree &t, int64_t n, int bucket, int nsys, int cs);
// clear / nclear: device words the build's first launch zeroes on the way
// (counters of the caller that must start at zero), or none.
int octree_build(sfcnl_ctx ctx, Octree &t, const uint64_t *keys, const float *x, const float *y,
                 const float *z, const float *h, const float4 *cluster_box, const SegTable &seg,
                 uint32_t *clear = nullptr, int nclear = 0);
// The two halves of octree_build: the nodes, ranges and child slots from the
// sorted keys alone, then the node boxes from the cluster boxes and particles.
int octree_topology(sfcnl_ctx ctx, Octree &t, const uint64_t *keys, const SegTable &seg, uint32_t *clear = nullptr,
                    int nclear = 0);
int octree_geometry(sfcnl_ctx ctx, Octree &t, const float *x, const float *y, const float *z, const float *h,
                    const float4 *cluster_box, const SegTable &seg);

// build_nlist without argument checks; `readback` waits for the stream and
// reports capacity and input errors (otherwise the flags stay on the device).
size_t nlist_ws_bytes(int64_t n, const sfcnl_nlist_opts &o, int nsys);
// `active` (nullable, one flag per super-cluster): only super-clusters with a
// nonzero flag get a list (full lists only); the others get an empty one.
// `p_active` (nullable, one flag per particle): the lists count only the
// flagged particles' own-radius pairs (d2 < h_i^2), so boxes need no radii;
// `reuse_tree` keeps the octree of the previous build (same keys, bucket and
// cluster size: its positions and ranges are still exact).
// `gate` (device word, nullable): when *gate <= gate_max every super-cluster
// gets an empty list (the moved particles are recounted by count_moved_impl).
int nlist_build_impl(sfcnl_ctx ctx, int64_t n, const uint64_t *keys, const float *x, const float *y, const float *z,
                     const float *h, const float *bbox, const sfcnl_nlist_opts &o, void *ws, size_t ws_bytes,
                     uint32_t *sc_info, uint32_t *pool, size_t pool_bytes, const SegTable &seg, bool readback,
                     size_t *used_bytes, int64_t *max_nj, const uint32_t *active = nullptr,
                     const uint8_t *p_active = nullptr, bool reuse_tree = false, const uint32_t *gate = nullptr,
                     uint32_t gate_max = 0);
// arrays for restricted rebuilds inside a build_nlist workspace
struct ActiveWs {
    uint32_t *sc;      // per super-cluster: particles that moved
    uint32_t *scan;    // nsc + 1 words: exclusive prefix sum, then the total
    uint8_t *p;        // per particle: moved
    void *scan_tmp;
    uint32_t *plist;   // n words: the moved particles, in order
    const float4 *cs_box;  // the octree's child slots (boxes and records)
    const uint4 *cs_rec;
    uint32_t nslots;
};
// Recount of the moved particles without a list (h-iteration rounds after the
// first): compacts act.p into act.plist, then one wavefront per listed
// particle walks the octree of the last full build with the particle's own
// sphere and writes rho and nnb as the restricted pass would. With `gate`
// (device word, nullable) both kernels run only if *gate <= gate_max; the
// per-particle kernel grid is `blocks` workgroups of 4 waves.
int count_moved_impl(sfcnl_ctx ctx, int64_t n, const ActiveWs &act, const float *x, const float *y, const float *z,
                     const float *h, const float *m, float *rho, int32_t *nnb, const SegTable &seg, const Period &per,
                     const uint32_t *gate, uint32_t gate_max, unsigned blocks);
ActiveWs nlist_ws_active(void *ws, int64_t n, const sfcnl_nlist_opts &o, int nsys);
int clusters_impl(sfcnl_ctx ctx, int64_t n, const float *x, const float *y, const float *z, const float *h, int cs,
                  float *bbox, const SegTable &seg);
// `active` as for nlist_build_impl: the pass leaves rho and nnb of inactive
// super-clusters unchanged (full lists only).
int pass_impl(sfcnl_ctx ctx, int64_t n, int cs, int compress, int half, const uint32_t *sc_info, const uint32_t *pool,
              const float *x, const float *y, const float *z, const float *h, const float *m, float *rho, int32_t *nnb,
              const SegTable &seg, const Period &per, const uint32_t *active = nullptr,
              const uint8_t *p_active = nullptr, const uint32_t *gate = nullptr, uint32_t gate_max = 0);
int features_impl(sfcnl_ctx ctx, int64_t n, const uint64_t *keys, const float *x, const float *y, const float *z,
                  const float *h, const int32_t *nnb, float box_edge, int target, uint16_t *feat,
                  const SegTable &seg);
// reads the status block into pinned memory (kStWords words) and waits
int read_status(sfcnl_ctx ctx);
// Locates sfc_sort_noalloc's fixed device scratch array on the current device
// (once per device; sort.hip) and returns its device address in *ptr.
int sort_scratch_setup(int device, void **ptr);
// build_nlist's sizes and errors from a copied status block (hs)
// (nsc: super-clusters of the build; on a staging overflow *h_max_nj is the
// max_j_per_sc that holds every list)
int nlist_status(sfcnl_ctx ctx, const uint32_t *hs, size_t pool_bytes, int max_j_per_sc, uint32_t nsc,
                 size_t *h_used_bytes, int64_t *h_max_nj);
// The max_j_per_sc whose staging holds the lists of a build over nsc
// super-clusters that requested hs[kStChunks] shared chunks.
inline int64_t staging_fit(const uint32_t *hs, uint32_t nsc) {
    const uint64_t need = (uint64_t)nsc + hs[kStChunks];
    return (int64_t)((need + nsc - 1) / (nsc ? nsc : 1)) * kWave;
}

}  // namespace sfcnl

// ---------------------------------------------------------------------------
// Device helpers (wave64)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int sfc_lane() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t sfc_lt_mask() { return (1ull << sfc_lane()) - 1ull; }

__device__ __forceinline__ uint64_t sfc_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ int sfc_popc(uint64_t v) { return __popcll(v); }

// Uniform-lane read (index must be wave-uniform).
__device__ __forceinline__ uint32_t sfc_readlane(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

__device__ __forceinline__ float sfc_readlane_f(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ uint32_t sfc_incl_scan(uint32_t v) {
    const int l = sfc_lane();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (l >= d) v += t;
    }
    return v;
}

// Gap along one axis between two boxes (or a point and a box), from
// d1 = blo - ahi and d2 = alo - bhi (the separations of the direct images). On
// a periodic axis the gap is also taken to the images one period away,
// min(d1, d2) + L; both lie within one period, so no other image is closer.
// Every step rounds monotonically, so the gap never exceeds the |d| of a
// particle pair across the two after its minimum image is taken.
template <bool kPbc>
__device__ __forceinline__ float axis_gap(float d1, float d2, float L) {
    const float g = fmaxf(fmaxf(d1, d2), 0.0f);
    if (!kPbc) return g;
    return fminf(g, fmaxf(fminf(d1, d2) + L, 0.0f));
}

// Minimum images of a pair's components on periodic axes, skipped for the
// whole wave when no lane's component exceeds half its period (then none
// changes): only tiles that straddle a periodic face pay for the selects.
__device__ __forceinline__ void wave_min_image(float &dx, float &dy, float &dz, const sfcnl::Period &p) {
    const bool far = fabsf(dx) > p.hL[0] || fabsf(dy) > p.hL[1] || fabsf(dz) > p.hL[2];
    if (sfc_ballot(far)) {
        dx = sfcnl::min_image(dx, p.L[0], p.hL[0]);
        dy = sfcnl::min_image(dy, p.L[1], p.hL[1]);
        dz = sfcnl::min_image(dz, p.L[2], p.hL[2]);
    }
}

// Common leading 3-bit digits of two 63-bit keys (21 if equal).
__device__ __forceinline__ int sfc_common_digits(uint64_t a, uint64_t b) {
    uint64_t x = a ^ b;
    if (x == 0) return 21;
    return (__clzll((long long)x) - 1) / 3;
}
