// Octree over SFC-sorted Hilbert keys (Sec. II-A: the neighbour search walks
// the octree whose nodes are key-prefix cells, i.e. contiguous particle
// ranges).
//
// A cell is "heavy" if it holds more than `bucket` particles; the leaves are
// the light cells whose parent is heavy. Everything is derived in parallel
// from the sorted keys with a fixed number of launches:
//   * particle p lies in a heavy level-L cell iff some window of bucket+1
//     consecutive particles containing p shares its first L digits, so the
//     leaf level of p is 1 + max over the windows around p of their common
//     digit count (capped at the finest level, 21);
//   * a leaf starts at p iff p and p-1 differ in a digit above that level;
//   * the nodes beginning at a leaf start p are the cells of levels
//     (common digits with p-1, leaf level], so one prefix sum over particles
//     numbers all nodes in depth-first pre-order;
//   * a node's particle range ends at the first key leaving its cell (a
//     binary search), and the node after its subtree is the first node
//     starting at that particle (the escape index); the children of a node
//     are found by following escape indices from the next node.
// Node boxes are exact: the union over the node's particles, answered by a
// range query over a fixed hierarchy of boxes (clusters of 8 particles, then
// groups of 8 clusters, and so on): at most 7 ragged items per level and end.
#include "internal.h"

namespace sfcnl {
namespace {

constexpr int kMaxLevel = 21;
constexpr int kMaxBucket = 256;

// Node count, clamped to the arrays' capacity. The capacity is a proven upper
// bound, so the clamp only keeps a broken invariant from touching memory
// outside the arrays; it is reported through the status block.
__device__ __forceinline__ uint32_t node_count(const uint32_t *d_nnodes, uint32_t cap) {
    const uint32_t nn = *d_nnodes;
    return nn < cap ? nn : cap;
}

// Real particle range [lo, hi) of the system holding particle p (the whole
// array for one system); the padding after hi belongs to no node.
__device__ __forceinline__ void seg_range(const SegTable &seg, int64_t p, int64_t n, int64_t &lo, int64_t &hi) {
    if (seg.on()) {
        const int sy = seg.sc_sys[p / kScSize];
        lo = seg.pbase[sy];
        hi = lo + seg.count[sy];
    } else {
        lo = 0;
        hi = n;
    }
}

// lam(a) below: the common digits of key[a] and key[a + bucket] when both lie
// in a's system, else -1 (the window [a, a + bucket] is not one system's).

// Leaf level of particle p: one more than the largest lam over the bucket + 1
// windows [a, a + bucket] that hold p (a in [p - bucket, p]). The maximum over
// that sliding window comes from a doubling table in LDS: after the step of
// width d, entry k holds the largest of the d values from k on, and two
// overlapping runs of the largest width d <= bucket + 1 cover the window.
// A block takes kLeafPer consecutive groups of 256 particles, the keys they
// need staged once in LDS. Also writes the common digits with the previous key
// (cdig) and the node count of every group of 256 particles (nodes start at p
// for the levels (cdig, leaf level]). Block 0 also zeroes the nclear words at
// clear (the caller's counters that must start at zero; this saves their own
// launch).
constexpr int kLeafPer = 4;
constexpr int kLeafSpan = 256 * kLeafPer;

__global__ __launch_bounds__(256) void k_leaf_level(const uint64_t *__restrict__ keys, int64_t n, int bucket,
                                                    SegTable seg, int8_t *__restrict__ cdig,
                                                    int8_t *__restrict__ lleaf, uint32_t *__restrict__ blk,
                                                    uint32_t *__restrict__ clear, int nclear) {
    __shared__ uint64_t s_key[kLeafSpan + 2 * kMaxBucket];  // keys b0 - bucket .. b0 + span + bucket - 1
    __shared__ int8_t s_tab[2][kLeafSpan + kMaxBucket];  // bytes (measured faster than words)
    __shared__ uint32_t s_w[kLeafPer][256 / kWave];
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < nclear; k += 256) clear[k] = 0u;
    const int len = kLeafSpan + bucket;  // window starts b0 - bucket .. b0 + span - 1
    const int nkey = len + bucket;
    const int64_t b0 = (int64_t)blockIdx.x * kLeafSpan;
    // keys from clamped indices, loaded unconditionally (in flight together)
    {
        constexpr int kRounds = (kLeafSpan + 2 * kMaxBucket) / 256;
        uint64_t kv[kRounds];
#pragma unroll
        for (int r = 0; r < kRounds; r++) {
            const int64_t a = b0 - bucket + r * 256 + threadIdx.x;
            kv[r] = keys[a < 0 ? 0 : (a >= n ? n - 1 : a)];
        }
#pragma unroll
        for (int r = 0; r < kRounds; r++)
            if (r * 256 + (int)threadIdx.x < nkey) s_key[r * 256 + threadIdx.x] = kv[r];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < len; k += 256) {
        const int64_t a = b0 - bucket + k;
        int lam = -1;
        if (a >= 0 && a < n) {
            int64_t lo, hi;
            seg_range(seg, a, n, lo, hi);
            if (a < hi && a + bucket < hi) lam = sfc_common_digits(s_key[k], s_key[k + bucket]);
        }
        s_tab[0][k] = (int8_t)lam;
    }
    __syncthreads();
    const int win = bucket + 1;
    int d = 1, cur = 0;
    while (2 * d <= win) {
        // entries k with k + 2d <= len are exact; the rest are never read
        for (int k = threadIdx.x; k < len; k += 256) {
            const int u = s_tab[cur][k];
            const int v = k + d < len ? s_tab[cur][k + d] : -1;
            s_tab[cur ^ 1][k] = (int8_t)(u > v ? u : v);
        }
        __syncthreads();
        cur ^= 1;
        d *= 2;
    }
#pragma unroll
    for (int r = 0; r < kLeafPer; r++) {
        const int k = r * 256 + threadIdx.x;  // particle b0 + k; its window starts at table entry k
        const int64_t p = b0 + k;
        uint32_t cnt = 0;
        if (p < n) {
            int64_t lo, hi;
            seg_range(seg, p, n, lo, hi);  // systems never share a cell: each starts its own root
            int c, L;
            if (p >= hi) {  // padding: starts no node (cdig >= every leaf level)
                c = 127;
                L = 0;
            } else {
                c = p == lo ? -1 : sfc_common_digits(s_key[bucket + k - 1], s_key[bucket + k]);
                const int u = s_tab[cur][k], v = s_tab[cur][k + win - d];
                const int m = u > v ? u : v;
                L = m + 1 < kMaxLevel ? m + 1 : kMaxLevel;
                cnt = c < L ? (uint32_t)(L - c) : 0u;
            }
            cdig[p] = (int8_t)c;
            lleaf[p] = (int8_t)L;
        }
        // the group's total of the node counts
        const uint32_t tot = sfc_readlane(sfc_incl_scan(cnt), kWave - 1);
        if (sfc_lane() == 0) s_w[r][threadIdx.x / kWave] = tot;
    }
    __syncthreads();
    if (threadIdx.x < kLeafPer) {
        const int r = threadIdx.x;
        const int64_t g = (int64_t)blockIdx.x * kLeafPer + r;  // group of 256 particles
        if (g * 256 < n) blk[g] = s_w[r][0] + s_w[r][1] + s_w[r][2] + s_w[r][3];
    }
}

// Node numbers in depth-first pre-order: the prefix of the node counts over
// the particles (the block's offset from the scanned block totals, plus an
// exclusive scan inside the block). node_at[p] is the first node starting at
// p or after it; the nodes starting at p are written.
__global__ __launch_bounds__(256) void k_emit_nodes(const int8_t *__restrict__ cdig, const int8_t *__restrict__ lleaf,
                                                    const uint32_t *__restrict__ blk_off, int64_t n, uint32_t cap,
                                                    uint32_t *__restrict__ node_at, uint32_t *__restrict__ nfirst,
                                                    uint8_t *__restrict__ nlevel, uint8_t *__restrict__ nleaf) {
    __shared__ uint32_t s_w[256 / kWave];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int c = 0, L = 0;
    if (p < n) {
        c = cdig[p];
        L = lleaf[p];
    }
    const uint32_t cnt = c < L ? (uint32_t)(L - c) : 0u;
    const int lane = sfc_lane(), w = threadIdx.x / kWave;
    const uint32_t inc = sfc_incl_scan(cnt);
    if (lane == kWave - 1) s_w[w] = inc;
    __syncthreads();
    uint32_t before = blk_off[blockIdx.x];
    for (int k = 0; k < w; k++) before += s_w[k];
    uint32_t k = before + inc - cnt;
    if (p >= n) return;
    node_at[p] = k;
    for (int l = c + 1; l <= L && k < cap; l++, k++) {
        nfirst[k] = (uint32_t)p;
        nlevel[k] = (uint8_t)l;
        nleaf[k] = (uint8_t)(l == L);
    }
}

// Kernels over the nodes: the count is only known on the device, so a fixed
// grid strides over it.
constexpr unsigned kNodeGrid = 2048;

__global__ __launch_bounds__(256) void k_node_range(const uint64_t *__restrict__ keys, int64_t n,
                                                    const uint32_t *__restrict__ node_at,
                                                    const uint32_t *__restrict__ d_nnodes, uint32_t cap,
                                                    const uint32_t *__restrict__ nfirst,
                                                    const uint8_t *__restrict__ nlevel, uint32_t *__restrict__ nend,
                                                    uint32_t *__restrict__ nesc, uint32_t *status, SegTable seg) {
    const uint32_t nn = node_count(d_nnodes, cap);
    const uint32_t k0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (k0 == 0 && *d_nnodes > cap) atomicOr(&status[kStTree], 1u);
    for (uint32_t k = k0; k < nn; k += gridDim.x * blockDim.x) {
        uint32_t f = nfirst[k];
        int L = nlevel[k];
        int64_t slo, shi;
        seg_range(seg, f, n, slo, shi);
        uint32_t end = (uint32_t)shi;  // a root spans its whole system
        if (L > 0) {
            const int shift = 3 * (kMaxLevel - L);
            const uint64_t pre = keys[f] >> shift;
            uint32_t lo = f + 1, hi = (uint32_t)shi;
            while (lo < hi) {
                uint32_t mid = lo + (hi - lo) / 2;
                if ((keys[mid] >> shift) == pre)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            end = lo;
        }
        nend[k] = end;
        const uint32_t e = end == (uint32_t)n ? nn : node_at[end];
        nesc[k] = e < nn ? e : nn;
    }
}

// Children of every node (up to 8, in key order, by following escape indices
// from the next node): each child learns its parent and its index among the
// siblings; the parent's count goes to cbase for the prefix sum that places
// the children in child slots.
__global__ __launch_bounds__(256) void k_children(const uint32_t *__restrict__ d_nnodes, uint32_t cap,
                                                  const uint8_t *__restrict__ nleaf, const uint32_t *__restrict__ nesc,
                                                  uint32_t *__restrict__ parent, uint8_t *__restrict__ pidx,
                                                  uint8_t *__restrict__ nnchild, uint32_t *__restrict__ cbase,
                                                  uint32_t *status) {
    const uint32_t nn = node_count(d_nnodes, cap);
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nn; k += gridDim.x * blockDim.x) {
        if (nleaf[k]) {
            nnchild[k] = 0;
            cbase[k] = 0;
            continue;
        }
        uint32_t e = nesc[k], c = k + 1;
        int i = 0;
        while (c < e && i < 8) {
            parent[c] = k;
            pidx[c] = (uint8_t)i;
            i++;
            c = nesc[c];
        }
        if (c < e || i == 0) atomicOr(&status[kStTree], 2u);  // an octree node has 1..8 children
        nnchild[k] = (uint8_t)i;
        cbase[k] = (uint32_t)i;
    }
}

__device__ __forceinline__ void add_box(float4 &lo, float4 &hi, const float4 l, const float4 u) {
    lo.x = fminf(lo.x, l.x);
    lo.y = fminf(lo.y, l.y);
    lo.z = fminf(lo.z, l.z);
    lo.w = fmaxf(lo.w, l.w);
    hi.x = fmaxf(hi.x, u.x);
    hi.y = fmaxf(hi.y, u.y);
    hi.z = fmaxf(hi.z, u.z);
}

// Up to three levels of the box hierarchy in one launch: box b of a level =
// the union of boxes 8b .. 8b+7 of the level below. Each thread forms one box
// of the first level from `below`; the block's first 32 threads then join
// each 8 of those (from LDS) into the second level, and its first 4 threads
// into the third (a block covers 256 boxes of the first level, so 32 of the
// second and 4 of the third; boxes past a level's end are empty and join as
// no-ops). nlev (1..3) levels are written.
__global__ __launch_bounds__(256) void k_box_levels(const float4 *__restrict__ below, int64_t nbelow, int nlev,
                                                    float4 *__restrict__ l1, int64_t n1, float4 *__restrict__ l2,
                                                    int64_t n2, float4 *__restrict__ l3, int64_t n3) {
    __shared__ float4 s_lo[256], s_hi[256];
    const int t = threadIdx.x;
    const int64_t b = (int64_t)blockIdx.x * 256 + t;
    float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
    float4 hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
    if (b < n1) {
        for (int64_t c = 8 * b; c < 8 * b + 8 && c < nbelow; c++) add_box(lo, hi, below[2 * c], below[2 * c + 1]);
        l1[2 * b] = lo;
        l1[2 * b + 1] = hi;
    }
    if (nlev < 2) return;
    s_lo[t] = lo;
    s_hi[t] = hi;
    __syncthreads();
    float4 l2o = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
    float4 h2o = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
    if (t < 32) {
        for (int k = 0; k < 8; k++) add_box(l2o, h2o, s_lo[8 * t + k], s_hi[8 * t + k]);
        const int64_t a = (int64_t)blockIdx.x * 32 + t;
        if (a < n2) {
            l2[2 * a] = l2o;
            l2[2 * a + 1] = h2o;
        }
    }
    if (nlev < 3) return;
    __syncthreads();
    if (t < 32) {
        s_lo[t] = l2o;
        s_hi[t] = h2o;
    }
    __syncthreads();
    if (t < 4) {
        float4 l3o = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
        float4 h3o = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
        for (int k = 0; k < 8; k++) add_box(l3o, h3o, s_lo[8 * t + k], s_hi[8 * t + k]);
        const int64_t a = (int64_t)blockIdx.x * 4 + t;
        if (a < n3) {
            l3[2 * a] = l3o;
            l3[2 * a + 1] = h3o;
        }
    }
}

struct BoxLevels {
    const float4 *lvl[kMaxBoxLevels + 1];  // lvl[0] = cluster boxes (cs particles each)
    int nlvl;
    int cshift;  // log2 of the cluster size
};

// Exact box of every node (the union over its particles, answered by a range
// query over the box hierarchy: ragged particles at both ends, then whole
// groups coarsening one level at a time), written with the node's record
// {first, end, child count (0 = leaf), first child slot} into the node's own
// child slot: slot 0 for the root, 1 + cbase[parent] + index among the
// parent's children otherwise (other systems' roots have no slot; their
// records are kept apart). The traversal reads everything about a child with
// one round trip.
//
// A node's range [first, end) leaves, at level l (level 0: particles; level
// l >= 1: the boxes of L.lvl[l - 1], each covering 2^sh particles), the whole
// units [A, B) with A = ceil(first / 2^sh) and B = floor(end / 2^sh); of
// these, the level takes the ragged ones at both ends (those whose unit of
// the next level is not whole inside), and the coarsest level takes them
// all. So every (level, end) part is known up front: 16 lanes share a node,
// lane q taking the parts q, q + 16, ... (part 2l + e: level l, end e), with
// its loads issued together, and the lanes then join their boxes. Minimum
// and maximum are exact and idempotent, so neither the order of the joins
// nor the repeats of a clamped index change the box.
constexpr int kSlotLanes = 16;

__global__ __launch_bounds__(256) void k_node_slots(const uint32_t *__restrict__ d_nnodes, uint32_t cap,
                                                    const uint32_t *__restrict__ nfirst,
                                                    const uint32_t *__restrict__ nend,
                                                    const uint8_t *__restrict__ nlevel,
                                                    const uint8_t *__restrict__ nnchild,
                                                    const uint32_t *__restrict__ parent,
                                                    const uint8_t *__restrict__ pidx, const uint32_t *__restrict__ cbase,
                                                    const float *__restrict__ x, const float *__restrict__ y,
                                                    const float *__restrict__ z, const float *__restrict__ h,
                                                    BoxLevels L, float4 *__restrict__ cs_box,
                                                    uint4 *__restrict__ cs_rec) {
    const uint32_t nn = node_count(d_nnodes, cap);
    const int q = threadIdx.x % kSlotLanes;
    const uint32_t gstride = gridDim.x * (blockDim.x / kSlotLanes);
    // a node's lanes share k and so every branch below
    for (uint32_t k = (blockIdx.x * blockDim.x + threadIdx.x) / kSlotLanes; k < nn; k += gstride) {
        uint32_t slot;
        if (nlevel[k] == 0) {
            if (k != 0) continue;  // another system's root
            slot = 0;
        } else {
            slot = 1u + cbase[parent[k]] + pidx[k];
            if (slot >= cap) continue;  // only on a broken tree (reported elsewhere)
        }
        const uint32_t first = nfirst[k], end = nend[k];
        float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
        float4 hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
        for (int part = q; part < 2 * (L.nlvl + 1); part += kSlotLanes) {
            const int l = part >> 1;
            const int sh = l == 0 ? 0 : L.cshift + 3 * (l - 1);
            const uint64_t A = ((uint64_t)first + ((1ull << sh) - 1ull)) >> sh;
            const uint64_t B = (uint64_t)end >> sh;
            if (A >= B) continue;
            // the ragged units: [A, f) at the front, [b, B) at the back
            uint64_t i0, i1;
            if (l == L.nlvl) {  // the coarsest level takes all (with the front part)
                i0 = A;
                i1 = (part & 1) ? A : B;
            } else {
                const uint64_t m = l == 0 ? (1ull << L.cshift) - 1ull : 7ull;
                const uint64_t f = ((A + m) & ~m) < B ? (A + m) & ~m : B;
                const uint64_t b = (B & ~m) > f ? B & ~m : f;
                i0 = (part & 1) ? b : A;
                i1 = (part & 1) ? B : f;
            }
            if (l == 0) {
                for (uint64_t t0 = i0; t0 < i1; t0 += 4) {
                    float px[4], py[4], pz[4], ph[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const uint64_t t = t0 + u < i1 ? t0 + u : i1 - 1;
                        px[u] = x[t];
                        py[u] = y[t];
                        pz[u] = z[t];
                        ph[u] = h[t];
                    }
#pragma unroll
                    for (int u = 0; u < 4; u++)
                        add_box(lo, hi, make_float4(px[u], py[u], pz[u], ph[u]), make_float4(px[u], py[u], pz[u], 0.0f));
                }
            } else {
                const float4 *bx = L.lvl[l - 1];
                for (uint64_t t0 = i0; t0 < i1; t0 += 4) {
                    float4 bl[4], bh[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const uint64_t t = t0 + u < i1 ? t0 + u : i1 - 1;
                        bl[u] = bx[2 * t];
                        bh[u] = bx[2 * t + 1];
                    }
#pragma unroll
                    for (int u = 0; u < 4; u++) add_box(lo, hi, bl[u], bh[u]);
                }
            }
        }
        // join the lanes' boxes (groups of kSlotLanes aligned lanes)
#pragma unroll
        for (int d = 1; d < kSlotLanes; d <<= 1) {
            lo.x = fminf(lo.x, __shfl_xor(lo.x, d, kSlotLanes));
            lo.y = fminf(lo.y, __shfl_xor(lo.y, d, kSlotLanes));
            lo.z = fminf(lo.z, __shfl_xor(lo.z, d, kSlotLanes));
            lo.w = fmaxf(lo.w, __shfl_xor(lo.w, d, kSlotLanes));
            hi.x = fmaxf(hi.x, __shfl_xor(hi.x, d, kSlotLanes));
            hi.y = fmaxf(hi.y, __shfl_xor(hi.y, d, kSlotLanes));
            hi.z = fmaxf(hi.z, __shfl_xor(hi.z, d, kSlotLanes));
        }
        if (q == 0) {
            cs_box[2 * (size_t)slot] = lo;
            cs_box[2 * (size_t)slot + 1] = hi;
            cs_rec[slot] = make_uint4(first, end, nnchild[k], 1u + cbase[k]);
        }
    }
}

// Root record of every system (the level-0 node at its first particle).
__global__ void k_roots(SegTable seg, const uint32_t *__restrict__ node_at, const uint32_t *__restrict__ nfirst,
                        const uint32_t *__restrict__ nend, const uint8_t *__restrict__ nnchild,
                        const uint32_t *__restrict__ cbase, const uint32_t *__restrict__ d_nnodes, uint32_t cap) {
    const int sy = blockIdx.x * blockDim.x + threadIdx.x;
    if (sy >= seg.nsys) return;
    const uint32_t nn = node_count(d_nnodes, cap);
    const uint32_t p = seg.pbase[sy];
    uint4 r = make_uint4(p, p, 0u, 0u);  // empty system: no super-cluster ever reads it
    if (seg.count[sy] > 0) {
        const uint32_t k = node_at[p];
        if (k < nn) r = make_uint4(nfirst[k], nend[k], nnchild[k], 1u + cbase[k]);
    }
    seg.roots[sy] = r;
}

}  // namespace

static size_t node_capacity(int64_t n, int bucket, int nsys) {
    // heavy cells of one level are disjoint and hold > bucket particles each;
    // levels 0..20 can be heavy and every node is a heavy cell or its child
    int64_t heavy = 21 * (n / (bucket + 1) + nsys);
    int64_t cap = 9 * heavy + 2;
    int64_t lim = 22 * n + 2 * nsys;
    return (size_t)(cap < lim ? cap : lim);
}

// Sizes of the box hierarchy above the cluster boxes: level 1 groups 8
// clusters, level 2 groups 8 of those, ... until one box remains.
static int box_levels(int64_t n, int cs, int64_t *sizes) {
    int64_t m = (n + cs - 1) / cs;
    int nl = 0;
    while (m > 1 && nl < kMaxBoxLevels) {
        m = (m + 7) / 8;
        sizes[nl++] = m;
    }
    return nl;
}

// Grid of the kernels over nodes (they stride over the device-side count).
static unsigned node_grid(const Octree &t) {
    const unsigned g = blocks_for((int64_t)t.node_cap, 256);
    return g < kNodeGrid ? g : kNodeGrid;
}

void octree_carve(Carver &cv, Octree &t, int64_t n, int bucket, int nsys, int cs) {
    t.n = n;
    t.bucket = bucket;
    t.cs = cs;
    size_t nc = node_capacity(n, bucket, nsys);
    t.node_cap = (uint32_t)nc;
    t.cdig = cv.take<int8_t>((size_t)n);
    t.lleaf = cv.take<int8_t>((size_t)n);
    t.node_at = cv.take<uint32_t>((size_t)n + 1);
    t.blk = cv.take<uint32_t>((size_t)blocks_for(n, 256) + 1);
    t.nfirst = cv.take<uint32_t>(nc);
    t.nend = cv.take<uint32_t>(nc);
    t.nesc = cv.take<uint32_t>(nc);
    t.nlevel = cv.take<uint8_t>(nc);
    t.nleaf = cv.take<uint8_t>(nc);
    t.nnchild = cv.take<uint8_t>(nc);
    t.parent = cv.take<uint32_t>(nc);
    t.pidx = cv.take<uint8_t>(nc);
    t.cbase = cv.take<uint32_t>(nc);
    t.cs_box = cv.take<float4>(2 * nc);
    t.cs_rec = cv.take<uint4>(nc);
    int64_t sizes[kMaxBoxLevels];
    t.nboxlvl = box_levels(n, cs, sizes);
    for (int l = 0; l < t.nboxlvl; l++) t.boxlvl[l] = cv.take<float4>(2 * (size_t)sizes[l]);
    t.d_nnodes = cv.take<uint32_t>(4);
    t.scan_tmp = cv.take<char>(scan_tmp_bytes((int64_t)blocks_for(n, 256) + 1));
}

int octree_topology(sfcnl_ctx ctx, Octree &t, const uint64_t *keys, const SegTable &seg, uint32_t *clear, int nclear) {
    const int64_t n = t.n;
    const int B = t.bucket;
    if (B < 1 || B > kMaxBucket) return set_err(ctx, SFCNL_E_ARG, "octree: bucket %d out of range", B);
    hipStream_t st = ctx->stream;
    const unsigned gp = blocks_for(n, 256);
    // leaf levels and per-block node counts, their prefix sum (the total is
    // the node count), then the nodes in depth-first pre-order
    k_leaf_level<<<blocks_for(n, kLeafSpan), 256, 0, st>>>(keys, n, B, seg, t.cdig, t.lleaf, t.blk, clear,
                                                          clear ? nclear : 0);
    SFCNL_LAUNCHED(ctx);
    int rc = scan_u32(ctx, t.blk, t.blk, (int64_t)gp, t.d_nnodes, t.scan_tmp);
    if (rc) return rc;
    const uint32_t cap = t.node_cap;
    k_emit_nodes<<<gp, 256, 0, st>>>(t.cdig, t.lleaf, t.blk, n, cap, t.node_at, t.nfirst, t.nlevel, t.nleaf);
    SFCNL_LAUNCHED(ctx);
    // the node count is only known on the device: a fixed grid strides over it
    const unsigned gn = node_grid(t);
    k_node_range<<<gn, 256, 0, st>>>(keys, n, t.node_at, t.d_nnodes, cap, t.nfirst, t.nlevel, t.nend, t.nesc,
                                     ctx->d_status, seg);
    SFCNL_LAUNCHED(ctx);
    k_children<<<gn, 256, 0, st>>>(t.d_nnodes, cap, t.nleaf, t.nesc, t.parent, t.pidx, t.nnchild, t.cbase,
                                   ctx->d_status);
    SFCNL_LAUNCHED(ctx);
    // contiguous child slots: prefix sum of the child counts over the nodes
    return scan_u32_dyn(ctx, t.cbase, t.cbase, t.d_nnodes, (int64_t)cap);
}

int octree_geometry(sfcnl_ctx ctx, Octree &t, const float *x, const float *y, const float *z, const float *h,
                    const float4 *cluster_box, const SegTable &seg) {
    const int64_t n = t.n;
    hipStream_t st = ctx->stream;
    const uint32_t cap = t.node_cap;
    const unsigned gn = node_grid(t);
    // box hierarchy over the cluster boxes (three levels per launch), then the
    // exact node boxes and records in their slots
    int64_t sizes[kMaxBoxLevels];
    const int nl = box_levels(n, t.cs, sizes);
    BoxLevels L;
    L.lvl[0] = cluster_box;
    L.nlvl = nl + 1;
    L.cshift = t.cs == 4 ? 2 : (t.cs == 16 ? 4 : 3);
    int64_t below = (n + t.cs - 1) / t.cs;
    for (int l = 0; l < nl;) {
        const int nlev = nl - l < 3 ? nl - l : 3;
        k_box_levels<<<blocks_for(sizes[l], 256), 256, 0, st>>>(
            L.lvl[l], below, nlev, t.boxlvl[l], sizes[l], nlev > 1 ? t.boxlvl[l + 1] : nullptr,
            nlev > 1 ? sizes[l + 1] : 0, nlev > 2 ? t.boxlvl[l + 2] : nullptr, nlev > 2 ? sizes[l + 2] : 0);
        SFCNL_LAUNCHED(ctx);
        for (int k = 0; k < nlev; k++) L.lvl[l + 1 + k] = t.boxlvl[l + k];
        below = sizes[l + nlev - 1];
        l += nlev;
    }
    // kSlotLanes lanes per node: a grid of twice the node kernels' blocks
    k_node_slots<<<2 * gn, 256, 0, st>>>(t.d_nnodes, cap, t.nfirst, t.nend, t.nlevel, t.nnchild, t.parent, t.pidx,
                                     t.cbase, x, y, z, h, L, t.cs_box, t.cs_rec);
    SFCNL_LAUNCHED(ctx);
    if (seg.on()) {
        k_roots<<<blocks_for(seg.nsys, 64), 64, 0, st>>>(seg, t.node_at, t.nfirst, t.nend, t.nnchild, t.cbase,
                                                         t.d_nnodes, cap);
        SFCNL_LAUNCHED(ctx);
    }
    return SFCNL_OK;
}

int octree_build(sfcnl_ctx ctx, Octree &t, const uint64_t *keys, const float *x, const float *y, const float *z,
                 const float *h, const float4 *cluster_box, const SegTable &seg, uint32_t *clear, int nclear) {
    const int rc = octree_topology(ctx, t, keys, seg, clear, nclear);
    if (rc) return rc;
    return octree_geometry(ctx, t, x, y, z, h, cluster_box, seg);
}

}  // namespace sfcnl
