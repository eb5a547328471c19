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
//     starting at that particle (the escape index);
//   * node boxes are refitted bottom-up, the last child to finish doing the
//     parent (atomic visit counters, no waiting).
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

__global__ __launch_bounds__(256) void k_digits(const uint64_t *__restrict__ keys, int64_t n, int bucket,
                                                int8_t *__restrict__ cdig, int8_t *__restrict__ lam) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint64_t k = keys[p];
    cdig[p] = (int8_t)(p == 0 ? -1 : sfc_common_digits(keys[p - 1], k));
    lam[p] = (int8_t)(p + bucket < n ? sfc_common_digits(k, keys[p + bucket]) : -1);
}

__global__ __launch_bounds__(256) void k_leaf_level(const int8_t *__restrict__ cdig, const int8_t *__restrict__ lam,
                                                    int64_t n, int bucket, int8_t *__restrict__ lleaf,
                                                    uint32_t *__restrict__ cnt) {
    __shared__ int8_t s_lam[256 + kMaxBucket];
    const int64_t b0 = (int64_t)blockIdx.x * 256;
    for (int k = threadIdx.x; k < 256 + bucket; k += 256) {
        int64_t a = b0 - bucket + k;
        s_lam[k] = (a >= 0 && a < n) ? lam[a] : (int8_t)-1;
    }
    __syncthreads();
    int64_t p = b0 + threadIdx.x;
    if (p >= n) return;
    int m = -1;
    for (int k = 0; k <= bucket; k++) {
        int v = s_lam[threadIdx.x + k];  // window start a = p - bucket + k
        m = v > m ? v : m;
    }
    int L = m + 1 < kMaxLevel ? m + 1 : kMaxLevel;
    int c = cdig[p];
    lleaf[p] = (int8_t)L;
    cnt[p] = c < L ? (uint32_t)(L - c) : 0u;
}

__global__ __launch_bounds__(256) void k_emit_nodes(const int8_t *__restrict__ cdig, const int8_t *__restrict__ lleaf,
                                                    const uint32_t *__restrict__ node_at, int64_t n, uint32_t cap,
                                                    uint32_t *__restrict__ nfirst, uint8_t *__restrict__ nlevel,
                                                    uint8_t *__restrict__ nleaf) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int c = cdig[p], L = lleaf[p];
    if (c >= L) return;
    uint32_t k = node_at[p];
    for (int l = c + 1; l <= L && k < cap; l++, k++) {
        nfirst[k] = (uint32_t)p;
        nlevel[k] = (uint8_t)l;
        nleaf[k] = (uint8_t)(l == L);
    }
}

__global__ __launch_bounds__(256) void k_node_range(const uint64_t *__restrict__ keys, int64_t n,
                                                    const uint32_t *__restrict__ node_at,
                                                    const uint32_t *__restrict__ d_nnodes, uint32_t cap,
                                                    const uint32_t *__restrict__ nfirst,
                                                    const uint8_t *__restrict__ nlevel, uint32_t *__restrict__ nend,
                                                    uint32_t *__restrict__ nesc, uint32_t *__restrict__ nvisit,
                                                    uint32_t *__restrict__ nparent, uint32_t *status) {
    const uint32_t nn = node_count(d_nnodes, cap);
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0 && *d_nnodes > cap) atomicOr(&status[kStTree], 1u);
    if (k >= nn) return;
    uint32_t f = nfirst[k];
    int L = nlevel[k];
    uint32_t end = (uint32_t)n;
    if (L > 0) {
        const int shift = 3 * (kMaxLevel - L);
        const uint64_t pre = keys[f] >> shift;
        uint32_t lo = f + 1, hi = (uint32_t)n;
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
    nvisit[k] = 0;
    nparent[k] = 0xFFFFFFFFu;
}

__global__ __launch_bounds__(256) void k_children(const uint32_t *__restrict__ d_nnodes, uint32_t cap,
                                                  const uint8_t *__restrict__ nleaf, const uint32_t *__restrict__ nesc,
                                                  uint32_t *__restrict__ nchild, uint8_t *__restrict__ nnchild,
                                                  uint32_t *__restrict__ nparent, uint32_t *status) {
    const uint32_t nn = node_count(d_nnodes, cap);
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    if (nleaf[k]) {
        nnchild[k] = 0;
        return;
    }
    uint32_t e = nesc[k], c = k + 1;
    int i = 0;
    while (c < e && i < 8) {
        nchild[8 * (size_t)k + i] = c;
        nparent[c] = k;
        i++;
        c = nesc[c];
    }
    if (c < e || i == 0) atomicOr(&status[kStTree], 2u);  // an octree node has 1..8 children
    nnchild[k] = (uint8_t)i;
}

__global__ __launch_bounds__(256) void k_refit(const uint32_t *__restrict__ d_nnodes, uint32_t cap,
                                               const uint8_t *__restrict__ nleaf,
                                               const uint32_t *__restrict__ nfirst, const uint32_t *__restrict__ nend,
                                               const uint32_t *__restrict__ nchild, const uint8_t *__restrict__ nnchild,
                                               const uint32_t *__restrict__ nparent, uint32_t *nvisit,
                                               const float *__restrict__ x, const float *__restrict__ y,
                                               const float *__restrict__ z, const float *__restrict__ h, float4 *nbox,
                                               uint32_t *status) {
    const uint32_t nn = node_count(d_nnodes, cap);
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn || !nleaf[k]) return;
    float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
    float4 hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
    for (uint32_t p = nfirst[k]; p < nend[k]; p++) {
        float px = x[p], py = y[p], pz = z[p], ph = h[p];
        lo.x = fminf(lo.x, px);
        lo.y = fminf(lo.y, py);
        lo.z = fminf(lo.z, pz);
        lo.w = fmaxf(lo.w, ph);
        hi.x = fmaxf(hi.x, px);
        hi.y = fmaxf(hi.y, py);
        hi.z = fmaxf(hi.z, pz);
    }
    nbox[2 * (size_t)k] = lo;
    nbox[2 * (size_t)k + 1] = hi;
    uint32_t c = k;
    while (c != 0) {
        __threadfence();
        uint32_t par = nparent[c];
        if (par >= nn) {  // every non-root node has a parent
            atomicOr(&status[kStTree], 4u);
            return;
        }
        uint32_t old = atomicAdd(&nvisit[par], 1u);
        if (old + 1 != nnchild[par]) return;  // a sibling finishes the parent
        __threadfence();
        float4 l = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
        float4 u = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
        for (int i = 0; i < nnchild[par]; i++) {
            uint32_t ch = nchild[8 * (size_t)par + i];
            const float4 a = nbox[2 * (size_t)ch];
            const float4 b = nbox[2 * (size_t)ch + 1];
            l.x = fminf(l.x, a.x);
            l.y = fminf(l.y, a.y);
            l.z = fminf(l.z, a.z);
            l.w = fmaxf(l.w, a.w);
            u.x = fmaxf(u.x, b.x);
            u.y = fmaxf(u.y, b.y);
            u.z = fmaxf(u.z, b.z);
        }
        nbox[2 * (size_t)par] = l;
        nbox[2 * (size_t)par + 1] = u;
        c = par;
    }
}

}  // namespace

static size_t node_capacity(int64_t n, int bucket) {
    // heavy cells of one level are disjoint and hold > bucket particles each;
    // levels 0..20 can be heavy and every node is a heavy cell or its child
    int64_t heavy = 21 * (n / (bucket + 1) + 1);
    int64_t cap = 9 * heavy + 2;
    int64_t lim = 22 * n + 2;
    return (size_t)(cap < lim ? cap : lim);
}

void octree_carve(Carver &cv, Octree &t, int64_t n, int bucket) {
    t.n = n;
    t.bucket = bucket;
    size_t nc = node_capacity(n, bucket);
    t.cdig = cv.take<int8_t>((size_t)n);
    t.lam = cv.take<int8_t>((size_t)n);
    t.lleaf = cv.take<int8_t>((size_t)n);
    t.node_at = cv.take<uint32_t>((size_t)n + 1);
    t.nfirst = cv.take<uint32_t>(nc);
    t.nend = cv.take<uint32_t>(nc);
    t.nesc = cv.take<uint32_t>(nc);
    t.nlevel = cv.take<uint8_t>(nc);
    t.nleaf = cv.take<uint8_t>(nc);
    t.nnchild = cv.take<uint8_t>(nc);
    t.nchild = cv.take<uint32_t>(8 * nc);
    t.nparent = cv.take<uint32_t>(nc);
    t.nvisit = cv.take<uint32_t>(nc);
    t.nbox = cv.take<float4>(2 * nc);
    t.d_nnodes = cv.take<uint32_t>(4);
    t.scan_tmp = cv.take<char>(scan_tmp_bytes(n + 1));
}

int octree_build(sfcnl_ctx ctx, Octree &t, const uint64_t *keys, const float *x, const float *y, const float *z,
                 const float *h) {
    const int64_t n = t.n;
    const int B = t.bucket;
    if (B < 1 || B > kMaxBucket) return set_err(ctx, SFCNL_E_ARG, "octree: bucket %d out of range", B);
    hipStream_t st = ctx->stream;
    const unsigned gp = blocks_for(n, 256);
    k_digits<<<gp, 256, 0, st>>>(keys, n, B, t.cdig, t.lam);
    SFCNL_LAUNCHED(ctx);
    uint32_t *cnt = t.node_at;  // counts, scanned in place
    k_leaf_level<<<gp, 256, 0, st>>>(t.cdig, t.lam, n, B, t.lleaf, cnt);
    SFCNL_LAUNCHED(ctx);
    int rc = scan_u32(ctx, cnt, t.node_at, n, t.d_nnodes, t.scan_tmp);
    if (rc) return rc;
    const uint32_t cap = (uint32_t)node_capacity(n, B);
    k_emit_nodes<<<gp, 256, 0, st>>>(t.cdig, t.lleaf, t.node_at, n, cap, t.nfirst, t.nlevel, t.nleaf);
    SFCNL_LAUNCHED(ctx);
    const unsigned gn = blocks_for((int64_t)cap, 256);
    k_node_range<<<gn, 256, 0, st>>>(keys, n, t.node_at, t.d_nnodes, cap, t.nfirst, t.nlevel, t.nend, t.nesc,
                                     t.nvisit, t.nparent, ctx->d_status);
    SFCNL_LAUNCHED(ctx);
    k_children<<<gn, 256, 0, st>>>(t.d_nnodes, cap, t.nleaf, t.nesc, t.nchild, t.nnchild, t.nparent, ctx->d_status);
    SFCNL_LAUNCHED(ctx);
    k_refit<<<gn, 256, 0, st>>>(t.d_nnodes, cap, t.nleaf, t.nfirst, t.nend, t.nchild, t.nnchild, t.nparent, t.nvisit,
                                x, y, z, h, t.nbox, ctx->d_status);
    SFCNL_LAUNCHED(ctx);
    return SFCNL_OK;
}

}  // namespace sfcnl
