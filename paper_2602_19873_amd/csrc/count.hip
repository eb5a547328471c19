// Recount of the particles whose radius moved in an h-iteration round,
// without a list. A particle's own-radius count depends on its radius alone,
// so after the first round only the moved particles need new counts; when
// few moved, building their super-clusters' lists leaves most of the GPU
// idle while one wavefront walks a large sphere. Here every moved particle
// gets a wavefront of its own: it walks the octree of the last full build
// (positions and key ranges are unchanged) with its own sphere, pushing the
// children whose boxes come within its radius, and at a leaf tests the
// leaf's particles 64 at a time with the exact FP32 pair formula. Counts are
// exact and densities are the sums of the restricted pass in another order.
#include "internal.h"

namespace sfcnl {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kStackCap = 160;  // 1 + 7 * 21 pushes at most

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Writes the moved particles of super-cluster s to plist[off[s] + rank].
__global__ __launch_bounds__(256) void k_compact_moved(int64_t n, const uint32_t *__restrict__ cnt,
                                                       const uint32_t *__restrict__ off,
                                                       const uint8_t *__restrict__ moved, uint32_t *__restrict__ plist,
                                                       const uint32_t *gate, uint32_t gate_max) {
    const int lane = sfc_lane();
    const uint32_t s = (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave));
    const uint32_t nsc = (uint32_t)((n + kScSize - 1) / kScSize);
    if (s >= nsc || (gate && *gate > gate_max) || cnt[s] == 0) return;
    const int64_t i = (int64_t)s * kScSize + lane;
    const bool f = i < n && moved[i] != 0;
    const uint64_t b = sfc_ballot(f);
    if (f) plist[off[s] + (uint32_t)sfc_popc(b & sfc_lt_mask())] = (uint32_t)i;
}

struct CountArgs {
    int64_t n;
    const uint32_t *plist;
    const uint32_t *total;  // listed particles (device word)
    const uint32_t *gate;   // nullable: run only if *gate <= gate_max
    uint32_t gate_max;
    const float *x, *y, *z, *h, *m;
    const float4 *cs_box;   // octree child slots (slot 0 = root)
    const uint4 *cs_rec;
    uint32_t nslots;
    SegTable seg;
    Period per;
    float *rho;
    int32_t *nnb;
    uint32_t *status;
};

// One wavefront per listed particle, waves striding over the list.
template <bool kMass, bool kPbc>
__global__ __launch_bounds__(256) void k_count_moved(CountArgs a) {
    __shared__ uint4 s_stack[kWavesPerBlock][kStackCap];
    const int lane = sfc_lane();
    const int w = threadIdx.x / kWave;
    if (a.gate && *a.gate > a.gate_max) return;
    const uint32_t total = *a.total;
    const uint32_t nw = gridDim.x * kWavesPerBlock;
    uint4 *stack = s_stack[w];
    for (uint32_t t = blockIdx.x * kWavesPerBlock + w; t < total; t += nw) {
        const uint32_t i = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.plist[t]);
        const float xi = a.x[i], yi = a.y[i], zi = a.z[i], hi = a.h[i];
        const float h2 = hi * hi;
        const float hinv = 1.0f / hi;
        float acc = 0.0f;  // m_j times the halved spline shape, summed
        uint32_t cnt = 0;
        wave_sync();  // the previous particle's last stack reads are done
        if (lane == 0) stack[0] = a.seg.on() ? a.seg.roots[a.seg.sc_sys[i / kScSize]] : a.cs_rec[0];
        int sp = 1;
        wave_sync();
        while (sp > 0) {
            sp--;
            const uint4 rv = stack[sp];
            const uint32_t nfirst = (uint32_t)__builtin_amdgcn_readfirstlane((int)rv.x);
            const uint32_t nend = (uint32_t)__builtin_amdgcn_readfirstlane((int)rv.y);
            const uint32_t nchild = (uint32_t)__builtin_amdgcn_readfirstlane((int)rv.z);
            const uint32_t cslot = (uint32_t)__builtin_amdgcn_readfirstlane((int)rv.w);
            if (nend > (uint64_t)a.n || nfirst >= nend || cslot + nchild > a.nslots) {  // only on a broken tree
                if (lane == 0) atomicOr(&a.status[kStTree], 16u);
                break;
            }
            if (nchild == 0) {
                for (uint32_t p0 = nfirst; p0 < nend; p0 += kWave) {
                    const uint32_t j = p0 + (uint32_t)lane;
                    const bool v = j < nend;
                    float dx = v ? a.x[j] - xi : 0.0f;
                    float dy = v ? a.y[j] - yi : 0.0f;
                    float dz = v ? a.z[j] - zi : 0.0f;
                    if (kPbc) wave_min_image(dx, dy, dz, a.per);
                    const float dxx = dx * dx;
                    const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
                    const bool in = v && j != i && d2 < h2;
                    const uint64_t bal = sfc_ballot(in);
                    if (bal) {
                        cnt += (uint32_t)sfc_popc(bal);
                        const float q = __builtin_amdgcn_sqrtf(d2) * hinv;
                        const float t1 = q - 1.0f;
                        const float q2 = q * q;
                        const float inner = __builtin_fmaf(3.0f * q2, t1, 0.5f);
                        const float outer = -(t1 * t1) * t1;
                        const float wq = q < 0.5f ? inner : outer;
                        const float mj = kMass ? (in ? a.m[j] : 0.0f) : 1.0f;
                        acc = in ? __builtin_fmaf(mj, wq, acc) : acc;
                    }
                }
            } else {
                // lane jl < nchild tests child jl against the particle's sphere
                const int jl = lane;
                bool hit = false;
                uint4 crec = make_uint4(0u, 0u, 0u, 0u);
                if (jl < (int)nchild) {
                    const uint32_t slot = cslot + (uint32_t)jl;
                    const float4 lo = a.cs_box[2 * (size_t)slot], hb = a.cs_box[2 * (size_t)slot + 1];
                    crec = a.cs_rec[slot];
                    const float gx = axis_gap<kPbc>(lo.x - xi, xi - hb.x, a.per.L[0]);
                    const float gy = axis_gap<kPbc>(lo.y - yi, yi - hb.y, a.per.L[1]);
                    const float gz = axis_gap<kPbc>(lo.z - zi, zi - hb.z, a.per.L[2]);
                    const float gxx = gx * gx;
                    hit = __builtin_fmaf(gz, gz, __builtin_fmaf(gy, gy, gxx)) < h2;
                }
                const uint64_t keep = sfc_ballot(hit);
                const int c = sfc_popc(keep);
                if (sp + c > kStackCap) {  // cannot happen in a valid octree (depth <= 21)
                    if (lane == 0) atomicOr(&a.status[kStTree], 8u);
                    break;
                }
                if (hit) stack[sp + sfc_popc(keep & sfc_lt_mask())] = crec;
                sp += c;
                wave_sync();
            }
        }
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) acc += __shfl_xor(acc, d, 64);
        if (lane == 0) {
            const float norm = 2.5464790894703255f * hinv * hinv * hinv;  // 8 / pi
            a.rho[i] = norm * __builtin_fmaf(2.0f, acc, kMass ? a.m[i] : 1.0f);
            a.nnb[i] = (int32_t)cnt;
        }
    }
}

}  // namespace
}  // namespace sfcnl

using namespace sfcnl;

int sfcnl::count_moved_impl(sfcnl_ctx ctx, int64_t n, const ActiveWs &act, const float *x, const float *y,
                            const float *z, const float *h, const float *m, float *rho, int32_t *nnb,
                            const SegTable &seg, const Period &per, const uint32_t *gate, uint32_t gate_max,
                            unsigned blocks) {
    if (n == 0) return SFCNL_OK;
    const uint32_t nsc = (uint32_t)((n + kScSize - 1) / kScSize);
    hipStream_t st = ctx->stream;
    prof_mark(ctx, kStagePass, false);
    k_compact_moved<<<blocks_for(nsc, kWavesPerBlock), 256, 0, st>>>(n, act.sc, act.scan, act.p, act.plist, gate,
                                                                     gate_max);
    SFCNL_LAUNCHED(ctx);
    CountArgs a{n, act.plist, act.scan + nsc, gate, gate_max, x, y, z, h, m, act.cs_box, act.cs_rec, act.nslots,
                seg, per, rho, nnb, ctx->d_status};
    const unsigned g = blocks ? blocks : 1u;
    if (per.on()) {
        if (m)
            k_count_moved<true, true><<<g, 256, 0, st>>>(a);
        else
            k_count_moved<false, true><<<g, 256, 0, st>>>(a);
    } else {
        if (m)
            k_count_moved<true, false><<<g, 256, 0, st>>>(a);
        else
            k_count_moved<false, false><<<g, 256, 0, st>>>(a);
    }
    SFCNL_LAUNCHED(ctx);
    prof_mark(ctx, kStagePass, true);
    return SFCNL_OK;
}
