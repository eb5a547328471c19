// Neighbour pass (Sec. II-A "neighbor pass", Sec. II-D Listing 1): decode a
// super-cluster's compressed list 64 entries at a time (Sec. II-B, "set the
// output to one where the bitmask is zero", info nibbles, data nibbles), then
// evaluate one 8x8 particle tile per (j-cluster, set mask bit) on one
// wavefront and accumulate the SPH density and the neighbour count.
//
// Lane (il, jl) = (lane / 8, lane % 8) keeps i-particle il of every i-cluster
// in registers and loads j-particle jl of the current j-cluster, so a tile is
// one 64-lane step with no cross-lane traffic; the 8 partial sums per
// i-particle are combined once at the end.
#include "internal.h"

namespace sfcnl {
namespace {

constexpr int kWavesPerBlock = 4;
// Position for absent particles: any distance to it overflows to +inf.
constexpr float kFar = 3.0e38f;

__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned g) {
    const unsigned per = g / 8, rem = g % 8, x = b % 8, i = b / 8;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

__device__ __forceinline__ uint32_t nibble_at(const uint8_t *stream, uint32_t t) {
    return (uint32_t)(stream[t >> 1] >> ((t & 1u) * 4u)) & 0xFu;
}

// Decodes one segment of `cnt` differences at pool[p..] whose previous index
// is prevj; lane k returns index k (lanes >= cnt return garbage). Advances p
// past the segment.
__device__ __forceinline__ uint32_t decode_segment(const uint32_t *__restrict__ pool, uint32_t &p, uint32_t cnt,
                                                   uint32_t prevj) {
    const int lane = sfc_lane();
    const uint32_t lo = pool[p], hi = pool[p + 1];
    const uint64_t m = ((uint64_t)hi << 32) | lo;
    const uint8_t *stream = reinterpret_cast<const uint8_t *>(pool + p + 2);
    const bool valid = (uint32_t)lane < cnt;
    const bool nonone = valid && ((m >> lane) & 1ull);
    const uint32_t ninfo = (uint32_t)sfc_popc(m);
    uint32_t v = 1u, nd = 0u;
    if (nonone) {
        const uint32_t inf = nibble_at(stream, (uint32_t)sfc_popc(m & sfc_lt_mask()));
        if (inf >= 8u)
            v = inf - 6u;
        else
            nd = inf + 1u;
    }
    const uint32_t incl = sfc_incl_scan(nd);
    if (nd) {
        uint32_t t = ninfo + incl - nd;
        v = 0u;
        for (uint32_t d = 0; d < nd; d++) v = (v << 4) | nibble_at(stream, t + d);
    }
    const uint32_t total_nib = ninfo + sfc_readlane(incl, kWave - 1);
    p += 2u + (total_nib + 7u) / 8u;
    return prevj + sfc_incl_scan(valid ? v : 0u);
}

struct PassArgs {
    int64_t n;
    uint32_t nsc;
    const uint32_t *sc_info, *pool;
    const float *x, *y, *z, *h, *m;
    float *rho;
    int32_t *nnb;
    SegTable seg;  // batched systems: list indices are relative to the system's first cluster
};

template <bool kCompress, bool kMass, bool kCount>
__global__ __launch_bounds__(256) void k_pass(PassArgs a) {
    const int lane = sfc_lane();
    const int w = threadIdx.x / kWave;
    const uint32_t s = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + w;
    if (s >= a.nsc) return;
    const int il = lane >> 3, jl = lane & 7;
    const int64_t n = a.n;

    // i particles: lane holds particle il of every i-cluster c; absent ones
    // get a negative squared radius so that no pair is accepted
    float ix[kSub], iy[kSub], iz[kSub], ih2[kSub], ihinv[kSub];
#pragma unroll
    for (int c = 0; c < kSub; c++) {
        const int64_t i = (int64_t)s * kScSize + c * kCs + il;
        const bool v = i < n;
        ix[c] = v ? a.x[i] : 0.0f;
        iy[c] = v ? a.y[i] : 0.0f;
        iz[c] = v ? a.z[i] : 0.0f;
        const float hh = v ? a.h[i] : 1.0f;
        ih2[c] = v ? hh * hh : -1.0f;
        ihinv[c] = 1.0f / hh;
    }
    // acc[c] sums m_j f(q)/2 with f the spline shape (f(0) = 1)
    float acc[kSub];
    int cnt_nb[kSub];
#pragma unroll
    for (int c = 0; c < kSub; c++) {
        acc[c] = 0.0f;
        cnt_nb[c] = 0;
    }

    const uint32_t own_c0 = s * kSub;
    const uint32_t off = a.sc_info[2 * s], nj = a.sc_info[2 * s + 1];
    const uint8_t *mbytes = reinterpret_cast<const uint8_t *>(a.pool + off);
    const uint32_t jbase = a.seg.on() ? a.seg.pbase[a.seg.sc_sys[s]] / kCs : 0u;
    uint32_t p = off + (nj + 3u) / 4u;
    uint32_t prevj = 0xFFFFFFFFu;
    for (uint32_t b0 = 0; b0 < nj; b0 += kWave) {
        const uint32_t cnt = nj - b0 < (uint32_t)kWave ? nj - b0 : (uint32_t)kWave;
        uint32_t jv;
        if (kCompress) {
            jv = decode_segment(a.pool, p, cnt, prevj);
        } else {
            jv = (uint32_t)lane < cnt ? a.pool[p + b0 + lane] : 0u;
        }
        const uint32_t mv = (uint32_t)lane < cnt ? mbytes[b0 + lane] : 0u;
        prevj = sfc_readlane(jv, (int)cnt - 1);
        jv += jbase;
        // software pipeline: the next entry's j-particles load while the
        // current entry's tiles run
        uint32_t cj = sfc_readlane(jv, 0);
        int64_t jp = (int64_t)cj * kCs + jl;
        float xj, yj, zj, mj;
        {
            const bool vj = jp < n;
            xj = vj ? a.x[jp] : kFar;
            yj = vj ? a.y[jp] : kFar;
            zj = vj ? a.z[jp] : kFar;
            mj = kMass ? (vj ? a.m[jp] : 0.0f) : 1.0f;
        }
        for (uint32_t e = 0; e < cnt; e++) {
            const uint32_t mk = sfc_readlane(mv, (int)e);
            const uint32_t ccur = cj;
            const float cx = xj, cy = yj, cz = zj, cm = mj;
            if (e + 1 < cnt) {
                cj = sfc_readlane(jv, (int)e + 1);
                jp = (int64_t)cj * kCs + jl;
                const bool vj = jp < n;
                xj = vj ? a.x[jp] : kFar;
                yj = vj ? a.y[jp] : kFar;
                zj = vj ? a.z[jp] : kFar;
                mj = kMass ? (vj ? a.m[jp] : 0.0f) : 1.0f;
            }
            // the j-cluster is one of our own i-clusters: exclude i == j
            const int self_c = (ccur >= own_c0 && ccur < own_c0 + kSub) ? (int)(ccur - own_c0) : -1;
#pragma unroll
            for (int c = 0; c < kSub; c++) {
                if ((mk >> c) & 1u) {
                    const float dx = cx - ix[c];
                    const float dy = cy - iy[c];
                    const float dz = cz - iz[c];
                    const float dxx = dx * dx;
                    const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
                    bool in = d2 < ih2[c];
                    if (c == self_c) in = in && il != jl;
                    if (sfc_ballot(in)) {
                        // M4 spline with support h, halved: 1/2 - 3q^2 + 3q^3
                        // below q = 1/2, (1-q)^3 above
                        const float q = __builtin_amdgcn_sqrtf(d2) * ihinv[c];
                        const float t1 = q - 1.0f;
                        const float q2 = q * q;
                        const float inner = __builtin_fmaf(3.0f * q2, t1, 0.5f);
                        const float outer = -(t1 * t1) * t1;
                        const float wq = q < 0.5f ? inner : outer;
                        const float nacc = __builtin_fmaf(cm, wq, acc[c]);
                        acc[c] = in ? nacc : acc[c];
                        cnt_nb[c] += in ? 1 : 0;
                    }
                }
            }
        }
    }
    // sum the 8 partials of each i-particle (lanes differing in jl)
#pragma unroll
    for (int c = 0; c < kSub; c++) {
#pragma unroll
        for (int d = 1; d < 8; d <<= 1) {
            acc[c] += __shfl_xor(acc[c], d, 64);
            if (kCount) cnt_nb[c] += __shfl_xor(cnt_nb[c], d, 64);
        }
    }
    // lane (il, jl) stores particle il of i-cluster jl
    float r = acc[0];
    int nb = cnt_nb[0];
#pragma unroll
    for (int c = 1; c < kSub; c++) {
        r = jl == c ? acc[c] : r;
        nb = jl == c ? cnt_nb[c] : nb;
    }
    const int64_t io = (int64_t)s * kScSize + jl * kCs + il;
    if (io < n) {
        const float hh = a.h[io];
        const float hinv = 1.0f / hh;
        const float mi = kMass ? a.m[io] : 1.0f;
        const float norm = 2.5464790894703255f * hinv * hinv * hinv;  // 8 / pi
        a.rho[io] = norm * __builtin_fmaf(2.0f, r, mi);
        if (kCount) a.nnb[io] = nb;
    }
}

struct DecodeArgs {
    uint32_t nsc;
    const uint32_t *sc_info, *pool, *offsets;
    uint32_t *j;
    uint16_t *mask;
};

template <bool kCompress>
__global__ __launch_bounds__(256) void k_decode(DecodeArgs a) {
    const int lane = sfc_lane();
    const uint32_t s = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (s >= a.nsc) return;
    const uint32_t off = a.sc_info[2 * s], nj = a.sc_info[2 * s + 1];
    const uint8_t *mbytes = reinterpret_cast<const uint8_t *>(a.pool + off);
    uint32_t p = off + (nj + 3u) / 4u;
    uint32_t prevj = 0xFFFFFFFFu;
    const uint32_t o = a.offsets[s];
    for (uint32_t b0 = 0; b0 < nj; b0 += kWave) {
        const uint32_t cnt = nj - b0 < (uint32_t)kWave ? nj - b0 : (uint32_t)kWave;
        uint32_t jv;
        if (kCompress)
            jv = decode_segment(a.pool, p, cnt, prevj);
        else
            jv = (uint32_t)lane < cnt ? a.pool[p + b0 + lane] : 0u;
        prevj = sfc_readlane(jv, (int)cnt - 1);
        if ((uint32_t)lane < cnt) {
            a.j[o + b0 + lane] = jv;
            a.mask[o + b0 + lane] = mbytes[b0 + lane];
        }
    }
}

}  // namespace
}  // namespace sfcnl

using namespace sfcnl;

int sfcnl::pass_impl(sfcnl_ctx ctx, int64_t n, int compress, const uint32_t *d_sc_info, const uint32_t *d_pool,
                     const float *d_x, const float *d_y, const float *d_z, const float *d_h, const float *d_m,
                     float *d_rho, int32_t *d_nnb, const SegTable &seg) {
    PassArgs a{n, (uint32_t)((n + kScSize - 1) / kScSize), d_sc_info, d_pool, d_x, d_y, d_z, d_h, d_m, d_rho, d_nnb,
               seg};
    const unsigned g = blocks_for(a.nsc, kWavesPerBlock);
    hipStream_t st = ctx->stream;
    const bool hm = d_m != nullptr, hc = d_nnb != nullptr;
#define SFCNL_PASS(C, M, K) k_pass<C, M, K><<<g, 256, 0, st>>>(a)
    prof_mark(ctx, kStagePass, false);
    if (compress) {
        if (hm) {
            if (hc) SFCNL_PASS(true, true, true); else SFCNL_PASS(true, true, false);
        } else {
            if (hc) SFCNL_PASS(true, false, true); else SFCNL_PASS(true, false, false);
        }
    } else {
        if (hm) {
            if (hc) SFCNL_PASS(false, true, true); else SFCNL_PASS(false, true, false);
        } else {
            if (hc) SFCNL_PASS(false, false, true); else SFCNL_PASS(false, false, false);
        }
    }
#undef SFCNL_PASS
    SFCNL_LAUNCHED(ctx);
    prof_mark(ctx, kStagePass, true);
    return SFCNL_OK;
}

extern "C" int nlist_pass(sfcnl_ctx ctx, int64_t n, int cluster_size, int compress, const uint32_t *d_sc_info,
                          const uint32_t *d_pool, const float *d_x, const float *d_y, const float *d_z,
                          const float *d_h, const float *d_m, float *d_rho, int32_t *d_nnb) {
    if (!ctx) return SFCNL_E_ARG;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "nlist_pass: n out of range");
    if (cluster_size != kCs) return set_err(ctx, SFCNL_E_ARG, "nlist_pass: cluster_size %d not supported", cluster_size);
    if (compress != 0 && compress != 1) return set_err(ctx, SFCNL_E_ARG, "nlist_pass: compress must be 0 or 1");
    if (n == 0) return SFCNL_OK;
    if (!d_sc_info || !d_pool || !d_x || !d_y || !d_z || !d_h || !d_rho)
        return set_err(ctx, SFCNL_E_ARG, "nlist_pass: null pointer");
    return pass_impl(ctx, n, compress, d_sc_info, d_pool, d_x, d_y, d_z, d_h, d_m, d_rho, d_nnb, SegTable{});
}

extern "C" int nlist_decode(sfcnl_ctx ctx, int64_t n, int cluster_size, int compress, const uint32_t *d_sc_info,
                            const uint32_t *d_pool, const uint32_t *d_offsets, uint32_t *d_j, uint16_t *d_mask) {
    if (!ctx) return SFCNL_E_ARG;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "nlist_decode: n out of range");
    if (cluster_size != kCs) return set_err(ctx, SFCNL_E_ARG, "nlist_decode: cluster_size %d not supported", cluster_size);
    if (n == 0) return SFCNL_OK;
    if (!d_sc_info || !d_pool || !d_offsets || !d_j || !d_mask)
        return set_err(ctx, SFCNL_E_ARG, "nlist_decode: null pointer");
    DecodeArgs a{(uint32_t)((n + kScSize - 1) / kScSize), d_sc_info, d_pool, d_offsets, d_j, d_mask};
    const unsigned g = blocks_for(a.nsc, kWavesPerBlock);
    if (compress)
        k_decode<true><<<g, 256, 0, ctx->stream>>>(a);
    else
        k_decode<false><<<g, 256, 0, ctx->stream>>>(a);
    SFCNL_LAUNCHED(ctx);
    return SFCNL_OK;
}
