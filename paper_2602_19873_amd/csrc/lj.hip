// Lennard-Jones 12/6 + Coulomb pass (the benchmark pass of Sec. III): the
// list is built once at the list cutoff and reused, and the pass keeps the
// pairs inside the shorter interaction cutoff (a Verlet buffer), evaluating
// the force of each on the tile layout of the density pass.
//
// Full list: lane roles of the density pass (i-particle registers, the j
// side loaded per entry); per-lane force partials are summed over the lanes
// that share an i-particle at the end and stored. Half list: lane roles of
// the symmetric density pass; each stored pair adds its force to i and the
// opposite force to j (Newton's third law), the j side reduced over its DPP
// row group before one atomic per component. At cluster size 8 both passes
// take list entries 8 at a time, their j-particles fetched into LDS with one
// load per field, and the half pass adds the j sums of 8 entries with one
// atomic per lane and component.
//
// Absent i-particles sit at +kAway and absent j-particles at -kAway: every
// squared distance that involves one overflows to +inf and fails the cutoff
// test, while the differences themselves stay finite (zero force times a
// finite difference is zero).
#include <cmath>

#include "internal.h"

#include "pass_common.h"

namespace sfcnl {
namespace {

using namespace passk;

constexpr float kAway = 1.0e38f;

// One wavefront (one super-cluster) per block, as for the density passes.
constexpr int kLjWaves = 1;

struct LjArgs {
    int64_t n;
    uint32_t nsc;
    const uint32_t *sc_info, *pool;
    const float *x, *y, *z, *q;
    float rc2;    // f32(r_cut^2)
    float sig2;   // sigma^2
    float eps24;  // 24 eps
    float eps4;   // 4 eps
    float kc;     // Coulomb prefactor
    float *fx, *fy, *fz, *ep;
    Period per;   // periodic axes (used by the kPbc kernels)
};

// orders a wave's LDS accesses around it (the wave runs in lockstep)
__device__ __forceinline__ void lj_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// minimum images of a pair's components on periodic axes
template <bool kPbc>
__device__ __forceinline__ void wrap3(float &dx, float &dy, float &dz, const Period &p) {
    if (kPbc) wave_min_image(dx, dy, dz, p);
}

// fr = -(dU/dr) / r of one pair at squared distance d2, and (kE) the pair
// energy U; kqq = coulomb * q_i * q_j.
template <bool kQ, bool kE>
__device__ __forceinline__ void lj_factor(float d2, float kqq, const LjArgs &a, float &fr, float &u) {
    const float ir2 = __builtin_amdgcn_rcpf(d2);
    const float s2 = a.sig2 * ir2;
    const float s6 = s2 * s2 * s2;
    fr = a.eps24 * ir2 * s6 * __builtin_fmaf(2.0f, s6, -1.0f);
    if (kE) u = a.eps4 * s6 * (s6 - 1.0f);
    if (kQ) {
        const float c = kqq * __builtin_amdgcn_rsqf(d2);  // k q_i q_j / r
        fr = __builtin_fmaf(c, ir2, fr);
        if (kE) u += c;
    }
}

// One pair of a full-list tile. g accumulates fr * (x_j - x_i) (the force on
// i is its negative), ge the pair energies. wrap (wave-uniform) false: no
// pair of the tile can need a minimum image.
template <bool kQ, bool kE, bool kPbc>
__device__ __forceinline__ void lj_tile(float xj, float yj, float zj, float qj, float xi, float yi, float zi,
                                        float kqi, bool self_pair, const LjArgs &a, float &gx, float &gy, float &gz,
                                        float &ge, bool wrap = true) {
    float dx = xj - xi;
    float dy = yj - yi;
    float dz = zj - zi;
    if (wrap) wrap3<kPbc>(dx, dy, dz, a.per);
    const float dxx = dx * dx;
    const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
    const bool in = d2 < a.rc2 && !self_pair;
    if (sfc_ballot(in)) {
        float fr, u = 0.0f;
        lj_factor<kQ, kE>(d2, kqi * qj, a, fr, u);
        fr = in ? fr : 0.0f;
        gx = __builtin_fmaf(fr, dx, gx);
        gy = __builtin_fmaf(fr, dy, gy);
        gz = __builtin_fmaf(fr, dz, gz);
        if (kE) ge += in ? u : 0.0f;
    }
}

// Six waves per SIMD for cluster sizes 4 and 8 (a few registers spilled, 3 %
// faster); cluster size 16 spills heavily under that cap and keeps its own
// register count.
template <int CS, bool kCompress, bool kQ, bool kE, bool kPbc>
__global__ __launch_bounds__(kWave * kLjWaves) __attribute__((amdgpu_waves_per_eu(CS == 16 ? 1 : 6))) void k_pass_lj(LjArgs a) {
    constexpr int kNsub = kScSize / CS;
    constexpr int kNreg = CS == 8 ? 8 : 4;
    constexpr int kNj = CS == 16 ? 4 : 1;
    constexpr int kGroup = CS == 8 ? 8 : 4;
    const int lane = sfc_lane();
    const int w = threadIdx.x / kWave;
    const uint32_t s = (uint32_t)__builtin_amdgcn_readfirstlane((int)(xcd_remap(blockIdx.x, gridDim.x) * kLjWaves + w));
    if (s >= a.nsc) return;
    const int64_t n = a.n;
    const int jl = lane & (kGroup - 1);

    float ix[kNreg], iy[kNreg], iz[kNreg], ikq[kNreg];
#pragma unroll
    for (int k = 0; k < kNreg; k++) {
        const int64_t i = (int64_t)s * kScSize + ipart<CS>(k, lane);
        const bool v = i < n;
        ix[k] = v ? a.x[i] : kAway;
        iy[k] = v ? a.y[i] : kAway;
        iz[k] = v ? a.z[i] : kAway;
        ikq[k] = kQ ? (v ? a.kc * a.q[i] : 0.0f) : 0.0f;
    }
    float gx[kNreg], gy[kNreg], gz[kNreg], ge[kNreg];
#pragma unroll
    for (int k = 0; k < kNreg; k++) gx[k] = gy[k] = gz[k] = ge[k] = 0.0f;

    const uint32_t own_c0 = s * kNsub;
    const uint32_t off = a.sc_info[2 * s], nj = a.sc_info[2 * s + 1];
    const uint8_t *mbytes = reinterpret_cast<const uint8_t *>(a.pool + off);
    const uint16_t *mshorts = reinterpret_cast<const uint16_t *>(a.pool + off);
    uint32_t p = off + (nj * (CS == 4 ? 2u : 1u) + 3u) / 4u;
    uint32_t prevj = 0xFFFFFFFFu;
    auto load_j = [&](uint32_t cj, float (&xj)[kNj], float (&yj)[kNj], float (&zj)[kNj], float (&qj)[kNj]) {
#pragma unroll
        for (int t = 0; t < kNj; t++) {
            const int64_t jp = (int64_t)cj * CS + (CS == 16 ? 4 * t + jl : jl);
            const bool vj = jp < n;
            xj[t] = vj ? a.x[jp] : -kAway;
            yj[t] = vj ? a.y[jp] : -kAway;
            zj[t] = vj ? a.z[jp] : -kAway;
            qj[t] = kQ ? (vj ? a.q[jp] : 0.0f) : 0.0f;
        }
    };
    // Cluster size 8: the entries of a decoded segment 8 at a time. Lane
    // (q, r) = (lane / 8, lane % 8) loads particle r of the batch's entry q
    // (one load per field for the batch) into LDS, where the tile lanes of
    // entry q read j-particle jl.
    const IBox ib = kPbc && CS == 8 ? ibox_of<kNreg>(ix, iy, iz) : IBox{};
    auto batch_wraps = [&](float4 jp, bool used) __attribute__((always_inline)) {
        return sfc_ballot(used && far_from_box(jp, ib, a.per)) != 0;
    };
    __shared__ float4 s_jb[kLjWaves][CS == 8 ? kWave : 1];  // x, y, z, charge
    auto entries8 = [&](uint32_t mvl, uint32_t jvl, uint32_t cnt) __attribute__((always_inline)) {
        const int il = lane >> 3;
        for (uint32_t q0 = 0; q0 < cnt; q0 += 8) {
            const uint32_t e = q0 + (uint32_t)(lane >> 3);
            const bool ev = e < cnt;
            const uint32_t cjb = (uint32_t)__shfl((int)jvl, (int)(ev ? e : q0), kWave);
            const uint32_t pq = cjb * CS + (uint32_t)(lane & 7);  // n < 2^31
            const bool pv = ev && pq < n;
            const uint32_t pc = pq < n ? pq : (uint32_t)(n - 1);  // loads of a clamped index go out together
            const float bx = a.x[pc], by = a.y[pc], bz = a.z[pc];
            const float bq = kQ ? a.q[pc] : 0.0f;
            lj_wave_sync();  // the previous batch's reads are done
            const float4 jv4 = make_float4(pv ? bx : -kAway, pv ? by : -kAway, pv ? bz : -kAway, pv ? bq : 0.0f);
            s_jb[w][lane] = jv4;
            lj_wave_sync();
            const uint32_t bn = cnt - q0 < 8u ? cnt - q0 : 8u;
            const bool wrap = kPbc && batch_wraps(jv4, (uint32_t)(lane >> 3) < bn);
            for (uint32_t q = 0; q < bn; q++) {
                const uint32_t mk = sfc_readlane(mvl, (int)(q0 + q));
                const uint32_t cj = sfc_readlane(jvl, (int)(q0 + q));
                const float4 jb = s_jb[w][q * 8 + jl];
                const int self_c = (cj >= own_c0 && cj < own_c0 + kNsub) ? (int)(cj - own_c0) : -1;
#pragma unroll
                for (int c = 0; c < kNreg; c++)
                    if ((mk >> c) & 1u)
                        lj_tile<kQ, kE, kPbc>(jb.x, jb.y, jb.z, jb.w, ix[c], iy[c], iz[c], ikq[c], c == self_c && il == jl,
                                              a, gx[c], gy[c], gz[c], ge[c], wrap);
            }
        }
    };
    for (uint32_t b0 = 0; b0 < nj; b0 += kWave) {
        const uint32_t cnt = nj - b0 < (uint32_t)kWave ? nj - b0 : (uint32_t)kWave;
        uint32_t jv;
        if (kCompress)
            jv = decode_segment(a.pool, p, cnt, prevj);
        else
            jv = (uint32_t)lane < cnt ? a.pool[p + b0 + lane] : 0u;
        uint32_t mv = 0u;
        if ((uint32_t)lane < cnt) mv = CS == 4 ? (uint32_t)mshorts[b0 + lane] : (uint32_t)mbytes[b0 + lane];
        prevj = sfc_readlane(jv, (int)cnt - 1);
        if constexpr (CS == 8) {
            entries8(mv, jv, cnt);
            continue;
        }
        // the next entry's j-particles load while the current entry's tiles run
        uint32_t cj = sfc_readlane(jv, 0);
        float xj[kNj], yj[kNj], zj[kNj], qj[kNj];
        load_j(cj, xj, yj, zj, qj);
        for (uint32_t e = 0; e < cnt; e++) {
            const uint32_t mk = sfc_readlane(mv, (int)e);
            const uint32_t ccur = cj;
            float cx[kNj], cy[kNj], cz[kNj], cq[kNj];
#pragma unroll
            for (int t = 0; t < kNj; t++) {
                cx[t] = xj[t];
                cy[t] = yj[t];
                cz[t] = zj[t];
                cq[t] = qj[t];
            }
            if (e + 1 < cnt) {
                cj = sfc_readlane(jv, (int)e + 1);
                load_j(cj, xj, yj, zj, qj);
            }
            const int self_c = (ccur >= own_c0 && ccur < own_c0 + kNsub) ? (int)(ccur - own_c0) : -1;
            if (CS == 8) {
                const int il = lane >> 3;
#pragma unroll
                for (int c = 0; c < kNreg; c++)
                    if ((mk >> c) & 1u)
                        lj_tile<kQ, kE, kPbc>(cx[0], cy[0], cz[0], cq[0], ix[c], iy[c], iz[c], ikq[c],
                                        c == self_c && il == jl, a, gx[c], gy[c], gz[c], ge[c]);
            } else if (CS == 4) {
                const int il = (lane >> 2) & 3, q = lane >> 4;
#pragma unroll
                for (int k = 0; k < kNreg; k++)
                    if ((mk >> (4 * k)) & 0xFu)
                        lj_tile<kQ, kE, kPbc>(cx[0], cy[0], cz[0], cq[0], ix[k], iy[k], iz[k], ikq[k],
                                        4 * k + q == self_c && il == jl, a, gx[k], gy[k], gz[k], ge[k]);
            } else {
                const int il = lane >> 2;
#pragma unroll
                for (int c = 0; c < kNreg; c++)
                    if ((mk >> c) & 1u) {
#pragma unroll
                        for (int t = 0; t < 4; t++)
                            lj_tile<kQ, kE, kPbc>(cx[t], cy[t], cz[t], cq[t], ix[c], iy[c], iz[c], ikq[c],
                                            c == self_c && il == 4 * t + jl, a, gx[c], gy[c], gz[c], ge[c]);
                    }
            }
        }
    }
    // sum the partials of each i-particle over the kGroup lanes sharing it;
    // the lane with j slot k then stores register k
#pragma unroll
    for (int k = 0; k < kNreg; k++) {
#pragma unroll
        for (int d = 1; d < kGroup; d <<= 1) {
            gx[k] += __shfl_xor(gx[k], d, 64);
            gy[k] += __shfl_xor(gy[k], d, 64);
            gz[k] += __shfl_xor(gz[k], d, 64);
            if (kE) ge[k] += __shfl_xor(ge[k], d, 64);
        }
    }
    float rx = gx[0], ry = gy[0], rz = gz[0], re = ge[0];
#pragma unroll
    for (int k = 1; k < kNreg; k++) {
        rx = jl == k ? gx[k] : rx;
        ry = jl == k ? gy[k] : ry;
        rz = jl == k ? gz[k] : rz;
        re = jl == k ? ge[k] : re;
    }
    const int64_t io = (int64_t)s * kScSize + ipart<CS>(jl, lane);
    if (io < n) {
        a.fx[io] = -rx;
        a.fy[io] = -ry;
        a.fz[io] = -rz;
        if (kE) a.ep[io] = 0.5f * re;
    }
}

// The batched entries of cluster size 8 need more registers: five waves per
// SIMD without spills run faster than six with them.
template <int CS, bool kCompress, bool kQ, bool kE, bool kPbc>
__global__ __launch_bounds__(kWave * kLjWaves) __attribute__((amdgpu_waves_per_eu(CS == 16 ? 1 : (CS == 8 ? 5 : 6)))) void k_pass_lj_half(LjArgs a) {
    constexpr int kNsub = kScSize / CS;
    constexpr int kNreg = CS == 8 ? 8 : 4;
    constexpr int kNj = CS == 16 ? 4 : 1;
    constexpr int kIL = CS == 8 ? 8 : 16;  // lanes per j-particle (the i side, low bits)
    const int lane = sfc_lane();
    const int w = threadIdx.x / kWave;
    const uint32_t s = (uint32_t)__builtin_amdgcn_readfirstlane((int)(xcd_remap(blockIdx.x, gridDim.x) * kLjWaves + w));
    if (s >= a.nsc) return;
    const int64_t n = a.n;
    const int jq = CS == 8 ? lane >> 3 : lane >> 4;

    float ix[kNreg], iy[kNreg], iz[kNreg], ikq[kNreg];
#pragma unroll
    for (int k = 0; k < kNreg; k++) {
        const int64_t i = (int64_t)s * kScSize + ipart_sym<CS>(k, lane);
        const bool v = i < n;
        ix[k] = v ? a.x[i] : kAway;
        iy[k] = v ? a.y[i] : kAway;
        iz[k] = v ? a.z[i] : kAway;
        ikq[k] = kQ ? (v ? a.kc * a.q[i] : 0.0f) : 0.0f;
    }
    float gx[kNreg], gy[kNreg], gz[kNreg], ge[kNreg];
#pragma unroll
    for (int k = 0; k < kNreg; k++) gx[k] = gy[k] = gz[k] = ge[k] = 0.0f;

    const uint32_t own_c0 = s * kNsub;
    const uint32_t off = a.sc_info[2 * s], nj = a.sc_info[2 * s + 1];
    const uint8_t *mbytes = reinterpret_cast<const uint8_t *>(a.pool + off);
    const uint16_t *mshorts = reinterpret_cast<const uint16_t *>(a.pool + off);
    // Cluster size 8: the entries of a decoded segment 8 at a time. Lane
    // (q, r) = (lane / 8, lane % 8) loads particle r of the batch's entry q
    // (one load per field for the batch) and leaves it in LDS, where the tile
    // lanes of entry q read j-particle jq. An entry's j-side sums (over the 8
    // lanes of each j-particle, by DPP) and whether the j-particle formed a
    // pair go to LDS too, and after the batch lane (q, r) adds its particle's
    // sums with one atomic per component.
    const IBox ib = kPbc && CS == 8 ? ibox_of<kNreg>(ix, iy, iz) : IBox{};
    auto batch_wraps = [&](float4 jp, bool used) __attribute__((always_inline)) {
        return sfc_ballot(used && far_from_box(jp, ib, a.per)) != 0;
    };
    __shared__ float4 s_jb[kLjWaves][CS == 8 ? kWave : 1];  // x, y, z, charge
    __shared__ float4 s_jh[kLjWaves][CS == 8 ? kWave : 1];  // j-side force (and energy) sums
    __shared__ uint32_t s_jhit[kLjWaves][CS == 8 ? kWave : 1];
    auto entries8 = [&](uint32_t mvl, uint32_t jvl, uint32_t cnt) __attribute__((always_inline)) {
        const int il = lane & 7;
        for (uint32_t q0 = 0; q0 < cnt; q0 += 8) {
            const uint32_t e = q0 + (uint32_t)(lane >> 3);
            bool ev = e < cnt;
            const uint32_t cjb = (uint32_t)__shfl((int)jvl, (int)(ev ? e : q0), kWave);
            const uint32_t pq = cjb * CS + (uint32_t)(lane & 7);  // n < 2^31
            ev = ev && pq < n;
            const uint32_t pc = pq < n ? pq : (uint32_t)(n - 1);  // loads of a clamped index go out together
            const float bx = a.x[pc], by = a.y[pc], bz = a.z[pc];
            const float bq = kQ ? a.q[pc] : 0.0f;
            const float4 jv4 = make_float4(ev ? bx : -kAway, ev ? by : -kAway, ev ? bz : -kAway, ev ? bq : 0.0f);
            s_jb[w][lane] = jv4;
            lj_wave_sync();
            const uint32_t bn = cnt - q0 < 8u ? cnt - q0 : 8u;
            const bool wrap = kPbc && batch_wraps(jv4, (uint32_t)(lane >> 3) < bn);
            for (uint32_t q = 0; q < bn; q++) {
                const uint32_t mk = sfc_readlane(mvl, (int)(q0 + q));
                const uint32_t cj = sfc_readlane(jvl, (int)(q0 + q));
                const float4 jb = s_jb[w][q * 8 + jq];
                float hx = 0.0f, hy = 0.0f, hz = 0.0f, he = 0.0f;
                uint64_t jm = 0;  // lanes that formed a pair
                // inside the super-cluster only j > i counts
                const int self_c = (cj >= own_c0 && cj < own_c0 + kNsub) ? (int)(cj - own_c0) : -1;
#pragma unroll
                for (int c = 0; c < kNreg; c++) {
                    if (!((mk >> c) & 1u)) continue;
                    const bool kp = self_c < 0 || c < self_c || (c == self_c && jq > il);
                    float dx = jb.x - ix[c];
                    float dy = jb.y - iy[c];
                    float dz = jb.z - iz[c];
                    if (wrap) wrap3<kPbc>(dx, dy, dz, a.per);  // wave-uniform
                    const float dxx = dx * dx;
                    const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
                    const bool in = kp && d2 < a.rc2;
                    const uint64_t bal = sfc_ballot(in);
                    if (bal) {
                        jm |= bal;
                        float fr, u = 0.0f;
                        lj_factor<kQ, kE>(d2, ikq[c] * jb.w, a, fr, u);
                        fr = in ? fr : 0.0f;
                        const float px = fr * dx, py = fr * dy, pz = fr * dz;
                        gx[c] += px;
                        gy[c] += py;
                        gz[c] += pz;
                        hx += px;
                        hy += py;
                        hz += pz;
                        if (kE) {
                            const float uu = in ? u : 0.0f;
                            ge[c] += uu;
                            he += uu;
                        }
                    }
                }
                if (jm) {
                    group_sum<kIL>(hx);
                    group_sum<kIL>(hy);
                    group_sum<kIL>(hz);
                    if (kE) group_sum<kIL>(he);
                }
                if (il == 0) {
                    s_jh[w][q * 8 + jq] = make_float4(hx, hy, hz, he);
                    s_jhit[w][q * 8 + jq] = ((jm >> (8 * jq)) & 0xFFull) != 0 ? 1u : 0u;
                }
            }
            lj_wave_sync();
            // lane (q, r): j-particle r of entry q
            if (ev && (uint32_t)(lane >> 3) < bn && s_jhit[w][lane]) {
                const float4 hv = s_jh[w][lane];
                atomicAdd(&a.fx[pq], hv.x);
                atomicAdd(&a.fy[pq], hv.y);
                atomicAdd(&a.fz[pq], hv.z);
                if (kE) atomicAdd(&a.ep[pq], 0.5f * hv.w);
            }
            lj_wave_sync();  // the next batch rewrites the LDS arrays
        }
    };

    uint32_t p = off + (nj * (CS == 4 ? 2u : 1u) + 3u) / 4u;
    uint32_t prevj = 0xFFFFFFFFu;
    for (uint32_t b0 = 0; b0 < nj; b0 += kWave) {
        const uint32_t cnt = nj - b0 < (uint32_t)kWave ? nj - b0 : (uint32_t)kWave;
        uint32_t jv;
        if (kCompress)
            jv = decode_segment(a.pool, p, cnt, prevj);
        else
            jv = (uint32_t)lane < cnt ? a.pool[p + b0 + lane] : 0u;
        uint32_t mv = 0u;
        if ((uint32_t)lane < cnt) mv = CS == 4 ? (uint32_t)mshorts[b0 + lane] : (uint32_t)mbytes[b0 + lane];
        prevj = sfc_readlane(jv, (int)cnt - 1);
        if constexpr (CS == 8) {
            entries8(mv, jv, cnt);
            continue;
        }
        float nx[kNj], ny[kNj], nz[kNj], nq[kNj];
        auto load_j = [&](uint32_t cjn) {
#pragma unroll
            for (int t = 0; t < kNj; t++) {
                const int64_t jp = (int64_t)cjn * CS + (CS == 16 ? 4 * t + jq : jq);
                const bool vj = jp < n;
                nx[t] = vj ? a.x[jp] : -kAway;
                ny[t] = vj ? a.y[jp] : -kAway;
                nz[t] = vj ? a.z[jp] : -kAway;
                nq[t] = kQ ? (vj ? a.q[jp] : 0.0f) : 0.0f;
            }
        };
        load_j(sfc_readlane(jv, 0));
        for (uint32_t e = 0; e < cnt; e++) {
            const uint32_t mk = sfc_readlane(mv, (int)e);
            const uint32_t cj = sfc_readlane(jv, (int)e);
            float xj[kNj], yj[kNj], zj[kNj], qj[kNj], hx[kNj], hy[kNj], hz[kNj], he[kNj];
            int64_t jp[kNj];
#pragma unroll
            for (int t = 0; t < kNj; t++) {
                jp[t] = (int64_t)cj * CS + (CS == 16 ? 4 * t + jq : jq);
                xj[t] = nx[t];
                yj[t] = ny[t];
                zj[t] = nz[t];
                qj[t] = nq[t];
                hx[t] = hy[t] = hz[t] = he[t] = 0.0f;
            }
            if (e + 1 < cnt) load_j(sfc_readlane(jv, (int)e + 1));
            // inside the super-cluster only j > i counts
            const int self_c = (cj >= own_c0 && cj < own_c0 + kNsub) ? (int)(cj - own_c0) : -1;
            auto keep = [&](int ci, int ipos, int jpos) {
                return self_c < 0 || ci < self_c || (ci == self_c && jpos > ipos);
            };
            uint64_t jm[kNj];  // lanes that formed a pair with j-slot t
#pragma unroll
            for (int t = 0; t < kNj; t++) jm[t] = 0;
            // one pair: g (i side) and h (j side) accumulate fr * (x_j - x_i)
            auto pair = [&](int t, int k, bool kp) {
                float dx = xj[t] - ix[k];
                float dy = yj[t] - iy[k];
                float dz = zj[t] - iz[k];
                wrap3<kPbc>(dx, dy, dz, a.per);
                const float dxx = dx * dx;
                const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
                const bool in = kp && d2 < a.rc2;
                const uint64_t bal = sfc_ballot(in);
                if (bal) {
                    jm[t] |= bal;
                    float fr, u = 0.0f;
                    lj_factor<kQ, kE>(d2, ikq[k] * qj[t], a, fr, u);
                    fr = in ? fr : 0.0f;
                    const float px = fr * dx, py = fr * dy, pz = fr * dz;
                    gx[k] += px;
                    gy[k] += py;
                    gz[k] += pz;
                    hx[t] += px;
                    hy[t] += py;
                    hz[t] += pz;
                    if (kE) {
                        const float uu = in ? u : 0.0f;
                        ge[k] += uu;
                        he[t] += uu;
                    }
                }
            };
            if (CS == 8) {
                const int il = lane & 7;
#pragma unroll
                for (int c = 0; c < kNreg; c++)
                    if ((mk >> c) & 1u) pair(0, c, keep(c, il, jq));
            } else if (CS == 4) {
                const int il = lane & 3, q = (lane >> 2) & 3;
#pragma unroll
                for (int k = 0; k < kNreg; k++)
                    if ((mk >> (4 * k)) & 0xFu) pair(0, k, keep(4 * k + q, il, jq));
            } else {
                const int il = lane & 15;
#pragma unroll
                for (int c = 0; c < kNreg; c++)
                    if ((mk >> c) & 1u) {
#pragma unroll
                        for (int t = 0; t < 4; t++) pair(t, c, keep(c, il, 4 * t + jq));
                    }
            }
            // j side: the force on j is +fr (x_j - x_i) summed; reduce over the
            // i lanes of each j-particle (one DPP row group), one atomic each
            uint64_t jany = 0;
#pragma unroll
            for (int t = 0; t < kNj; t++) jany |= jm[t];
            if (jany) {
                constexpr uint64_t kGrp = (1ull << kIL) - 1ull;
#pragma unroll
                for (int t = 0; t < kNj; t++) {
                    group_sum<kIL>(hx[t]);
                    group_sum<kIL>(hy[t]);
                    group_sum<kIL>(hz[t]);
                    if (kE) group_sum<kIL>(he[t]);
                    const bool hit = ((jm[t] >> (jq * kIL)) & kGrp) != 0;
                    if ((lane & (kIL - 1)) == 0 && hit && jp[t] < n) {
                        atomicAdd(&a.fx[jp[t]], hx[t]);
                        atomicAdd(&a.fy[jp[t]], hy[t]);
                        atomicAdd(&a.fz[jp[t]], hz[t]);
                        if (kE) atomicAdd(&a.ep[jp[t]], 0.5f * he[t]);
                    }
                }
            }
        }
    }
    // i side: sum over the j lanes (the high lane bits); the lane with j slot
    // k adds register k
#pragma unroll
    for (int k = 0; k < kNreg; k++) {
#pragma unroll
        for (int d = kIL; d < kWave; d <<= 1) {
            gx[k] += __shfl_xor(gx[k], d, 64);
            gy[k] += __shfl_xor(gy[k], d, 64);
            gz[k] += __shfl_xor(gz[k], d, 64);
            if (kE) ge[k] += __shfl_xor(ge[k], d, 64);
        }
    }
    float rx = gx[0], ry = gy[0], rz = gz[0], re = ge[0];
#pragma unroll
    for (int k = 1; k < kNreg; k++) {
        rx = jq == k ? gx[k] : rx;
        ry = jq == k ? gy[k] : ry;
        rz = jq == k ? gz[k] : rz;
        re = jq == k ? ge[k] : re;
    }
    const int64_t io = (int64_t)s * kScSize + ipart_sym<CS>(jq, lane);
    if (io < n) {
        atomicAdd(&a.fx[io], -rx);
        atomicAdd(&a.fy[io], -ry);
        atomicAdd(&a.fz[io], -rz);
        if (kE) atomicAdd(&a.ep[io], 0.5f * re);
    }
}

template <int CS, bool kHalf, bool kPbc>
void launch_lj(int variant, unsigned g, hipStream_t st, const LjArgs &a) {
#define SFCNL_LJ(C, Q, E) \
    (kHalf ? k_pass_lj_half<CS, C, Q, E, kPbc> : k_pass_lj<CS, C, Q, E, kPbc>)<<<g, kWave * kLjWaves, 0, st>>>(a)
    switch (variant) {
        case 7: SFCNL_LJ(true, true, true); break;
        case 6: SFCNL_LJ(true, true, false); break;
        case 5: SFCNL_LJ(true, false, true); break;
        case 4: SFCNL_LJ(true, false, false); break;
        case 3: SFCNL_LJ(false, true, true); break;
        case 2: SFCNL_LJ(false, true, false); break;
        case 1: SFCNL_LJ(false, false, true); break;
        default: SFCNL_LJ(false, false, false); break;
    }
#undef SFCNL_LJ
}

template <bool kPbc>
void launch_lj_any(int cs, int half, int variant, unsigned g, hipStream_t st, const LjArgs &a) {
    if (half) {
        if (cs == 4)
            launch_lj<4, true, kPbc>(variant, g, st, a);
        else if (cs == 16)
            launch_lj<16, true, kPbc>(variant, g, st, a);
        else
            launch_lj<8, true, kPbc>(variant, g, st, a);
    } else if (cs == 4) {
        launch_lj<4, false, kPbc>(variant, g, st, a);
    } else if (cs == 16) {
        launch_lj<16, false, kPbc>(variant, g, st, a);
    } else {
        launch_lj<8, false, kPbc>(variant, g, st, a);
    }
}

}  // namespace
}  // namespace sfcnl

using namespace sfcnl;

extern "C" int nlist_pass_lj(sfcnl_ctx ctx, int64_t n, int cluster_size, int compress, int half,
                             const uint32_t *d_sc_info, const uint32_t *d_pool, const float *d_x, const float *d_y,
                             const float *d_z, const float *d_q, const sfcnl_lj_params *params, float *d_fx,
                             float *d_fy, float *d_fz, float *d_epot, const float *h_period) {
    if (!ctx) return SFCNL_E_ARG;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "nlist_pass_lj: n out of range");
    if (cluster_size != 4 && cluster_size != 8 && cluster_size != 16)
        return set_err(ctx, SFCNL_E_ARG, "nlist_pass_lj: cluster_size %d not supported", cluster_size);
    if (compress != 0 && compress != 1) return set_err(ctx, SFCNL_E_ARG, "nlist_pass_lj: compress must be 0 or 1");
    if (half != 0 && half != 1) return set_err(ctx, SFCNL_E_ARG, "nlist_pass_lj: half must be 0 or 1");
    if (!params) return set_err(ctx, SFCNL_E_ARG, "nlist_pass_lj: null params");
    const sfcnl_lj_params pr = *params;
    if (!(pr.r_cut > 0.0f) || !std::isfinite(pr.r_cut) || !(pr.sigma > 0.0f) || !std::isfinite(pr.sigma) ||
        !std::isfinite(pr.eps) || !std::isfinite(pr.coulomb))
        return set_err(ctx, SFCNL_E_ARG, "nlist_pass_lj: parameters must be finite, sigma and r_cut > 0");
    if (!period_ok(h_period)) return set_err(ctx, SFCNL_E_ARG, "nlist_pass_lj: period must be 3 finite values >= 0");
    if (n == 0) return SFCNL_OK;
    if (!d_sc_info || !d_pool || !d_x || !d_y || !d_z || !d_fx || !d_fy || !d_fz)
        return set_err(ctx, SFCNL_E_ARG, "nlist_pass_lj: null pointer");
    LjArgs a{n, (uint32_t)((n + kScSize - 1) / kScSize), d_sc_info, d_pool, d_x, d_y, d_z, d_q,
             pr.r_cut * pr.r_cut, pr.sigma * pr.sigma, 24.0f * pr.eps, 4.0f * pr.eps, pr.coulomb,
             d_fx, d_fy, d_fz, d_epot, make_period(h_period)};
    const unsigned g = blocks_for(a.nsc, kLjWaves);
    hipStream_t st = ctx->stream;
    const int variant = (compress ? 4 : 0) | (d_q ? 2 : 0) | (d_epot ? 1 : 0);
    prof_mark(ctx, kStagePass, false);
    if (half) {
        // accumulators start at zero (fill kernels, so the call can sit in a graph)
        int rc = fill2_u32(ctx, reinterpret_cast<uint32_t *>(d_fx), reinterpret_cast<uint32_t *>(d_fy), n, 0u);
        if (rc) return rc;
        rc = fill2_u32(ctx, reinterpret_cast<uint32_t *>(d_fz), reinterpret_cast<uint32_t *>(d_epot), n, 0u);
        if (rc) return rc;
    }
    if (a.per.on())
        launch_lj_any<true>(cluster_size, half, variant, g, st, a);
    else
        launch_lj_any<false>(cluster_size, half, variant, g, st, a);
    SFCNL_LAUNCHED(ctx);
    prof_mark(ctx, kStagePass, true);
    return SFCNL_OK;
}
