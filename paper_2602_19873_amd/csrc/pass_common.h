// Pieces shared by the list passes (the SPH density pass and the
// Lennard-Jones + Coulomb pass): the wave-level decoder of one compressed
// segment (Sec. II-B), the XCD-aware block order, the lane roles that map
// list tiles onto a wavefront, DPP sums inside lane groups, and the wave's
// i-box that the periodic batch test (far_from_box) takes.
#pragma once
#include "internal.h"

namespace sfcnl {
namespace passk {

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

// i-particle held in register k by a lane (the traversal's lane roles):
// CS = 8: 8k + lane / 8; CS = 4 and 16: 16k + lane / 4.
template <int CS>
__device__ __forceinline__ int ipart(int k, int lane) {
    return CS == 8 ? 8 * k + (lane >> 3) : 16 * k + (lane >> 2);
}

// Cross-lane sums inside groups of 8 or 16 consecutive lanes with DPP
// (quad swaps, then the mirrored half row, then the mirrored row): every lane
// of a group ends with the group total.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int kLanes>
__device__ __forceinline__ void group_sum(float &f, int &c) {
    f += dpp_f<0xB1>(f);  // quad_perm [1, 0, 3, 2]
    c += dpp_i<0xB1>(c);
    f += dpp_f<0x4E>(f);  // quad_perm [2, 3, 0, 1]
    c += dpp_i<0x4E>(c);
    f += dpp_f<0x141>(f);  // row_half_mirror
    c += dpp_i<0x141>(c);
    if (kLanes == 16) {
        f += dpp_f<0x140>(f);  // row_mirror
        c += dpp_i<0x140>(c);
    }
}

template <int kLanes>
__device__ __forceinline__ void group_sum(float &f) {
    f += dpp_f<0xB1>(f);
    f += dpp_f<0x4E>(f);
    f += dpp_f<0x141>(f);
    if (kLanes == 16) f += dpp_f<0x140>(f);
}

// Lane roles of the symmetric pass (the i-particles in the low lane bits, so
// that a j-particle's sum over the i side stays inside a DPP row):
//   CS = 8:  lane = 8 jl + il; register k holds i-particle 8k + il;
//   CS = 4:  lane = 16 jl + 4q + il; register k holds i-particle 16k + 4q + il
//            (i-cluster 4k + q);
//   CS = 16: lane = 16 jq + il; register k holds i-particle 16k + il; the
//            lane takes j-particles 4t + jq.
template <int CS>
__device__ __forceinline__ int ipart_sym(int k, int lane) {
    return CS == 8 ? 8 * k + (lane & 7) : 16 * k + (lane & 15);
}

template <int kNreg>
__device__ __forceinline__ void wave_range(const float (&v)[kNreg], float &lo, float &hi) {
    lo = v[0];
    hi = v[0];
#pragma unroll
    for (int k = 1; k < kNreg; k++) {
        lo = fminf(lo, v[k]);
        hi = fmaxf(hi, v[k]);
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        lo = fminf(lo, __shfl_xor(lo, d, kWave));
        hi = fmaxf(hi, __shfl_xor(hi, d, kWave));
    }
    // wave-uniform: scalar registers
    lo = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, lo)));
    hi = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, hi)));
}
template <int kNreg>
__device__ __forceinline__ IBox ibox_of(const float (&ix)[kNreg], const float (&iy)[kNreg], const float (&iz)[kNreg]) {
    IBox b;
    wave_range<kNreg>(ix, b.lo[0], b.hi[0]);
    wave_range<kNreg>(iy, b.lo[1], b.hi[1]);
    wave_range<kNreg>(iz, b.lo[2], b.hi[2]);
    return b;
}

}  // namespace passk
}  // namespace sfcnl
