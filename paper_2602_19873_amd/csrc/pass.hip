// Neighbour pass (Sec. II-A, Sec. II-D Listing 1): decode a super-cluster's
// compressed list 64 entries at a time (Sec. II-B: lanes whose bitmask bit is
// clear take difference 1, the others read an info nibble and then any data
// nibbles), then evaluate one 8x8 particle tile per (j-cluster, set mask bit)
// on one wavefront and accumulate the SPH density and the neighbour count.
//
// Lane (il, jl) = (lane / 8, lane % 8) keeps i-particle il of every i-cluster
// in registers and takes j-particle jl of the current j-cluster, so a tile is
// one 64-lane step with no cross-lane traffic; the 8 partial sums per
// i-particle are combined once at the end. (The symmetric pass puts the
// i-side in the low lane bits instead, and for cluster size 8 takes its list
// entries in batches of 8; see k_pass_half.)
#include "internal.h"
#include "pass_common.h"

namespace sfcnl {
namespace {

using namespace passk;

// Waves (super-clusters) per block of the density passes: a launch-shape
// knob of the context (sfcnl_set_pass_waves, 1, 2 or 4). One wave per block
// lets a block release its slots as soon as its one list is done (7 % faster
// than four for the half-list pass on the uniform benchmark); the batch
// autotuner times all three.
constexpr int kPassWavesMax = 4;
// LDS per wave of the cluster-size-8 symmetric pass: a batch's 64
// j-particles (x, y, z, h^2), their 1/h and masses, and every tile lane's
// j-side partial sum and count for each of the batch's 8 entries
constexpr int kPassLds8 = (6 + 2 * 8) * kWave * 4;

// orders a wave's LDS accesses around it (the wave runs in lockstep)
__device__ __forceinline__ void pass_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

struct PassArgs {
    int64_t n;
    uint32_t nsc;
    const uint32_t *sc_info, *pool;
    const float *x, *y, *z, *h, *m;
    float *rho;
    int32_t *nnb;
    SegTable seg;  // batched systems: list indices are relative to the system's first cluster
    Period per;    // periodic axes (used by the kPbc kernels)
    const uint32_t *active;  // nullable: skip super-clusters with active[s] == 0 (full pass)
    const uint8_t *p_active;  // nullable: write only particles with p_active[i] != 0 (full pass)
    const uint32_t *gate;     // nullable: nothing to do when *gate <= gate_max
    uint32_t gate_max;
};

// A quarter of the halved M4 shape as two clamped cubes: with
// a = sat(c (1 - q)), c = 4^(-1/3), and u = sat(1/2 - q) (sat clamps to
// [0, 1], a free output modifier), a^3 - u^3 equals (1/2 - 3q^2 + 3q^3) / 4
// below q = 1/2, (1 - q)^3 / 4 up to q = 1 and zero beyond, so a pair
// outside the radius adds nothing and the sum needs no select. Adds
// m f(q) / 8 to acc (f(0) = 1) for q = r hinv, given rc = r c.
constexpr float kCubeC = 0.62996052494743658f;  // 4^(-1/3)

template <bool kMass>
__device__ __forceinline__ float add_shape(float acc, float m, float r, float rc, float hinv) {
    const float a = __builtin_amdgcn_fmed3f(__builtin_fmaf(-rc, hinv, kCubeC), 0.0f, 1.0f);
    const float u = __builtin_amdgcn_fmed3f(__builtin_fmaf(-r, hinv, 0.5f), 0.0f, 1.0f);
    const float a2 = a * a;
    const float u2 = u * u;
    if (!kMass) return __builtin_fmaf(-u2, u, __builtin_fmaf(a2, a, acc));
    return __builtin_fmaf(m, __builtin_fmaf(a2, a, -(u2 * u)), acc);
}

// One particle pair of a tile: the own-radius test (the self pair excluded)
// counts and adds m_j f(q)/8. Folding the self pair into the test measured
// faster here than masking it off around the call.
template <bool kMass, bool kPbc>
__device__ __forceinline__ void tile_pair(float xj, float yj, float zj, float mj, float xi, float yi, float zi,
                                          float h2, float hinv, bool self_pair, float &acc, int &cnt,
                                          const Period &per) {
    float dx = xj - xi;
    float dy = yj - yi;
    float dz = zj - zi;
    if (kPbc) wave_min_image(dx, dy, dz, per);  // minimum images on periodic axes
    const float dxx = dx * dx;
    const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
    const bool in = d2 < h2 && !self_pair;
    if (sfc_ballot(in)) {
        const float r = __builtin_amdgcn_sqrtf(d2);
        const float nacc = add_shape<kMass>(acc, mj, r, r * kCubeC, hinv);
        acc = in ? nacc : acc;
        cnt += in ? 1 : 0;
    }
}

// Lane roles for cluster size CS (64 / CS i-clusters per super-cluster):
//   CS = 8:  lane (il, jl) = (lane / 8, lane % 8) takes j-particle jl of the
//            listed j-cluster against i-particle il of every set i-cluster;
//   CS = 4:  lane (q, il, jl) = (lane / 16, lane / 4 % 4, lane % 4) takes
//            j-particle jl against i-particle il of i-clusters 4k + q;
//   CS = 16: lane (il, jq) = (lane / 4, lane % 4) takes j-particles 4t + jq
//            (t = 0..3) against i-particle il of every set i-cluster.
// Both passes are bound by VALU issue; for cluster sizes 4 and 8 six waves
// per SIMD (at most 80 VGPRs, a few registers spilled) hide more of the load
// latency than five without spills: measured 8 % faster for either list
// form. The symmetric pass of cluster size 8, which takes its entries in
// batches, needs more registers and runs five waves (2 registers spilled
// with compression; six waves spilled more and ran 2 % slower). Cluster size
// 16 holds four j-particles per lane; under the same cap it spills heavily,
// so it keeps its own register count.
template <int CS, bool kCompress, bool kMass, bool kCount, bool kPbc>
__global__ __launch_bounds__(kWave * kPassWavesMax) __attribute__((amdgpu_waves_per_eu(CS == 16 ? 1 : 6))) void k_pass(PassArgs a) {
    constexpr int kNsub = kScSize / CS;
    constexpr int kNreg = CS == 8 ? 8 : 4;
    constexpr int kNj = CS == 16 ? 4 : 1;     // j-particles per lane and entry
    constexpr int kGroup = CS == 8 ? 8 : 4;   // lanes sharing an i-particle
    const int lane = sfc_lane();
    const int w = threadIdx.x / kWave;
    // wave-uniform: keep the super-cluster index (and all derived from it) scalar
    const uint32_t s = (uint32_t)__builtin_amdgcn_readfirstlane((int)(xcd_remap(blockIdx.x, gridDim.x) * (blockDim.x / kWave) + w));
    if (s >= a.nsc || (a.active && !a.active[s]) || (a.gate && *a.gate <= a.gate_max)) return;
    const int64_t n = a.n;
    const int jl = lane & (kGroup - 1);

    // i particles; absent ones get a negative squared radius so that no pair
    // is accepted
    float ix[kNreg], iy[kNreg], iz[kNreg], ih2[kNreg], ihinv[kNreg];
#pragma unroll
    for (int k = 0; k < kNreg; k++) {
        const int64_t i = (int64_t)s * kScSize + ipart<CS>(k, lane);
        const bool v = i < n;
        ix[k] = v ? a.x[i] : 0.0f;
        iy[k] = v ? a.y[i] : 0.0f;
        iz[k] = v ? a.z[i] : 0.0f;
        const float hh = v ? a.h[i] : 1.0f;
        ih2[k] = v ? hh * hh : -1.0f;
        ihinv[k] = 1.0f / hh;
    }
    // acc[k] sums m_j f(q)/8 with f the spline shape (f(0) = 1)
    float acc[kNreg];
    int cnt_nb[kNreg];
#pragma unroll
    for (int k = 0; k < kNreg; k++) {
        acc[k] = 0.0f;
        cnt_nb[k] = 0;
    }

    const uint32_t own_c0 = s * kNsub;
    const uint32_t off = a.sc_info[2 * s], nj = a.sc_info[2 * s + 1];
    const uint8_t *mbytes = reinterpret_cast<const uint8_t *>(a.pool + off);
    const uint16_t *mshorts = reinterpret_cast<const uint16_t *>(a.pool + off);
    const uint32_t jbase = a.seg.on() ? a.seg.pbase[a.seg.sc_sys[s]] / CS : 0u;
    uint32_t p = off + (nj * (CS == 4 ? 2u : 1u) + 3u) / 4u;
    uint32_t prevj = 0xFFFFFFFFu;
    auto load_j = [&](uint32_t cj, float (&xj)[kNj], float (&yj)[kNj], float (&zj)[kNj], float (&mj)[kNj]) {
#pragma unroll
        for (int t = 0; t < kNj; t++) {
            const int64_t jp = (int64_t)cj * CS + (CS == 16 ? 4 * t + jl : jl);
            const bool vj = jp < n;
            xj[t] = vj ? a.x[jp] : kFar;
            yj[t] = vj ? a.y[jp] : kFar;
            zj[t] = vj ? a.z[jp] : kFar;
            mj[t] = kMass ? (vj ? a.m[jp] : 0.0f) : 1.0f;
        }
    };
    for (uint32_t b0 = 0; b0 < nj; b0 += kWave) {
        const uint32_t cnt = nj - b0 < (uint32_t)kWave ? nj - b0 : (uint32_t)kWave;
        uint32_t jv;
        if (kCompress) {
            jv = decode_segment(a.pool, p, cnt, prevj);
        } else {
            jv = (uint32_t)lane < cnt ? a.pool[p + b0 + lane] : 0u;
        }
        uint32_t mv = 0u;
        if ((uint32_t)lane < cnt) mv = CS == 4 ? (uint32_t)mshorts[b0 + lane] : (uint32_t)mbytes[b0 + lane];
        prevj = sfc_readlane(jv, (int)cnt - 1);
        jv += jbase;
        // software pipeline: the next entry's j-particles load while the
        // current entry's tiles run
        uint32_t cj = sfc_readlane(jv, 0);
        float xj[kNj], yj[kNj], zj[kNj], mj[kNj];
        load_j(cj, xj, yj, zj, mj);
        for (uint32_t e = 0; e < cnt; e++) {
            const uint32_t mk = sfc_readlane(mv, (int)e);
            const uint32_t ccur = cj;
            float cx[kNj], cy[kNj], cz[kNj], cm[kNj];
#pragma unroll
            for (int t = 0; t < kNj; t++) {
                cx[t] = xj[t];
                cy[t] = yj[t];
                cz[t] = zj[t];
                cm[t] = mj[t];
            }
            if (e + 1 < cnt) {
                cj = sfc_readlane(jv, (int)e + 1);
                load_j(cj, xj, yj, zj, mj);
            }
            // the j-cluster is one of our own i-clusters: exclude i == j
            const int self_c = (ccur >= own_c0 && ccur < own_c0 + kNsub) ? (int)(ccur - own_c0) : -1;
            if (CS == 8) {
                const int il = lane >> 3;
#pragma unroll
                for (int c = 0; c < kNreg; c++)
                    if ((mk >> c) & 1u)
                        tile_pair<kMass, kPbc>(cx[0], cy[0], cz[0], cm[0], ix[c], iy[c], iz[c], ih2[c], ihinv[c],
                                               c == self_c && il == jl, acc[c], cnt_nb[c], a.per);
            } else if (CS == 4) {
                const int il = (lane >> 2) & 3, q = lane >> 4;
#pragma unroll
                for (int k = 0; k < kNreg; k++)
                    if ((mk >> (4 * k)) & 0xFu)
                        tile_pair<kMass, kPbc>(cx[0], cy[0], cz[0], cm[0], ix[k], iy[k], iz[k], ih2[k], ihinv[k],
                                               4 * k + q == self_c && il == jl, acc[k], cnt_nb[k], a.per);
            } else {
                const int il = lane >> 2;
#pragma unroll
                for (int c = 0; c < kNreg; c++)
                    if ((mk >> c) & 1u) {
#pragma unroll
                        for (int t = 0; t < 4; t++)
                                tile_pair<kMass, kPbc>(cx[t], cy[t], cz[t], cm[t], ix[c], iy[c], iz[c], ih2[c],
                                                       ihinv[c], c == self_c && il == 4 * t + jl, acc[c], cnt_nb[c], a.per);
                    }
            }
        }
    }
    // sum the partials of each i-particle (the kGroup lanes sharing it)
#pragma unroll
    for (int k = 0; k < kNreg; k++) {
#pragma unroll
        for (int d = 1; d < kGroup; d <<= 1) {
            acc[k] += __shfl_xor(acc[k], d, 64);
            if (kCount) cnt_nb[k] += __shfl_xor(cnt_nb[k], d, 64);
        }
    }
    // lane stores register jl (its group has kGroup lanes, one per register)
    float r = acc[0];
    int nb = cnt_nb[0];
#pragma unroll
    for (int k = 1; k < kNreg; k++) {
        r = jl == k ? acc[k] : r;
        nb = jl == k ? cnt_nb[k] : nb;
    }
    const int64_t io = (int64_t)s * kScSize + ipart<CS>(jl, lane);
    if (io < n && (!a.p_active || a.p_active[io])) {
        const float hh = a.h[io];
        const float hinv = 1.0f / hh;
        const float mi = kMass ? a.m[io] : 1.0f;
        const float norm = 2.5464790894703255f * hinv * hinv * hinv;  // 8 / pi
        a.rho[io] = norm * __builtin_fmaf(8.0f, r, mi);
        if (kCount) a.nnb[io] = nb;
    }
}

// ---------------------------------------------------------------------------
// Half list: every stored pair (i, j), j > i, is evaluated once and feeds both
// particles: rho_i gets m_j W(r, h_i) when d2 < h_i^2 and rho_j gets m_i
// W(r, h_j) when d2 < h_j^2 (the symmetric evaluation of Sec. II-D). Shape
// sums (times masses) and counts are added atomically to rho and nnb, which
// start at zero; the j side is first reduced over the lanes that share a
// j-particle. k_pass_finalize then applies each particle's normalisation and
// self term. Float atomics make the summation order, and so the last bits of
// rho, vary from run to run; the counts are exact.
// ---------------------------------------------------------------------------

// One stored pair feeding both particles: own-radius counts on either side
// and the two shape sums (zero outside each radius). The caller masks pairs
// that the half list does not hold off.
template <bool kMass, bool kPbc>
__device__ __forceinline__ void half_pair(float xj, float yj, float zj, float mj, float hj2, float hjinv, float xi,
                                          float yi, float zi, float mi, float hi2, float hiinv, float &acc_i,
                                          int &cnt_i, float &acc_j, int &cnt_j, const Period &per, bool wrap = true) {
    float dx = xj - xi;
    float dy = yj - yi;
    float dz = zj - zi;
    if (kPbc && wrap) wave_min_image(dx, dy, dz, per);  // minimum images on periodic axes (wrap: wave-uniform)
    const float dxx = dx * dx;
    const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
    cnt_i += d2 < hi2 ? 1 : 0;
    cnt_j += d2 < hj2 ? 1 : 0;
    const float r = __builtin_amdgcn_sqrtf(d2);
    const float rc = r * kCubeC;
    acc_i = add_shape<kMass>(acc_i, mj, r, rc, hiinv);
    acc_j = add_shape<kMass>(acc_j, mi, r, rc, hjinv);
}

template <int CS, bool kCompress, bool kMass, bool kCount, bool kPbc>
__global__ __launch_bounds__(kWave * kPassWavesMax) __attribute__((amdgpu_waves_per_eu(CS == 16 ? 1 : (CS == 8 ? 5 : 6)))) void k_pass_half(PassArgs a) {
    constexpr int kNsub = kScSize / CS;
    constexpr int kNreg = CS == 8 ? 8 : 4;
    constexpr int kNj = CS == 16 ? 4 : 1;
    constexpr int kIL = CS == 8 ? 8 : 16;  // lanes per j-particle (the i side, low bits)
    const int lane = sfc_lane();
    const int w = threadIdx.x / kWave;
    // wave-uniform: keep the super-cluster index (and all derived from it) scalar
    const uint32_t s = (uint32_t)__builtin_amdgcn_readfirstlane((int)(xcd_remap(blockIdx.x, gridDim.x) * (blockDim.x / kWave) + w));
    if (s >= a.nsc) return;
    const int64_t n = a.n;
    const int jq = CS == 8 ? lane >> 3 : lane >> 4;  // j-particle slot of the lane

    // i particles; absent ones are put far away (every distance overflows)
    float ix[kNreg], iy[kNreg], iz[kNreg], ih2[kNreg], ihinv[kNreg], im[kNreg];
#pragma unroll
    for (int k = 0; k < kNreg; k++) {
        const int64_t i = (int64_t)s * kScSize + ipart_sym<CS>(k, lane);
        const bool v = i < n;
        ix[k] = v ? a.x[i] : kFar;
        iy[k] = v ? a.y[i] : kFar;
        iz[k] = v ? a.z[i] : kFar;
        const float hh = v ? a.h[i] : 1.0f;
        ih2[k] = v ? hh * hh : -1.0f;
        ihinv[k] = 1.0f / hh;
        // a batch's padding particles (index < n, NaN radius and mass) get a
        // zero mass: their shape is zero, but 0 * NaN would not be
        im[k] = kMass ? ((v && hh > 0.0f) ? a.m[i] : 0.0f) : 1.0f;
    }
    float acc[kNreg];
    int cnt_nb[kNreg];
#pragma unroll
    for (int k = 0; k < kNreg; k++) {
        acc[k] = 0.0f;
        cnt_nb[k] = 0;
    }

    const uint32_t own_c0 = s * kNsub;
    const uint32_t off = a.sc_info[2 * s], nj = a.sc_info[2 * s + 1];
    const uint8_t *mbytes = reinterpret_cast<const uint8_t *>(a.pool + off);
    const uint16_t *mshorts = reinterpret_cast<const uint16_t *>(a.pool + off);
    const uint32_t jbase = a.seg.on() ? a.seg.pbase[a.seg.sc_sys[s]] / CS : 0u;
    // periodic: a batch whose j-particles all lie within half a period of
    // both ends of the i-box skips the minimum image (far_from_box)
    const IBox ib = kPbc && CS == 8 ? ibox_of<kNreg>(ix, iy, iz) : IBox{};
    // Cluster size 8: the entries of a decoded segment 8 at a time. Lane
    // (q, r) = (lane / 8, lane % 8) loads particle r of the batch's entry q
    // (one load per field for the batch; loading the next batch behind the
    // current one's tiles measured slower, the extra registers spilled),
    // derives its squared radius and reciprocal once and leaves them in LDS,
    // where the tile lanes of entry q read j-particle jq. Every tile lane's
    // j-side partial sum and count of an entry go to LDS too, and after the
    // batch lane (q, r) adds the 8 partials of its particle and updates rho
    // and nnb with one atomic each.
    // this wave's LDS (one wave-uniform base; the arrays at fixed offsets)
    extern __shared__ float4 s_pass_dyn[];
    float *const s_base = reinterpret_cast<float *>(s_pass_dyn) +
                          (size_t)__builtin_amdgcn_readfirstlane(w) * (kPassLds8 / 4);
    float4 *const s_jb = reinterpret_cast<float4 *>(s_base);
    float *const s_jh = s_base + 4 * kWave;
    float *const s_jm = s_base + 5 * kWave;
    float *const s_ja = s_base + 6 * kWave;
    int *const s_jc = reinterpret_cast<int *>(s_base + 14 * kWave);
    struct JLoad {
        float x, y, z, h, m;
        uint32_t q;  // particle index (n < 2^31)
        bool v;
    };
    auto load_batch8 = [&](uint32_t jvl, uint32_t q0, uint32_t cnt, JLoad &f) {
        const uint32_t e = q0 + (uint32_t)(lane >> 3);
        f.v = e < cnt;
        const uint32_t cjb = (uint32_t)__shfl((int)jvl, (int)(f.v ? e : q0), kWave);
        f.q = cjb * CS + (uint32_t)(lane & 7);
        f.v = f.v && f.q < n;
        const uint32_t qc = f.q < n ? f.q : (uint32_t)(n - 1);  // loads of a clamped index stay in flight
        f.x = a.x[qc];
        f.y = a.y[qc];
        f.z = a.z[qc];
        f.h = a.h[qc];
        f.m = kMass ? a.m[qc] : 1.0f;
    };
    auto half_entries8 = [&](uint32_t mvl, uint32_t jvl, uint32_t cnt) {
        JLoad f;
        load_batch8(jvl, 0, cnt, f);
        for (uint32_t q0 = 0; q0 < cnt; q0 += 8) {
            // the batch's j-particles into LDS (absent ones: far away, radius
            // -1, mass 0; NaN padding never pairs either)
            const float hh = f.v ? f.h : -1.0f;
            const bool vh = hh > 0.0f;
            const float4 jv4 = make_float4(f.v ? f.x : kFar, f.v ? f.y : kFar, f.v ? f.z : kFar, vh ? hh * hh : -1.0f);
            s_jb[lane] = jv4;
            s_jh[lane] = vh ? __builtin_amdgcn_rcpf(hh) : 1.0f;
            if (kMass) s_jm[lane] = vh ? f.m : 0.0f;
            const bool ev = f.v;
            const uint32_t jq_p = f.q;  // this lane's batch particle (for the atomics)
            pass_wave_sync();
            const uint32_t bn = cnt - q0 < 8u ? cnt - q0 : 8u;
            const bool wrap = kPbc && sfc_ballot((uint32_t)(lane >> 3) < bn && far_from_box(jv4, ib, a.per)) != 0;
            const int il = lane & 7;
            for (uint32_t q = 0; q < bn; q++) {
                const uint32_t mk = sfc_readlane(mvl, (int)(q0 + q));
                const uint32_t cj = sfc_readlane(jvl, (int)(q0 + q));
                const float4 jb = s_jb[q * 8 + jq];
                const float hjinv = s_jh[q * 8 + jq];
                const float mj = kMass ? s_jm[q * 8 + jq] : 1.0f;
                float accj = 0.0f;
                int cntj = 0;
                // inside the super-cluster only j > i counts
                const int self_c = (cj >= own_c0 && cj < own_c0 + kNsub) ? (int)(cj - own_c0) : -1;
#pragma unroll
                for (int c = 0; c < kNreg; c++)
                    if (((mk >> c) & 1u) && (self_c < 0 || c < self_c || (c == self_c && jq > il)))
                        half_pair<kMass, kPbc>(jb.x, jb.y, jb.z, mj, jb.w, hjinv, ix[c], iy[c], iz[c], im[c], ih2[c],
                                               ihinv[c], acc[c], cnt_nb[c], accj, cntj, a.per, wrap);
                s_ja[q * kWave + lane] = accj;
                s_jc[q * kWave + lane] = cntj;
            }
            pass_wave_sync();
            // lane (q, r): j-particle r of entry q, whose 8 partials (tile
            // lanes 8r .. 8r + 7 of entry q) sit at 8 lane .. 8 lane + 7
            if (ev && (uint32_t)(lane >> 3) < bn) {
                const int4 c0 = reinterpret_cast<const int4 *>(s_jc)[2 * lane];
                const int4 c1 = reinterpret_cast<const int4 *>(s_jc)[2 * lane + 1];
                const int c = ((c0.x + c0.y) + (c0.z + c0.w)) + ((c1.x + c1.y) + (c1.z + c1.w));
                if (c != 0) {
                    const float4 a0 = reinterpret_cast<const float4 *>(s_ja)[2 * lane];
                    const float4 a1 = reinterpret_cast<const float4 *>(s_ja)[2 * lane + 1];
                    atomicAdd(&a.rho[jq_p], ((a0.x + a0.y) + (a0.z + a0.w)) + ((a1.x + a1.y) + (a1.z + a1.w)));
                    if (kCount) atomicAdd(&a.nnb[jq_p], c);
                }
            }
            pass_wave_sync();  // the next batch rewrites the LDS arrays
            if (q0 + 8 < cnt) load_batch8(jvl, q0 + 8, cnt, f);
        }
    };

    uint32_t p = off + (nj * (CS == 4 ? 2u : 1u) + 3u) / 4u;
    uint32_t prevj = 0xFFFFFFFFu;
    for (uint32_t b0 = 0; b0 < nj; b0 += kWave) {
        const uint32_t cnt = nj - b0 < (uint32_t)kWave ? nj - b0 : (uint32_t)kWave;
        uint32_t jv;
        if (kCompress) {
            jv = decode_segment(a.pool, p, cnt, prevj);
        } else {
            jv = (uint32_t)lane < cnt ? a.pool[p + b0 + lane] : 0u;
        }
        uint32_t mv = 0u;
        if ((uint32_t)lane < cnt) mv = CS == 4 ? (uint32_t)mshorts[b0 + lane] : (uint32_t)mbytes[b0 + lane];
        prevj = sfc_readlane(jv, (int)cnt - 1);
        jv += jbase;
        if constexpr (CS == 8) {
            half_entries8(mv, jv, cnt);
            continue;
        }
        // software pipeline: the next entry's j-particles load while the
        // current entry's tiles run
        float nx[kNj], ny[kNj], nz[kNj], nm[kNj], nh[kNj];
        auto load_j = [&](uint32_t cjn) {
#pragma unroll
            for (int t = 0; t < kNj; t++) {
                const int64_t q = (int64_t)cjn * CS + (CS == 16 ? 4 * t + jq : jq);
                const bool vj = q < n;
                nx[t] = vj ? a.x[q] : kFar;
                ny[t] = vj ? a.y[q] : kFar;
                nz[t] = vj ? a.z[q] : kFar;
                nh[t] = vj ? a.h[q] : -1.0f;
                nm[t] = kMass ? ((vj && nh[t] > 0.0f) ? a.m[q] : 0.0f) : 1.0f;
            }
        };
        load_j(sfc_readlane(jv, 0));
        for (uint32_t e = 0; e < cnt; e++) {
            const uint32_t mk = sfc_readlane(mv, (int)e);
            const uint32_t cj = sfc_readlane(jv, (int)e);
            float xj[kNj], yj[kNj], zj[kNj], mj[kNj], hj2[kNj], hjinv[kNj], accj[kNj];
            int cntj[kNj];
            int64_t jp[kNj];
#pragma unroll
            for (int t = 0; t < kNj; t++) {
                jp[t] = (int64_t)cj * CS + (CS == 16 ? 4 * t + jq : jq);
                xj[t] = nx[t];
                yj[t] = ny[t];
                zj[t] = nz[t];
                mj[t] = nm[t];
                const bool vj = nh[t] > 0.0f;  // absent: -1 (NaN padding never pairs)
                hj2[t] = vj ? nh[t] * nh[t] : -1.0f;
                hjinv[t] = vj ? __builtin_amdgcn_rcpf(nh[t]) : 1.0f;
                accj[t] = 0.0f;
                cntj[t] = 0;
            }
            if (e + 1 < cnt) load_j(sfc_readlane(jv, (int)e + 1));
            // inside the super-cluster only j > i counts
            const int self_c = (cj >= own_c0 && cj < own_c0 + kNsub) ? (int)(cj - own_c0) : -1;
            auto keep = [&](int ci, int ipos, int jpos) {
                return self_c < 0 || ci < self_c || (ci == self_c && jpos > ipos);
            };
            // (cluster size 8 takes its entries in batches, above)
            if constexpr (CS == 4) {
                const int il = lane & 3, q = (lane >> 2) & 3;
#pragma unroll
                for (int k = 0; k < kNreg; k++)
                    if (((mk >> (4 * k)) & 0xFu) && keep(4 * k + q, il, jq))
                        half_pair<kMass, kPbc>(xj[0], yj[0], zj[0], mj[0], hj2[0], hjinv[0], ix[k], iy[k], iz[k],
                                               im[k], ih2[k], ihinv[k], acc[k], cnt_nb[k], accj[0], cntj[0], a.per);
            } else {
                const int il = lane & 15;
#pragma unroll
                for (int c = 0; c < kNreg; c++)
                    if ((mk >> c) & 1u) {
#pragma unroll
                        for (int t = 0; t < 4; t++)
                            if (keep(c, il, 4 * t + jq))
                                half_pair<kMass, kPbc>(xj[t], yj[t], zj[t], mj[t], hj2[t], hjinv[t], ix[c], iy[c],
                                                       iz[c], im[c], ih2[c], ihinv[c], acc[c], cnt_nb[c], accj[t],
                                                       cntj[t], a.per);
                    }
            }
            // j side: sum over the i lanes of each j-particle (one DPP row
            // group), then one atomic per j-particle
            bool any = false;
#pragma unroll
            for (int t = 0; t < kNj; t++) any = any || cntj[t] != 0;
            if (sfc_ballot(any)) {
#pragma unroll
                for (int t = 0; t < kNj; t++) {
                    group_sum<kIL>(accj[t], cntj[t]);
                    if ((lane & (kIL - 1)) == 0 && cntj[t] != 0) {
                        atomicAdd(&a.rho[jp[t]], accj[t]);
                        if (kCount) atomicAdd(&a.nnb[jp[t]], cntj[t]);
                    }
                }
            }
        }
    }
    // i side: sum the partials of each i-particle over the j lanes (the high
    // lane bits), then one atomic per particle; the lane with j slot k takes
    // register k
#pragma unroll
    for (int k = 0; k < kNreg; k++) {
#pragma unroll
        for (int d = kIL; d < kWave; d <<= 1) {
            acc[k] += __shfl_xor(acc[k], d, 64);
            cnt_nb[k] += __shfl_xor(cnt_nb[k], d, 64);
        }
    }
    float r = acc[0];
    int nb = cnt_nb[0];
#pragma unroll
    for (int k = 1; k < kNreg; k++) {
        r = jq == k ? acc[k] : r;
        nb = jq == k ? cnt_nb[k] : nb;
    }
    const int64_t io = (int64_t)s * kScSize + ipart_sym<CS>(jq, lane);
    if (io < n && nb != 0) {
        atomicAdd(&a.rho[io], r);
        if (kCount) atomicAdd(&a.nnb[io], nb);
    }
}

// rho_i = 8 / (pi h_i^3) (m_i + 8 S_i), S_i the summed m_j f / 8.
template <bool kMass>
__global__ __launch_bounds__(256) void k_pass_finalize(int64_t n, const float *__restrict__ h,
                                                       const float *__restrict__ m, float *__restrict__ rho) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float hinv = 1.0f / h[i];
    const float norm = 2.5464790894703255f * hinv * hinv * hinv;  // 8 / pi
    rho[i] = norm * __builtin_fmaf(8.0f, rho[i], kMass ? m[i] : 1.0f);
}

struct DecodeArgs {
    uint32_t nsc;
    int mask_bytes;
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
    const uint16_t *mshorts = reinterpret_cast<const uint16_t *>(a.pool + off);
    uint32_t p = off + (nj * (uint32_t)a.mask_bytes + 3u) / 4u;
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
            a.mask[o + b0 + lane] = a.mask_bytes == 2 ? mshorts[b0 + lane] : (uint16_t)mbytes[b0 + lane];
        }
    }
}

template <int CS, bool kPbc>
void launch_pass(int variant, unsigned g, unsigned tpb, hipStream_t st, const PassArgs &a) {
    switch (variant) {
        case 7: k_pass<CS, true, true, true, kPbc><<<g, tpb, 0, st>>>(a); break;
        case 6: k_pass<CS, true, true, false, kPbc><<<g, tpb, 0, st>>>(a); break;
        case 5: k_pass<CS, true, false, true, kPbc><<<g, tpb, 0, st>>>(a); break;
        case 4: k_pass<CS, true, false, false, kPbc><<<g, tpb, 0, st>>>(a); break;
        case 3: k_pass<CS, false, true, true, kPbc><<<g, tpb, 0, st>>>(a); break;
        case 2: k_pass<CS, false, true, false, kPbc><<<g, tpb, 0, st>>>(a); break;
        case 1: k_pass<CS, false, false, true, kPbc><<<g, tpb, 0, st>>>(a); break;
        default: k_pass<CS, false, false, false, kPbc><<<g, tpb, 0, st>>>(a); break;
    }
}

template <int CS, bool kPbc>
void launch_pass_half(int variant, unsigned g, unsigned tpb, hipStream_t st, const PassArgs &a) {
    const size_t lds = CS == 8 ? (size_t)(tpb / kWave) * kPassLds8 : 0;
    switch (variant) {
        case 7: k_pass_half<CS, true, true, true, kPbc><<<g, tpb, lds, st>>>(a); break;
        case 6: k_pass_half<CS, true, true, false, kPbc><<<g, tpb, lds, st>>>(a); break;
        case 5: k_pass_half<CS, true, false, true, kPbc><<<g, tpb, lds, st>>>(a); break;
        case 4: k_pass_half<CS, true, false, false, kPbc><<<g, tpb, lds, st>>>(a); break;
        case 3: k_pass_half<CS, false, true, true, kPbc><<<g, tpb, lds, st>>>(a); break;
        case 2: k_pass_half<CS, false, true, false, kPbc><<<g, tpb, lds, st>>>(a); break;
        case 1: k_pass_half<CS, false, false, true, kPbc><<<g, tpb, lds, st>>>(a); break;
        default: k_pass_half<CS, false, false, false, kPbc><<<g, tpb, lds, st>>>(a); break;
    }
}

template <bool kPbc>
void launch_any(int cs, bool half, int variant, unsigned g, unsigned tpb, hipStream_t st, const PassArgs &a) {
    if (half) {
        if (cs == 4)
            launch_pass_half<4, kPbc>(variant, g, tpb, st, a);
        else if (cs == 16)
            launch_pass_half<16, kPbc>(variant, g, tpb, st, a);
        else
            launch_pass_half<8, kPbc>(variant, g, tpb, st, a);
    } else if (cs == 4) {
        launch_pass<4, kPbc>(variant, g, tpb, st, a);
    } else if (cs == 16) {
        launch_pass<16, kPbc>(variant, g, tpb, st, a);
    } else {
        launch_pass<8, kPbc>(variant, g, tpb, st, a);
    }
}

}  // namespace
}  // namespace sfcnl

using namespace sfcnl;

int sfcnl::pass_impl(sfcnl_ctx ctx, int64_t n, int cs, int compress, int half, const uint32_t *d_sc_info,
                     const uint32_t *d_pool, const float *d_x, const float *d_y, const float *d_z, const float *d_h,
                     const float *d_m, float *d_rho, int32_t *d_nnb, const SegTable &seg, const Period &per,
                     const uint32_t *active, const uint8_t *p_active, const uint32_t *gate, uint32_t gate_max) {
    if ((active || p_active || gate) && half)
        return set_err(ctx, SFCNL_E_ARG, "nlist_pass: a restricted pass needs the full list");
    PassArgs a{n, (uint32_t)((n + kScSize - 1) / kScSize), d_sc_info, d_pool, d_x, d_y, d_z, d_h, d_m, d_rho, d_nnb,
               seg, per, active, p_active, gate, gate_max};
    const int waves = ctx->pass_waves;
    const unsigned g = blocks_for(a.nsc, waves);
    const unsigned tpb = (unsigned)(kWave * waves);
    hipStream_t st = ctx->stream;
    const int variant = (compress ? 4 : 0) | (d_m ? 2 : 0) | (d_nnb ? 1 : 0);
    prof_mark(ctx, kStagePass, false);
    if (half) {
        // accumulators start at zero (fill kernels, so the call can sit in a graph)
        int rc = fill2_u32(ctx, reinterpret_cast<uint32_t *>(d_rho), reinterpret_cast<uint32_t *>(d_nnb), n, 0u);
        if (rc) return rc;
    }
    if (per.on())
        launch_any<true>(cs, half, variant, g, tpb, st, a);
    else
        launch_any<false>(cs, half, variant, g, tpb, st, a);
    SFCNL_LAUNCHED(ctx);
    if (half) {
        if (d_m)
            k_pass_finalize<true><<<blocks_for(n, 256), 256, 0, st>>>(n, d_h, d_m, d_rho);
        else
            k_pass_finalize<false><<<blocks_for(n, 256), 256, 0, st>>>(n, d_h, d_m, d_rho);
        SFCNL_LAUNCHED(ctx);
    }
    prof_mark(ctx, kStagePass, true);
    return SFCNL_OK;
}

static bool cs_ok(int cs) { return cs == 4 || cs == 8 || cs == 16; }

extern "C" int nlist_pass(sfcnl_ctx ctx, int64_t n, int cluster_size, int compress, int half,
                          const uint32_t *d_sc_info, const uint32_t *d_pool, const float *d_x, const float *d_y,
                          const float *d_z, const float *d_h, const float *d_m, float *d_rho, int32_t *d_nnb,
                          const float *h_period) {
    if (!ctx) return SFCNL_E_ARG;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "nlist_pass: n out of range");
    if (!cs_ok(cluster_size)) return set_err(ctx, SFCNL_E_ARG, "nlist_pass: cluster_size %d not supported", cluster_size);
    if (compress != 0 && compress != 1) return set_err(ctx, SFCNL_E_ARG, "nlist_pass: compress must be 0 or 1");
    if (half != 0 && half != 1) return set_err(ctx, SFCNL_E_ARG, "nlist_pass: half must be 0 or 1");
    if (!period_ok(h_period)) return set_err(ctx, SFCNL_E_ARG, "nlist_pass: period must be 3 finite values >= 0");
    if (n == 0) return SFCNL_OK;
    if (!d_sc_info || !d_pool || !d_x || !d_y || !d_z || !d_h || !d_rho)
        return set_err(ctx, SFCNL_E_ARG, "nlist_pass: null pointer");
    return pass_impl(ctx, n, cluster_size, compress, half, d_sc_info, d_pool, d_x, d_y, d_z, d_h, d_m, d_rho, d_nnb,
                     SegTable{}, make_period(h_period));
}

extern "C" int nlist_decode(sfcnl_ctx ctx, int64_t n, int cluster_size, int compress, const uint32_t *d_sc_info,
                            const uint32_t *d_pool, const uint32_t *d_offsets, uint32_t *d_j, uint16_t *d_mask) {
    if (!ctx) return SFCNL_E_ARG;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "nlist_decode: n out of range");
    if (!cs_ok(cluster_size))
        return set_err(ctx, SFCNL_E_ARG, "nlist_decode: cluster_size %d not supported", cluster_size);
    if (n == 0) return SFCNL_OK;
    if (!d_sc_info || !d_pool || !d_offsets || !d_j || !d_mask)
        return set_err(ctx, SFCNL_E_ARG, "nlist_decode: null pointer");
    DecodeArgs a{(uint32_t)((n + kScSize - 1) / kScSize), cluster_size == 4 ? 2 : 1, d_sc_info, d_pool, d_offsets,
                 d_j, d_mask};
    const unsigned g = blocks_for(a.nsc, kWavesPerBlock);
    if (compress)
        k_decode<true><<<g, 256, 0, ctx->stream>>>(a);
    else
        k_decode<false><<<g, 256, 0, ctx->stream>>>(a);
    SFCNL_LAUNCHED(ctx);
    return SFCNL_OK;
}
