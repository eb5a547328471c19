// Compressed 1x1 list: the combination of the index compression with a full
// neighbour list that the paper leaves as future work (Sec. V). Row i holds
// particle i's neighbours in the pair set (j != i, d2 < max(h_i, h_j)^2) in
// ascending order, encoded as the index stream of a super-cluster list
// without masks (differences from -1, nibble segments of 64 values,
// Sec. II-B/II-C); rows follow each other in particle order.
//
// Build: from a full cluster list. One wavefront per particle decodes its
// super-cluster's list 64 entries at a time, keeps the entries whose mask has
// the particle's i-cluster bit (a ballot compaction into LDS), tests the
// particles of 64 / CS of those j-clusters per step with the exact FP32 pair
// formula, appends the survivors (already in ascending order) to a pending
// buffer in LDS and encodes a segment whenever 64 are pending. A sizing run
// and a writing run around a prefix sum place the rows deterministically.
//
// Pass: one wavefront per particle decodes 64 neighbours per step and
// evaluates each lane's pair once; no tile of a cluster pair is wasted.
#include "internal.h"
#include "pass_common.h"

namespace sfcnl {
namespace {

using namespace passk;

constexpr int kSegCap = 80;  // words of one 64-value segment: 2 + (64 + 512 + 7) / 8

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t nibbles_of(uint32_t v) { return (32u - (uint32_t)__clz((int)v) + 3u) >> 2; }

struct RowArgs {
    int64_t n;
    const uint32_t *sc_info, *pool;  // the full cluster list
    const float *x, *y, *z, *h;
    Period per;
    int compress;                    // encoding of the rows
    uint32_t *row_words;             // sizing run: words of each row
    const uint32_t *row_off;         // writing run: prefix sum of row_words (n + 1)
    uint32_t *row_info;              // writing run: {word offset, count} per particle
    uint32_t *out;
    uint64_t out_words;
    uint32_t *status;
};

template <int CS, bool kCompIn, bool kWrite, bool kPbc>
__global__ __launch_bounds__(256) void k_rows(RowArgs a) {
    constexpr int kPerStep = kWave / CS;  // candidate j-clusters tested per step
    __shared__ uint32_t s_cand[kWavesPerBlock][kWave];
    __shared__ uint32_t s_pend[kWavesPerBlock][2 * kWave];
    __shared__ uint32_t s_seg[kWavesPerBlock][kSegCap];
    const int lane = sfc_lane();
    const int w = threadIdx.x / kWave;
    const uint64_t lt = sfc_lt_mask();
    const uint32_t i =
        (uint32_t)__builtin_amdgcn_readfirstlane((int)(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + w));
    if (i >= a.n) return;
    const uint32_t s = i / kScSize, c = (i % kScSize) / CS;
    const float xi = a.x[i], yi = a.y[i], zi = a.z[i], hi = a.h[i];
    const float hi2 = hi * hi;
    const uint32_t off = a.sc_info[2 * s], nj = a.sc_info[2 * s + 1];
    const uint8_t *mbytes = reinterpret_cast<const uint8_t *>(a.pool + off);
    const uint16_t *mshorts = reinterpret_cast<const uint16_t *>(a.pool + off);
    uint32_t p = off + (nj * (CS == 4 ? 2u : 1u) + 3u) / 4u;

    uint32_t *out = nullptr;
    if (kWrite) {
        const uint32_t ro = a.row_off[i], re = a.row_off[i + 1];
        if ((uint64_t)re > a.out_words) {  // the pool is too small: an empty row, reported
            if (lane == 0) {
                a.row_info[2 * (size_t)i] = ro;
                a.row_info[2 * (size_t)i + 1] = 0u;
                atomicOr(&a.status[kStPoolOverflow], 1u);
            }
            return;
        }
        out = a.out + ro;
    }
    uint32_t *cand = s_cand[w];
    uint32_t *pend = s_pend[w];
    uint32_t *seg = s_seg[w];
    uint32_t npend = 0, count = 0, words = 0;
    uint32_t prevrow = 0xFFFFFFFFu;  // last neighbour emitted (differences start from -1)

    // emits the first m pending neighbours as one segment (or raw words)
    auto flush = [&](uint32_t m) {
        const bool valid = (uint32_t)lane < m;
        const uint32_t j = valid ? pend[lane] : 0u;
        if (a.compress) {
            uint32_t jprev = __shfl_up(j, 1, 64);
            if (lane == 0) jprev = prevrow;
            const uint32_t v = j - jprev;
            const bool nonone = valid && v != 1u;
            const uint64_t mk = sfc_ballot(nonone);
            const bool small = v <= 9u;
            const uint32_t nn = nibbles_of(v);
            const uint32_t ndata = (nonone && !small) ? nn : 0u;
            const uint32_t ninfo = (uint32_t)sfc_popc(mk);
            const uint32_t incl = sfc_incl_scan(ndata);
            const uint32_t total_nib = ninfo + sfc_readlane(incl, kWave - 1);
            const uint32_t segw = 2u + (total_nib + 7u) / 8u;
            if (kWrite) {
                const uint32_t info = small ? v + 6u : nn - 1u;
                const uint32_t ipos = (uint32_t)sfc_popc(mk & lt);
                const uint32_t dpos = ninfo + incl - ndata;
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
                for (uint32_t q = lane; q < segw; q += kWave) out[words + q] = seg[q];
            }
            words += segw;
        } else {
            if (kWrite && valid) out[words + lane] = j;
            words += m;
        }
        prevrow = sfc_readlane(j, (int)m - 1);
        count += m;
        wave_sync();
    };

    uint32_t prevj = 0xFFFFFFFFu;  // decoding state of the cluster list
    for (uint32_t b0 = 0; b0 < nj; b0 += kWave) {
        const uint32_t cntb = nj - b0 < (uint32_t)kWave ? nj - b0 : (uint32_t)kWave;
        uint32_t jv;
        if (kCompIn)
            jv = decode_segment(a.pool, p, cntb, prevj);
        else
            jv = (uint32_t)lane < cntb ? a.pool[p + b0 + lane] : 0u;
        uint32_t mv = 0u;
        if ((uint32_t)lane < cntb) mv = CS == 4 ? (uint32_t)mshorts[b0 + lane] : (uint32_t)mbytes[b0 + lane];
        prevj = sfc_readlane(jv, (int)cntb - 1);
        // the entries whose mask holds our i-cluster, in list (ascending) order
        const bool sel = (uint32_t)lane < cntb && ((mv >> c) & 1u);
        const uint64_t bsel = sfc_ballot(sel);
        const uint32_t ncand = (uint32_t)sfc_popc(bsel);
        if (sel) cand[sfc_popc(bsel & lt)] = jv;
        wave_sync();
        for (uint32_t k0 = 0; k0 < ncand; k0 += kPerStep) {
            const uint32_t kk = k0 + (uint32_t)(lane / CS);
            const uint32_t j = (kk < ncand ? cand[kk < ncand ? kk : 0] : 0u) * CS + (uint32_t)(lane % CS);
            const bool valid = kk < ncand && j < a.n;
            float dx = valid ? a.x[j] - xi : 0.0f;
            float dy = valid ? a.y[j] - yi : 0.0f;
            float dz = valid ? a.z[j] - zi : 0.0f;
            if (kPbc) wave_min_image(dx, dy, dz, a.per);
            const float hj = valid ? a.h[j] : 0.0f;
            const float dxx = dx * dx;
            const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
            const bool in = valid && j != i && d2 < fmaxf(hi2, hj * hj);
            const uint64_t b = sfc_ballot(in);
            if (in) pend[npend + (uint32_t)sfc_popc(b & lt)] = j;
            npend += (uint32_t)sfc_popc(b);
            wave_sync();
            if (npend >= (uint32_t)kWave) {
                flush(kWave);
                const uint32_t rest = npend - kWave;
                const uint32_t tmp = (uint32_t)lane < rest ? pend[kWave + lane] : 0u;
                wave_sync();
                if ((uint32_t)lane < rest) pend[lane] = tmp;
                npend = rest;
                wave_sync();
            }
        }
        wave_sync();  // cand is refilled by the next block
    }
    if (npend) flush(npend);
    if (lane == 0) {
        if (kWrite) {
            a.row_info[2 * (size_t)i] = a.row_off[i];
            a.row_info[2 * (size_t)i + 1] = count;
        } else {
            a.row_words[i] = words;
        }
    }
}

struct RowPassArgs {
    int64_t n;
    const uint32_t *row_info, *pool;
    const float *x, *y, *z, *h, *m;
    Period per;
    float *rho;
    int32_t *nnb;
};

// Density and counts from the rows: the own-radius subset of each row.
template <bool kCompress, bool kMass, bool kCount, bool kPbc>
__global__ __launch_bounds__(256) void k_pass_rows(RowPassArgs a) {
    const int lane = sfc_lane();
    const int w = threadIdx.x / kWave;
    const uint32_t i =
        (uint32_t)__builtin_amdgcn_readfirstlane((int)(xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + w));
    if (i >= a.n) return;
    const float xi = a.x[i], yi = a.y[i], zi = a.z[i], hi = a.h[i];
    const float hi2 = hi * hi;
    const float hinv = 1.0f / hi;
    const uint32_t off = a.row_info[2 * (size_t)i], cnt = a.row_info[2 * (size_t)i + 1];
    uint32_t p = off;
    uint32_t prevj = 0xFFFFFFFFu;
    float acc = 0.0f;
    uint32_t nb = 0;
    for (uint32_t b0 = 0; b0 < cnt; b0 += kWave) {
        const uint32_t c = cnt - b0 < (uint32_t)kWave ? cnt - b0 : (uint32_t)kWave;
        uint32_t jv;
        if (kCompress)
            jv = decode_segment(a.pool, p, c, prevj);
        else
            jv = (uint32_t)lane < c ? a.pool[off + b0 + lane] : 0u;
        prevj = sfc_readlane(jv, (int)c - 1);
        const bool valid = (uint32_t)lane < c;
        float dx = valid ? a.x[jv] - xi : 0.0f;
        float dy = valid ? a.y[jv] - yi : 0.0f;
        float dz = valid ? a.z[jv] - zi : 0.0f;
        if (kPbc) wave_min_image(dx, dy, dz, a.per);
        const float dxx = dx * dx;
        const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dxx));
        const bool in = valid && d2 < hi2;
        const uint64_t bal = sfc_ballot(in);
        if (bal) {
            nb += (uint32_t)sfc_popc(bal);
            const float q = __builtin_amdgcn_sqrtf(d2) * hinv;
            const float t1 = q - 1.0f;
            const float q2 = q * q;
            const float inner = __builtin_fmaf(3.0f * q2, t1, 0.5f);
            const float outer = -(t1 * t1) * t1;
            const float wq = q < 0.5f ? inner : outer;
            const float mj = kMass ? (in ? a.m[jv] : 0.0f) : 1.0f;
            acc = in ? __builtin_fmaf(mj, wq, acc) : acc;
        }
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) acc += __shfl_xor(acc, d, 64);
    if (lane == 0) {
        const float norm = 2.5464790894703255f * hinv * hinv * hinv;  // 8 / pi
        a.rho[i] = norm * __builtin_fmaf(2.0f, acc, kMass ? a.m[i] : 1.0f);
        if (kCount) a.nnb[i] = (int32_t)nb;
    }
}

template <int CS, bool kWrite, bool kPbc>
void launch_rows(bool comp_in, unsigned g, hipStream_t st, const RowArgs &a) {
    if (comp_in)
        k_rows<CS, true, kWrite, kPbc><<<g, 256, 0, st>>>(a);
    else
        k_rows<CS, false, kWrite, kPbc><<<g, 256, 0, st>>>(a);
}

template <bool kWrite, bool kPbc>
void launch_rows_cs(int cs, bool comp_in, unsigned g, hipStream_t st, const RowArgs &a) {
    if (cs == 4)
        launch_rows<4, kWrite, kPbc>(comp_in, g, st, a);
    else if (cs == 16)
        launch_rows<16, kWrite, kPbc>(comp_in, g, st, a);
    else
        launch_rows<8, kWrite, kPbc>(comp_in, g, st, a);
}

template <bool kPbc>
void launch_pass_rows(int variant, unsigned g, hipStream_t st, const RowPassArgs &a) {
    switch (variant) {
        case 7: k_pass_rows<true, true, true, kPbc><<<g, 256, 0, st>>>(a); break;
        case 6: k_pass_rows<true, true, false, kPbc><<<g, 256, 0, st>>>(a); break;
        case 5: k_pass_rows<true, false, true, kPbc><<<g, 256, 0, st>>>(a); break;
        case 4: k_pass_rows<true, false, false, kPbc><<<g, 256, 0, st>>>(a); break;
        case 3: k_pass_rows<false, true, true, kPbc><<<g, 256, 0, st>>>(a); break;
        case 2: k_pass_rows<false, true, false, kPbc><<<g, 256, 0, st>>>(a); break;
        case 1: k_pass_rows<false, false, true, kPbc><<<g, 256, 0, st>>>(a); break;
        default: k_pass_rows<false, false, false, kPbc><<<g, 256, 0, st>>>(a); break;
    }
}

__global__ void k_rows_total(const uint32_t *total, uint32_t *status) { status[kStTotalLo] = *total; }

struct RowsWs {
    uint32_t *row_words, *row_off;
    void *scan_tmp;
};

size_t carve_rows(RowsWs &ws, void *base, int64_t n) {
    Carver cv{reinterpret_cast<char *>(base), 0};
    ws.row_words = cv.take<uint32_t>((size_t)n);
    ws.row_off = cv.take<uint32_t>((size_t)n + 1);
    ws.scan_tmp = cv.take<char>(scan_tmp_bytes(n));
    return cv.used;
}

}  // namespace
}  // namespace sfcnl

using namespace sfcnl;

extern "C" int build_rows_workspace(int64_t n, size_t *ws_bytes) {
    if (n < 0 || n >= (int64_t(1) << 31) || !ws_bytes) return SFCNL_E_ARG;
    RowsWs ws;
    *ws_bytes = align_up(carve_rows(ws, nullptr, n), 256) + 256;
    return SFCNL_OK;
}

extern "C" int build_rows(sfcnl_ctx ctx, int64_t n, int cluster_size, int list_compress, const uint32_t *d_sc_info,
                          const uint32_t *d_pool, const float *d_x, const float *d_y, const float *d_z,
                          const float *d_h, int compress, const float *h_period, void *d_ws, size_t ws_bytes,
                          uint32_t *d_row_info, uint32_t *d_row_pool, size_t pool_bytes, size_t *h_used_bytes) {
    if (!ctx) return SFCNL_E_ARG;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "build_rows: n out of range");
    if (cluster_size != 4 && cluster_size != 8 && cluster_size != 16)
        return set_err(ctx, SFCNL_E_ARG, "build_rows: cluster_size %d not supported", cluster_size);
    if ((list_compress != 0 && list_compress != 1) || (compress != 0 && compress != 1))
        return set_err(ctx, SFCNL_E_ARG, "build_rows: compress flags must be 0 or 1");
    if (!period_ok(h_period)) return set_err(ctx, SFCNL_E_ARG, "build_rows: period must be 3 finite values >= 0");
    if (!h_used_bytes) return set_err(ctx, SFCNL_E_ARG, "build_rows: null result pointer");
    *h_used_bytes = 0;
    if (n == 0) return SFCNL_OK;
    if (!d_sc_info || !d_pool || !d_x || !d_y || !d_z || !d_h || !d_ws || !d_row_info || (!d_row_pool && pool_bytes))
        return set_err(ctx, SFCNL_E_ARG, "build_rows: null pointer");
    RowsWs ws;
    const size_t need = carve_rows(ws, d_ws, n);
    if (need > ws_bytes) return set_err(ctx, SFCNL_E_ARG, "build_rows: workspace %zu < %zu bytes", ws_bytes, need);
    const Period per = make_period(h_period);
    RowArgs a{n, d_sc_info, d_pool, d_x, d_y, d_z, d_h, per, compress, ws.row_words, ws.row_off, d_row_info,
              d_row_pool, pool_bytes / 4, ctx->d_status};
    hipStream_t st = ctx->stream;
    const unsigned g = blocks_for(n, kWavesPerBlock);
    int rc = fill_u32(ctx, ctx->d_status + kStPoolOverflow, 1, 0u);
    if (rc) return rc;
    if (per.on())
        launch_rows_cs<false, true>(cluster_size, list_compress, g, st, a);
    else
        launch_rows_cs<false, false>(cluster_size, list_compress, g, st, a);
    SFCNL_LAUNCHED(ctx);
    rc = scan_u32(ctx, ws.row_words, ws.row_off, n, ws.row_off + n, ws.scan_tmp);
    if (rc) return rc;
    if (per.on())
        launch_rows_cs<true, true>(cluster_size, list_compress, g, st, a);
    else
        launch_rows_cs<true, false>(cluster_size, list_compress, g, st, a);
    SFCNL_LAUNCHED(ctx);
    k_rows_total<<<1, 1, 0, st>>>(ws.row_off + n, ctx->d_status);
    SFCNL_LAUNCHED(ctx);
    rc = read_status(ctx);
    if (rc) return rc;
    *h_used_bytes = (size_t)ctx->h_status[kStTotalLo] * 4;
    if (ctx->h_status[kStPoolOverflow])
        return set_err(ctx, SFCNL_E_CAPACITY, "build_rows: pool of %zu bytes < %zu needed", pool_bytes, *h_used_bytes);
    return SFCNL_OK;
}

extern "C" int rows_pass(sfcnl_ctx ctx, int64_t n, int compress, const uint32_t *d_row_info,
                         const uint32_t *d_row_pool, const float *d_x, const float *d_y, const float *d_z,
                         const float *d_h, const float *d_m, float *d_rho, int32_t *d_nnb, const float *h_period) {
    if (!ctx) return SFCNL_E_ARG;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "rows_pass: n out of range");
    if (compress != 0 && compress != 1) return set_err(ctx, SFCNL_E_ARG, "rows_pass: compress must be 0 or 1");
    if (!period_ok(h_period)) return set_err(ctx, SFCNL_E_ARG, "rows_pass: period must be 3 finite values >= 0");
    if (n == 0) return SFCNL_OK;
    if (!d_row_info || !d_row_pool || !d_x || !d_y || !d_z || !d_h || !d_rho)
        return set_err(ctx, SFCNL_E_ARG, "rows_pass: null pointer");
    RowPassArgs a{n, d_row_info, d_row_pool, d_x, d_y, d_z, d_h, d_m, make_period(h_period), d_rho, d_nnb};
    const int variant = (compress ? 4 : 0) | (d_m ? 2 : 0) | (d_nnb ? 1 : 0);
    const unsigned g = blocks_for(n, kWavesPerBlock);
    prof_mark(ctx, kStagePass, false);
    if (a.per.on())
        launch_pass_rows<true>(variant, g, ctx->stream, a);
    else
        launch_pass_rows<false>(variant, g, ctx->stream, a);
    SFCNL_LAUNCHED(ctx);
    prof_mark(ctx, kStagePass, true);
    return SFCNL_OK;
}
