// Batches of independent particle systems: one padded layout, one set of
// launches over every system's super-clusters, per-system octrees and
// per-system list indices (so that each system's list is exactly the list it
// would get on its own).
#include <stdlib.h>
#include <string.h>

#include "internal.h"

using namespace sfcnl;

namespace {

void free_batch(sfcnl_batch b) {
    if (!b) return;
    (void)hipFree(b->d_sc_sys);
    (void)hipFree(b->d_pbase);
    (void)hipFree(b->d_count);
    (void)hipFree(b->d_in_off);
    (void)hipFree(b->d_edge);
    (void)hipFree(b->d_lo);
    (void)hipFree(b->d_scale);
    (void)hipFree(b->d_roots);
    (void)hipFree(b->d_sys_moved);
    if (b->h_sys_moved) (void)hipHostFree(b->h_sys_moved);
    if (b->h_rstat) (void)hipHostFree(b->h_rstat);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    free(b->h_in_off);
    free(b->h_pbase);
    free(b->h_box);
    free(b);
}

int check_batch(sfcnl_ctx ctx, sfcnl_batch b, const char *fn) {
    if (!b) return set_err(ctx, SFCNL_E_ARG, "%s: null batch", fn);
    if (b->device != ctx->device) return set_err(ctx, SFCNL_E_ARG, "%s: batch on another device", fn);
    return SFCNL_OK;
}

}  // namespace

extern "C" int sfcnl_batch_create(sfcnl_ctx ctx, int nsys, const int64_t *h_counts, const float *h_boxes,
                                  sfcnl_batch *out) {
    if (!ctx) return SFCNL_E_ARG;
    if (!out) return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_create: null output");
    *out = nullptr;
    if (nsys < 1 || nsys > SFCNL_BATCH_MAX_SYSTEMS || !h_counts || !h_boxes)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_create: need 1..%d systems with counts and boxes",
                       SFCNL_BATCH_MAX_SYSTEMS);
    int64_t n_in = 0, n_pad = 0;
    for (int s = 0; s < nsys; s++) {
        if (h_counts[s] < 0) return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_create: system %d has a negative count", s);
        for (int a = 0; a < 3; a++) {
            const float lo = h_boxes[6 * s + 2 * a], hi = h_boxes[6 * s + 2 * a + 1];
            if (!(hi > lo) || !__builtin_isfinite(lo) || !__builtin_isfinite(hi))
                return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_create: system %d box axis %d empty or not finite", s, a);
        }
        n_in += h_counts[s];
        n_pad += (h_counts[s] + kScSize - 1) / kScSize * kScSize;
        if (n_pad >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_create: batch too large");
    }
    sfcnl_batch b = static_cast<sfcnl_batch>(calloc(1, sizeof(sfcnl_batch_s)));
    if (!b) return set_err(ctx, SFCNL_E_HIP, "sfcnl_batch_create: out of host memory");
    b->device = ctx->device;
    b->nsys = nsys;
    b->n_in = n_in;
    b->n_pad = n_pad;
    b->h_in_off = static_cast<int64_t *>(malloc(sizeof(int64_t) * (nsys + 1)));
    b->h_pbase = static_cast<int64_t *>(malloc(sizeof(int64_t) * (nsys + 1)));
    b->h_box = static_cast<float *>(malloc(sizeof(float) * 6 * nsys));
    const int64_t nsc = n_pad / kScSize;
    uint16_t *sc_sys = static_cast<uint16_t *>(malloc(sizeof(uint16_t) * (nsc > 0 ? nsc : 1)));
    uint32_t *tab = static_cast<uint32_t *>(malloc(sizeof(uint32_t) * (3 * nsys + 2)));
    float *ftab = static_cast<float *>(malloc(sizeof(float) * 7 * nsys));
    int rc = SFCNL_OK;
    if (!b->h_in_off || !b->h_pbase || !b->h_box || !sc_sys || !tab || !ftab) {
        rc = set_err(ctx, SFCNL_E_HIP, "sfcnl_batch_create: out of host memory");
    } else {
        memcpy(b->h_box, h_boxes, sizeof(float) * 6 * nsys);
        uint32_t *pbase = tab, *count = tab + nsys + 1, *in_off = tab + 2 * nsys + 1;
        float *edge = ftab, *lo = ftab + nsys, *scale = ftab + 4 * nsys;
        int64_t ib = 0, pb = 0;
        for (int s = 0; s < nsys; s++) {
            b->h_in_off[s] = ib;
            b->h_pbase[s] = pb;
            in_off[s] = (uint32_t)ib;
            pbase[s] = (uint32_t)pb;
            count[s] = (uint32_t)h_counts[s];
            const int64_t padded = (h_counts[s] + kScSize - 1) / kScSize * kScSize;
            for (int64_t c = pb / kScSize; c < (pb + padded) / kScSize; c++) sc_sys[c] = (uint16_t)s;
            ib += h_counts[s];
            pb += padded;
            float e = 0.0f;
            for (int a = 0; a < 3; a++) {
                const float l = h_boxes[6 * s + 2 * a], h = h_boxes[6 * s + 2 * a + 1];
                lo[3 * s + a] = l;
                // the single-system key scale: 2^21 over the side, rounded once
                scale[3 * s + a] = (float)(2097152.0 / ((double)h - (double)l));
                e = fmaxf(e, h - l);
            }
            edge[s] = e;
        }
        b->h_in_off[nsys] = ib;
        b->h_pbase[nsys] = pb;
        in_off[nsys] = (uint32_t)ib;
        pbase[nsys] = (uint32_t)pb;
#define SFCNL_ALLOC(ptr, cnt)                                                                                    \
    if (rc == SFCNL_OK && hipMalloc((void **)&(ptr), sizeof(*(ptr)) * ((cnt) > 0 ? (size_t)(cnt) : 1)) != hipSuccess) \
        rc = set_err(ctx, SFCNL_E_HIP, "sfcnl_batch_create: device allocation failed");
        SFCNL_ALLOC(b->d_sc_sys, nsc);
        SFCNL_ALLOC(b->d_pbase, nsys + 1);
        SFCNL_ALLOC(b->d_count, nsys);
        SFCNL_ALLOC(b->d_in_off, nsys + 1);
        SFCNL_ALLOC(b->d_edge, nsys);
        SFCNL_ALLOC(b->d_lo, 3 * nsys);
        SFCNL_ALLOC(b->d_scale, 3 * nsys);
        SFCNL_ALLOC(b->d_roots, nsys);
        SFCNL_ALLOC(b->d_sys_moved, nsys);
#undef SFCNL_ALLOC
        if (rc == SFCNL_OK &&
            (hipHostMalloc((void **)&b->h_sys_moved, sizeof(uint32_t) * nsys * kGraphRounds) != hipSuccess ||
             hipHostMalloc((void **)&b->h_rstat, sizeof(uint32_t) * kStWords * kGraphRounds) != hipSuccess))
            rc = set_err(ctx, SFCNL_E_HIP, "sfcnl_batch_create: pinned allocation failed");
        if (rc == SFCNL_OK && (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
                               hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
                               hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess))
            rc = set_err(ctx, SFCNL_E_HIP, "sfcnl_batch_create: stream or event creation failed");
        const hipMemcpyKind h2d = hipMemcpyHostToDevice;
        if (rc == SFCNL_OK &&
            (hipMemcpy(b->d_sc_sys, sc_sys, sizeof(uint16_t) * nsc, h2d) != hipSuccess ||
             hipMemcpy(b->d_pbase, pbase, sizeof(uint32_t) * (nsys + 1), h2d) != hipSuccess ||
             hipMemcpy(b->d_count, count, sizeof(uint32_t) * nsys, h2d) != hipSuccess ||
             hipMemcpy(b->d_in_off, in_off, sizeof(uint32_t) * (nsys + 1), h2d) != hipSuccess ||
             hipMemcpy(b->d_edge, edge, sizeof(float) * nsys, h2d) != hipSuccess ||
             hipMemcpy(b->d_lo, lo, sizeof(float) * 3 * nsys, h2d) != hipSuccess ||
             hipMemcpy(b->d_scale, scale, sizeof(float) * 3 * nsys, h2d) != hipSuccess))
            rc = set_err(ctx, SFCNL_E_HIP, "sfcnl_batch_create: table upload failed");
    }
    free(sc_sys);
    free(tab);
    free(ftab);
    if (rc != SFCNL_OK) {
        free_batch(b);
        return rc;
    }
    *out = b;
    return SFCNL_OK;
}

extern "C" void sfcnl_batch_destroy(sfcnl_batch b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    free_batch(b);
}

extern "C" int sfcnl_batch_layout(sfcnl_batch b, int64_t *n_in, int64_t *n_padded, int64_t *h_in_off,
                                  int64_t *h_pbase) {
    if (!b) return SFCNL_E_ARG;
    if (n_in) *n_in = b->n_in;
    if (n_padded) *n_padded = b->n_pad;
    if (h_in_off) memcpy(h_in_off, b->h_in_off, sizeof(int64_t) * (b->nsys + 1));
    if (h_pbase) memcpy(h_pbase, b->h_pbase, sizeof(int64_t) * (b->nsys + 1));
    return SFCNL_OK;
}

extern "C" int sfcnl_batch_nlist_workspace(sfcnl_batch b, const sfcnl_nlist_opts *opts, size_t *ws_bytes) {
    if (!b || !opts || !ws_bytes) return SFCNL_E_ARG;
    size_t single;
    int rc = build_nlist_workspace(b->n_pad, opts, &single);  // validates the options
    if (rc) return rc;
    *ws_bytes = nlist_ws_bytes(b->n_pad, *opts, b->nsys);
    return SFCNL_OK;
}

extern "C" int sfcnl_batch_build_clusters(sfcnl_ctx ctx, sfcnl_batch b, const float *d_x, const float *d_y,
                                          const float *d_z, const float *d_h, int cluster_size, float *d_bbox_out) {
    if (!ctx) return SFCNL_E_ARG;
    int rc = check_batch(ctx, b, "sfcnl_batch_build_clusters");
    if (rc) return rc;
    if (cluster_size != 4 && cluster_size != 8 && cluster_size != 16)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_build_clusters: cluster_size %d not supported", cluster_size);
    if (b->n_pad == 0) return SFCNL_OK;
    if (!d_x || !d_y || !d_z || !d_h || !d_bbox_out)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_build_clusters: null pointer");
    return clusters_impl(ctx, b->n_pad, d_x, d_y, d_z, d_h, cluster_size, d_bbox_out, seg_of(b));
}

extern "C" int sfcnl_batch_build_nlist(sfcnl_ctx ctx, sfcnl_batch b, const uint64_t *d_keys, const float *d_x,
                                       const float *d_y, const float *d_z, const float *d_h, const float *d_bbox,
                                       const sfcnl_nlist_opts *opts, void *d_ws, size_t ws_bytes,
                                       uint32_t *d_sc_info, uint32_t *d_pool, size_t pool_bytes, size_t *h_used_bytes,
                                       int64_t *h_max_nj) {
    if (!ctx) return SFCNL_E_ARG;
    int rc = check_batch(ctx, b, "sfcnl_batch_build_nlist");
    if (rc) return rc;
    size_t need;
    if (!opts || sfcnl_batch_nlist_workspace(b, opts, &need))
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_build_nlist: bad options");
    if (!h_used_bytes || !h_max_nj) return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_build_nlist: null result pointer");
    *h_used_bytes = 0;
    *h_max_nj = 0;
    if (b->n_pad == 0) return SFCNL_OK;
    if (!d_keys || !d_x || !d_y || !d_z || !d_h || !d_bbox || !d_ws || !d_sc_info || (!d_pool && pool_bytes))
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_build_nlist: null pointer");
    return nlist_build_impl(ctx, b->n_pad, d_keys, d_x, d_y, d_z, d_h, d_bbox, *opts, d_ws, ws_bytes, d_sc_info,
                            d_pool, pool_bytes, seg_of(b), true, h_used_bytes, h_max_nj);
}

extern "C" int sfcnl_batch_pass(sfcnl_ctx ctx, sfcnl_batch b, int cluster_size, int compress, int half,
                                const uint32_t *d_sc_info, const uint32_t *d_pool, const float *d_x, const float *d_y,
                                const float *d_z, const float *d_h, const float *d_m, float *d_rho, int32_t *d_nnb) {
    if (!ctx) return SFCNL_E_ARG;
    int rc = check_batch(ctx, b, "sfcnl_batch_pass");
    if (rc) return rc;
    if (cluster_size != 4 && cluster_size != 8 && cluster_size != 16)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_pass: cluster_size %d not supported", cluster_size);
    if (compress != 0 && compress != 1) return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_pass: compress must be 0 or 1");
    if (half != 0 && half != 1) return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_pass: half must be 0 or 1");
    if (b->n_pad == 0) return SFCNL_OK;
    if (!d_sc_info || !d_pool || !d_x || !d_y || !d_z || !d_h || !d_rho)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_pass: null pointer");
    return pass_impl(ctx, b->n_pad, cluster_size, compress, half, d_sc_info, d_pool, d_x, d_y, d_z, d_h, d_m, d_rho, d_nnb,
                     seg_of(b), Period{});
}
