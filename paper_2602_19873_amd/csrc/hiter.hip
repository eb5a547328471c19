// Smoothing-length iteration: every particle's radius is driven to a target
// own-radius neighbour count by rebuilding the list (the paper rebuilds its
// list every step with per-particle radii, Sec. IV; the update rule is this
// library's, stated in sfcnl.h).
#include "internal.h"

namespace sfcnl {
namespace {

__global__ __launch_bounds__(256) void k_bracket_init(int64_t n, float2 *__restrict__ br) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) br[i] = make_float2(0.0f, INFINITY);
}

__global__ __launch_bounds__(256) void k_h_update(int64_t n, const int32_t *__restrict__ nnb, float *__restrict__ h,
                                                  float2 *__restrict__ br, int target, int tol,
                                                  uint32_t *unconverged) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool moved = false;
    if (i < n) {
        const int c = nnb[i];
        const int dev = c - target;
        if (dev > tol || dev < -tol) {
            moved = true;
            const float hc = h[i];
            float2 b = br[i];
            if (dev < 0)
                b.x = fmaxf(b.x, hc);  // too few neighbours: h is a lower bound
            else
                b.y = fminf(b.y, hc);  // too many: an upper bound
            float hn;
            if (c == 0) {
                hn = 2.0f * hc;
            } else {
                hn = hc * cbrtf((float)target / (float)c);
                hn = fminf(fmaxf(hn, 0.5f * hc), 2.0f * hc);
            }
            if (!(hn > b.x && hn < b.y)) {
                if (b.y == INFINITY)
                    hn = 2.0f * b.x;
                else if (b.x == 0.0f)
                    hn = 0.5f * b.y;
                else
                    hn = 0.5f * (b.x + b.y);
            }
            h[i] = hn;
            br[i] = b;
        }
    }
    const uint64_t m = sfc_ballot(moved);
    if (sfc_lane() == 0 && m) atomicAdd(unconverged, (uint32_t)sfc_popc(m));
}

}  // namespace
}  // namespace sfcnl

using namespace sfcnl;

extern "C" int sfcnl_h_iterate(sfcnl_ctx ctx, int64_t n, const uint64_t *d_keys, const float *d_x, const float *d_y,
                               const float *d_z, float *d_h, float *d_bracket, const float *d_m,
                               const sfcnl_nlist_opts *nl_opts, const sfcnl_hiter_opts *it_opts, float *d_bbox,
                               void *d_ws, size_t ws_bytes, uint32_t *d_sc_info, uint32_t *d_pool, size_t pool_bytes,
                               float *d_rho, int32_t *d_nnb, int *h_iters, int64_t *h_unconverged,
                               size_t *h_used_bytes, int64_t *h_max_nj) {
    if (!ctx) return SFCNL_E_ARG;
    if (!it_opts || !nl_opts || !h_iters || !h_unconverged || !h_used_bytes || !h_max_nj)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: null argument");
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: n out of range");
    if (it_opts->target < 1 || it_opts->tol < 0 || it_opts->max_iters < 1)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: target >= 1, tol >= 0, max_iters >= 1 required");
    *h_iters = 0;
    *h_unconverged = n;
    *h_used_bytes = 0;
    *h_max_nj = 0;
    if (n == 0) {
        *h_unconverged = 0;
        return SFCNL_OK;
    }
    if (!d_keys || !d_x || !d_y || !d_z || !d_h || !d_bracket || !d_bbox || !d_rho || !d_nnb)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: null pointer");
    hipStream_t st = ctx->stream;
    float2 *br = reinterpret_cast<float2 *>(d_bracket);
    if (!it_opts->resume) {
        k_bracket_init<<<blocks_for(n, 256), 256, 0, st>>>(n, br);
        SFCNL_LAUNCHED(ctx);
    }
    for (int it = 0; it < it_opts->max_iters; it++) {
        int rc = build_clusters(ctx, n, d_x, d_y, d_z, d_h, nl_opts->cluster_size, d_bbox);
        if (rc) return rc;
        rc = build_nlist(ctx, n, d_keys, d_x, d_y, d_z, d_h, d_bbox, nl_opts, d_ws, ws_bytes, d_sc_info, d_pool,
                         pool_bytes, h_used_bytes, h_max_nj);
        if (rc) return rc;
        rc = nlist_pass(ctx, n, nl_opts->cluster_size, nl_opts->compress, d_sc_info, d_pool, d_x, d_y, d_z, d_h, d_m,
                        d_rho, d_nnb);
        if (rc) return rc;
        rc = fill_u32(ctx, ctx->d_status + kStUnconverged, 1, 0);
        if (rc) return rc;
        k_h_update<<<blocks_for(n, 256), 256, 0, st>>>(n, d_nnb, d_h, br, it_opts->target, it_opts->tol,
                                                        ctx->d_status + kStUnconverged);
        SFCNL_LAUNCHED(ctx);
        SFCNL_HIP(ctx, hipMemcpyAsync(ctx->h_status + kStUnconverged, ctx->d_status + kStUnconverged,
                                      sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        SFCNL_HIP(ctx, hipStreamSynchronize(st));
        *h_iters = it + 1;
        *h_unconverged = ctx->h_status[kStUnconverged];
        if (*h_unconverged == 0) return SFCNL_OK;
    }
    return set_err(ctx, SFCNL_E_NOCONV, "sfcnl_h_iterate: %lld particles unconverged after %d rounds",
                   (long long)*h_unconverged, it_opts->max_iters);
}
