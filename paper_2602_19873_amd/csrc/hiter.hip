// Smoothing-length iteration: every particle's radius is driven to a target
// own-radius neighbour count by rebuilding the list (the paper rebuilds its
// list every step with per-particle radii, Sec. IV; the update rule is this
// library's, stated in sfcnl.h).
#include "internal.h"

namespace sfcnl {
namespace {

constexpr float kLn8 = 2.0794415416798357f;

__global__ __launch_bounds__(256) void k_bracket_init(int64_t n, float2 *__restrict__ br) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) br[i] = make_float2(0.0f, INFINITY);
}

// One round of the update rule; `proposal` (nullable) holds learned
// log(h_new / h) values that replace the cube-root step where they are finite
// and within a factor 8.
__global__ __launch_bounds__(256) void k_h_update(int64_t n, const int32_t *__restrict__ nnb, float *__restrict__ h,
                                                  float2 *__restrict__ br, int target, int tol,
                                                  const float *__restrict__ proposal, uint32_t *unconverged) {
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
            const float d = proposal ? proposal[i] : NAN;
            if (d >= -kLn8 && d <= kLn8) {  // false for NaN
                hn = hc * expf(d);
            } else if (c == 0) {
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
                               float *d_rho, int32_t *d_nnb, const sfcnl_hseed *seed, sfcnl_hiter_stats *st_out) {
    if (!ctx) return SFCNL_E_ARG;
    if (!it_opts || !nl_opts || !st_out) return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: null argument");
    sfcnl_hiter_stats &S = *st_out;
    S.iters = 0;
    S.unconverged = n;
    S.moved = 0;
    S.used_bytes = 0;
    S.max_nj = 0;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: n out of range");
    if (it_opts->target < 1 || it_opts->tol < 0 || it_opts->max_iters < 1)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: target >= 1, tol >= 0, max_iters >= 1 required");
    if (n == 0) {
        S.unconverged = 0;
        return SFCNL_OK;
    }
    if (!d_keys || !d_x || !d_y || !d_z || !d_h || !d_bracket || !d_bbox || !d_rho || !d_nnb)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: null pointer");
    if (seed && (!seed->d_params || !seed->d_feat || !seed->d_delta || !(seed->box_edge > 0.0f)))
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: incomplete seed");
    hipStream_t strm = ctx->stream;
    float2 *br = reinterpret_cast<float2 *>(d_bracket);
    if (!it_opts->resume) {
        k_bracket_init<<<blocks_for(n, 256), 256, 0, strm>>>(n, br);
        SFCNL_LAUNCHED(ctx);
    }
    for (int it = 0; it < it_opts->max_iters; it++) {
        int rc = build_clusters(ctx, n, d_x, d_y, d_z, d_h, nl_opts->cluster_size, d_bbox);
        if (rc) return rc;
        rc = build_nlist(ctx, n, d_keys, d_x, d_y, d_z, d_h, d_bbox, nl_opts, d_ws, ws_bytes, d_sc_info, d_pool,
                         pool_bytes, &S.used_bytes, &S.max_nj);
        if (rc) return rc;
        rc = nlist_pass(ctx, n, nl_opts->cluster_size, nl_opts->compress, d_sc_info, d_pool, d_x, d_y, d_z, d_h, d_m,
                        d_rho, d_nnb);
        if (rc) return rc;
        const float *proposal = nullptr;
        if (seed && it == 0) {  // learned first step from the first round's counts
            rc = sfcnl_hseed_features(ctx, n, d_keys, d_h, d_nnb, d_bbox, seed->box_edge, it_opts->target,
                                      seed->d_feat);
            if (rc) return rc;
            rc = sfcnl_mlp_infer(ctx, seed->d_params, n, seed->d_feat, seed->d_delta);
            if (rc) return rc;
            proposal = seed->d_delta;
        }
        rc = fill_u32(ctx, ctx->d_status + kStUnconverged, 1, 0);
        if (rc) return rc;
        k_h_update<<<blocks_for(n, 256), 256, 0, strm>>>(n, d_nnb, d_h, br, it_opts->target, it_opts->tol, proposal,
                                                        ctx->d_status + kStUnconverged);
        SFCNL_LAUNCHED(ctx);
        SFCNL_HIP(ctx, hipMemcpyAsync(ctx->h_status + kStUnconverged, ctx->d_status + kStUnconverged,
                                      sizeof(uint32_t), hipMemcpyDeviceToHost, strm));
        SFCNL_HIP(ctx, hipStreamSynchronize(strm));
        S.iters = it + 1;
        S.unconverged = ctx->h_status[kStUnconverged];
        S.moved += S.unconverged;
        if (S.unconverged == 0) return SFCNL_OK;
    }
    return set_err(ctx, SFCNL_E_NOCONV, "sfcnl_h_iterate: %lld particles unconverged after %d rounds",
                   (long long)S.unconverged, it_opts->max_iters);
}
