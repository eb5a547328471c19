// Smoothing-length iteration: every particle's radius is driven to a target
// own-radius neighbour count by rebuilding the list (the paper rebuilds its
// list every step with per-particle radii, Sec. IV; the update rule is this
// library's, stated in sfcnl.h).
#include <vector>

#include "internal.h"

namespace sfcnl {
namespace {

constexpr float kLn8 = 2.0794415416798357f;

__global__ __launch_bounds__(256) void k_bracket_init(int64_t n, float2 *__restrict__ br) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) br[i] = make_float2(0.0f, INFINITY);
}

// Learned step before the first round: h *= exp(clamp(d, -ln 8, ln 8)) where
// d is finite (real particles only).
__global__ __launch_bounds__(256) void k_seed_apply(int64_t n, float *__restrict__ h, const float *__restrict__ d,
                                                    SegTable seg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (seg.on()) {
        const int sy = seg.sc_sys[i / kScSize];
        if ((uint32_t)i - seg.pbase[sy] >= seg.count[sy]) return;
    }
    const float v = d[i];
    if (__builtin_isfinite(v)) h[i] = h[i] * expf(fminf(fmaxf(v, -kLn8), kLn8));
}

// One round of the update rule; `proposal` (nullable) holds learned
// log(h_new / h) values that replace the cube-root step where they are finite
// and within a factor 8. Nothing changes when the round's list could not be
// built (input, capacity or tree flags set in the status block), so that a
// round launched without a host check can be repeated after the fix.
// Batched systems skip their padding and count moves per system (a wave's 64
// particles are one super-cluster, hence one system).
__global__ __launch_bounds__(256) void k_h_update(int64_t n, const int32_t *__restrict__ nnb, float *__restrict__ h,
                                                  float2 *__restrict__ br, int target, int tol,
                                                  const float *__restrict__ proposal, const uint32_t *status,
                                                  SegTable seg, uint32_t *sys_moved, uint32_t *sc_moved,
                                                  uint8_t *p_moved) {
    if (status[kStInputErr] | status[kStPoolOverflow] | status[kStScratch] | status[kStTree]) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool moved = false;
    int sy = 0;
    bool real = i < n;
    if (seg.on() && i < n) {
        sy = seg.sc_sys[i / kScSize];
        real = (uint32_t)i - seg.pbase[sy] < seg.count[sy];
    }
    if (real) {
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
    // per particle and per super-cluster (a wave's 64 particles are one
    // super-cluster) what moved: the next round recounts only those; the
    // total is a prefix sum over the super-clusters (no contended atomics)
    if (i < n) p_moved[i] = moved ? 1 : 0;
    const uint64_t m = sfc_ballot(moved);
    if (sfc_lane() == 0 && i < n) {
        sc_moved[i / kScSize] = (uint32_t)sfc_popc(m);
        if (sys_moved && m) sys_moved[sy] = 1u;  // same value from every wave
    }
}

// The moved total for the host's status read (the next round's list build
// clears the status block; the total itself stays in the scan output).
__global__ void k_publish_total(const uint32_t *total, uint32_t *status) { status[kStUnconverged] = *total; }

// Rounds after the first recount the moved particles one wavefront each
// (count_moved_impl) when they are at most this many; above it, building the
// lists of their super-clusters shares each walk among up to 64 particles.
// Measured on the 1/r sphere and the 64-system batch: the per-particle walk
// wins up to about a quarter of the particles.
uint32_t count_path_limit(int64_t n) { return (uint32_t)(n / 4 + 64); }



// Grid of the per-particle recount: up to 8192 wavefronts.
unsigned count_blocks(uint32_t total) {
    const uint32_t b = (total + 3u) / 4u;
    return b < 1u ? 1u : (b > 2048u ? 2048u : b);
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
    if (it_opts->recount < 0 || it_opts->recount > 2)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: recount must be 0, 1 or 2");
    if (n == 0) {
        S.unconverged = 0;
        return SFCNL_OK;
    }
    if (!d_keys || !d_x || !d_y || !d_z || !d_h || !d_bracket || !d_bbox || !d_rho || !d_nnb || !d_ws ||
        !d_sc_info || (!d_pool && pool_bytes))
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: null pointer");
    size_t need;
    if (build_nlist_workspace(n, nl_opts, &need) != SFCNL_OK)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: bad list options");
    if (ws_bytes < need) return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: workspace %zu < %zu bytes", ws_bytes, need);
    if (seed && (!seed->d_params || !seed->d_feat || !seed->d_delta || !(seed->box_edge > 0.0f) ||
                 (seed->mode != SFCNL_SEED_AFTER_FIRST && seed->mode != SFCNL_SEED_BEFORE_FIRST)))
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_h_iterate: incomplete seed");
    hipStream_t strm = ctx->stream;
    float2 *br = reinterpret_cast<float2 *>(d_bracket);
    if (!it_opts->resume) {
        k_bracket_init<<<blocks_for(n, 256), 256, 0, strm>>>(n, br);
        SFCNL_LAUNCHED(ctx);
        if (seed && seed->mode == SFCNL_SEED_BEFORE_FIRST) {
            int rc = features_impl(ctx, n, d_keys, d_x, d_y, d_z, d_h, nullptr, seed->box_edge, it_opts->target,
                                   seed->d_feat, SegTable{});
            if (rc) return rc;
            rc = sfcnl_mlp_infer(ctx, seed->d_params, n, seed->d_feat, seed->d_delta);
            if (rc) return rc;
            k_seed_apply<<<blocks_for(n, 256), 256, 0, strm>>>(n, d_h, seed->d_delta, SegTable{});
            SFCNL_LAUNCHED(ctx);
        }
    }
    // The first round counts every particle with the requested list form;
    // later rounds rebuild full lists only for super-clusters where a radius
    // moved (the counts of the others cannot change: n_i depends on h_i only),
    // (with a half list requested and the automatic recount, those rounds
    // rebuild every super-cluster's half list instead), and a converged run
    // ends with one list build in the requested form.
    sfcnl_nlist_opts it_nl = *nl_opts;
    it_nl.half = 0;
    const ActiveWs act = nlist_ws_active(d_ws, n, it_nl, 1);
    const int64_t nsc = (n + kScSize - 1) / kScSize;
    bool list_final = false;
    for (int it = 0; it < it_opts->max_iters; it++) {
        const bool first = it == 0;
        const bool per_particle = !first && (it_opts->recount == 2 ||
                                             (it_opts->recount == 0 && S.unconverged <= count_path_limit(n)));
        // every super-cluster in the requested form: the first round, and with
        // the automatic recount and a half list every round that builds lists.
        // The counting lists are full lists (each pair twice): on the 8M 1/r
        // sphere, where nearly every super-cluster holds a moved particle in
        // those rounds, they cost more than the half list and its symmetric
        // pass (27.5 against 31.4 ms to converge). Counts, and so rounds and
        // radii, are the same either way (n_i depends on h_i only).
        const bool full = first || (it_opts->recount == 0 && nl_opts->half && !per_particle);
        const sfcnl_nlist_opts &o = full ? *nl_opts : it_nl;
        int rc = SFCNL_OK;
        if (full) {
            rc = clusters_impl(ctx, n, d_x, d_y, d_z, d_h, o.cluster_size, d_bbox, SegTable{});
            if (rc) return rc;
        }
        if (per_particle) {
            // few moved: one wavefront per moved particle on the last octree
            rc = count_moved_impl(ctx, n, act, d_x, d_y, d_z, d_h, d_m, d_rho, d_nnb, SegTable{},
                                  make_period(o.period), nullptr, 0, count_blocks((uint32_t)S.unconverged));
            if (rc) return rc;
        } else {
            // full rounds: every super-cluster in the requested form; the
            // others: counting lists of the moved particles, same octree
            rc = nlist_build_impl(ctx, n, d_keys, d_x, d_y, d_z, d_h, d_bbox, o, d_ws, ws_bytes, d_sc_info, d_pool,
                                  pool_bytes, SegTable{}, true, &S.used_bytes, &S.max_nj, full ? nullptr : act.sc,
                                  full ? nullptr : act.p, !full);
            if (rc) return rc;
            rc = pass_impl(ctx, n, o.cluster_size, o.compress, o.half, d_sc_info, d_pool, d_x, d_y, d_z, d_h, d_m,
                           d_rho, d_nnb, SegTable{}, make_period(o.period), full ? nullptr : act.sc,
                           full ? nullptr : act.p);
            if (rc) return rc;
        }
        list_final = full;
        const float *proposal = nullptr;
        if (seed && seed->mode == SFCNL_SEED_AFTER_FIRST && first) {  // learned step from the first counts
            rc = sfcnl_hseed_features(ctx, n, d_keys, d_x, d_y, d_z, d_h, d_nnb, seed->box_edge, it_opts->target,
                                      seed->d_feat);
            if (rc) return rc;
            rc = sfcnl_mlp_infer(ctx, seed->d_params, n, seed->d_feat, seed->d_delta);
            if (rc) return rc;
            proposal = seed->d_delta;
        }
        k_h_update<<<blocks_for(n, 256), 256, 0, strm>>>(n, d_nnb, d_h, br, it_opts->target, it_opts->tol, proposal,
                                                        ctx->d_status, SegTable{}, nullptr, act.sc, act.p);
        SFCNL_LAUNCHED(ctx);
        rc = scan_u32(ctx, act.sc, act.scan, nsc, act.scan + nsc, act.scan_tmp);
        if (rc) return rc;
        k_publish_total<<<1, 1, 0, strm>>>(act.scan + nsc, ctx->d_status);
        SFCNL_LAUNCHED(ctx);
        SFCNL_HIP(ctx, hipMemcpyAsync(ctx->h_status + kStUnconverged, ctx->d_status + kStUnconverged,
                                      sizeof(uint32_t), hipMemcpyDeviceToHost, strm));
        SFCNL_HIP(ctx, hipStreamSynchronize(strm));
        S.iters = it + 1;
        S.unconverged = ctx->h_status[kStUnconverged];
        S.moved += S.unconverged;
        if (S.unconverged == 0) {
            if (!list_final) {  // the list of the final radii, every super-cluster, requested form
                rc = clusters_impl(ctx, n, d_x, d_y, d_z, d_h, nl_opts->cluster_size, d_bbox, SegTable{});
                if (rc) return rc;
                rc = nlist_build_impl(ctx, n, d_keys, d_x, d_y, d_z, d_h, d_bbox, *nl_opts, d_ws, ws_bytes,
                                      d_sc_info, d_pool, pool_bytes, SegTable{}, true, &S.used_bytes, &S.max_nj);
                if (rc) return rc;
            }
            return SFCNL_OK;
        }
    }
    return set_err(ctx, SFCNL_E_NOCONV, "sfcnl_h_iterate: %lld particles unconverged after %d rounds",
                   (long long)S.unconverged, it_opts->max_iters);
}

// ---------------------------------------------------------------------------
// Batched iteration: every round is one fixed sequence of launches over all
// systems (cluster boxes, octrees, traversal, encode, pass, update, status
// copy), captured once into a graph and replayed; the host only reads the
// status block between rounds.
// ---------------------------------------------------------------------------

namespace {

struct RoundArgs {
    sfcnl_batch b;
    const uint64_t *keys;
    const float *x, *y, *z, *m;
    float *h;
    float2 *br;
    const sfcnl_nlist_opts *nl;
    const sfcnl_hiter_opts *it;
    float *bbox;
    void *ws;
    size_t ws_bytes;
    uint32_t *sc_info, *pool;
    size_t pool_bytes;
    float *rho;
    int32_t *nnb;
};

// Enqueues one round on ctx->stream with list options `o`; `seed` adds the
// learned first step; `restricted` limits the list build and the pass to the
// super-clusters flagged in `act` (which receives the next round's flags);
// the round's status block and per-system moved flags are copied to host
// slot `slot`.
int enqueue_round(sfcnl_ctx ctx, const RoundArgs &r, const sfcnl_nlist_opts &o, const sfcnl_hseed *seed,
                  bool restricted, const ActiveWs &act, int slot) {
    const SegTable seg = seg_of(r.b);
    const int64_t n = r.b->n_pad;
    int rc = SFCNL_OK;
    if (!restricted) {
        rc = clusters_impl(ctx, n, r.x, r.y, r.z, r.h, o.cluster_size, r.bbox, seg);
        if (rc) return rc;
    }
    // restricted rounds hold both recounts; the moved total (left in the scan
    // output by the previous round) selects one on the device: the lists of
    // the moved particles' super-clusters, or one wavefront per moved particle
    const uint32_t *gate = restricted ? act.scan + n / kScSize : nullptr;
    // recount 1: lists only (the per-particle path runs for a zero total,
    // where it has nothing to do); 2: per particle only
    const uint32_t limit = r.it->recount == 1 ? 0u : (r.it->recount == 2 ? 0xFFFFFFFFu : count_path_limit(n));
    rc = nlist_build_impl(ctx, n, r.keys, r.x, r.y, r.z, r.h, r.bbox, o, r.ws, r.ws_bytes, r.sc_info, r.pool,
                          r.pool_bytes, seg, false, nullptr, nullptr, restricted ? act.sc : nullptr,
                          restricted ? act.p : nullptr, restricted, gate, limit);
    if (rc) return rc;
    rc = pass_impl(ctx, n, o.cluster_size, o.compress, o.half, r.sc_info, r.pool, r.x, r.y, r.z, r.h, r.m, r.rho,
                   r.nnb, seg, Period{}, restricted ? act.sc : nullptr, restricted ? act.p : nullptr, gate, limit);
    if (rc) return rc;
    if (restricted) {
        rc = count_moved_impl(ctx, n, act, r.x, r.y, r.z, r.h, r.m, r.rho, r.nnb, seg, Period{}, gate, limit,
                              count_blocks(r.it->recount == 2 ? 8192u : limit));
        if (rc) return rc;
    }
    const float *proposal = nullptr;
    if (seed) {
        rc = features_impl(ctx, n, r.keys, r.x, r.y, r.z, r.h, r.nnb, 1.0f, r.it->target, seed->d_feat, seg);
        if (rc) return rc;
        rc = sfcnl_mlp_infer(ctx, seed->d_params, n, seed->d_feat, seed->d_delta);
        if (rc) return rc;
        proposal = seed->d_delta;
    }
    rc = fill_u32(ctx, r.b->d_sys_moved, r.b->nsys, 0);
    if (rc) return rc;
    k_h_update<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, r.nnb, r.h, r.br, r.it->target, r.it->tol, proposal,
                                                           ctx->d_status, seg, r.b->d_sys_moved, act.sc, act.p);
    SFCNL_LAUNCHED(ctx);
    rc = scan_u32(ctx, act.sc, act.scan, n / kScSize, act.scan + n / kScSize, act.scan_tmp);
    if (rc) return rc;
    k_publish_total<<<1, 1, 0, ctx->stream>>>(act.scan + n / kScSize, ctx->d_status);
    SFCNL_LAUNCHED(ctx);
    SFCNL_HIP(ctx, hipMemcpyAsync(r.b->h_rstat + (size_t)slot * kStWords, ctx->d_status, kStWords * sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, ctx->stream));
    SFCNL_HIP(ctx, hipMemcpyAsync(r.b->h_sys_moved + (size_t)slot * r.b->nsys, r.b->d_sys_moved,
                                  r.b->nsys * sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
    return SFCNL_OK;
}

// Runs the batch's work on its own stream, ordered after the caller's stream
// and before the caller's later work; restores the context on every exit.
struct OnBatchStream {
    sfcnl_ctx ctx;
    sfcnl_batch b;
    hipStream_t user;
    int prof_slots;
    OnBatchStream(sfcnl_ctx c, sfcnl_batch bb) : ctx(c), b(bb), user(c->stream), prof_slots(c->prof_slots) {
        (void)hipEventRecord(b->ev_in, user);
        (void)hipStreamWaitEvent(b->stream, b->ev_in, 0);
        ctx->stream = b->stream;
    }
    ~OnBatchStream() {
        (void)hipEventRecord(b->ev_out, b->stream);
        (void)hipStreamWaitEvent(user, b->ev_out, 0);
        ctx->stream = user;
        ctx->prof_slots = prof_slots;
    }
};

struct GraphHolder {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    ~GraphHolder() {
        if (e) (void)hipGraphExecDestroy(e);
        if (g) (void)hipGraphDestroy(g);
    }
};

}  // namespace

extern "C" int sfcnl_batch_h_iterate(sfcnl_ctx ctx, sfcnl_batch b, const uint64_t *d_keys, const float *d_x,
                                     const float *d_y, const float *d_z, float *d_h, float *d_bracket,
                                     const float *d_m, const sfcnl_nlist_opts *nl_opts,
                                     const sfcnl_hiter_opts *it_opts, float *d_bbox, void *d_ws, size_t ws_bytes,
                                     uint32_t *d_sc_info, uint32_t *d_pool, size_t pool_bytes, float *d_rho,
                                     int32_t *d_nnb, const sfcnl_hseed *seed, int use_graph,
                                     sfcnl_hiter_stats *st_out, int32_t *h_sys_rounds) {
    if (!ctx) return SFCNL_E_ARG;
    if (!b || b->device != ctx->device) return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_h_iterate: bad batch");
    if (!it_opts || !nl_opts || !st_out) return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_h_iterate: null argument");
    sfcnl_hiter_stats &S = *st_out;
    S.iters = 0;
    S.unconverged = b->n_in;
    S.moved = 0;
    S.used_bytes = 0;
    S.max_nj = 0;
    if (h_sys_rounds)
        for (int s = 0; s < b->nsys; s++) h_sys_rounds[s] = 0;
    if (it_opts->target < 1 || it_opts->tol < 0 || it_opts->max_iters < 1)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_h_iterate: target >= 1, tol >= 0, max_iters >= 1 required");
    if (it_opts->recount < 0 || it_opts->recount > 2)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_h_iterate: recount must be 0, 1 or 2");
    size_t need;
    if (sfcnl_batch_nlist_workspace(b, nl_opts, &need))
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_h_iterate: bad list options");
    if (ws_bytes < need)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_h_iterate: workspace %zu < %zu bytes", ws_bytes, need);
    if (b->n_in == 0) {
        S.unconverged = 0;
        return SFCNL_OK;
    }
    if (!d_keys || !d_x || !d_y || !d_z || !d_h || !d_bracket || !d_bbox || !d_ws || !d_sc_info || !d_rho || !d_nnb ||
        (!d_pool && pool_bytes))
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_h_iterate: null pointer");
    if (seed && (!seed->d_params || !seed->d_feat || !seed->d_delta ||
                 (seed->mode != SFCNL_SEED_AFTER_FIRST && seed->mode != SFCNL_SEED_BEFORE_FIRST)))
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_batch_h_iterate: incomplete seed");

    RoundArgs r{b,     d_keys, d_x,    d_y,     d_z,       d_m,    d_h,  reinterpret_cast<float2 *>(d_bracket),
                nl_opts, it_opts, d_bbox, d_ws, ws_bytes, d_sc_info, d_pool, pool_bytes, d_rho, d_nnb};
    OnBatchStream on(ctx, b);
    hipStream_t st = ctx->stream;
    if (!it_opts->resume) {
        k_bracket_init<<<blocks_for(b->n_pad, 256), 256, 0, st>>>(b->n_pad, r.br);
        SFCNL_LAUNCHED(ctx);
        if (seed && seed->mode == SFCNL_SEED_BEFORE_FIRST) {
            const SegTable seg = seg_of(b);
            int rc = features_impl(ctx, b->n_pad, d_keys, d_x, d_y, d_z, d_h, nullptr, 1.0f, it_opts->target,
                                   seed->d_feat, seg);
            if (rc) return rc;
            rc = sfcnl_mlp_infer(ctx, seed->d_params, b->n_pad, seed->d_feat, seed->d_delta);
            if (rc) return rc;
            k_seed_apply<<<blocks_for(b->n_pad, 256), 256, 0, st>>>(b->n_pad, d_h, seed->d_delta, seg);
            SFCNL_LAUNCHED(ctx);
        }
    }
    // Round 0 counts every particle with the requested list form; later
    // rounds rebuild full lists only for super-clusters where a radius moved
    // (the same rounds, and so the same radii, as recounting everything); a
    // converged run ends with one list build in the requested form.
    sfcnl_nlist_opts it_nl = *nl_opts;
    it_nl.half = 0;
    const ActiveWs act = nlist_ws_active(d_ws, b->n_pad, it_nl, b->nsys);
    bool list_final = false;
    // restricted rounds replay a graph of kGraphRounds rounds (one of a single
    // round when fewer are left): rounds after convergence in a replay find
    // nothing flagged and change nothing, so the host reads the status
    // blocks of a replay in order and stops at the first converged one
    GraphHolder gh_many, gh_one;
    std::vector<char> active((size_t)b->nsys, 1);
    int it = 0;
    while (it < it_opts->max_iters) {
        int nr = 1;
        if (it == 0) {
            const sfcnl_hseed *sd = (seed && seed->mode == SFCNL_SEED_AFTER_FIRST) ? seed : nullptr;
            int rc = enqueue_round(ctx, r, *nl_opts, sd, false, act, 0);
            if (rc) return rc;
        } else if (use_graph) {
            nr = it + kGraphRounds <= it_opts->max_iters ? kGraphRounds : 1;
            GraphHolder &gh = nr > 1 ? gh_many : gh_one;
            if (!gh.e) {
                ctx->prof_slots = 0;  // no event records inside the graph
                SFCNL_HIP(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                int rc = SFCNL_OK;
                for (int k = 0; k < nr && rc == SFCNL_OK; k++) rc = enqueue_round(ctx, r, it_nl, nullptr, true, act, k);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(st, &g);
                gh.g = g;
                if (rc) return rc;
                if (e != hipSuccess) return set_err(ctx, SFCNL_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
                SFCNL_HIP(ctx, hipGraphInstantiate(&gh.e, gh.g, nullptr, nullptr, 0));
                ctx->prof_slots = on.prof_slots;
            }
            SFCNL_HIP(ctx, hipGraphLaunch(gh.e, st));
        } else {
            int rc = enqueue_round(ctx, r, it_nl, nullptr, true, act, 0);
            if (rc) return rc;
        }
        SFCNL_HIP(ctx, hipStreamSynchronize(st));
        for (int k = 0; k < nr; k++, it++) {
            list_final = it == 0;
            const uint32_t *hs = b->h_rstat + (size_t)k * kStWords;
            const uint32_t *hm = b->h_sys_moved + (size_t)k * b->nsys;
            S.used_bytes = (size_t)hs[kStTotalLo] * 4;
            S.max_nj = hs[kStMaxNj];
            if (hs[kStInputErr]) {
                const uint32_t e = hs[kStInputErr];
                int rc = fill_u32(ctx, ctx->d_status + kStInputErr, 1, 0);
                if (rc) return rc;
                return set_err(ctx, SFCNL_E_INPUT, "input error flags 0x%x (1: non-finite position, 2: bad radius, 8: positions span a "
                                       "period or a radius reaches half of it)", e);
            }
            if (hs[kStTree]) return set_err(ctx, SFCNL_E_HIP, "internal error: octree invariant broken (0x%x)", hs[kStTree]);
            if (hs[kStScratch]) {
                S.max_nj = staging_fit(hs, (uint32_t)(b->n_pad / kScSize));
                return set_err(ctx, SFCNL_E_CAPACITY, "staging list of max_j_per_sc %d too small: %lld holds the lists",
                               nl_opts->max_j_per_sc, (long long)S.max_nj);
            }
            if (hs[kStPoolOverflow])
                return set_err(ctx, SFCNL_E_CAPACITY, "pool of %zu bytes < %zu needed", pool_bytes, S.used_bytes);
            S.iters = it + 1;
            S.unconverged = hs[kStUnconverged];
            S.moved += S.unconverged;
            // a system takes part in a round while its previous round moved a
            // particle (every system takes part in the first)
            if (h_sys_rounds)
                for (int s = 0; s < b->nsys; s++)
                    if (it == 0 || active[s]) h_sys_rounds[s] = it + 1;
            for (int s = 0; s < b->nsys; s++) active[s] = hm[s] != 0;
            if (S.unconverged == 0) {
                if (!list_final) {  // the list of the final radii, every super-cluster, requested form
                    const SegTable seg = seg_of(b);
                    int rc = clusters_impl(ctx, b->n_pad, d_x, d_y, d_z, d_h, nl_opts->cluster_size, d_bbox, seg);
                    if (rc) return rc;
                    rc = nlist_build_impl(ctx, b->n_pad, d_keys, d_x, d_y, d_z, d_h, d_bbox, *nl_opts, d_ws, ws_bytes,
                                          d_sc_info, d_pool, pool_bytes, seg, true, &S.used_bytes, &S.max_nj);
                    if (rc) return rc;
                }
                return SFCNL_OK;
            }
        }
    }
    return set_err(ctx, SFCNL_E_NOCONV, "sfcnl_batch_h_iterate: %lld particles unconverged after %d rounds",
                   (long long)S.unconverged, it_opts->max_iters);
}
