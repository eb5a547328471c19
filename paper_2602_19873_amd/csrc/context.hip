// Context, error reporting and status read-back of the sfcnl library.
#include <stdlib.h>
#include <string.h>

#include <cmath>

#include "internal.h"

namespace sfcnl {

int set_err(sfcnl_ctx ctx, int code, const char *fmt, ...) {
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof ctx->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

bool period_ok(const float *period) {
    if (!period) return true;
    for (int a = 0; a < 3; a++)
        if (!(period[a] >= 0.0f) || !std::isfinite(period[a])) return false;
    return true;
}

Period make_period(const float *period) {
    Period p;
    if (!period) return p;
    for (int a = 0; a < 3; a++) {
        if (period[a] > 0.0f) {
            p.L[a] = period[a];
            p.hL[a] = 0.5f * period[a];
            if (p.hL[a] < p.hmin) p.hmin = p.hL[a];
        }
    }
    return p;
}

}  // namespace sfcnl

using namespace sfcnl;

extern "C" const char *sfcnl_version(void) { return "sfcnl 0.1 gfx950"; }

extern "C" int sfcnl_create(sfcnl_ctx *out, int device, void *stream) {
    if (!out) return SFCNL_E_ARG;
    *out = nullptr;
    sfcnl_ctx c = (sfcnl_ctx)calloc(1, sizeof(sfcnl_ctx_s));
    if (!c) return SFCNL_E_ARG;
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->pass_waves = 1;
    c->prof_mask = (1u << SFCNL_NSTAGE) - 1u;
    if (hipSetDevice(device) != hipSuccess) {
        free(c);
        return SFCNL_E_HIP;
    }
    if (sort_scratch_setup(device, &c->d_sort_scratch) != SFCNL_OK) {
        free(c);
        return SFCNL_E_HIP;
    }
    if (hipMalloc((void **)&c->d_status, kStatusAlloc * sizeof(uint32_t)) != hipSuccess) {
        free(c);
        return SFCNL_E_HIP;
    }
    if (hipHostMalloc((void **)&c->h_status, kStWords * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(c->d_status);
        free(c);
        return SFCNL_E_HIP;
    }
    memset(c->h_status, 0, kStWords * sizeof(uint32_t));
    // coherent: the device's stores reach the host while later work still runs
    if (hipHostMalloc((void **)&c->h_pend, kStWords * sizeof(uint64_t), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess) {
        (void)hipHostFree(c->h_status);
        (void)hipFree(c->d_status);
        free(c);
        return SFCNL_E_HIP;
    }
    memset(c->h_pend, 0, kStWords * sizeof(uint64_t));
    if (hipHostGetDevicePointer((void **)&c->d_pend, c->h_pend, 0) != hipSuccess) {
        (void)hipHostFree(c->h_pend);
        (void)hipHostFree(c->h_status);
        (void)hipFree(c->d_status);
        free(c);
        return SFCNL_E_HIP;
    }
    if (fill_u32(c, c->d_status, kStatusAlloc, 0) != SFCNL_OK || hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipHostFree(c->h_pend);
        (void)hipHostFree(c->h_status);
        (void)hipFree(c->d_status);
        free(c);
        return SFCNL_E_HIP;
    }
    *out = c;
    return SFCNL_OK;
}

static void prof_release(sfcnl_ctx ctx) {
    for (int s = 0; s < SFCNL_NSTAGE; s++) {
        if (ctx->prof_ev[s]) {
            for (int k = 0; k < 2 * ctx->prof_slots; k++) (void)hipEventDestroy(ctx->prof_ev[s][k]);
            free(ctx->prof_ev[s]);
            ctx->prof_ev[s] = nullptr;
        }
        ctx->prof_used[s] = 0;
    }
    ctx->prof_slots = 0;
}

extern "C" int sfcnl_profile_begin(sfcnl_ctx ctx, int slots) {
    if (!ctx || slots < 1) return SFCNL_E_ARG;
    prof_release(ctx);
    for (int s = 0; s < SFCNL_NSTAGE; s++) {
        ctx->prof_ev[s] = (hipEvent_t *)calloc(2 * (size_t)slots, sizeof(hipEvent_t));
        if (!ctx->prof_ev[s]) return set_err(ctx, SFCNL_E_ARG, "profile: out of host memory");
        for (int k = 0; k < 2 * slots; k++) SFCNL_HIP(ctx, hipEventCreate(&ctx->prof_ev[s][k]));
    }
    ctx->prof_slots = slots;
    return SFCNL_OK;
}

extern "C" int sfcnl_profile_end(sfcnl_ctx ctx, double *h_ms, int64_t *h_calls) {
    if (!ctx || !h_ms || !h_calls) return SFCNL_E_ARG;
    SFCNL_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int s = 0; s < SFCNL_NSTAGE; s++) {
        double tot = 0.0;
        for (int k = 0; k < ctx->prof_used[s]; k++) {
            float ms = 0.0f;
            SFCNL_HIP(ctx, hipEventElapsedTime(&ms, ctx->prof_ev[s][2 * k], ctx->prof_ev[s][2 * k + 1]));
            tot += ms;
        }
        h_ms[s] = tot;
        h_calls[s] = ctx->prof_slots ? ctx->prof_used[s] : 0;
    }
    prof_release(ctx);
    return SFCNL_OK;
}

extern "C" int sfcnl_profile_stages(sfcnl_ctx ctx, uint32_t stage_mask) {
    if (!ctx) return SFCNL_E_ARG;
    if (stage_mask >> SFCNL_NSTAGE) return set_err(ctx, SFCNL_E_ARG, "profile: stage mask 0x%x has bits past the stages", stage_mask);
    ctx->prof_mask = stage_mask;
    return SFCNL_OK;
}

extern "C" void sfcnl_destroy(sfcnl_ctx ctx) {
    if (!ctx) return;
    prof_release(ctx);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipHostFree(ctx->h_pend);
    (void)hipHostFree(ctx->h_status);
    (void)hipFree(ctx->d_status);
    free(ctx);
}

extern "C" int sfcnl_set_stream(sfcnl_ctx ctx, void *stream) {
    if (!ctx) return SFCNL_E_ARG;
    ctx->stream = (hipStream_t)stream;
    return SFCNL_OK;
}

extern "C" int sfcnl_set_pass_waves(sfcnl_ctx ctx, int waves) {
    if (!ctx) return SFCNL_E_ARG;
    if (waves != 1 && waves != 2 && waves != 4) return set_err(ctx, SFCNL_E_ARG, "pass waves must be 1, 2 or 4");
    ctx->pass_waves = waves;
    return SFCNL_OK;
}

extern "C" const char *sfcnl_last_error(sfcnl_ctx ctx) { return ctx ? ctx->err : "null context"; }

extern "C" int sfcnl_sync(sfcnl_ctx ctx) {
    if (!ctx) return SFCNL_E_ARG;
    SFCNL_HIP(ctx, hipMemcpyAsync(ctx->h_status, ctx->d_status, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
    SFCNL_HIP(ctx, hipStreamSynchronize(ctx->stream));
    uint32_t e = ctx->h_status[kStInputErr];
    if (e) {
        int rc = fill_u32(ctx, ctx->d_status + kStInputErr, 1, 0);
        if (rc) return rc;
        return set_err(ctx, SFCNL_E_INPUT, "input error flags 0x%x (1: non-finite position, 2: bad radius, 4: bad permutation, 8: positions span a "
                       "period or a radius reaches half of it)", e);
    }
    return SFCNL_OK;
}
