// Learned smoothing-length seed: features, an 8 -> 64 -> 64 -> 1 ReLU MLP on
// the bf16 matrix cores (FP32 accumulate), its gradient and Adam. The network
// output is added to the cube-root rule's step, -feature0 / 3, so an untrained
// network reproduces the plain rule.
//
// Matrix-core layout (v_mfma_f32_16x16x16_bf16, wave64): for lane l with
// s = l % 16 and g = l / 16, the A operand holds A[s][4g .. 4g+3], the B
// operand B[4g .. 4g+3][s], and the accumulator D[4g .. 4g+3][s]. Activations
// are kept transposed (units x samples), so a layer's accumulator fragment is
// directly the next layer's B operand: W1 X^T, then W2 H1^T, 16 samples per
// tile. The backward pass forms W2^T delta2 the same way; the two weight
// gradients contract over samples and go through a per-wave LDS transpose.
#include "internal.h"

namespace sfcnl {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = SFCNL_HSEED_NFEAT;  // 8 features
constexpr int kHid = 64;
constexpr int kOffW1 = 0, kOffB1 = 512, kOffW2 = 576, kOffB2 = 4672, kOffW3 = 4736, kOffB3 = 4800;
constexpr int kNParam = SFCNL_MLP_NPARAM;  // 4801
constexpr int kWaves = 4;

// float -> bfloat16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ short f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (short)0x7FC0;
    return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(short b) { return __uint_as_float((uint32_t)(uint16_t)b << 16); }
__device__ __forceinline__ float qbf(float f) { return bf2f(f2bf(f)); }

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Weights of one block, rounded to bf16 once.
struct WeightsLds {
    short W1[kHid * 16];     // [unit][feature], features 8..15 zero
    short W2[kHid * kHid];   // [out unit][in unit]
    short W2T[kHid * kHid];  // [in unit][out unit]
    float b1[kHid], b2[kHid], w3q[kHid];
    float b3;
};

__device__ void load_weights(WeightsLds &L, const float *__restrict__ p) {
    for (int t = threadIdx.x; t < kHid * 16; t += blockDim.x) {
        const int u = t / 16, f = t % 16;
        L.W1[t] = f < kIn ? f2bf(p[kOffW1 + u * kIn + f]) : (short)0;
    }
    for (int t = threadIdx.x; t < kHid * kHid; t += blockDim.x) {
        const short w = f2bf(p[kOffW2 + t]);
        L.W2[t] = w;
        L.W2T[(t % kHid) * kHid + t / kHid] = w;
    }
    for (int t = threadIdx.x; t < kHid; t += blockDim.x) {
        L.b1[t] = p[kOffB1 + t];
        L.b2[t] = p[kOffB2 + t];
        L.w3q[t] = qbf(p[kOffW3 + t]);
    }
    if (threadIdx.x == 0) L.b3 = p[kOffB3];
    __syncthreads();
}

__device__ __forceinline__ bf16x4 lds4(const short *p) { return *reinterpret_cast<const bf16x4 *>(p); }

// Features of sample s as the B operand (lanes g = 0, 1 carry features
// 4g .. 4g+3; the K padding 8..15 is zero).
__device__ __forceinline__ bf16x4 load_x(const uint16_t *__restrict__ feat, int64_t idx, bool valid, int g) {
    bf16x4 x = {0, 0, 0, 0};
    if (valid && g < 2) {
        const uint2 w = *reinterpret_cast<const uint2 *>(feat + idx * kIn + 4 * g);
        x[0] = (short)(w.x & 0xFFFFu);
        x[1] = (short)(w.x >> 16);
        x[2] = (short)(w.y & 0xFFFFu);
        x[3] = (short)(w.y >> 16);
    }
    return x;
}

struct Fwd {
    f32x4 z1[4], z2[4];  // pre-activations (with bias)
    bf16x4 h1[4];        // relu(z1) in bf16: B operands of layer 2
    f32x4 h2[4];         // relu(z2) rounded to bf16
    float y;             // output of sample s (same in the 4 lanes of s)
};

__device__ __forceinline__ void forward_tile(const WeightsLds &L, bf16x4 x, int s, int g, Fwd &F) {
    // x: this lane's B-operand slice of the sample features (see load_x)
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        const f32x4 z = mfma(lds4(&L.W1[(mt * 16 + s) * 16 + 4 * g]), x, f32x4{0, 0, 0, 0});
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const float v = z[i] + L.b1[mt * 16 + 4 * g + i];
            F.z1[mt][i] = v;
            F.h1[mt][i] = f2bf(fmaxf(v, 0.0f));
        }
    }
    float part = 0.0f;
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        f32x4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int kt = 0; kt < 4; kt++) acc = mfma(lds4(&L.W2[(mt * 16 + s) * kHid + kt * 16 + 4 * g]), F.h1[kt], acc);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int u = mt * 16 + 4 * g + i;
            const float v = acc[i] + L.b2[u];
            F.z2[mt][i] = v;
            F.h2[mt][i] = qbf(fmaxf(v, 0.0f));
            part = __builtin_fmaf(L.w3q[u], F.h2[mt][i], part);
        }
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    // residual on the cube-root rule: -feature0 / 3 = log((target / (n+1))^(1/3));
    // lane s (g = 0) holds feature 0 of sample s
    const float f0 = __shfl(bf2f(x[0]), s, 64);
    F.y = part + L.b3 - f0 * (1.0f / 3.0f);
}

__global__ __launch_bounds__(256) void k_mlp_infer(const float *__restrict__ params, int64_t n,
                                                   const uint16_t *__restrict__ feat, float *__restrict__ out) {
    __shared__ WeightsLds L;
    load_weights(L, params);
    const int lane = sfc_lane(), s = lane & 15, g = lane >> 4;
    const int64_t ntiles = (n + 15) / 16;
    const int64_t wave = (int64_t)blockIdx.x * kWaves + threadIdx.x / kWave;
    const int64_t nw = (int64_t)gridDim.x * kWaves;
    for (int64_t t = wave; t < ntiles; t += nw) {
        const int64_t idx = t * 16 + s;
        const bool v = idx < n;
        Fwd F;
        forward_tile(L, load_x(feat, idx, v, g), s, g, F);
        if (v && g == 0) out[idx] = F.y;
    }
}

// Gradient of the mean squared error over a batch: each wave accumulates its
// tiles and writes one partial gradient (kNParam floats) and partial loss.
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ params, int64_t nsamp,
                                                  const uint16_t *__restrict__ feat, const float *__restrict__ target,
                                                  int64_t batch, int64_t start, int64_t mul, int64_t add,
                                                  float *__restrict__ partial) {
    __shared__ WeightsLds L;
    __shared__ short T1[kWaves][kHid * 16], T2[kWaves][kHid * 16], T3[kWaves][kHid * 16], TX[kWaves][16 * 16];
    load_weights(L, params);
    const int lane = sfc_lane(), s = lane & 15, g = lane >> 4;
    const int w = threadIdx.x / kWave;
    const int64_t ntiles = (batch + 15) / 16;
    const int64_t wave = (int64_t)blockIdx.x * kWaves + w;
    const int64_t nw = (int64_t)gridDim.x * kWaves;
    const float inv_b = 2.0f / (float)batch;

    f32x4 dW2[4][4], dW1[4];
    float dw3[4][4], db2[4][4], db1[4][4];
    float db3 = 0.0f, loss = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        dW1[a] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int b = 0; b < 4; b++) {
            dW2[a][b] = f32x4{0, 0, 0, 0};
            dw3[a][b] = db2[a][b] = db1[a][b] = 0.0f;
        }
    }
    for (int64_t t = wave; t < ntiles; t += nw) {
        const int64_t k = t * 16 + s;
        const bool v = k < batch;
        const int64_t idx = v ? (int64_t)(((unsigned __int128)(uint64_t)(start + k) * (uint64_t)mul + (uint64_t)add) %
                                          (uint64_t)nsamp)
                              : 0;
        const bf16x4 x = load_x(feat, idx, v, g);
        Fwd F;
        forward_tile(L, x, s, g, F);
        const float r = v ? F.y - target[idx] : 0.0f;
        if (g == 0) loss = __builtin_fmaf(r, r, loss);
        const float dy = r * inv_b;
        if (g == 0) db3 += dy;
        // layer 3 and the error entering layer 2
        bf16x4 d2b[4];
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int u = mt * 16 + 4 * g + i;
                dw3[mt][i] = __builtin_fmaf(dy, F.h2[mt][i], dw3[mt][i]);
                const float d2 = F.z2[mt][i] > 0.0f ? L.w3q[u] * dy : 0.0f;
                db2[mt][i] += d2;
                d2b[mt][i] = f2bf(d2);
            }
        }
        // error entering layer 1: W2^T delta2
        bf16x4 d1b[4];
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            f32x4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int kt = 0; kt < 4; kt++) acc = mfma(lds4(&L.W2T[(mt * 16 + s) * kHid + kt * 16 + 4 * g]), d2b[kt], acc);
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const float d1 = F.z1[mt][i] > 0.0f ? acc[i] : 0.0f;
                db1[mt][i] += d1;
                d1b[mt][i] = f2bf(d1);
            }
        }
        // transposes for the contractions over samples
        short *t1 = T1[w], *t2 = T2[w], *t3 = T3[w], *tx = TX[w];
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int u = mt * 16 + 4 * g + i;
                t1[u * 16 + s] = F.h1[mt][i];
                t2[u * 16 + s] = d2b[mt][i];
                t3[u * 16 + s] = d1b[mt][i];
            }
        }
#pragma unroll
        for (int i = 0; i < 4; i++) tx[(4 * g + i) * 16 + s] = x[i];  // feature 4g+i of sample s (zero for g >= 2)
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // dW2[u2][u1] += sum_s delta2[u2][s] h1[u1][s]
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            const bf16x4 a = lds4(&t2[(mt * 16 + s) * 16 + 4 * g]);
#pragma unroll
            for (int nt = 0; nt < 4; nt++) dW2[mt][nt] = mfma(a, lds4(&t1[(nt * 16 + s) * 16 + 4 * g]), dW2[mt][nt]);
        }
        // dW1[u1][f] += sum_s delta1[u1][s] x[f][s]
        const bf16x4 bx = lds4(&tx[s * 16 + 4 * g]);
#pragma unroll
        for (int mt = 0; mt < 4; mt++) dW1[mt] = mfma(lds4(&t3[(mt * 16 + s) * 16 + 4 * g]), bx, dW1[mt]);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    // sum the per-sample partials over the 16 lanes of each g
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
#pragma unroll
            for (int d = 1; d < 16; d <<= 1) {
                dw3[mt][i] += __shfl_xor(dw3[mt][i], d, 64);
                db2[mt][i] += __shfl_xor(db2[mt][i], d, 64);
                db1[mt][i] += __shfl_xor(db1[mt][i], d, 64);
            }
        }
    }
    for (int d = 1; d < 64; d <<= 1) {
        db3 += __shfl_xor(db3, d, 64);
        loss += __shfl_xor(loss, d, 64);
    }
    float *out = partial + wave * (kNParam + 1);
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int u = mt * 16 + 4 * g + i;
#pragma unroll
            for (int nt = 0; nt < 4; nt++) out[kOffW2 + u * kHid + nt * 16 + s] = dW2[mt][nt][i];
            if (s < kIn) out[kOffW1 + u * kIn + s] = dW1[mt][i];
            if (s == 0) {
                out[kOffW3 + u] = dw3[mt][i];
                out[kOffB2 + u] = db2[mt][i];
                out[kOffB1 + u] = db1[mt][i];
            }
        }
    }
    if (lane == 0) {
        out[kOffB3] = db3;
        out[kNParam] = loss;
    }
}

// Sum of the wave partials; index kNParam is the loss (mean over the batch).
__global__ __launch_bounds__(256) void k_mlp_reduce(const float *__restrict__ partial, int nwaves, int64_t batch,
                                                    float *__restrict__ grad, float *__restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNParam) return;
    float acc = 0.0f;
    for (int w = 0; w < nwaves; w++) acc += partial[(size_t)w * (kNParam + 1) + p];
    if (p < kNParam)
        grad[p] = acc;
    else if (loss)
        *loss = acc / (float)batch;
}

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, float lr, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParam) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

// splitmix64 (Steele, Lea & Flood 2014): one 64-bit output per counter value.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// He-uniform weights for the ReLU layers, small output weights, zero biases.
__global__ __launch_bounds__(256) void k_mlp_init(uint64_t seed, float *__restrict__ p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParam) return;
    const double u = (double)(splitmix64(seed * 0x100000001B3ull + (uint64_t)i) >> 11) * 0x1.0p-53;  // [0, 1)
    float bound = 0.0f;
    if (i < kOffB1)
        bound = sqrtf(6.0f / kIn);
    else if (i >= kOffW2 && i < kOffB2)
        bound = sqrtf(6.0f / kHid);
    else if (i >= kOffW3 && i < kOffB3)
        bound = 0.1f * sqrtf(6.0f / kHid);
    p[i] = (float)((2.0 * u - 1.0) * bound);
}

// Features of particle i (SFC order), all dimensionless:
//   0 log((n_prev + 1) / target)
//   1 log(cluster box diagonal / h)        2 log(super-cluster box diagonal / h)
//   3..5 log((1 + occupancy) / target) of the particle's key-prefix cell at
//        levels L0 - 1, L0, L0 + 1, with L0 the level whose cell edge is
//        closest to h
//   6 log2(edge_0 / h) - L0 (where h falls between levels)
//   7 log(target / 100)
__device__ __forceinline__ uint32_t lower_bound_key(const uint64_t *keys, uint32_t lo, uint32_t hi, uint64_t v) {
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (keys[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ float wave_min(float v, int from, int to) {
    for (int d = from; d < to; d <<= 1) v = fminf(v, __shfl_xor(v, d, 64));
    return v;
}
__device__ __forceinline__ float wave_max(float v, int from, int to) {
    for (int d = from; d < to; d <<= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
    return v;
}

__device__ __forceinline__ float diag(float lx, float ly, float lz, float hx, float hy, float hz) {
    return sqrtf((hx - lx) * (hx - lx) + (hy - ly) * (hy - ly) + (hz - lz) * (hz - lz));
}

// One wavefront = one 64-particle super-cluster (blocks of 256 start at
// multiples of 64): the 8-particle cluster box and the super-cluster box come
// from min / max over lane groups; absent particles are NaN, which fminf and
// fmaxf ignore.
__global__ __launch_bounds__(256) void k_features(int64_t n, const uint64_t *__restrict__ keys,
                                                  const float *__restrict__ x, const float *__restrict__ y,
                                                  const float *__restrict__ z, const float *__restrict__ h,
                                                  const int32_t *__restrict__ nnb, float edge0, int target,
                                                  uint16_t *__restrict__ feat, SegTable seg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i < n;
    const float px = in ? x[i] : NAN, py = in ? y[i] : NAN, pz = in ? z[i] : NAN;
    float clx = wave_min(px, 1, 8), cly = wave_min(py, 1, 8), clz = wave_min(pz, 1, 8);
    float chx = wave_max(px, 1, 8), chy = wave_max(py, 1, 8), chz = wave_max(pz, 1, 8);
    const float slx = wave_min(clx, 8, 64), sly = wave_min(cly, 8, 64), slz = wave_min(clz, 8, 64);
    const float shx = wave_max(chx, 8, 64), shy = wave_max(chy, 8, 64), shz = wave_max(chz, 8, 64);
    if (!in) return;
    // key searches stay inside the particle's own system
    uint32_t klo = 0, khi = (uint32_t)n;
    if (seg.on()) {
        const int sy = seg.sc_sys[i / kScSize];
        klo = seg.pbase[sy];
        khi = klo + seg.count[sy];
        edge0 = seg.edge[sy];
        if ((uint32_t)i >= khi) {  // padding
            *reinterpret_cast<uint4 *>(feat + i * kIn) = make_uint4(0u, 0u, 0u, 0u);
            return;
        }
    }
    const float hi = h[i];
    const float lt = logf((float)target);
    float f[kIn];
    f[0] = nnb ? logf((float)nnb[i] + 1.0f) - lt : 0.0f;  // no count yet: 0
    f[1] = logf(fmaxf(diag(clx, cly, clz, chx, chy, chz) / hi, 1e-3f));
    f[2] = logf(fmaxf(diag(slx, sly, slz, shx, shy, shz) / hi, 1e-3f));
    const float lev = log2f(edge0 / hi);
    int L0 = (int)rintf(lev);
    L0 = L0 < 2 ? 2 : (L0 > 20 ? 20 : L0);
    const uint64_t key = keys[i];
#pragma unroll
    for (int d = -1; d <= 1; d++) {
        const int L = L0 + d;
        const int shift = 3 * (21 - L);
        const uint64_t pre = key >> shift;
        const uint32_t a = lower_bound_key(keys, klo, khi, pre << shift);
        const uint32_t b = lower_bound_key(keys, klo, khi, (pre + 1) << shift);
        f[4 + d] = logf(1.0f + (float)(b - a)) - lt;
    }
    f[6] = lev - (float)L0;
    f[7] = lt - logf(100.0f);
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; k++)
        w[k] = (uint32_t)(uint16_t)f2bf(f[2 * k]) | ((uint32_t)(uint16_t)f2bf(f[2 * k + 1]) << 16);
    *reinterpret_cast<uint4 *>(feat + i * kIn) = make_uint4(w[0], w[1], w[2], w[3]);
}

constexpr int kGradMaxWaves = 256;

}  // namespace
}  // namespace sfcnl

using namespace sfcnl;

extern "C" int sfcnl_mlp_init(sfcnl_ctx ctx, uint64_t seed, float *d_params) {
    if (!ctx) return SFCNL_E_ARG;
    if (!d_params) return set_err(ctx, SFCNL_E_ARG, "sfcnl_mlp_init: null params");
    k_mlp_init<<<blocks_for(kNParam, 256), 256, 0, ctx->stream>>>(seed, d_params);
    SFCNL_LAUNCHED(ctx);
    return SFCNL_OK;
}

extern "C" int sfcnl_mlp_infer(sfcnl_ctx ctx, const float *d_params, int64_t n, const uint16_t *d_feat, float *d_out) {
    if (!ctx) return SFCNL_E_ARG;
    if (n < 0) return set_err(ctx, SFCNL_E_ARG, "sfcnl_mlp_infer: n < 0");
    if (n == 0) return SFCNL_OK;
    if (!d_params || !d_feat || !d_out) return set_err(ctx, SFCNL_E_ARG, "sfcnl_mlp_infer: null pointer");
    const int64_t ntiles = (n + 15) / 16;
    int64_t blocks = (ntiles + kWaves - 1) / kWaves;
    if (blocks > 4096) blocks = 4096;
    k_mlp_infer<<<(unsigned)blocks, 256, 0, ctx->stream>>>(d_params, n, d_feat, d_out);
    SFCNL_LAUNCHED(ctx);
    return SFCNL_OK;
}

extern "C" int sfcnl_mlp_grad_workspace(int64_t batch, size_t *ws_bytes) {
    if (batch < 1 || !ws_bytes) return SFCNL_E_ARG;
    *ws_bytes = (size_t)kGradMaxWaves * (kNParam + 1) * sizeof(float);
    return SFCNL_OK;
}

extern "C" int sfcnl_mlp_grad(sfcnl_ctx ctx, const float *d_params, int64_t nsamp, const uint16_t *d_feat,
                              const float *d_target, int64_t batch, int64_t start, int64_t mul, int64_t add,
                              void *d_ws, size_t ws_bytes, float *d_grad, float *d_loss) {
    if (!ctx) return SFCNL_E_ARG;
    if (nsamp < 1 || batch < 1 || mul < 1 || add < 0)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_mlp_grad: need nsamp, batch, mul >= 1 and add >= 0");
    if (!d_params || !d_feat || !d_target || !d_ws || !d_grad)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_mlp_grad: null pointer");
    size_t need;
    sfcnl_mlp_grad_workspace(batch, &need);
    if (ws_bytes < need) return set_err(ctx, SFCNL_E_ARG, "sfcnl_mlp_grad: workspace %zu < %zu", ws_bytes, need);
    const int64_t ntiles = (batch + 15) / 16;
    int64_t waves = ntiles < kGradMaxWaves ? ntiles : kGradMaxWaves;
    waves = (waves + kWaves - 1) / kWaves * kWaves;
    float *partial = reinterpret_cast<float *>(d_ws);
    k_mlp_grad<<<(unsigned)(waves / kWaves), 256, 0, ctx->stream>>>(d_params, nsamp, d_feat, d_target, batch, start,
                                                                    mul, add, partial);
    SFCNL_LAUNCHED(ctx);
    k_mlp_reduce<<<blocks_for(kNParam + 1, 256), 256, 0, ctx->stream>>>(partial, (int)waves, batch, d_grad, d_loss);
    SFCNL_LAUNCHED(ctx);
    return SFCNL_OK;
}

extern "C" int sfcnl_mlp_adam(sfcnl_ctx ctx, float *d_params, const float *d_grad, float *d_m, float *d_v, int64_t t,
                              float lr) {
    if (!ctx) return SFCNL_E_ARG;
    if (t < 1 || !(lr > 0.0f)) return set_err(ctx, SFCNL_E_ARG, "sfcnl_mlp_adam: need step >= 1 and lr > 0");
    if (!d_params || !d_grad || !d_m || !d_v) return set_err(ctx, SFCNL_E_ARG, "sfcnl_mlp_adam: null pointer");
    const float c1 = (float)(1.0 / (1.0 - pow(0.9, (double)t)));
    const float c2 = (float)(1.0 / (1.0 - pow(0.999, (double)t)));
    k_adam<<<blocks_for(kNParam, 256), 256, 0, ctx->stream>>>(d_params, d_grad, d_m, d_v, lr, c1, c2);
    SFCNL_LAUNCHED(ctx);
    return SFCNL_OK;
}

int sfcnl::features_impl(sfcnl_ctx ctx, int64_t n, const uint64_t *d_keys, const float *d_x, const float *d_y,
                         const float *d_z, const float *d_h, const int32_t *d_nnb, float box_edge, int target,
                         uint16_t *d_feat, const SegTable &seg) {
    k_features<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, d_keys, d_x, d_y, d_z, d_h, d_nnb, box_edge, target,
                                                            d_feat, seg);
    SFCNL_LAUNCHED(ctx);
    return SFCNL_OK;
}

extern "C" int sfcnl_hseed_features(sfcnl_ctx ctx, int64_t n, const uint64_t *d_keys, const float *d_x,
                                    const float *d_y, const float *d_z, const float *d_h, const int32_t *d_nnb,
                                    float box_edge, int target, uint16_t *d_feat) {
    if (!ctx) return SFCNL_E_ARG;
    if (n < 0 || n >= (int64_t(1) << 31)) return set_err(ctx, SFCNL_E_ARG, "sfcnl_hseed_features: n out of range");
    if (n == 0) return SFCNL_OK;
    if (!d_keys || !d_x || !d_y || !d_z || !d_h || !d_feat || !(box_edge > 0.0f) || target < 1)
        return set_err(ctx, SFCNL_E_ARG, "sfcnl_hseed_features: bad argument");
    return features_impl(ctx, n, d_keys, d_x, d_y, d_z, d_h, d_nnb, box_edge, target, d_feat, SegTable{});
}
