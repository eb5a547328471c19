/*
 * sfcnl -- compressed space-filling-curve cluster neighbour lists on gfx950.
 *
 * C ABI of the GPU library. The operations follow "GPU-Native Compressed
 * Neighbor Lists with a Space-Filling-Curve Data Layout":
 *   sfc_sort        Hilbert keys and SFC order of the particles (Sec. II-A)
 *   sfc_gather      particle fields into SFC order (Sec. II-A, II-C); the
 *                   sfc_gather_ws form stages them through a workspace
 *   build_clusters  fixed-size clusters of SFC-consecutive particles and their
 *                   bounding boxes (Sec. II-A)
 *   build_nlist     octree traversal, cluster-pair list with per-i-cluster
 *                   bitmasks, nibble compression (Sec. II-A, II-B, II-C)
 *   nlist_pass      decompress and compute the SPH density sum and neighbour
 *                   counts (Sec. II-A "neighbor pass", Sec. II-D, Listing 1)
 *   nlist_pass_lj   the Lennard-Jones 12/6 + Coulomb force pass of the
 *                   Sec. III benchmark (interaction cutoff inside the list's)
 *   build_rows      the compressed 1x1 list derived from a cluster list, and
 *   rows_pass       its density pass (the paper's future work, Sec. V)
 *
 * Conventions shared by every call:
 *   - d_* arguments are device pointers, h_* arguments are host pointers. The
 *     caller owns every buffer; the library only borrows them for the call.
 *   - Work is enqueued on the context's HIP stream. Calls return as soon as
 *     the work is enqueued, except build_nlist, which waits for its own
 *     kernels to read back list size and error flags (build_nlist_async and
 *     build_nlist_result split that wait off).
 *   - Every call returns an sfcnl status (0 on success, negative on failure)
 *     and never throws. sfcnl_last_error() gives a text for the last failure
 *     on that context.
 *   - Particle indices are 32-bit: n must be below 2^31.
 *   - Errors found on the device (non-finite coordinates, radii <= 0 or
 *     non-finite) are latched in the context and returned as SFCNL_E_INPUT by
 *     the next build_nlist or sfcnl_sync.
 */
#ifndef SFCNL_H
#define SFCNL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SFCNL_OK 0
#define SFCNL_E_ARG (-1)      /* bad argument; nothing was enqueued */
#define SFCNL_E_INPUT (-2)    /* non-finite position or bad radius found on the device */
#define SFCNL_E_CAPACITY (-3) /* output or workspace too small; required sizes reported */
#define SFCNL_E_HIP (-4)      /* a HIP runtime call failed */
#define SFCNL_E_NOCONV (-5)   /* sfcnl_h_iterate: iteration limit reached, particles unconverged */

/* Super-cluster size: 64 particles, one wavefront (Sec. II-A). */
#define SFCNL_SC_SIZE 64
/* Hilbert key resolution: 21 bits per axis, 63-bit keys. */
#define SFCNL_KEY_BITS 21

typedef struct sfcnl_ctx_s *sfcnl_ctx;

/* Creates a context bound to `device` and `stream` (a hipStream_t, NULL for
 * the null stream). Allocates a few KiB of device status memory and pinned
 * host memory for the read-back of build_nlist. */
int sfcnl_create(sfcnl_ctx *out, int device, void *stream);
void sfcnl_destroy(sfcnl_ctx ctx);
/* Re-binds the context to another stream of the same device. */
int sfcnl_set_stream(sfcnl_ctx ctx, void *stream);
/* Launch shape of the density passes (nlist_pass and the batched passes) of
 * this context: 1, 2 or 4 wavefronts (super-clusters) per workgroup (default
 * 1). Results do not depend on it; the batch autotuner times the choices.
 * Other values return SFCNL_E_ARG. */
int sfcnl_set_pass_waves(sfcnl_ctx ctx, int waves);
const char *sfcnl_last_error(sfcnl_ctx ctx);
/* Waits for the stream and returns the latched device-side error, if any
 * (the latch is cleared). */
int sfcnl_sync(sfcnl_ctx ctx);
/* Library version string. */
const char *sfcnl_version(void);

/* ---- 1. SFC order (Sec. II-A) ------------------------------------------
 * Positions are quantised to 21 bits per axis inside h_box = {xmin, xmax,
 * ymin, ymax, zmin, zmax} (host array; max > min on every axis):
 *   q = trunc(f32(f32(x - xmin) * s)), s = f32(2^21 / (xmax - xmin)),
 *   clamped to [0, 2^21 - 1],
 * and mapped to a 63-bit Hilbert key (Skilling's transpose form, x the most
 * significant axis of each 3-bit digit). The particles are then ordered by key
 * with a stable sort (ties keep input order).
 *   d_keys_out [n] u64: sorted keys.
 *   d_perm_out [n] u32: perm[k] = input index of the k-th particle in order.
 *   d_ws / ws_bytes: scratch of at least sfc_sort_workspace(n) bytes. */
int sfc_sort_workspace(int64_t n, size_t *ws_bytes);
int sfc_sort(sfcnl_ctx ctx, int64_t n, const float *d_x, const float *d_y, const float *d_z,
             const float *h_box, uint64_t *d_keys_out, uint32_t *d_perm_out, void *d_ws, size_t ws_bytes);

/* sfc_sort without a caller workspace and without any device allocation, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. Same arguments, kernels and results
 * as sfc_sort (bit for bit); the scratch is a fixed device array of the
 * library (about 13 MiB per GPU, held until the process ends), located once
 * per device by sfcnl_create.
 *   n: 0 .. SFCNL_SORT_NOALLOC_MAX_N; larger n returns SFCNL_E_ARG and
 *     enqueues nothing.
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (contexts on different streams, or host threads) race and must be ordered
 * by the caller. The array keeps the last call's contents; nothing in it needs
 * to start at zero. */
#define SFCNL_SORT_NOALLOC_MAX_N (1 << 20)
int sfc_sort_noalloc(sfcnl_ctx ctx, int64_t n, const float *d_x, const float *d_y, const float *d_z,
                     const float *h_box, uint64_t *d_keys_out, uint32_t *d_perm_out);

/* out[f][k] = in[f][perm[k]] for nfields (1..8) float arrays of length n.
 * h_in / h_out are host arrays of device pointers; out must not alias in. */
int sfc_gather(sfcnl_ctx ctx, int64_t n, const uint32_t *d_perm, int nfields, const float *const *h_in,
               float *const *h_out);

/* The same gather staged through a workspace: up to four fields at a time are
 * first packed into 16-byte records in input order (one coalesced pass), so
 * that every particle's fields arrive with one random read instead of one per
 * field. Results are identical to sfc_gather, bit for bit.
 *   d_ws / ws_bytes: at least sfc_gather_workspace(n) bytes (16 n + 256), any
 *   alignment; reused from one call to the next. */
int sfc_gather_workspace(int64_t n, size_t *ws_bytes);
int sfc_gather_ws(sfcnl_ctx ctx, int64_t n, const uint32_t *d_perm, int nfields, const float *const *h_in,
                  float *const *h_out, void *d_ws, size_t ws_bytes);

/* ---- 2. Clusters (Sec. II-A) ---------------------------------------------
 * Cluster c holds SFC-ordered particles [cs*c, min(cs*c + cs, n)). For each
 * cluster: d_bbox_out[8c .. 8c+7] = {lo.x, lo.y, lo.z, max h, hi.x, hi.y,
 * hi.z, 0} (exact FP32 min / max). cluster_size is 4, 8 or 16 (the paper uses
 * 8 on wave64 hardware, Sec. II-D; the cluster overhead grows with the size,
 * Sec. III-A). Inputs must be in SFC order. Also checks inputs (latched as
 * SFCNL_E_INPUT). */
int build_clusters(sfcnl_ctx ctx, int64_t n, const float *d_x, const float *d_y, const float *d_z,
                   const float *d_h, int cluster_size, float *d_bbox_out);

/* ---- 3. Neighbour list (Sec. II-A, II-B, II-C) ---------------------------
 * Pair set: (i, j) with i != j and d2 < f32(max(h_i, h_j)^2), where
 * dx = f32(x_j - x_i) (likewise y, z) and d2 = fma(dz, dz, fma(dy, dy, dx*dx)).
 * Super-cluster s = particles [64 s, 64 s + 64) = the S = 64 / cs i-clusters
 * S s .. S s + S - 1 (cs = cluster size). Its list holds every j-cluster (cs
 * particles) containing a j paired with some i of s, in ascending order, each
 * with an S-bit mask whose bit c is set iff some i of i-cluster S s + c has a
 * pair in the j-cluster.
 *
 * Output layout (all little-endian 32-bit words):
 *   d_sc_info [n_sc][2] u32: {word offset into the pool, n_j}, n_sc = ceil(n / 64).
 *   pool at that offset: n_j masks of 1 byte (2 bytes, little-endian, for
 *     cs = 4), padded to 4 bytes; then
 *     compress == 0: n_j u32 j-cluster indices;
 *     compress == 1: per block of 64 index differences (the first from -1):
 *       u64 bitmask (bit k set iff difference k is not 1), then one info
 *       nibble per set bit (v + 6 for v in [2, 9], else number of data
 *       nibbles - 1), then the data nibbles of every value above 9, most
 *       significant first; nibble t in byte t/2, low half first; padded to
 *       4 bytes (Sec. II-B, Table I; segments one wavefront wide, Sec. II-C).
 * Super-clusters are laid out in order, so the pool is deterministic.
 *
 * Inputs: SFC-ordered d_keys (from sfc_sort), positions, radii, and the
 * cluster boxes of build_clusters. opts:
 *   cluster_size  4, 8 or 16 (the size given to build_clusters).
 *   compress      0 or 1.
 *   leaf_bucket   octree leaves hold at most this many particles (8..256).
 *   max_j_per_sc  staging room per super-cluster on average: the workspace
 *                 stages n_sc * ceil(max_j_per_sc / 64) chunks of 64 list
 *                 entries (6 bytes each); every super-cluster fills its own
 *                 first chunk and a longer list continues in chunks shared
 *                 by all super-clusters, so only the total length counts.
 *   half          0: the full list above; 1: the half list, which keeps only
 *                 the pairs with j > i (the symmetric option of Sec. II-D,
 *                 each pair stored once): masks count only such pairs, and a
 *                 super-cluster lists no j-cluster that ends before it.
 *   period        periodic boundaries without shift vectors (Sec. II-A):
 *                 period[a] > 0 makes axis a periodic with that length, 0
 *                 leaves it open (finite, >= 0). Every distance test then
 *                 uses the minimum image of each periodic component in FP32,
 *                 d - L if d > f32(L/2), d + L if d < -f32(L/2), before the
 *                 pair formula; the list stores one entry per j-cluster, with
 *                 no image index, and the passes recompute the image. The
 *                 positions must span less than one period and every radius
 *                 must stay below half of it (else SFCNL_E_INPUT, flag 8).
 *                 Batched calls take open boundaries only. A zeroed field
 *                 (the C default of an initialised struct) means open.
 * Workspace: at least build_nlist_workspace(n, opts) bytes.
 * Returns SFCNL_OK, or SFCNL_E_CAPACITY when the pool (pool_bytes) or the
 * staging list is too small: then *h_used_bytes is the pool size needed and
 * *h_max_nj the largest list length, or, when the staging list was too small,
 * the max_j_per_sc that holds every list; a retry with enough room yields the
 * identical list, and the lists that did not fit are recorded as empty in
 * sc_info (so a pass over it stays inside the pool). On success *h_used_bytes
 * is the pool size used and *h_max_nj the largest list length. Waits for the
 * stream. */
typedef struct {
    int cluster_size;
    int compress;
    int leaf_bucket;
    int max_j_per_sc;
    int half;
    float period[3];
} sfcnl_nlist_opts;

int build_nlist_workspace(int64_t n, const sfcnl_nlist_opts *opts, size_t *ws_bytes);
int build_nlist(sfcnl_ctx ctx, int64_t n, const uint64_t *d_keys, const float *d_x, const float *d_y,
                const float *d_z, const float *d_h, const float *d_bbox, const sfcnl_nlist_opts *opts,
                void *d_ws, size_t ws_bytes, uint32_t *d_sc_info, uint32_t *d_pool, size_t pool_bytes,
                size_t *h_used_bytes, int64_t *h_max_nj);

/* The same build without the wait: build_nlist_async returns once the work
 * is enqueued, so that a pass (or the next step's work) can be enqueued behind
 * it at once, and build_nlist_result waits until the build's status has
 * reached the host (not for work enqueued after the build) and returns what
 * build_nlist would have returned, with the same *h_used_bytes and *h_max_nj.
 * One build may be pending per context; build_nlist_result without one is
 * SFCNL_E_ARG. A list that does not fit is recorded as empty in sc_info, so a
 * pass enqueued before the result stays inside the pool; on SFCNL_E_CAPACITY
 * the build (and such a pass) must be redone with the sizes reported. The
 * buffers must stay untouched until the result call. The result call polls
 * pinned host memory that a one-wave kernel behind the build writes (no
 * event, whose barrier would stall the stream), so it keeps the calling
 * thread busy while it waits; a stream error ends the wait with SFCNL_E_HIP. */
int build_nlist_async(sfcnl_ctx ctx, int64_t n, const uint64_t *d_keys, const float *d_x, const float *d_y,
                      const float *d_z, const float *d_h, const float *d_bbox, const sfcnl_nlist_opts *opts,
                      void *d_ws, size_t ws_bytes, uint32_t *d_sc_info, uint32_t *d_pool, size_t pool_bytes);
int build_nlist_result(sfcnl_ctx ctx, size_t *h_used_bytes, int64_t *h_max_nj);

/* ---- 4. Neighbour pass (Sec. II-A, Sec. II-D Listing 1) ------------------
 * Decompresses each super-cluster's list and evaluates every cs x cs particle
 * tile of a listed (j-cluster, set mask bit) pair:
 *   rho_i = m_i W(0, h_i) + sum_{j != i, d2 < f32(h_i^2)} m_j W(r_ij, h_i)
 *   nnb_i = number of such j,
 * W the M4 cubic spline of compact support h (3-D norm 8 / (pi h^3)), in
 * FP32. d_m == NULL means unit masses; d_nnb may be NULL. Outputs in SFC
 * order. cluster_size and compress as given to build_nlist; half = 1 for a
 * half list (built with opts->half): each stored pair then feeds both
 * particles (Sec. II-D's symmetric evaluation), added with atomics, so the
 * last bits of rho may differ from run to run (nnb stays exact). A full list
 * must be passed with half = 0. h_period: host pointer to the 3 periods the
 * list was built with (opts->period), or NULL for open boundaries. */
int nlist_pass(sfcnl_ctx ctx, int64_t n, int cluster_size, int compress, int half, const uint32_t *d_sc_info,
               const uint32_t *d_pool, const float *d_x, const float *d_y, const float *d_z,
               const float *d_h, const float *d_m, float *d_rho, int32_t *d_nnb, const float *h_period);

/* ---- 4b. Lennard-Jones 12/6 + Coulomb pass (Sec. III, Lennard-Jones benchmark)
 * The benchmark pass of Sec. III with a Verlet buffer: the list is built once
 * with a radius h_i >= r_cut for every particle (the list cutoff) and reused;
 * the pass keeps only the pairs with d2 < f32(r_cut^2) (the interaction
 * cutoff), decided by the pair formula of build_nlist. For those pairs
 *   U(r) = 4 eps ((sigma/r)^12 - (sigma/r)^6) + coulomb q_i q_j / r
 *   F_i  = sum_j [24 eps (2 (sigma/r)^12 - (sigma/r)^6) / r^2 + coulomb q_i q_j / r^3] (x_i - x_j)
 *   E_i  = 1/2 sum_j U(r_ij)
 * in FP32 (reciprocal and reciprocal square root at 1 ulp). Pairs within
 * r_cut that the list does not hold (a list built with radii below r_cut)
 * are not seen. Outputs in SFC order: d_fx, d_fy, d_fz forces, d_epot
 * (nullable) per-particle energies. d_q == NULL means no charges (pure
 * Lennard-Jones). cluster_size, compress and half as given to build_nlist; a
 * half list feeds both particles of every stored pair (Newton's third law)
 * through float atomics, so the last bits vary from run to run. Two particles
 * at the same position give non-finite forces. h_period: the 3 periods of the
 * list (opts->period) or NULL for open boundaries; periodic pairs use their
 * minimum images. */
typedef struct {
    float eps;      /* Lennard-Jones well depth, finite */
    float sigma;    /* Lennard-Jones length, > 0 */
    float coulomb;  /* Coulomb prefactor k, finite (ignored without charges) */
    float r_cut;    /* interaction cutoff, > 0 */
} sfcnl_lj_params;
int nlist_pass_lj(sfcnl_ctx ctx, int64_t n, int cluster_size, int compress, int half, const uint32_t *d_sc_info,
                  const uint32_t *d_pool, const float *d_x, const float *d_y, const float *d_z, const float *d_q,
                  const sfcnl_lj_params *params, float *d_fx, float *d_fy, float *d_fz, float *d_epot,
                  const float *h_period);

/* ---- 4c. Compressed 1x1 list (the paper's future work, Sec. V) -----------
 * The combination of the index compression with a full neighbour list: row i
 * holds particle i's neighbours in the pair set (j != i,
 * d2 < f32(max(h_i, h_j)^2), minimum images on periodic axes) in ascending
 * order, encoded as the index stream of a super-cluster list without masks
 * (differences from -1 in 64-value nibble segments, or raw u32 indices when
 * compress = 0). Rows follow each other in particle order; d_row_info [n][2]
 * u32 holds {word offset, count} per particle (caller-owned, like the pool).
 * build_rows derives the rows from a FULL cluster list (build_nlist with
 * half = 0) of the same positions and radii, given with its cluster size and
 * encoding; h_period as given to that build (NULL: open). The workspace is
 * build_rows_workspace(n) bytes. Waits for the stream; returns
 * SFCNL_E_CAPACITY with *h_used_bytes = the pool size needed when pool_bytes
 * is too small (rows that did not fit are recorded empty; a retry with room
 * gives the identical rows). rows_pass computes the density and counts of
 * nlist_pass from the rows (the own-radius subset of each row), one wavefront
 * per particle, in FP32. */
int build_rows_workspace(int64_t n, size_t *ws_bytes);
int build_rows(sfcnl_ctx ctx, int64_t n, int cluster_size, int list_compress, const uint32_t *d_sc_info,
               const uint32_t *d_pool, const float *d_x, const float *d_y, const float *d_z, const float *d_h,
               int compress, const float *h_period, void *d_ws, size_t ws_bytes, uint32_t *d_row_info,
               uint32_t *d_row_pool, size_t pool_bytes, size_t *h_used_bytes);
int rows_pass(sfcnl_ctx ctx, int64_t n, int compress, const uint32_t *d_row_info, const uint32_t *d_row_pool,
              const float *d_x, const float *d_y, const float *d_z, const float *d_h, const float *d_m,
              float *d_rho, int32_t *d_nnb, const float *h_period);

/* Decodes the whole list on the device into flat arrays: super-cluster s's
 * entries go to [d_offsets[s], d_offsets[s] + n_j), with d_offsets the
 * exclusive prefix sum of n_j (caller-computed, n_sc + 1 entries). Used to
 * check the device decoder on its own. */
int nlist_decode(sfcnl_ctx ctx, int64_t n, int cluster_size, int compress, const uint32_t *d_sc_info,
                 const uint32_t *d_pool, const uint32_t *d_offsets, uint32_t *d_j, uint16_t *d_mask);

/* ---- 5. Smoothing-length iteration -----------------------------------------
 * Drives every particle's radius h_i to `target` +- `tol` own-radius
 * neighbours (the count n_i of nlist_pass) by rebuilding the list. The paper
 * rebuilds its list every step with variable radii (Sec. IV); the iteration
 * rule itself is this library's:
 *   converged      |n_i - target| <= tol: h_i is left unchanged (n_i depends on
 *                  h_i only, so it stays converged);
 *   otherwise      the bracket is narrowed (lo_i = h_i if n_i < target - tol,
 *                  hi_i = h_i if n_i > target + tol), then
 *                  h' = 2 h_i if n_i = 0, else h_i * cbrt(target / n_i) clamped
 *                  to [h_i / 2, 2 h_i]; if h' is not strictly inside
 *                  (lo_i, hi_i), h' = (lo_i + hi_i) / 2 (or hi_i / 2 while
 *                  lo_i = 0, 2 lo_i while hi_i is unbounded).
 * Each round: build_clusters, build_nlist, nlist_pass, update; it stops when no
 * particle moved, after max_iters rounds, or on an error. The first round of a
 * call counts every particle with the requested list form; later rounds
 * recount only the particles whose radius moved in the previous round (n_i
 * depends on h_i alone, so the other counts cannot change and the rounds,
 * radii and counts are those of recounting everything), and a converged run
 * that needed more than one round ends with one list build of every
 * super-cluster in the requested form. A later round recounts either through
 * full lists of the super-clusters holding a moved particle (each octree walk
 * shared by up to 64 particles) or, when few moved, with one wavefront per
 * moved particle walking the octree with its own sphere and no list;
 * opts->recount chooses: 0 by the number moved (at most n / 4 + 64: per
 * particle), 1 lists, 2 per particle. Counts and radii are the same either
 * way; densities differ in summation order only. The workspace
 * is build_nlist_workspace(n, nl_opts) bytes. If only that closing build does
 * not fit, SFCNL_E_CAPACITY comes back with h_stats->unconverged == 0: radii,
 * d_rho and d_nnb are final and the list can be built with build_nlist after
 * growing the buffers.
 * Arrays are in SFC order (sfc_sort + sfc_gather). d_h is updated in place.
 * d_bracket [2n] holds {lo_i, hi_i}; it is initialised to {0, +inf} unless
 * opts->resume is set, which continues an interrupted run (for instance after
 * SFCNL_E_CAPACITY, with larger buffers). On SFCNL_OK the list, d_rho and
 * d_nnb describe the final radii. Returns SFCNL_E_NOCONV when max_iters rounds
 * left particles unconverged. d_bbox is caller scratch of 8 floats per
 * cluster. */
typedef struct {
    int target;
    int tol;
    int max_iters;
    int resume;
    int recount;  /* 0 automatic, 1 lists, 2 one wavefront per moved particle */
} sfcnl_hiter_opts;

/* Optional learned step (see section 6), used when `seed` is not NULL:
 *   mode SFCNL_SEED_AFTER_FIRST: the update of the call's first round uses
 *     h * exp(d), d = MLP(features at that round's counts) (the cube-root
 *     rule is the fallback wherever d is not finite or |d| > ln 8; the
 *     bracket test applies as usual);
 *   mode SFCNL_SEED_BEFORE_FIRST: before the first round (unless resuming),
 *     every radius becomes h * exp(clamp(d, -ln 8, ln 8)), d = MLP(features
 *     with no count: feature 0 is 0), computed from the cluster boxes at the
 *     starting radii and the keys; h is unchanged where d is not finite. The
 *     rounds then follow the rule above.
 * Scratch: d_feat n x 8 bf16, d_delta n floats. box_edge = largest edge of
 * the key box given to sfc_sort. */
#define SFCNL_SEED_AFTER_FIRST 0
#define SFCNL_SEED_BEFORE_FIRST 1
typedef struct {
    const float *d_params;
    uint16_t *d_feat;
    float *d_delta;
    float box_edge;
    int mode;
} sfcnl_hseed;

/* Results of sfcnl_h_iterate (host struct): rounds run by this call,
 * particles still outside target +- tol, the sum over rounds of the particles
 * that moved (so moved / n + 1 is the mean number of rounds a particle needed
 * when all converged), and the list sizes of build_nlist. */
typedef struct {
    int iters;
    int64_t unconverged;
    int64_t moved;
    size_t used_bytes;
    int64_t max_nj;
} sfcnl_hiter_stats;

int sfcnl_h_iterate(sfcnl_ctx ctx, int64_t n, const uint64_t *d_keys, const float *d_x, const float *d_y,
                    const float *d_z, float *d_h, float *d_bracket, const float *d_m,
                    const sfcnl_nlist_opts *nl_opts, const sfcnl_hiter_opts *it_opts, float *d_bbox, void *d_ws,
                    size_t ws_bytes, uint32_t *d_sc_info, uint32_t *d_pool, size_t pool_bytes, float *d_rho,
                    int32_t *d_nnb, const sfcnl_hseed *seed, sfcnl_hiter_stats *h_stats);

/* ---- 6. Learned smoothing-length seed (this library's addition) ------------
 * An MLP 8 -> 64 -> 64 -> 1 with ReLU predicts a correction to the cube-root
 * step, d = log(h_converged / h) = -feature0 / 3 + MLP(features), from 8
 * dimensionless features of a particle at radius h with n own-radius
 * neighbours: log((n+1)/target); log(cluster box diagonal / h); log(super-
 * cluster box diagonal / h); log((1 + occupancy)/target) of the particle's
 * Hilbert-key cell at the three levels around the one whose edge is closest to
 * h; the fractional part of that level; log(target / 100).
 * Parameters: SFCNL_MLP_NPARAM floats, W1[64][8], b1[64], W2[64][64], b2[64],
 * w3[64], b3 (FP32 master copy, caller-owned). The kernels round weights,
 * inputs and hidden activations to bfloat16 (nearest even) and use the bf16
 * matrix cores with FP32 accumulation; the back-propagated errors are rounded
 * to bf16 before entering matrix products (bias gradients are not).
 *   sfcnl_hseed_features: d_feat [n][8] bf16 for SFC-ordered d_keys,
 *     positions, d_h and d_nnb; the boxes are those of 8 consecutive
 *     particles and of the 64-particle super-cluster whatever the list's
 *     cluster size; box_edge as above; d_nnb NULL means no count yet
 *     (feature 0 = 0).
 *   sfcnl_mlp_init: deterministic He-uniform initialisation from `seed`
 *     (splitmix64 counter stream), zero biases.
 *   sfcnl_mlp_infer: d_out[i] = MLP(d_feat[i]) - feature0 / 3.
 *   sfcnl_mlp_grad: loss = mean over the batch of (d(f_k) - t_k)^2 and its
 *     gradient d_grad [SFCNL_MLP_NPARAM]; sample k of the batch is
 *     ((start + k) * mul + add) mod nsamp (a permutation of the samples when
 *     gcd(mul, nsamp) = 1). d_loss (nullable) gets the loss.
 *   sfcnl_mlp_adam: one Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected,
 *     step t >= 1) on params with moments d_m, d_v. */
#define SFCNL_MLP_NPARAM 4801
#define SFCNL_HSEED_NFEAT 8
int sfcnl_hseed_features(sfcnl_ctx ctx, int64_t n, const uint64_t *d_keys, const float *d_x, const float *d_y,
                         const float *d_z, const float *d_h, const int32_t *d_nnb, float box_edge, int target,
                         uint16_t *d_feat);
int sfcnl_mlp_init(sfcnl_ctx ctx, uint64_t seed, float *d_params);
int sfcnl_mlp_infer(sfcnl_ctx ctx, const float *d_params, int64_t n, const uint16_t *d_feat, float *d_out);
int sfcnl_mlp_grad_workspace(int64_t batch, size_t *ws_bytes);
int sfcnl_mlp_grad(sfcnl_ctx ctx, const float *d_params, int64_t nsamp, const uint16_t *d_feat,
                   const float *d_target, int64_t batch, int64_t start, int64_t mul, int64_t add, void *d_ws,
                   size_t ws_bytes, float *d_grad, float *d_loss);
int sfcnl_mlp_adam(sfcnl_ctx ctx, float *d_params, const float *d_grad, float *d_m, float *d_v, int64_t t,
                   float lr);

/* ---- 7. Batches of independent systems (this library's addition) ----------
 * Many systems of uneven sizes go through one set of launches: every kernel
 * covers the super-clusters of all systems, each system keeps its own octree
 * (its root is found per super-cluster), its list stores j-cluster indices
 * relative to the system's first cluster, and the result for each system is
 * bit-identical to the single-system calls above on that system alone.
 *
 * Layouts. Input particles are the systems concatenated: system s is
 * [in_off[s], in_off[s+1]) with in_off[0] = 0. The padded (SFC) layout puts
 * system s at pbase[s] (a multiple of 64) and fills up to pbase[s+1] with
 * padding: key all ones, permutation entry 0xFFFFFFFF, fields NaN. Outputs for
 * padding slots are unspecified. Every array below named "padded" has n_padded
 * entries (d_bbox: 8 floats per cluster of padded particles).
 *
 *   sfcnl_batch_create: nsys in [1, SFCNL_BATCH_MAX_SYSTEMS]; h_counts[s] >= 0
 *     particles of system s; h_boxes 6 floats per system (xlo, xhi, ylo, yhi,
 *     zlo, zhi, as the box of sfc_sort). Copies the tables to the context's
 *     device and creates a stream of default priority; the batch belongs to
 *     that device. Total padded size < 2^31.
 *   sfcnl_batch_layout: sizes; h_in_off / h_pbase (nullable) get nsys + 1
 *     entries.
 *   sfcnl_batch_sort: keys of each particle in its system's box (sfc_sort's
 *     definition), sorted stably by (system, key), spread into the padded
 *     layout: d_keys_out, d_perm_out padded (perm entries index the input).
 *   sfcnl_batch_gather: d_out[f][q] = d_in[f][perm[q]], NaN for padding.
 *   sfcnl_batch_build_clusters / _build_nlist / _pass: build_clusters,
 *     build_nlist and nlist_pass on padded arrays; sc_info is per padded
 *     super-cluster (system s owns super-clusters [pbase[s]/64,
 *     pbase[s+1]/64)) and offsets are into the one shared pool.
 *   sfcnl_batch_h_iterate: sfcnl_h_iterate on every system at once, with the
 *     same rule per particle; a converged system is left unchanged while
 *     others continue. With use_graph, the launches of one round are captured
 *     once into a HIP graph on the batch's stream and replayed each round
 *     (the host reads the status block between rounds); the batch's stream is
 *     ordered after the context's stream on entry and before it on return.
 *     The seed (nullable) works as in section 5, except that each system's
 *     box edge comes from its box (seed->box_edge is ignored). h_sys_rounds
 *     (nullable, nsys entries) gets, per system, the rounds it took part in
 *     (the rounds up to and including its first round with no particle
 *     moved). On SFCNL_E_CAPACITY no radius of the failing round changed,
 *     so a call with resume set and larger buffers continues the run.
 * The batch calls enqueue on the context's stream, except _h_iterate (see
 * above), which waits for its stream. */
#define SFCNL_BATCH_MAX_SYSTEMS 65535
typedef struct sfcnl_batch_s *sfcnl_batch;
int sfcnl_batch_create(sfcnl_ctx ctx, int nsys, const int64_t *h_counts, const float *h_boxes, sfcnl_batch *out);
void sfcnl_batch_destroy(sfcnl_batch b);
int sfcnl_batch_layout(sfcnl_batch b, int64_t *n_in, int64_t *n_padded, int64_t *h_in_off, int64_t *h_pbase);
int sfcnl_batch_sort_workspace(sfcnl_batch b, size_t *ws_bytes);
int sfcnl_batch_sort(sfcnl_ctx ctx, sfcnl_batch b, const float *d_x, const float *d_y, const float *d_z,
                     uint64_t *d_keys_out, uint32_t *d_perm_out, void *d_ws, size_t ws_bytes);
int sfcnl_batch_gather(sfcnl_ctx ctx, sfcnl_batch b, const uint32_t *d_perm, int nfields, const float *const *h_in,
                       float *const *h_out);
int sfcnl_batch_nlist_workspace(sfcnl_batch b, const sfcnl_nlist_opts *opts, size_t *ws_bytes);
int sfcnl_batch_build_clusters(sfcnl_ctx ctx, sfcnl_batch b, const float *d_x, const float *d_y, const float *d_z,
                               const float *d_h, int cluster_size, float *d_bbox_out);
int sfcnl_batch_build_nlist(sfcnl_ctx ctx, sfcnl_batch b, const uint64_t *d_keys, const float *d_x,
                            const float *d_y, const float *d_z, const float *d_h, const float *d_bbox,
                            const sfcnl_nlist_opts *opts, void *d_ws, size_t ws_bytes, uint32_t *d_sc_info,
                            uint32_t *d_pool, size_t pool_bytes, size_t *h_used_bytes, int64_t *h_max_nj);
int sfcnl_batch_pass(sfcnl_ctx ctx, sfcnl_batch b, int cluster_size, int compress, int half, const uint32_t *d_sc_info,
                     const uint32_t *d_pool, const float *d_x, const float *d_y, const float *d_z, const float *d_h,
                     const float *d_m, float *d_rho, int32_t *d_nnb);
int sfcnl_batch_h_iterate(sfcnl_ctx ctx, sfcnl_batch b, const uint64_t *d_keys, const float *d_x, const float *d_y,
                          const float *d_z, float *d_h, float *d_bracket, const float *d_m,
                          const sfcnl_nlist_opts *nl_opts, const sfcnl_hiter_opts *it_opts, float *d_bbox,
                          void *d_ws, size_t ws_bytes, uint32_t *d_sc_info, uint32_t *d_pool, size_t pool_bytes,
                          float *d_rho, int32_t *d_nnb, const sfcnl_hseed *seed, int use_graph,
                          sfcnl_hiter_stats *h_stats, int32_t *h_sys_rounds);

/* ---- Stage timing -------------------------------------------------------
 * When enabled, every call brackets each of its stages with a pair of HIP
 * events on the context's stream (no synchronisation). Stages:
 *   0 keys, 1 radix sort, 2 gather, 3 clusters, 4 octree, 5 traversal,
 *   6 encode (prefix sum + encoder), 7 pass.
 * sfcnl_profile_begin allocates `slots` event pairs per stage; recording past
 * that many calls of a stage is skipped. sfcnl_profile_end waits for the
 * stream, writes per stage the summed milliseconds (h_ms[8]) and the number of
 * recorded calls (h_calls[8]), and releases the events. */
#define SFCNL_NSTAGE 8
int sfcnl_profile_begin(sfcnl_ctx ctx, int slots);
int sfcnl_profile_end(sfcnl_ctx ctx, double *h_ms, int64_t *h_calls);
/* Restricts the event recording of the context's stage timing to the stages
 * whose bit is set in stage_mask (bit s = stage s; the default, set by
 * sfcnl_create, is all stages). A timing event makes the stream drain the work
 * before it, so a step timed with every stage bracketed runs slower than
 * without; timing one stage keeps that cost to its own two events. Bits above
 * the stage count return SFCNL_E_ARG. */
int sfcnl_profile_stages(sfcnl_ctx ctx, uint32_t stage_mask);

#ifdef __cplusplus
}
#endif

#endif /* SFCNL_H */
