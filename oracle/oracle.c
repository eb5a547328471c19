/*
 * CPU oracle for the SFC cluster neighbour list and the SPH density pass.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against. It shares no code with
 * the GPU library and the product path never calls it.
 *
 * What it computes (paper: "GPU-Native Compressed Neighbor Lists with a
 * Space-Filling-Curve Data Layout"):
 *   - Hilbert keys of quantised positions (Sec. II-A: particles are kept in
 *     Hilbert order; the curve variant is Skilling's transpose algorithm,
 *     J. Skilling, AIP Conf. Proc. 707, 2004).
 *   - The particle pair set P = {(i,j): i != j, d2 < max(h_i,h_j)^2} under one
 *     fixed FP32 formula (Sec. II-A, per-particle interaction radii).
 *   - The cluster-pair list: per super-cluster of 64 particles, the ascending
 *     j-cluster indices with one bit per i-cluster (Sec. II-A).
 *   - The nibble encoding of Sec. II-B / Table I, laid out in segments of one
 *     wavefront width (Sec. II-C).
 *   - SPH densities rho_i = sum_j m_j W(r_ij, h_i) and neighbour counts in
 *     FP64 (Sec. II-D, Listing 1).
 *   - Lennard-Jones 12/6 + Coulomb forces of the pairs inside an interaction
 *     cutoff shorter than the list cutoff (Sec. III, Lennard-Jones benchmark).
 *   - Periodic boundaries without shift vectors: every distance test takes
 *     the minimum image of each component on periodic axes (Sec. II-A).
 *
 * Must be compiled with -ffp-contract=off: the FP32 pair test below spells
 * out every rounding step and no other contraction is allowed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_KEY_BITS 21

/* ------------------------------------------------------------------------- */
/* Hilbert keys                                                               */
/* ------------------------------------------------------------------------- */

/* Skilling's AxesToTranspose for three axes of `bits` bits, then the
 * transposed words are read out most-significant bit first, x before y
 * before z, three bits per level. */
uint64_t orc_hilbert3(uint32_t x, uint32_t y, uint32_t z, int bits)
{
    uint32_t X[3] = {x, y, z};
    uint32_t top = 1u << (bits - 1);
    /* undo excess work: walk the levels from the top */
    for (uint32_t q = top; q > 1; q >>= 1) {
        uint32_t p = q - 1;
        for (int i = 0; i < 3; i++) {
            if (X[i] & q) {
                X[0] ^= p; /* invert low bits of axis 0 */
            } else {
                uint32_t t = (X[0] ^ X[i]) & p; /* swap low bits of axes 0 and i */
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    /* Gray encode */
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t q = top; q > 1; q >>= 1)
        if (X[2] & q) t ^= q - 1;
    for (int i = 0; i < 3; i++) X[i] ^= t;
    /* interleave */
    uint64_t key = 0;
    for (int b = bits - 1; b >= 0; b--) {
        uint64_t d = ((uint64_t)((X[0] >> b) & 1u) << 2) | ((uint64_t)((X[1] >> b) & 1u) << 1) |
                     (uint64_t)((X[2] >> b) & 1u);
        key = (key << 3) | d;
    }
    return key;
}

/* Quantise one coordinate to 21 bits: q = trunc(f32(f32(x - lo) * s)),
 * clamped to [0, 2^21 - 1]; s = f32(2^21 / (hi - lo)) in double. */
static float orc_scale(float lo, float hi)
{
    return (float)(2097152.0 / ((double)hi - (double)lo));
}

static uint32_t orc_quantise(float x, float lo, float s)
{
    float t = x - lo;
    t = t * s;
    if (!(t > 0.0f)) return 0u;
    if (t >= 2097151.0f) return 2097151u;
    return (uint32_t)t;
}

void orc_hilbert_keys(int64_t n, const float *x, const float *y, const float *z, const float *box,
                      uint64_t *keys)
{
    float sx = orc_scale(box[0], box[1]), sy = orc_scale(box[2], box[3]), sz = orc_scale(box[4], box[5]);
    for (int64_t i = 0; i < n; i++) {
        uint32_t qx = orc_quantise(x[i], box[0], sx);
        uint32_t qy = orc_quantise(y[i], box[2], sy);
        uint32_t qz = orc_quantise(z[i], box[4], sz);
        keys[i] = orc_hilbert3(qx, qy, qz, ORC_KEY_BITS);
    }
}

/* ------------------------------------------------------------------------- */
/* The FP32 pair test                                                         */
/* ------------------------------------------------------------------------- */

/* Periodic axes (Sec. II-A: periodic boundaries without shift vectors, the
 * periodic distance of a pair computed whenever it is needed): per[a] > 0
 * makes axis a periodic with length per[a], 0 leaves it open. A component
 * difference d = f32(x_j - x_i) becomes its minimum image in FP32: d - L if
 * d > f32(L/2), d + L if d < -f32(L/2). Positions lie within one period, so
 * |d| < L and one step suffices. */
static float orc_min_image(float d, float L)
{
    if (L > 0.0f) {
        float hl = 0.5f * L;
        if (d > hl)
            d = d - L;
        else if (d < -hl)
            d = d + L;
    }
    return d;
}

/* The same image choice on the exact FP64 difference of two FP32 coordinates,
 * for the values computed on accepted pairs (their distance is below every
 * radius, which is below L/2, so both rules pick the same image). */
static double orc_diff64(float xj, float xi, float L)
{
    double d = (double)xj - (double)xi;
    if (L > 0.0f) {
        if (d > 0.5 * (double)L)
            d -= (double)L;
        else if (d < -0.5 * (double)L)
            d += (double)L;
    }
    return d;
}

/* d2 = fma(dz, dz, fma(dy, dy, dx*dx)) with dx = f32(x_j - x_i) etc. (minimum
 * images on periodic axes); the pair is in P iff d2 < f32(max(h_i, h_j)^2),
 * strictly. */
static float orc_d2(const float *per, float xi, float yi, float zi, float xj, float yj, float zj)
{
    float dx = orc_min_image(xj - xi, per[0]);
    float dy = orc_min_image(yj - yi, per[1]);
    float dz = orc_min_image(zj - zi, per[2]);
    float dxx = dx * dx;
    return fmaf(dz, dz, fmaf(dy, dy, dxx));
}

static int is_pair_p(const float *per, float xi, float yi, float zi, float hi, float xj, float yj, float zj,
                     float hj)
{
    float d2 = orc_d2(per, xi, yi, zi, xj, yj, zj);
    float r = hi > hj ? hi : hj;
    float r2 = r * r;
    return d2 < r2;
}

static const float orc_open[3] = {0.0f, 0.0f, 0.0f};

int orc_is_pair(float xi, float yi, float zi, float hi, float xj, float yj, float zj, float hj)
{
    return is_pair_p(orc_open, xi, yi, zi, hi, xj, yj, zj, hj);
}

/* Own-radius (gather) test used by the density and the neighbour count. */
static int orc_in_own_radius(const float *per, float xi, float yi, float zi, float hi, float xj, float yj,
                             float zj)
{
    float d2 = orc_d2(per, xi, yi, zi, xj, yj, zj);
    float r2 = hi * hi;
    return d2 < r2;
}

/* ------------------------------------------------------------------------- */
/* Cell list (a textbook uniform grid, Quentrec & Brot 1973)                  */
/* ------------------------------------------------------------------------- */

typedef struct {
    double lo[3], edge[3];
    int64_t dim[3];
    float per[3];   /* periods (0: open axis) */
    int64_t *start; /* ncell + 1 */
    int64_t *idx;   /* particles sorted by cell */
} orc_grid;

static void grid_init(orc_grid *g, const float *period)
{
    memset(g, 0, sizeof *g);
    for (int a = 0; a < 3; a++) g->per[a] = (period && period[a] > 0.0f) ? period[a] : 0.0f;
}

static int64_t grid_cell1(const orc_grid *g, int a, double v)
{
    int64_t c = (int64_t)floor((v - g->lo[a]) / g->edge[a]);
    if (c < 0) c = 0;
    if (c >= g->dim[a]) c = g->dim[a] - 1;
    return c;
}

/* Cells of edge >= max radius * (1 + 2^-20): every FP32-accepted pair lies in
 * adjacent cells, since FP32 rounding accepts pairs at most a few ulp beyond R.
 * On a periodic axis the cells tile the period exactly (edge = L / dim), so a
 * pair whose minimum image wraps lies in the first and last cells. */
static void grid_build(orc_grid *g, int64_t n, const float *x, const float *y, const float *z,
                       const float *h)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double hmax = 0.0;
    const float *p[3] = {x, y, z};
    for (int64_t i = 0; i < n; i++) {
        for (int a = 0; a < 3; a++) {
            if (p[a][i] < lo[a]) lo[a] = p[a][i];
            if (p[a][i] > hi[a]) hi[a] = p[a][i];
        }
        if (h[i] > hmax) hmax = h[i];
    }
    if (n == 0) { lo[0] = lo[1] = lo[2] = 0.0; hi[0] = hi[1] = hi[2] = 0.0; }
    double need = hmax * (1.0 + ldexp(1.0, -20));
    double edge = need;
    double ext = 0.0;
    for (int a = 0; a < 3; a++) if (hi[a] - lo[a] > ext) ext = hi[a] - lo[a];
    /* keep the cell count near N: a coarser grid is still exact, just slower */
    double cap = ceil(cbrt((double)(n > 1 ? n : 1))) + 1.0;
    if (edge <= 0.0 || ext / edge > cap) edge = ext / cap;
    if (edge <= 0.0) edge = 1.0;
    int64_t ncell = 1;
    for (int a = 0; a < 3; a++) {
        g->lo[a] = lo[a];
        if (g->per[a] > 0.0f) {
            double L = (double)g->per[a];
            int64_t d = need > 0.0 ? (int64_t)floor(L / need) : (int64_t)cap;
            if (d > (int64_t)cap) d = (int64_t)cap;
            if (d < 1) d = 1;
            g->dim[a] = d;
            g->edge[a] = L / (double)d;
        } else {
            g->edge[a] = edge;
            g->dim[a] = (int64_t)floor((hi[a] - lo[a]) / edge) + 1;
        }
        ncell *= g->dim[a];
    }
    g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->idx = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *cell = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) {
        int64_t c = (grid_cell1(g, 2, z[i]) * g->dim[1] + grid_cell1(g, 1, y[i])) * g->dim[0] +
                    grid_cell1(g, 0, x[i]);
        cell[i] = c;
        g->start[c + 1]++;
    }
    for (int64_t c = 0; c < ncell; c++) g->start[c + 1] += g->start[c];
    int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
    memcpy(fill, g->start, (size_t)ncell * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) g->idx[fill[cell[i]]++] = i;
    free(fill);
    free(cell);
}

static void grid_free(orc_grid *g)
{
    free(g->start);
    free(g->idx);
}

/* Cells along axis a next to cell c (c - 1, c, c + 1; wrapped on a periodic
 * axis), each once. */
static int axis_cells(const orc_grid *g, int a, int64_t c, int64_t *out)
{
    int k = 0;
    for (int64_t dc = -1; dc <= 1; dc++) {
        int64_t v = c + dc;
        if (g->per[a] > 0.0f)
            v = ((v % g->dim[a]) + g->dim[a]) % g->dim[a];
        else if (v < 0 || v >= g->dim[a])
            continue;
        int dup = 0;
        for (int t = 0; t < k; t++) dup |= out[t] == v;
        if (!dup) out[k++] = v;
    }
    return k;
}

/* The cells that can hold a partner of a particle at (xi, yi, zi): the 3x3x3
 * block around its cell (at most 27 cells). */
static int cells_around(const orc_grid *g, float xi, float yi, float zi, int64_t *cells)
{
    int64_t cx[3], cy[3], cz[3];
    int nx = axis_cells(g, 0, grid_cell1(g, 0, xi), cx);
    int ny = axis_cells(g, 1, grid_cell1(g, 1, yi), cy);
    int nz = axis_cells(g, 2, grid_cell1(g, 2, zi), cz);
    int k = 0;
    for (int iz = 0; iz < nz; iz++)
        for (int iy = 0; iy < ny; iy++)
            for (int ix = 0; ix < nx; ix++) cells[k++] = (cz[iz] * g->dim[1] + cy[iy]) * g->dim[0] + cx[ix];
    return k;
}

/* Candidate range t of particle i: cell t of its block (grid) or all particles. */
static int candidate_ranges(const orc_grid *g, int use_grid, int64_t n, float xi, float yi, float zi,
                            int64_t *cells)
{
    if (!use_grid) {
        cells[0] = -1;
        return 1;
    }
    (void)n;
    return cells_around(g, xi, yi, zi, cells);
}

static void range_of(const orc_grid *g, int64_t n, int64_t cell, int64_t *k0, int64_t *k1)
{
    if (cell < 0) {
        *k0 = 0;
        *k1 = n;
    } else {
        *k0 = g->start[cell];
        *k1 = g->start[cell + 1];
    }
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Neighbours of particle i in P, ascending, written to out (capacity cap).
 * Returns the count (which may exceed cap; then only cap are written). */
static int64_t neighbours_of(const orc_grid *g, int use_grid, int64_t n, const float *x, const float *y,
                             const float *z, const float *h, int64_t i, int64_t *out, int64_t cap)
{
    int64_t cnt = 0;
    int64_t cells[27];
    int nc = candidate_ranges(g, use_grid, n, x[i], y[i], z[i], cells);
    for (int t = 0; t < nc; t++) {
        int64_t k0, k1;
        range_of(g, n, cells[t], &k0, &k1);
        for (int64_t k = k0; k < k1; k++) {
            int64_t j = cells[t] < 0 ? k : g->idx[k];
            if (j == i) continue;
            if (is_pair_p(g->per, x[i], y[i], z[i], h[i], x[j], y[j], z[j], h[j])) {
                if (cnt < cap) out[cnt] = j;
                cnt++;
            }
        }
    }
    if (cnt <= cap && cnt > 1) qsort(out, (size_t)cnt, sizeof(int64_t), cmp_i64);
    return cnt;
}

/* Maximum |P_i| over all i (to size buffers). */
int64_t orc_max_degree(int64_t n, const float *x, const float *y, const float *z, const float *h,
                       int use_grid, const float *period)
{
    orc_grid g;
    grid_init(&g, period);
    if (use_grid) grid_build(&g, n, x, y, z, h);
    int64_t mx = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(max : mx)
    for (int64_t i = 0; i < n; i++) {
        int64_t c = neighbours_of(&g, use_grid, n, x, y, z, h, i, NULL, 0);
        if (c > mx) mx = c;
    }
    if (use_grid) grid_free(&g);
    return mx;
}

/* Pair set as CSR: offs[n+1], nbr[offs[i]..offs[i+1]) ascending.
 * Call with nbr == NULL to get the counts in offs only. period: 3 floats
 * (0 = open axis) or NULL (all open). */
void orc_pairs_csr(int64_t n, const float *x, const float *y, const float *z, const float *h, int use_grid,
                   int64_t *offs, int64_t *nbr, const float *period)
{
    orc_grid g;
    grid_init(&g, period);
    if (use_grid) grid_build(&g, n, x, y, z, h);
    if (nbr == NULL) {
        offs[0] = 0;
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; i++) offs[i + 1] = neighbours_of(&g, use_grid, n, x, y, z, h, i, NULL, 0);
        for (int64_t i = 0; i < n; i++) offs[i + 1] += offs[i];
    } else {
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; i++)
            neighbours_of(&g, use_grid, n, x, y, z, h, i, nbr + offs[i], offs[i + 1] - offs[i]);
    }
    if (use_grid) grid_free(&g);
}

/* ------------------------------------------------------------------------- */
/* Cluster-pair list (Sec. II-A)                                              */
/* ------------------------------------------------------------------------- */

/* Super-cluster s holds particles [64 s, 64 s + 64); its i-clusters are the
 * cs-sized runs inside it (bit c of a mask = i-cluster c of the super-cluster).
 * Its list holds every j-cluster that contains a j with (i, j) in P for some i
 * of the super-cluster, ascending, with bit c set iff such an i lies in
 * i-cluster c. The half list (the symmetric option of Sec. II-D: each pair
 * stored once) counts only pairs with j > i, so every pair of P appears in
 * exactly one super-cluster's list, under its smaller index. */
typedef struct {
    int64_t count;
    uint32_t *j;
    uint16_t *mask;
} orc_sc_list;

static void sc_list_one(const orc_grid *g, int use_grid, int64_t n, const float *x, const float *y,
                        const float *z, const float *h, int cs, int half, int64_t s, uint16_t *marks,
                        int64_t *touched, int64_t **nbp, int64_t *nbcap, orc_sc_list *out)
{
    int64_t nt = 0;
    for (int64_t i = 64 * s; i < 64 * s + 64 && i < n; i++) {
        int c = (int)((i - 64 * s) / cs);
        int64_t cnt = neighbours_of(g, use_grid, n, x, y, z, h, i, *nbp, *nbcap);
        if (cnt > *nbcap) { /* grow the buffer and search again */
            free(*nbp);
            *nbcap = cnt;
            *nbp = (int64_t *)malloc((size_t)cnt * sizeof(int64_t));
            if (!*nbp) abort();
            cnt = neighbours_of(g, use_grid, n, x, y, z, h, i, *nbp, *nbcap);
        }
        const int64_t *nb = *nbp;
        for (int64_t k = 0; k < cnt; k++) {
            if (half && nb[k] <= i) continue;
            int64_t cj = nb[k] / cs;
            if (marks[cj] == 0) touched[nt++] = cj;
            marks[cj] |= (uint16_t)(1u << c);
        }
    }
    qsort(touched, (size_t)nt, sizeof(int64_t), cmp_i64);
    out->count = nt;
    out->j = (uint32_t *)malloc((size_t)(nt > 0 ? nt : 1) * sizeof(uint32_t));
    out->mask = (uint16_t *)malloc((size_t)(nt > 0 ? nt : 1) * sizeof(uint16_t));
    for (int64_t k = 0; k < nt; k++) {
        out->j[k] = (uint32_t)touched[k];
        out->mask[k] = marks[touched[k]];
        marks[touched[k]] = 0;
    }
}

/* Builds the list for the super-clusters in sc_ids (or all if sc_ids == NULL,
 * nsel = number of super-clusters). max_degree is only the initial size of the
 * per-thread neighbour buffer, which grows on demand. Results are returned as CSR over the
 * selection: *out_offs (nsel+1), *out_j, *out_mask, malloc'ed here and
 * released with orc_free. Returns 0, or -1 on allocation failure. */
int orc_cluster_list(int64_t n, const float *x, const float *y, const float *z, const float *h, int cs, int half,
                     int use_grid, int64_t nsel, const int64_t *sc_ids, int64_t max_degree,
                     int64_t **out_offs, uint32_t **out_j, uint16_t **out_mask, const float *period)
{
    int64_t nclu = (n + cs - 1) / cs;
    orc_grid g;
    grid_init(&g, period);
    if (use_grid) grid_build(&g, n, x, y, z, h);
    orc_sc_list *lists = (orc_sc_list *)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(orc_sc_list));
    int64_t nbcap = max_degree > 0 ? max_degree : 1;
#pragma omp parallel
    {
        uint16_t *marks = (uint16_t *)calloc((size_t)(nclu > 0 ? nclu : 1), sizeof(uint16_t));
        int64_t *touched = (int64_t *)malloc((size_t)(nclu > 0 ? nclu : 1) * sizeof(int64_t));
        int64_t cap = nbcap;
        int64_t *nb = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
#pragma omp for schedule(dynamic, 4)
        for (int64_t k = 0; k < nsel; k++) {
            int64_t s = sc_ids ? sc_ids[k] : k;
            sc_list_one(&g, use_grid, n, x, y, z, h, cs, half, s, marks, touched, &nb, &cap, &lists[k]);
        }
        free(marks);
        free(touched);
        free(nb);
    }
    if (use_grid) grid_free(&g);
    int64_t *offs = (int64_t *)malloc((size_t)(nsel + 1) * sizeof(int64_t));
    offs[0] = 0;
    for (int64_t k = 0; k < nsel; k++) offs[k + 1] = offs[k] + lists[k].count;
    uint32_t *jj = (uint32_t *)malloc((size_t)(offs[nsel] > 0 ? offs[nsel] : 1) * sizeof(uint32_t));
    uint16_t *mm = (uint16_t *)malloc((size_t)(offs[nsel] > 0 ? offs[nsel] : 1) * sizeof(uint16_t));
    for (int64_t k = 0; k < nsel; k++) {
        memcpy(jj + offs[k], lists[k].j, (size_t)lists[k].count * sizeof(uint32_t));
        memcpy(mm + offs[k], lists[k].mask, (size_t)lists[k].count * sizeof(uint16_t));
        free(lists[k].j);
        free(lists[k].mask);
    }
    free(lists);
    *out_offs = offs;
    *out_j = jj;
    *out_mask = mm;
    return 0;
}

void orc_free(void *p) { free(p); }

/* ------------------------------------------------------------------------- */
/* Nibble encoding (Sec. II-B, Tables I and II; layout Sec. II-C)            */
/* ------------------------------------------------------------------------- */

/* Number of hexadecimal digits of v >= 1. */
static int nibbles_of(uint32_t v)
{
    int k = 0;
    while (v) {
        k++;
        v >>= 4;
    }
    return k;
}

/* One block of `count` (<= w) difference values, in symbols:
 *   bits[k]  = 1 iff v_k != 1 (Table I: the bitmask marks the non-one values)
 *   info     = one nibble per non-one value, in order: v + 6 for v in [2, 9],
 *              otherwise (number of data nibbles) - 1
 *   data     = for every value above 9, its hexadecimal digits, most
 *              significant first, in order.
 * Returns 0, or -1 if a value is 0 (a sorted unique list never has one). */
int orc_encode_block_symbols(const uint32_t *v, int count, uint8_t *bits, uint8_t *info, int *ninfo,
                             uint8_t *data, int *ndata)
{
    int ni = 0, nd = 0;
    for (int k = 0; k < count; k++) {
        uint32_t val = v[k];
        if (val == 0) return -1;
        if (val == 1) {
            bits[k] = 0;
            continue;
        }
        bits[k] = 1;
        if (val <= 9) {
            info[ni++] = (uint8_t)(val + 6);
        } else {
            int nn = nibbles_of(val);
            info[ni++] = (uint8_t)(nn - 1);
            for (int d = nn - 1; d >= 0; d--) data[nd++] = (uint8_t)((val >> (4 * d)) & 0xFu);
        }
    }
    *ninfo = ni;
    *ndata = nd;
    return 0;
}

/* Size in 4-byte words of one super-cluster's stream.
 *   nsub = 64 / cs i-clusters; mask bytes per entry = 2 if nsub == 16 else 1.
 *   mask area: n_j mask entries, padded to 4 bytes.
 *   uncompressed: n_j u32 j-cluster indices.
 *   compressed: per block of 64 differences (first difference taken from -1):
 *     8-byte bitmask (bit k = lane k), then the info nibbles and the data
 *     nibbles as one nibble stream (nibble t in byte t/2, low half first),
 *     padded to 4 bytes. */
static int64_t mask_bytes_per_entry(int cs) { return (64 / cs == 16) ? 2 : 1; }

/* The index stream of a list: raw u32 indices, or the differences (from -1)
 * in nibble segments of up to 64 values. */
static int64_t encode_values(int64_t nj, const uint32_t *j, int compress, uint32_t *out /* may be NULL */)
{
    int64_t w = 0;
    if (!compress) {
        if (out)
            for (int64_t k = 0; k < nj; k++) out[k] = j[k];
        return nj;
    }
    uint32_t v[64];
    uint8_t bits[64], info[64], data[64 * 8];
    for (int64_t b0 = 0; b0 < nj; b0 += 64) {
        int cnt = (int)(nj - b0 < 64 ? nj - b0 : 64);
        for (int k = 0; k < cnt; k++) {
            int64_t idx = b0 + k;
            uint32_t prev = idx == 0 ? 0xFFFFFFFFu : j[idx - 1]; /* j_{-1} = -1 */
            v[k] = j[idx] - prev;
        }
        int ni, nd;
        if (orc_encode_block_symbols(v, cnt, bits, info, &ni, data, &nd) != 0) return -1;
        int64_t nib = ni + nd;
        int64_t seg_words = 2 + (nib + 7) / 8;
        if (out) {
            uint64_t m = 0;
            for (int k = 0; k < cnt; k++) m |= (uint64_t)bits[k] << k;
            uint32_t *seg = out + w;
            memset(seg, 0, (size_t)seg_words * 4);
            seg[0] = (uint32_t)(m & 0xFFFFFFFFu);
            seg[1] = (uint32_t)(m >> 32);
            uint8_t *stream = (uint8_t *)(seg + 2);
            for (int64_t t = 0; t < nib; t++) {
                uint8_t nbl = t < ni ? info[t] : data[t - ni];
                stream[t / 2] |= (uint8_t)(nbl << (4 * (t % 2)));
            }
        }
        w += seg_words;
    }
    return w;
}

int64_t orc_encode_sc(int64_t nj, const uint32_t *j, const uint16_t *mask, int cs, int compress,
                      uint32_t *out /* may be NULL to size */)
{
    int64_t mb = mask_bytes_per_entry(cs);
    int64_t mwords = (nj * mb + 3) / 4;
    if (out) {
        memset(out, 0, (size_t)mwords * 4);
        uint8_t *mbytes = (uint8_t *)out;
        for (int64_t k = 0; k < nj; k++) {
            if (mb == 2) {
                mbytes[2 * k] = (uint8_t)(mask[k] & 0xFF);
                mbytes[2 * k + 1] = (uint8_t)(mask[k] >> 8);
            } else {
                mbytes[k] = (uint8_t)mask[k];
            }
        }
    }
    int64_t vw = encode_values(nj, j, compress, out ? out + mwords : NULL);
    return vw < 0 ? -1 : mwords + vw;
}

/* One row of the 1x1 list (the combination of the compression with a full
 * neighbour list that the paper names as future work, Sec. V): particle i's
 * ascending neighbour indices, encoded as the index stream of a super-cluster
 * list without masks. */
int64_t orc_encode_row(int64_t nj, const uint32_t *j, int compress, uint32_t *out /* may be NULL to size */)
{
    return encode_values(nj, j, compress, out);
}

/* Inverse of orc_encode_sc. Returns words consumed, or -1 on a malformed
 * stream. */
static int64_t decode_values(const uint32_t *in, int64_t nj, int compress, uint32_t *j)
{
    if (!compress) {
        for (int64_t k = 0; k < nj; k++) j[k] = in[k];
        return nj;
    }
    int64_t w = 0;
    uint32_t prev = 0xFFFFFFFFu;
    for (int64_t b0 = 0; b0 < nj; b0 += 64) {
        int cnt = (int)(nj - b0 < 64 ? nj - b0 : 64);
        const uint32_t *seg = in + w;
        uint64_t m = (uint64_t)seg[0] | ((uint64_t)seg[1] << 32);
        const uint8_t *stream = (const uint8_t *)(seg + 2);
        int ni = 0;
        for (int k = 0; k < cnt; k++) ni += (int)((m >> k) & 1u);
        int64_t ti = 0, td = ni;
        for (int k = 0; k < cnt; k++) {
            uint32_t val = 1;
            if ((m >> k) & 1u) {
                uint32_t inf = (stream[ti / 2] >> (4 * (ti % 2))) & 0xFu;
                ti++;
                if (inf >= 8) {
                    val = inf - 6;
                } else {
                    val = 0;
                    for (uint32_t d = 0; d <= inf; d++) {
                        val = (val << 4) | ((stream[td / 2] >> (4 * (td % 2))) & 0xFu);
                        td++;
                    }
                    if (val < 10) return -1;
                }
            }
            prev = prev + val;
            j[b0 + k] = prev;
        }
        w += 2 + (td + 7) / 8;
    }
    return w;
}

int64_t orc_decode_sc(const uint32_t *in, int64_t nj, int cs, int compress, uint32_t *j, uint16_t *mask)
{
    int64_t mb = mask_bytes_per_entry(cs);
    int64_t mwords = (nj * mb + 3) / 4;
    const uint8_t *mbytes = (const uint8_t *)in;
    for (int64_t k = 0; k < nj; k++)
        mask[k] = mb == 2 ? (uint16_t)(mbytes[2 * k] | (mbytes[2 * k + 1] << 8)) : mbytes[k];
    int64_t vw = decode_values(in + mwords, nj, compress, j);
    return vw < 0 ? -1 : mwords + vw;
}

int64_t orc_decode_row(const uint32_t *in, int64_t nj, int compress, uint32_t *j)
{
    return decode_values(in, nj, compress, j);
}

/* ------------------------------------------------------------------------- */
/* SPH density (Sec. II-D, Listing 1) in FP64                                 */
/* ------------------------------------------------------------------------- */

/* M4 cubic spline with compact support h, 3-D normalisation 8/(pi h^3):
 *   W = 8/(pi h^3) * (1 - 6 q^2 + 6 q^3)  for 0 <= q < 1/2
 *     = 8/(pi h^3) * 2 (1 - q)^3          for 1/2 <= q < 1
 *     = 0                                  otherwise, q = r/h. */
double orc_kernel_w(double r, double h)
{
    double q = r / h;
    double norm = 8.0 / (M_PI * h * h * h);
    if (q < 0.5) return norm * (1.0 - 6.0 * q * q + 6.0 * q * q * q);
    if (q < 1.0) {
        double t = 1.0 - q;
        return norm * 2.0 * t * t * t;
    }
    return 0.0;
}

/* rho_i = m_i W(0, h_i) + sum over j != i with d2 < f32(h_i^2) of m_j W(r_ij, h_i),
 * r_ij from the exact FP64 differences of the FP32 coordinates (minimum
 * images on periodic axes). The set of j is decided by the same FP32 test as
 * the pair set. nnb_i = size of that set. m == NULL means unit masses. */
void orc_density(int64_t n, const float *x, const float *y, const float *z, const float *h, const float *m,
                 int use_grid, double *rho, int32_t *nnb, const float *period)
{
    orc_grid g;
    grid_init(&g, period);
    if (use_grid) grid_build(&g, n, x, y, z, h);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; i++) {
        double mi = m ? (double)m[i] : 1.0;
        double acc = mi * orc_kernel_w(0.0, (double)h[i]);
        int32_t cnt = 0;
        int64_t cells[27];
        int nc = candidate_ranges(&g, use_grid, n, x[i], y[i], z[i], cells);
        for (int t = 0; t < nc; t++) {
            int64_t k0, k1;
            range_of(&g, n, cells[t], &k0, &k1);
            for (int64_t k = k0; k < k1; k++) {
                int64_t j = cells[t] < 0 ? k : g.idx[k];
                if (j == i) continue;
                if (!orc_in_own_radius(g.per, x[i], y[i], z[i], h[i], x[j], y[j], z[j])) continue;
                double dx = orc_diff64(x[j], x[i], g.per[0]);
                double dy = orc_diff64(y[j], y[i], g.per[1]);
                double dz = orc_diff64(z[j], z[i], g.per[2]);
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                double mj = m ? (double)m[j] : 1.0;
                acc += mj * orc_kernel_w(r, (double)h[i]);
                cnt++;
            }
        }
        rho[i] = acc;
        if (nnb) nnb[i] = cnt;
    }
    if (use_grid) grid_free(&g);
}

/* ------------------------------------------------------------------------- */
/* Lennard-Jones 12/6 + Coulomb pair forces (Sec. III, Lennard-Jones benchmark) */
/* ------------------------------------------------------------------------- */

/* The benchmark pass of Sec. III: every pair closer than the interaction
 * cutoff r_c (fewer than the list cutoff, the Verlet buffer) feels the 12/6
 * Lennard-Jones force plus the Coulomb force of the two charges. Which pairs
 * interact is decided by the same FP32 test as everything else,
 * d2 < f32(r_c^2); the force of an accepted pair is evaluated in FP64 from the
 * exact differences of the FP32 coordinates:
 *   U(r) = 4 eps ((sigma/r)^12 - (sigma/r)^6) + k q_i q_j / r
 *   F_i  = sum_j -dU/dr (x_i - x_j)/r
 *        = sum_j [24 eps (2 (sigma/r)^12 - (sigma/r)^6) / r^2 + k q_i q_j / r^3] (x_i - x_j)
 *   E_i  = 1/2 sum_j U(r_ij)   (each pair's energy shared by its two particles)
 * scale_i = sum_j |F_ij| and escale_i = 1/2 sum_j |U(r_ij)| (the sizes of the
 * terms, for rounding-error bounds).
 * q == NULL means no charges. idx (nullable, count nidx) restricts the output
 * to those particles: row t of the outputs is particle idx[t]. Periodic axes
 * as for the pair set (minimum images). */
void orc_lj(int64_t n, const float *x, const float *y, const float *z, const float *q, double eps, double sigma,
            double kc, float rc, int use_grid, const int64_t *idx, int64_t nidx, double *f, double *e,
            double *scale, double *escale, int32_t *nnb, const float *period)
{
    float *hr = (float *)malloc((size_t)(n > 0 ? n : 1) * sizeof(float));
    for (int64_t i = 0; i < n; i++) hr[i] = rc;
    orc_grid g;
    grid_init(&g, period);
    if (use_grid) grid_build(&g, n, x, y, z, hr);
    int64_t rows = idx ? nidx : n;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t t = 0; t < rows; t++) {
        int64_t i = idx ? idx[t] : t;
        double fx = 0.0, fy = 0.0, fz = 0.0, en = 0.0, sc = 0.0, esc = 0.0;
        int32_t cnt = 0;
        int64_t cells[27];
        int nc = candidate_ranges(&g, use_grid, n, x[i], y[i], z[i], cells);
        for (int u = 0; u < nc; u++) {
            int64_t k0, k1;
            range_of(&g, n, cells[u], &k0, &k1);
            for (int64_t k = k0; k < k1; k++) {
                int64_t j = cells[u] < 0 ? k : g.idx[k];
                if (j == i) continue;
                if (!orc_in_own_radius(g.per, x[i], y[i], z[i], rc, x[j], y[j], z[j])) continue;
                double dx = -orc_diff64(x[j], x[i], g.per[0]);
                double dy = -orc_diff64(y[j], y[i], g.per[1]);
                double dz = -orc_diff64(z[j], z[i], g.per[2]);
                double r2 = dx * dx + dy * dy + dz * dz;
                double r = sqrt(r2);
                double sr6 = pow(sigma / r, 6.0);
                double qq = q ? (double)q[i] * (double)q[j] : 0.0;
                /* -dU/dr divided by r */
                double fr = (24.0 * eps * (2.0 * sr6 * sr6 - sr6) + kc * qq / r) / r2;
                fx += fr * dx;
                fy += fr * dy;
                fz += fr * dz;
                double u_ = 4.0 * eps * (sr6 * sr6 - sr6) + kc * qq / r;
                en += 0.5 * u_;
                esc += 0.5 * fabs(u_);
                sc += fabs(fr) * r;
                cnt++;
            }
        }
        f[3 * t] = fx;
        f[3 * t + 1] = fy;
        f[3 * t + 2] = fz;
        if (e) e[t] = en;
        if (scale) scale[t] = sc;
        if (escale) escale[t] = esc;
        if (nnb) nnb[t] = cnt;
    }
    if (use_grid) grid_free(&g);
    free(hr);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following parallel loops (timing at one thread). */
void orc_set_num_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}
