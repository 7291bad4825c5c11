/*
 * CPU ORACLE -- test infrastructure only.  Plain serial C for the Hilbert
 * space-filling-curve partition of a structured grid (Space-filling
 * Partitioning Method section): cell centroids are mapped linearly into
 * [0,1)^3, each is given its position along a 3-D Hilbert curve, and the
 * cells, in curve order, are cut into nparts runs of equal size (Algorithm
 * "Space-filling curve method").  The partition-quality measures follow the
 * Partition Quality subsection.  Shares no code with the GPU library.
 *
 * The curve is the table-driven one of the paper's Hilbert order figures:
 * 24 orientation states; at each level the three coordinate bits of that
 * level (x weight 4, y weight 2, z weight 1) select, through the ordering
 * table, the base-8 digit of the key and, through the orientation table, the
 * state of the next level.  The two tables below are the paper's (ordering
 * table and orientation table figures), one row of eight per state; the pins
 * check that they give a curve through every lattice point whose consecutive
 * points are face neighbours.
 */
#include "oracle.h"
#include <stdlib.h>
#include <string.h>

static const unsigned char ORDER[24][8] = {
    {0, 7, 3, 4, 1, 6, 2, 5},
    {0, 1, 3, 2, 7, 6, 4, 5},
    {0, 3, 7, 4, 1, 2, 6, 5},
    {2, 3, 5, 4, 1, 0, 6, 7},
    {4, 5, 3, 2, 7, 6, 0, 1},
    {4, 7, 3, 0, 5, 6, 2, 1},
    {6, 7, 5, 4, 1, 0, 2, 3},
    {0, 1, 7, 6, 3, 2, 4, 5},
    {2, 1, 5, 6, 3, 0, 4, 7},
    {6, 1, 5, 2, 7, 0, 4, 3},
    {0, 7, 1, 6, 3, 4, 2, 5},
    {2, 1, 3, 0, 5, 6, 4, 7},
    {4, 7, 5, 6, 3, 0, 2, 1},
    {4, 5, 7, 6, 3, 2, 0, 1},
    {6, 1, 7, 0, 5, 2, 4, 3},
    {0, 3, 1, 2, 7, 4, 6, 5},
    {2, 3, 1, 0, 5, 4, 6, 7},
    {6, 7, 1, 0, 5, 4, 2, 3},
    {2, 5, 1, 6, 3, 4, 0, 7},
    {4, 3, 7, 0, 5, 2, 6, 1},
    {4, 3, 5, 2, 7, 0, 6, 1},
    {6, 5, 1, 2, 7, 4, 0, 3},
    {2, 5, 3, 4, 1, 6, 0, 7},
    {6, 5, 7, 4, 1, 2, 0, 3},
};

static const unsigned char NEXT_STATE[24][8] = {
    {1, 6, 3, 4, 2, 5, 0, 0},
    {0, 7, 8, 1, 9, 4, 5, 1},
    {15, 22, 23, 20, 0, 2, 19, 2},
    {3, 23, 3, 15, 6, 20, 16, 22},
    {11, 4, 12, 4, 20, 1, 22, 13},
    {22, 12, 20, 11, 5, 0, 5, 19},
    {17, 0, 6, 21, 3, 9, 6, 2},
    {10, 1, 14, 13, 11, 7, 12, 7},
    {8, 9, 8, 18, 14, 12, 10, 11},
    {21, 8, 9, 9, 1, 6, 17, 7},
    {7, 17, 15, 12, 16, 13, 10, 10},
    {11, 14, 9, 5, 11, 22, 0, 8},
    {18, 5, 12, 10, 19, 8, 12, 20},
    {8, 13, 19, 7, 5, 13, 18, 4},
    {23, 11, 7, 17, 14, 14, 6, 1},
    {2, 18, 10, 15, 21, 19, 20, 15},
    {16, 21, 17, 19, 16, 2, 3, 18},
    {6, 10, 16, 14, 17, 23, 17, 15},
    {18, 18, 21, 8, 17, 7, 13, 16},
    {3, 4, 13, 16, 19, 19, 2, 5},
    {16, 13, 20, 20, 4, 3, 15, 12},
    {9, 21, 18, 21, 15, 14, 23, 10},
    {22, 22, 6, 1, 23, 11, 4, 3},
    {14, 23, 2, 9, 22, 23, 21, 0},
};

/* Integer coordinate of a point of [0,1]: the paper's scaling by 2^32 - 1
 * with truncation, in FP64. */
static uint32_t coord_u32(double c)
{
    return (uint32_t)(c * 4294967295.0);
}

int orc_hsfc_key3(const double *c, int32_t levels, uint64_t *key)
{
    if (!c || !key || levels < 1 || levels > 21) return ORC_ERR_ARG;
    for (int a = 0; a < 3; ++a)
        if (!(c[a] >= 0.0 && c[a] <= 1.0)) return ORC_ERR_ARG;
    const uint32_t u[3] = {coord_u32(c[0]), coord_u32(c[1]), coord_u32(c[2])};
    unsigned state = 0;
    uint64_t k = 0;
    for (int l = 0; l < levels; ++l) {
        const int bit = 31 - l;   /* level l reads bit 31 - l of each coordinate */
        const unsigned oct = (((u[0] >> bit) & 1u) << 2) | (((u[1] >> bit) & 1u) << 1) | ((u[2] >> bit) & 1u);
        k = (k << 3) | ORDER[state][oct];
        state = NEXT_STATE[state][oct];
    }
    *key = k;
    return ORC_OK;
}

/* centroid of cell (i, j, k) scaled by the largest extent, so cells stay cubes */
static void centroid(int nx, int ny, int nz, int i, int j, int k, double *c)
{
    int L = nx;
    if (ny > L) L = ny;
    if (nz > L) L = nz;
    c[0] = ((double)i + 0.5) / (double)L;
    c[1] = ((double)j + 0.5) / (double)L;
    c[2] = ((double)k + 0.5) / (double)L;
}

int orc_hsfc_grid_keys(int32_t nx, int32_t ny, int32_t nz, int32_t levels, uint64_t *keys)
{
    if (nx < 1 || ny < 1 || nz < 1 || !keys) return ORC_ERR_ARG;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double c[3];
                centroid(nx, ny, nz, i, j, k, c);
                int rc = orc_hsfc_key3(c, levels, keys + i + (int64_t)nx * (j + (int64_t)ny * k));
                if (rc != ORC_OK) return rc;
            }
    return ORC_OK;
}

typedef struct { uint64_t key; int64_t idx; } kv_t;

static int kv_cmp(const void *a, const void *b)
{
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Cells in increasing key order (equal keys by index) cut into nparts runs:
 * the cell of rank r goes to part floor(r * nparts / n), so part sizes differ
 * by at most one. */
int orc_hsfc_partition(int64_t n, const uint64_t *keys, int32_t nparts, int32_t *part)
{
    if (n < 0 || !keys || !part || nparts < 1) return ORC_ERR_ARG;
    kv_t *v = (kv_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(kv_t));
    if (!v) return ORC_ERR_OOM;
    for (int64_t q = 0; q < n; ++q) { v[q].key = keys[q]; v[q].idx = q; }
    qsort(v, (size_t)n, sizeof(kv_t), kv_cmp);
    for (int64_t r = 0; r < n; ++r) part[v[r].idx] = (int32_t)((r * (int64_t)nparts) / n);
    free(v);
    return ORC_OK;
}

/* Partition quality of a structured-grid partition (faces between
 * face-neighbour cells and on the grid boundary).  Per part i: size |G_i|,
 * f_i = faces of its cells counted once, b_i = those faces shared with a
 * cell of another part, c_i = number of other parts it shares a face with.
 * q[0] load imbalance N_p max|G_i| / sum|G_i|; q[1] max_i b_i/f_i; q[2]
 * sum b_i / (sum f_i - sum b_i); q[3] the average (1/N_p) sum_i b_i/f_i;
 * q[4] max_i c_i.  per_part (nullable): [nparts][4] = |G_i|, f_i, b_i, c_i. */
int orc_partition_quality(int32_t nx, int32_t ny, int32_t nz, const int32_t *part, int32_t nparts, double *q,
                          int64_t *per_part)
{
    if (nx < 1 || ny < 1 || nz < 1 || !part || nparts < 1 || !q) return ORC_ERR_ARG;
    const int64_t n = (int64_t)nx * ny * nz;
    int64_t *sz = (int64_t *)calloc((size_t)nparts, sizeof(int64_t));
    int64_t *f = (int64_t *)calloc((size_t)nparts, sizeof(int64_t));
    int64_t *b = (int64_t *)calloc((size_t)nparts, sizeof(int64_t));
    unsigned char *adj = (unsigned char *)calloc((size_t)nparts * (size_t)nparts, 1);
    if (!sz || !f || !b || !adj) { free(sz); free(f); free(b); free(adj); return ORC_ERR_OOM; }
    for (int64_t c = 0; c < n; ++c)
        if (part[c] < 0 || part[c] >= nparts) { free(sz); free(f); free(b); free(adj); return ORC_ERR_ARG; }
    static const int D[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int64_t c = i + (int64_t)nx * (j + (int64_t)ny * k);
                const int p = part[c];
                sz[p]++;
                for (int s = 0; s < 6; ++s) {
                    const int ii = i + D[s][0], jj = j + D[s][1], kk = k + D[s][2];
                    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) { f[p]++; continue; }
                    const int64_t m = ii + (int64_t)nx * (jj + (int64_t)ny * kk);
                    const int pm = part[m];
                    if (pm != p) { f[p]++; b[p]++; adj[(size_t)p * nparts + pm] = 1; }
                    else if (m > c) f[p]++;   /* a face inside the part, counted once */
                }
            }
    int64_t mx = 0, sf = 0, sb = 0, cmax = 0;
    double rmax = 0.0, ravg = 0.0;
    for (int p = 0; p < nparts; ++p) {
        if (sz[p] > mx) mx = sz[p];
        sf += f[p];
        sb += b[p];
        const double r = f[p] > 0 ? (double)b[p] / (double)f[p] : 0.0;
        if (r > rmax) rmax = r;
        ravg += r;
        int64_t cp = 0;
        for (int o = 0; o < nparts; ++o) cp += adj[(size_t)p * nparts + o];
        if (cp > cmax) cmax = cp;
        if (per_part) {
            per_part[4 * p] = sz[p];
            per_part[4 * p + 1] = f[p];
            per_part[4 * p + 2] = b[p];
            per_part[4 * p + 3] = cp;
        }
    }
    q[0] = (double)nparts * (double)mx / (double)n;
    q[1] = rmax;
    q[2] = (sf - sb) > 0 ? (double)sb / (double)(sf - sb) : 0.0;
    q[3] = ravg / (double)nparts;
    q[4] = (double)cmax;
    free(sz); free(f); free(b); free(adj);
    return ORC_OK;
}
