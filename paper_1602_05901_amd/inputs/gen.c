/*
 * Seeded synthetic reservoir Jacobians (inputs only; see gen.h).
 */
#include "gen.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream)
{
    return mix64(seed ^ (stream * 0xD1B54A32D192ED03ULL + 0x632BE59BD9B4E019ULL));
}

static inline double u_from_key(uint64_t key, uint64_t index)
{
    uint64_t h = mix64(key + (index + 1ULL) * 0x9E3779B97F4A7C15ULL);
    return (double)(h >> 11) * 0x1.0p-53;
}

static inline double n_from_key(uint64_t key, uint64_t index)
{
    double u1 = u_from_key(key, 2 * index);
    double u2 = u_from_key(key, 2 * index + 1);
    return sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586476925 * u2);
}

double gen_uniform(uint64_t seed, uint64_t stream, uint64_t index)
{
    return u_from_key(stream_key(seed, stream), index);
}

double gen_normal(uint64_t seed, uint64_t stream, uint64_t index)
{
    return n_from_key(stream_key(seed, stream), index);
}

void gen_uniform_vec(uint64_t seed, uint64_t stream, int64_t n, double lo, double hi, double *out)
{
    uint64_t key = stream_key(seed, stream);
    for (int64_t i = 0; i < n; ++i) out[i] = lo + (hi - lo) * u_from_key(key, (uint64_t)i);
}

void gen_normal_vec(uint64_t seed, uint64_t stream, int64_t n, double *out)
{
    uint64_t key = stream_key(seed, stream);
    for (int64_t i = 0; i < n; ++i) out[i] = n_from_key(key, (uint64_t)i);
}

static int cfg_ok(const gen_cfg *c)
{
    if (!c || c->nx < 1 || c->ny < 1 || c->nz < 1) return 0;
    if (c->dt <= 0.0) return 0;
    if (c->nsrc != 0 && c->nsrc != 4 && c->nsrc != 8) return 0;
    return 1;
}

int gen_source_cells(const gen_cfg *c, int64_t *cells)
{
    if (!cfg_ok(c)) return -1;
    const int64_t nx = c->nx, ny = c->ny, nz = c->nz;
#define CID(i, j, k) ((int64_t)(k) * nx * ny + (int64_t)(j) * nx + (int64_t)(i))
    int n = 0;
    if (c->nsrc == 4) {
        /* two injectors on the bottom layer, two producers on the top layer */
        cells[n++] = CID(0, 0, 0);
        cells[n++] = CID(nx - 1, ny - 1, 0);
        cells[n++] = CID(nx - 1, 0, nz - 1);
        cells[n++] = CID(0, ny - 1, nz - 1);
    } else if (c->nsrc == 8) {
        for (int kk = 0; kk < 2; ++kk)
            for (int jj = 0; jj < 2; ++jj)
                for (int ii = 0; ii < 2; ++ii)
                    cells[n++] = CID(ii ? nx - 1 : 0, jj ? ny - 1 : 0, kk ? nz - 1 : 0);
    }
#undef CID
    /* de-duplicate (degenerate grids with a dimension of 1) */
    int m = 0;
    for (int a = 0; a < n; ++a) {
        int dup = 0;
        for (int b = 0; b < m; ++b) dup |= (cells[b] == cells[a]);
        if (!dup) cells[m++] = cells[a];
    }
    return m;
}

/* Straight channels of permeability 1e3 in a background of 1: each channel is
 * a band of half-width w/2 (perpendicular to its xy axis, azimuth theta) and
 * thickness h layers; channels are added until >= 25% of cells are channel. */
static void channel_mask(const gen_cfg *c, unsigned char *mask)
{
    const int64_t nx = c->nx, ny = c->ny, nz = c->nz, ncell = nx * ny * nz;
    const uint64_t key = stream_key(c->seed, 5);
    memset(mask, 0, (size_t)ncell);
    int64_t inside = 0;
    const double diag = sqrt((double)nx * nx + (double)ny * ny);
    for (int ch = 0; ch < 4096 && inside * 4 < ncell; ++ch) {
        const uint64_t b = (uint64_t)ch * 8;
        double theta = 3.14159265358979323846 * u_from_key(key, b + 0);
        int w = 4 + (int)(9.0 * u_from_key(key, b + 1));      /* 4..12 */
        int h = 4 + (int)(9.0 * u_from_key(key, b + 2));      /* 4..12 */
        if (h > nz) h = (int)nz;
        int z0 = (int)((double)(nz - h + 1) * u_from_key(key, b + 3));
        double off = (u_from_key(key, b + 4) - 0.5) * diag;
        double ncx = -sin(theta), ncy = cos(theta);
        double cx = 0.5 * (double)nx, cy = 0.5 * (double)ny;
        for (int k = z0; k < z0 + h; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    double dist = ((double)i + 0.5 - cx) * ncx + ((double)j + 0.5 - cy) * ncy - off;
                    if (fabs(dist) <= 0.5 * (double)w) {
                        int64_t C = (int64_t)k * nx * ny + j * nx + i;
                        if (!mask[C]) { mask[C] = 1; ++inside; }
                    }
                }
    }
}

int gen_lnk(const gen_cfg *c, double *lnk)
{
    if (!cfg_ok(c) || !lnk) return -1;
    const int64_t nx = c->nx, ny = c->ny, nz = c->nz, nxy = nx * ny, ncell = nxy * nz;
    const uint64_t k0 = stream_key(c->seed, 0), k1 = stream_key(c->seed, 1);
    switch (c->lnk_kind) {
    case GEN_LNK_IID:
        for (int64_t C = 0; C < ncell; ++C) lnk[C] = c->sigma * n_from_key(k0, (uint64_t)C);
        return 0;
    case GEN_LNK_LAYERED:
        for (int64_t k = 0; k < nz; ++k) {
            double mu = c->sigma_layer * n_from_key(k1, (uint64_t)k);
            for (int64_t r = 0; r < nxy; ++r) {
                int64_t C = k * nxy + r;
                lnk[C] = mu + c->sigma * n_from_key(k0, (uint64_t)C);
            }
        }
        return 0;
    case GEN_LNK_CHANNELS: {
        unsigned char *mask = (unsigned char *)malloc((size_t)ncell);
        if (!mask) return -2;
        channel_mask(c, mask);
        const double lk = log(1.0e3);
        for (int64_t C = 0; C < ncell; ++C)
            lnk[C] = (mask[C] ? lk : 0.0) + c->sigma * n_from_key(k0, (uint64_t)C);
        free(mask);
        return 0;
    }
    default:
        return -1;
    }
}

int gen_blocks(const gen_cfg *c, const double *lnk, double *blocks)
{
    if (!cfg_ok(c) || !lnk || !blocks) return -1;
    const int64_t nx = c->nx, ny = c->ny, nz = c->nz, nxy = nx * ny;
    const uint64_t km = stream_key(c->seed, 2), ka = stream_key(c->seed, 3);
    int64_t src[8];
    int nsrc = gen_source_cells(c, src);
    /* neighbour offsets for slots 0..6 (slot 3 is the cell itself) */
    const int di[7] = {0, 0, -1, 0, 1, 0, 0};
    const int dj[7] = {0, -1, 0, 0, 0, 1, 0};
    const int dk[7] = {-1, 0, 0, 0, 0, 0, 1};
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t C = k * nxy + j * nx + i;
                double *blk = blocks + C * 63;
                memset(blk, 0, 63 * sizeof(double));
                const double ka_ = exp(lnk[C]);
                for (int s = 0; s < 7; ++s) {
                    if (s == 3) continue;
                    const int64_t ii = i + di[s], jj = j + dj[s], kk = k + dk[s];
                    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) continue;
                    const int64_t N = kk * nxy + jj * nx + ii;
                    const double kb = exp(lnk[N]);
                    const double T = 2.0 * ka_ * kb / (ka_ + kb); /* harmonic mean, unit geometry */
                    for (int p = 0; p < 3; ++p)
                        for (int q = 0; q < 3; ++q) {
                            uint64_t idx = (uint64_t)((C * 7 + s) * 9 + 3 * p + q);
                            double m = 0.1 + 0.9 * u_from_key(km, idx) + (p == q ? c->m_shift : 0.0);
                            blk[s * 9 + 3 * p + q] = -T * m;
                        }
                }
                /* diagonal block: minus the sum of the off-diagonal blocks,
                 * plus the accumulation term on its diagonal */
                for (int e = 0; e < 9; ++e) {
                    double acc = 0.0;
                    for (int s = 0; s < 7; ++s)
                        if (s != 3) acc += blk[s * 9 + e];
                    blk[3 * 9 + e] = -acc;
                }
                int is_src = 0;
                for (int q = 0; q < nsrc; ++q) is_src |= (src[q] == C);
                for (int p = 0; p < 3; ++p) {
                    double a = (1.0 + 9.0 * u_from_key(ka, (uint64_t)(3 * C + p))) / c->dt;
                    if (is_src) a += c->src_add;
                    blk[3 * 9 + 4 * p] += a;
                }
            }
    return 0;
}

int gen_poisson(const gen_cfg *c, const double *lnk, double *coef)
{
    if (!cfg_ok(c) || !coef) return -1;
    const int64_t nx = c->nx, ny = c->ny, nz = c->nz;
    static const int OFF[7][3] = {{0, 0, -1}, {0, -1, 0}, {-1, 0, 0}, {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t cc = (k * ny + j) * nx + i;
                const double kc = lnk ? exp(lnk[cc]) : 1.0;
                double *row = coef + 7 * cc;
                double diag = 0.0;
                for (int s = 0; s < 7; ++s) {
                    if (s == 3) continue;
                    const int64_t ii = i + OFF[s][0], jj = j + OFF[s][1], kk = k + OFF[s][2];
                    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) {
                        row[s] = 0.0;
                        diag += kc;                      /* boundary face, u = 0 outside */
                        continue;
                    }
                    const double kn = lnk ? exp(lnk[(kk * ny + jj) * nx + ii]) : 1.0;
                    const double T = lnk ? 2.0 * kc * kn / (kc + kn) : 1.0;
                    row[s] = -T;
                    diag += T;
                }
                row[3] = diag;
            }
    return 0;
}
