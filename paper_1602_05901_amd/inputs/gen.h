/*
 * Seeded synthetic inputs: log-normal permeability fields and the 3x3-block,
 * 7-point cell-centred Jacobians built from them, plus random vectors.
 *
 * This module builds INPUTS only.  It holds none of the solver's arithmetic
 * (no products with the assembled matrix, no factorisation, no Krylov step);
 * both the CPU oracle and the GPU path consume what it writes.
 *
 * Grid and cell numbering follow the paper's Grid section: a structured
 * nx*ny*nz grid, cell (i,j,k) has index C = nx*ny*k + nx*j + i (bottom layer
 * first); interior cells have six neighbours, boundary cells three to five.
 *
 * Random numbers: every draw is a pure function of (seed, stream, index),
 * made with the SplitMix64 output function (Steele, Lea & Flood 2014):
 *   key  = mix64(seed ^ (stream * 0xD1B54A32D192ED03 + 0x632BE59BD9B4E019))
 *   h    = mix64(key + (index + 1) * 0x9E3779B97F4A7C15)
 *   u    = (h >> 11) * 2^-53                       in [0, 1)
 * Normals use Box-Muller on draws 2*index and 2*index+1 of the same stream.
 * Streams: 0 cell ln k noise, 1 layer means, 2 coupling-matrix entries,
 *          3 accumulation terms, 4 x_true, 5 channel geometry, 6 test vectors.
 */
#ifndef RSV_GEN_H
#define RSV_GEN_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { GEN_LNK_IID = 0, GEN_LNK_LAYERED = 1, GEN_LNK_CHANNELS = 2 };

typedef struct gen_cfg {
    int32_t nx, ny, nz;
    int32_t lnk_kind;     /* GEN_LNK_* */
    double  sigma;        /* std of the iid ln k part (channels: std of log noise) */
    double  sigma_layer;  /* std of the per-layer mean (layered only) */
    double  m_shift;      /* shift s of M = s*I + U(0.1,1)^{3x3} per directed block */
    int32_t nsrc;         /* 0, 4 (two injectors + two producers) or 8 (corners) */
    double  src_add;      /* added to the three scalar diagonal entries of a source cell */
    double  dt;           /* accumulation term = U(1,10)/dt */
    uint64_t seed;
} gen_cfg;

/* One counter-based uniform draw in [0,1). */
double gen_uniform(uint64_t seed, uint64_t stream, uint64_t index);
/* One standard normal draw. */
double gen_normal(uint64_t seed, uint64_t stream, uint64_t index);

/* ln k per cell, length nx*ny*nz, natural cell order.  Returns 0 or <0 on bad cfg. */
int gen_lnk(const gen_cfg *cfg, double *lnk);

/* Jacobian blocks, layout double[ncell][7][3][3]; slots ordered by ascending
 * column: 0:-z 1:-y 2:-x 3:diagonal 4:+x 5:+y 6:+z; absent neighbours are zero
 * blocks.  lnk is the field from gen_lnk (or any caller field). */
int gen_blocks(const gen_cfg *cfg, const double *lnk, double *blocks);

/* Scalar 7-point coefficients of a Poisson-type equation -div(k grad u) = f
 * (the paper's Poisson Equation and pressure-system examples), layout
 * double[ncell][7], slots as above.  Face transmissibility T = harmonic mean
 * of the two cells' k = exp(ln k); off-diagonal = -T; diagonal = sum of the
 * cell's face T plus k of the cell for every face on the grid boundary (a
 * homogeneous Dirichlet condition); lnk = NULL means k = 1 (the 7-point
 * Laplacian: diagonal 6, off-diagonals -1). */
int gen_poisson(const gen_cfg *cfg, const double *lnk, double *coef);

/* Fills out[i] = lo + (hi-lo)*u(seed, stream, i) for i < n. */
void gen_uniform_vec(uint64_t seed, uint64_t stream, int64_t n, double lo, double hi, double *out);
/* Fills out[i] = normal(seed, stream, i). */
void gen_normal_vec(uint64_t seed, uint64_t stream, int64_t n, double *out);

/* Source cell list for nsrc in {0,4,8}: writes up to 8 cell indices, returns count. */
int gen_source_cells(const gen_cfg *cfg, int64_t *cells);

#ifdef __cplusplus
}
#endif
#endif
