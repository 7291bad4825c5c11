/*
 * CPU ORACLE -- test infrastructure only.  Plain FP64 loops for the learned
 * residual -> correction network used as a flexible-GMRES preconditioner:
 * a 3-level 3-D U-Net (channels c0/c1/c2, 3x3x3 kernels, zero padding 1,
 * average-pool down, nearest-neighbour up followed by a convolution,
 * additive skips, ReLU, final 1x1x1 linear layer to 3 channels).
 *
 * Layout: channels last, x[v*C + c], voxel v = i + nx*(j + ny*k).
 * Conv weights w[tap][ci][co], tap = (dk+1)*9 + (dj+1)*3 + (di+1), bias b[co].
 * Parameter vector: for layers 0..9 (3x3x3) w then b, then layer 10 (1x1x1)
 * w[ci][co] then b.  Layers: 0 enc1a 4->c0, 1 enc1b c0->c0, 2 enc2a c0->c1,
 * 3 enc2b c1->c1, 4 enc3a c1->c2, 5 enc3b c2->c2, 6 dec2a c2->c1 (on the
 * up-sampled enc3b), 7 dec2b c1->c1, 8 dec1a c1->c0 (on the up-sampled dec2b),
 * 9 dec1b c0->c0, 10 final c0->3.
 *
 * With emulate = 1 every tensor the GPU stores in BF16 (the network input,
 * the ReLU outputs, the pooled tensors, the weights) is rounded to BF16 here
 * too (round to nearest even), and everything else stays FP64.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

static double bf16_round(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f;   /* inf / nan */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

double orc_bf16(double x) { return bf16_round(x); }

/* y = conv3d(x) + b  (no activation) */
void orc_conv3d_fwd(int nx, int ny, int nz, int cin, int cout, const double *x, const double *w,
                    const double *b, double *y)
{
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int64_t v = i + (int64_t)nx * (j + (int64_t)ny * k);
                double *yo = y + v * cout;
                for (int co = 0; co < cout; ++co) yo[co] = b ? b[co] : 0.0;
                for (int dk = -1; dk <= 1; ++dk)
                    for (int dj = -1; dj <= 1; ++dj)
                        for (int di = -1; di <= 1; ++di) {
                            const int ii = i + di, jj = j + dj, kk = k + dk;
                            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) continue;
                            const int tap = (dk + 1) * 9 + (dj + 1) * 3 + (di + 1);
                            const double *xi = x + (ii + (int64_t)nx * (jj + (int64_t)ny * kk)) * cin;
                            const double *wt = w + (int64_t)tap * cin * cout;
                            for (int ci = 0; ci < cin; ++ci)
                                for (int co = 0; co < cout; ++co) yo[co] += wt[ci * cout + co] * xi[ci];
                        }
            }
}

/* adjoints of y = conv3d(x) + b: dx (transposed correlation), dw, db; any may be NULL */
void orc_conv3d_bwd(int nx, int ny, int nz, int cin, int cout, const double *x, const double *w,
                    const double *dy, double *dx, double *dw, double *db)
{
    const int64_t V = (int64_t)nx * ny * nz;
    if (dx) memset(dx, 0, (size_t)(V * cin) * sizeof(double));
    if (dw) memset(dw, 0, (size_t)(27 * cin * cout) * sizeof(double));
    if (db) memset(db, 0, (size_t)cout * sizeof(double));
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int64_t v = i + (int64_t)nx * (j + (int64_t)ny * k);
                const double *g = dy + v * cout;
                if (db)
                    for (int co = 0; co < cout; ++co) db[co] += g[co];
                for (int dk = -1; dk <= 1; ++dk)
                    for (int dj = -1; dj <= 1; ++dj)
                        for (int di = -1; di <= 1; ++di) {
                            const int ii = i + di, jj = j + dj, kk = k + dk;
                            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) continue;
                            const int tap = (dk + 1) * 9 + (dj + 1) * 3 + (di + 1);
                            const int64_t u = ii + (int64_t)nx * (jj + (int64_t)ny * kk);
                            const double *wt = w + (int64_t)tap * cin * cout;
                            for (int ci = 0; ci < cin; ++ci)
                                for (int co = 0; co < cout; ++co) {
                                    if (dx) dx[u * cin + ci] += wt[ci * cout + co] * g[co];
                                    if (dw) dw[((int64_t)tap * cin + ci) * cout + co] += x[u * cin + ci] * g[co];
                                }
                        }
            }
}

/* ---------------------------------------------------------------- the network */

typedef struct {
    int c[3];
    int cin[11], cout[11];
    int64_t woff[11], boff[11];
    int64_t np;
} arch_t;

static void arch_init(arch_t *a, int c0, int c1, int c2)
{
    a->c[0] = c0; a->c[1] = c1; a->c[2] = c2;
    const int ci[11] = {4, c0, c0, c1, c1, c2, c2, c1, c1, c0, c0};
    const int co[11] = {c0, c0, c1, c1, c2, c2, c1, c1, c0, c0, 3};
    int64_t off = 0;
    for (int l = 0; l < 11; ++l) {
        a->cin[l] = ci[l];
        a->cout[l] = co[l];
        a->woff[l] = off;
        off += (int64_t)(l < 10 ? 27 : 1) * ci[l] * co[l];
        a->boff[l] = off;
        off += co[l];
    }
    a->np = off;
}

int64_t orc_unet_nparams(int c0, int c1, int c2)
{
    arch_t a;
    arch_init(&a, c0, c1, c2);
    return a.np;
}

static void pool_fwd(int nx, int ny, int nz, int C, const double *x, double *y)
{
    const int mx = nx / 2, my = ny / 2, mz = nz / 2;
    for (int k = 0; k < mz; ++k)
        for (int j = 0; j < my; ++j)
            for (int i = 0; i < mx; ++i) {
                double *yo = y + (i + (int64_t)mx * (j + (int64_t)my * k)) * C;
                for (int c = 0; c < C; ++c) yo[c] = 0.0;
                for (int q = 0; q < 8; ++q) {
                    const int ii = 2 * i + (q & 1), jj = 2 * j + ((q >> 1) & 1), kk = 2 * k + (q >> 2);
                    const double *xi = x + (ii + (int64_t)nx * (jj + (int64_t)ny * kk)) * C;
                    for (int c = 0; c < C; ++c) yo[c] += xi[c];
                }
                for (int c = 0; c < C; ++c) yo[c] *= 0.125;
            }
}

/* adjoint of the average pool: every child gets 1/8 of its parent's gradient */
static void pool_bwd(int nx, int ny, int nz, int C, const double *dy, double *dx)
{
    const int mx = nx / 2, my = ny / 2;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const double *g = dy + ((i / 2) + (int64_t)mx * ((j / 2) + (int64_t)my * (k / 2))) * C;
                double *o = dx + (i + (int64_t)nx * (j + (int64_t)ny * k)) * C;
                for (int c = 0; c < C; ++c) o[c] = 0.125 * g[c];
            }
}

/* nearest up-sampling of a (nx/2,ny/2,nz/2) tensor to (nx,ny,nz) */
static void up_fwd(int nx, int ny, int nz, int C, const double *x, double *y)
{
    const int mx = nx / 2, my = ny / 2;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const double *xi = x + ((i / 2) + (int64_t)mx * ((j / 2) + (int64_t)my * (k / 2))) * C;
                double *o = y + (i + (int64_t)nx * (j + (int64_t)ny * k)) * C;
                for (int c = 0; c < C; ++c) o[c] = xi[c];
            }
}

/* adjoint of nearest up-sampling: parents sum their eight children */
static void up_bwd(int nx, int ny, int nz, int C, const double *dy, double *dx)
{
    const int mx = nx / 2, my = ny / 2, mz = nz / 2;
    memset(dx, 0, (size_t)((int64_t)mx * my * mz * C) * sizeof(double));
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double *o = dx + ((i / 2) + (int64_t)mx * ((j / 2) + (int64_t)my * (k / 2))) * C;
                const double *g = dy + (i + (int64_t)nx * (j + (int64_t)ny * k)) * C;
                for (int c = 0; c < C; ++c) o[c] += g[c];
            }
}

typedef struct {
    int64_t V1, V2, V3;
    double *x0, *a1, *s1, *p1, *a2, *s2, *p2, *a3, *b3, *u3, *d2a, *d2, *u2, *d1a, *d1, *y;
    double *z6, *z8;   /* pre-activation of the skip layers (conv + skip) */
} acts_t;

static void acts_free(acts_t *t)
{
    double **p[] = {&t->x0, &t->a1, &t->s1, &t->p1, &t->a2, &t->s2, &t->p2, &t->a3, &t->b3, &t->u3,
                    &t->d2a, &t->d2, &t->u2, &t->d1a, &t->d1, &t->y, &t->z6, &t->z8};
    for (size_t q = 0; q < sizeof(p) / sizeof(p[0]); ++q) { free(*p[q]); *p[q] = NULL; }
}

static int acts_alloc(acts_t *t, const arch_t *a, int nx, int ny, int nz)
{
    memset(t, 0, sizeof(*t));
    t->V1 = (int64_t)nx * ny * nz;
    t->V2 = t->V1 / 8;
    t->V3 = t->V2 / 8;
    const int c0 = a->c[0], c1 = a->c[1], c2 = a->c[2];
#define AL(f, n) if (!(t->f = (double *)calloc((size_t)(n), sizeof(double)))) { acts_free(t); return -1; }
    AL(x0, t->V1 * 4) AL(a1, t->V1 * c0) AL(s1, t->V1 * c0) AL(p1, t->V2 * c0) AL(a2, t->V2 * c1)
    AL(s2, t->V2 * c1) AL(p2, t->V3 * c1) AL(a3, t->V3 * c2) AL(b3, t->V3 * c2) AL(u3, t->V2 * c2)
    AL(d2a, t->V2 * c1) AL(d2, t->V2 * c1) AL(u2, t->V1 * c1) AL(d1a, t->V1 * c0) AL(d1, t->V1 * c0)
    AL(y, t->V1 * 3) AL(z6, t->V2 * c1) AL(z8, t->V1 * c0)
#undef AL
    return 0;
}

static void relu_round(double *x, int64_t n, int emulate)
{
    for (int64_t q = 0; q < n; ++q) {
        double v = x[q] > 0.0 ? x[q] : 0.0;
        x[q] = emulate ? bf16_round(v) : v;
    }
}

static void round_all(double *x, int64_t n, int emulate)
{
    if (!emulate) return;
    for (int64_t q = 0; q < n; ++q) x[q] = bf16_round(x[q]);
}

/* forward pass keeping every intermediate (params already BF16-rounded when emulating) */
static void unet_forward(const arch_t *a, int nx, int ny, int nz, const double *P, acts_t *t, int emulate)
{
    const int c0 = a->c[0], c1 = a->c[1], c2 = a->c[2];
    const int mx = nx / 2, my = ny / 2, mz = nz / 2, lx = nx / 4, ly = ny / 4, lz = nz / 4;
#define W(l) (P + a->woff[l])
#define B(l) (P + a->boff[l])
    round_all(t->x0, t->V1 * 4, emulate);
    orc_conv3d_fwd(nx, ny, nz, 4, c0, t->x0, W(0), B(0), t->a1); relu_round(t->a1, t->V1 * c0, emulate);
    orc_conv3d_fwd(nx, ny, nz, c0, c0, t->a1, W(1), B(1), t->s1); relu_round(t->s1, t->V1 * c0, emulate);
    pool_fwd(nx, ny, nz, c0, t->s1, t->p1); round_all(t->p1, t->V2 * c0, emulate);
    orc_conv3d_fwd(mx, my, mz, c0, c1, t->p1, W(2), B(2), t->a2); relu_round(t->a2, t->V2 * c1, emulate);
    orc_conv3d_fwd(mx, my, mz, c1, c1, t->a2, W(3), B(3), t->s2); relu_round(t->s2, t->V2 * c1, emulate);
    pool_fwd(mx, my, mz, c1, t->s2, t->p2); round_all(t->p2, t->V3 * c1, emulate);
    orc_conv3d_fwd(lx, ly, lz, c1, c2, t->p2, W(4), B(4), t->a3); relu_round(t->a3, t->V3 * c2, emulate);
    orc_conv3d_fwd(lx, ly, lz, c2, c2, t->a3, W(5), B(5), t->b3); relu_round(t->b3, t->V3 * c2, emulate);
    up_fwd(mx, my, mz, c2, t->b3, t->u3);
    orc_conv3d_fwd(mx, my, mz, c2, c1, t->u3, W(6), B(6), t->z6);
    for (int64_t q = 0; q < t->V2 * c1; ++q) { t->z6[q] += t->s2[q]; t->d2a[q] = t->z6[q]; }
    relu_round(t->d2a, t->V2 * c1, emulate);
    orc_conv3d_fwd(mx, my, mz, c1, c1, t->d2a, W(7), B(7), t->d2); relu_round(t->d2, t->V2 * c1, emulate);
    up_fwd(nx, ny, nz, c1, t->d2, t->u2);
    orc_conv3d_fwd(nx, ny, nz, c1, c0, t->u2, W(8), B(8), t->z8);
    for (int64_t q = 0; q < t->V1 * c0; ++q) { t->z8[q] += t->s1[q]; t->d1a[q] = t->z8[q]; }
    relu_round(t->d1a, t->V1 * c0, emulate);
    orc_conv3d_fwd(nx, ny, nz, c0, c0, t->d1a, W(9), B(9), t->d1); relu_round(t->d1, t->V1 * c0, emulate);
    /* final 1x1x1 linear layer */
    const double *w10 = W(10), *b10 = B(10);
    for (int64_t v = 0; v < t->V1; ++v)
        for (int co = 0; co < 3; ++co) {
            double s = b10[co];
            for (int ci = 0; ci < c0; ++ci) s += w10[ci * 3 + co] * t->d1[v * c0 + ci];
            t->y[v * 3 + co] = s;
        }
#undef W
#undef B
}

static double *params_copy(const arch_t *a, const double *P, int emulate)
{
    double *Q = (double *)malloc((size_t)a->np * sizeof(double));
    if (!Q) return NULL;
    for (int64_t q = 0; q < a->np; ++q) Q[q] = emulate ? bf16_round(P[q]) : P[q];
    return Q;
}

static int dims_ok(int nx, int ny, int nz) { return nx > 0 && ny > 0 && nz > 0 && nx % 4 == 0 && ny % 4 == 0 && nz % 4 == 0; }

int orc_unet_forward(int c0, int c1, int c2, int nx, int ny, int nz, const double *params, const double *x0,
                     double *y, int emulate)
{
    if (!dims_ok(nx, ny, nz)) return ORC_ERR_ARG;
    arch_t a;
    arch_init(&a, c0, c1, c2);
    acts_t t;
    if (acts_alloc(&t, &a, nx, ny, nz)) return ORC_ERR_OOM;
    double *P = params_copy(&a, params, emulate);
    if (!P) { acts_free(&t); return ORC_ERR_OOM; }
    memcpy(t.x0, x0, (size_t)(t.V1 * 4) * sizeof(double));
    unet_forward(&a, nx, ny, nz, P, &t, emulate);
    memcpy(y, t.y, (size_t)(t.V1 * 3) * sizeof(double));
    free(P);
    acts_free(&t);
    return ORC_OK;
}

/* gradient through ReLU: g <- g where the activation is positive, else 0 */
static void relu_bwd(double *g, const double *act, int64_t n)
{
    for (int64_t q = 0; q < n; ++q)
        if (!(act[q] > 0.0)) g[q] = 0.0;
}

/* Loss L = ||y - t||^2 / ||t||^2 for one sample and its gradient with respect
 * to every parameter (exact adjoint of the forward pass, FP64). */
int orc_unet_loss_grad(int c0, int c1, int c2, int nx, int ny, int nz, const double *params, const double *x0,
                       const double *target, double *grad, double *loss, int emulate)
{
    if (!dims_ok(nx, ny, nz)) return ORC_ERR_ARG;
    arch_t a;
    arch_init(&a, c0, c1, c2);
    acts_t t;
    if (acts_alloc(&t, &a, nx, ny, nz)) return ORC_ERR_OOM;
    double *P = params_copy(&a, params, emulate);
    const int64_t V1 = t.V1, V2 = t.V2, V3 = t.V3;
    const int mx = nx / 2, my = ny / 2, mz = nz / 2, lx = nx / 4, ly = ny / 4, lz = nz / 4;
    const int64_t big = V1 * (c0 > c1 ? (c0 > c2 ? c0 : c2) : (c1 > c2 ? c1 : c2)) + V1 * 4;
    double *g1 = (double *)calloc((size_t)big, sizeof(double));
    double *g2 = (double *)calloc((size_t)big, sizeof(double));
    double *gs1 = (double *)calloc((size_t)(V1 * c0), sizeof(double));
    double *gs2 = (double *)calloc((size_t)(V2 * c1), sizeof(double));
    if (!P || !g1 || !g2 || !gs1 || !gs2) {
        free(P); free(g1); free(g2); free(gs1); free(gs2); acts_free(&t);
        return ORC_ERR_OOM;
    }
    memcpy(t.x0, x0, (size_t)(V1 * 4) * sizeof(double));
    unet_forward(&a, nx, ny, nz, P, &t, emulate);
    double tt = 0.0, ee = 0.0;
    for (int64_t q = 0; q < V1 * 3; ++q) {
        tt += target[q] * target[q];
        ee += (t.y[q] - target[q]) * (t.y[q] - target[q]);
    }
    *loss = ee / tt;
    memset(grad, 0, (size_t)a.np * sizeof(double));
#define W(l) (P + a.woff[l])
#define GW(l) (grad + a.woff[l])
#define GB(l) (grad + a.boff[l])
    /* dL/dy */
    double *gy = g2;
    for (int64_t q = 0; q < V1 * 3; ++q) gy[q] = 2.0 * (t.y[q] - target[q]) / tt;
    /* final layer */
    double *gd1 = g1;
    for (int64_t v = 0; v < V1; ++v)
        for (int ci = 0; ci < c0; ++ci) {
            double s = 0.0;
            for (int co = 0; co < 3; ++co) {
                s += W(10)[ci * 3 + co] * gy[v * 3 + co];
                GW(10)[ci * 3 + co] += t.d1[v * c0 + ci] * gy[v * 3 + co];
            }
            gd1[v * c0 + ci] = s;
        }
    for (int64_t v = 0; v < V1; ++v)
        for (int co = 0; co < 3; ++co) GB(10)[co] += gy[v * 3 + co];
    /* dec1b */
    relu_bwd(gd1, t.d1, V1 * c0);
    double *gd1a = g2;
    orc_conv3d_bwd(nx, ny, nz, c0, c0, t.d1a, W(9), gd1, gd1a, GW(9), GB(9));
    /* dec1a: d1a = relu(conv8(up(d2)) + s1) */
    relu_bwd(gd1a, t.d1a, V1 * c0);
    for (int64_t q = 0; q < V1 * c0; ++q) gs1[q] = gd1a[q];
    double *gu2 = g1;
    orc_conv3d_bwd(nx, ny, nz, c1, c0, t.u2, W(8), gd1a, gu2, GW(8), GB(8));
    double *gd2 = g2;
    up_bwd(nx, ny, nz, c1, gu2, gd2);
    /* dec2b */
    relu_bwd(gd2, t.d2, V2 * c1);
    double *gd2a = g1;
    orc_conv3d_bwd(mx, my, mz, c1, c1, t.d2a, W(7), gd2, gd2a, GW(7), GB(7));
    /* dec2a: d2a = relu(conv6(up(b3)) + s2) */
    relu_bwd(gd2a, t.d2a, V2 * c1);
    for (int64_t q = 0; q < V2 * c1; ++q) gs2[q] = gd2a[q];
    double *gu3 = g2;
    orc_conv3d_bwd(mx, my, mz, c2, c1, t.u3, W(6), gd2a, gu3, GW(6), GB(6));
    double *gb3 = g1;
    up_bwd(mx, my, mz, c2, gu3, gb3);
    /* enc3b, enc3a */
    relu_bwd(gb3, t.b3, V3 * c2);
    double *ga3 = g2;
    orc_conv3d_bwd(lx, ly, lz, c2, c2, t.a3, W(5), gb3, ga3, GW(5), GB(5));
    relu_bwd(ga3, t.a3, V3 * c2);
    double *gp2 = g1;
    orc_conv3d_bwd(lx, ly, lz, c1, c2, t.p2, W(4), ga3, gp2, GW(4), GB(4));
    /* pool 2 */
    double *gs2b = g2;
    pool_bwd(mx, my, mz, c1, gp2, gs2b);
    for (int64_t q = 0; q < V2 * c1; ++q) gs2b[q] += gs2[q];
    /* enc2b, enc2a */
    relu_bwd(gs2b, t.s2, V2 * c1);
    double *ga2 = g1;
    orc_conv3d_bwd(mx, my, mz, c1, c1, t.a2, W(3), gs2b, ga2, GW(3), GB(3));
    relu_bwd(ga2, t.a2, V2 * c1);
    double *gp1 = g2;
    orc_conv3d_bwd(mx, my, mz, c0, c1, t.p1, W(2), ga2, gp1, GW(2), GB(2));
    /* pool 1 */
    double *gs1b = g1;
    pool_bwd(nx, ny, nz, c0, gp1, gs1b);
    for (int64_t q = 0; q < V1 * c0; ++q) gs1b[q] += gs1[q];
    /* enc1b, enc1a */
    relu_bwd(gs1b, t.s1, V1 * c0);
    double *ga1 = g2;
    orc_conv3d_bwd(nx, ny, nz, c0, c0, t.a1, W(1), gs1b, ga1, GW(1), GB(1));
    relu_bwd(ga1, t.a1, V1 * c0);
    orc_conv3d_bwd(nx, ny, nz, 4, c0, t.x0, W(0), ga1, NULL, GW(0), GB(0));
#undef W
#undef GW
#undef GB
    free(P); free(g1); free(g2); free(gs1); free(gs2);
    acts_free(&t);
    return ORC_OK;
}

/* Network input from a residual: channels 0..2 = r / s with s = rms(r) over
 * all 3*ncell entries, channel 3 = standardised ln k; returns s. */
double orc_unet_prepare(int nx, int ny, int nz, const double *r, const double *lnk, double *x0)
{
    const int64_t V = (int64_t)nx * ny * nz;
    double ss = 0.0, m = 0.0, m2 = 0.0;
    for (int64_t q = 0; q < 3 * V; ++q) ss += r[q] * r[q];
    for (int64_t v = 0; v < V; ++v) m += lnk[v];
    m /= (double)V;
    for (int64_t v = 0; v < V; ++v) m2 += (lnk[v] - m) * (lnk[v] - m);
    const double sd = sqrt(m2 / (double)V);
    const double s = sqrt(ss / (double)(3 * V));
    for (int64_t v = 0; v < V; ++v) {
        for (int p = 0; p < 3; ++p) x0[v * 4 + p] = (s > 0.0) ? r[3 * v + p] / s : 0.0;
        x0[v * 4 + 3] = (sd > 0.0) ? (lnk[v] - m) / sd : 0.0;
    }
    return s;
}

/* One Adam step (Kingma & Ba 2015), beta1 0.9, beta2 0.999, eps 1e-8, step t >= 1. */
void orc_adam(int64_t n, double *p, const double *g, double *m, double *v, int64_t t, double lr)
{
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t q = 0; q < n; ++q) {
        m[q] = b1 * m[q] + (1.0 - b1) * g[q];
        v[q] = b2 * v[q] + (1.0 - b2) * g[q] * g[q];
        p[q] -= lr * (m[q] / c1) / (sqrt(v[q] / c2) + eps);
    }
}
