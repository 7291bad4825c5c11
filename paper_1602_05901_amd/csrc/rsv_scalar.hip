// Scalar (one unknown per cell) 7-point systems, for the paper's Poisson
// Equation example: GMRES(30) with restricted additive Schwarz, overlap one,
// ILU(0) on every subdomain (Restricted Additive Schwarz Method subsection,
// RAS default parameters; Poisson Equation example).
//
// Storage: the seven coefficients of every row as seven row-ordered arrays
// coef[s][row] (slots -z,-y,-x,D,+x,+y,+z by cell direction), vectors in row
// order; the product is one thread per row with the residual, norm and dot
// epilogues of the block product.
//
// RAS: px x py x pz boxes (the first n mod p boxes one cell longer), each
// extended to Omega_s = the cells within graph distance `overlap` of the box
// (L1 distance on the lattice: faces, no edges or corners for overlap 1).
// Every Omega_s cell is an entry of one long list, grouped by subdomain and,
// inside a subdomain, by local hyperplane (i - ex0) + (j - ey0) + (k - ez0),
// ascending cell index inside a plane.  The local ILU(0) in ascending global
// order has no fill on the 7-point graph (two neighbours of a cell are never
// neighbours), so D_c = a_cc - sum_{k lower} a_ck a_kc / D_k and every plane
// depends only on the one before: one workgroup per subdomain walks its
// planes with a barrier between them, for the factorisation and for both
// sweeps of an apply; only the owner of a cell writes its result.
#include "rsv_internal.h"

#include <algorithm>
#include <cmath>
#include <new>
#include <thread>
#include <vector>

namespace {

constexpr int SB = 256;          // product / assembly threads per block
constexpr int RAS_T = 1024;      // threads of a subdomain's workgroup

// row -> cell (inverse of row_of)
__host__ __device__ inline void cell_of_row(const Geo &g, int64_t r, int &i, int &j, int &k)
{
    i = (int)(r % g.nx);
    j = (int)((r / g.nx) % g.ny);
    const int kk = (int)(r / ((int64_t)g.nx * g.ny));
    k = (g.ordering == RSV_TOP_DOWN) ? g.nz - 1 - kk : kk;
}

__device__ inline double sblock_sum(double v, double *lds)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < nw; ++q) s += lds[q];
    return s;
}

__global__ __launch_bounds__(SB) void k_sassemble(Geo g, const double *__restrict__ src, double *__restrict__ coef,
                                                  int32_t *flags)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t r = (int64_t)blockIdx.x * SB + threadIdx.x;
    if (r >= n) return;
    int i, j, k;
    cell_of_row(g, r, i, j, k);
    for (int s = 0; s < 7; ++s) {
        int di, dj, dk;
        dir_off(s, di, dj, dk);
        const bool inside = i + di >= 0 && i + di < g.nx && j + dj >= 0 && j + dj < g.ny && k + dk >= 0 && k + dk < g.nz;
        const double v = src[7 * r + s];
        if (!isfinite(v)) {
            atomicOr(&flags[0], (int32_t)FLAG_NAN);
            atomicMin(&flags[1], (int32_t)r);
        } else if (!inside && v != 0.0) {
            atomicOr(&flags[0], (int32_t)FLAG_PATTERN);
            atomicMin(&flags[1], (int32_t)r);
        }
        coef[s * n + r] = inside ? v : 0.0;
    }
}

template <int MODE>
__global__ __launch_bounds__(SB) void k_sspmv(Geo g, const double *__restrict__ coef, const double *__restrict__ x,
                                              double *__restrict__ y, const double *__restrict__ aux,
                                              double alpha, double beta, double *__restrict__ partials)
{
    __shared__ double lds[SB / 64];
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t r = (int64_t)blockIdx.x * SB + threadIdx.x;
    double r0 = 0.0, r1 = 0.0;
    if (r < n) {
        int i, j, k;
        cell_of_row(g, r, i, j, k);
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < 7; ++s) {
            int di, dj, dk;
            dir_off(s, di, dj, dk);
            const int a = i + di, b = j + dj, c = k + dk;
            if (a >= 0 && a < g.nx && b >= 0 && b < g.ny && c >= 0 && c < g.nz)
                acc += coef[s * n + r] * x[(s == 3) ? r : row_of(g, a, b, c)];
        }
        double o = acc;
        if (MODE == SPMV_AXPBY) {
            o *= alpha;
            if (beta != 0.0) o += beta * y[r];
        } else if (MODE == SPMV_RESID) {
            o = aux[r] - acc;
        }
        y[r] = o;
        if (MODE == SPMV_RESID || MODE == SPMV_NORM) r0 = o * o;
        if (MODE == SPMV_DOT1 || MODE == SPMV_DOT2) r0 = aux[r] * o;
        if (MODE == SPMV_DOT2) r1 = o * o;
    }
    if (MODE >= SPMV_RESID) {
        const int K = (MODE == SPMV_DOT2) ? 2 : 1;
        const double s0 = sblock_sum(r0, lds);
        if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * K] = s0;
        if (MODE == SPMV_DOT2) {
            const double s1 = sblock_sum(r1, lds);
            if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * K + 1] = s1;
        }
    }
}

// ---------------------------------------------------------------- RAS
// Entry arrays (length nent, structure of arrays): grow = row of the entry's
// cell, orow = that row if the subdomain owns the cell else -1, lo[q] / hi[q]
// = entry of the lower (-z, -y, -x) / upper (+x, +y, +z) neighbour inside the
// same Omega_s or -1; l[q] = a_ck / D_k, u[q] = a_cm, dinv = 1 / D_c; y = the
// sweeps' working values.  pl[pl_off[s] + p] .. pl[pl_off[s] + p + 1] = the
// entries of plane p of subdomain s (pl_cnt[s] planes).
struct SRasDev {
    int64_t nent;
    const int32_t *grow, *orow, *lo, *hi;
    double *l, *u, *dinv, *y;
    const int64_t *pl;
    const int32_t *pl_off, *pl_cnt;
};

__device__ constexpr int LO_SLOT[3] = {0, 1, 2};   // -z, -y, -x (ascending column)
__device__ constexpr int HI_SLOT[3] = {4, 5, 6};   // +x, +y, +z (ascending column)

__global__ __launch_bounds__(RAS_T) void k_sras_factor(Geo g, const double *__restrict__ coef, SRasDev d,
                                                       int32_t *flags)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int s = blockIdx.x;
    const int np = d.pl_cnt[s];
    const int64_t *pl = d.pl + d.pl_off[s];
    for (int p = 0; p < np; ++p) {
        for (int64_t e = pl[p] + threadIdx.x; e < pl[p + 1]; e += RAS_T) {
            const int64_t r = d.grow[e];
            double dd = coef[3 * n + r];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int32_t ke = d.lo[q * d.nent + e];
                double lv = 0.0;
                if (ke >= 0) {
                    const double a_ck = coef[LO_SLOT[q] * n + r];
                    const double a_kc = coef[(6 - LO_SLOT[q]) * n + d.grow[ke]];
                    lv = a_ck * d.dinv[ke];
                    dd -= lv * a_kc;
                }
                d.l[q * d.nent + e] = lv;
            }
#pragma unroll
            for (int q = 0; q < 3; ++q)
                d.u[q * d.nent + e] = (d.hi[q * d.nent + e] >= 0) ? coef[HI_SLOT[q] * n + r] : 0.0;
            if (!(fabs(dd) > 1e-300) || !isfinite(dd)) {
                atomicOr(&flags[0], (int32_t)FLAG_PIVOT);
                atomicMin(&flags[1], (int32_t)r);
                d.dinv[e] = 0.0;
            } else {
                d.dinv[e] = 1.0 / dd;
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(RAS_T) void k_sras_apply(SRasDev d, const double *__restrict__ rin,
                                                      double *__restrict__ zout)
{
    const int s = blockIdx.x;
    const int np = d.pl_cnt[s];
    const int64_t *pl = d.pl + d.pl_off[s];
    for (int p = 0; p < np; ++p) {          // forward: y_c = r_c - sum L_ck y_k
        for (int64_t e = pl[p] + threadIdx.x; e < pl[p + 1]; e += RAS_T) {
            double v = rin[d.grow[e]];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int32_t ke = d.lo[q * d.nent + e];
                if (ke >= 0) v -= d.l[q * d.nent + e] * d.y[ke];
            }
            d.y[e] = v;
        }
        __syncthreads();
    }
    for (int p = np - 1; p >= 0; --p) {     // backward: z_c = (y_c - sum a_cm z_m) / D_c
        for (int64_t e = pl[p] + threadIdx.x; e < pl[p + 1]; e += RAS_T) {
            double v = d.y[e];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int32_t me = d.hi[q * d.nent + e];
                if (me >= 0) v -= d.u[q * d.nent + e] * d.y[me];
            }
            v *= d.dinv[e];
            d.y[e] = v;
            const int32_t o = d.orow[e];
            if (o >= 0) zout[o] = v;
        }
        __syncthreads();
    }
}

int64_t box_start(int64_t b, int64_t len, int64_t p)
{
    const int64_t base = len / p, rem = len % p;
    return b * base + std::min(b, rem);
}

struct SRas final : PcImpl {
    rsv_matrix *M = nullptr;
    rsv_ctx *c = nullptr;
    int nsub = 0;
    int64_t nent = 0;
    std::vector<void *> mem;
    SRasDev d{};

    ~SRas() override
    {
        if (c) (void)hipStreamSynchronize(c->stream);
        for (void *p : mem) dev_free(p);
    }
    int64_t bytes() const override { return nent * (4 * 8 + 8 * 8) + nsub * 12; }
    // per Omega_s entry: row and owner ids, 3 + 3 neighbour entries, 3 + 3
    // coefficients, the pivot (88 B); r in, y out, y in, y out, z out (40 B)
    int64_t apply_bytes() const override { return nent * 128; }

    template <class T> rsv_status alloc(T **p, size_t n)
    {
        rsv_status s = dev_alloc(c, (void **)p, n * sizeof(T));
        if (s == RSV_OK) mem.push_back(*p);
        return s;
    }

    rsv_status apply(const double *r, double *z) override
    {
        ProfScope ps(c, RSV_K_RAS);
        hipLaunchKernelGGL(k_sras_apply, dim3(nsub), dim3(RAS_T), 0, c->stream, d, r, z);
        RSV_LAUNCH(c);
        return RSV_OK;
    }

    rsv_status setup(int px, int py, int pz, int ov, int64_t *bad_cell)
    {
        const Geo &G = M->g->geo;
        const int64_t nx = G.nx, ny = G.ny, nz = G.nz;
        nsub = px * py * pz;
        // per subdomain: its box, extended box and the count of its Omega_s cells
        struct Box { int64_t x0, x1, y0, y1, z0, z1, ex0, ex1, ey0, ey1, ez0, ez1, count, first; int nplane; };
        std::vector<Box> B(nsub);
        for (int s = 0; s < nsub; ++s) {
            Box &b = B[s];
            const int sx = s % px, sy = (s / px) % py, sz = s / (px * py);
            b.x0 = box_start(sx, nx, px); b.x1 = box_start(sx + 1, nx, px);
            b.y0 = box_start(sy, ny, py); b.y1 = box_start(sy + 1, ny, py);
            b.z0 = box_start(sz, nz, pz); b.z1 = box_start(sz + 1, nz, pz);
            b.ex0 = std::max<int64_t>(0, b.x0 - ov); b.ex1 = std::min<int64_t>(nx, b.x1 + ov);
            b.ey0 = std::max<int64_t>(0, b.y0 - ov); b.ey1 = std::min<int64_t>(ny, b.y1 + ov);
            b.ez0 = std::max<int64_t>(0, b.z0 - ov); b.ez1 = std::min<int64_t>(nz, b.z1 + ov);
            b.nplane = (int)((b.ex1 - b.ex0) + (b.ey1 - b.ey0) + (b.ez1 - b.ez0) - 2);
        }
        auto dist = [](int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo - v : (v >= hi ? v - hi + 1 : 0); };
        auto inside = [&](const Box &b, int64_t i, int64_t j, int64_t k) {
            return dist(i, b.x0, b.x1) + dist(j, b.y0, b.y1) + dist(k, b.z0, b.z1) <= ov;
        };
        int64_t total = 0, tplanes = 0;
        for (int s = 0; s < nsub; ++s) {
            Box &b = B[s];
            int64_t cnt = 0;
            for (int64_t k = b.ez0; k < b.ez1; ++k)
                for (int64_t j = b.ey0; j < b.ey1; ++j) {
                    // the cells of row (j, k) inside Omega_s form one x-interval
                    const int64_t rest = dist(j, b.y0, b.y1) + dist(k, b.z0, b.z1);
                    if (rest > ov) continue;
                    const int64_t lo = std::max(b.ex0, b.x0 - (ov - rest)), hi = std::min(b.ex1, b.x1 + (ov - rest));
                    cnt += std::max<int64_t>(0, hi - lo);
                }
            b.count = cnt;
            b.first = total;
            total += cnt;
            tplanes += b.nplane + 1;
        }
        if (total >= ((int64_t)1 << 31)) return set_err(c, RSV_ERR_ARG, "RAS: more than 2^31 subdomain cells");
        nent = total;
        std::vector<int32_t> grow(total), orow(total), lo(3 * total), hi(3 * total);
        std::vector<int64_t> pl(tplanes);
        std::vector<int32_t> pl_off(nsub), pl_cnt(nsub);
        {
            int64_t off = 0;
            for (int s = 0; s < nsub; ++s) {
                pl_off[s] = (int32_t)off;
                pl_cnt[s] = B[s].nplane;
                off += B[s].nplane + 1;
            }
        }
        auto build = [&](int s) {
            const Box &b = B[s];
            const int64_t EX = b.ex1 - b.ex0, EY = b.ey1 - b.ey0, EZ = b.ez1 - b.ez0;
            std::vector<int32_t> cntp(b.nplane + 1, 0);
            for (int64_t k = b.ez0; k < b.ez1; ++k)
                for (int64_t j = b.ey0; j < b.ey1; ++j)
                    for (int64_t i = b.ex0; i < b.ex1; ++i)
                        if (inside(b, i, j, k)) cntp[(i - b.ex0) + (j - b.ey0) + (k - b.ez0) + 1]++;
            for (int p = 0; p < b.nplane; ++p) cntp[p + 1] += cntp[p];
            int64_t *plp = pl.data() + pl_off[s];
            for (int p = 0; p <= b.nplane; ++p) plp[p] = b.first + cntp[p];
            std::vector<int32_t> lmap((size_t)(EX * EY * EZ), -1);
            std::vector<int32_t> fill(cntp.begin(), cntp.end() - 1);
            for (int64_t k = b.ez0; k < b.ez1; ++k)           // natural order inside every plane
                for (int64_t j = b.ey0; j < b.ey1; ++j)
                    for (int64_t i = b.ex0; i < b.ex1; ++i) {
                        if (!inside(b, i, j, k)) continue;
                        const int p = (int)((i - b.ex0) + (j - b.ey0) + (k - b.ez0));
                        const int64_t e = b.first + fill[p]++;
                        lmap[((k - b.ez0) * EY + (j - b.ey0)) * EX + (i - b.ex0)] = (int32_t)e;
                        const int64_t row = row_of(G, (int)i, (int)j, (int)k);
                        grow[e] = (int32_t)row;
                        const bool own = i >= b.x0 && i < b.x1 && j >= b.y0 && j < b.y1 && k >= b.z0 && k < b.z1;
                        orow[e] = own ? (int32_t)row : -1;
                    }
            auto at = [&](int64_t i, int64_t j, int64_t k) -> int32_t {
                if (i < b.ex0 || i >= b.ex1 || j < b.ey0 || j >= b.ey1 || k < b.ez0 || k >= b.ez1) return -1;
                return lmap[((k - b.ez0) * EY + (j - b.ey0)) * EX + (i - b.ex0)];
            };
            for (int64_t k = b.ez0; k < b.ez1; ++k)
                for (int64_t j = b.ey0; j < b.ey1; ++j)
                    for (int64_t i = b.ex0; i < b.ex1; ++i) {
                        const int32_t e = at(i, j, k);
                        if (e < 0) continue;
                        lo[0 * total + e] = at(i, j, k - 1);
                        lo[1 * total + e] = at(i, j - 1, k);
                        lo[2 * total + e] = at(i - 1, j, k);
                        hi[0 * total + e] = at(i + 1, j, k);
                        hi[1 * total + e] = at(i, j + 1, k);
                        hi[2 * total + e] = at(i, j, k + 1);
                    }
        };
        {
            const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
            std::vector<std::thread> th;
            for (int t = 0; t < nth; ++t)
                th.emplace_back([&, t] { for (int s = t; s < nsub; s += nth) build(s); });
            for (auto &x : th) x.join();
        }
        int32_t *dgrow, *dorow, *dlo, *dhi, *dploff, *dplcnt;
        int64_t *dpl;
        double *dl, *du, *ddinv, *dy;
        rsv_status st = alloc(&dgrow, (size_t)total);
        if (st == RSV_OK) st = alloc(&dorow, (size_t)total);
        if (st == RSV_OK) st = alloc(&dlo, (size_t)3 * total);
        if (st == RSV_OK) st = alloc(&dhi, (size_t)3 * total);
        if (st == RSV_OK) st = alloc(&dl, (size_t)3 * total);
        if (st == RSV_OK) st = alloc(&du, (size_t)3 * total);
        if (st == RSV_OK) st = alloc(&ddinv, (size_t)total);
        if (st == RSV_OK) st = alloc(&dy, (size_t)total);
        if (st == RSV_OK) st = alloc(&dpl, (size_t)tplanes);
        if (st == RSV_OK) st = alloc(&dploff, (size_t)nsub);
        if (st == RSV_OK) st = alloc(&dplcnt, (size_t)nsub);
        if (st != RSV_OK) return st;
        RSV_HIP(c, hipMemcpyAsync(dgrow, grow.data(), total * 4, hipMemcpyHostToDevice, c->stream));
        RSV_HIP(c, hipMemcpyAsync(dorow, orow.data(), total * 4, hipMemcpyHostToDevice, c->stream));
        RSV_HIP(c, hipMemcpyAsync(dlo, lo.data(), 3 * total * 4, hipMemcpyHostToDevice, c->stream));
        RSV_HIP(c, hipMemcpyAsync(dhi, hi.data(), 3 * total * 4, hipMemcpyHostToDevice, c->stream));
        RSV_HIP(c, hipMemcpyAsync(dpl, pl.data(), tplanes * 8, hipMemcpyHostToDevice, c->stream));
        RSV_HIP(c, hipMemcpyAsync(dploff, pl_off.data(), nsub * 4, hipMemcpyHostToDevice, c->stream));
        RSV_HIP(c, hipMemcpyAsync(dplcnt, pl_cnt.data(), nsub * 4, hipMemcpyHostToDevice, c->stream));
        d = SRasDev{total, dgrow, dorow, dlo, dhi, dl, du, ddinv, dy, dpl, dploff, dplcnt};
        rsv_status fs = flags_reset(c);   // synchronises: the host arrays may be released after it
        if (fs != RSV_OK) return fs;
        {
            ProfScope ps(c, RSV_K_FACTOR);
            hipLaunchKernelGGL(k_sras_factor, dim3(nsub), dim3(RAS_T), 0, c->stream, G, M->d_coef, d, c->d_flags);
        }
        RSV_LAUNCH(c);
        return flags_check(c, bad_cell);
    }
};

}  // namespace

rsv_status launch_sspmv(rsv_ctx *c, const Geo &g, const double *coef, int mode, const double *x, double *y,
                        const double *aux, double alpha, double beta, int k0)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int nb = (int)((n + SB - 1) / SB);
    if (mode >= SPMV_RESID) {
        rsv_status s = partials_reserve(c, (int64_t)nb * 2);
        if (s != RSV_OK) return s;
    }
    double *P = c->d_partials;
    const int tok = prof_begin(c, RSV_K_SPMV);
    const dim3 grid(nb), blk(SB);
    switch (mode) {
    case SPMV_Y: hipLaunchKernelGGL(k_sspmv<SPMV_Y>, grid, blk, 0, c->stream, g, coef, x, y, aux, alpha, beta, P); break;
    case SPMV_AXPBY: hipLaunchKernelGGL(k_sspmv<SPMV_AXPBY>, grid, blk, 0, c->stream, g, coef, x, y, aux, alpha, beta, P); break;
    case SPMV_RESID: hipLaunchKernelGGL(k_sspmv<SPMV_RESID>, grid, blk, 0, c->stream, g, coef, x, y, aux, alpha, beta, P); break;
    case SPMV_NORM: hipLaunchKernelGGL(k_sspmv<SPMV_NORM>, grid, blk, 0, c->stream, g, coef, x, y, aux, alpha, beta, P); break;
    case SPMV_DOT1: hipLaunchKernelGGL(k_sspmv<SPMV_DOT1>, grid, blk, 0, c->stream, g, coef, x, y, aux, alpha, beta, P); break;
    case SPMV_DOT2: hipLaunchKernelGGL(k_sspmv<SPMV_DOT2>, grid, blk, 0, c->stream, g, coef, x, y, aux, alpha, beta, P); break;
    default: return set_err(c, RSV_ERR_ARG, "bad spmv mode");
    }
    prof_end(c, tok);
    RSV_LAUNCH(c);
    if (mode >= SPMV_RESID) return launch_reduce(c, nb, mode == SPMV_DOT2 ? 2 : 1, k0);
    return RSV_OK;
}

rsv_status mat_spmv(rsv_matrix *M, int mode, const double *x, double *y, const double *aux, double alpha,
                    double beta, int k0)
{
    if (M->bs == 1) return launch_sspmv(M->g->ctx, M->g->geo, M->d_coef, mode, x, y, aux, alpha, beta, k0);
    return launch_spmv(M->g->ctx, M->g->geo, M->d_A, mode, x, y, aux, alpha, beta, k0);
}

rsv_status mat_in(rsv_matrix *M, const double *nat, double *v)
{
    if (M->bs == 1) return launch_copy(M->g->ctx, M->nv, nat, v);
    return launch_nat_to_tl(M->g->ctx, M->g->geo, nat, v);
}

rsv_status mat_out(rsv_matrix *M, const double *v, double *nat, double alpha, double beta)
{
    if (M->bs == 1) return launch_axpby(M->g->ctx, M->nv, alpha, v, beta, nat);
    return launch_tl_to_nat(M->g->ctx, M->g->geo, v, nat, alpha, beta);
}

rsv_status sras_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, int64_t *bad_cell)
{
    rsv_ctx *c = A->g->ctx;
    const Geo &G = A->g->geo;
    int px = 1, py = 1, pz = 1, ov = 0;      // BILU0 of a scalar matrix: one subdomain, no overlap
    if (p->type == RSV_PC_RAS) {
        px = p->ras_px; py = p->ras_py; pz = p->ras_pz; ov = p->ras_overlap;
        if (px < 1 || py < 1 || pz < 1 || px > G.nx || py > G.ny || pz > G.nz || ov < 0)
            return set_err(c, RSV_ERR_ARG, "bad RAS subdomain counts or overlap");
    }
    if (p->precision != RSV_FP64) return set_err(c, RSV_ERR_ARG, "scalar systems have FP64 preconditioners only");
    SRas *R = new (std::nothrow) SRas();
    if (!R) return set_err(c, RSV_ERR_OOM, "scalar RAS");
    R->M = A;
    R->c = c;
    rsv_status s = R->setup(px, py, pz, ov, bad_cell);
    if (s != RSV_OK) {
        delete R;
        return s;
    }
    *out = R;
    return RSV_OK;
}

extern "C" {

rsv_status rsv_matrix_assemble_scalar(rsv_grid *g, const double *coef, int32_t where, rsv_matrix **out)
{
    if (!g || !coef || !out) return set_err(g ? g->ctx : nullptr, RSV_ERR_ARG, "NULL argument");
    *out = nullptr;
    rsv_ctx *c = g->ctx;
    rsv_matrix *M = new (std::nothrow) rsv_matrix();
    if (!M) return set_err(c, RSV_ERR_OOM, "matrix");
    M->g = g;
    M->bs = 1;
    M->nv = g->ncell;
    rsv_status s = dev_alloc(c, (void **)&M->d_coef, (size_t)g->ncell * 7 * sizeof(double));
    if (s == RSV_OK) {
        M->bytes = g->ncell * 7 * (int64_t)sizeof(double);
        s = scalar_assemble_values(M, coef, where);
    }
    if (s != RSV_OK) {
        rsv_matrix_destroy(M);
        return s;
    }
    *out = M;
    return RSV_OK;
}

}  // extern "C"

rsv_status scalar_assemble_values(rsv_matrix *M, const double *coef, int32_t where)
{
    rsv_grid *g = M->g;
    rsv_ctx *c = g->ctx;
    const size_t bytes = (size_t)g->ncell * 7 * sizeof(double);
    const double *src = coef;
    double *stage = nullptr;
    if (where == RSV_MEM_HOST) {
        rsv_status s = dev_alloc(c, (void **)&stage, bytes);
        if (s != RSV_OK) return s;
        hipError_t e = hipMemcpyAsync(stage, coef, bytes, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) {
            dev_free(stage);
            return set_err(c, RSV_ERR_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
        }
        src = stage;
    } else if (where != RSV_MEM_DEVICE) {
        return set_err(c, RSV_ERR_ARG, "bad memory kind");
    }
    rsv_status s = flags_reset(c);
    if (s == RSV_OK) {
        hipLaunchKernelGGL(k_sassemble, dim3((unsigned)((g->ncell + SB - 1) / SB)), dim3(SB), 0, c->stream, g->geo, src,
                           M->d_coef, c->d_flags);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) s = set_err(c, RSV_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    if (s == RSV_OK) s = flags_check(c, nullptr);
    if (stage) dev_free(stage);
    return s;
}
