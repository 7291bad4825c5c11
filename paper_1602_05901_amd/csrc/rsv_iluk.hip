// ILU(k) local solvers for restricted additive Schwarz (the ILUK local
// solver of the RAS data structure and its level parameter, Restricted
// Additive Schwarz Method subsection), for 3x3-block matrices.
//
// Subdomains, overlap and owner-only write-back are those of the ILU(0) RAS:
// px x py x pz boxes (the first n mod p one cell longer), Omega_s = the cells
// within graph distance `overlap` of the box, local order = ascending global
// (bottom-up natural) index.  ILU(k) keeps the fill positions whose level of
// fill is at most k: the stencil positions have level 0, and eliminating row
// m from row i gives (i, j) the level lev(i,m) + lev(m,j) + 1.  With fill
// the hyperplane schedule of ILU(0) no longer holds (level-1 fill couples
// cell c to c + e_x - e_y, a cell of the same plane i + j + k), so rows are
// scheduled by dependency levels computed from the symbolic pattern: a row's
// forward level is one more than that of every column of its L part, its
// backward level one more than that of every column of its U part.
//
// Host: the symbolic factorisation and the schedules, per subdomain (threads
// over subdomains).  Device: one workgroup per subdomain walks its levels
// with a barrier between them -- the IKJ numeric factorisation (a row's L
// blocks times the inverted pivots of the rows they reference, each update
// merged into the row's sorted pattern, then the row's own pivot inverted by
// cofactors), and for an apply the forward sweep y_i = r_i - sum L_ij y_j and
// the backward sweep z_i = U_ii^-1 (y_i - sum U_ij z_j), the owner writing
// z_i into the tile-lane result.
#include "rsv_internal.h"

#include <algorithm>
#include <new>
#include <thread>
#include <vector>

namespace {

constexpr int KT = 256;   // threads of a subdomain's workgroup

struct IlukDev {
    int64_t nrow;
    const int32_t *gslot, *own;          // per row: tile-lane slot of its cell; 1 if the subdomain owns it
    const int64_t *lptr, *uptr;          // per row: ranges in the L / U position arrays
    const int32_t *lcol, *ucol;          // column = row index (global across subdomains)
    const int64_t *lsrc, *usrc;          // A-entry base index of a stencil position, -1 for fill
    double *lval, *uval, *dval, *dinv;   // 9 per position / row, row-major blocks
    double *y;                           // 3 per row
    const int32_t *fo, *bo;              // rows in forward / backward level order
    const int64_t *fl, *bl;              // level boundaries into fo / bo
    const int32_t *fl_off, *bl_off, *fl_cnt, *bl_cnt;   // per subdomain: first boundary, level count
    const int64_t *dbase;                // per row: A-entry base index of the diagonal block
};

__device__ inline void mm3_sub(const double *a, const double *b, double *c)   // c -= a b
{
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) c[3 * p + q] -= a[3 * p] * b[q] + a[3 * p + 1] * b[3 + q] + a[3 * p + 2] * b[6 + q];
}

// initial values: the blocks of A at stencil positions (tile-lane entries
// 64 apart), zero at fill positions
__global__ __launch_bounds__(256) void k_iluk_load(const double *__restrict__ A, IlukDev d, int64_t nl, int64_t nu)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t tot = nl + nu + d.nrow;
    if (t >= tot) return;
    int64_t src;
    double *dst;
    if (t < nl) { src = d.lsrc[t]; dst = d.lval + 9 * t; }
    else if (t < nl + nu) { src = d.usrc[t - nl]; dst = d.uval + 9 * (t - nl); }
    else { src = d.dbase[t - nl - nu]; dst = d.dval + 9 * (t - nl - nu); }
#pragma unroll
    for (int e = 0; e < 9; ++e) dst[e] = (src >= 0) ? A[src + 64 * e] : 0.0;
}

__global__ __launch_bounds__(KT) void k_iluk_factor(IlukDev d, int32_t *flags)
{
    const int s = blockIdx.x;
    const int nlev = d.fl_cnt[s];
    const int64_t *fl = d.fl + d.fl_off[s];
    for (int lv = 0; lv < nlev; ++lv) {
        for (int64_t t = fl[lv] + threadIdx.x; t < fl[lv + 1]; t += KT) {
            const int32_t i = d.fo[t];
            const int64_t l0 = d.lptr[i], l1 = d.lptr[i + 1], u0 = d.uptr[i], u1 = d.uptr[i + 1];
            for (int64_t p = l0; p < l1; ++p) {
                const int32_t k = d.lcol[p];
                double lik[9], a[9];
#pragma unroll
                for (int e = 0; e < 9; ++e) a[e] = d.lval[9 * p + e];
                const double *dk = d.dinv + 9 * k;
#pragma unroll
                for (int pp = 0; pp < 3; ++pp)
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        lik[3 * pp + q] = a[3 * pp] * dk[q] + a[3 * pp + 1] * dk[3 + q] + a[3 * pp + 2] * dk[6 + q];
#pragma unroll
                for (int e = 0; e < 9; ++e) d.lval[9 * p + e] = lik[e];
                // row i -= L_ik (row k's U part), merged into the sorted pattern of row i
                int64_t pl = p + 1, pu = u0;
                for (int64_t q = d.uptr[k]; q < d.uptr[k + 1]; ++q) {
                    const int32_t j = d.ucol[q];
                    double *tgt = nullptr;
                    if (j < i) {
                        while (pl < l1 && d.lcol[pl] < j) ++pl;
                        if (pl < l1 && d.lcol[pl] == j) tgt = d.lval + 9 * pl;
                    } else if (j == i) {
                        tgt = d.dval + 9 * (int64_t)i;
                    } else {
                        while (pu < u1 && d.ucol[pu] < j) ++pu;
                        if (pu < u1 && d.ucol[pu] == j) tgt = d.uval + 9 * pu;
                    }
                    if (tgt) mm3_sub(lik, d.uval + 9 * q, tgt);
                }
            }
            double D[9], Di[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) D[e] = d.dval[9 * (int64_t)i + e];
            if (!inv3(D, Di)) {
                atomicOr(&flags[0], (int32_t)FLAG_PIVOT);
                atomicMin(&flags[1], (int32_t)d.own[i] >> 1);   // the row's cell, stored with the owner bit
#pragma unroll
                for (int e = 0; e < 9; ++e) Di[e] = 0.0;
            }
#pragma unroll
            for (int e = 0; e < 9; ++e) d.dinv[9 * (int64_t)i + e] = Di[e];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(KT) void k_iluk_apply(IlukDev d, const double *__restrict__ r, double *__restrict__ z)
{
    const int s = blockIdx.x;
    {
        const int nlev = d.fl_cnt[s];
        const int64_t *fl = d.fl + d.fl_off[s];
        for (int lv = 0; lv < nlev; ++lv) {
            for (int64_t t = fl[lv] + threadIdx.x; t < fl[lv + 1]; t += KT) {
                const int32_t i = d.fo[t];
                const int64_t sl = d.gslot[i];
                double v0 = r[vidx(sl, 0)], v1 = r[vidx(sl, 1)], v2 = r[vidx(sl, 2)];
                for (int64_t p = d.lptr[i]; p < d.lptr[i + 1]; ++p) {
                    const double *L = d.lval + 9 * p, *yk = d.y + 3 * (int64_t)d.lcol[p];
                    const double y0 = yk[0], y1 = yk[1], y2 = yk[2];
                    v0 -= L[0] * y0 + L[1] * y1 + L[2] * y2;
                    v1 -= L[3] * y0 + L[4] * y1 + L[5] * y2;
                    v2 -= L[6] * y0 + L[7] * y1 + L[8] * y2;
                }
                d.y[3 * (int64_t)i] = v0;
                d.y[3 * (int64_t)i + 1] = v1;
                d.y[3 * (int64_t)i + 2] = v2;
            }
            __syncthreads();
        }
    }
    {
        const int nlev = d.bl_cnt[s];
        const int64_t *bl = d.bl + d.bl_off[s];
        for (int lv = 0; lv < nlev; ++lv) {
            for (int64_t t = bl[lv] + threadIdx.x; t < bl[lv + 1]; t += KT) {
                const int32_t i = d.bo[t];
                double v0 = d.y[3 * (int64_t)i], v1 = d.y[3 * (int64_t)i + 1], v2 = d.y[3 * (int64_t)i + 2];
                for (int64_t q = d.uptr[i]; q < d.uptr[i + 1]; ++q) {
                    const double *U = d.uval + 9 * q, *zj = d.y + 3 * (int64_t)d.ucol[q];
                    const double z0 = zj[0], z1 = zj[1], z2 = zj[2];
                    v0 -= U[0] * z0 + U[1] * z1 + U[2] * z2;
                    v1 -= U[3] * z0 + U[4] * z1 + U[5] * z2;
                    v2 -= U[6] * z0 + U[7] * z1 + U[8] * z2;
                }
                const double *Di = d.dinv + 9 * (int64_t)i;
                const double w0 = Di[0] * v0 + Di[1] * v1 + Di[2] * v2;
                const double w1 = Di[3] * v0 + Di[4] * v1 + Di[5] * v2;
                const double w2 = Di[6] * v0 + Di[7] * v1 + Di[8] * v2;
                d.y[3 * (int64_t)i] = w0;
                d.y[3 * (int64_t)i + 1] = w1;
                d.y[3 * (int64_t)i + 2] = w2;
                if (d.own[i] & 1) {
                    const int64_t sl = d.gslot[i];
                    z[vidx(sl, 0)] = w0;
                    z[vidx(sl, 1)] = w1;
                    z[vidx(sl, 2)] = w2;
                }
            }
            __syncthreads();
        }
    }
}

int64_t kbox_start(int64_t b, int64_t len, int64_t p)
{
    const int64_t base = len / p, rem = len % p;
    return b * base + std::min(b, rem);
}

// symbolic ILU(k) of one subdomain's local matrix, rows in local order
struct SubPlan {
    std::vector<int64_t> cells;                  // global natural cell index, ascending
    std::vector<int32_t> owned;
    std::vector<std::vector<int32_t>> lcol, ucol; // local columns, ascending
    std::vector<int32_t> flev, blev;
    int nfl = 0, nbl = 0;
};

struct RasK final : PcImpl {
    rsv_matrix *M = nullptr;
    rsv_ctx *c = nullptr;
    int nsub = 0;
    int64_t nrow = 0, nl = 0, nu = 0;
    std::vector<void *> mem;
    IlukDev d{};

    ~RasK() override
    {
        if (c) (void)hipStreamSynchronize(c->stream);
        for (void *p : mem) dev_free(p);
    }
    int64_t bytes() const override { return (nl + nu) * (72 + 12) + nrow * (2 * 72 + 24 + 32); }

    template <class T> rsv_status upload(T **dp, const std::vector<T> &h)
    {
        rsv_status s = dev_alloc(c, (void **)dp, std::max<size_t>(h.size(), 1) * sizeof(T));
        if (s != RSV_OK) return s;
        mem.push_back(*dp);
        if (!h.empty()) RSV_HIP(c, hipMemcpyAsync(*dp, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
        return RSV_OK;
    }
    template <class T> rsv_status alloc(T **dp, size_t n)
    {
        rsv_status s = dev_alloc(c, (void **)dp, std::max<size_t>(n, 1) * sizeof(T));
        if (s == RSV_OK) mem.push_back(*dp);
        return s;
    }

    rsv_status apply(const double *r, double *z) override
    {
        ProfScope ps(c, RSV_K_RAS);
        hipLaunchKernelGGL(k_iluk_apply, dim3(nsub), dim3(KT), 0, c->stream, d, r, z);
        RSV_LAUNCH(c);
        return RSV_OK;
    }

    rsv_status setup(int px, int py, int pz, int ov, int level, int64_t *bad_cell)
    {
        const Geo &G = M->g->geo;
        const int64_t nx = G.nx, ny = G.ny, nz = G.nz;
        nsub = px * py * pz;
        std::vector<SubPlan> P(nsub);
        auto dist = [](int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo - v : (v >= hi ? v - hi + 1 : 0); };
        auto plan = [&](int s) {
            SubPlan &sp = P[s];
            const int64_t sx = s % px, sy = (s / px) % py, sz = s / ((int64_t)px * py);
            const int64_t x0 = kbox_start(sx, nx, px), x1 = kbox_start(sx + 1, nx, px);
            const int64_t y0 = kbox_start(sy, ny, py), y1 = kbox_start(sy + 1, ny, py);
            const int64_t z0 = kbox_start(sz, nz, pz), z1 = kbox_start(sz + 1, nz, pz);
            const int64_t ex0 = std::max<int64_t>(0, x0 - ov), ex1 = std::min<int64_t>(nx, x1 + ov);
            const int64_t ey0 = std::max<int64_t>(0, y0 - ov), ey1 = std::min<int64_t>(ny, y1 + ov);
            const int64_t ez0 = std::max<int64_t>(0, z0 - ov), ez1 = std::min<int64_t>(nz, z1 + ov);
            const int64_t EX = ex1 - ex0, EY = ey1 - ey0, EZ = ez1 - ez0;
            std::vector<int32_t> lmap((size_t)(EX * EY * EZ), -1);
            for (int64_t k = ez0; k < ez1; ++k)
                for (int64_t j = ey0; j < ey1; ++j)
                    for (int64_t i = ex0; i < ex1; ++i) {
                        if (dist(i, x0, x1) + dist(j, y0, y1) + dist(k, z0, z1) > ov) continue;
                        lmap[((k - ez0) * EY + (j - ey0)) * EX + (i - ex0)] = (int32_t)sp.cells.size();
                        sp.cells.push_back((k * ny + j) * nx + i);
                        sp.owned.push_back(i >= x0 && i < x1 && j >= y0 && j < y1 && k >= z0 && k < z1);
                    }
            const int64_t m = (int64_t)sp.cells.size();
            auto at = [&](int64_t i, int64_t j, int64_t k) -> int32_t {
                if (i < ex0 || i >= ex1 || j < ey0 || j >= ey1 || k < ez0 || k >= ez1) return -1;
                return lmap[((k - ez0) * EY + (j - ey0)) * EX + (i - ex0)];
            };
            sp.lcol.assign(m, {});
            sp.ucol.assign(m, {});
            std::vector<std::vector<int32_t>> ulev(m);
            std::vector<int32_t> lev(m, -1), row;
            for (int64_t r = 0; r < m; ++r) {
                const int64_t cc = sp.cells[r];
                const int64_t i = cc % nx, j = (cc / nx) % ny, k = cc / (nx * ny);
                row.clear();
                const int32_t nb[7] = {at(i, j, k - 1), at(i, j - 1, k), at(i - 1, j, k), (int32_t)r,
                                       at(i + 1, j, k), at(i, j + 1, k), at(i, j, k + 1)};
                for (int q = 0; q < 7; ++q)
                    if (nb[q] >= 0) { row.push_back(nb[q]); lev[nb[q]] = 0; }
                std::sort(row.begin(), row.end());
                for (size_t t = 0; t < row.size() && row[t] < r; ++t) {
                    const int32_t mm = row[t];
                    for (size_t q = 0; q < sp.ucol[mm].size(); ++q) {
                        const int32_t jj = sp.ucol[mm][q];
                        const int32_t l = lev[mm] + ulev[mm][q] + 1;
                        if (l > level) continue;
                        if (lev[jj] < 0) {
                            row.insert(std::upper_bound(row.begin() + t + 1, row.end(), jj), jj);
                            lev[jj] = l;
                        } else if (l < lev[jj]) {
                            lev[jj] = l;
                        }
                    }
                }
                for (int32_t col : row) {
                    if (col < r) sp.lcol[r].push_back(col);
                    else if (col > r) { sp.ucol[r].push_back(col); ulev[r].push_back(lev[col]); }
                    lev[col] = -1;
                }
            }
            sp.flev.assign(m, 0);
            sp.blev.assign(m, 0);
            for (int64_t r = 0; r < m; ++r) {
                int32_t v = 0;
                for (int32_t k2 : sp.lcol[r]) v = std::max(v, sp.flev[k2] + 1);
                sp.flev[r] = v;
                sp.nfl = std::max(sp.nfl, v + 1);
            }
            for (int64_t r = m - 1; r >= 0; --r) {
                int32_t v = 0;
                for (int32_t j2 : sp.ucol[r]) v = std::max(v, sp.blev[j2] + 1);
                sp.blev[r] = v;
                sp.nbl = std::max(sp.nbl, v + 1);
            }
        };
        {
            const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
            std::vector<std::thread> th;
            for (int t = 0; t < nth; ++t)
                th.emplace_back([&, t] { for (int s = t; s < nsub; s += nth) plan(s); });
            for (auto &x : th) x.join();
        }
        // concatenate: rows of subdomain s start at base[s]
        std::vector<int64_t> base(nsub + 1, 0);
        for (int s = 0; s < nsub; ++s) base[s + 1] = base[s] + (int64_t)P[s].cells.size();
        nrow = base[nsub];
        if (nrow >= ((int64_t)1 << 31)) return set_err(c, RSV_ERR_ARG, "RAS: more than 2^31 subdomain cells");
        std::vector<int32_t> gslot(nrow), own(nrow), lcol, ucol, fo(nrow), bo(nrow);
        std::vector<int64_t> lptr(nrow + 1), uptr(nrow + 1), lsrc, usrc, dbase(nrow), fl, bl;
        std::vector<int32_t> fl_off(nsub), bl_off(nsub), fl_cnt(nsub), bl_cnt(nsub);
        auto abase = [&](int64_t cell, int slotdir) -> int64_t {   // A entry of block (cell, stencil slot) at element 0
            const int i = (int)(cell % nx), j = (int)((cell / nx) % ny), k = (int)(cell / (nx * ny));
            return aidx(slot_of(G, i, j, k), slotdir * 9);
        };
        // stencil slot of the position (cell a, column cell b), or -1 for a fill position
        auto stencil_dir = [&](int64_t a, int64_t b) -> int {
            const int64_t di = b % nx - a % nx, dj = (b / nx) % ny - (a / nx) % ny, dk = b / (nx * ny) - a / (nx * ny);
            if (di == 0 && dj == 0 && dk == -1) return 0;
            if (di == 0 && dj == -1 && dk == 0) return 1;
            if (di == -1 && dj == 0 && dk == 0) return 2;
            if (di == 1 && dj == 0 && dk == 0) return 4;
            if (di == 0 && dj == 1 && dk == 0) return 5;
            if (di == 0 && dj == 0 && dk == 1) return 6;
            return -1;
        };
        for (int s = 0; s < nsub; ++s) {
            const SubPlan &sp = P[s];
            const int64_t m = (int64_t)sp.cells.size();
            for (int64_t r = 0; r < m; ++r) {
                const int64_t g = base[s] + r, cc = sp.cells[r];
                const int i = (int)(cc % nx), j = (int)((cc / nx) % ny), k = (int)(cc / (nx * ny));
                gslot[g] = (int32_t)slot_of(G, i, j, k);
                // the owner bit, and the cell's row for error reports
                own[g] = (int32_t)((row_of(G, i, j, k) << 1) | (sp.owned[r] ? 1 : 0));
                dbase[g] = abase(cc, 3);
                lptr[g] = (int64_t)lcol.size();
                for (int32_t col : sp.lcol[r]) {
                    lcol.push_back((int32_t)(base[s] + col));
                    const int dir = stencil_dir(cc, sp.cells[col]);
                    lsrc.push_back(dir >= 0 ? abase(cc, dir) : -1);
                }
                uptr[g] = (int64_t)ucol.size();
                for (int32_t col : sp.ucol[r]) {
                    ucol.push_back((int32_t)(base[s] + col));
                    const int dir = stencil_dir(cc, sp.cells[col]);
                    usrc.push_back(dir >= 0 ? abase(cc, dir) : -1);
                }
            }
        }
        lptr[nrow] = (int64_t)lcol.size();
        uptr[nrow] = (int64_t)ucol.size();
        nl = (int64_t)lcol.size();
        nu = (int64_t)ucol.size();
        // level schedules: rows of a subdomain bucketed by level
        int64_t pos = 0;
        for (int s = 0; s < nsub; ++s) {
            const SubPlan &sp = P[s];
            const int64_t m = (int64_t)sp.cells.size();
            for (int pass = 0; pass < 2; ++pass) {
                const std::vector<int32_t> &lv = pass ? sp.blev : sp.flev;
                const int nlv = pass ? sp.nbl : sp.nfl;
                std::vector<int64_t> cnt(nlv + 1, 0);
                for (int64_t r = 0; r < m; ++r) cnt[lv[r] + 1]++;
                for (int q = 0; q < nlv; ++q) cnt[q + 1] += cnt[q];
                std::vector<int64_t> &bounds = pass ? bl : fl;
                (pass ? bl_off : fl_off)[s] = (int32_t)bounds.size();
                (pass ? bl_cnt : fl_cnt)[s] = nlv;
                for (int q = 0; q <= nlv; ++q) bounds.push_back(pos + cnt[q]);
                std::vector<int32_t> &ord = pass ? bo : fo;
                std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
                for (int64_t r = 0; r < m; ++r) ord[pos + fill[lv[r]]++] = (int32_t)(base[s] + r);
            }
            pos += m;
        }
        P.clear();
        int32_t *dgslot, *down, *dlcol, *ducol, *dfo, *dbo, *dfloff, *dbloff, *dflcnt, *dblcnt;
        int64_t *dlptr, *duptr, *dlsrc, *dusrc, *ddbase, *dfl, *dbl;
        double *dlval, *duval, *ddval, *ddinv, *dy;
        rsv_status st = upload(&dgslot, gslot);
        if (st == RSV_OK) st = upload(&down, own);
        if (st == RSV_OK) st = upload(&dlptr, lptr);
        if (st == RSV_OK) st = upload(&duptr, uptr);
        if (st == RSV_OK) st = upload(&dlcol, lcol);
        if (st == RSV_OK) st = upload(&ducol, ucol);
        if (st == RSV_OK) st = upload(&dlsrc, lsrc);
        if (st == RSV_OK) st = upload(&dusrc, usrc);
        if (st == RSV_OK) st = upload(&ddbase, dbase);
        if (st == RSV_OK) st = upload(&dfo, fo);
        if (st == RSV_OK) st = upload(&dbo, bo);
        if (st == RSV_OK) st = upload(&dfl, fl);
        if (st == RSV_OK) st = upload(&dbl, bl);
        if (st == RSV_OK) st = upload(&dfloff, fl_off);
        if (st == RSV_OK) st = upload(&dbloff, bl_off);
        if (st == RSV_OK) st = upload(&dflcnt, fl_cnt);
        if (st == RSV_OK) st = upload(&dblcnt, bl_cnt);
        if (st == RSV_OK) st = alloc(&dlval, (size_t)9 * nl);
        if (st == RSV_OK) st = alloc(&duval, (size_t)9 * nu);
        if (st == RSV_OK) st = alloc(&ddval, (size_t)9 * nrow);
        if (st == RSV_OK) st = alloc(&ddinv, (size_t)9 * nrow);
        if (st == RSV_OK) st = alloc(&dy, (size_t)3 * nrow);
        if (st != RSV_OK) return st;
        d = IlukDev{nrow, dgslot, down, dlptr, duptr, dlcol, ducol, dlsrc, dusrc, dlval, duval, ddval, ddinv,
                    dy, dfo, dbo, dfl, dbl, dfloff, dbloff, dflcnt, dblcnt, ddbase};
        rsv_status fs = flags_reset(c);      // synchronises: the host arrays may go after this
        if (fs != RSV_OK) return fs;
        {
            ProfScope ps(c, RSV_K_FACTOR);
            const int64_t tot = nl + nu + nrow;
            hipLaunchKernelGGL(k_iluk_load, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, M->d_A, d,
                               nl, nu);
            hipLaunchKernelGGL(k_iluk_factor, dim3(nsub), dim3(KT), 0, c->stream, d, c->d_flags);
        }
        RSV_LAUNCH(c);
        return flags_check(c, bad_cell);
    }
};

}  // namespace

rsv_status rasK_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, int64_t *bad_cell)
{
    rsv_ctx *c = A->g->ctx;
    const Geo &G = A->g->geo;
    int px = 1, py = 1, pz = 1, ov = 0;      // BILU(k) of the whole grid: one subdomain, no overlap
    if (p->type == RSV_PC_RAS) {
        px = p->ras_px; py = p->ras_py; pz = p->ras_pz; ov = p->ras_overlap;
        if (px < 1 || py < 1 || pz < 1 || px > G.nx || py > G.ny || pz > G.nz || ov < 0)
            return set_err(c, RSV_ERR_ARG, "bad RAS subdomain counts or overlap");
    }
    if (p->precision != RSV_FP64) return set_err(c, RSV_ERR_ARG, "ILU(k) with k > 0 has FP64 factors only");
    if (p->iluk_level < 1 || p->iluk_level > 8) return set_err(c, RSV_ERR_ARG, "iluk_level must be in [0, 8]");
    RasK *R = new (std::nothrow) RasK();
    if (!R) return set_err(c, RSV_ERR_OOM, "ILU(k) RAS");
    R->M = A;
    R->c = c;
    rsv_status s = R->setup(px, py, pz, ov, p->iluk_level, bad_cell);
    if (s != RSV_OK) {
        delete R;
        return s;
    }
    *out = R;
    return RSV_OK;
}
