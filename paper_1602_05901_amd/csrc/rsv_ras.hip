// Restricted additive Schwarz (Cai & Sarkis; the paper's RAS subsection and
// its RAS_DATA / default-parameter figures): the grid is cut into px*py*pz
// boxes; subdomain s is its box plus every cell within matrix-graph distance
// `overlap`; the local matrix (A restricted to Omega_s, couplings leaving it
// dropped) gets a block ILU(0) in ascending global order; the apply restricts
// r to Omega_s, solves with the local factors and writes back only the cells
// s owns (restricted prolongation, no atomics, no averaging).
//
// Two GPU mappings compute the same local solves.
//
// Boxed (the default, `pipelined`): the subdomains' extended boxes (a box
// grown by `overlap` cells per side, clipped to the grid) are placed side by
// side in groups of G x G, each group padded to whole 8x8 tiles, in an array
// of boxes that forms one auxiliary grid (boxes stacked in z share tile
// columns: longer columns, fewer tiles, less of each column spent on the
// tile's diagonal ramp).  The local matrix is stored there with every
// coupling that leaves Omega_s set to zero; cells outside every Omega_s get an
// identity diagonal and no couplings.  The block-diagonal ILU(0) of that grid
// is exactly the set of local ILU(0)s (the natural order inside a box is the
// global order, and boxes share no couplings), and its pipelined tile sweeps
// exchange faces only inside a group, so every group advances at once, each
// tile's data streamed by its loader waves.  G = 1 pads every box alone; a
// larger G wastes less padding but chains the boxes of a group through the
// tiles they share.
// The apply gathers r into the auxiliary grid and runs both sweeps there; the
// backward sweep stores each cell's result into z only from the box that owns
// the cell (an index map delivered with the sweep's operands).
//
// Per subdomain: one workgroup per subdomain.  Omega_s's cells are listed by
// hyperplane i+j+k (ascending global index inside a plane); all local lower
// neighbours of a cell lie on the previous hyperplane, so a workgroup walks
// the planes with one barrier between planes.  Factors are stored
// structure-of-arrays over the concatenated local cell lists so that each
// plane's loads are coalesced.
#include "rsv_internal.h"

#include <algorithm>
#include <new>

namespace {

constexpr int RB = 1024;   // threads per subdomain workgroup

struct RasDev {
    int64_t n;                  // total local cells (sum |Omega_s|)
    const int32_t *slot;        // [n] tile-lane slot of the cell
    const int32_t *nb;          // [6][n] local index of neighbour -z,-y,-x,+x,+y,+z in Omega_s, or -1
    const uint8_t *owned;       // [n]
    const int64_t *pp;          // plane pointers (global offsets into the local arrays)
    const int32_t *sub_pp0;     // [nsub] first entry of subdomain s in pp
    const int32_t *sub_np;      // [nsub] number of planes
};

__global__ __launch_bounds__(RB) void k_ras_factor(RasDev R, const double *__restrict__ A, double *__restrict__ Lf,
                                                   double *__restrict__ Dinv, double *__restrict__ U,
                                                   int32_t *flags, Geo g)
{
    const int s = blockIdx.x;
    const int64_t n = R.n;
    const int np = R.sub_np[s];
    const int64_t *pp = R.pp + R.sub_pp0[s];
    for (int p = 0; p < np; ++p) {
        for (int64_t c = pp[p] + threadIdx.x; c < pp[p + 1]; c += RB) {
            const int64_t slot = R.slot[c];
            double D[9];
            for (int e = 0; e < 9; ++e) D[e] = A[aidx(slot, 27 + e)];
            for (int q = 0; q < 3; ++q) {   // -z, -y, -x
                const int32_t m = R.nb[q * n + c];
                double L[9];
                if (m >= 0) {
                    const int64_t ms = R.slot[m];
                    double Ack[9], Dk[9], Akc[9];
                    for (int e = 0; e < 9; ++e) {
                        Ack[e] = A[aidx(slot, q * 9 + e)];
                        Dk[e] = Dinv[e * n + m];
                        Akc[e] = A[aidx(ms, (6 - q) * 9 + e)];
                    }
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b)
                            L[3 * a + b] = Ack[3 * a] * Dk[b] + Ack[3 * a + 1] * Dk[3 + b] + Ack[3 * a + 2] * Dk[6 + b];
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b)
                            D[3 * a + b] -= L[3 * a] * Akc[b] + L[3 * a + 1] * Akc[3 + b] + L[3 * a + 2] * Akc[6 + b];
                } else {
                    for (int e = 0; e < 9; ++e) L[e] = 0.0;
                }
                for (int e = 0; e < 9; ++e) Lf[(q * 9 + e) * n + c] = L[e];
            }
            for (int q = 0; q < 3; ++q) {   // +x, +y, +z: A's blocks if the neighbour is in Omega_s
                const int32_t m = R.nb[(3 + q) * n + c];
                for (int e = 0; e < 9; ++e) U[(q * 9 + e) * n + c] = (m >= 0) ? A[aidx(slot, (4 + q) * 9 + e)] : 0.0;
            }
            double Di[9];
            if (!inv3(D, Di)) {
                int gx, gy, k;
                cell_of(g, slot, gx, gy, k);
                atomicOr(&flags[0], FLAG_PIVOT);
                atomicMin(&flags[1], (int32_t)row_of(g, gx, gy, k));
                for (int e = 0; e < 9; ++e) Di[e] = 0.0;
            }
            for (int e = 0; e < 9; ++e) Dinv[e * n + c] = Di[e];
        }
        __syncthreads();
    }
}

// Local vectors yl, zl are [3][n + 1]: entry n of each component is a
// permanent zero, the value of an absent neighbour.  Every load of a cell is
// issued unconditionally (absent neighbours read the zero entry; their factor
// blocks are zero), and the neighbour indices of a thread's first cell in the
// next plane are fetched during the current plane, so after each barrier a
// plane costs one memory round trip (the neighbour values, with the factor
// blocks and r loaded alongside) instead of one per branch.
template <typename T, int DIR>
struct RasCell {
    int64_t c, slot, m[3];
    __device__ void fetch(const RasDev &R, int64_t cc)
    {
        c = cc;
        slot = R.slot[cc];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int32_t mq = R.nb[(DIR == 0 ? q : 3 + q) * R.n + cc];
            m[q] = mq >= 0 ? mq : R.n;
        }
    }
};

template <typename T>
__device__ __forceinline__ void ras_fwd_cell(const RasCell<T, 0> &C, int64_t n, int64_t n1, const T *__restrict__ Lf,
                                             const double *__restrict__ r, T *__restrict__ yl)
{
    T l[27], rr[3], y[3][3];
#pragma unroll
    for (int e = 0; e < 27; ++e) l[e] = Lf[e * n + C.c];
#pragma unroll
    for (int a = 0; a < 3; ++a) rr[a] = (T)r[vidx(C.slot, a)];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int b = 0; b < 3; ++b) y[q][b] = yl[b * n1 + C.m[q]];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T acc = 0;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            acc += l[q * 9 + 3 * a] * y[q][0] + l[q * 9 + 3 * a + 1] * y[q][1] + l[q * 9 + 3 * a + 2] * y[q][2];
        yl[a * n1 + C.c] = rr[a] - acc;
    }
}

template <typename T>
__device__ __forceinline__ void ras_bwd_cell(const RasCell<T, 1> &C, const RasDev &R, int64_t n1, const T *__restrict__ U,
                                             const T *__restrict__ Dinv, const T *__restrict__ yl, T *__restrict__ zl,
                                             double *__restrict__ z)
{
    const int64_t n = R.n;
    T u[27], dd[9], yy[3], zz[3][3];
#pragma unroll
    for (int e = 0; e < 27; ++e) u[e] = U[e * n + C.c];
#pragma unroll
    for (int e = 0; e < 9; ++e) dd[e] = Dinv[e * n + C.c];
#pragma unroll
    for (int a = 0; a < 3; ++a) yy[a] = yl[a * n1 + C.c];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int b = 0; b < 3; ++b) zz[q][b] = zl[b * n1 + C.m[q]];
    T tv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T acc = 0;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            acc += u[q * 9 + 3 * a] * zz[q][0] + u[q * 9 + 3 * a + 1] * zz[q][1] + u[q * 9 + 3 * a + 2] * zz[q][2];
        tv[a] = yy[a] - acc;
    }
    T out[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a] = dd[3 * a] * tv[0] + dd[3 * a + 1] * tv[1] + dd[3 * a + 2] * tv[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) zl[a * n1 + C.c] = out[a];
    if (R.owned[C.c])
#pragma unroll
        for (int a = 0; a < 3; ++a) z[vidx(C.slot, a)] = (double)out[a];
}

template <typename T>
__global__ __launch_bounds__(RB) void k_ras_apply(RasDev R, const T *__restrict__ Lf, const T *__restrict__ Dinv,
                                                  const T *__restrict__ U, const double *__restrict__ r,
                                                  T *__restrict__ yl, T *__restrict__ zl, double *__restrict__ z)
{
    const int s = blockIdx.x;
    const int64_t n = R.n, n1 = n + 1;
    const int np = R.sub_np[s];
    const int64_t *pp = R.pp + R.sub_pp0[s];
    const int tid = threadIdx.x;
    {
        RasCell<T, 0> nxt{};
        if (pp[0] + tid < pp[1]) nxt.fetch(R, pp[0] + tid);
        for (int p = 0; p < np; ++p) {
            const int64_t c0 = pp[p] + tid, end = pp[p + 1];
            const RasCell<T, 0> cur = nxt;
            if (p + 1 < np && pp[p + 1] + tid < pp[p + 2]) nxt.fetch(R, pp[p + 1] + tid);
            if (c0 < end) ras_fwd_cell<T>(cur, n, n1, Lf, r, yl);
            for (int64_t c = c0 + RB; c < end; c += RB) {
                RasCell<T, 0> C;
                C.fetch(R, c);
                ras_fwd_cell<T>(C, n, n1, Lf, r, yl);
            }
            __syncthreads();
        }
    }
    {
        RasCell<T, 1> nxt{};
        if (np > 0 && pp[np - 1] + tid < pp[np]) nxt.fetch(R, pp[np - 1] + tid);
        for (int p = np - 1; p >= 0; --p) {
            const int64_t c0 = pp[p] + tid, end = pp[p + 1];
            const RasCell<T, 1> cur = nxt;
            if (p > 0 && pp[p - 1] + tid < pp[p]) nxt.fetch(R, pp[p - 1] + tid);
            if (c0 < end) ras_bwd_cell<T>(cur, R, n1, U, Dinv, yl, zl, z);
            for (int64_t c = c0 + RB; c < end; c += RB) {
                RasCell<T, 1> C;
                C.fetch(R, c);
                ras_bwd_cell<T>(C, R, n1, U, Dinv, yl, zl, z);
            }
            __syncthreads();
        }
    }
}

__global__ void k_cvt(int64_t n, const double *__restrict__ a, float *__restrict__ b)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) b[e] = (float)a[e];
}

static int64_t split_index(int64_t v, int64_t len, int64_t p)
{
    const int64_t base = len / p, rem = len % p, big = rem * (base + 1);
    if (v < big) return v / (base + 1);
    return rem + (v - big) / base;
}
static int64_t split_start(int64_t b, int64_t len, int64_t p)
{
    const int64_t base = len / p, rem = len % p;
    return b * base + std::min(b, rem);
}

struct Ras : PcImpl {
    rsv_matrix *M = nullptr;
    rsv_ctx *c = nullptr;
    bool fp32 = false;
    int nsub = 0;
    int64_t n = 0;
    int32_t *slot = nullptr, *nb = nullptr, *sub_pp0 = nullptr, *sub_np = nullptr;
    uint8_t *owned = nullptr;
    int64_t *pp = nullptr;
    double *Lf = nullptr, *Dinv = nullptr, *U = nullptr;
    float *Lf32 = nullptr, *Dinv32 = nullptr, *U32 = nullptr;
    void *yl = nullptr, *zl = nullptr;
    int64_t nbytes = 0;

    ~Ras() override
    {
        dev_free(slot); dev_free(nb); dev_free(sub_pp0); dev_free(sub_np); dev_free(owned); dev_free(pp);
        dev_free(Lf); dev_free(Dinv); dev_free(U); dev_free(Lf32); dev_free(Dinv32); dev_free(U32);
        dev_free(yl); dev_free(zl);
    }
    int64_t bytes() const override { return nbytes; }

    rsv_status alloc(void **p, size_t b)
    {
        rsv_status s = dev_alloc(c, p, b);
        if (s == RSV_OK) nbytes += (int64_t)b;
        return s;
    }
    template <typename V>
    rsv_status upload(V **p, const std::vector<V> &h)
    {
        rsv_status s = alloc((void **)p, h.size() * sizeof(V));
        if (s != RSV_OK) return s;
        RSV_HIP(c, hipMemcpy(*p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
        return RSV_OK;
    }

    RasDev dev() const { return RasDev{n, slot, nb, owned, pp, sub_pp0, sub_np}; }

    rsv_status setup(const rsv_pc_params *p, int64_t *bad_cell)
    {
        const Geo &g = M->g->geo;
        const int px = p->ras_px, py = p->ras_py, pz = p->ras_pz, ov = p->ras_overlap;
        if (px < 1 || py < 1 || pz < 1 || px > g.nx || py > g.ny || pz > g.nz || ov < 0)
            return set_err(c, RSV_ERR_ARG, "bad RAS partition");
        nsub = px * py * pz;
        const int64_t ncell = M->g->ncell;
        auto cid = [&](int i, int j, int k) { return ((int64_t)k * g.ny + j) * g.nx + i; };
        std::vector<int32_t> stamp(ncell, -1), dist(ncell, 0);
        std::vector<int32_t> h_slot, h_nb6;   // nb filled after sizes are known
        std::vector<uint8_t> h_owned;
        std::vector<int64_t> h_pp;
        std::vector<int32_t> h_pp0(nsub), h_np(nsub);
        std::vector<std::vector<int64_t>> lists(nsub);
        std::vector<int64_t> queue;
        for (int s = 0; s < nsub; ++s) {
            const int sx = s % px, sy = (s / px) % py, sz = s / (px * py);
            const int x0 = (int)split_start(sx, g.nx, px), x1 = (int)split_start(sx + 1, g.nx, px);
            const int y0 = (int)split_start(sy, g.ny, py), y1 = (int)split_start(sy + 1, g.ny, py);
            const int z0 = (int)split_start(sz, g.nz, pz), z1 = (int)split_start(sz + 1, g.nz, pz);
            queue.clear();
            for (int k = z0; k < z1; ++k)
                for (int j = y0; j < y1; ++j)
                    for (int i = x0; i < x1; ++i) {
                        const int64_t C = cid(i, j, k);
                        stamp[C] = s;
                        dist[C] = 0;
                        queue.push_back(C);
                    }
            // breadth-first search over the stencil graph up to distance `ov`
            for (size_t h = 0; h < queue.size(); ++h) {
                const int64_t C = queue[h];
                if (dist[C] >= ov) continue;
                const int i = (int)(C % g.nx), j = (int)((C / g.nx) % g.ny), k = (int)(C / ((int64_t)g.nx * g.ny));
                for (int d = 0; d < 7; ++d) {
                    if (d == 3) continue;
                    int di, dj, dk;
                    dir_off(d, di, dj, dk);
                    const int a = i + di, b = j + dj, e = k + dk;
                    if (a < 0 || a >= g.nx || b < 0 || b >= g.ny || e < 0 || e >= g.nz) continue;
                    const int64_t N = cid(a, b, e);
                    if (stamp[N] == s) continue;
                    stamp[N] = s;
                    dist[N] = dist[C] + 1;
                    queue.push_back(N);
                }
            }
            // order: hyperplane, then ascending global index
            std::vector<int64_t> &lst = lists[s];
            lst = queue;
            std::sort(lst.begin(), lst.end(), [&](int64_t a, int64_t b) {
                const int64_t pa = a % g.nx + (a / g.nx) % g.ny + a / ((int64_t)g.nx * g.ny);
                const int64_t pb = b % g.nx + (b / g.nx) % g.ny + b / ((int64_t)g.nx * g.ny);
                return pa != pb ? pa < pb : a < b;
            });
        }
        int64_t total = 0;
        for (int s = 0; s < nsub; ++s) total += (int64_t)lists[s].size();
        if (total >= ((int64_t)1 << 31)) return set_err(c, RSV_ERR_ARG, "RAS local size exceeds int32");
        n = total;
        h_slot.resize(n);
        h_owned.resize(n);
        h_nb6.assign(6 * n, -1);
        std::vector<int32_t> loc(ncell, -1);
        int64_t off = 0;
        for (int s = 0; s < nsub; ++s) {
            const std::vector<int64_t> &lst = lists[s];
            for (size_t q = 0; q < lst.size(); ++q) loc[lst[q]] = (int32_t)(off + q);
            h_pp0[s] = (int32_t)h_pp.size();
            int64_t prev_plane = -1;
            int nplanes = 0;
            for (size_t q = 0; q < lst.size(); ++q) {
                const int64_t C = lst[q];
                const int i = (int)(C % g.nx), j = (int)((C / g.nx) % g.ny), k = (int)(C / ((int64_t)g.nx * g.ny));
                const int64_t pl = i + j + k;
                if (pl != prev_plane) {
                    // planes are contiguous (every plane between first and last is non-empty
                    // for a face-connected set); record empty planes too for safety
                    if (prev_plane >= 0)
                        for (int64_t e = prev_plane + 1; e < pl; ++e) { h_pp.push_back(off + (int64_t)q); ++nplanes; }
                    h_pp.push_back(off + (int64_t)q);
                    ++nplanes;
                    prev_plane = pl;
                }
                const int64_t L = off + (int64_t)q;
                h_slot[L] = (int32_t)slot_of(g, i, j, k);
                const int sx = (int)split_index(i, g.nx, px), sy = (int)split_index(j, g.ny, py),
                          sz = (int)split_index(k, g.nz, pz);
                h_owned[L] = ((sz * py + sy) * px + sx) == s;
            }
            h_pp.push_back(off + (int64_t)lst.size());
            h_np[s] = nplanes;
            // local neighbour indices
            const int dirs[6] = {0, 1, 2, 4, 5, 6};
            for (size_t q = 0; q < lst.size(); ++q) {
                const int64_t C = lst[q];
                const int i = (int)(C % g.nx), j = (int)((C / g.nx) % g.ny), k = (int)(C / ((int64_t)g.nx * g.ny));
                for (int d6 = 0; d6 < 6; ++d6) {
                    int di, dj, dk;
                    dir_off(dirs[d6], di, dj, dk);
                    const int a = i + di, b = j + dj, e = k + dk;
                    if (a < 0 || a >= g.nx || b < 0 || b >= g.ny || e < 0 || e >= g.nz) continue;
                    const int32_t m = loc[cid(a, b, e)];
                    h_nb6[(int64_t)d6 * n + off + (int64_t)q] = m;
                }
            }
            for (size_t q = 0; q < lst.size(); ++q) loc[lst[q]] = -1;
            off += (int64_t)lst.size();
        }
        rsv_status st = upload(&slot, h_slot);
        if (st == RSV_OK) st = upload(&nb, h_nb6);
        if (st == RSV_OK) st = upload(&owned, h_owned);
        if (st == RSV_OK) st = upload(&pp, h_pp);
        if (st == RSV_OK) st = upload(&sub_pp0, h_pp0);
        if (st == RSV_OK) st = upload(&sub_np, h_np);
        if (st == RSV_OK) st = alloc((void **)&Lf, (size_t)n * 27 * sizeof(double));
        if (st == RSV_OK) st = alloc((void **)&Dinv, (size_t)n * 9 * sizeof(double));
        if (st == RSV_OK) st = alloc((void **)&U, (size_t)n * 27 * sizeof(double));
        if (st != RSV_OK) return st;
        st = flags_reset(c);
        if (st != RSV_OK) return st;
        {
            ProfScope ps(c, RSV_K_FACTOR);
            hipLaunchKernelGGL(k_ras_factor, dim3(nsub), dim3(RB), 0, c->stream, dev(), M->d_A, Lf, Dinv, U, c->d_flags, g);
        }
        RSV_LAUNCH(c);
        st = flags_check(c, bad_cell);
        if (st != RSV_OK) return st;
        if (fp32) {
            st = alloc((void **)&Lf32, (size_t)n * 27 * sizeof(float));
            if (st == RSV_OK) st = alloc((void **)&Dinv32, (size_t)n * 9 * sizeof(float));
            if (st == RSV_OK) st = alloc((void **)&U32, (size_t)n * 27 * sizeof(float));
            if (st == RSV_OK) st = alloc(&yl, (size_t)(n + 1) * 3 * sizeof(float));
            if (st == RSV_OK) st = alloc(&zl, (size_t)(n + 1) * 3 * sizeof(float));
            if (st != RSV_OK) return st;
            hipLaunchKernelGGL(k_cvt, dim3(2048), dim3(256), 0, c->stream, n * 27, Lf, Lf32);
            hipLaunchKernelGGL(k_cvt, dim3(2048), dim3(256), 0, c->stream, n * 9, Dinv, Dinv32);
            hipLaunchKernelGGL(k_cvt, dim3(2048), dim3(256), 0, c->stream, n * 27, U, U32);
            RSV_LAUNCH(c);
            RSV_HIP(c, hipStreamSynchronize(c->stream));
            dev_free(Lf); Lf = nullptr;
            dev_free(Dinv); Dinv = nullptr;
            dev_free(U); U = nullptr;
            nbytes -= n * 63 * (int64_t)sizeof(double);
        } else {
            st = alloc(&yl, (size_t)(n + 1) * 3 * sizeof(double));
            if (st == RSV_OK) st = alloc(&zl, (size_t)(n + 1) * 3 * sizeof(double));
            if (st != RSV_OK) return st;
        }
        // the zero entries (index n of each component) of the local vectors
        RSV_HIP(c, hipMemsetAsync(yl, 0, (size_t)(n + 1) * 3 * (fp32 ? sizeof(float) : sizeof(double)), c->stream));
        RSV_HIP(c, hipMemsetAsync(zl, 0, (size_t)(n + 1) * 3 * (fp32 ? sizeof(float) : sizeof(double)), c->stream));
        RSV_HIP(c, hipStreamSynchronize(c->stream));
        return RSV_OK;
    }

    rsv_status apply(const double *r, double *z) override
    {
        ProfScope ps(c, RSV_K_RAS);
        if (fp32)
            hipLaunchKernelGGL(k_ras_apply<float>, dim3(nsub), dim3(RB), 0, c->stream, dev(), Lf32, Dinv32, U32, r,
                               (float *)yl, (float *)zl, z);
        else
            hipLaunchKernelGGL(k_ras_apply<double>, dim3(nsub), dim3(RB), 0, c->stream, dev(), Lf, Dinv, U, r,
                               (double *)yl, (double *)zl, z);
        RSV_LAUNCH(c);
        return RSV_OK;
    }
};


// ---------------------------------------------------------------- boxed mapping

// Placement of the subdomain boxes in the auxiliary grid.  Boxes sit in
// groups of G x G, side by side at a pitch of BW (BH) cells, each group padded
// to whole 8 x 8 tiles (GXp x GYp cells); SX box columns (a multiple of G) per
// row, SZ boxes stacked per tile column, EZ layers each.  A box's slot in the
// arrangement is s = (by * SX + bx) * SZ + bz.
struct BoxDev {
    int32_t nsub, SX, SZ, G, BW, BH, GXp, GYp, EZ, ov;
    const int32_t *box;   // [nsub][9]: core x0,x1,y0,y1,z0,z1; extended-box origin ex,ey,ez
};

__host__ __device__ inline int box_dist(int v, int lo, int hi) { return v < lo ? lo - v : (v >= hi ? v - hi + 1 : 0); }

// Omega_s: cells within graph distance ov of the core box
__host__ __device__ inline bool in_omega(const int32_t *q, int x, int y, int z, int ov)
{
    return box_dist(x, q[0], q[1]) + box_dist(y, q[2], q[3]) + box_dist(z, q[4], q[5]) <= ov;
}

// The global cell that auxiliary cell (X, Y, k) stands for; false when it is
// padding, outside the grid or outside Omega_s of its box s.
__host__ __device__ inline bool aux_cell(const BoxDev &B, const int32_t *box, const Geo &g, int X, int Y, int k, int &s,
                                         int &gx, int &gy, int &gz)
{
    const int gxi = X / B.GXp, xx = X - gxi * B.GXp, bi = xx / B.BW;
    const int gyi = Y / B.GYp, yy = Y - gyi * B.GYp, bj = yy / B.BH;
    if (bi >= B.G || bj >= B.G) return false;   // group padding
    const int bx = gxi * B.G + bi, by = gyi * B.G + bj, bz = k / B.EZ;
    s = (by * B.SX + bx) * B.SZ + bz;
    if (s >= B.nsub) return false;
    const int32_t *q = box + 9 * s;
    gx = q[6] + (xx - bi * B.BW);
    gy = q[7] + (yy - bj * B.BH);
    gz = q[8] + k % B.EZ;
    if (gx >= g.nx || gy >= g.ny || gz >= g.nz) return false;
    return in_omega(q, gx, gy, gz, B.ov);
}

// local matrix of every subdomain in the auxiliary grid
__global__ __launch_bounds__(256) void k_rasb_build(Geo ga, Geo g, BoxDev B, const double *__restrict__ A,
                                                   double *__restrict__ Aa)
{
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= ga.nslot) return;
    int X, Y, k, s = 0, gx = 0, gy = 0, gz = 0;
    const bool real = cell_of(ga, slot, X, Y, k);
    const bool in = real && aux_cell(B, B.box, g, X, Y, k, s, gx, gy, gz);
    const int64_t gsl = in ? slot_of(g, gx, gy, gz) : 0;
    for (int d = 0; d < 7; ++d) {
        bool keep = in;
        if (in && d != 3) {
            int di, dj, dk;
            dir_off(d, di, dj, dk);
            const int a = gx + di, b = gy + dj, e = gz + dk;
            keep = a >= 0 && a < g.nx && b >= 0 && b < g.ny && e >= 0 && e < g.nz && in_omega(B.box + 9 * s, a, b, e, B.ov);
        }
        for (int e = 0; e < 9; ++e) {
            const double id = (d == 3 && real && (e == 0 || e == 4 || e == 8)) ? 1.0 : 0.0;
            Aa[aidx(slot, d * 9 + e)] = keep ? A[aidx(gsl, d * 9 + e)] : (in ? 0.0 : id);
        }
    }
}

// index maps of the auxiliary grid: gin[s] = the grid slot of the Omega cell
// that auxiliary slot s holds (-1: none); gout[s] = the same when the cell's
// own box is s's box (restricted prolongation), else -1
__global__ __launch_bounds__(256) void k_rasb_maps(Geo ga, Geo g, BoxDev B, int32_t *__restrict__ gin,
                                                  int32_t *__restrict__ gout)
{
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= ga.nslot) return;
    int X, Y, k, s, gx, gy, gz;
    const bool in = cell_of(ga, slot, X, Y, k) && aux_cell(B, B.box, g, X, Y, k, s, gx, gy, gz);
    const int32_t m = in ? (int32_t)slot_of(g, gx, gy, gz) : -1;
    gin[slot] = m;
    gout[slot] = (in && in_omega(B.box + 9 * s, gx, gy, gz, 0)) ? m : -1;
}

// restriction: r on Omega_s into each box (zero elsewhere)
__global__ __launch_bounds__(256) void k_rasb_gather(int64_t nslot, const int32_t *__restrict__ gin,
                                                    const double *__restrict__ r, double *__restrict__ ra)
{
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= nslot) return;
    const int32_t m = gin[slot];
    const int64_t mm = m >= 0 ? m : 0;
#pragma unroll
    for (int p = 0; p < 3; ++p) ra[vidx(slot, p)] = m >= 0 ? r[vidx(mm, p)] : 0.0;
}

struct RasBoxed : PcImpl {
    rsv_matrix *M = nullptr;
    rsv_ctx *c = nullptr;
    BoxDev B{};
    std::vector<int32_t> h_box;
    int32_t *d_box = nullptr;
    rsv_grid *ga = nullptr;          // auxiliary grid of boxes
    rsv_matrix Ma{};                 // local matrices in it
    PcImpl *ilu = nullptr;           // its block-diagonal BILU0, writing z through gout
    int32_t *gin = nullptr, *gout = nullptr;
    double *ra = nullptr;
    int64_t nbytes = 0;
    bool too_large = false;          // the boxes do not fit one auxiliary grid

    ~RasBoxed() override
    {
        delete ilu;
        dev_free(Ma.d_A);
        dev_free(ra);
        dev_free(gin);
        dev_free(gout);
        dev_free(d_box);
        rsv_grid_destroy(ga);
    }
    int64_t bytes() const override { return nbytes + (ilu ? ilu->bytes() : 0); }

    rsv_status alloc(void **p, size_t b)
    {
        rsv_status s = dev_alloc(c, p, b);
        if (s == RSV_OK) nbytes += (int64_t)b;
        return s;
    }

    rsv_status setup(const rsv_pc_params *p, int64_t *bad_cell)
    {
        const Geo &g = M->g->geo;
        const int px = p->ras_px, py = p->ras_py, pz = p->ras_pz, ov = p->ras_overlap;
        if (px < 1 || py < 1 || pz < 1 || px > g.nx || py > g.ny || pz > g.nz || ov < 0 || p->ras_stack < 0 ||
            p->ras_group < 0 || p->ras_group > 16)
            return set_err(c, RSV_ERR_ARG, "bad RAS partition");
        const int nsub = px * py * pz;
        h_box.assign((size_t)nsub * 9, 0);
        int EX = 1, EY = 1, EZ = 1;
        for (int s = 0; s < nsub; ++s) {
            const int sx = s % px, sy = (s / px) % py, sz = s / (px * py);
            int32_t *q = h_box.data() + 9 * s;
            q[0] = (int32_t)split_start(sx, g.nx, px); q[1] = (int32_t)split_start(sx + 1, g.nx, px);
            q[2] = (int32_t)split_start(sy, g.ny, py); q[3] = (int32_t)split_start(sy + 1, g.ny, py);
            q[4] = (int32_t)split_start(sz, g.nz, pz); q[5] = (int32_t)split_start(sz + 1, g.nz, pz);
            q[6] = std::max(0, q[0] - ov); q[7] = std::max(0, q[2] - ov); q[8] = std::max(0, q[4] - ov);
            EX = std::max(EX, std::min(g.nx, q[1] + ov) - q[6]);
            EY = std::max(EY, std::min(g.ny, q[3] + ov) - q[7]);
            EZ = std::max(EZ, std::min(g.nz, q[5] + ov) - q[8]);
        }
        // boxes per tile column (SZ) and per group side (G); a group of G x G boxes
        // padded to whole tiles wastes less than G^2 boxes padded one by one
        auto arrange = [&](int sz, int gg, int &ngx, int &ngy) {
            const int nl = (nsub + sz - 1) / sz;
            const int ng = (nl + gg * gg - 1) / (gg * gg);
            ngx = 1;
            while (ngx * ngx < ng) ++ngx;
            ngy = (ng + ngx - 1) / ngx;
        };
        int grp = p->ras_group > 0 ? p->ras_group : 1;
        auto fit = [&](int sz, int gg) {     // no group larger than the boxes of one layer fill
            const int nl = (nsub + sz - 1) / sz;
            while (gg > 1 && gg * gg > nl) --gg;
            return gg;
        };
        auto tiles = [&](int sz, int gg) {   // tiles of the filled groups
            const int nl = (nsub + sz - 1) / sz;
            gg = fit(sz, gg);
            return (int64_t)((nl + gg * gg - 1) / (gg * gg)) * ((gg * EX + 7) / 8) * ((gg * EY + 7) / 8);
        };
        // as many boxes per tile column as keep at least four tiles per CU
        int SZ = 1;
        if (p->ras_stack > 0)
            SZ = std::min(nsub, p->ras_stack);
        else
            while (SZ < nsub && tiles(2 * SZ, grp) >= 4 * (int64_t)c->num_cu) SZ *= 2;
        grp = fit(SZ, grp);
        int ngx, ngy;
        arrange(SZ, grp, ngx, ngy);
        const int GXp = (grp * EX + 7) / 8 * 8, GYp = (grp * EY + 7) / 8 * 8;
        const int SX = ngx * grp;
        B = BoxDev{nsub, SX, SZ, grp, EX, EY, GXp, GYp, EZ, ov, nullptr};
        // the auxiliary grid must fit the tile-lane index range (3 * slots < 2^31);
        // otherwise the caller falls back to the per-subdomain mapping
        const int64_t aux_slots = (int64_t)ngx * (GXp / 8) * ngy * (GYp / 8) * SZ * EZ * 64;
        if (3 * aux_slots >= ((int64_t)1 << 31)) {
            too_large = true;
            return set_err(c, RSV_ERR_ARG, "RAS boxes exceed the auxiliary grid's index range");
        }
        // factorisation planes inside each box (the boxes share no couplings)
        rsv_status st = grid_create_planes(c, ngx * GXp, ngy * GYp, SZ * EZ, RSV_BOTTOM_UP, GXp, GYp, EZ, &ga);
        if (st != RSV_OK) return st;
        const Geo &G = ga->geo;
        st = alloc((void **)&d_box, h_box.size() * sizeof(int32_t));
        if (st == RSV_OK) st = alloc((void **)&Ma.d_A, (size_t)(G.nslot / 64) * 63 * 64 * sizeof(double));
        if (st == RSV_OK) st = alloc((void **)&ra, (size_t)ga->nv * sizeof(double));
        if (st == RSV_OK) st = alloc((void **)&gin, (size_t)G.nslot * sizeof(int32_t));
        if (st == RSV_OK) st = alloc((void **)&gout, (size_t)G.nslot * sizeof(int32_t));
        if (st != RSV_OK) return st;
        RSV_HIP(c, hipMemcpy(d_box, h_box.data(), h_box.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        B.box = d_box;
        Ma.g = ga;
        hipLaunchKernelGGL(k_rasb_build, dim3((unsigned)((G.nslot + 255) / 256)), dim3(256), 0, c->stream, G, g, B,
                           M->d_A, Ma.d_A);
        hipLaunchKernelGGL(k_rasb_maps, dim3((unsigned)((G.nslot + 255) / 256)), dim3(256), 0, c->stream, G, g, B,
                           gin, gout);
        RSV_LAUNCH(c);
        int64_t bad = -1;
        st = bilu0_create_boxed(&Ma, p, GXp / 8, GYp / 8, gout, &ilu, &bad);
        if (st == RSV_ERR_ZERO_PIVOT && bad >= 0 && bad_cell) {
            // the auxiliary row of the failing pivot, as the cell of the grid
            const int X = (int)(bad % G.nx), Y = (int)((bad / G.nx) % G.ny), k = (int)(bad / ((int64_t)G.nx * G.ny));
            int s, gx, gy, gz;
            if (aux_cell(B, h_box.data(), g, X, Y, k, s, gx, gy, gz)) *bad_cell = row_of(g, gx, gy, gz);
        }
        return st;
    }

    rsv_status apply(const double *r, double *z) override
    {
        ProfScope ps(c, RSV_K_RAS);
        const Geo &G = ga->geo;
        hipLaunchKernelGGL(k_rasb_gather, dim3((unsigned)((G.nslot + 255) / 256)), dim3(256), 0, c->stream, G.nslot, gin,
                           r, ra);
        RSV_LAUNCH(c);
        // the backward sweep stores each owned cell's result straight into z
        return ilu->apply(ra, z);
    }
};

}  // namespace

rsv_status ras_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, int64_t *bad_cell)
{
    rsv_ctx *c = A->g->ctx;
    if (p->pipelined) {
        RasBoxed *R = new (std::nothrow) RasBoxed();
        if (!R) return set_err(c, RSV_ERR_OOM, "ras");
        R->M = A;
        R->c = c;
        rsv_status s = R->setup(p, bad_cell);
        if (s == RSV_OK) {
            *out = R;
            return RSV_OK;
        }
        const bool fall_back = R->too_large;
        delete R;
        if (!fall_back) return s;
        // too many or too large boxes for one auxiliary grid: per-subdomain mapping
    }
    Ras *R = new (std::nothrow) Ras();
    if (!R) return set_err(c, RSV_ERR_OOM, "ras");
    R->M = A;
    R->c = c;
    R->fp32 = (p->precision == RSV_FP32);
    rsv_status s = R->setup(p, bad_cell);
    if (s != RSV_OK) {
        delete R;
        return s;
    }
    *out = R;
    return RSV_OK;
}
