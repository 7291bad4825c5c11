// Hilbert space-filling-curve keys of points and grid cells, the equal-count
// cut of the curve into parts, and the partition-quality measures
// (Space-filling Partitioning Method section: Hilbert orders, the table-driven
// algorithm, Algorithm "Space-filling curve method", Partition Quality).
//
// Keys: each point of [0,1]^3 is scaled by 2^32 - 1 and truncated to three
// 32-bit coordinates; level l (l = 0 first) reads bit 31 - l of each (x
// weight 4, y 2, z 1 in the octant index) and walks the 24-state machine of
// the paper's ordering and orientation tables, emitting one base-8 digit per
// level, most significant first (a 3*levels-bit integer key).
//
// Partition: the cells in (key, index) order are cut into nparts runs of
// sizes differing by at most one (the cell of rank r goes to part
// floor(r nparts / n)).  The order comes from a stable least-significant-
// digit radix sort over the 3*levels key bits, 8 bits per pass: per-tile
// digit histograms, one exclusive scan, and a scatter in which each tile
// ranks its elements by digit with wave ballots (eight ballots match the
// lanes holding the same digit) so equal digits keep their input order.
#include "rsv_internal.h"

#include <algorithm>
#include <vector>

namespace {

// The paper's ordering table: per state, the digit of octant t in bits 3t..3t+2.
__constant__ uint32_t c_digits[24] = {
    0xab18f8u, 0xb374c8u, 0xb919d8u, 0xf8195au,
    0x2374ecu, 0x2b50fcu, 0x68197eu, 0xb13dc8u,
    0xf03d4au, 0x70754eu, 0xaa3c78u, 0xf350cau,
    0x283d7cu, 0x213decu, 0x7151ceu, 0xba7458u,
    0xfa505au, 0x6a507eu, 0xe23c6au, 0x3951dcu,
    0x38755cu, 0x62746eu, 0xe318eau, 0x6119eeu,
};
// The paper's orientation table: per state, the next state of octant t in bits 5t..5t+4.
__constant__ uint64_t c_next[24] = {
    0x000a220cc1ull, 0x094890a0e0ull, 0x14c40a5ecfull, 0xb428678ee3ull,
    0x6d8342308bull, 0x994055d196ull, 0x11923a9811ull, 0x3b0eb6b82aull,
    0x5a98e92128ull, 0x3c4c14a515ull, 0x529b063e27ull, 0x402cb2a5cbull,
    0xa3113530b2ull, 0x249a53cda8ull, 0x099ce89d77ull, 0x7d2757aa42ull,
    0x90c509c6b0ull, 0x7c6f174146ull, 0x834f145652ull, 0x28a7383483ull,
    0x63c64a51b0ull, 0x55dcfacaa9ull, 0x1917709ad6ull, 0x056f648aeeull,
};

enum { FLAG_RANGE = 16 };

__device__ inline uint32_t unit_to_u32(double c) { return (uint32_t)(c * 4294967295.0); }

__device__ inline uint64_t hilbert_key(const uint32_t *dig, const uint64_t *nxt, uint32_t u0, uint32_t u1,
                                       uint32_t u2, int levels)
{
    uint32_t st = 0;
    uint64_t k = 0;
    for (int l = 0; l < levels; ++l) {
        const int b = 31 - l;
        const uint32_t t = (((u0 >> b) & 1u) << 2) | (((u1 >> b) & 1u) << 1) | ((u2 >> b) & 1u);
        k = (k << 3) | ((dig[st] >> (3 * t)) & 7u);
        st = (uint32_t)((nxt[st] >> (5 * t)) & 31u);
    }
    return k;
}

// the two tables staged in LDS (per-lane state indices differ)
#define RSV_HSFC_TABLES                                   \
    __shared__ uint32_t s_dig[24];                        \
    __shared__ uint64_t s_nxt[24];                        \
    if (threadIdx.x < 24) {                               \
        s_dig[threadIdx.x] = c_digits[threadIdx.x];       \
        s_nxt[threadIdx.x] = c_next[threadIdx.x];         \
    }                                                     \
    __syncthreads();

__global__ __launch_bounds__(256) void k_hsfc_points(int64_t n, const double *__restrict__ xyz, int levels,
                                                     uint64_t *__restrict__ keys, int32_t *flags)
{
    RSV_HSFC_TABLES
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const double x = xyz[3 * e], y = xyz[3 * e + 1], z = xyz[3 * e + 2];
        if (!(x >= 0.0 && x <= 1.0 && y >= 0.0 && y <= 1.0 && z >= 0.0 && z <= 1.0)) {
            atomicOr(&flags[0], (int32_t)FLAG_RANGE);
            keys[e] = 0;
            continue;
        }
        keys[e] = hilbert_key(s_dig, s_nxt, unit_to_u32(x), unit_to_u32(y), unit_to_u32(z), levels);
    }
}

// keys of the grid's cells by block row: centroid ((i, j, k) + 1/2) / L with
// L the largest extent, so the cells stay cubes in [0,1)^3
__global__ __launch_bounds__(256) void k_hsfc_grid(Geo g, int levels, uint64_t *__restrict__ keys)
{
    RSV_HSFC_TABLES
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const double L = (double)max(g.nx, max(g.ny, g.nz));
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) {
        const int i = (int)(r % g.nx), j = (int)((r / g.nx) % g.ny);
        const int kk = (int)(r / ((int64_t)g.nx * g.ny));
        const int k = (g.ordering == RSV_TOP_DOWN) ? g.nz - 1 - kk : kk;
        keys[r] = hilbert_key(s_dig, s_nxt, unit_to_u32(((double)i + 0.5) / L), unit_to_u32(((double)j + 0.5) / L),
                              unit_to_u32(((double)k + 0.5) / L), levels);
    }
}

// ---------------------------------------------------------------- radix sort
constexpr int RS_ITEMS = 16, RS_TILE = 256 * RS_ITEMS;

// per-tile histogram of the digit at `shift`, stored digit-major: hist[d * ntile + tile]
__global__ __launch_bounds__(256) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                 uint32_t *__restrict__ hist, int ntile)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int it = 0; it < RS_ITEMS; ++it) {
        const int64_t e = base + it * 256 + threadIdx.x;
        if (e < n) atomicAdd(&h[(uint32_t)(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntile + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of a tile of 4096 counts (16 consecutive per thread); the
// tile total goes to sums[tile]
__global__ __launch_bounds__(256) void k_scan_tile(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                   int64_t m, uint32_t *__restrict__ sums)
{
    __shared__ uint32_t t[256];
    const int64_t base = (int64_t)blockIdx.x * RS_TILE + (int64_t)threadIdx.x * RS_ITEMS;
    uint32_t v[RS_ITEMS], s = 0;
#pragma unroll
    for (int q = 0; q < RS_ITEMS; ++q) {
        v[q] = (base + q < m) ? in[base + q] : 0u;
        s += v[q];
    }
    t[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {   // inclusive scan of the thread totals
        const uint32_t a = ((int)threadIdx.x >= off) ? t[threadIdx.x - off] : 0u;
        __syncthreads();
        t[threadIdx.x] += a;
        __syncthreads();
    }
    uint32_t run = t[threadIdx.x] - s;
#pragma unroll
    for (int q = 0; q < RS_ITEMS; ++q) {
        if (base + q < m) out[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == 255) sums[blockIdx.x] = t[255];
}

__global__ __launch_bounds__(256) void k_scan_add(uint32_t *__restrict__ out, int64_t m,
                                                  const uint32_t *__restrict__ add)
{
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const uint32_t a = add[blockIdx.x];
    for (int q = threadIdx.x; q < RS_TILE; q += 256)
        if (base + q < m) out[base + q] += a;
}

// stable scatter of one digit pass; iin == nullptr: the indices are the positions
__global__ __launch_bounds__(256) void k_rs_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ iin,
                                                    uint64_t *__restrict__ kout, uint32_t *__restrict__ iout,
                                                    int64_t n, int shift, const uint32_t *__restrict__ offs, int ntile)
{
    __shared__ uint32_t base_off[256];
    __shared__ uint32_t wcnt[4][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    base_off[tid] = offs[(int64_t)tid * ntile + blockIdx.x];
    for (int q = 0; q < 4; ++q) wcnt[q][tid] = 0;
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int it = 0; it < RS_ITEMS; ++it) {
        const int64_t e = (int64_t)blockIdx.x * RS_TILE + it * 256 + tid;
        const bool valid = e < n;
        const uint64_t key = valid ? kin[e] : 0ull;
        const uint32_t idx = valid ? (iin ? iin[e] : (uint32_t)e) : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t ones = __ballot(valid && ((d >> b) & 1u));
            same &= ((d >> b) & 1u) ? ones : ~ones;
        }
        const uint64_t earlier = same & below;
        if (valid && earlier == 0ull) wcnt[w][d] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t pos = base_off[d] + (uint32_t)__popcll(earlier);
            for (int q = 0; q < w; ++q) pos += wcnt[q][d];
            kout[pos] = key;
            iout[pos] = idx;
        }
        __syncthreads();
        base_off[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        for (int q = 0; q < 4; ++q) wcnt[q][tid] = 0;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_assign_parts(const uint32_t *__restrict__ idx, int64_t n, int32_t nparts,
                                                      int32_t *__restrict__ part)
{
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256)
        part[idx[r]] = (int32_t)((r * (int64_t)nparts) / n);
}

// ---------------------------------------------------------------- partition quality
// per part: cnt[p] = {|G_p|, f_p, b_p}; adjacency bit (p, q) set when a face
// joins parts p and q.  A face inside a part is counted by its lower cell.
__global__ __launch_bounds__(256) void k_quality(Geo g, const int32_t *__restrict__ part, int32_t nparts,
                                                 unsigned long long *__restrict__ cnt, uint32_t *__restrict__ adj,
                                                 int words, int32_t *flags)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int lane = threadIdx.x & 63;
    for (int64_t r0 = (int64_t)blockIdx.x * 256; r0 < n; r0 += (int64_t)gridDim.x * 256) {
        const int64_t r = r0 + threadIdx.x;
        const bool valid = r < n;
        int p = valid ? part[r] : -1;
        if (valid && (p < 0 || p >= nparts)) {
            atomicOr(&flags[0], (int32_t)FLAG_RANGE);
            p = -1;
        }
        unsigned long long f = 0, b = 0;
        if (p >= 0) {
            const int i = (int)(r % g.nx), j = (int)((r / g.nx) % g.ny), kk = (int)(r / ((int64_t)g.nx * g.ny));
            const int k = (g.ordering == RSV_TOP_DOWN) ? g.nz - 1 - kk : kk;
            for (int s = 0; s < 7; ++s) {
                if (s == 3) continue;
                int di, dj, dk;
                dir_off(s, di, dj, dk);
                const int ii = i + di, jj = j + dj, k2 = k + dk;
                if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny || k2 < 0 || k2 >= g.nz) { ++f; continue; }
                const int64_t m = row_of(g, ii, jj, k2);
                const int q = part[m];
                if (q != p) {
                    ++f;
                    ++b;
                    if (q >= 0 && q < nparts) atomicOr(&adj[(int64_t)p * words + (q >> 5)], 1u << (q & 31));
                } else if (s > 3) {
                    ++f;   // +x, +y, +z neighbour in the same part: the shared face once
                }
            }
        }
        // one atomic per wave when the wave's cells share a part
        const int p0 = __shfl(p, 0);
        const bool uniform = __ballot(valid && p == p0) == __ballot(valid);
        if (uniform && p0 >= 0) {
            unsigned long long sf = f, sb = b, sc = valid ? 1ull : 0ull;
            for (int off = 32; off > 0; off >>= 1) {
                sf += __shfl_xor(sf, off);
                sb += __shfl_xor(sb, off);
                sc += __shfl_xor(sc, off);
            }
            if (lane == 0) {
                atomicAdd(&cnt[3 * (int64_t)p0], sc);
                atomicAdd(&cnt[3 * (int64_t)p0 + 1], sf);
                atomicAdd(&cnt[3 * (int64_t)p0 + 2], sb);
            }
        } else if (p >= 0) {
            atomicAdd(&cnt[3 * (int64_t)p], 1ull);
            atomicAdd(&cnt[3 * (int64_t)p + 1], f);
            atomicAdd(&cnt[3 * (int64_t)p + 2], b);
        }
    }
}

// per part: connectivity (set bits of its adjacency row) into cnt4[p] = {|G|, f, b, c}
__global__ __launch_bounds__(256) void k_quality_rows(const unsigned long long *__restrict__ cnt,
                                                      const uint32_t *__restrict__ adj, int words, int32_t nparts,
                                                      long long *__restrict__ per)
{
    for (int p = blockIdx.x * 256 + threadIdx.x; p < nparts; p += gridDim.x * 256) {
        long long c = 0;
        for (int q = 0; q < words; ++q) c += __popc(adj[(int64_t)p * words + q]);
        per[4 * (int64_t)p] = (long long)cnt[3 * (int64_t)p];
        per[4 * (int64_t)p + 1] = (long long)cnt[3 * (int64_t)p + 1];
        per[4 * (int64_t)p + 2] = (long long)cnt[3 * (int64_t)p + 2];
        per[4 * (int64_t)p + 3] = c;
    }
}

// the five measures from the per-part counts (one workgroup, fixed order)
__global__ __launch_bounds__(256) void k_quality_final(const long long *__restrict__ per, int32_t nparts, int64_t n,
                                                       double *__restrict__ q)
{
    __shared__ long long s_max[256], s_f[256], s_b[256], s_c[256];
    __shared__ double s_r[256], s_rsum[256];
    long long mx = 0, sf = 0, sb = 0, cm = 0;
    double rm = 0.0, rs = 0.0;
    for (int p = threadIdx.x; p < nparts; p += 256) {
        const long long sz = per[4 * (int64_t)p], f = per[4 * (int64_t)p + 1], b = per[4 * (int64_t)p + 2];
        const long long c = per[4 * (int64_t)p + 3];
        mx = max(mx, sz);
        sf += f;
        sb += b;
        cm = max(cm, c);
        const double r = f > 0 ? (double)b / (double)f : 0.0;
        rm = fmax(rm, r);
        rs += r;
    }
    const int t = threadIdx.x;
    s_max[t] = mx; s_f[t] = sf; s_b[t] = sb; s_c[t] = cm; s_r[t] = rm; s_rsum[t] = rs;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            s_max[t] = max(s_max[t], s_max[t + off]);
            s_f[t] += s_f[t + off];
            s_b[t] += s_b[t + off];
            s_c[t] = max(s_c[t], s_c[t + off]);
            s_r[t] = fmax(s_r[t], s_r[t + off]);
            s_rsum[t] += s_rsum[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        q[0] = (double)nparts * (double)s_max[0] / (double)n;
        q[1] = s_r[0];
        q[2] = (s_f[0] - s_b[0]) > 0 ? (double)s_b[0] / (double)(s_f[0] - s_b[0]) : 0.0;
        q[3] = s_rsum[0] / (double)nparts;
        q[4] = (double)s_c[0];
    }
}

int grid_for(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 16384); }

rsv_status flags_range_check(rsv_ctx *c, const char *what)
{
    int32_t f[2];
    RSV_HIP(c, hipMemcpyAsync(f, c->d_flags, sizeof(f), hipMemcpyDeviceToHost, c->stream));
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    if (f[0] & FLAG_RANGE) return set_err(c, RSV_ERR_ARG, what);
    return RSV_OK;
}

// exclusive scan of m counts in place of out (out may equal in), recursing on tile sums
rsv_status scan_counts(rsv_ctx *c, const uint32_t *in, uint32_t *out, int64_t m, std::vector<void *> &tmp)
{
    const int64_t ntile = (m + RS_TILE - 1) / RS_TILE;
    uint32_t *sums = nullptr;
    rsv_status s = dev_alloc(c, (void **)&sums, (size_t)ntile * sizeof(uint32_t));
    if (s != RSV_OK) return s;
    tmp.push_back(sums);
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)ntile), dim3(256), 0, c->stream, in, out, m, sums);
    RSV_LAUNCH(c);
    if (ntile > 1) {
        s = scan_counts(c, sums, sums, ntile, tmp);
        if (s != RSV_OK) return s;
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)ntile), dim3(256), 0, c->stream, out, m, sums);
        RSV_LAUNCH(c);
    }
    return RSV_OK;
}

struct Tmp {
    std::vector<void *> p;
    ~Tmp() { for (void *q : p) dev_free(q); }
};

}  // namespace

extern "C" {

rsv_status rsv_hsfc_keys(rsv_ctx *c, int64_t n, const double *coords, int32_t levels, uint64_t *keys)
{
    if (!c || n < 0 || (n > 0 && (!coords || !keys))) return set_err(c, RSV_ERR_ARG, "bad argument");
    if (levels < 1 || levels > 21) return set_err(c, RSV_ERR_ARG, "levels must be in [1, 21]");
    if (n == 0) return RSV_OK;
    rsv_status s = flags_reset(c);
    if (s != RSV_OK) return s;
    hipLaunchKernelGGL(k_hsfc_points, dim3(grid_for(n)), dim3(256), 0, c->stream, n, coords, levels, keys, c->d_flags);
    RSV_LAUNCH(c);
    return flags_range_check(c, "a coordinate is outside [0, 1] or not a number");
}

rsv_status rsv_grid_hsfc_keys(rsv_grid *g, int32_t levels, uint64_t *keys)
{
    if (!g || !keys) return set_err(g ? g->ctx : nullptr, RSV_ERR_ARG, "NULL argument");
    rsv_ctx *c = g->ctx;
    if (levels < 1 || levels > 21) return set_err(c, RSV_ERR_ARG, "levels must be in [1, 21]");
    hipLaunchKernelGGL(k_hsfc_grid, dim3(grid_for(g->ncell)), dim3(256), 0, c->stream, g->geo, levels, keys);
    RSV_LAUNCH(c);
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    return RSV_OK;
}

rsv_status rsv_hsfc_partition(rsv_ctx *c, int64_t n, const uint64_t *keys, int32_t levels, int32_t nparts,
                              int32_t *part)
{
    if (!c || n < 0 || (n > 0 && (!keys || !part))) return set_err(c, RSV_ERR_ARG, "bad argument");
    if (levels < 1 || levels > 21) return set_err(c, RSV_ERR_ARG, "levels must be in [1, 21]");
    if (nparts < 1) return set_err(c, RSV_ERR_ARG, "nparts must be >= 1");
    if (n > ((int64_t)1 << 31)) return set_err(c, RSV_ERR_ARG, "at most 2^31 keys");
    if (n == 0) return RSV_OK;
    const int64_t ntile = (n + RS_TILE - 1) / RS_TILE;
    Tmp t;
    uint64_t *k2[2] = {nullptr, nullptr};
    uint32_t *i2[2] = {nullptr, nullptr}, *hist = nullptr;
    rsv_status s = RSV_OK;
    for (int q = 0; q < 2 && s == RSV_OK; ++q) {
        s = dev_alloc(c, (void **)&k2[q], (size_t)n * sizeof(uint64_t));
        if (s == RSV_OK) { t.p.push_back(k2[q]); s = dev_alloc(c, (void **)&i2[q], (size_t)n * sizeof(uint32_t)); }
        if (s == RSV_OK) t.p.push_back(i2[q]);
    }
    if (s == RSV_OK) s = dev_alloc(c, (void **)&hist, (size_t)ntile * 256 * sizeof(uint32_t));
    if (s != RSV_OK) return s;
    t.p.push_back(hist);
    const int bits = 3 * levels, passes = (bits + 7) / 8;
    const uint64_t *kin = keys;
    const uint32_t *iin = nullptr;
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = 8 * ps;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)ntile), dim3(256), 0, c->stream, kin, n, shift, hist, (int)ntile);
        RSV_LAUNCH(c);
        s = scan_counts(c, hist, hist, ntile * 256, t.p);
        if (s != RSV_OK) return s;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntile), dim3(256), 0, c->stream, kin, iin, k2[ps & 1],
                           i2[ps & 1], n, shift, hist, (int)ntile);
        RSV_LAUNCH(c);
        kin = k2[ps & 1];
        iin = i2[ps & 1];
    }
    hipLaunchKernelGGL(k_assign_parts, dim3(grid_for(n)), dim3(256), 0, c->stream, iin, n, nparts, part);
    RSV_LAUNCH(c);
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    return RSV_OK;
}

rsv_status rsv_partition_quality(rsv_grid *g, const int32_t *part, int32_t nparts, double *q, int64_t *per_part)
{
    if (!g || !part || !q) return set_err(g ? g->ctx : nullptr, RSV_ERR_ARG, "NULL argument");
    rsv_ctx *c = g->ctx;
    if (nparts < 1 || nparts > 16384) return set_err(c, RSV_ERR_ARG, "nparts must be in [1, 16384]");
    const int words = (nparts + 31) / 32;
    Tmp t;
    unsigned long long *cnt = nullptr;
    uint32_t *adj = nullptr;
    long long *per = nullptr;
    double *dq = nullptr;
    rsv_status s = dev_alloc(c, (void **)&cnt, (size_t)nparts * 3 * sizeof(unsigned long long));
    if (s == RSV_OK) { t.p.push_back(cnt); s = dev_alloc(c, (void **)&adj, (size_t)nparts * words * sizeof(uint32_t)); }
    if (s == RSV_OK) { t.p.push_back(adj); s = dev_alloc(c, (void **)&per, (size_t)nparts * 4 * sizeof(long long)); }
    if (s == RSV_OK) { t.p.push_back(per); s = dev_alloc(c, (void **)&dq, 5 * sizeof(double)); }
    if (s != RSV_OK) return s;
    t.p.push_back(dq);
    RSV_HIP(c, hipMemsetAsync(cnt, 0, (size_t)nparts * 3 * sizeof(unsigned long long), c->stream));
    RSV_HIP(c, hipMemsetAsync(adj, 0, (size_t)nparts * words * sizeof(uint32_t), c->stream));
    s = flags_reset(c);
    if (s != RSV_OK) return s;
    hipLaunchKernelGGL(k_quality, dim3(grid_for(g->ncell)), dim3(256), 0, c->stream, g->geo, part, nparts, cnt, adj,
                       words, c->d_flags);
    RSV_LAUNCH(c);
    hipLaunchKernelGGL(k_quality_rows, dim3(grid_for(nparts)), dim3(256), 0, c->stream, cnt, adj, words, nparts, per);
    RSV_LAUNCH(c);
    hipLaunchKernelGGL(k_quality_final, dim3(1), dim3(256), 0, c->stream, per, nparts, g->ncell, dq);
    RSV_LAUNCH(c);
    s = flags_range_check(c, "a part number is outside [0, nparts)");
    if (s != RSV_OK) return s;
    RSV_HIP(c, hipMemcpyAsync(q, dq, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (per_part)
        RSV_HIP(c, hipMemcpyAsync(per_part, per, (size_t)nparts * 4 * sizeof(long long), hipMemcpyDeviceToHost,
                                  c->stream));
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    return RSV_OK;
}

}  // extern "C"
