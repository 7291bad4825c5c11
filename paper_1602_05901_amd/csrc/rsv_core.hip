// Context, grid (cell <-> row map), matrix assembly and the ABI SpMV.
#include "rsv_internal.h"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>

static thread_local std::string g_last_static_err;

rsv_status set_err(rsv_ctx *c, rsv_status s, const std::string &msg)
{
    if (c) c->err = msg;
    else g_last_static_err = msg;
    return s;
}

rsv_status dev_alloc(rsv_ctx *c, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return set_err(c, RSV_ERR_OOM, std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    return RSV_OK;
}

void dev_free(void *p)
{
    if (p) (void)hipFree(p);
}

rsv_status flags_reset(rsv_ctx *c)
{
    int32_t init[2] = {0, 0x7fffffff};
    RSV_HIP(c, hipMemcpyAsync(c->d_flags, init, sizeof(init), hipMemcpyHostToDevice, c->stream));
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    return RSV_OK;
}

rsv_status flags_check(rsv_ctx *c, int64_t *bad_cell)
{
    int32_t f[2];
    RSV_HIP(c, hipMemcpyAsync(f, c->d_flags, sizeof(f), hipMemcpyDeviceToHost, c->stream));
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    if (bad_cell) *bad_cell = (f[1] == 0x7fffffff) ? -1 : f[1];
    if (f[0] & FLAG_TIMEOUT) return set_err(c, RSV_ERR_TIMEOUT, "wavefront wait exceeded its bound");
    if (f[0] & FLAG_PATTERN) return set_err(c, RSV_ERR_PATTERN, "nonzero block toward a missing neighbour");
    if (f[0] & FLAG_NAN) return set_err(c, RSV_ERR_NAN, "non-finite matrix entry");
    if (f[0] & FLAG_PIVOT) return set_err(c, RSV_ERR_ZERO_PIVOT, "zero or near-singular 3x3 pivot");
    return RSV_OK;
}

// ------------------------------------------------------------------ fixed scratch
// The device memory of the entry points that allocate nothing: one
// file-scope array, a copy of which each device holds from the first context
// created on it until the process ends.  On the host the array's name is only
// a stand-in, never a device address: host code uses the address that
// hipGetSymbolAddress returns, looked up once per device (with that device
// current) and kept per device.
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[MAX_DEVICES] = {};

rsv_status scratch_lookup(rsv_ctx *c)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (c->device < 0 || c->device >= MAX_DEVICES) return set_err(c, RSV_ERR_ARG, "device ordinal beyond the scratch table");
    if (!g_scratch_ptr[c->device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_err(c, RSV_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[c->device] = (double *)p;
    }
    c->d_scratch = g_scratch_ptr[c->device];
    return RSV_OK;
}

// ------------------------------------------------------------------ kernel timing
static constexpr int PROF_POOL = 4096;   // events (2048 launches) between resolutions

static void prof_resolve(rsv_ctx *c)
{
    if (c->prof_used == 0) return;
    (void)hipEventSynchronize(c->prof_ev[c->prof_used - 1]);
    for (int p = 0; p < c->prof_used / 2; ++p) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->prof_ev[2 * p], c->prof_ev[2 * p + 1]) == hipSuccess) {
            c->prof_ms[c->prof_kind[p]] += ms;
            c->prof_cnt[c->prof_kind[p]] += 1;
        }
    }
    c->prof_used = 0;
}

int prof_begin(rsv_ctx *c, int kind)
{
    if (!c->prof_on || !((c->prof_mask >> kind) & 1u)) return -1;
    if (c->prof_used + 2 > (int)c->prof_ev.size()) prof_resolve(c);
    const int tok = c->prof_used;
    c->prof_used += 2;
    c->prof_kind[tok / 2] = kind;
    (void)hipEventRecord(c->prof_ev[tok], c->stream);
    return tok;
}

void prof_end(rsv_ctx *c, int tok)
{
    if (tok < 0) return;
    (void)hipEventRecord(c->prof_ev[tok + 1], c->stream);
}

extern "C" {

rsv_status rsv_profile_enable(rsv_ctx *c, int32_t on)
{
    if (!c) return set_err(nullptr, RSV_ERR_ARG, "ctx is NULL");
    if (on) {
        if (c->prof_ev.empty()) {
            c->prof_ev.resize(PROF_POOL);
            c->prof_kind.resize(PROF_POOL / 2);
            for (auto &e : c->prof_ev) RSV_HIP(c, hipEventCreate(&e));
        }
        prof_resolve(c);
        for (int k = 0; k < RSV_K_COUNT; ++k) { c->prof_ms[k] = 0.0; c->prof_cnt[k] = 0; }
        c->prof_on = true;
    } else {
        prof_resolve(c);
        c->prof_on = false;
    }
    return RSV_OK;
}

rsv_status rsv_profile_classes(rsv_ctx *c, uint32_t mask)
{
    if (!c) return set_err(nullptr, RSV_ERR_ARG, "ctx is NULL");
    c->prof_mask = mask;
    return RSV_OK;
}

rsv_status rsv_profile_read(rsv_ctx *c, double *ms, int64_t *cnt)
{
    if (!c) return set_err(nullptr, RSV_ERR_ARG, "ctx is NULL");
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    prof_resolve(c);
    for (int k = 0; k < RSV_K_COUNT; ++k) {
        if (ms) ms[k] = c->prof_ms[k];
        if (cnt) cnt[k] = c->prof_cnt[k];
    }
    return RSV_OK;
}

int32_t rsv_version(void) { return RSV_VERSION; }

rsv_status rsv_set_wait_limit(rsv_ctx *c, double seconds)
{
    if (!c || !(seconds > 0.0) || seconds > 60.0) return set_err(c, RSV_ERR_ARG, "wait limit must be in (0, 60] s");
    c->wait_ticks = (uint64_t)(seconds * 1e8);   // the device wall clock runs at 100 MHz
    if (c->wait_ticks == 0) c->wait_ticks = 1;
    return RSV_OK;
}

rsv_status rsv_device_info(const rsv_ctx *c, int64_t *info, int32_t n)
{
    if (!c || !info || n < 0) return set_err(nullptr, RSV_ERR_ARG, "NULL argument");
    const int64_t v[5] = {c->num_cu, c->lds_max, c->lds_per_cu, sweep_ring_depth(c, 0, 0), sweep_ring_depth(c, 1, 0)};
    for (int i = 0; i < n && i < 5; ++i) info[i] = v[i];
    return RSV_OK;
}

const char *rsv_status_str(rsv_status s)
{
    switch (s) {
    case RSV_OK: return "RSV_OK";
    case RSV_NOT_CONVERGED: return "RSV_NOT_CONVERGED";
    case RSV_BREAKDOWN: return "RSV_BREAKDOWN";
    case RSV_ERR_ARG: return "RSV_ERR_ARG";
    case RSV_ERR_OOM: return "RSV_ERR_OOM";
    case RSV_ERR_HIP: return "RSV_ERR_HIP";
    case RSV_ERR_ZERO_PIVOT: return "RSV_ERR_ZERO_PIVOT";
    case RSV_ERR_NAN: return "RSV_ERR_NAN";
    case RSV_ERR_PATTERN: return "RSV_ERR_PATTERN";
    case RSV_ERR_TIMEOUT: return "RSV_ERR_TIMEOUT";
    default: return "RSV_UNKNOWN";
    }
}

const char *rsv_last_error(const rsv_ctx *c)
{
    return c ? c->err.c_str() : g_last_static_err.c_str();
}

rsv_status rsv_create(int32_t dev, rsv_ctx **out)
{
    if (!out) return set_err(nullptr, RSV_ERR_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return set_err(nullptr, RSV_ERR_HIP, std::string("hipGetDeviceCount: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= n) return set_err(nullptr, RSV_ERR_ARG, "device ordinal out of range");
    e = hipSetDevice(dev);
    if (e != hipSuccess) return set_err(nullptr, RSV_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    rsv_ctx *c = new (std::nothrow) rsv_ctx();
    if (!c) return set_err(nullptr, RSV_ERR_OOM, "ctx");
    c->device = dev;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        c->num_cu = prop.multiProcessorCount;
        size_t lds = prop.sharedMemPerBlock;
        if (prop.sharedMemPerBlockOptin > lds) lds = prop.sharedMemPerBlockOptin;
        if (prop.maxSharedMemoryPerMultiProcessor > 0 && prop.maxSharedMemoryPerMultiProcessor < lds)
            lds = prop.maxSharedMemoryPerMultiProcessor;
        c->lds_max = (int)lds;
        c->lds_per_cu = (int)prop.maxSharedMemoryPerMultiProcessor;
    }
    rsv_status s = RSV_OK;
    if (hipHostMalloc((void **)&c->h_scal, SC_COUNT * sizeof(double), hipHostMallocDefault) != hipSuccess) s = RSV_ERR_OOM;
    if (s == RSV_OK) s = dev_alloc(c, (void **)&c->d_scal, SC_COUNT * sizeof(double));
    if (s == RSV_OK) s = dev_alloc(c, (void **)&c->d_tickets, 8 * sizeof(uint64_t));
    if (s == RSV_OK) s = dev_alloc(c, (void **)&c->d_flags, 4 * sizeof(int32_t));
    if (s == RSV_OK && hipMemset(c->d_tickets, 0, 8 * sizeof(uint64_t)) != hipSuccess) s = RSV_ERR_HIP;
    if (s == RSV_OK && hipMemset(c->d_scal, 0, SC_COUNT * sizeof(double)) != hipSuccess) s = RSV_ERR_HIP;
    if (s == RSV_OK) s = flags_reset(c);
    if (s == RSV_OK) s = scratch_lookup(c);   // device current: set above
    if (s != RSV_OK) {
        g_last_static_err = c->err.empty() ? "context allocation failed" : c->err;
        rsv_destroy(c);
        return s;
    }
    *out = c;
    return RSV_OK;
}

rsv_status rsv_set_stream(rsv_ctx *c, void *stream)
{
    if (!c) return set_err(nullptr, RSV_ERR_ARG, "ctx is NULL");
    c->stream = (hipStream_t)stream;
    return RSV_OK;
}

void rsv_destroy(rsv_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto &e : c->prof_ev) (void)hipEventDestroy(e);
    if (c->h_scal) (void)hipHostFree(c->h_scal);
    if (c->h_spec) (void)hipHostFree(c->h_spec);
    for (auto &e : c->spec_ev)
        if (e) (void)hipEventDestroy(e);
    dev_free(c->d_scal);
    dev_free(c->d_partials);
    dev_free(c->d_tickets);
    dev_free(c->d_flags);
    delete c;
}

}  // extern "C"

rsv_status grid_create_planes(rsv_ctx *c, int32_t nx, int32_t ny, int32_t nz, int32_t ordering, int mx, int my,
                              int mz, rsv_grid **out)
{
    if (!c || !out) return set_err(c, RSV_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return set_err(c, RSV_ERR_ARG, "grid dimensions must be >= 1");
    if (ordering != RSV_BOTTOM_UP && ordering != RSV_TOP_DOWN) return set_err(c, RSV_ERR_ARG, "bad ordering");
    if (mx < 1 || my < 1 || mz < 1) return set_err(c, RSV_ERR_ARG, "bad plane moduli");
    const int ntx = (nx + 7) / 8, nty = (ny + 7) / 8;
    const int64_t nslot = (int64_t)ntx * nty * nz * 64;
    if (nslot * 3 >= ((int64_t)1 << 31)) return set_err(c, RSV_ERR_ARG, "grid too large (3*padded cells must fit int32)");
    rsv_grid *g = new (std::nothrow) rsv_grid();
    if (!g) return set_err(c, RSV_ERR_OOM, "grid");
    g->ctx = c;
    g->geo = Geo{nx, ny, nz, ntx, nty, ordering, nslot};
    g->ncell = (int64_t)nx * ny * nz;
    g->nv = 3 * nslot;
    g->nplanes = std::min(mx, nx) + std::min(my, ny) + std::min(mz, nz) - 2;
    // real slots bucketed by plane (i mod mx) + (j mod my) + (k mod mz),
    // ascending slot within a plane
    std::vector<int64_t> cnt(g->nplanes + 1, 0);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) cnt[i % mx + j % my + k % mz + 1]++;
    for (int p = 0; p < g->nplanes; ++p) cnt[p + 1] += cnt[p];
    g->plane_ptr = cnt;
    std::vector<int32_t> slots(g->ncell);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    int li[64], lj[64];
    for (int L = 0; L < 64; ++L) lane_ij(L, li[L], lj[L]);
    int64_t s = 0;
    for (int T = 0; T < ntx * nty; ++T) {
        const int x0 = (T % ntx) * 8, y0 = (T / ntx) * 8;
        for (int r = 0; r < nz; ++r)
            for (int L = 0; L < 64; ++L, ++s) {
                const int gx = x0 + li[L], gy = y0 + lj[L];
                if (gx >= nx || gy >= ny) continue;
                const int k = wrap_nz(r - li[L] - lj[L], nz);
                slots[fill[gx % mx + gy % my + k % mz]++] = (int32_t)s;
            }
    }
    rsv_status st = dev_alloc(c, (void **)&g->d_plane_slots, slots.size() * sizeof(int32_t));
    if (st != RSV_OK) { delete g; return st; }
    hipError_t e = hipMemcpy(g->d_plane_slots, slots.data(), slots.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        dev_free(g->d_plane_slots);
        delete g;
        return set_err(c, RSV_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    *out = g;
    return RSV_OK;
}

extern "C" {

rsv_status rsv_grid_create(rsv_ctx *c, int32_t nx, int32_t ny, int32_t nz, int32_t ordering, rsv_grid **out)
{
    return grid_create_planes(c, nx, ny, nz, ordering, nx, ny, nz, out);
}

void rsv_grid_destroy(rsv_grid *g)
{
    if (!g) return;
    dev_free(g->d_plane_slots);
    delete g;
}

int64_t rsv_grid_ncell(const rsv_grid *g) { return g ? g->ncell : 0; }

rsv_status rsv_cell_to_row(const rsv_grid *g, int32_t i, int32_t j, int32_t k, int64_t *row)
{
    if (!g || !row) return set_err(nullptr, RSV_ERR_ARG, "NULL argument");
    const Geo &G = g->geo;
    if (i < 0 || i >= G.nx || j < 0 || j >= G.ny || k < 0 || k >= G.nz) return set_err(g->ctx, RSV_ERR_ARG, "cell out of range");
    *row = row_of(G, i, j, k);
    return RSV_OK;
}

rsv_status rsv_row_to_cell(const rsv_grid *g, int64_t row, int32_t *i, int32_t *j, int32_t *k)
{
    if (!g || !i || !j || !k) return set_err(nullptr, RSV_ERR_ARG, "NULL argument");
    if (row < 0 || row >= g->ncell) return set_err(g->ctx, RSV_ERR_ARG, "row out of range");
    const Geo &G = g->geo;
    *i = (int32_t)(row % G.nx);
    *j = (int32_t)((row / G.nx) % G.ny);
    const int32_t kk = (int32_t)(row / ((int64_t)G.nx * G.ny));
    *k = (G.ordering == RSV_TOP_DOWN) ? G.nz - 1 - kk : kk;
    return RSV_OK;
}

static rsv_status assemble_values(rsv_matrix *M, const double *blocks, int32_t where)
{
    rsv_grid *g = M->g;
    rsv_ctx *c = g->ctx;
    const size_t bytes = (size_t)g->ncell * 63 * sizeof(double);
    const double *src = blocks;
    double *stage = nullptr;
    if (where == RSV_MEM_HOST) {
        rsv_status s = dev_alloc(c, (void **)&stage, bytes);
        if (s != RSV_OK) return s;
        hipError_t e = hipMemcpyAsync(stage, blocks, bytes, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) {
            dev_free(stage);
            return set_err(c, RSV_ERR_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
        }
        src = stage;
    } else if (where != RSV_MEM_DEVICE) {
        return set_err(c, RSV_ERR_ARG, "bad memory kind");
    }
    rsv_status s = flags_reset(c);
    if (s == RSV_OK) s = launch_assemble(c, g->geo, src, M->d_A);
    if (s == RSV_OK) s = flags_check(c, nullptr);
    if (stage) dev_free(stage);
    return s;
}

rsv_status rsv_matrix_assemble(rsv_grid *g, const double *blocks, int32_t where, rsv_matrix **out)
{
    if (!g || !blocks || !out) return set_err(g ? g->ctx : nullptr, RSV_ERR_ARG, "NULL argument");
    *out = nullptr;
    rsv_ctx *c = g->ctx;
    rsv_matrix *M = new (std::nothrow) rsv_matrix();
    if (!M) return set_err(c, RSV_ERR_OOM, "matrix");
    M->g = g;
    M->bs = 3;
    M->nv = g->nv;
    const size_t abytes = (size_t)(g->geo.nslot / 64) * 63 * 64 * sizeof(double);
    rsv_status s = dev_alloc(c, (void **)&M->d_A, abytes);
    if (s == RSV_OK) {
        M->bytes = (int64_t)abytes;
        s = assemble_values(M, blocks, where);
    }
    if (s != RSV_OK) {
        rsv_matrix_destroy(M);
        return s;
    }
    *out = M;
    return RSV_OK;
}

rsv_status rsv_matrix_update(rsv_matrix *M, const double *blocks, int32_t where)
{
    if (!M || !blocks) return set_err(M ? M->g->ctx : nullptr, RSV_ERR_ARG, "NULL argument");
    if (M->bs == 1) return scalar_assemble_values(M, blocks, where);
    return assemble_values(M, blocks, where);
}

// rsv_spmv and rsv_matrix_device_bytes are defined with the solver workspace

void rsv_pc_params_default(rsv_pc_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->type = RSV_PC_BILU0;
    p->precision = RSV_FP64;
    p->ras_px = p->ras_py = p->ras_pz = 4;
    p->ras_overlap = 1;
    p->iluk_level = 0;
    p->pipelined = 1;
    p->theta = 0.9;
    p->cpr_variant = RSV_CPR_FPF;
    p->cpr_stage = RSV_PC_RAS;
    p->cpr_decouple = RSV_DECOUPLE_NONE;
    p->mg_pre = 1;
    p->mg_post = 1;
    p->mg_coarse = 128;
    p->local_solver = RSV_LOCAL_ILUK;
    p->ilut_p = -1;
    p->ilut_tol = 1e-3;
}

void rsv_solver_params_default(rsv_solver_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->method = RSV_GMRES;
    p->restart = 30;
    p->tol = 1e-8;
    p->maxit = 10000;
    p->ortho = RSV_CGS2;
}

}  // extern "C"
