// Learned preconditioner: a 3-level 3-D U-Net residual -> correction map used
// inside flexible GMRES, with block ILU(0) as the fallback (the paper's
// user-defined preconditioner hook, PC_USER with assemble / solve / destroy).
//
// Network (channels c0/c1/c2, default 16/32/64, 3x3x3 kernels, zero padding):
//   x0 = [r/s (3 channels), standardised ln k]           s = rms(r)
//   a1 = relu(conv0(x0)),  s1 = relu(conv1(a1))           full resolution
//   a2 = relu(conv2(pool(s1))), s2 = relu(conv3(a2))     1/2
//   a3 = relu(conv4(pool(s2))), b3 = relu(conv5(a3))     1/4
//   d2a = relu(conv6(up(b3)) + s2), d2 = relu(conv7(d2a))
//   d1a = relu(conv8(up(d2)) + s1), d1 = relu(conv9(d1a))
//   y = conv10(d1)  (1x1x1 linear to 3 channels),  z = s * y
// pool = 2x2x2 average, up = nearest-neighbour x2.  Activations and weights
// are BF16; every convolution is an implicit GEMM on the CDNA matrix cores
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation).  Training: the backward
// data pass is the same kernel on transposed, tap-flipped weights; the weight
// gradient is a split-K MFMA GEMM over voxels with a fixed-order reduction;
// Adam keeps FP32 master weights.
#include "rsv_internal.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

__device__ __host__ inline uint16_t f2bf(float f)
{
#ifdef __HIP_DEVICE_COMPILE__
    uint32_t u = __float_as_uint(f);
#else
    uint32_t u;
    std::memcpy(&u, &f, 4);
#endif
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int NL = 11;   // layers (10 convolutions 3x3x3 + final 1x1x1)

struct Arch {
    int c[3];
    int cin[NL], cout[NL];
    int64_t woff[NL], boff[NL], np;
    void init(int c0, int c1, int c2)
    {
        c[0] = c0; c[1] = c1; c[2] = c2;
        const int ci[NL] = {4, c0, c0, c1, c1, c2, c2, c1, c1, c0, c0};
        const int co[NL] = {c0, c0, c1, c1, c2, c2, c1, c1, c0, c0, 3};
        int64_t off = 0;
        for (int l = 0; l < NL; ++l) {
            cin[l] = ci[l];
            cout[l] = co[l];
            woff[l] = off;
            off += (int64_t)(l < 10 ? 27 : 1) * ci[l] * co[l];
            boff[l] = off;
            off += co[l];
        }
        np = off;
    }
    // K blocks (of 32 for inputs with a multiple of 8 channels, else 16): forward, backward data
    int kb(int l) const { return (27 * cin[l] + (cin[l] % 8 ? 15 : 31)) / (cin[l] % 8 ? 16 : 32); }
    int kbt(int l) const { return (27 * cout[l] + (cout[l] % 8 ? 15 : 31)) / (cout[l] % 8 ? 16 : 32); }
};

struct ConvGeo {
    int nx, ny, nz;   // output resolution
    int up;           // input is the half-resolution tensor, read nearest-up-sampled
    int cin, cout;
    int64_t V;
};

__device__ inline int64_t src_voxel(const ConvGeo &g, int x, int y, int z, int dx, int dy, int dz)
{
    const int a = x + dx, b = y + dy, c = z + dz;
    if (a < 0 || a >= g.nx || b < 0 || b >= g.ny || c < 0 || c >= g.nz) return -1;
    if (g.up) {
        const int hx = g.nx >> 1, hy = g.ny >> 1;
        return (a >> 1) + (int64_t)hx * ((b >> 1) + (int64_t)hy * (c >> 1));
    }
    return a + (int64_t)g.nx * (b + (int64_t)g.ny * c);
}

// ---------------------------------------------------------------- convolution as implicit GEMM
// K per MFMA: 32 (v_mfma_f32_16x16x32_bf16, 8 k per lane) when the input has a
// multiple of 8 channels, so that a lane's 8 consecutive k are 8 channels of
// one tap; else 16 (v_mfma_f32_16x16x16_bf16, 4 k per lane).
__host__ __device__ constexpr int conv_kw(int cin) { return cin % 8 == 0 ? 32 : 16; }
__host__ __device__ constexpr int conv_kblocks(int cin) { return (27 * cin + conv_kw(cin) - 1) / conv_kw(cin); }
// bytes of one lane's packed weight fragment
__host__ __device__ constexpr int conv_frag_bytes(int cin) { return conv_kw(cin) / 2; }
template <bool K32> struct Frag { using T = v4s; static constexpr int KW = 16; };
template <> struct Frag<true> { using T = v8s; static constexpr int KW = 32; };
__device__ inline v4f mfma_k(v4s a, v4s b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
__device__ inline v4f mfma_k(v8s a, v8s b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

// One wavefront: 16*MB output voxels x (16*NB) output channels.  GEMM row m =
// voxel, column n = output channel, k = tap*cin + ci.  Operand fragments
// (KW = 16 or 32, w = KW / 4 k per lane): lane l holds A[m = l%16][k = w*(l/16)
// .. + w-1] and B[k = w*(l/16) .. + w-1][n = l%16]; the result holds
// D[m = 4*(l/16) + i][n = l%16].  Weights are pre-packed so that B fragments
// are one load per lane; an A fragment's lane reads w consecutive channels of
// one voxel.  Each B fragment feeds MB products and each A fragment NB.
template <int MB, int NB, bool OUT_BF16, bool K32>
__global__ __launch_bounds__(256) void k_conv(ConvGeo g, const uint16_t *__restrict__ X, const void *__restrict__ Wfv,
                                              int KB, const float *__restrict__ bias,
                                              const uint16_t *__restrict__ skip, int relu, void *__restrict__ out)
{
    using FT = typename Frag<K32>::T;
    constexpr int KW = Frag<K32>::KW;
    const FT *Wf = (const FT *)Wfv;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t v0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * MB);
    if (v0 >= g.V) return;
    const int m = lane & 15, kq = (KW / 4) * (lane >> 4);
    int px[MB], py[MB], pz[MB];
    bool live[MB];   // the last tile of a level may be partial
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const int64_t v = v0 + mb * 16 + m;
        live[mb] = v < g.V;
        px[mb] = (int)(v % g.nx);
        py[mb] = (int)((v / g.nx) % g.ny);
        pz[mb] = (int)(v / ((int64_t)g.nx * g.ny));
    }
    v4f acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = v4f{0.f, 0.f, 0.f, 0.f};
    const int K = 27 * g.cin;
    for (int kb = 0; kb < KB; ++kb) {
        const int k = kb * KW + kq;
        const bool kin = k < K;
        const int tap = kin ? k / g.cin : 0, ci = k - tap * g.cin;
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
        FT a[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            a[mb] = FT{};
            if (kin && live[mb]) {
                const int64_t u = src_voxel(g, px[mb], py[mb], pz[mb], dx, dy, dz);
                if (u >= 0) a[mb] = *(const FT *)(X + u * g.cin + ci);
            }
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const FT b = Wf[((int64_t)kb * NB + nb) * 64 + lane];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb][nb] = mfma_k(a[mb], b, acc[mb][nb]);
        }
    }
    const int n = lane & 15, mr = 4 * (lane >> 4);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int co = nb * 16 + n;
        const float bb = bias ? bias[co] : 0.f;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t vo = v0 + mb * 16 + mr + i;
                if (vo >= g.V) continue;
                float val = acc[mb][nb][i] + bb;
                if (skip) val += bf2f(skip[vo * g.cout + co]);
                if (relu) val = val > 0.f ? val : 0.f;
                if (OUT_BF16) ((uint16_t *)out)[vo * g.cout + co] = f2bf(val);
                else ((float *)out)[vo * g.cout + co] = val;
            }
    }
}

// LDS-tiled variant for inputs of at most 32 channels: a workgroup computes a
// 16 (x) x 4 (y) x 4 (z) output block; the 18 x 6 x 6 input halo (zero outside
// the grid, nearest-up-sampled when `up`) and the packed weights are staged in
// LDS once, so every MFMA operand comes from LDS.  Wave w owns output plane
// z0 + w; its voxel block mb is the x-run at y0 + mb.
constexpr int CT_X = 16, CT_Y = 4, CT_Z = 4, CH_X = CT_X + 2, CH_Y = CT_Y + 2, CH_Z = CT_Z + 2;
constexpr int CH_N = CH_X * CH_Y * CH_Z;   // 648 halo voxels

// the epilogue of one or two output blocks stages each wave's results in the
// halo area ([64 voxels][16 NB + 1] floats per wave), made larger if needed
__host__ __device__ constexpr size_t conv_stage_bytes(int nb) { return nb <= 2 ? (size_t)4 * 64 * (16 * nb + 1) * 4 : 0; }
inline size_t conv_lds_bytes(int cin, int KB, int NB)
{
    return std::max((size_t)CH_N * cin * 2, conv_stage_bytes(NB)) + (size_t)KB * NB * 64 * conv_frag_bytes(cin);
}

// Global -> LDS copy of n 16-byte words by the workgroup, eight loads in
// flight per thread before their stores.
__device__ inline void stage_words(const v4s *__restrict__ src, v4s *dst, int n)
{
    for (int e0 = 0; e0 < n; e0 += 8 * 256) {
        v4s v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = e0 + i * 256 + (int)threadIdx.x;
            if (e < n) v[i] = src[e];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = e0 + i * 256 + (int)threadIdx.x;
            if (e < n) dst[e] = v[i];
        }
    }
}

// LDS-tiled variant for inputs of CIN = 4, 16 or 32 channels.  A workgroup
// stages the packed weights in LDS once and then walks bricks of 16 (x) x 4
// (y) x 4 (z) output voxels (brick b, b + gridDim.x, ...): the brick's
// 18 x 6 x 6 input halo (zero outside the grid, nearest-up-sampled when `up`)
// goes to LDS from registers that were loaded during the previous brick's
// MFMAs, so every MFMA operand comes from LDS and no load waits on the
// critical path.  Wave w owns output plane z0 + w; its voxel block mb is the
// x-run at y0 + mb.
template <int NB, bool OUT_BF16, int CIN>
__global__ __launch_bounds__(256) void k_conv_lds(ConvGeo g, const uint16_t *__restrict__ X, const void *__restrict__ Wfv,
                                                  int KB, const float *__restrict__ bias,
                                                  const uint16_t *__restrict__ skip, int relu, void *__restrict__ out)
{
    constexpr bool K32 = CIN % 8 == 0;
    using FT = typename Frag<K32>::T;
    constexpr int KW = Frag<K32>::KW;
    constexpr int C4 = CIN / 4, NI = (CH_N * C4 + 255) / 256;   // halo words (4 channels) per thread
    extern __shared__ __align__(16) unsigned char cl[];
    FT *wl = (FT *)cl;                                          // [KB][NB][64]
    uint16_t *xl = (uint16_t *)(cl + (size_t)KB * NB * 64 * sizeof(FT));   // [648][CIN]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ntx = (g.nx + CT_X - 1) / CT_X, nty = (g.ny + CT_Y - 1) / CT_Y, ntz = (g.nz + CT_Z - 1) / CT_Z;
    const int nbricks = ntx * nty * ntz;
    stage_words((const v4s *)Wfv, (v4s *)wl, KB * NB * 64 * (int)(sizeof(FT) / sizeof(v4s)));
    v4s hv[NI];
    auto load = [&](int b) {
        const int x0 = (b % ntx) * CT_X, y0 = ((b / ntx) % nty) * CT_Y, z0 = (b / (ntx * nty)) * CT_Z;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int e = tid + 256 * i;
            const int h = e / C4, q = e - h * C4;
            const int hx = h % CH_X, hy = (h / CH_X) % CH_Y, hz = h / (CH_X * CH_Y);
            hv[i] = v4s{0, 0, 0, 0};
            if (e < CH_N * C4) {
                const int64_t u = src_voxel(g, x0, y0, z0, hx - 1, hy - 1, hz - 1);
                if (u >= 0) hv[i] = *(const v4s *)(X + u * CIN + 4 * q);
            }
        }
    };
    const int m = lane & 15, kq = (KW / 4) * (lane >> 4);
    const int n = lane & 15, mr = 4 * (lane >> 4);
    const int K = 27 * CIN;
    if ((int)blockIdx.x < nbricks) load(blockIdx.x);
    for (int b = blockIdx.x; b < nbricks; b += gridDim.x) {
        const int x0 = (b % ntx) * CT_X, y0 = ((b / ntx) % nty) * CT_Y, z0 = (b / (ntx * nty)) * CT_Z;
        __syncthreads();   // the previous brick's operands have been read (and the weights written)
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int e = tid + 256 * i;
            if (e < CH_N * C4) *(v4s *)(xl + (size_t)e * 4) = hv[i];   // [h][CIN] = word e
        }
        __syncthreads();
        if (b + (int)gridDim.x < nbricks) load(b + gridDim.x);
        v4f acc[CT_Y][NB];
#pragma unroll
        for (int mb = 0; mb < CT_Y; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = v4f{0.f, 0.f, 0.f, 0.f};
        for (int kb = 0; kb < KB; ++kb) {
            const int k = kb * KW + kq;
            const bool kin = k < K;
            const int tap = kin ? k / CIN : 0, ci = k - tap * CIN;
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;   // halo offsets (0..2)
            FT a[CT_Y];
#pragma unroll
            for (int mb = 0; mb < CT_Y; ++mb) {
                const int h = ((wave + dz) * CH_Y + (mb + dy)) * CH_X + (m + dx);
                a[mb] = kin ? *(const FT *)(xl + (size_t)h * CIN + ci) : FT{};
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const FT bf = wl[(kb * NB + nb) * 64 + lane];
#pragma unroll
                for (int mb = 0; mb < CT_Y; ++mb) acc[mb][nb] = mfma_k(a[mb], bf, acc[mb][nb]);
            }
        }
        if constexpr (NB <= 2) {
            // epilogue through LDS (16 or 32 output channels): each wave puts
            // its 64 voxels x 16 NB channels into the halo area, which no wave
            // reads any more, then lane v takes voxel v whole (x = v % 16,
            // y = v / 16), adds bias and skip, applies the ReLU and stores the
            // voxel with 16-byte accesses instead of one channel per lane and store
            constexpr int C = 16 * NB, SC = C + 1;          // channels; staging row (one word of padding)
            float *stg = (float *)xl + wave * (64 * SC);
            __syncthreads();   // every wave is done with the halo
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int mb = 0; mb < CT_Y; ++mb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) stg[(mb * 16 + mr + i) * SC + nb * 16 + n] = acc[mb][nb][i];
            __syncthreads();
            const int x = x0 + (lane & 15), y = y0 + (lane >> 4), z = z0 + wave;
            if (x < g.nx && y < g.ny && z < g.nz) {
                const int64_t vo = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
                float v[C];
#pragma unroll
                for (int c = 0; c < C; ++c) v[c] = stg[lane * SC + c] + (bias ? bias[c] : 0.f);
                if (skip) {
                    const uint4 *sp = (const uint4 *)(skip + vo * C);
#pragma unroll
                    for (int q = 0; q < C / 8; ++q) {
                        const uint4 sq = sp[q];
                        const uint32_t sw[4] = {sq.x, sq.y, sq.z, sq.w};
#pragma unroll
                        for (int c = 0; c < 8; ++c) v[8 * q + c] += bf2f((uint16_t)(sw[c >> 1] >> (16 * (c & 1))));
                    }
                }
                if (relu)
#pragma unroll
                    for (int c = 0; c < C; ++c) v[c] = v[c] > 0.f ? v[c] : 0.f;
                if (OUT_BF16) {
                    uint4 *op = (uint4 *)((uint16_t *)out + vo * C);
#pragma unroll
                    for (int q = 0; q < C / 8; ++q) {
                        uint32_t pw[4];
#pragma unroll
                        for (int h = 0; h < 4; ++h)
                            pw[h] = (uint32_t)f2bf(v[8 * q + 2 * h]) | ((uint32_t)f2bf(v[8 * q + 2 * h + 1]) << 16);
                        op[q] = uint4{pw[0], pw[1], pw[2], pw[3]};
                    }
                } else {
                    float4 *op = (float4 *)((float *)out + vo * C);
#pragma unroll
                    for (int q = 0; q < C / 4; ++q) op[q] = float4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
                }
            }
        } else {
            // epilogue: the skip inputs are loaded together, then bias, skip, ReLU, store
            const int z = z0 + wave;
            float sk[NB][CT_Y][4];
    #pragma unroll
            for (int nb = 0; nb < NB; ++nb)
    #pragma unroll
                for (int mb = 0; mb < CT_Y; ++mb)
    #pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int x = x0 + mr + i, y = y0 + mb;
                        sk[nb][mb][i] = 0.f;
                        if (skip && x < g.nx && y < g.ny && z < g.nz)
                            sk[nb][mb][i] = bf2f(skip[(x + (int64_t)g.nx * (y + (int64_t)g.ny * z)) * g.cout + nb * 16 + n]);
                    }
    #pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int co = nb * 16 + n;
                const float bb = bias ? bias[co] : 0.f;
    #pragma unroll
                for (int mb = 0; mb < CT_Y; ++mb) {
                    const int y = y0 + mb;
    #pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int x = x0 + mr + i;
                        if (x >= g.nx || y >= g.ny || z >= g.nz) continue;
                        const int64_t vo = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
                        float val = acc[mb][nb][i] + bb + sk[nb][mb][i];
                        if (relu) val = val > 0.f ? val : 0.f;
                        if (OUT_BF16) ((uint16_t *)out)[vo * g.cout + co] = f2bf(val);
                        else ((float *)out)[vo * g.cout + co] = val;
                    }
                }
            }
        }
    }
}

constexpr size_t CONV_LDS_MAX = 96 * 1024;

// launch of k_conv: NB = cout / 16 column blocks; 4 voxel blocks per wave on
// large levels (weight fragments reused four times), 1 on small ones (more waves)
template <bool OUT_BF16>
hipError_t launch_conv(hipStream_t st, const ConvGeo &g, const uint16_t *X, const void *Wf, int KB, const float *bias,
                       const uint16_t *skip, int relu, void *out)
{
    const int NB = (g.cout + 15) / 16;
    if ((g.cin == 4 || g.cin == 16 || g.cin == 32) && conv_lds_bytes(g.cin, KB, NB) <= CONV_LDS_MAX && g.V >= 4096) {
        static bool attr[2][5][3] = {};
        const size_t sh = conv_lds_bytes(g.cin, KB, NB);
        const int64_t nbricks = (int64_t)((g.nx + CT_X - 1) / CT_X) * ((g.ny + CT_Y - 1) / CT_Y) * ((g.nz + CT_Z - 1) / CT_Z);
        // a few workgroups per CU, each walking many bricks with its weights staged once
        const unsigned nwg = (unsigned)std::min<int64_t>(nbricks, 1024);
        const int ci = g.cin == 4 ? 0 : (g.cin == 16 ? 1 : 2);
#define RSV_CONVL(nb, cin)                                                                                                \
    do {                                                                                                                  \
        if (!attr[OUT_BF16][nb][ci]) {                                                                                    \
            hipError_t e_ = hipFuncSetAttribute((const void *)k_conv_lds<nb, OUT_BF16, cin>,                              \
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)CONV_LDS_MAX);           \
            if (e_ != hipSuccess) return e_;                                                                              \
            attr[OUT_BF16][nb][ci] = true;                                                                                \
        }                                                                                                                 \
        hipLaunchKernelGGL((k_conv_lds<nb, OUT_BF16, cin>), dim3(nwg), dim3(256), sh, st, g, X, Wf, KB, bias, skip, relu, \
                           out);                                                                                          \
    } while (0)
#define RSV_CONVL_NB(cin)                          \
    do {                                           \
        if (NB == 1) RSV_CONVL(1, cin);            \
        else if (NB == 2) RSV_CONVL(2, cin);       \
        else if (NB == 4) RSV_CONVL(4, cin);       \
        else return hipErrorInvalidValue;          \
    } while (0)
        if (g.cin == 4) RSV_CONVL_NB(4);
        else if (g.cin == 16) RSV_CONVL_NB(16);
        else RSV_CONVL_NB(32);
#undef RSV_CONVL_NB
#undef RSV_CONVL
        return hipGetLastError();
    }
    const int MB = g.V >= 131072 ? 4 : 1;
    const int64_t waves = (g.V + 16 * MB - 1) / (16 * MB);
    const dim3 grid((unsigned)((waves + 3) / 4)), blk(256);
#define RSV_CONV(mb, nb)                                                                                                \
    do {                                                                                                                \
        if (g.cin % 8 == 0)                                                                                             \
            hipLaunchKernelGGL((k_conv<mb, nb, OUT_BF16, true>), grid, blk, 0, st, g, X, Wf, KB, bias, skip, relu, out);  \
        else                                                                                                            \
            hipLaunchKernelGGL((k_conv<mb, nb, OUT_BF16, false>), grid, blk, 0, st, g, X, Wf, KB, bias, skip, relu, out); \
    } while (0)
    if (MB == 4) {
        if (NB == 1) RSV_CONV(4, 1);
        else if (NB == 2) RSV_CONV(4, 2);
        else if (NB == 4) RSV_CONV(4, 4);
        else return hipErrorInvalidValue;
    } else {
        if (NB == 1) RSV_CONV(1, 1);
        else if (NB == 2) RSV_CONV(1, 2);
        else if (NB == 4) RSV_CONV(1, 4);
        else return hipErrorInvalidValue;
    }
#undef RSV_CONV
    return hipGetLastError();
}

// Weight and bias gradients, dW[tap][ci][co] = sum_v X[v + off(tap)][ci] G[v][co]
// and db[co] = sum_v G[v][co], as an MFMA GEMM over voxels on
// v_mfma_f32_16x16x32_bf16 (rows m = ci, columns n = co, k = voxel; lane l
// holds A[m = l%16][k = 8*(l/16) .. +7], B[k = 8*(l/16) .. +7][n = l%16], and
// D[m = 4*(l/16) + i][n = l%16]).  A workgroup owns one 16 x 16 channel pair
// (ci block, co block) and a chunk of bricks of 16 (x) x 4 (y) x 4 (z)
// voxels.  Per brick it stages in LDS, channel-major with 16 voxels per row,
// the input halo three times (shifted by dx = 0, 1, 2, so every A fragment is
// one aligned 16-byte read) and the gradient tile; wave w then computes the
// taps t = w, w + 4, ... for all 256 voxels (the B fragment of a k-step serves
// all its taps).  The next brick's global loads are issued before the MFMAs
// of the current one.  The rows of a channel are padded so that the 16
// channels of a fragment fall on distinct LDS banks.
//
// Split over voxels: each chunk writes one partial (taps, then the bias sums
// for ci block 0); k_dw_reduce adds them in a fixed order into the gradients.
// (Summing them inside this kernel, by the last workgroup to finish, needs a
// device-scope release per workgroup, which writes back the XCD's L2: 5x the
// time of this kernel and the reduction together at 64x64x32.)
constexpr int DW_XS = CH_Z * CH_Y * 16 + 8;   // bf16 per input channel and shift (576 + padding)
constexpr int DW_GS = CT_Z * CT_Y * 16 + 8;   // bf16 per output channel (256 + padding)
constexpr int DW_PART = 27 * 256 + 16;        // floats per partial: 27 taps x 16 x 16, then 16 bias sums
constexpr int DW_MAXCHUNK = 256;              // chunks per pair (16 groups of at most 16 in the reduction)
constexpr int DW_XU = CH_Z * CH_Y * 2 * 4;    // input staging units: (halo row, x octet, channel quad) = 288
constexpr size_t DW_LDS = (size_t)(3 * 16 * DW_XS + 16 * DW_GS) * 2;
static_assert(DW_LDS >= 256 * 16 * sizeof(float), "the bias reduction reuses the staging area");

struct DwRegs {
    v4s x[2][10];   // input units: 10 voxels (x octet + 2) x 4 channels
    v4s gq[8];      // gradient unit: 8 voxels x 4 channels
};

__global__ __launch_bounds__(256) void k_conv_dw(ConvGeo g, const uint16_t *__restrict__ X,
                                                 const uint16_t *__restrict__ G, int npairs,
                                                 int bricks_per_chunk, float *__restrict__ partials)
{
    extern __shared__ __align__(16) unsigned char dl[];
    uint16_t *xs = (uint16_t *)dl;                  // [3 dx][16 ci][DW_XS]
    uint16_t *gs = xs + 3 * 16 * DW_XS;             // [16 co][DW_GS]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int pair = blockIdx.x % npairs, chunk = blockIdx.x / npairs;
    const int cob_n = g.cout / 16, cib = pair / cob_n, cob = pair % cob_n;
    const int ntx = (g.nx + CT_X - 1) / CT_X, nty = (g.ny + CT_Y - 1) / CT_Y, ntz = (g.nz + CT_Z - 1) / CT_Z;
    const int nbricks = ntx * nty * ntz;
    const int b_begin = chunk * bricks_per_chunk;
    const int b_end = b_begin + bricks_per_chunk < nbricks ? b_begin + bricks_per_chunk : nbricks;
    const int m = lane & 15, kx = 8 * ((lane >> 4) & 1), krow = lane >> 5;
    // gradient unit of threads 0..127: channel quad gq_q, x octet gq_o, row gq_r (y = r & 3, z = r >> 2)
    const int gq_q = tid & 3, gq_o = (tid >> 2) & 1, gq_r = (tid >> 3) & 15;
    v4f acc[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
    float bq[4] = {0.f, 0.f, 0.f, 0.f};   // bias sums of channels 4 gq_q .. + 3
    DwRegs R;
    auto load = [&](int b) {
        const int x0 = (b % ntx) * CT_X, y0 = ((b / ntx) % nty) * CT_Y, z0 = (b / (ntx * nty)) * CT_Z;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int u = tid + 256 * k;
            const int q = u & 3, o = (u >> 2) & 1, r = u >> 3;
            const int hy = r % CH_Y, hz = r / CH_Y;
            const int c0 = cib * 16 + 4 * q;
            const bool ok = u < DW_XU && c0 < g.cin;
#pragma unroll
            for (int i = 0; i < 10; ++i) {
                R.x[k][i] = v4s{0, 0, 0, 0};
                if (ok) {
                    const int64_t sv = src_voxel(g, x0, y0, z0, 8 * o + i - 1, hy - 1, hz - 1);
                    if (sv >= 0) R.x[k][i] = *(const v4s *)(X + sv * g.cin + c0);
                }
            }
        }
        const int y = y0 + (gq_r & 3), z = z0 + (gq_r >> 2);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int x = x0 + 8 * gq_o + i;
            R.gq[i] = v4s{0, 0, 0, 0};
            if (tid < 128 && x < g.nx && y < g.ny && z < g.nz)
                R.gq[i] = *(const v4s *)(G + (x + (int64_t)g.nx * (y + (int64_t)g.ny * z)) * g.cout + cob * 16 + 4 * gq_q);
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int u = tid + 256 * k;
            if (u >= DW_XU) continue;
            const int q = u & 3, o = (u >> 2) & 1, r = u >> 3;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    v8s row;
#pragma unroll
                    for (int i = 0; i < 8; ++i) row[i] = R.x[k][dx + i][j];
                    *(v8s *)(xs + (size_t)(dx * 16 + 4 * q + j) * DW_XS + r * 16 + 8 * o) = row;
                }
        }
        if (tid < 128) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v8s row;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    row[i] = R.gq[i][j];
                    bq[j] += bf2f((uint16_t)R.gq[i][j]);
                }
                *(v8s *)(gs + (size_t)(4 * gq_q + j) * DW_GS + gq_r * 16 + 8 * gq_o) = row;
            }
        }
    };
    if (b_begin < b_end) load(b_begin);
    for (int b = b_begin; b < b_end; ++b) {
        __syncthreads();   // the previous brick's fragments have been read
        store();
        __syncthreads();
        if (b + 1 < b_end) load(b + 1);
        // k-step s: plane s / 2, rows 2 (s % 2) + krow, x from kx
#pragma unroll 2
        for (int s = 0; s < 8; ++s) {
            const int z = s >> 1, row = 2 * (s & 1) + krow;
            const v8bf bf = __builtin_bit_cast(v8bf, *(const v8s *)(gs + (size_t)m * DW_GS + (z * CT_Y + row) * 16 + kx));
#pragma unroll
            for (int j = 0; j < 7; ++j) {
                const int t = wave + 4 * j;
                if (t < 27) {
                    const int tdz = t / 9, tdy = (t / 3) % 3, tdx = t % 3;
                    const v8bf af = __builtin_bit_cast(
                        v8bf, *(const v8s *)(xs + (size_t)(tdx * 16 + m) * DW_XS + ((z + tdz) * CH_Y + row + tdy) * 16 + kx));
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, acc[j], 0, 0, 0);
                }
            }
        }
    }
    // this chunk's partial: taps of this wave, then (ci block 0) the bias sums
    float *part = partials + ((int64_t)chunk * npairs + pair) * DW_PART;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const int t = wave + 4 * j;
        if (t < 27)
#pragma unroll
            for (int i = 0; i < 4; ++i) part[t * 256 + (4 * (lane >> 4) + i) * 16 + m] = acc[j][i];
    }
    if (cib == 0) {
        __syncthreads();
        float *red = (float *)dl;   // [16 channels][256 threads]
#pragma unroll
        for (int c = 0; c < 16; ++c) red[c * 256 + tid] = (tid < 128 && c / 4 == gq_q) ? bq[c % 4] : 0.f;
        __syncthreads();
        if (tid < 16) {
            float t = 0.f;
            for (int q = 0; q < 256; ++q) t += red[tid * 256 + q];
            part[27 * 256 + tid] = t;
        }
    }
}

// grad_w += scale * (sum of the chunks' weight partials), grad_b likewise for
// the bias sums, in a fixed order: a workgroup owns 16 float4 of one pair's
// partial; thread t sums chunk group t / 16 (chunks t / 16, + 16, ...: up to
// 16 loads in flight), then 16 threads add the 16 group sums in group order.
__global__ __launch_bounds__(256) void k_dw_reduce(const float *__restrict__ partials, int npairs, int nchunks,
                                                   int cin, int cout, float scale, float *__restrict__ grad_w,
                                                   float *__restrict__ grad_b)
{
    __shared__ float4 gsum[16][16];
    constexpr int NE4 = DW_PART / 4, SLICES = (NE4 + 15) / 16;
    const int pair = blockIdx.x / SLICES, slice = blockIdx.x % SLICES;
    const int cob_n = cout / 16, cib = pair / cob_n, cob = pair % cob_n;
    const int gr = threadIdx.x >> 4, e4 = slice * 16 + (threadIdx.x & 15);
    const int64_t stride = (int64_t)npairs * DW_PART;
    float4 v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int ch = gr + 16 * i;
        v[i] = (e4 < NE4 && ch < nchunks) ? *(const float4 *)(partials + ch * stride + (int64_t)pair * DW_PART + 4 * e4)
                                          : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float4 s4 = v[0];
#pragma unroll
    for (int i = 1; i < 16; ++i) { s4.x += v[i].x; s4.y += v[i].y; s4.z += v[i].z; s4.w += v[i].w; }
    gsum[gr][threadIdx.x & 15] = s4;
    __syncthreads();
    if (threadIdx.x >= 16 || e4 >= NE4) return;
    float4 t4 = gsum[0][threadIdx.x];
    for (int q = 1; q < 16; ++q) {
        const float4 u = gsum[q][threadIdx.x];
        t4.x += u.x; t4.y += u.y; t4.z += u.z; t4.w += u.w;
    }
    const float sv[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int e = 4 * e4 + i;
        if (e < 27 * 256) {
            const int t = e >> 8, ci = cib * 16 + ((e >> 4) & 15), co = cob * 16 + (e & 15);
            if (ci < cin) grad_w[((int64_t)t * cin + ci) * cout + co] += scale * sv[i];
        } else if (cib == 0) {
            grad_b[cob * 16 + (e - 27 * 256)] += scale * sv[i];
        }
    }
}


// sum over chunks (fixed order), added to the gradient
__global__ void k_sum_chunks(const float *__restrict__ partials, int nchunk, int64_t n, float scale,
                             float *__restrict__ grad)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        float s = 0.f;
        for (int c = 0; c < nchunk; ++c) s += partials[(int64_t)c * n + e];
        grad[e] += scale * s;
    }
}

// ---------------------------------------------------------------- elementwise pieces

__global__ void k_pool(int nx, int ny, int nz, int C, const uint16_t *__restrict__ x, uint16_t *__restrict__ y)
{
    const int mx = nx / 2, my = ny / 2;
    const int64_t n = (int64_t)mx * my * (nz / 2) * C;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int c = (int)(e % C);
        const int64_t u = e / C;
        const int i = (int)(u % mx), j = (int)((u / mx) % my), k = (int)(u / ((int64_t)mx * my));
        float s = 0.f;
        for (int q = 0; q < 8; ++q) {
            const int ii = 2 * i + (q & 1), jj = 2 * j + ((q >> 1) & 1), kk = 2 * k + (q >> 2);
            s += bf2f(x[(ii + (int64_t)nx * (jj + (int64_t)ny * kk)) * C + c]);
        }
        y[e] = f2bf(0.125f * s);
    }
}

// adjoint of the average pool (fine grid nx,ny,nz): dx += dy(parent) / 8
__global__ void k_pool_bwd(int nx, int ny, int nz, int C, const float *__restrict__ dy, float *__restrict__ dx)
{
    const int mx = nx / 2, my = ny / 2;
    const int64_t n = (int64_t)nx * ny * nz * C;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int c = (int)(e % C);
        const int64_t v = e / C;
        const int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((int64_t)nx * ny));
        dx[e] += 0.125f * dy[((i / 2) + (int64_t)mx * ((j / 2) + (int64_t)my * (k / 2))) * C + c];
    }
}

// adjoint of nearest up-sampling (fine grid nx,ny,nz): parent = sum of 8 children
__global__ void k_up_bwd(int nx, int ny, int nz, int C, const float *__restrict__ dyf, float *__restrict__ dx)
{
    const int mx = nx / 2, my = ny / 2;
    const int64_t n = (int64_t)mx * my * (nz / 2) * C;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int c = (int)(e % C);
        const int64_t u = e / C;
        const int i = (int)(u % mx), j = (int)((u / mx) % my), k = (int)(u / ((int64_t)mx * my));
        float s = 0.f;
        for (int q = 0; q < 8; ++q) {
            const int ii = 2 * i + (q & 1), jj = 2 * j + ((q >> 1) & 1), kk = 2 * k + (q >> 2);
            s += dyf[(ii + (int64_t)nx * (jj + (int64_t)ny * kk)) * C + c];
        }
        dx[e] = s;
    }
}

// G = bf16(g * [y > 0]); optional FP32 copy of the masked gradient (skip paths)
__global__ void k_mask(int64_t n, const float *__restrict__ g, const uint16_t *__restrict__ y,
                       uint16_t *__restrict__ G, float *__restrict__ gm)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const float v = bf2f(y[e]) > 0.f ? g[e] : 0.f;
        G[e] = f2bf(v);
        if (gm) gm[e] = v;
    }
}

__global__ void k_add(int64_t n, const float *__restrict__ a, float *__restrict__ b)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) b[e] += a[e];
}

__global__ void k_f2bf(int64_t n, const float *__restrict__ a, uint16_t *__restrict__ b)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) b[e] = f2bf(a[e]);
}

// final 1x1x1 layer: y[v][co] = b[co] + sum_ci W[ci][co] d1[v][ci]
__global__ void k_final(int64_t V, int C, const uint16_t *__restrict__ d1, const float *__restrict__ W,
                        const float *__restrict__ b, float *__restrict__ y)
{
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (int64_t)gridDim.x * 256) {
        float o[3] = {b[0], b[1], b[2]};
        for (int ci = 0; ci < C; ++ci) {
            const float a = bf2f(d1[v * C + ci]);
            for (int co = 0; co < 3; ++co) o[co] += W[ci * 3 + co] * a;
        }
        for (int co = 0; co < 3; ++co) y[v * 3 + co] = o[co];
    }
}

// backward of the final layer, data part: gd1[v][ci] = sum_co W[ci][co] gy[v][co]
__global__ void k_final_bwd_data(int64_t V, int C, const float *__restrict__ W, const float *__restrict__ gy,
                                 float *__restrict__ gd1)
{
    const int64_t n = V * C;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int ci = (int)(e % C);
        const int64_t v = e / C;
        gd1[e] = W[ci * 3] * gy[v * 3] + W[ci * 3 + 1] * gy[v * 3 + 1] + W[ci * 3 + 2] * gy[v * 3 + 2];
    }
}

// weight part: partials[chunk][q] for q = ci*3 + co (sum_v d1[v][ci] gy[v][co]) and
// q = 3C + co (sum_v gy[v][co]); grid.x = q, grid.y = voxel chunk
__global__ __launch_bounds__(256) void k_final_dw(int64_t V, int C, int64_t chunk, const uint16_t *__restrict__ d1,
                                                  const float *__restrict__ gy, float *__restrict__ partials)
{
    __shared__ float red[256];
    const int q = blockIdx.x, nw = 3 * C + 3;
    const int co = q % 3, ci = q / 3;
    const int64_t v_begin = (int64_t)blockIdx.y * chunk;
    const int64_t v_end = v_begin + chunk < V ? v_begin + chunk : V;
    float s = 0.f;
    for (int64_t v = v_begin + threadIdx.x; v < v_end; v += 256)
        s += (ci < C ? bf2f(d1[v * C + ci]) : 1.f) * gy[v * 3 + co];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.y * nw + q] = red[0];
}

// network input from a residual.  rtl: tile-lane FP64 vector (or NULL), rnat:
// natural block-row FP64 vector (or NULL); s2 = sum r^2 over all entries.
// x0[v][0..2] = r/s (s = rms), x0[v][3] = standardised ln k (precomputed).
__global__ void k_prep(Geo geo, const double *__restrict__ rtl, const double *__restrict__ rnat,
                       const double *__restrict__ s2, const uint16_t *__restrict__ lnk_std,
                       uint16_t *__restrict__ x0)
{
    const int64_t V = (int64_t)geo.nx * geo.ny * geo.nz;
    const double s = sqrt(s2[0] / (double)(3 * V));
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (int64_t)gridDim.x * 256) {
        const int i = (int)(v % geo.nx), j = (int)((v / geo.nx) % geo.ny), k = (int)(v / ((int64_t)geo.nx * geo.ny));
        double r[3];
        if (rtl) {
            const int64_t sl = slot_of(geo, i, j, k);
            for (int p = 0; p < 3; ++p) r[p] = rtl[vidx(sl, p)];
        } else {
            const int64_t row = row_of(geo, i, j, k);
            for (int p = 0; p < 3; ++p) r[p] = rnat[3 * row + p];
        }
        for (int p = 0; p < 3; ++p) x0[v * 4 + p] = f2bf((float)(r[p] * inv));
        x0[v * 4 + 3] = lnk_std[v];
    }
}

// z = s * y (+ add, tile-lane, when given) back to a tile-lane (ztl) or natural (znat) FP64 vector
__global__ void k_post(Geo geo, const float *__restrict__ y, const double *__restrict__ s2, double *__restrict__ ztl,
                       double *__restrict__ znat, const double *__restrict__ add = nullptr)
{
    const int64_t V = (int64_t)geo.nx * geo.ny * geo.nz;
    const double s = sqrt(s2[0] / (double)(3 * V));
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (int64_t)gridDim.x * 256) {
        const int i = (int)(v % geo.nx), j = (int)((v / geo.nx) % geo.ny), k = (int)(v / ((int64_t)geo.nx * geo.ny));
        if (ztl) {
            const int64_t sl = slot_of(geo, i, j, k);
            for (int p = 0; p < 3; ++p)
                ztl[vidx(sl, p)] = (add ? add[vidx(sl, p)] : 0.0) + s * (double)y[v * 3 + p];
        } else {
            const int64_t row = row_of(geo, i, j, k);
            for (int p = 0; p < 3; ++p) znat[3 * row + p] = s * (double)y[v * 3 + p];
        }
    }
}

// standardised ln k (mean/std given) in voxel order, BF16; lnk given per block row
__global__ void k_lnk_std(Geo geo, const float *__restrict__ lnk, double mean, double inv_sd, uint16_t *__restrict__ out)
{
    const int64_t V = (int64_t)geo.nx * geo.ny * geo.nz;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (int64_t)gridDim.x * 256) {
        const int i = (int)(v % geo.nx), j = (int)((v / geo.nx) % geo.ny), k = (int)(v / ((int64_t)geo.nx * geo.ny));
        out[v] = f2bf((float)(((double)lnk[row_of(geo, i, j, k)] - mean) * inv_sd));
    }
}

// loss partials: sum (y - e/s)^2 and sum (e/s)^2 for one sample; e natural FP64
__global__ __launch_bounds__(256) void k_loss(Geo geo, const float *__restrict__ y, const double *__restrict__ e,
                                              const double *__restrict__ s2, double *__restrict__ partials)
{
    __shared__ double r0[256], r1[256];
    const int64_t V = (int64_t)geo.nx * geo.ny * geo.nz;
    const double s = sqrt(s2[0] / (double)(3 * V));
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    double a = 0.0, b = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (int64_t)gridDim.x * 256) {
        const int i = (int)(v % geo.nx), j = (int)((v / geo.nx) % geo.ny), k = (int)(v / ((int64_t)geo.nx * geo.ny));
        const int64_t row = row_of(geo, i, j, k);
        for (int p = 0; p < 3; ++p) {
            const double t = e[3 * row + p] * inv;
            const double d = (double)y[v * 3 + p] - t;
            a += d * d;
            b += t * t;
        }
    }
    r0[threadIdx.x] = a;
    r1[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) { r0[threadIdx.x] += r0[threadIdx.x + w]; r1[threadIdx.x] += r1[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { partials[2 * blockIdx.x] = r0[0]; partials[2 * blockIdx.x + 1] = r1[0]; }
}

// gy = scale * 2 (y - e/s) / ||e/s||^2   (tt = ||e/s||^2 in sc[0])
__global__ void k_gy(Geo geo, const float *__restrict__ y, const double *__restrict__ e, const double *__restrict__ s2,
                     const double *__restrict__ tt, float scale, float *__restrict__ gy)
{
    const int64_t V = (int64_t)geo.nx * geo.ny * geo.nz;
    const double s = sqrt(s2[0] / (double)(3 * V));
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    const double f = 2.0 * (double)scale / tt[0];
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (int64_t)gridDim.x * 256) {
        const int i = (int)(v % geo.nx), j = (int)((v / geo.nx) % geo.ny), k = (int)(v / ((int64_t)geo.nx * geo.ny));
        const int64_t row = row_of(geo, i, j, k);
        for (int p = 0; p < 3; ++p) gy[v * 3 + p] = (float)(f * ((double)y[v * 3 + p] - e[3 * row + p] * inv));
    }
}

__global__ void k_adam(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float c1, float c2)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const float mm = 0.9f * m[e] + 0.1f * g[e];
        const float vv = 0.999f * v[e] + 0.001f * g[e] * g[e];
        m[e] = mm;
        v[e] = vv;
        p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
    }
}

// pack W[tap][ci][co] (FP32) into B fragments of kw k per block (kw / 4 per
// lane): forward (k = tap*cin + ci, n = co) or transposed for the data
// gradient (k = tap'*cout + co with tap' = 26 - tap, n = ci)
__global__ void k_pack(const float *__restrict__ W, int cin, int cout, int transposed, int KB, int NB, int kw,
                       short *__restrict__ Wf)
{
    const int64_t n = (int64_t)KB * NB * 64;
    const int w = kw / 4;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int lane = (int)(e % 64);
        const int nb = (int)((e / 64) % NB);
        const int kb = (int)(e / (64 * NB));
        const int col = nb * 16 + (lane & 15);
        for (int i = 0; i < w; ++i) {
            const int k = kb * kw + w * (lane >> 4) + i;
            float wv = 0.f;
            if (!transposed) {
                if (k < 27 * cin && col < cout) wv = W[(int64_t)k * cout + col];   // k = tap*cin + ci
            } else {
                if (k < 27 * cout && col < cin) {
                    const int tp = k / cout, co = k - tp * cout;
                    wv = W[((int64_t)(26 - tp) * cin + col) * cout + co];
                }
            }
            Wf[e * w + i] = (short)f2bf(wv);
        }
    }
}

// seeded He-uniform initialisation (SplitMix64 counter hash), biases zero
__global__ void k_init(int64_t n, float *__restrict__ p, const int64_t *__restrict__ seg, int nseg, uint64_t seed)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        // seg: [woff, boff, fan_in, scale*1e6] per layer
        float val = 0.f;
        for (int l = 0; l < nseg; ++l) {
            const int64_t wo = seg[4 * l], bo = seg[4 * l + 1];
            if (e >= wo && e < bo) {
                uint64_t z = seed + (uint64_t)(e + 1) * 0x9E3779B97F4A7C15ull;
                z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
                z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
                z ^= z >> 31;
                const double u = (double)(z >> 11) * 0x1.0p-53;
                const double a = sqrt(6.0 / (double)seg[4 * l + 2]) * (double)seg[4 * l + 3] * 1e-6;
                val = (float)((2.0 * u - 1.0) * a);
            }
        }
        p[e] = val;
    }
}

inline int nblk(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 4096); }

}  // namespace

// ---------------------------------------------------------------- the network object

struct rsv_net {
    rsv_ctx *c = nullptr;
    Arch a;
    int64_t step = 0;
    float *P = nullptr, *G = nullptr, *M = nullptr, *Vv = nullptr;   // FP32 master, gradient, Adam moments
    v4s *wf[10] = {nullptr}, *wt[10] = {nullptr};                    // packed BF16 weights
    bool packed = false;
    // workspace for one grid
    int wx = 0, wy = 0, wz = 0;
    uint16_t *x0 = nullptr, *a1 = nullptr, *s1 = nullptr, *p1 = nullptr, *a2 = nullptr, *s2 = nullptr, *p2 = nullptr,
             *a3 = nullptr, *b3 = nullptr, *d2a = nullptr, *d2 = nullptr, *d1a = nullptr, *d1 = nullptr;
    uint16_t *Gb = nullptr, *lnk_std = nullptr;
    float *y = nullptr, *gy = nullptr, *g1 = nullptr, *g2 = nullptr, *gs1 = nullptr, *gs2 = nullptr, *part = nullptr;
    double *d_sc = nullptr;   // [0] sum r^2, [1] sum (e/s)^2
    int64_t part_cap = 0;

    ~rsv_net() { release(); }
    void free_ws()
    {
        void *ps[] = {x0, a1, s1, p1, a2, s2, p2, a3, b3, d2a, d2, d1a, d1, Gb, lnk_std, y, gy, g1, g2, gs1, gs2, part};
        for (void *p : ps) dev_free(p);
        x0 = a1 = s1 = p1 = a2 = s2 = p2 = a3 = b3 = d2a = d2 = d1a = d1 = Gb = lnk_std = nullptr;
        y = gy = g1 = g2 = gs1 = gs2 = part = nullptr;
        part_cap = 0;
        wx = wy = wz = 0;
    }
    void release()
    {
        free_ws();
        dev_free(P); dev_free(G); dev_free(M); dev_free(Vv); dev_free(d_sc);
        for (int l = 0; l < 10; ++l) { dev_free(wf[l]); dev_free(wt[l]); }
    }
};

static rsv_status net_pack(rsv_net *n)
{
    rsv_ctx *c = n->c;
    for (int l = 0; l < 10; ++l) {
        const int NB = n->a.cout[l] / 16, NBt = (n->a.cin[l] + 15) / 16;
        hipLaunchKernelGGL(k_pack, dim3(nblk((int64_t)n->a.kb(l) * NB * 64)), dim3(256), 0, c->stream, n->P + n->a.woff[l],
                           n->a.cin[l], n->a.cout[l], 0, n->a.kb(l), NB, conv_kw(n->a.cin[l]), (short *)n->wf[l]);
        if (l > 0)
            hipLaunchKernelGGL(k_pack, dim3(nblk((int64_t)n->a.kbt(l) * NBt * 64)), dim3(256), 0, c->stream,
                               n->P + n->a.woff[l], n->a.cin[l], n->a.cout[l], 1, n->a.kbt(l), NBt, conv_kw(n->a.cout[l]),
                               (short *)n->wt[l]);
    }
    RSV_LAUNCH(c);
    n->packed = true;
    return RSV_OK;
}

static rsv_status net_ws(rsv_net *n, int nx, int ny, int nz)
{
    if (n->wx == nx && n->wy == ny && n->wz == nz) return RSV_OK;
    rsv_ctx *c = n->c;
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    n->free_ws();
    const int64_t V1 = (int64_t)nx * ny * nz, V2 = V1 / 8, V3 = V2 / 8;
    const int c0 = n->a.c[0], c1 = n->a.c[1], c2 = n->a.c[2];
    // largest data-path gradient: full resolution with c0 or c1 channels (the
    // up-sampled input of the last decoder level), half resolution with c2
    const int64_t gmax = std::max(V1 * std::max(c0, c1), V2 * std::max(c1, c2));
    struct { void **p; size_t b; } L[] = {
        {(void **)&n->x0, (size_t)V1 * 4 * 2}, {(void **)&n->a1, (size_t)V1 * c0 * 2}, {(void **)&n->s1, (size_t)V1 * c0 * 2},
        {(void **)&n->p1, (size_t)V2 * c0 * 2}, {(void **)&n->a2, (size_t)V2 * c1 * 2}, {(void **)&n->s2, (size_t)V2 * c1 * 2},
        {(void **)&n->p2, (size_t)V3 * c1 * 2}, {(void **)&n->a3, (size_t)V3 * c2 * 2}, {(void **)&n->b3, (size_t)V3 * c2 * 2},
        {(void **)&n->d2a, (size_t)V2 * c1 * 2}, {(void **)&n->d2, (size_t)V2 * c1 * 2}, {(void **)&n->d1a, (size_t)V1 * c0 * 2},
        {(void **)&n->d1, (size_t)V1 * c0 * 2}, {(void **)&n->Gb, (size_t)gmax * 2}, {(void **)&n->lnk_std, (size_t)V1 * 2},
        {(void **)&n->y, (size_t)V1 * 3 * 4}, {(void **)&n->gy, (size_t)V1 * 3 * 4},
        {(void **)&n->g1, (size_t)gmax * 4}, {(void **)&n->g2, (size_t)gmax * 4},
        {(void **)&n->gs1, (size_t)V1 * c0 * 4}, {(void **)&n->gs2, (size_t)V2 * c1 * 4},
    };
    for (auto &e : L) {
        rsv_status s = dev_alloc(c, e.p, e.b);
        if (s != RSV_OK) { n->free_ws(); return s; }
    }
    n->wx = nx; n->wy = ny; n->wz = nz;
    return RSV_OK;
}

static rsv_status part_reserve(rsv_net *n, int64_t nfloat)
{
    if (nfloat <= n->part_cap) return RSV_OK;
    RSV_HIP(n->c, hipStreamSynchronize(n->c->stream));
    dev_free(n->part);
    n->part = nullptr;
    rsv_status s = dev_alloc(n->c, (void **)&n->part, (size_t)nfloat * sizeof(float));
    if (s == RSV_OK) n->part_cap = nfloat;
    return s;
}

// y = conv(X) + b [+ skip], relu, BF16 out
static rsv_status conv_fwd(rsv_net *n, int l, int nx, int ny, int nz, int up, const uint16_t *X, const uint16_t *skip,
                           int relu, uint16_t *out)
{
    rsv_ctx *c = n->c;
    ConvGeo g{nx, ny, nz, up, n->a.cin[l], n->a.cout[l], (int64_t)nx * ny * nz};
    if (g.cout % 16) return set_err(c, RSV_ERR_ARG, "channel count must be 16, 32 or 64");
    const hipError_t e = launch_conv<true>(c->stream, g, X, n->wf[l], n->a.kb(l), n->P + n->a.boff[l], skip, relu, out);
    if (e != hipSuccess) return set_err(c, RSV_ERR_HIP, std::string("conv launch: ") + hipGetErrorString(e));
    return RSV_OK;
}

// dX (FP32, resolution of G) = transposed conv of the BF16 gradient G
static rsv_status conv_bwd_data(rsv_net *n, int l, int nx, int ny, int nz, const uint16_t *G, float *dX)
{
    rsv_ctx *c = n->c;
    ConvGeo g{nx, ny, nz, 0, n->a.cout[l], n->a.cin[l], (int64_t)nx * ny * nz};
    if (g.cout % 16) return set_err(c, RSV_ERR_ARG, "channel count must be 16, 32 or 64");
    const hipError_t e = launch_conv<false>(c->stream, g, G, n->wt[l], n->a.kbt(l), nullptr, nullptr, 0, dX);
    if (e != hipSuccess) return set_err(c, RSV_ERR_HIP, std::string("conv launch: ") + hipGetErrorString(e));
    return RSV_OK;
}

// grad(W_l) += scale * X^T G, grad(b_l) += scale * colsum(G)
static rsv_status conv_bwd_weight(rsv_net *n, int l, int nx, int ny, int nz, int up, const uint16_t *X,
                                  const uint16_t *G, float scale, float *grad_w, float *grad_b)
{
    rsv_ctx *c = n->c;
    ConvGeo g{nx, ny, nz, up, n->a.cin[l], n->a.cout[l], (int64_t)nx * ny * nz};
    if (g.cout % 16 || g.cin > 64) return set_err(c, RSV_ERR_ARG, "channel count must be 16, 32 or 64");
    const int npairs = ((g.cin + 15) / 16) * (g.cout / 16);
    const int64_t nbricks = (int64_t)((nx + CT_X - 1) / CT_X) * ((ny + CT_Y - 1) / CT_Y) * ((nz + CT_Z - 1) / CT_Z);
    // about 256 workgroups (two per CU fit the 63 KB of LDS) of at least two bricks
    const int64_t want = std::max<int64_t>(1, std::min<int64_t>((nbricks + 1) / 2, std::max(1, 256 / npairs)));
    const int per = (int)((nbricks + want - 1) / want);
    const int nchunks = (int)((nbricks + per - 1) / per);
    if (nchunks > DW_MAXCHUNK) return set_err(c, RSV_ERR_ARG, "weight gradient: too many voxel chunks");
    rsv_status s = part_reserve(n, (int64_t)nchunks * npairs * DW_PART);
    if (s != RSV_OK) return s;
    hipLaunchKernelGGL(k_conv_dw, dim3(nchunks * npairs), dim3(256), DW_LDS, c->stream, g, X, G, npairs, per, n->part);
    constexpr int slices = (DW_PART / 4 + 15) / 16;
    hipLaunchKernelGGL(k_dw_reduce, dim3(npairs * slices), dim3(256), 0, c->stream, (const float *)n->part, npairs, nchunks,
                       g.cin, g.cout, scale, grad_w, grad_b);
    RSV_LAUNCH(c);
    return RSV_OK;
}

// forward pass; x0 must be filled; result y (FP32 [V][3])
static rsv_status net_forward(rsv_net *n, int nx, int ny, int nz)
{
    if (!n->packed) {
        rsv_status s = net_pack(n);
        if (s != RSV_OK) return s;
    }
    const int mx = nx / 2, my = ny / 2, mz = nz / 2, lx = nx / 4, ly = ny / 4, lz = nz / 4;
    const int c0 = n->a.c[0], c1 = n->a.c[1];
    rsv_ctx *c = n->c;
    ProfScope ps(c, RSV_K_NET);
    rsv_status s;
    if ((s = conv_fwd(n, 0, nx, ny, nz, 0, n->x0, nullptr, 1, n->a1)) != RSV_OK) return s;
    if ((s = conv_fwd(n, 1, nx, ny, nz, 0, n->a1, nullptr, 1, n->s1)) != RSV_OK) return s;
    hipLaunchKernelGGL(k_pool, dim3(nblk((int64_t)mx * my * mz * c0)), dim3(256), 0, c->stream, nx, ny, nz, c0, n->s1, n->p1);
    if ((s = conv_fwd(n, 2, mx, my, mz, 0, n->p1, nullptr, 1, n->a2)) != RSV_OK) return s;
    if ((s = conv_fwd(n, 3, mx, my, mz, 0, n->a2, nullptr, 1, n->s2)) != RSV_OK) return s;
    hipLaunchKernelGGL(k_pool, dim3(nblk((int64_t)lx * ly * lz * c1)), dim3(256), 0, c->stream, mx, my, mz, c1, n->s2, n->p2);
    if ((s = conv_fwd(n, 4, lx, ly, lz, 0, n->p2, nullptr, 1, n->a3)) != RSV_OK) return s;
    if ((s = conv_fwd(n, 5, lx, ly, lz, 0, n->a3, nullptr, 1, n->b3)) != RSV_OK) return s;
    if ((s = conv_fwd(n, 6, mx, my, mz, 1, n->b3, n->s2, 1, n->d2a)) != RSV_OK) return s;
    if ((s = conv_fwd(n, 7, mx, my, mz, 0, n->d2a, nullptr, 1, n->d2)) != RSV_OK) return s;
    if ((s = conv_fwd(n, 8, nx, ny, nz, 1, n->d2, n->s1, 1, n->d1a)) != RSV_OK) return s;
    if ((s = conv_fwd(n, 9, nx, ny, nz, 0, n->d1a, nullptr, 1, n->d1)) != RSV_OK) return s;
    const int64_t V1 = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL(k_final, dim3(nblk(V1)), dim3(256), 0, c->stream, V1, c0, n->d1, n->P + n->a.woff[10],
                       n->P + n->a.boff[10], n->y);
    RSV_LAUNCH(c);
    return RSV_OK;
}

// backward pass for gy (in n->g2 as [V1][3] FP32 on entry is not assumed: gy pointer given)
static rsv_status net_backward(rsv_net *n, int nx, int ny, int nz, const float *gy, float scale)
{
    rsv_ctx *c = n->c;
    ProfScope ps(c, RSV_K_NET);
    const int mx = nx / 2, my = ny / 2, mz = nz / 2, lx = nx / 4, ly = ny / 4, lz = nz / 4;
    const int c0 = n->a.c[0], c1 = n->a.c[1], c2 = n->a.c[2];
    const int64_t V1 = (int64_t)nx * ny * nz, V2 = V1 / 8, V3 = V2 / 8;
    float *gw = n->G;
#define GW(l) (gw + n->a.woff[l])
#define GB(l) (gw + n->a.boff[l])
    rsv_status s;
    // final layer: gd1 -> g1, weight and bias gradients by voxel chunks
    {
        const int nwf = c0 * 3 + 3;
        const int64_t chunk = 4096;
        const int nch = (int)((V1 + chunk - 1) / chunk);
        if ((s = part_reserve(n, (int64_t)nch * nwf)) != RSV_OK) return s;
        hipLaunchKernelGGL(k_final_bwd_data, dim3(nblk(V1 * c0)), dim3(256), 0, c->stream, V1, c0,
                           (const float *)(n->P + n->a.woff[10]), gy, n->g1);
        hipLaunchKernelGGL(k_final_dw, dim3(nwf, nch), dim3(256), 0, c->stream, V1, c0, chunk, (const uint16_t *)n->d1,
                           gy, n->part);
        hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(256), 0, c->stream, (const float *)n->part, nch, (int64_t)nwf, scale,
                           GW(10));
        RSV_LAUNCH(c);
    }
    // data-path gradients are unscaled; weight gradients are multiplied by `scale`
    auto layer = [&](int l, int lnx, int lny, int lnz, int up, const uint16_t *X, const uint16_t *Y, float *gY,
                     float *gX, float *gskip) -> rsv_status {
        const int64_t V = (int64_t)lnx * lny * lnz;
        const int64_t ne = V * n->a.cout[l];
        hipLaunchKernelGGL(k_mask, dim3(nblk(ne)), dim3(256), 0, c->stream, ne, (const float *)gY, Y, n->Gb, gskip);
        RSV_LAUNCH(c);
        rsv_status st = conv_bwd_weight(n, l, lnx, lny, lnz, up, X, n->Gb, scale, GW(l), GB(l));
        if (st != RSV_OK) return st;
        if (gX) st = conv_bwd_data(n, l, lnx, lny, lnz, n->Gb, gX);
        return st;
    };
    // dec1b: in d1a, out d1
    if ((s = layer(9, nx, ny, nz, 0, n->d1a, n->d1, n->g1, n->g2, nullptr)) != RSV_OK) return s;
    // dec1a: out d1a = relu(conv8(up(d2)) + s1); skip gradient -> gs1
    if ((s = layer(8, nx, ny, nz, 1, n->d2, n->d1a, n->g2, n->g1, n->gs1)) != RSV_OK) return s;
    hipLaunchKernelGGL(k_up_bwd, dim3(nblk(V2 * c1)), dim3(256), 0, c->stream, nx, ny, nz, c1, (const float *)n->g1, n->g2);
    // dec2b
    if ((s = layer(7, mx, my, mz, 0, n->d2a, n->d2, n->g2, n->g1, nullptr)) != RSV_OK) return s;
    // dec2a: skip gradient -> gs2
    if ((s = layer(6, mx, my, mz, 1, n->b3, n->d2a, n->g1, n->g2, n->gs2)) != RSV_OK) return s;
    hipLaunchKernelGGL(k_up_bwd, dim3(nblk(V3 * c2)), dim3(256), 0, c->stream, mx, my, mz, c2, (const float *)n->g2, n->g1);
    // enc3b, enc3a
    if ((s = layer(5, lx, ly, lz, 0, n->a3, n->b3, n->g1, n->g2, nullptr)) != RSV_OK) return s;
    if ((s = layer(4, lx, ly, lz, 0, n->p2, n->a3, n->g2, n->g1, nullptr)) != RSV_OK) return s;
    // pool 2: gs2 += pool_bwd(gp2)
    hipLaunchKernelGGL(k_pool_bwd, dim3(nblk(V2 * c1)), dim3(256), 0, c->stream, mx, my, mz, c1, (const float *)n->g1, n->gs2);
    // enc2b, enc2a
    if ((s = layer(3, mx, my, mz, 0, n->a2, n->s2, n->gs2, n->g1, nullptr)) != RSV_OK) return s;
    if ((s = layer(2, mx, my, mz, 0, n->p1, n->a2, n->g1, n->g2, nullptr)) != RSV_OK) return s;
    hipLaunchKernelGGL(k_pool_bwd, dim3(nblk(V1 * c0)), dim3(256), 0, c->stream, nx, ny, nz, c0, (const float *)n->g2, n->gs1);
    // enc1b, enc1a
    if ((s = layer(1, nx, ny, nz, 0, n->a1, n->s1, n->gs1, n->g1, nullptr)) != RSV_OK) return s;
    if ((s = layer(0, nx, ny, nz, 0, n->x0, n->a1, n->g1, nullptr, nullptr)) != RSV_OK) return s;
#undef GW
#undef GB
    RSV_LAUNCH(c);
    return RSV_OK;
}

static rsv_status dims_check(rsv_ctx *c, const rsv_grid *g)
{
    if (g->geo.nx % 4 || g->geo.ny % 4 || g->geo.nz % 4)
        return set_err(c, RSV_ERR_ARG, "learned preconditioner needs grid dimensions that are multiples of 4");
    return RSV_OK;
}

// standardised ln k channel (mean/std over the grid, FP64 on the host) into out[V]
static rsv_status set_lnk(rsv_net *n, const rsv_grid *g, const float *lnk_dev, uint16_t *out)
{
    rsv_ctx *c = n->c;
    const int64_t V = g->ncell;
    std::vector<float> h(V);
    RSV_HIP(c, hipMemcpyAsync(h.data(), lnk_dev, V * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    double m = 0.0, m2 = 0.0;
    for (float v : h) m += v;
    m /= (double)V;
    for (float v : h) m2 += ((double)v - m) * ((double)v - m);
    const double sd = std::sqrt(m2 / (double)V);
    hipLaunchKernelGGL(k_lnk_std, dim3(nblk(V)), dim3(256), 0, c->stream, g->geo, lnk_dev, m, sd > 0 ? 1.0 / sd : 0.0,
                       out);
    RSV_LAUNCH(c);
    return RSV_OK;
}

// Fills x0 from r (tile-lane rtl or natural rnat) and leaves sum r^2 in n->d_sc[0]
static rsv_status prep(rsv_net *n, const rsv_grid *g, const double *rtl, const double *rnat, const uint16_t *lnk_std)
{
    rsv_ctx *c = n->c;
    const int64_t len = rtl ? g->nv : 3 * g->ncell;
    rsv_status s = launch_dot(c, len, rtl ? rtl : rnat, rtl ? rtl : rnat, SC_MISC);
    if (s != RSV_OK) return s;
    RSV_HIP(c, hipMemcpyAsync(n->d_sc, c->d_scal + SC_MISC, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    hipLaunchKernelGGL(k_prep, dim3(nblk(g->ncell)), dim3(256), 0, c->stream, g->geo, rtl, rnat, (const double *)n->d_sc,
                       lnk_std, n->x0);
    RSV_LAUNCH(c);
    return RSV_OK;
}

struct Learned : PcImpl {
    rsv_matrix *M = nullptr;
    rsv_net *net = nullptr;
    uint16_t *lnk_std = nullptr;   // this preconditioner's standardised ln k channel
    PcImpl *base = nullptr;        // mode 1: the BILU0 step the network corrects
    double *t1 = nullptr, *r1 = nullptr;   // mode 1: BILU0^-1 r and r - A t1 (tile-lane)
    ~Learned() override
    {
        dev_free(lnk_std);
        dev_free(t1);
        dev_free(r1);
    }
    int64_t bytes() const override { return M->g->ncell * 2 + (base ? 2 * M->g->nv * (int64_t)sizeof(double) : 0); }
    rsv_status apply(const double *r, double *z) override
    {
        rsv_grid *g = M->g;
        rsv_ctx *c = net->c;
        rsv_status s = net_ws(net, g->geo.nx, g->geo.ny, g->geo.nz);
        const double *in = r;
        if (s == RSV_OK && base) {
            s = base->apply(r, t1);
            if (s == RSV_OK) s = launch_spmv(c, g->geo, M->d_A, SPMV_RESID, t1, r1, r, 0.0, 0.0, SC_MISC);
            in = r1;
        }
        if (s == RSV_OK) s = prep(net, g, in, nullptr, lnk_std);
        if (s == RSV_OK) s = net_forward(net, g->geo.nx, g->geo.ny, g->geo.nz);
        if (s != RSV_OK) return s;
        hipLaunchKernelGGL(k_post, dim3(nblk(g->ncell)), dim3(256), 0, c->stream, g->geo, (const float *)net->y,
                           (const double *)net->d_sc, z, (double *)nullptr, (const double *)(base ? t1 : nullptr));
        RSV_LAUNCH(c);
        return RSV_OK;
    }
};

rsv_status learned_create(rsv_matrix *A, const rsv_pc_params *p, PcImpl **out, PcImpl *base)
{
    rsv_ctx *c = A->g->ctx;
    if (!p->net || !p->lnk) return set_err(c, RSV_ERR_ARG, "learned preconditioner needs net and lnk");
    rsv_status s = dims_check(c, A->g);
    if (s != RSV_OK) return s;
    rsv_net *n = p->net;
    if (n->c != c) return set_err(c, RSV_ERR_ARG, "network belongs to another context");
    Learned *L = new (std::nothrow) Learned();
    if (!L) return set_err(c, RSV_ERR_OOM, "learned");
    L->M = A;
    L->net = n;
    s = dev_alloc(c, (void **)&L->lnk_std, (size_t)A->g->ncell * 2);
    if (s == RSV_OK) s = set_lnk(n, A->g, p->lnk, L->lnk_std);
    if (s == RSV_OK) s = net_ws(n, A->g->geo.nx, A->g->geo.ny, A->g->geo.nz);
    if (s == RSV_OK && p->learned_mode == 1) {
        if (!base) s = set_err(c, RSV_ERR_ARG, "learned mode 1 needs the BILU0 base");
        L->base = base;
        if (s == RSV_OK) s = dev_alloc(c, (void **)&L->t1, (size_t)A->g->nv * sizeof(double));
        if (s == RSV_OK) s = dev_alloc(c, (void **)&L->r1, (size_t)A->g->nv * sizeof(double));
        // phantom slots of the tile-lane vectors stay zero
        if (s == RSV_OK && (hipMemsetAsync(L->t1, 0, (size_t)A->g->nv * sizeof(double), c->stream) != hipSuccess ||
                            hipMemsetAsync(L->r1, 0, (size_t)A->g->nv * sizeof(double), c->stream) != hipSuccess))
            s = set_err(c, RSV_ERR_HIP, "hipMemsetAsync");
    } else if (s == RSV_OK && p->learned_mode != 0) {
        s = set_err(c, RSV_ERR_ARG, "learned_mode must be 0 or 1");
    }
    if (s != RSV_OK) { delete L; return s; }
    *out = L;
    return RSV_OK;
}

extern "C" {

rsv_status rsv_net_create(rsv_ctx *c, const rsv_net_arch *arch, uint64_t seed, rsv_net **out)
{
    if (!c || !arch || !out) return set_err(c, RSV_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (arch->levels != 3) return set_err(c, RSV_ERR_ARG, "only 3-level networks are supported");
    for (int q : {arch->c0, arch->c1, arch->c2})
        if (q != 16 && q != 32 && q != 64) return set_err(c, RSV_ERR_ARG, "channel counts must be 16, 32 or 64");
    rsv_net *n = new (std::nothrow) rsv_net();
    if (!n) return set_err(c, RSV_ERR_OOM, "net");
    n->c = c;
    n->a.init(arch->c0, arch->c1, arch->c2);
    const size_t pb = (size_t)n->a.np * sizeof(float);
    rsv_status s = dev_alloc(c, (void **)&n->P, pb);
    if (s == RSV_OK) s = dev_alloc(c, (void **)&n->G, pb);
    if (s == RSV_OK) s = dev_alloc(c, (void **)&n->M, pb);
    if (s == RSV_OK) s = dev_alloc(c, (void **)&n->Vv, pb);
    if (s == RSV_OK) s = dev_alloc(c, (void **)&n->d_sc, 8 * sizeof(double));
    for (int l = 0; l < 10 && s == RSV_OK; ++l) {
        s = dev_alloc(c, (void **)&n->wf[l], (size_t)n->a.kb(l) * (n->a.cout[l] / 16) * 64 * conv_frag_bytes(n->a.cin[l]));
        if (s == RSV_OK)
            s = dev_alloc(c, (void **)&n->wt[l],
                          (size_t)n->a.kbt(l) * ((n->a.cin[l] + 15) / 16) * 64 * conv_frag_bytes(n->a.cout[l]));
    }
    if (s != RSV_OK) { delete n; return s; }
    // He-uniform init; the final layer is scaled by 0.1 so an untrained net starts small
    std::vector<int64_t> seg(4 * NL);
    for (int l = 0; l < NL; ++l) {
        seg[4 * l] = n->a.woff[l];
        seg[4 * l + 1] = n->a.boff[l];
        seg[4 * l + 2] = (int64_t)(l < 10 ? 27 : 1) * n->a.cin[l];
        seg[4 * l + 3] = l < 10 ? 1000000 : 100000;
    }
    int64_t *dseg = nullptr;
    s = dev_alloc(c, (void **)&dseg, seg.size() * sizeof(int64_t));
    if (s == RSV_OK && hipMemcpy(dseg, seg.data(), seg.size() * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess)
        s = set_err(c, RSV_ERR_HIP, "hipMemcpy");
    if (s == RSV_OK) {
        hipLaunchKernelGGL(k_init, dim3(nblk(n->a.np)), dim3(256), 0, c->stream, n->a.np, n->P, (const int64_t *)dseg, NL,
                           seed * 0xD1B54A32D192ED03ull + 0x632BE59BD9B4E019ull);
        if (hipMemsetAsync(n->M, 0, pb, c->stream) != hipSuccess || hipMemsetAsync(n->Vv, 0, pb, c->stream) != hipSuccess)
            s = set_err(c, RSV_ERR_HIP, "hipMemsetAsync");
        if (hipStreamSynchronize(c->stream) != hipSuccess) s = set_err(c, RSV_ERR_HIP, "sync");
    }
    dev_free(dseg);
    if (s == RSV_OK) s = net_pack(n);
    if (s != RSV_OK) { delete n; return s; }
    *out = n;
    return RSV_OK;
}

void rsv_net_destroy(rsv_net *n)
{
    if (!n) return;
    (void)hipStreamSynchronize(n->c->stream);
    delete n;
}

int64_t rsv_net_num_params(const rsv_net *n) { return n ? n->a.np : 0; }

rsv_status rsv_net_get_params(rsv_net *n, float *h, int64_t cnt)
{
    if (!n || !h || cnt != n->a.np) return set_err(n ? n->c : nullptr, RSV_ERR_ARG, "bad parameter buffer");
    RSV_HIP(n->c, hipMemcpyAsync(h, n->P, cnt * sizeof(float), hipMemcpyDeviceToHost, n->c->stream));
    RSV_HIP(n->c, hipStreamSynchronize(n->c->stream));
    return RSV_OK;
}

rsv_status rsv_net_set_params(rsv_net *n, const float *h, int64_t cnt)
{
    if (!n || !h || cnt != n->a.np) return set_err(n ? n->c : nullptr, RSV_ERR_ARG, "bad parameter buffer");
    RSV_HIP(n->c, hipMemcpyAsync(n->P, h, cnt * sizeof(float), hipMemcpyHostToDevice, n->c->stream));
    RSV_HIP(n->c, hipMemsetAsync(n->M, 0, cnt * sizeof(float), n->c->stream));
    RSV_HIP(n->c, hipMemsetAsync(n->Vv, 0, cnt * sizeof(float), n->c->stream));
    n->step = 0;
    rsv_status s = net_pack(n);
    if (s != RSV_OK) return s;
    RSV_HIP(n->c, hipStreamSynchronize(n->c->stream));
    return RSV_OK;
}

rsv_status rsv_net_save(rsv_net *n, const char *path)
{
    if (!n || !path) return set_err(n ? n->c : nullptr, RSV_ERR_ARG, "NULL argument");
    std::vector<float> h(n->a.np);
    rsv_status s = rsv_net_get_params(n, h.data(), n->a.np);
    if (s != RSV_OK) return s;
    FILE *f = fopen(path, "wb");
    if (!f) return set_err(n->c, RSV_ERR_ARG, std::string("cannot open ") + path);
    const char magic[8] = {'R', 'S', 'V', 'N', 'E', 'T', '1', 0};
    const int32_t hdr[4] = {3, n->a.c[0], n->a.c[1], n->a.c[2]};
    const int64_t meta[2] = {n->a.np, n->step};
    bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(hdr, 4, 4, f) == 4 && fwrite(meta, 8, 2, f) == 2 &&
              fwrite(h.data(), 4, h.size(), f) == h.size();
    fclose(f);
    return ok ? RSV_OK : set_err(n->c, RSV_ERR_ARG, "write failed");
}

rsv_status rsv_net_load(rsv_net *n, const char *path)
{
    if (!n || !path) return set_err(n ? n->c : nullptr, RSV_ERR_ARG, "NULL argument");
    FILE *f = fopen(path, "rb");
    if (!f) return set_err(n->c, RSV_ERR_ARG, std::string("cannot open ") + path);
    char magic[8];
    int32_t hdr[4];
    int64_t meta[2];
    bool ok = fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "RSVNET1", 7) == 0 && fread(hdr, 4, 4, f) == 4 &&
              fread(meta, 8, 2, f) == 2 && hdr[1] == n->a.c[0] && hdr[2] == n->a.c[1] && hdr[3] == n->a.c[2] &&
              meta[0] == n->a.np;
    std::vector<float> h(ok ? n->a.np : 0);
    if (ok) ok = fread(h.data(), 4, h.size(), f) == h.size();
    fclose(f);
    if (!ok) return set_err(n->c, RSV_ERR_ARG, "not a network file of this architecture");
    rsv_status s = rsv_net_set_params(n, h.data(), n->a.np);
    n->step = meta[1];
    return s;
}

rsv_status rsv_net_forward(rsv_net *n, rsv_grid *g, const double *r, const float *lnk, double *z)
{
    if (!n || !g || !r || !lnk || !z) return set_err(n ? n->c : nullptr, RSV_ERR_ARG, "NULL argument");
    rsv_ctx *c = n->c;
    rsv_status s = dims_check(c, g);
    if (s == RSV_OK) s = net_ws(n, g->geo.nx, g->geo.ny, g->geo.nz);
    if (s == RSV_OK) s = set_lnk(n, g, lnk, n->lnk_std);
    if (s == RSV_OK) s = prep(n, g, nullptr, r, n->lnk_std);
    if (s == RSV_OK) s = net_forward(n, g->geo.nx, g->geo.ny, g->geo.nz);
    if (s != RSV_OK) return s;
    hipLaunchKernelGGL(k_post, dim3(nblk(g->ncell)), dim3(256), 0, c->stream, g->geo, (const float *)n->y,
                       (const double *)n->d_sc, (double *)nullptr, z);
    RSV_LAUNCH(c);
    RSV_HIP(c, hipStreamSynchronize(c->stream));
    return RSV_OK;
}

static rsv_status loss_grad_batch(rsv_net *n, rsv_grid *g, int32_t nb, const double *r, const double *e,
                                  const float *lnk, float *loss_out)
{
    rsv_ctx *c = n->c;
    if (nb < 1) return set_err(c, RSV_ERR_ARG, "batch must be >= 1");
    rsv_status s = dims_check(c, g);
    if (s == RSV_OK) s = net_ws(n, g->geo.nx, g->geo.ny, g->geo.nz);
    if (s != RSV_OK) return s;
    if (!n->packed && (s = net_pack(n)) != RSV_OK) return s;
    const int64_t V = g->ncell, N = 3 * V;
    RSV_HIP(c, hipMemsetAsync(n->G, 0, (size_t)n->a.np * sizeof(float), c->stream));
    double total = 0.0;
    const int nbk = nblk(V) < 1024 ? nblk(V) : 1024;
    if ((s = partials_reserve(c, 2 * nbk)) != RSV_OK) return s;
    for (int b = 0; b < nb; ++b) {
        if ((s = set_lnk(n, g, lnk + (int64_t)b * V, n->lnk_std)) != RSV_OK) return s;
        if ((s = prep(n, g, nullptr, r + (int64_t)b * N, n->lnk_std)) != RSV_OK) return s;
        if ((s = net_forward(n, g->geo.nx, g->geo.ny, g->geo.nz)) != RSV_OK) return s;
        hipLaunchKernelGGL(k_loss, dim3(nbk), dim3(256), 0, c->stream, g->geo, (const float *)n->y, e + (int64_t)b * N,
                           (const double *)n->d_sc, c->d_partials);
        RSV_LAUNCH(c);
        if ((s = launch_reduce(c, nbk, 2, SC_MISC)) != RSV_OK) return s;
        if ((s = scal_to_host(c, SC_MISC, 2)) != RSV_OK) return s;
        total += c->h_scal[SC_MISC] / c->h_scal[SC_MISC + 1];
        RSV_HIP(c, hipMemcpyAsync(n->d_sc + 1, c->d_scal + SC_MISC + 1, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        // gy = (2 / nb) (y - e/s) / ||e/s||^2
        hipLaunchKernelGGL(k_gy, dim3(nblk(V)), dim3(256), 0, c->stream, g->geo, (const float *)n->y, e + (int64_t)b * N,
                           (const double *)n->d_sc, (const double *)(n->d_sc + 1), 1.0f / (float)nb, n->gy);
        RSV_LAUNCH(c);
        if ((s = net_backward(n, g->geo.nx, g->geo.ny, g->geo.nz, n->gy, 1.0f)) != RSV_OK) return s;
    }
    if (loss_out) *loss_out = (float)(total / nb);
    return RSV_OK;
}

rsv_status rsv_net_loss_grad(rsv_net *n, rsv_grid *g, int32_t nb, const double *r, const double *e, const float *lnk,
                             float *loss_out, float *grad_out)
{
    if (!n || !g || !r || !e || !lnk) return set_err(n ? n->c : nullptr, RSV_ERR_ARG, "NULL argument");
    rsv_status s = loss_grad_batch(n, g, nb, r, e, lnk, loss_out);
    if (s != RSV_OK) return s;
    if (grad_out) {
        RSV_HIP(n->c, hipMemcpyAsync(grad_out, n->G, (size_t)n->a.np * sizeof(float), hipMemcpyDeviceToHost, n->c->stream));
    }
    RSV_HIP(n->c, hipStreamSynchronize(n->c->stream));
    return RSV_OK;
}

rsv_status rsv_net_train_step(rsv_net *n, rsv_grid *g, int32_t nb, const double *r, const double *e, const float *lnk,
                              float lr, float *loss_out)
{
    if (!n || !g || !r || !e || !lnk) return set_err(n ? n->c : nullptr, RSV_ERR_ARG, "NULL argument");
    rsv_status s = loss_grad_batch(n, g, nb, r, e, lnk, loss_out);
    if (s != RSV_OK) return s;
    n->step += 1;
    const float c1 = 1.0f - powf(0.9f, (float)n->step), c2 = 1.0f - powf(0.999f, (float)n->step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(n->a.np)), dim3(256), 0, n->c->stream, n->a.np, n->P, (const float *)n->G, n->M,
                       n->Vv, lr, c1, c2);
    RSV_LAUNCH(n->c);
    s = net_pack(n);
    if (s != RSV_OK) return s;
    RSV_HIP(n->c, hipStreamSynchronize(n->c->stream));
    return RSV_OK;
}

// ---------------------------------------------------------------- single-layer entry points

rsv_status rsv_conv3d(rsv_ctx *c, int32_t nx, int32_t ny, int32_t nz, int32_t cin, int32_t cout, const uint16_t *x,
                      const float *w, const float *b, float *y)
{
    if (!c || !x || !w || !y) return set_err(c, RSV_ERR_ARG, "NULL argument");
    if (cin % 4 || cin < 4 || cin > 64 || (cout != 16 && cout != 32 && cout != 64) || nx < 1 || ny < 1 || nz < 1)
        return set_err(c, RSV_ERR_ARG, "conv3d needs cin a multiple of 4 up to 64, cout 16/32/64, positive dims");
    const int KB = conv_kblocks(cin), NB = cout / 16;
    short *wf = nullptr;
    rsv_status s = dev_alloc(c, (void **)&wf, (size_t)KB * NB * 64 * conv_frag_bytes(cin));
    if (s != RSV_OK) return s;
    hipLaunchKernelGGL(k_pack, dim3(nblk((int64_t)KB * NB * 64)), dim3(256), 0, c->stream, w, cin, cout, 0, KB, NB,
                       conv_kw(cin), wf);
    ConvGeo g{nx, ny, nz, 0, cin, cout, (int64_t)nx * ny * nz};
    hipError_t e = launch_conv<false>(c->stream, g, x, wf, KB, b, nullptr, 0, y);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dev_free(wf);
    if (e != hipSuccess) return set_err(c, RSV_ERR_HIP, std::string("conv3d: ") + hipGetErrorString(e));
    return RSV_OK;
}

rsv_status rsv_conv3d_bwd(rsv_ctx *c, int32_t nx, int32_t ny, int32_t nz, int32_t cin, int32_t cout, const uint16_t *x,
                          const float *w, const uint16_t *dy, float *dx, float *dw, float *db)
{
    if (!c || !x || !w || !dy) return set_err(c, RSV_ERR_ARG, "NULL argument");
    if (cin % 4 || cin < 4 || cin > 64 || (cout != 16 && cout != 32 && cout != 64) || nx < 1 || ny < 1 || nz < 1)
        return set_err(c, RSV_ERR_ARG, "conv3d needs cin a multiple of 4 up to 64, cout 16/32/64, positive dims");
    if (dx && cin % 16) return set_err(c, RSV_ERR_ARG, "the data gradient needs cin in {16, 32, 64}");
    // a one-layer network-like view to reuse the layer kernels
    rsv_net tmp;
    tmp.c = c;
    tmp.a.init(16, 16, 16);
    tmp.a.cin[1] = cin;
    tmp.a.cout[1] = cout;
    const int KBt = conv_kblocks(cout), NBt = (cin + 15) / 16;
    rsv_status s = RSV_OK;
    ConvGeo g{nx, ny, nz, 0, cin, cout, (int64_t)nx * ny * nz};
    if (dx) {
        s = dev_alloc(c, (void **)&tmp.wt[1], (size_t)KBt * NBt * 64 * conv_frag_bytes(cout));
        if (s == RSV_OK) {
            hipLaunchKernelGGL(k_pack, dim3(nblk((int64_t)KBt * NBt * 64)), dim3(256), 0, c->stream, w, cin, cout, 1, KBt,
                               NBt, conv_kw(cout), (short *)tmp.wt[1]);
            s = conv_bwd_data(&tmp, 1, nx, ny, nz, dy, dx);
        }
    }
    if (s == RSV_OK && (dw || db)) {
        float *gw = nullptr;
        const int64_t nwb = 27LL * cin * cout + cout;
        s = dev_alloc(c, (void **)&gw, (size_t)nwb * sizeof(float));
        if (s == RSV_OK && hipMemsetAsync(gw, 0, (size_t)nwb * sizeof(float), c->stream) != hipSuccess)
            s = set_err(c, RSV_ERR_HIP, "hipMemsetAsync");
        if (s == RSV_OK) s = conv_bwd_weight(&tmp, 1, nx, ny, nz, 0, x, dy, 1.0f, gw, gw + 27LL * cin * cout);
        if (s == RSV_OK && dw)
            if (hipMemcpyAsync(dw, gw, 27LL * cin * cout * sizeof(float), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
                s = set_err(c, RSV_ERR_HIP, "hipMemcpyAsync");
        if (s == RSV_OK && db)
            if (hipMemcpyAsync(db, gw + 27LL * cin * cout, cout * sizeof(float), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
                s = set_err(c, RSV_ERR_HIP, "hipMemcpyAsync");
        if (hipStreamSynchronize(c->stream) != hipSuccess && s == RSV_OK) s = set_err(c, RSV_ERR_HIP, "sync");
        dev_free(gw);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess && s == RSV_OK) s = set_err(c, RSV_ERR_HIP, "sync");
    (void)g;
    return s;
}

}  // extern "C"
