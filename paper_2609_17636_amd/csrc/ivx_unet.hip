// Learned warm start: a U-Net (Ronneberger et al. 2015) on the dirty mosaic, trained on
// converged cold-start solutions of the Classic3D objective.  Every layer is a kernel
// here; the 3x3 convolutions are implicit GEMMs on the bf16 matrix cores.
//
// Implicit GEMM of a 3x3 convolution, NHWC: rows = output pixels p, columns = output
// channels o, reduction index k = (dy * 3 + dx) * Cin + c.  A[p][k] is the input pixel
// shifted by (dy - 1, dx - 1) (zero outside), B[k][o] = W[o][dy][dx][c].  The products run on
// gfx950's v_mfma_f32_16x16x32_bf16, one per 32-wide k step of a 16 x 16 output tile:
//   A operand : lane l holds A[l % 16][8 (l / 16) + v], v = 0..7 (8 consecutive k)
//   B operand : lane l holds B[8 (l / 16) + v][l % 16]  (the same 8 k of one column)
//   result    : lane l holds D[4 (l / 16) + v][l % 16], v = 0..3
// (A and B give each lane the same k indices, so the product does not depend on the order in
// which the instruction walks them.)
// The transposed correlation (gradient of the input) is the same kernel on flipped
// weights, and the weight gradient is a second implicit GEMM (rows o, columns k, reduction
// over pixels) split over pixel ranges with a fixed-order reduction of the partials.
#include "ivx_internal.hpp"
#include "ivx_unet.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <vector>

namespace ivx {
ivx_status set_error(ivx_status s, const std::string &msg); // defined with the objective ABI
}

using namespace ivx;

namespace {

constexpr int NT = 256;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// 8 bf16 values (as raw 16-bit patterns, element 0 in the low half of word 0) as an operand
__device__ __forceinline__ bf16x8 as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }
__device__ __forceinline__ uint4 pack8(const uint16_t *e) {
    return uint4{e[0] | ((uint32_t)e[1] << 16), e[2] | ((uint32_t)e[3] << 16), e[4] | ((uint32_t)e[5] << 16),
                 e[6] | ((uint32_t)e[7] << 16)};
}
__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------- 3x3 convolution
template <int NTW>
__global__ __launch_bounds__(NT) void k_conv3x3(const float *__restrict__ x, int n, int h, int w, int cin,
                                                const uint16_t *__restrict__ wt, const float *__restrict__ bias,
                                                int cout, int relu, const float *__restrict__ mask, int accumulate,
                                                float *__restrict__ y) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t P = (int64_t)n * h * w;
    const int64_t pbase = (int64_t)blockIdx.x * 64 + wave * 16;
    const int cobase = blockIdx.y * (16 * NTW);
    const int K = 9 * cin;
    const int row = lane & 15, kq = lane >> 4;
    const int64_t p = pbase + row;
    const bool pv = p < P;
    int pn = 0, py = 0, px = 0;
    if (pv) {
        pn = (int)(p / ((int64_t)h * w));
        const int r = (int)(p - (int64_t)pn * h * w);
        py = r / w;
        px = r - py * w;
    }
    f32x4 acc[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        // the lane's 8 k: two runs of 4 channels (cin % 4 == 0: each run stays in one tap)
        uint16_t ae[8];
#pragma unroll
        for (int hlf = 0; hlf < 2; ++hlf) {
            const int k = k0 + 8 * kq + 4 * hlf;
            float4 v = float4{0.f, 0.f, 0.f, 0.f};
            if (pv && k < K) {
                const int tap = k / cin, c = k - (k / cin) * cin;
                const int yy = py + tap / 3 - 1, xx = px + tap % 3 - 1;
                if (yy >= 0 && yy < h && xx >= 0 && xx < w)
                    v = *reinterpret_cast<const float4 *>(x + (((int64_t)pn * h + yy) * w + xx) * cin + c);
            }
            ae[4 * hlf + 0] = f2bf(v.x);
            ae[4 * hlf + 1] = f2bf(v.y);
            ae[4 * hlf + 2] = f2bf(v.z);
            ae[4 * hlf + 3] = f2bf(v.w);
        }
        const bf16x8 a = as_bf16x8(pack8(ae));
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const int co = cobase + t * 16 + row;
            uint2 u[2] = {uint2{0u, 0u}, uint2{0u, 0u}};
#pragma unroll
            for (int hlf = 0; hlf < 2; ++hlf) {
                const int k = k0 + 8 * kq + 4 * hlf;
                if (co < cout && k < K) u[hlf] = *reinterpret_cast<const uint2 *>(wt + (int64_t)co * K + k);
            }
            acc[t] = mma(a, as_bf16x8(uint4{u[0].x, u[0].y, u[1].x, u[1].y}), acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        const int co = cobase + t * 16 + row;
        if (co >= cout) continue;
        const float bb = bias ? bias[co] : 0.f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t pp = pbase + 4 * kq + v;
            if (pp >= P) continue;
            const int64_t o = pp * cout + co;
            float val = acc[t][v] + bb;
            if (relu) val = fmaxf(val, 0.f);
            if (mask && !(mask[o] > 0.f)) val = 0.f;
            if (accumulate) val += y[o];
            y[o] = val;
        }
    }
}

// LDS-tiled implicit GEMM for the 3x3 convolution: block tile 64 pixels x BN channels
// (BN = 32 NJ), k chunks of 32 staged in LDS as bf16 (A: [pixel][k], B: [channel][k], rows
// padded to 40 elements), 4 waves in a 2 x 2 arrangement, each wave 2 x NJ tiles of
// v_mfma_f32_16x16x32_bf16 (one per chunk).  The next chunk's global loads are issued before
// the current chunk's matrix products.
constexpr int TBM = 64, TBK = 32, TLD = 40;
template <int NJ>
__global__ __launch_bounds__(NT) void k_conv3x3_tiled(const float *__restrict__ x, int n, int h, int w, int cin,
                                                      const uint16_t *__restrict__ wt, const float *__restrict__ bias,
                                                      int cout, int relu, const float *__restrict__ mask,
                                                      int accumulate, float *__restrict__ y) {
    constexpr int BN = 32 * NJ;
    __shared__ __align__(16) uint16_t As[TBM * TLD];
    __shared__ __align__(16) uint16_t Bs[BN * TLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t P = (int64_t)n * h * w;
    const int K = 9 * cin;
    const int64_t m0 = (int64_t)blockIdx.x * TBM;
    const int n0 = blockIdx.y * BN;
    // ---- global -> register staging: A (pixel am, k quarter aq), B (channel rows)
    const int am = tid >> 2, aq = (tid & 3) * 8;
    const int64_t ap = m0 + am;
    int apn = 0, apy = 0, apx = 0;
    const bool apv = ap < P;
    if (apv) {
        apn = (int)(ap / ((int64_t)h * w));
        const int r = (int)(ap - (int64_t)apn * h * w);
        apy = r / w;
        apx = r - apy * w;
    }
    constexpr int BPIECES = BN * (TBK / 8);           // 8-element pieces of one B chunk
    constexpr int BROWS = (BPIECES + NT - 1) / NT;    // per thread (1 or 2)
    uint16_t ra[8];
    uint16_t rb[BROWS][8];
    auto gload = [&](int k0) {
#pragma unroll
        for (int hlf = 0; hlf < 2; ++hlf) {
            const int k = k0 + aq + 4 * hlf;
            float4 v = float4{0.f, 0.f, 0.f, 0.f};
            if (apv && k < K) {
                const int tap = k / cin, c = k - tap * cin;
                const int yy = apy + tap / 3 - 1, xx = apx + tap % 3 - 1;
                if (yy >= 0 && yy < h && xx >= 0 && xx < w)
                    v = *reinterpret_cast<const float4 *>(x + (((int64_t)apn * h + yy) * w + xx) * cin + c);
            }
            ra[4 * hlf + 0] = f2bf(v.x);
            ra[4 * hlf + 1] = f2bf(v.y);
            ra[4 * hlf + 2] = f2bf(v.z);
            ra[4 * hlf + 3] = f2bf(v.w);
        }
#pragma unroll
        for (int b = 0; b < BROWS; ++b) {
            const int e = tid + b * NT;
            const int o = e >> 2, bq = (e & 3) * 8;
#pragma unroll
            for (int hlf = 0; hlf < 2; ++hlf) {
                const int k = k0 + bq + 4 * hlf;
                uint2 u = uint2{0u, 0u};
                if (e < BPIECES && n0 + o < cout && k < K) u = *reinterpret_cast<const uint2 *>(wt + (int64_t)(n0 + o) * K + k);
                rb[b][4 * hlf + 0] = (uint16_t)(u.x & 0xFFFFu);
                rb[b][4 * hlf + 1] = (uint16_t)(u.x >> 16);
                rb[b][4 * hlf + 2] = (uint16_t)(u.y & 0xFFFFu);
                rb[b][4 * hlf + 3] = (uint16_t)(u.y >> 16);
            }
        }
    };
    auto sstore = [&]() {
        uint4 va;
        va.x = ra[0] | ((uint32_t)ra[1] << 16);
        va.y = ra[2] | ((uint32_t)ra[3] << 16);
        va.z = ra[4] | ((uint32_t)ra[5] << 16);
        va.w = ra[6] | ((uint32_t)ra[7] << 16);
        *reinterpret_cast<uint4 *>(&As[am * TLD + aq]) = va;
#pragma unroll
        for (int b = 0; b < BROWS; ++b) {
            const int e = tid + b * NT;
            if (e >= BPIECES) continue;
            const int o = e >> 2, bq = (e & 3) * 8;
            uint4 vb;
            vb.x = rb[b][0] | ((uint32_t)rb[b][1] << 16);
            vb.y = rb[b][2] | ((uint32_t)rb[b][3] << 16);
            vb.z = rb[b][4] | ((uint32_t)rb[b][5] << 16);
            vb.w = rb[b][6] | ((uint32_t)rb[b][7] << 16);
            *reinterpret_cast<uint4 *>(&Bs[o * TLD + bq]) = vb;
        }
    };
    // ---- matrix products: wave (wr, wc) owns rows 32 wr .. +32, columns 16 NJ wc .. +16 NJ
    const int wr = wave >> 1, wc = wave & 1;
    const int row = lane & 15, kq = lane >> 4;
    f32x4 acc[2][NJ];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nch = (K + TBK - 1) / TBK;
    gload(0);
    for (int kc = 0; kc < nch; ++kc) {
        __syncthreads();
        sstore();
        __syncthreads();
        if (kc + 1 < nch) gload((kc + 1) * TBK);
        static_assert(TBK == 32, "one 16x16x32 product per chunk");
        bf16x8 af[2], bfr[NJ];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            af[i] = as_bf16x8(*reinterpret_cast<const uint4 *>(&As[(wr * 32 + i * 16 + row) * TLD + 8 * kq]));
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            bfr[j] = as_bf16x8(*reinterpret_cast<const uint4 *>(&Bs[(wc * 16 * NJ + j * 16 + row) * TLD + 8 * kq]));
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[i][j] = mma(af[i], bfr[j], acc[i][j]);
    }
    // ---- epilogue: D row (pixel) 4 kq + v, column (channel) = row index of the lane
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int co = n0 + wc * 16 * NJ + j * 16 + row;
            if (co >= cout) continue;
            const float bb = bias ? bias[co] : 0.f;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t pp = m0 + wr * 32 + i * 16 + 4 * kq + v;
                if (pp >= P) continue;
                const int64_t o = pp * cout + co;
                float val = acc[i][j][v] + bb;
                if (relu) val = fmaxf(val, 0.f);
                if (mask && !(mask[o] > 0.f)) val = 0.f;
                if (accumulate) val += y[o];
                y[o] = val;
            }
        }
}

// 3x3 convolution for cin % 32 == 0 on a 2-D output patch: a block computes 4 x 16 output
// pixels (one image) x BN = 32 NJ channels.  Per chunk of 32 input channels it stages the
// patch with its one-pixel halo (6 x 18 pixels, bf16) and the chunk's weights of all nine taps
// in LDS once, and takes the A operand of every tap from the staged patch: each input value
// is read from memory once per block instead of once per tap.  4 waves in a 2 x 2
// arrangement as in k_conv3x3_tiled; one v_mfma_f32_16x16x32_bf16 per tap and chunk.
constexpr int HX_TH = 4, HX_TW = 16, HX_PH = HX_TH + 2, HX_PW = HX_TW + 2, HX_LD = 40;
template <int NJ>
__global__ __launch_bounds__(NT) void k_conv3x3_halo(const float *__restrict__ x, int n, int h, int w, int cin,
                                                     const uint16_t *__restrict__ wt, const float *__restrict__ bias,
                                                     int cout, int relu, const float *__restrict__ mask,
                                                     int accumulate, float *__restrict__ y) {
    constexpr int BN = 32 * NJ;
    __shared__ __align__(16) uint16_t Ps[HX_PH * HX_PW * HX_LD];
    __shared__ __align__(16) uint16_t Bs[9 * BN * HX_LD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x = (w + HX_TW - 1) / HX_TW, tiles_y = (h + HX_TH - 1) / HX_TH;
    const int64_t t = blockIdx.x;
    const int img = (int)(t / ((int64_t)tiles_x * tiles_y));
    const int rem = (int)(t - (int64_t)img * tiles_x * tiles_y);
    const int y0 = (rem / tiles_x) * HX_TH, x0 = (rem % tiles_x) * HX_TW;
    const int n0 = blockIdx.y * BN;
    const int K = 9 * cin;
    const int wr = wave >> 1, wc = wave & 1;
    const int row = lane & 15, kq = lane >> 4;
    f32x4 acc[2][NJ];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < cin; c0 += 32) {
        __syncthreads(); // the previous chunk's products are done with the LDS
        // patch: (6 x 18 positions) x (8 groups of 4 channels), zero outside the image
        for (int e = tid; e < HX_PH * HX_PW * 8; e += NT) {
            const int pos = e >> 3, q = e & 7;
            const int py = y0 - 1 + pos / HX_PW, px = x0 - 1 + pos % HX_PW;
            float4 v = float4{0.f, 0.f, 0.f, 0.f};
            if (py >= 0 && py < h && px >= 0 && px < w)
                v = *reinterpret_cast<const float4 *>(x + (((int64_t)img * h + py) * w + px) * cin + c0 + 4 * q);
            uint2 u;
            u.x = f2bf(v.x) | ((uint32_t)f2bf(v.y) << 16);
            u.y = f2bf(v.z) | ((uint32_t)f2bf(v.w) << 16);
            *reinterpret_cast<uint2 *>(&Ps[pos * HX_LD + 4 * q]) = u;
        }
        // weights of the nine taps: (tap, channel o) rows of 32 k, 4 pieces of 8 each
        for (int e = tid; e < 9 * BN * 4; e += NT) {
            const int r = e >> 2, piece = e & 3;
            const int tap = r / BN, o = r - tap * BN;
            uint4 u = uint4{0u, 0u, 0u, 0u};
            if (n0 + o < cout)
                u = *reinterpret_cast<const uint4 *>(wt + (int64_t)(n0 + o) * K + tap * cin + c0 + 8 * piece);
            *reinterpret_cast<uint4 *>(&Bs[r * HX_LD + 8 * piece]) = u;
        }
        __syncthreads();
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;
            bf16x8 af[2], bfr[NJ];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                // output pixel (prow, pcol) = (2 wr + i, row) of the patch reads position
                // (prow + dy, pcol + dx) of the staged patch
                const int pos = (2 * wr + i + dy) * HX_PW + row + dx;
                af[i] = as_bf16x8(*reinterpret_cast<const uint4 *>(&Ps[pos * HX_LD + 8 * kq]));
            }
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                bfr[j] = as_bf16x8(
                    *reinterpret_cast<const uint4 *>(&Bs[(tap * BN + wc * 16 * NJ + j * 16 + row) * HX_LD + 8 * kq]));
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < NJ; ++j) acc[i][j] = mma(af[i], bfr[j], acc[i][j]);
        }
    }
    // epilogue: D row 4 kq + v is the output pixel (2 wr + i, 4 kq + v) of the patch, column the
    // channel
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int co = n0 + wc * 16 * NJ + j * 16 + row;
            if (co >= cout) continue;
            const float bb = bias ? bias[co] : 0.f;
            const int py = y0 + 2 * wr + i;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int px = x0 + 4 * kq + v;
                if (py >= h || px >= w) continue;
                const int64_t o = (((int64_t)img * h + py) * w + px) * cout + co;
                float val = acc[i][j][v] + bb;
                if (relu) val = fmaxf(val, 0.f);
                if (mask && !(mask[o] > 0.f)) val = 0.f;
                if (accumulate) val += y[o];
                y[o] = val;
            }
        }
}

// Weight-gradient partials: block (k tile of 64, o tile of 64, pixel range z).
constexpr int GW_PIX = 1024;
__global__ __launch_bounds__(NT) void k_conv3x3_gw(const float *__restrict__ x, const float *__restrict__ dy,
                                                   int n, int h, int w, int cin, int cout,
                                                   float *__restrict__ part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t P = (int64_t)n * h * w;
    const int K = 9 * cin;
    const int row = lane & 15, q = lane >> 4;
    const int co = blockIdx.y * 64 + wave * 16 + row;   // A row
    const int kbase = blockIdx.x * 64;                   // 4 column tiles
    const int64_t p0 = (int64_t)blockIdx.z * GW_PIX;
    const int64_t p1 = p0 + GW_PIX < P ? p0 + GW_PIX : P;
    int tapy[4], tapx[4], tc[4];
    bool kv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int k = kbase + t * 16 + row;
        kv[t] = k < K;
        const int tap = kv[t] ? k / cin : 0;
        tc[t] = kv[t] ? k - tap * cin : 0;
        tapy[t] = tap / 3 - 1;
        tapx[t] = tap % 3 - 1;
    }
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t pb = p0; pb < p1; pb += 32) {
        uint16_t a[8], b[4][8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            a[v] = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) b[t][v] = 0;
            const int64_t p = pb + 8 * q + v;
            if (p >= p1) continue;
            if (co < cout) a[v] = f2bf(dy[p * cout + co]);
            const int pn = (int)(p / ((int64_t)h * w));
            const int r = (int)(p - (int64_t)pn * h * w);
            const int py = r / w, px = r - (r / w) * w;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int yy = py + tapy[t], xx = px + tapx[t];
                if (kv[t] && yy >= 0 && yy < h && xx >= 0 && xx < w)
                    b[t][v] = f2bf(x[(((int64_t)pn * h + yy) * w + xx) * cin + tc[t]]);
            }
        }
        const bf16x8 av = as_bf16x8(pack8(a));
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = mma(av, as_bf16x8(pack8(b[t])), acc[t]);
    }
    // D rows = output channels (4 q + v of this wave's 16), columns = k
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int k = kbase + t * 16 + row;
        if (k >= K) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int o = blockIdx.y * 64 + wave * 16 + 4 * q + v;
            if (o < cout) part[((int64_t)blockIdx.z * cout + o) * K + k] = acc[t][v];
        }
    }
}

// Weight and bias gradient partials, LDS-tiled: block (k tile of 64, o tile of 64, pixel
// range z of `ps` pixels).  The pixel range is walked in chunks of 32: dy (A, [o][pixel]) and
// the im2col view of x (B, [k][pixel]) are staged in LDS as bf16, transposed so that each
// lane's eight reduction elements are contiguous; 4 waves in a 2 x 2 arrangement each own
// 32 x 32 outputs (2 x 2 tiles of v_mfma_f32_16x16x32_bf16, one product per chunk).  Blocks of the first k tile also
// sum dy in FP32 for the bias.  part[z] = [dw partial (cout x K) | db partial (cout)].
// Requires cin % 4 == 0 and cout % 4 == 0.
constexpr int GW_PC = 32, GW_LD = 40, GW_TARGET_BLOCKS = 2048, GW_MIN_PIX = 256;
__global__ __launch_bounds__(NT) void k_conv3x3_gw_tiled(const float *__restrict__ x, const float *__restrict__ dy,
                                                         int n, int h, int w, int cin, int cout, int64_t ps,
                                                         float *__restrict__ part) {
    __shared__ __align__(16) uint16_t As[64 * GW_LD];
    __shared__ __align__(16) uint16_t Bs[64 * GW_LD];
    __shared__ float sb[16][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t P = (int64_t)n * h * w;
    const int64_t hw = (int64_t)h * w;
    const int K = 9 * cin;
    const int64_t len = (int64_t)cout * K + cout;
    const int o0 = blockIdx.y * 64, k0 = blockIdx.x * 64;
    const int64_t p0 = (int64_t)blockIdx.z * ps;
    const int64_t p1 = p0 + ps < P ? p0 + ps : P;
    // staging: pixel pair 2 sp (fastest within a wave), 4 rows g4 .. g4 + 3 of A and of B
    const int sp = tid & 15, g4 = (tid >> 4) * 4;
    const bool ov = o0 + g4 < cout;
    const int kk = k0 + g4;
    const bool kv = kk < K;
    const int tap = kv ? kk / cin : 0;
    const int tc = kk - tap * cin, tdy = tap / 3 - 1, tdx = tap % 3 - 1;
    const bool do_bias = blockIdx.x == 0;
    float4 ra[2], rb[2];
    float bs[4] = {0.f, 0.f, 0.f, 0.f};
    auto gload = [&](int64_t pc) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int64_t p = pc + 2 * sp + e;
            ra[e] = float4{0.f, 0.f, 0.f, 0.f};
            rb[e] = float4{0.f, 0.f, 0.f, 0.f};
            if (p < p1) {
                if (ov) ra[e] = *reinterpret_cast<const float4 *>(dy + p * cout + o0 + g4);
                const int pn = (int)(p / hw);
                const int r = (int)(p - pn * hw);
                const int yy = r / w + tdy, xx = r % w + tdx;
                if (kv && yy >= 0 && yy < h && xx >= 0 && xx < w)
                    rb[e] = *reinterpret_cast<const float4 *>(x + (((int64_t)pn * h + yy) * w + xx) * cin + tc);
            }
        }
    };
    auto sstore = [&]() {
        const float *a0 = reinterpret_cast<const float *>(&ra[0]), *a1 = reinterpret_cast<const float *>(&ra[1]);
        const float *b0 = reinterpret_cast<const float *>(&rb[0]), *b1 = reinterpret_cast<const float *>(&rb[1]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            *reinterpret_cast<uint32_t *>(&As[(g4 + i) * GW_LD + 2 * sp]) = f2bf(a0[i]) | ((uint32_t)f2bf(a1[i]) << 16);
            *reinterpret_cast<uint32_t *>(&Bs[(g4 + i) * GW_LD + 2 * sp]) = f2bf(b0[i]) | ((uint32_t)f2bf(b1[i]) << 16);
            bs[i] += a0[i] + a1[i];
        }
    };
    const int wr = wave >> 1, wc = wave & 1;
    const int row = lane & 15, kq = lane >> 4;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    gload(p0);
    for (int64_t pc = p0; pc < p1; pc += GW_PC) {
        __syncthreads();
        sstore();
        __syncthreads();
        if (pc + GW_PC < p1) gload(pc + GW_PC);
        static_assert(GW_PC == 32, "one 16x16x32 product per chunk");
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            af[i] = as_bf16x8(*reinterpret_cast<const uint4 *>(&As[(wr * 32 + i * 16 + row) * GW_LD + 8 * kq]));
            bfr[i] = as_bf16x8(*reinterpret_cast<const uint4 *>(&Bs[(wc * 32 + i * 16 + row) * GW_LD + 8 * kq]));
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = mma(af[i], bfr[j], acc[i][j]);
    }
    float *pz = part + (int64_t)blockIdx.z * len;
    // D row (o) 4 kq + v, column (k) = the lane's row index
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int k = k0 + wc * 32 + j * 16 + row;
            if (k >= K) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = o0 + wr * 32 + i * 16 + 4 * kq + v;
                if (o < cout) pz[(int64_t)o * K + k] = acc[i][j][v];
            }
        }
    if (do_bias) {
#pragma unroll
        for (int i = 0; i < 4; ++i) sb[sp][g4 + i] = bs[i];
        __syncthreads();
        if (tid < 64 && o0 + tid < cout) {
            float s = 0.f;
            for (int q = 0; q < 16; ++q) s += sb[q][tid];
            pz[(int64_t)cout * K + o0 + tid] = s;
        }
    }
}

// out[i] = sum over splits of part[z][i] in a fixed order: block = 64 consecutive i x 4
// interleaved split groups, combined in LDS.  i < nw goes to dw, the rest to db.
__global__ __launch_bounds__(NT) void k_sum_splits(const float *__restrict__ part, int splits, int64_t len,
                                                   int64_t nw, float *__restrict__ dw, float *__restrict__ db) {
    __shared__ float sh[4][64];
    const int64_t i = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    const int g = threadIdx.x >> 6;
    float s = 0.f;
    if (i < len)
        for (int z = g; z < splits; z += 4) s += part[(int64_t)z * len + i];
    sh[g][threadIdx.x & 63] = s;
    __syncthreads();
    if (g == 0 && i < len) {
        const float t = (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
        if (i < nw) dw[i] = t;
        else db[i - nw] = t;
    }
}

// dw[i] = sum over splits of part[s][i] (fixed order)
__global__ __launch_bounds__(NT) void k_sum_parts(const float *__restrict__ part, int splits, int64_t len,
                                                  float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= len) return;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[(int64_t)z * len + i];
    out[i] = s;
}

// db[o] = sum over pixels of dy[p][o]; one block per channel, fixed-order tree
__global__ __launch_bounds__(NT) void k_colsum(const float *__restrict__ dy, int64_t P, int c, float *__restrict__ out) {
    __shared__ float sh[NT];
    const int o = blockIdx.x;
    float s = 0.f;
    for (int64_t p = threadIdx.x; p < P; p += NT) s += dy[p * c + o];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int m = NT / 2; m >= 1; m >>= 1) {
        if (threadIdx.x < m) sh[threadIdx.x] += sh[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[o] = sh[0];
}

// wt[c][a][b][o] = W[o][2-a][2-b][c]
__global__ __launch_bounds__(NT) void k_flip(const uint16_t *__restrict__ W, int cin, int cout, uint16_t *__restrict__ wt) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int64_t tot = (int64_t)9 * cin * cout;
    if (i >= tot) return;
    const int o = (int)(i % cout);
    const int ab = (int)((i / cout) % 9);
    const int c = (int)(i / ((int64_t)cout * 9));
    const int a = ab / 3, b = ab % 3;
    wt[i] = W[((int64_t)o * 9 + (2 - a) * 3 + (2 - b)) * cin + c];
}

__global__ __launch_bounds__(NT) void k_to_bf16(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// ---------------------------------------------------------------- other layers
__global__ __launch_bounds__(NT) void k_pool2(const float *__restrict__ x, int n, int h, int w, int c,
                                              float *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int ho = h / 2, wo = w / 2;
    const int64_t tot = (int64_t)n * ho * wo * c;
    if (i >= tot) return;
    const int ch = (int)(i % c);
    const int64_t pix = i / c;
    const int xo = (int)(pix % wo), yo = (int)((pix / wo) % ho), nn = (int)(pix / ((int64_t)wo * ho));
    const float *b = x + (((int64_t)nn * h + 2 * yo) * w + 2 * xo) * c + ch;
    y[i] = fmaxf(fmaxf(b[0], b[c]), fmaxf(b[(int64_t)w * c], b[(int64_t)w * c + c]));
}

__global__ __launch_bounds__(NT) void k_pool2_grad(const float *__restrict__ x, const float *__restrict__ dy, int n,
                                                   int h, int w, int c, int accumulate, float *__restrict__ dx) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int ho = h / 2, wo = w / 2;
    const int64_t tot = (int64_t)n * ho * wo * c;
    if (i >= tot) return;
    const int ch = (int)(i % c);
    const int64_t pix = i / c;
    const int xo = (int)(pix % wo), yo = (int)((pix / wo) % ho), nn = (int)(pix / ((int64_t)wo * ho));
    const int64_t o00 = (((int64_t)nn * h + 2 * yo) * w + 2 * xo) * c + ch;
    const int64_t off[4] = {o00, o00 + c, o00 + (int64_t)w * c, o00 + (int64_t)w * c + c};
    float m = x[off[0]];
    for (int q = 1; q < 4; ++q) m = fmaxf(m, x[off[q]]);
    bool taken = false;
    for (int q = 0; q < 4; ++q) {
        float g = 0.f;
        if (!taken && x[off[q]] == m) {
            g = dy[i];
            taken = true;
        }
        dx[off[q]] = accumulate ? dx[off[q]] + g : g;
    }
}

__global__ __launch_bounds__(NT) void k_up2(const float *__restrict__ x, int n, int h, int w, int c,
                                            float *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int64_t tot = (int64_t)n * (2 * h) * (2 * w) * c;
    if (i >= tot) return;
    const int ch = (int)(i % c);
    const int64_t pix = i / c;
    const int xo = (int)(pix % (2 * w)), yo = (int)((pix / (2 * w)) % (2 * h)), nn = (int)(pix / ((int64_t)4 * w * h));
    y[i] = x[(((int64_t)nn * h + yo / 2) * w + xo / 2) * c + ch];
}

__global__ __launch_bounds__(NT) void k_up2_grad(const float *__restrict__ dy, int n, int h, int w, int c,
                                                 float *__restrict__ dx) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int64_t tot = (int64_t)n * h * w * c;
    if (i >= tot) return;
    const int ch = (int)(i % c);
    const int64_t pix = i / c;
    const int xx = (int)(pix % w), yy = (int)((pix / w) % h), nn = (int)(pix / ((int64_t)w * h));
    const int W2 = 2 * w;
    const int64_t b = (((int64_t)nn * 2 * h + 2 * yy) * W2 + 2 * xx) * c + ch;
    dx[i] = dy[b] + dy[b + c] + dy[b + (int64_t)W2 * c] + dy[b + (int64_t)W2 * c + c];
}

// out[p] = [a[p] (ca channels), b[p] (cb channels)]
__global__ __launch_bounds__(NT) void k_concat(const float *__restrict__ a, int ca, const float *__restrict__ b, int cb,
                                               int64_t P, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int c = ca + cb;
    if (i >= P * c) return;
    const int ch = (int)(i % c);
    const int64_t p = i / c;
    out[i] = ch < ca ? a[p * ca + ch] : b[p * cb + ch - ca];
}

// da[p] = d[p][:ca]; db[p] (+)= d[p][ca:]
__global__ __launch_bounds__(NT) void k_split(const float *__restrict__ d, int ca, int cb, int64_t P,
                                              float *__restrict__ da, float *__restrict__ db, int accumulate_b) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int c = ca + cb;
    if (i >= P * c) return;
    const int ch = (int)(i % c);
    const int64_t p = i / c;
    if (ch < ca) {
        da[p * ca + ch] = d[i];
    } else {
        const int64_t o = p * cb + ch - ca;
        db[o] = accumulate_b ? db[o] + d[i] : d[i];
    }
}

// network input [n][h][w] -> [n][h][w][4] (channel 0)
__global__ __launch_bounds__(NT) void k_pad_input(const float *__restrict__ x, int64_t P, float *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= P) return;
    reinterpret_cast<float4 *>(y)[i] = float4{x[i], 0.f, 0.f, 0.f};
}

// 1x1 head: y[p] = b + sum_c w[c] x[p][c]
// Head (1x1 convolution to one channel) on c-channel pixels, c % 4 == 0: G = c / 4 threads per
// pixel hold 4 channels each (float4 loads, contiguous across the threads of a block), NT / G
// pixels per block; the per-pixel and per-channel sums run over LDS in a fixed order.
__global__ __launch_bounds__(NT) void k_head(const float *__restrict__ x, int c, int64_t P, const float *__restrict__ wt,
                                             const float *__restrict__ b, float *__restrict__ y) {
    __shared__ float sh[NT];
    const int G = c >> 2, ppb = NT / G;
    const int t = threadIdx.x, g = t % G, lp = t / G;
    const int64_t p = (int64_t)blockIdx.x * ppb + lp;
    float s = 0.f;
    if (lp < ppb && p < P) {
        const float4 v = *reinterpret_cast<const float4 *>(x + p * c + 4 * g); // c % 4 == 0: aligned
        s = wt[4 * g] * v.x + wt[4 * g + 1] * v.y + wt[4 * g + 2] * v.z + wt[4 * g + 3] * v.w;
    }
    sh[t] = s;
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * ppb + t;
    if (t < ppb && q < P) {
        float acc = b[0];
        for (int i = 0; i < G; ++i) acc += sh[t * G + i];
        y[q] = acc;
    }
}

// head backward: dx[p][k] = w[k] dy[p] [x > 0]; per-block partials of dw[k] = sum_p dy x[p][k]
// and db = sum_p dy (blocks walk the pixels grid-stride; part[block][0..c]).
constexpr int HEAD_BLOCKS = 512;
__global__ __launch_bounds__(NT) void k_head_grad(const float *__restrict__ x, int c, int64_t P,
                                                  const float *__restrict__ wt, const float *__restrict__ dy,
                                                  float *__restrict__ dx, float *__restrict__ part) {
    __shared__ float4 sw[NT];
    __shared__ float sb[NT];
    const int G = c >> 2, ppb = NT / G;
    const int t = threadIdx.x, g = t % G, lp = t / G;
    const bool act = lp < ppb;
    const float4 w4 = act ? float4{wt[4 * g], wt[4 * g + 1], wt[4 * g + 2], wt[4 * g + 3]} : float4{0.f, 0.f, 0.f, 0.f};
    float4 a4 = float4{0.f, 0.f, 0.f, 0.f};
    float ab = 0.f;
    if (act) {
        for (int64_t p = (int64_t)blockIdx.x * ppb + lp; p < P; p += (int64_t)gridDim.x * ppb) {
            const float gy = dy[p];
            const float4 v = *reinterpret_cast<const float4 *>(x + p * c + 4 * g);
            *reinterpret_cast<float4 *>(dx + p * c + 4 * g) =
                float4{v.x > 0.f ? w4.x * gy : 0.f, v.y > 0.f ? w4.y * gy : 0.f, v.z > 0.f ? w4.z * gy : 0.f,
                       v.w > 0.f ? w4.w * gy : 0.f};
            a4.x += gy * v.x;
            a4.y += gy * v.y;
            a4.z += gy * v.z;
            a4.w += gy * v.w;
            ab += gy;
        }
    }
    sw[t] = a4;
    sb[t] = ab;
    __syncthreads();
    float *pz = part + (int64_t)blockIdx.x * (c + 1);
    for (int k = t; k <= c; k += NT) {
        float s = 0.f;
        if (k < c) {
            const int gg = k >> 2, e = k & 3;
            for (int i = 0; i < ppb; ++i) {
                const float4 v = sw[i * G + gg];
                s += e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
            }
        } else {
            for (int i = 0; i < ppb; ++i) s += sb[i * G];
        }
        pz[k] = s;
    }
}

// MSE: dy = 2 (y - t) / count; per-block partial sums of (y - t)^2
__global__ __launch_bounds__(NT) void k_mse(const float *__restrict__ y, const float *__restrict__ t, int64_t count,
                                            float *__restrict__ dy, double *__restrict__ part) {
    __shared__ double sh[NT];
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    double v = 0.0;
    if (i < count) {
        const float d = y[i] - t[i];
        dy[i] = 2.f * d / (float)count;
        v = (double)d * (double)d;
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int m = NT / 2; m >= 1; m >>= 1) {
        if (threadIdx.x < m) sh[threadIdx.x] += sh[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(NT) void k_sum_double(const double *__restrict__ part, int n, double scale,
                                                   double *__restrict__ out) {
    __shared__ double sh[NT];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int m = NT / 2; m >= 1; m >>= 1) {
        if (threadIdx.x < m) sh[threadIdx.x] += sh[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0] * scale;
}

// head gradient partials -> grads (fixed order)
// One wave per output k: lane i sums partials i, i + 64, ... in order, then a fixed xor tree.
__global__ __launch_bounds__(NT) void k_head_reduce(const float *__restrict__ part, int nblk, int c,
                                                    float *__restrict__ dw, float *__restrict__ db) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = wave; k <= c; k += NT / 64) {
        float s = 0.f;
        for (int i = lane; i < nblk; i += 64) s += part[(int64_t)i * (c + 1) + k];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
        if (lane == 0) {
            if (k < c) dw[k] = s;
            else db[0] = s;
        }
    }
}

// Adam (Kingma & Ba 2015) with bias correction folded into lr_t and eps_t
__global__ __launch_bounds__(NT) void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                                             float *__restrict__ v, int64_t n, float lr_t, float eps_t) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr_t * mi / (sqrtf(vi) + eps_t);
}

unsigned nblocks(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

// ------------------------------------------------------------------ launchers
hipError_t conv3x3(const float *x, int n, int h, int w, int cin, const uint16_t *wt, const float *bias, int cout,
                   int relu, const float *mask, int accumulate, float *y, hipStream_t st) {
    const int64_t P = (int64_t)n * h * w;
    const unsigned gx = (unsigned)((P + 63) / 64);
    // The halo patch pays where a block covers 32 output channels (measured on the warm-start
    // network: 197 against 247 us per call); with 64 the tiled kernel is faster (126 against
    // 141 us), its wider weight tile already amortising the input reads.
    if (cin % 32 == 0 && cout % 32 == 0 && cout % 64 != 0) {
        const unsigned gh = (unsigned)((int64_t)n * ((h + HX_TH - 1) / HX_TH) * ((w + HX_TW - 1) / HX_TW));
        k_conv3x3_halo<1><<<dim3(gh, cout / 32), NT, 0, st>>>(x, n, h, w, cin, wt, bias, cout, relu, mask,
                                                             accumulate, y);
        return hipGetLastError();
    }
    if (cin >= 16 && cout % 64 == 0)
        k_conv3x3_tiled<2><<<dim3(gx, cout / 64), NT, 0, st>>>(x, n, h, w, cin, wt, bias, cout, relu, mask, accumulate, y);
    else if (cin >= 16 && cout % 32 == 0)
        k_conv3x3_tiled<1><<<dim3(gx, cout / 32), NT, 0, st>>>(x, n, h, w, cin, wt, bias, cout, relu, mask, accumulate, y);
    else if (cout % 64 == 0) k_conv3x3<4><<<dim3(gx, cout / 64), NT, 0, st>>>(x, n, h, w, cin, wt, bias, cout, relu, mask, accumulate, y);
    else if (cout % 32 == 0) k_conv3x3<2><<<dim3(gx, cout / 32), NT, 0, st>>>(x, n, h, w, cin, wt, bias, cout, relu, mask, accumulate, y);
    else k_conv3x3<1><<<dim3(gx, (cout + 15) / 16), NT, 0, st>>>(x, n, h, w, cin, wt, bias, cout, relu, mask, accumulate, y);
    return hipGetLastError();
}

int64_t gw_splits(int n, int h, int w) { return ((int64_t)n * h * w + GW_PIX - 1) / GW_PIX; }

bool gw_tiled(int cin, int cout) { return cin % 4 == 0 && cout % 4 == 0; }

// Split count asked for by the tiled weight gradient: about GW_TARGET_BLOCKS blocks in all
// and at least GW_MIN_PIX pixels per split; non-decreasing in P.
int64_t gw_want_splits(int64_t P, int cin, int cout) {
    const int64_t tiles = (int64_t)((9 * cin + 63) / 64) * ((cout + 63) / 64);
    const int64_t want = std::min((GW_TARGET_BLOCKS + tiles - 1) / tiles, (P + GW_MIN_PIX - 1) / GW_MIN_PIX);
    return std::max<int64_t>(want, 1);
}

// Pixels per split: a whole number of 32-pixel chunks, so at most gw_want_splits splits.
int64_t gw_split_pixels(int64_t P, int cin, int cout) {
    const int64_t want = gw_want_splits(P, cin, cout);
    const int64_t ps = (P + want - 1) / want;
    return (ps + GW_PC - 1) / GW_PC * GW_PC;
}

// Floats of split partials conv3x3_grad_weight needs for this shape; enough for any
// smaller n as well.
int64_t gw_part_len(int n, int h, int w, int cin, int cout) {
    const int64_t P = (int64_t)n * h * w;
    if (!gw_tiled(cin, cout)) return gw_splits(n, h, w) * cout * 9 * cin;
    return gw_want_splits(P, cin, cout) * ((int64_t)cout * 9 * cin + cout);
}

hipError_t conv3x3_grad_weight(const float *x, const float *dy, int n, int h, int w, int cin, int cout, float *part,
                               float *dw, float *db, hipStream_t st) {
    const int K = 9 * cin;
    if (gw_tiled(cin, cout)) {
        const int64_t P = (int64_t)n * h * w;
        const int64_t ps = gw_split_pixels(P, cin, cout);
        const int64_t splits = (P + ps - 1) / ps;
        k_conv3x3_gw_tiled<<<dim3((K + 63) / 64, (cout + 63) / 64, (unsigned)splits), NT, 0, st>>>(
            x, dy, n, h, w, cin, cout, ps, part);
        const int64_t len = (int64_t)cout * K + cout;
        k_sum_splits<<<(unsigned)((len + 63) / 64), NT, 0, st>>>(part, (int)splits, len, (int64_t)cout * K, dw, db);
        return hipGetLastError();
    }
    const int64_t splits = gw_splits(n, h, w);
    k_conv3x3_gw<<<dim3((K + 63) / 64, (cout + 63) / 64, (unsigned)splits), NT, 0, st>>>(x, dy, n, h, w, cin, cout, part);
    const int64_t len = (int64_t)cout * K;
    k_sum_parts<<<nblocks(len), NT, 0, st>>>(part, (int)splits, len, dw);
    k_colsum<<<cout, NT, 0, st>>>(dy, (int64_t)n * h * w, cout, db);
    return hipGetLastError();
}

} // namespace

// ------------------------------------------------- allocation-free weight gradient
// Split partials of ivx_nn_conv3x3_grad_weight_noalloc live in this file-scope array: one
// copy on every device the library runs on, held until the process ends.  In host code the
// array's name is not a device address; its address on the current device comes from
// hipGetSymbolAddress, taken once per device and kept.  Every call on a device shares that
// device's copy (the partials are fully written before they are read, so nothing has to
// start at zero); calls that overlap on one device race.
constexpr int64_t NOALLOC_PART_FLOATS = int64_t(8) << 20; // 32 MiB
static __device__ __align__(256) float scratch[NOALLOC_PART_FLOATS];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first call there).
hipError_t scratch_on_current_device(float **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = static_cast<float *>(ptr);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// ======================================================================= network
struct ConvLayer {
    int cin, cout, h, w;       // input channels, output channels, spatial size
    int64_t w_off, b_off;      // offsets into the master parameter vector
    uint16_t *wbf = nullptr;   // bf16 weights [cout][3][3][cin]
    uint16_t *wflip = nullptr; // bf16 flipped weights [cin][3][3][cout]
};

struct ivx_unet {
    int L = 0, base = 0, maxb = 0, H = 0, W = 0;
    std::vector<int> ch;
    std::vector<ConvLayer> conv; // enc0a enc0b enc1a ... dec{L-2}a dec{L-2}b ... dec0a dec0b
    int64_t head_w = 0, head_b = 0, nparam = 0;
    int64_t step = 0;
    std::vector<void *> bufs;
    float *params = nullptr, *grads = nullptr, *mom = nullptr, *vel = nullptr;
    float *xin = nullptr, *xin_grad_dummy = nullptr;
    std::vector<float *> ea, eb, pool, up, cat, da, db; // forward activations
    std::vector<float *> g_ea, g_eb, g_pool, g_up, g_cat, g_da, g_db;
    float *out = nullptr, *gout = nullptr;
    float *part = nullptr;
    int64_t part_len = 0;
    float *head_part = nullptr;
    double *loss_part = nullptr, *loss = nullptr;
};

namespace {

template <typename T> ivx_status ualloc(ivx_unet *u, T **p, int64_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, (size_t)(count > 0 ? count : 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(IVX_ENOMEM, "hipMalloc failed in ivx_unet_create");
    }
    u->bufs.push_back(q);
    *p = (T *)q;
    return IVX_OK;
}

void ufree(ivx_unet *u) {
    for (void *p : u->bufs) (void)hipFree(p);
    u->bufs.clear();
}

int lvl_h(const ivx_unet *u, int l) { return u->H >> l; }
int lvl_w(const ivx_unet *u, int l) { return u->W >> l; }

// conv layer indices
int enc_a(int l) { return 2 * l; }
int enc_b(int l) { return 2 * l + 1; }
int dec_a(const ivx_unet *u, int l) { return 2 * u->L + 2 * (u->L - 2 - l); }
int dec_b(const ivx_unet *u, int l) { return dec_a(u, l) + 1; }

hipError_t refresh_bf16(ivx_unet *u, hipStream_t st) {
    for (ConvLayer &c : u->conv) {
        const int64_t nw = (int64_t)9 * c.cin * c.cout;
        k_to_bf16<<<nblocks(nw), NT, 0, st>>>(u->params + c.w_off, nw, c.wbf);
        k_flip<<<nblocks(nw), NT, 0, st>>>(c.wbf, c.cin, c.cout, c.wflip);
    }
    return hipGetLastError();
}

hipError_t forward(ivx_unet *u, const float *x, int B, hipStream_t st) {
    const int64_t P0 = (int64_t)B * u->H * u->W;
    k_pad_input<<<nblocks(P0), NT, 0, st>>>(x, P0, u->xin);
    hipError_t e;
    const float *hin = u->xin;
    for (int l = 0; l < u->L; ++l) {
        const int h = lvl_h(u, l), w = lvl_w(u, l);
        if (l > 0) {
            const int64_t tot = (int64_t)B * h * w * u->ch[l - 1];
            k_pool2<<<nblocks(tot), NT, 0, st>>>(u->eb[l - 1], B, 2 * h, 2 * w, u->ch[l - 1], u->pool[l]);
            hin = u->pool[l];
        }
        const ConvLayer &a = u->conv[enc_a(l)], &b = u->conv[enc_b(l)];
        if ((e = conv3x3(hin, B, h, w, a.cin, a.wbf, u->params + a.b_off, a.cout, 1, nullptr, 0, u->ea[l], st)) != hipSuccess) return e;
        if ((e = conv3x3(u->ea[l], B, h, w, b.cin, b.wbf, u->params + b.b_off, b.cout, 1, nullptr, 0, u->eb[l], st)) != hipSuccess) return e;
    }
    const float *hcur = u->eb[u->L - 1];
    for (int l = u->L - 2; l >= 0; --l) {
        const int h = lvl_h(u, l), w = lvl_w(u, l);
        const int64_t P = (int64_t)B * h * w;
        k_up2<<<nblocks(P * u->ch[l + 1]), NT, 0, st>>>(hcur, B, h / 2, w / 2, u->ch[l + 1], u->up[l]);
        k_concat<<<nblocks(P * (u->ch[l + 1] + u->ch[l])), NT, 0, st>>>(u->up[l], u->ch[l + 1], u->eb[l], u->ch[l], P, u->cat[l]);
        const ConvLayer &a = u->conv[dec_a(u, l)], &b = u->conv[dec_b(u, l)];
        if ((e = conv3x3(u->cat[l], B, h, w, a.cin, a.wbf, u->params + a.b_off, a.cout, 1, nullptr, 0, u->da[l], st)) != hipSuccess) return e;
        if ((e = conv3x3(u->da[l], B, h, w, b.cin, b.wbf, u->params + b.b_off, b.cout, 1, nullptr, 0, u->db[l], st)) != hipSuccess) return e;
        hcur = u->db[l];
    }
    const float *top = u->L > 1 ? u->db[0] : u->eb[0];
    const int hppb = NT / (u->ch[0] / 4);
    k_head<<<(unsigned)((P0 + hppb - 1) / hppb), NT, 0, st>>>(top, u->ch[0], P0, u->params + u->head_w,
                                                            u->params + u->head_b, u->out);
    return hipGetLastError();
}

// conv layer backward: weight/bias gradients into grads, input gradient (masked by the
// input activation > 0, accumulated if asked) unless gin is null
hipError_t conv_backward(ivx_unet *u, const ConvLayer &c, int B, const float *in, const float *gout, float *gin,
                         int accumulate, hipStream_t st) {
    hipError_t e;
    if ((e = conv3x3_grad_weight(in, gout, B, c.h, c.w, c.cin, c.cout, u->part, u->grads + c.w_off, u->grads + c.b_off,
                                 st)) != hipSuccess)
        return e;
    if (gin) return conv3x3(gout, B, c.h, c.w, c.cout, c.wflip, nullptr, c.cin, 0, in, accumulate, gin, st);
    return hipSuccess;
}

hipError_t backward(ivx_unet *u, int B, hipStream_t st) {
    hipError_t e;
    const int64_t P0 = (int64_t)B * u->H * u->W;
    const float *top = u->L > 1 ? u->db[0] : u->eb[0];
    float *gtop = u->L > 1 ? u->g_db[0] : u->g_eb[0];
    const int hppb = NT / (u->ch[0] / 4);
    const unsigned hb = (unsigned)std::min<int64_t>(HEAD_BLOCKS, (P0 + hppb - 1) / hppb);
    k_head_grad<<<hb, NT, 0, st>>>(top, u->ch[0], P0, u->params + u->head_w, u->gout, gtop, u->head_part);
    k_head_reduce<<<1, NT, 0, st>>>(u->head_part, (int)hb, u->ch[0], u->grads + u->head_w, u->grads + u->head_b);
    // decoder, top level first
    for (int l = 0; l <= u->L - 2; ++l) {
        const int h = lvl_h(u, l), w = lvl_w(u, l);
        const int64_t P = (int64_t)B * h * w;
        const ConvLayer &a = u->conv[dec_a(u, l)], &b = u->conv[dec_b(u, l)];
        if ((e = conv_backward(u, b, B, u->da[l], u->g_db[l], u->g_da[l], 0, st)) != hipSuccess) return e;
        if ((e = conv_backward(u, a, B, u->cat[l], u->g_da[l], u->g_cat[l], 0, st)) != hipSuccess) return e;
        // skip half goes to the encoder output of this level, upsampled half to the level below
        k_split<<<nblocks(P * (u->ch[l + 1] + u->ch[l])), NT, 0, st>>>(u->g_cat[l], u->ch[l + 1], u->ch[l], P,
                                                                        u->g_up[l], u->g_eb[l], 0);
        float *below = (l + 1 <= u->L - 2) ? u->g_db[l + 1] : u->g_eb[u->L - 1];
        k_up2_grad<<<nblocks((int64_t)B * (h / 2) * (w / 2) * u->ch[l + 1]), NT, 0, st>>>(u->g_up[l], B, h / 2, w / 2,
                                                                                           u->ch[l + 1], below);
    }
    // encoder, bottom level first; g_eb[l] for l < L-1 already holds the skip gradient
    for (int l = u->L - 1; l >= 0; --l) {
        const int h = lvl_h(u, l), w = lvl_w(u, l);
        const ConvLayer &a = u->conv[enc_a(l)], &b = u->conv[enc_b(l)];
        if ((e = conv_backward(u, b, B, u->ea[l], u->g_eb[l], u->g_ea[l], 0, st)) != hipSuccess) return e;
        if (l == 0) {
            if ((e = conv_backward(u, a, B, u->xin, u->g_ea[l], nullptr, 0, st)) != hipSuccess) return e;
        } else {
            if ((e = conv_backward(u, a, B, u->pool[l], u->g_ea[l], u->g_pool[l], 0, st)) != hipSuccess) return e;
            const int64_t tot = (int64_t)B * h * w * u->ch[l - 1];
            k_pool2_grad<<<nblocks(tot), NT, 0, st>>>(u->eb[l - 1], u->g_pool[l], B, 2 * h, 2 * w, u->ch[l - 1], 1,
                                                      u->g_eb[l - 1]);
        }
    }
    return hipGetLastError();
}

ivx_status check_net(const ivx_unet *u) {
    if (!u) return set_error(IVX_EINVAL, "network is NULL");
    return IVX_OK;
}

#define UHIP(call)                                                                            \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return set_error(IVX_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

} // namespace

extern "C" {

ivx_status ivx_unet_create(int32_t levels, int32_t base, int32_t max_batch, int32_t height, int32_t width, uint64_t seed,
                           ivx_unet **out) {
    if (!out) return set_error(IVX_EINVAL, "out is NULL");
    *out = nullptr;
    if (levels < 1 || levels > 5 || base < 16 || base % 16 || max_batch < 1 || height < 1 || width < 1 ||
        height % (1 << (levels - 1)) || width % (1 << (levels - 1)))
        return set_error(IVX_EINVAL, "bad network geometry");
    ivx_unet *u = new ivx_unet();
    u->L = levels;
    u->base = base;
    u->maxb = max_batch;
    u->H = height;
    u->W = width;
    for (int l = 0; l < levels; ++l) u->ch.push_back(base << l);
    int64_t off = 0;
    auto add_conv = [&](int cin, int cout, int l) {
        ConvLayer c;
        c.cin = cin;
        c.cout = cout;
        c.h = height >> l;
        c.w = width >> l;
        c.w_off = off;
        off += (int64_t)9 * cin * cout;
        c.b_off = off;
        off += cout;
        u->conv.push_back(c);
    };
    int prev = 4;
    for (int l = 0; l < levels; ++l) {
        add_conv(prev, u->ch[l], l);
        add_conv(u->ch[l], u->ch[l], l);
        prev = u->ch[l];
    }
    for (int l = levels - 2; l >= 0; --l) {
        add_conv(u->ch[l + 1] + u->ch[l], u->ch[l], l);
        add_conv(u->ch[l], u->ch[l], l);
    }
    u->head_w = off;
    off += u->ch[0];
    u->head_b = off;
    off += 1;
    u->nparam = off;
    ivx_status s;
    const int64_t B = max_batch;
    auto fail = [&](ivx_status st) {
        ufree(u);
        delete u;
        return st;
    };
    if ((s = ualloc(u, &u->params, off)) || (s = ualloc(u, &u->grads, off)) || (s = ualloc(u, &u->mom, off)) ||
        (s = ualloc(u, &u->vel, off)))
        return fail(s);
    for (ConvLayer &c : u->conv) {
        if ((s = ualloc(u, &c.wbf, (int64_t)9 * c.cin * c.cout)) || (s = ualloc(u, &c.wflip, (int64_t)9 * c.cin * c.cout)))
            return fail(s);
    }
    const int64_t P0 = B * height * width;
    if ((s = ualloc(u, &u->xin, P0 * 4))) return fail(s);
    u->ea.resize(levels); u->eb.resize(levels); u->pool.resize(levels); u->up.resize(levels); u->cat.resize(levels);
    u->da.resize(levels); u->db.resize(levels);
    u->g_ea.resize(levels); u->g_eb.resize(levels); u->g_pool.resize(levels); u->g_up.resize(levels);
    u->g_cat.resize(levels); u->g_da.resize(levels); u->g_db.resize(levels);
    int64_t maxpart = 1;
    for (int l = 0; l < levels; ++l) {
        const int64_t P = B * (height >> l) * (width >> l);
        const int c = u->ch[l];
        if ((s = ualloc(u, &u->ea[l], P * c)) || (s = ualloc(u, &u->eb[l], P * c)) || (s = ualloc(u, &u->g_ea[l], P * c)) ||
            (s = ualloc(u, &u->g_eb[l], P * c)))
            return fail(s);
        if (l > 0 && ((s = ualloc(u, &u->pool[l], P * u->ch[l - 1])) || (s = ualloc(u, &u->g_pool[l], P * u->ch[l - 1]))))
            return fail(s);
        if (l <= levels - 2) {
            const int cc = u->ch[l + 1] + c;
            if ((s = ualloc(u, &u->up[l], P * u->ch[l + 1])) || (s = ualloc(u, &u->cat[l], P * cc)) ||
                (s = ualloc(u, &u->da[l], P * c)) || (s = ualloc(u, &u->db[l], P * c)) ||
                (s = ualloc(u, &u->g_up[l], P * u->ch[l + 1])) || (s = ualloc(u, &u->g_cat[l], P * cc)) ||
                (s = ualloc(u, &u->g_da[l], P * c)) || (s = ualloc(u, &u->g_db[l], P * c)))
                return fail(s);
        }
    }
    for (const ConvLayer &c : u->conv) maxpart = std::max<int64_t>(maxpart, gw_part_len((int)B, c.h, c.w, c.cin, c.cout));
    if ((s = ualloc(u, &u->part, maxpart)) || (s = ualloc(u, &u->out, P0)) || (s = ualloc(u, &u->gout, P0)) ||
        (s = ualloc(u, &u->head_part, (int64_t)HEAD_BLOCKS * (u->ch[0] + 1))) ||
        (s = ualloc(u, &u->loss_part, (int64_t)nblocks(P0))) || (s = ualloc(u, &u->loss, 1)))
        return fail(s);
    u->part_len = maxpart;
    // He-normal initialisation, zero biases
    std::vector<float> h(off, 0.f);
    std::mt19937_64 rng(seed);
    for (const ConvLayer &c : u->conv) {
        std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / (9.0 * c.cin)));
        for (int64_t i = 0; i < (int64_t)9 * c.cin * c.cout; ++i) h[c.w_off + i] = (float)nd(rng);
    }
    {
        std::normal_distribution<double> nd(0.0, std::sqrt(1.0 / u->ch[0]));
        for (int k = 0; k < u->ch[0]; ++k) h[u->head_w + k] = (float)nd(rng);
    }
    if ((s = ivx_unet_set_params(u, h.data())) != IVX_OK) return fail(s);
    *out = u;
    return IVX_OK;
}

ivx_status ivx_unet_destroy(ivx_unet *u) {
    if (!u) return IVX_OK;
    ufree(u);
    delete u;
    return IVX_OK;
}

int64_t ivx_unet_param_count(const ivx_unet *u) { return u ? u->nparam : -1; }

ivx_status ivx_unet_get_params(const ivx_unet *u, float *params) {
    ivx_status s = check_net(u);
    if (s) return s;
    if (!params) return set_error(IVX_EINVAL, "params is NULL");
    UHIP(hipMemcpy(params, u->params, u->nparam * sizeof(float), hipMemcpyDefault));
    return IVX_OK;
}

ivx_status ivx_unet_set_params(ivx_unet *u, const float *params) {
    ivx_status s = check_net(u);
    if (s) return s;
    if (!params) return set_error(IVX_EINVAL, "params is NULL");
    UHIP(hipMemcpy(u->params, params, u->nparam * sizeof(float), hipMemcpyDefault));
    UHIP(hipMemset(u->mom, 0, u->nparam * sizeof(float)));
    UHIP(hipMemset(u->vel, 0, u->nparam * sizeof(float)));
    u->step = 0;
    UHIP(refresh_bf16(u, nullptr));
    UHIP(hipDeviceSynchronize());
    return IVX_OK;
}

ivx_status ivx_unet_forward(ivx_unet *u, const float *x, float *y, int32_t batch, void *stream) {
    ivx_status s = check_net(u);
    if (s) return s;
    if (!x || !y || batch < 1 || batch > u->maxb) return set_error(IVX_EINVAL, "bad forward arguments");
    hipStream_t st = (hipStream_t)stream;
    UHIP(forward(u, x, batch, st));
    UHIP(hipMemcpyAsync(y, u->out, (size_t)batch * u->H * u->W * sizeof(float), hipMemcpyDeviceToDevice, st));
    return IVX_OK;
}

ivx_status ivx_unet_train_step(ivx_unet *u, const float *x, const float *target, int32_t batch, float lr, double *loss,
                               void *stream) {
    ivx_status s = check_net(u);
    if (s) return s;
    if (!x || !target || batch < 1 || batch > u->maxb || !(lr > 0.f)) return set_error(IVX_EINVAL, "bad train arguments");
    hipStream_t st = (hipStream_t)stream;
    UHIP(forward(u, x, batch, st));
    const int64_t P0 = (int64_t)batch * u->H * u->W;
    k_mse<<<nblocks(P0), NT, 0, st>>>(u->out, target, P0, u->gout, u->loss_part);
    k_sum_double<<<1, NT, 0, st>>>(u->loss_part, (int)nblocks(P0), 1.0 / (double)P0, u->loss);
    UHIP(backward(u, batch, st));
    u->step += 1;
    const double b1t = 1.0 - std::pow(0.9, (double)u->step), b2t = 1.0 - std::pow(0.999, (double)u->step);
    // m_hat / (sqrt(v_hat) + eps) = (sqrt(b2t) / b1t) m / (sqrt(v) + eps sqrt(b2t))
    const float lr_t = (float)(lr * std::sqrt(b2t) / b1t), eps_t = (float)(1e-8 * std::sqrt(b2t));
    k_adam<<<nblocks(u->nparam), NT, 0, st>>>(u->params, u->grads, u->mom, u->vel, u->nparam, lr_t, eps_t);
    UHIP(refresh_bf16(u, st));
    if (loss) {
        UHIP(hipMemcpyAsync(loss, u->loss, sizeof(double), hipMemcpyDefault, st));
        hipPointerAttribute_t a;
        bool dev = false;
        if (hipPointerGetAttributes(&a, loss) == hipSuccess) dev = a.type == hipMemoryTypeDevice;
        else (void)hipGetLastError();
        if (!dev) UHIP(hipStreamSynchronize(st));
    }
    return IVX_OK;
}

ivx_status ivx_unet_loss_grad(ivx_unet *u, const float *x, const float *target, int32_t batch, float *grads, double *loss,
                              void *stream) {
    ivx_status s = check_net(u);
    if (s) return s;
    if (!x || !target || !grads || batch < 1 || batch > u->maxb) return set_error(IVX_EINVAL, "bad loss_grad arguments");
    hipStream_t st = (hipStream_t)stream;
    UHIP(forward(u, x, batch, st));
    const int64_t P0 = (int64_t)batch * u->H * u->W;
    k_mse<<<nblocks(P0), NT, 0, st>>>(u->out, target, P0, u->gout, u->loss_part);
    k_sum_double<<<1, NT, 0, st>>>(u->loss_part, (int)nblocks(P0), 1.0 / (double)P0, u->loss);
    UHIP(backward(u, batch, st));
    UHIP(hipMemcpyAsync(grads, u->grads, u->nparam * sizeof(float), hipMemcpyDefault, st));
    if (loss) UHIP(hipMemcpyAsync(loss, u->loss, sizeof(double), hipMemcpyDefault, st));
    UHIP(hipStreamSynchronize(st));
    return IVX_OK;
}

// ------------------------------------------------------------------ single layers
ivx_status ivx_nn_conv3x3(const float *x, int32_t n, int32_t h, int32_t w, int32_t cin, const uint16_t *weight,
                          const float *bias, int32_t cout, int32_t relu, const float *mask, int32_t accumulate, float *y,
                          void *stream) {
    if (!x || !weight || !y || n < 1 || h < 1 || w < 1 || cin < 4 || cin % 4 || cout < 16 || cout % 16)
        return set_error(IVX_EINVAL, "bad conv3x3 arguments");
    UHIP(conv3x3(x, n, h, w, cin, weight, bias, cout, relu, mask, accumulate, y, (hipStream_t)stream));
    return IVX_OK;
}

ivx_status ivx_nn_conv3x3_grad_weight(const float *x, const float *dy, int32_t n, int32_t h, int32_t w, int32_t cin,
                                      int32_t cout, float *dw, float *db, void *stream) {
    if (!x || !dy || !dw || !db || n < 1 || h < 1 || w < 1 || cin < 1 || cout < 1)
        return set_error(IVX_EINVAL, "bad conv3x3_grad_weight arguments");
    hipStream_t st = (hipStream_t)stream;
    float *part = nullptr;
    UHIP(hipMalloc(&part, (size_t)gw_part_len(n, h, w, cin, cout) * sizeof(float)));
    hipError_t e = conv3x3_grad_weight(x, dy, n, h, w, cin, cout, part, dw, db, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(part);
    if (e != hipSuccess) return set_error(IVX_EHIP, std::string("conv3x3_grad_weight: ") + hipGetErrorString(e));
    return IVX_OK;
}

ivx_status ivx_nn_conv3x3_grad_weight_noalloc(const float *x, const float *dy, int32_t n, int32_t h, int32_t w,
                                              int32_t cin, int32_t cout, float *dw, float *db, void *stream) {
    if (!x || !dy || !dw || !db || n < 1 || h < 1 || w < 1 || cin < 1 || cout < 1)
        return set_error(IVX_EINVAL, "bad conv3x3_grad_weight_noalloc arguments");
    const int64_t need = gw_part_len(n, h, w, cin, cout);
    if (need > NOALLOC_PART_FLOATS)
        return set_error(IVX_EINVAL, "conv3x3_grad_weight_noalloc: this shape needs " + std::to_string(need) +
                                         " floats of split partials, more than the " +
                                         std::to_string(NOALLOC_PART_FLOATS) +
                                         " of the static scratch (use ivx_nn_conv3x3_grad_weight)");
    float *part = nullptr;
    hipError_t e = scratch_on_current_device(&part);
    if (e != hipSuccess)
        return set_error(IVX_EHIP, std::string("conv3x3_grad_weight_noalloc: hipGetSymbolAddress: ") +
                                       hipGetErrorString(e));
    e = conv3x3_grad_weight(x, dy, n, h, w, cin, cout, part, dw, db, (hipStream_t)stream);
    if (e != hipSuccess) return set_error(IVX_EHIP, std::string("conv3x3_grad_weight_noalloc: ") + hipGetErrorString(e));
    return IVX_OK;
}

int64_t ivx_nn_conv3x3_grad_weight_noalloc_capacity(void) { return NOALLOC_PART_FLOATS; }

int64_t ivx_nn_conv3x3_grad_weight_scratch_floats(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout) {
    if (n < 1 || h < 1 || w < 1 || cin < 1 || cout < 1) return -1;
    return gw_part_len(n, h, w, cin, cout);
}

ivx_status ivx_nn_conv3x3_flip(const uint16_t *weight, int32_t cin, int32_t cout, uint16_t *flipped, void *stream) {
    if (!weight || !flipped || cin < 1 || cout < 1) return set_error(IVX_EINVAL, "bad flip arguments");
    const int64_t nw = (int64_t)9 * cin * cout;
    k_flip<<<nblocks(nw), NT, 0, (hipStream_t)stream>>>(weight, cin, cout, flipped);
    UHIP(hipGetLastError());
    return IVX_OK;
}

ivx_status ivx_nn_to_bf16(const float *x, int64_t count, uint16_t *out, void *stream) {
    if (!x || !out || count < 0) return set_error(IVX_EINVAL, "bad to_bf16 arguments");
    if (count) k_to_bf16<<<nblocks(count), NT, 0, (hipStream_t)stream>>>(x, count, out);
    UHIP(hipGetLastError());
    return IVX_OK;
}

ivx_status ivx_nn_pool2(const float *x, int32_t n, int32_t h, int32_t w, int32_t c, float *y, void *stream) {
    if (!x || !y || n < 1 || h < 2 || w < 2 || h % 2 || w % 2 || c < 1) return set_error(IVX_EINVAL, "bad pool2 arguments");
    k_pool2<<<nblocks((int64_t)n * (h / 2) * (w / 2) * c), NT, 0, (hipStream_t)stream>>>(x, n, h, w, c, y);
    UHIP(hipGetLastError());
    return IVX_OK;
}

ivx_status ivx_nn_pool2_grad(const float *x, const float *dy, int32_t n, int32_t h, int32_t w, int32_t c,
                             int32_t accumulate, float *dx, void *stream) {
    if (!x || !dy || !dx || n < 1 || h < 2 || w < 2 || h % 2 || w % 2 || c < 1)
        return set_error(IVX_EINVAL, "bad pool2_grad arguments");
    k_pool2_grad<<<nblocks((int64_t)n * (h / 2) * (w / 2) * c), NT, 0, (hipStream_t)stream>>>(x, dy, n, h, w, c,
                                                                                              accumulate, dx);
    UHIP(hipGetLastError());
    return IVX_OK;
}

ivx_status ivx_nn_up2(const float *x, int32_t n, int32_t h, int32_t w, int32_t c, float *y, void *stream) {
    if (!x || !y || n < 1 || h < 1 || w < 1 || c < 1) return set_error(IVX_EINVAL, "bad up2 arguments");
    k_up2<<<nblocks((int64_t)n * 4 * h * w * c), NT, 0, (hipStream_t)stream>>>(x, n, h, w, c, y);
    UHIP(hipGetLastError());
    return IVX_OK;
}

ivx_status ivx_nn_up2_grad(const float *dy, int32_t n, int32_t h, int32_t w, int32_t c, float *dx, void *stream) {
    if (!dy || !dx || n < 1 || h < 1 || w < 1 || c < 1) return set_error(IVX_EINVAL, "bad up2_grad arguments");
    k_up2_grad<<<nblocks((int64_t)n * h * w * c), NT, 0, (hipStream_t)stream>>>(dy, n, h, w, c, dx);
    UHIP(hipGetLastError());
    return IVX_OK;
}

} // extern "C"
