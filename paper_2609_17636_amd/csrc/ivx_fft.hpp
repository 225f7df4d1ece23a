// Device helpers shared by the kernel sources: complex arithmetic, the in-LDS Stockham FFT
// with its twiddle staging, the column-pass helpers and the bilinear sample of the sky.
#pragma once

#include "ivx_internal.hpp"

#include <math.h>

namespace ivx {

constexpr int NT = 256; // threads per block of every kernel

__device__ __forceinline__ cpx cmul(cpx a, cpx b) {
    return cpx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cpx cadd(cpx a, cpx b) { return cpx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cpx csub(cpx a, cpx b) { return cpx{a.re - b.re, a.im - b.im}; }

// ------------------------------------------------------------------------------ FFT
// In-LDS Stockham autosort FFT (mixed radix 2 then 4) of CB interleaved transforms of
// length N = 2^LOGN: element i of transform c is buf[i * CB + c].  Each stage reads all
// of a thread's butterfly inputs into registers, synchronises, then writes the outputs,
// so the transform runs in place.  Twiddles come from a table tw[t] = exp(-2 pi i t / N),
// t < 3N/4, staged in LDS through TwStage (conjugated for the inverse); no scaling is
// applied in either direction.
template <int LOGN> constexpr int tw_len() { return 3 * (1 << LOGN) / 4; }

// The twiddle table is fetched into registers at the start of a kernel and stored to LDS
// only after the kernel's own data loads have been issued, so the two global-memory
// latencies overlap instead of following each other.
template <int LOGN> struct TwStage {
    static constexpr int PER = (tw_len<LOGN>() + NT - 1) / NT;
    cpx v[PER];
    __device__ __forceinline__ void fetch(const cpx *__restrict__ tw) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * NT;
            if (i < tw_len<LOGN>()) v[u] = tw[i];
        }
    }
    __device__ __forceinline__ void store(cpx *tws) const {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * NT;
            if (i < tw_len<LOGN>()) tws[i] = v[u];
        }
    }
};

template <int LOGN, int CB, bool INV>
__device__ __forceinline__ void fft_lds(cpx *buf, const cpx *tw) {
    constexpr int N = 1 << LOGN;
    const int tid = threadIdx.x;
    int Ns = 1;
    if constexpr (LOGN & 1) {
        constexpr int TOT = CB * (N / 2);
        constexpr int BPT = (TOT + NT - 1) / NT;
        cpx v0[BPT], v1[BPT];
#pragma unroll
        for (int t = 0; t < BPT; ++t) {
            const int u = tid + t * NT;
            if (u < TOT) {
                const int c = u % CB, jj = u / CB;
                v0[t] = buf[jj * CB + c];
                v1[t] = buf[(jj + N / 2) * CB + c];
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < BPT; ++t) {
            const int u = tid + t * NT;
            if (u < TOT) {
                const int c = u % CB, jj = u / CB;
                buf[(2 * jj) * CB + c] = cadd(v0[t], v1[t]);
                buf[(2 * jj + 1) * CB + c] = csub(v0[t], v1[t]);
            }
        }
        __syncthreads();
        Ns = 2;
    }
#pragma unroll
    for (int s = 0; s < LOGN / 2; ++s) {
        constexpr int TOT = CB * (N / 4);
        constexpr int BPT = (TOT + NT - 1) / NT;
        cpx v[BPT][4];
        const int st = N / (4 * Ns);
#pragma unroll
        for (int t = 0; t < BPT; ++t) {
            const int u = tid + t * NT;
            if (u < TOT) {
                const int c = u % CB, jj = u / CB;
                const int k = jj & (Ns - 1);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    cpx x = buf[(jj + r * (N / 4)) * CB + c];
                    if (r > 0) {
                        cpx w = tw[k * r * st];
                        if (INV) w.im = -w.im;
                        x = cmul(x, w);
                    }
                    v[t][r] = x;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < BPT; ++t) {
            const int u = tid + t * NT;
            if (u < TOT) {
                const int c = u % CB, jj = u / CB;
                const int k = jj & (Ns - 1);
                const cpx a0 = v[t][0], a1 = v[t][1], a2 = v[t][2], a3 = v[t][3];
                const cpx s02 = cadd(a0, a2), d02 = csub(a0, a2);
                const cpx s13 = cadd(a1, a3), d13 = csub(a1, a3);
                // forward: y1 = d02 - i d13, y3 = d02 + i d13; inverse swaps the signs
                const cpx id13 = INV ? cpx{-d13.im, d13.re} : cpx{d13.im, -d13.re};
                const int o = ((jj - k) << 2) + k;
                buf[o * CB + c] = cadd(s02, s13);
                buf[(o + Ns) * CB + c] = cadd(d02, id13);
                buf[(o + 2 * Ns) * CB + c] = csub(s02, s13);
                buf[(o + 3 * Ns) * CB + c] = csub(d02, id13);
            }
        }
        __syncthreads();
        Ns *= 4;
    }
}

// Global loads each thread of a column pass issues before it waits for the first: with a few
// blocks of LDS-resident columns per compute unit, one load at a time leaves the latency of
// every row exposed.
constexpr int COL_LOADS = 8;

// Columns per block of a column pass: at most 32 KB of LDS columns, so that four blocks share
// a compute unit (at 1024-point columns 4 per block measured faster than 8 and 2).
// Work index of a column-pass block.  Blocks are dealt to the eight XCDs round-robin by
// launch index; block b takes work index (b % 8) * per + b / 8 of the (item, column group)
// pairs, so each XCD runs one contiguous range of them and neighbouring column groups, which
// share the cache lines of their row segments, meet in the same L2.  The launch has
// 8 * per blocks; false for the padding blocks past the last pair.
template <int CB> __device__ __forceinline__ bool col_block(const Geom &g, int &item, int &c0) {
    const int64_t ngrp = (g.rw + CB - 1) / CB, total = ngrp * g.C * g.P, per = (total + 7) / 8;
    const int64_t b = blockIdx.x, w = (b & 7) * per + (b >> 3);
    if (w >= total) return false;
    item = (int)(w / ngrp);
    c0 = (int)(w - (w / ngrp) * ngrp) * CB;
    return true;
}

template <int LOGN> constexpr int col_batch() {
    constexpr int b = 32768 / ((1 << LOGN) * (int)sizeof(cpx));
    return b > 16 ? 16 : (b < 1 ? 1 : b);
}

// --------------------------------------------------------------------- reprojection
// Bilinear sample at (row sy, col sx); pixel (i, j) sits at (i, j); outside pixels are 0.
// Branch-free: a tap outside the image reads a clamped pixel inside it and is scaled by 0, and
// a sample outside (or a NaN coordinate) evaluates at (0, 0) and is scaled by 0, so the loads
// of several samples can be in flight together (behind a branch each would wait for the last).
// Taps: the four pixel offsets (row-major, N^2 < 2^31) and their 0/1 masks; combine() forms
// the sample from the four loaded pixels.
struct BilinearTaps {
    int o[4];
    real m[4];
    real fy, fx, in;
    __device__ __forceinline__ real combine(real p00, real p01, real p10, real p11) const {
        const real x00 = p00 * m[0], x01 = p01 * m[1], x10 = p10 * m[2], x11 = p11 * m[3];
        const real v = (real(1) - fy) * ((real(1) - fx) * x00 + fx * x01) + fy * ((real(1) - fx) * x10 + fx * x11);
        return v * in;
    }
};

__device__ __forceinline__ BilinearTaps bilinear_taps(int N, real sy, real sx) {
    BilinearTaps t;
    const bool in = sy > real(-1) && sy < real(N) && sx > real(-1) && sx < real(N);
    const real cy = in ? sy : real(0), cx = in ? sx : real(0);
    const real fi = floor(cy), fj = floor(cx);
    const int i0 = (int)fi, j0 = (int)fj;
    t.fy = cy - fi;
    t.fx = cx - fj;
    t.in = in ? real(1) : real(0);
    const bool r0 = i0 >= 0, r1 = i0 + 1 < N, c0 = j0 >= 0, c1 = j0 + 1 < N;
    const int ia = (r0 ? i0 : 0) * N, ib = (r1 ? i0 + 1 : N - 1) * N;
    const int ja = c0 ? j0 : 0, jb = c1 ? j0 + 1 : N - 1;
    t.o[0] = ia + ja;
    t.o[1] = ia + jb;
    t.o[2] = ib + ja;
    t.o[3] = ib + jb;
    t.m[0] = (r0 && c0) ? real(1) : real(0);
    t.m[1] = (r0 && c1) ? real(1) : real(0);
    t.m[2] = (r1 && c0) ? real(1) : real(0);
    t.m[3] = (r1 && c1) ? real(1) : real(0);
    return t;
}

__device__ __forceinline__ real bilinear(const real *__restrict__ sky, int N, real sy, real sx) {
    const BilinearTaps t = bilinear_taps(N, sy, sx);
    return t.combine(sky[t.o[0]], sky[t.o[1]], sky[t.o[2]], sky[t.o[3]]);
}

} // namespace ivx
