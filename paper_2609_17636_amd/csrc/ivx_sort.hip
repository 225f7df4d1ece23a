// Stable least-significant-digit radix sort of 64-bit keys (optionally carrying 32-bit values)
// over bits [0, end_bit), 8 bits per pass.  Used for the plan-time binning of the visibility
// records and for the breakpoints of the bounded solver's Cauchy search.
//
// Per pass:
//   k_rs_hist     each block counts the digits of its tile (TILE = 256 threads x RS_ITEMS keys)
//                 into LDS and writes its 256 counts, digit-major (hist[d][block]); the digit
//                 totals are added into a 256-entry array (integer atomics: the sums do not
//                 depend on their order);
//   k_rs_offsets  one block per digit: exclusive prefix of that digit over the blocks, plus
//                 the number of keys with a smaller digit;
//   k_rs_scatter  each block walks its tile in RS_ITEMS rounds of 256 consecutive keys; a key's
//                 rank among the equal digits of its wave comes from eight ballots (one per
//                 digit bit), the waves of the round are ordered through per-wave digit counts
//                 in LDS, and a running count per digit carries the order across rounds, so
//                 equal digits keep their input order (stable).
// The passes ping-pong between the output arrays and a scratch copy so that the last pass
// writes the output.
#include "ivx_internal.hpp"

#include <algorithm>

namespace ivx {

namespace {

constexpr int RS_NT = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_NT * RS_ITEMS;
constexpr int RS_BINS = 256;

__global__ __launch_bounds__(RS_NT) void k_rs_zero(int *__restrict__ p) { p[threadIdx.x] = 0; }

__global__ __launch_bounds__(RS_NT) void k_rs_hist(const uint64_t *__restrict__ keys, int n, int shift,
                                                   int *__restrict__ hist, int nblk, int *__restrict__ total) {
    __shared__ int cnt[RS_BINS];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int64_t i = base + r * RS_NT + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(int)((keys[i] >> shift) & 0xFF)], 1);
    }
    __syncthreads();
    const int c = cnt[threadIdx.x];
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = c;
    if (c) atomicAdd(&total[threadIdx.x], c);
}

// block d: hist[d][*] -> exclusive prefix over blocks + (keys with a smaller digit)
__global__ __launch_bounds__(RS_NT) void k_rs_offsets(int *__restrict__ hist, int nblk, const int *__restrict__ total) {
    __shared__ int part[RS_NT];
    __shared__ int carry;
    const int d = blockIdx.x;
    if (threadIdx.x == 0) {
        int s = 0;
        for (int e = 0; e < d; ++e) s += total[e];
        carry = s;
    }
    __syncthreads();
    int *h = hist + (int64_t)d * nblk;
    for (int b0 = 0; b0 < nblk; b0 += RS_NT) {
        const int b = b0 + threadIdx.x;
        const int v = b < nblk ? h[b] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        // inclusive Hillis-Steele scan of the chunk
        for (int o = 1; o < RS_NT; o <<= 1) {
            const int add = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        const int c0 = carry;
        if (b < nblk) h[b] = c0 + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == RS_NT - 1) carry = c0 + part[RS_NT - 1];
        __syncthreads();
    }
}

__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                      int n, int shift, const int *__restrict__ offs, int nblk,
                                                      uint64_t *__restrict__ kout, uint32_t *__restrict__ vout) {
    __shared__ int run[RS_BINS];         // keys of each digit placed by earlier rounds
    __shared__ int wc[RS_NT / 64][RS_BINS]; // per-wave digit counts of the current round
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    run[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < RS_ITEMS; ++r) {
        for (int e = tid; e < (RS_NT / 64) * RS_BINS; e += RS_NT) (&wc[0][0])[e] = 0;
        __syncthreads();
        const int64_t i = base + r * RS_NT + tid;
        const bool valid = i < n;
        uint64_t key = 0;
        uint32_t val = 0;
        if (valid) {
            key = kin[i];
            if (vin) val = vin[i];
        }
        const int d = (int)((key >> shift) & 0xFF);
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t ones = __ballot(valid && ((d >> b) & 1));
            same &= ((d >> b) & 1) ? ones : ~ones;
        }
        const int rank = __popcll(same & below);
        if (valid && rank == 0) wc[wave][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            int pos = run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wc[w][d];
            kout[pos] = key;
            if (vin) vout[pos] = val;
        }
        __syncthreads();
        // advance the running counts by this round's digits
        int add = 0;
        for (int w = 0; w < RS_NT / 64; ++w) add += wc[w][tid];
        run[tid] += add;
        __syncthreads();
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

} // namespace

size_t radix_sort_temp_bytes(int n, bool pairs) {
    const int nblk = (n + RS_TILE - 1) / RS_TILE;
    size_t b = align256((size_t)n * sizeof(uint64_t));
    if (pairs) b += align256((size_t)n * sizeof(uint32_t));
    b += align256((size_t)RS_BINS * std::max(nblk, 1) * sizeof(int));
    b += align256(RS_BINS * sizeof(int));
    return b;
}

hipError_t radix_sort(void *temp, size_t temp_bytes, const uint64_t *kin, uint64_t *kout, const uint32_t *vin,
                      uint32_t *vout, int n, int end_bit, hipStream_t st) {
    if (n < 0 || end_bit < 1 || end_bit > 64) return hipErrorInvalidValue;
    const bool pairs = vin != nullptr;
    if (pairs && !vout) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    if (!temp || temp_bytes < radix_sort_temp_bytes(n, pairs)) return hipErrorInvalidValue;
    const int nblk = (n + RS_TILE - 1) / RS_TILE;
    char *p = static_cast<char *>(temp);
    uint64_t *ktmp = reinterpret_cast<uint64_t *>(p);
    p += align256((size_t)n * sizeof(uint64_t));
    uint32_t *vtmp = nullptr;
    if (pairs) {
        vtmp = reinterpret_cast<uint32_t *>(p);
        p += align256((size_t)n * sizeof(uint32_t));
    }
    int *hist = reinterpret_cast<int *>(p);
    p += align256((size_t)RS_BINS * nblk * sizeof(int));
    int *total = reinterpret_cast<int *>(p);
    const int passes = (end_bit + 7) / 8;
    // pass q writes to the output when (passes - 1 - q) is even, so that the last one does
    const uint64_t *ks = kin;
    const uint32_t *vs = vin;
    for (int q = 0; q < passes; ++q) {
        const bool to_out = ((passes - 1 - q) & 1) == 0;
        uint64_t *kd = to_out ? kout : ktmp;
        uint32_t *vd = to_out ? vout : vtmp;
        k_rs_zero<<<1, RS_BINS, 0, st>>>(total);
        k_rs_hist<<<nblk, RS_NT, 0, st>>>(ks, n, 8 * q, hist, nblk, total);
        k_rs_offsets<<<RS_BINS, RS_NT, 0, st>>>(hist, nblk, total);
        k_rs_scatter<<<nblk, RS_NT, 0, st>>>(ks, pairs ? vs : nullptr, n, 8 * q, hist, nblk, kd, pairs ? vd : nullptr);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        ks = kd;
        vs = vd;
    }
    return hipSuccess;
}

} // namespace ivx
