// Stable least-significant-digit radix sort of 64-bit keys (optionally carrying 32-bit values)
// over bits [0, end_bit), 8 bits per pass.  Used for the plan-time binning of the visibility
// records and for the breakpoints of the bounded solver's Cauchy search.
//
// A tile is `items` rounds of 256 consecutive keys, items chosen per sort (1..RS_ITEMS) so
// that small sorts still spread over ~256 blocks.  Per pass:
//   k_rs_hist     each block counts the digits of its tile into LDS and writes its 256
//                 counts, digit-major (hist[d][block]);
//   k_rs_offsets  one block per digit: exclusive prefix of that digit over the blocks (wave
//                 scans) and the digit's total;
//   k_rs_scatter  each block first turns the 256 totals into the start of every digit (an
//                 exclusive scan in the block), then walks its tile round by round; a key's
//                 rank among the equal digits of its wave comes from eight ballots (one per
//                 digit bit), the waves of the round are ordered through per-wave digit
//                 counts in LDS, and a running count per digit carries the order across
//                 rounds, so equal digits keep their input order (stable).
// No global atomics: every count is written by one block and read after the launch ends.
// The last pass ranks only the bits below end_bit, so keys equal on [0, end_bit) keep their
// order whatever their higher bits hold.
// The passes ping-pong between the output arrays and a scratch copy so that the last pass
// writes the output.
#include "ivx_internal.hpp"

#include <algorithm>

namespace ivx {

namespace {

constexpr int RS_NT = 256;
constexpr int RS_ITEMS = 8;            // most rounds per tile
constexpr int RS_BINS = 256;
constexpr int RS_FILL_BLOCKS = 256;    // blocks a sort aims for before tiles grow

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o);
        if (lane >= o) v += u;
    }
    return v;
}

__global__ __launch_bounds__(RS_NT) void k_rs_hist(const uint64_t *__restrict__ keys, int n, int shift, int dmask,
                                                   int items, int *__restrict__ hist, int nblk) {
    __shared__ int cnt[RS_BINS];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_NT * items;
    // RS_HU keys per thread requested together; past the end a thread reads key 0 and adds 0
    // (with the load or the add behind a branch, each key would wait for its own round trip)
    constexpr int RS_HU = 8;
    for (int r0 = 0; r0 < items; r0 += RS_HU) {
        uint64_t kv[RS_HU];
        bool ok[RS_HU];
#pragma unroll
        for (int u = 0; u < RS_HU; ++u) {
            const int64_t i = base + (int64_t)(r0 + u) * RS_NT + threadIdx.x;
            ok[u] = r0 + u < items && i < n;
            kv[u] = keys[ok[u] ? i : 0];
        }
#pragma unroll
        for (int u = 0; u < RS_HU; ++u) atomicAdd(&cnt[(int)(kv[u] >> shift) & dmask], ok[u] ? 1 : 0);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// block d: hist[d][*] -> exclusive prefix over blocks; total[d] = keys with digit d
__global__ __launch_bounds__(RS_NT) void k_rs_offsets(int *__restrict__ hist, int nblk, int *__restrict__ total) {
    __shared__ int wsum[RS_NT / 64];
    __shared__ int carry;
    const int d = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    int *h = hist + (int64_t)d * nblk;
    for (int b0 = 0; b0 < nblk; b0 += RS_NT) {
        const int b = b0 + tid;
        const int v = b < nblk ? h[b] : 0;
        const int inc = wave_incl_scan(v, lane);
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        int before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (b < nblk) h[b] = before + inc - v;
        __syncthreads();
        if (tid == RS_NT - 1) carry = before + inc;
        __syncthreads();
    }
    if (tid == 0) total[d] = carry;
}

__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                      int n, int shift, int dmask, int items,
                                                      const int *__restrict__ offs, int nblk,
                                                      const int *__restrict__ total, uint64_t *__restrict__ kout,
                                                      uint32_t *__restrict__ vout) {
    __shared__ int run[RS_BINS];         // keys of each digit placed by earlier rounds
    __shared__ int wc[RS_NT / 64][RS_BINS]; // per-wave digit counts of the current round
    __shared__ int wsum[RS_NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    {
        // start of digit tid = keys with a smaller digit (exclusive scan of the totals)
        const int tv = total[tid];
        const int inc = wave_incl_scan(tv, lane);
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        run[tid] = before + inc - tv + offs[(int64_t)tid * nblk + blockIdx.x];
    }
    const int64_t base = (int64_t)blockIdx.x * RS_NT * items;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < items; ++r) {
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
        const int d = (int)(key >> shift) & dmask;
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

int rs_items(int n) {
    const int64_t per = ((int64_t)n + (int64_t)RS_NT * RS_FILL_BLOCKS - 1) / ((int64_t)RS_NT * RS_FILL_BLOCKS);
    return (int)std::min<int64_t>(RS_ITEMS, std::max<int64_t>(1, per));
}

int rs_blocks(int n) {
    const int64_t tile = (int64_t)RS_NT * rs_items(n);
    return (int)std::max<int64_t>(1, ((int64_t)n + tile - 1) / tile);
}

// Block count is not monotone in n (tiles grow past RS_FILL_BLOCKS blocks), but a buffer
// sized for n must serve every shorter sort: bound the block count over all m <= n.
int rs_blocks_bound(int n) {
    const int64_t small = std::min<int64_t>(RS_FILL_BLOCKS, ((int64_t)n + RS_NT - 1) / RS_NT);
    return (int)std::max<int64_t>(rs_blocks(n), std::max<int64_t>(1, small));
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

} // namespace

size_t radix_sort_temp_bytes(int n, bool pairs) {
    const int nblk = rs_blocks_bound(n);
    size_t b = align256((size_t)n * sizeof(uint64_t));
    if (pairs) b += align256((size_t)n * sizeof(uint32_t));
    b += align256((size_t)RS_BINS * nblk * sizeof(int));
    b += align256((size_t)RS_BINS * sizeof(int));
    return b;
}

hipError_t radix_sort(void *temp, size_t temp_bytes, const uint64_t *kin, uint64_t *kout, const uint32_t *vin,
                      uint32_t *vout, int n, int end_bit, hipStream_t st) {
    if (n < 0 || end_bit < 1 || end_bit > 64) return hipErrorInvalidValue;
    const bool pairs = vin != nullptr;
    if (pairs && !vout) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    if (!temp || temp_bytes < radix_sort_temp_bytes(n, pairs)) return hipErrorInvalidValue;
    const int items = rs_items(n), nblk = rs_blocks(n);
    const int hist_blocks = rs_blocks_bound(n);
    char *p = static_cast<char *>(temp);
    uint64_t *ktmp = reinterpret_cast<uint64_t *>(p);
    p += align256((size_t)n * sizeof(uint64_t));
    uint32_t *vtmp = nullptr;
    if (pairs) {
        vtmp = reinterpret_cast<uint32_t *>(p);
        p += align256((size_t)n * sizeof(uint32_t));
    }
    int *hist = reinterpret_cast<int *>(p);
    p += align256((size_t)RS_BINS * hist_blocks * sizeof(int));
    int *total = reinterpret_cast<int *>(p);
    const int passes = (end_bit + 7) / 8;
    // pass q writes to the output when (passes - 1 - q) is even, so that the last one does
    const uint64_t *ks = kin;
    const uint32_t *vs = vin;
    for (int q = 0; q < passes; ++q) {
        const bool to_out = ((passes - 1 - q) & 1) == 0;
        uint64_t *kd = to_out ? kout : ktmp;
        uint32_t *vd = to_out ? vout : vtmp;
        // the last pass ranks only the bits below end_bit
        const int bits = std::min(8, end_bit - 8 * q);
        const int dmask = (1 << bits) - 1;
        k_rs_hist<<<nblk, RS_NT, 0, st>>>(ks, n, 8 * q, dmask, items, hist, nblk);
        k_rs_offsets<<<RS_BINS, RS_NT, 0, st>>>(hist, nblk, total);
        k_rs_scatter<<<nblk, RS_NT, 0, st>>>(ks, pairs ? vs : nullptr, n, 8 * q, dmask, items, hist, nblk, total,
                                             kd, pairs ? vd : nullptr);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        ks = kd;
        vs = vd;
    }
    return hipSuccess;
}

} // namespace ivx
