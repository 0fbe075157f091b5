// Exclusive scan of n uint32 counts in two launches over many workgroups, in
// a fixed order (no atomics), for the offset tables of the partition and list
// passes:
//   seg_reduce_kernel: workgroup g sums the values [g S, min(n, (g+1) S)) into
//                      partial[g];
//   seg_scan_kernel:   workgroup g adds partial[0 .. g) and scans its segment.
// out[i] = sum of in[0 .. i), out[n] = the total; out2 (optional) receives the
// same prefixes, total64 (optional) the total as int64, and a total above cap
// sets ST_CAPACITY in status.
#pragma once

#include "hf_internal.h"

namespace {

constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_MAX_GROUPS = 256;

struct ScanJob {
    const uint32_t *in;
    int64_t n;
    int64_t seg;          // values per workgroup
    uint64_t *partial;    // [SCAN_MAX_GROUPS]
    uint32_t *out;        // [n + 1]
    uint32_t *out2;       // [n] or null
    int64_t *total64;     // or null
    int64_t cap;          // capacity checked against the total (when total64 is set)
    uint32_t *status;
};

inline ScanJob scan_job(const uint32_t *in, int64_t n, uint64_t *partial, uint32_t *out, uint32_t *out2 = nullptr,
                        int64_t *total64 = nullptr, int64_t cap = 0, uint32_t *status = nullptr) {
    int64_t groups = (n + SCAN_THREADS - 1) / SCAN_THREADS;
    if (groups < 1) groups = 1;
    if (groups > SCAN_MAX_GROUPS) groups = SCAN_MAX_GROUPS;
    const int64_t seg = (n + groups - 1) / groups;
    return ScanJob{in, n, seg < 1 ? 1 : seg, partial, out, out2, total64, cap, status};
}

inline unsigned scan_groups(const ScanJob &j) {
    const int64_t g = (j.n + j.seg - 1) / j.seg;
    return unsigned(g > 0 ? g : 1);
}

constexpr int SCAN_TILES = 0, SCAN_MAXIMA = 1;  // TAG values of the two uses

// Workgroup sum of one value per thread (SCAN_THREADS threads).
__device__ __forceinline__ uint64_t scan_block_sum(uint64_t v, uint64_t *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    uint64_t t = 0;
    for (int w = 0; w < SCAN_THREADS / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

// TAG only tells the uses apart in profiles.
template <int TAG>
__global__ void __launch_bounds__(SCAN_THREADS) seg_reduce_kernel(ScanJob j) {
    __shared__ uint64_t red[SCAN_THREADS / 64];
    const int64_t lo = int64_t(blockIdx.x) * j.seg;
    const int64_t hi = lo + j.seg < j.n ? lo + j.seg : j.n;
    uint64_t s = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += SCAN_THREADS) s += j.in[i];
    const uint64_t t = scan_block_sum(s, red);
    if (threadIdx.x == 0) j.partial[blockIdx.x] = t;
}

template <int TAG>
__global__ void __launch_bounds__(SCAN_THREADS) seg_scan_kernel(ScanJob j) {
    __shared__ uint64_t red[SCAN_THREADS / 64];
    __shared__ uint32_t wsum[SCAN_THREADS / 64];
    const int g = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t carry = scan_block_sum(threadIdx.x < unsigned(g) ? j.partial[threadIdx.x] : 0ull, red);
    const int64_t lo = int64_t(g) * j.seg;
    const int64_t hi = lo + j.seg < j.n ? lo + j.seg : j.n;
    for (int64_t base = lo; base < hi; base += SCAN_THREADS) {
        const int64_t i = base + threadIdx.x;
        const uint32_t v = i < hi ? j.in[i] : 0u;
        uint32_t inc = v;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(inc, off, 64);
            if (lane >= off) inc += y;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        uint32_t before = 0, tile = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) {
            const uint32_t x = wsum[w];
            before += w < wave ? x : 0u;
            tile += x;
        }
        __syncthreads();
        if (i < hi) {
            const uint32_t e = uint32_t(carry) + before + inc - v;
            j.out[i] = e;
            if (j.out2) j.out2[i] = e;
        }
        carry += tile;
    }
    if (g == int(gridDim.x) - 1 && threadIdx.x == 0) {
        j.out[j.n] = uint32_t(carry);
        if (j.total64) {
            *j.total64 = int64_t(carry);
            if (int64_t(carry) > j.cap) atomicOr(j.status, hf::ST_CAPACITY);
        }
    }
}

}  // namespace
