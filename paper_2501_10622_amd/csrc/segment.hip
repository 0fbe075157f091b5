// Step 4 (local maxima of the grid CWT) and step 5 (segmentation of the grid
// by its maxima, Sec. 2.3) on the FP32 CWT field.
//
// Order on cells: (value, linear index), larger value first, equal values by
// larger index, -0 equal to +0.  It is encoded as a 64-bit key whose integer
// order is that order: high word = order-preserving bits of the float, low
// word = index.
#include "hf_internal.h"

using namespace hf;

namespace {

constexpr int MAX_BLOCK = 256;
constexpr int MAX_PER_THREAD = 16;
constexpr int MAX_CHUNK = MAX_BLOCK * MAX_PER_THREAD;  // cells per maxima workgroup

__device__ __forceinline__ uint64_t cell_key(float c, uint32_t idx, bool &nan) {
    uint32_t u = __float_as_uint(c);
    if ((u & 0x7fffffffu) > 0x7f800000u) nan = true;
    if (u == 0x80000000u) u = 0u;  // -0 -> +0
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return (uint64_t(u) << 32) | idx;
}

__device__ __forceinline__ uint32_t wrap(int v, int n) { return uint32_t(v < 0 ? v + n : (v >= n ? v - n : v)); }

// Largest key among the 26 neighbours of (x, y, z).
__device__ __forceinline__ uint64_t neighbour_max(const float *__restrict__ c, int n, int x, int y, int z,
                                                  bool &nan) {
    uint64_t best = 0;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
        const uint32_t zz = wrap(z + dz, n);
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const uint32_t yy = wrap(y + dy, n);
            const uint32_t row = (zz * uint32_t(n) + yy) * uint32_t(n);
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (dz == 0 && dy == 0 && dx == 0) continue;
                const uint32_t j = row + wrap(x + dx, n);
                const uint64_t k = cell_key(c[j], j, nan);
                best = k > best ? k : best;
            }
        }
    }
    return best;
}

// Pass 1: is-maximum bit mask (one 64-bit word per 64 consecutive cells) and
// the number of maxima in each workgroup's chunk of MAX_CHUNK cells.
__global__ void __launch_bounds__(MAX_BLOCK) maxima_mark_kernel(const float *__restrict__ c, int n, float tau,
                                                                unsigned long long *__restrict__ mask,
                                                                uint32_t *__restrict__ counts, uint32_t *status) {
    const uint32_t cells = uint32_t(n) * n * n;
    const uint32_t base = blockIdx.x * MAX_CHUNK;
    bool nan = false;
    uint32_t cnt = 0;
#pragma unroll 1
    for (int i = 0; i < MAX_PER_THREAD; ++i) {
        const uint32_t j = base + i * MAX_BLOCK + threadIdx.x;
        bool is_max = false;
        if (j < cells) {
            const int x = int(j % uint32_t(n)), y = int((j / uint32_t(n)) % uint32_t(n)), z = int(j / (uint32_t(n) * n));
            const float v = c[j];
            const uint64_t me = cell_key(v, j, nan);
            is_max = (v > tau) && me > neighbour_max(c, n, x, y, z, nan);
        }
        const unsigned long long bits = __ballot(is_max);
        if ((threadIdx.x & 63) == 0 && base + i * MAX_BLOCK + threadIdx.x < cells) mask[(j >> 6)] = bits;
        cnt += __popcll(bits);
    }
    __shared__ uint32_t red[MAX_BLOCK / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < MAX_BLOCK / 64; ++w) t += red[w];
        counts[blockIdx.x] = t;
    }
    if (nan) atomicOr(status, ST_INPUT);
}

// Pass 2: exclusive scan of the chunk counts (one workgroup, fixed order).
__global__ void __launch_bounds__(1024) maxima_scan_kernel(const uint32_t *__restrict__ counts, int nchunks,
                                                           uint32_t *__restrict__ offsets, int64_t cap,
                                                           int64_t *d_count, uint32_t *status) {
    __shared__ uint64_t part[1024];
    const int t = threadIdx.x;
    const int per = (nchunks + 1023) / 1024;
    const int lo = t * per, hi = min(nchunks, lo + per);
    uint64_t s = 0;
    for (int i = lo; i < hi; ++i) s += counts[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint64_t run = t > 0 ? part[t - 1] : 0;
    for (int i = lo; i < hi; ++i) {
        offsets[i] = uint32_t(run);
        run += counts[i];
    }
    if (t == 1023) {
        const uint64_t total = part[1023];
        *d_count = int64_t(total);
        if (int64_t(total) > cap) atomicOr(status, ST_CAPACITY);
    }
}

// Pass 3: write each chunk's maxima at its offset, in index order.
__global__ void __launch_bounds__(MAX_BLOCK) maxima_write_kernel(int n, const unsigned long long *__restrict__ mask,
                                                                 const uint32_t *__restrict__ offsets, int64_t cap,
                                                                 int32_t *__restrict__ out) {
    const uint32_t cells = uint32_t(n) * n * n;
    const uint32_t base = blockIdx.x * MAX_CHUNK;
    const uint32_t words = (min(cells - base, uint32_t(MAX_CHUNK)) + 63) / 64;
    __shared__ uint32_t pre[MAX_CHUNK / 64 + 1];
    if (threadIdx.x == 0) {
        uint32_t r = 0;
        for (uint32_t w = 0; w < words; ++w) {
            pre[w] = r;
            r += __popcll(mask[(base >> 6) + w]);
        }
    }
    __syncthreads();
    const uint32_t off0 = offsets[blockIdx.x];
    for (uint32_t w = threadIdx.x; w < words; w += blockDim.x) {
        unsigned long long bits = mask[(base >> 6) + w];
        uint32_t r = off0 + pre[w];
        while (bits) {
            const int b = __ffsll(bits) - 1;
            bits &= bits - 1;
            if (int64_t(r) < cap) out[r] = int32_t(base + w * 64 + b);
            ++r;
        }
    }
}

// Segmentation pass 1: parent = largest of self and the 26 neighbours.
__global__ void __launch_bounds__(256) parent_kernel(const float *__restrict__ c, int n,
                                                     int32_t *__restrict__ parent, uint32_t *status) {
    const uint32_t cells = uint32_t(n) * n * n;
    bool nan = false;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < cells; j += gridDim.x * blockDim.x) {
        const int x = int(j % uint32_t(n)), y = int((j / uint32_t(n)) % uint32_t(n)), z = int(j / (uint32_t(n) * n));
        const uint64_t me = cell_key(c[j], j, nan);
        const uint64_t nb = neighbour_max(c, n, x, y, z, nan);
        parent[j] = int32_t(uint32_t((nb > me ? nb : me) & 0xffffffffu));
    }
    if (nan) atomicOr(status, ST_INPUT);
}

__global__ void fill_flags_kernel(uint32_t *flags, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) flags[i] = (i == 0) ? 1u : 0u;
}

// One pointer-jumping round, in place: p <- p[p].  Round r runs only if round
// r-1 changed something (flags[r] set), so a fixed number of launches suffices.
__global__ void __launch_bounds__(256) jump_kernel(int32_t *__restrict__ ptr, uint32_t cells, uint32_t *flags,
                                                   int round) {
    if (flags[round] == 0u) return;
    bool changed = false;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < cells; j += gridDim.x * blockDim.x) {
        const int32_t p = ptr[j];
        const int32_t pp = ptr[p];
        if (pp != p) {
            ptr[j] = pp;
            changed = true;
        }
    }
    if (__any(changed) && (threadIdx.x & 63) == 0) flags[round + 1] = 1u;
}

__global__ void __launch_bounds__(256) finalize_kernel(int32_t *__restrict__ ptr, const float *__restrict__ c,
                                                       uint32_t cells, float tau) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < cells; j += gridDim.x * blockDim.x) {
        const int32_t r = ptr[j];
        ptr[j] = c[r] > tau ? r : -1;
    }
}

int rounds_for(uint32_t cells) {
    int k = 0;
    while ((uint64_t(1) << k) < cells) ++k;
    return k + 1;  // ceil(log2(longest path)) rounds, plus one that sees no change
}

struct MaximaLayout {
    size_t mask, counts, offsets, total;
    int nchunks;
};

MaximaLayout maxima_layout(int n) {
    MaximaLayout L{};
    const size_t cells = size_t(n) * n * n;
    L.nchunks = int((cells + MAX_CHUNK - 1) / MAX_CHUNK);
    size_t off = 0;
    L.mask = off;
    off = align_up(off + sizeof(unsigned long long) * ((cells + 63) / 64 + MAX_CHUNK / 64));
    L.counts = off;
    off = align_up(off + sizeof(uint32_t) * L.nchunks);
    L.offsets = off;
    off = align_up(off + sizeof(uint32_t) * L.nchunks);
    L.total = off;
    return L;
}

int stride_grid(uint32_t cells) {
    uint32_t g = (cells + 255) / 256;
    return int(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

}  // namespace

size_t hf::maxima_ws_bytes(const hf_box &box) { return maxima_layout(box.n).total; }

size_t hf::segment_ws_bytes(const hf_box &box) {
    const uint32_t cells = uint32_t(box.n) * box.n * box.n;
    return align_up(sizeof(uint32_t) * (rounds_for(cells) + 2));
}

extern "C" hf_status hf_maxima(hf_ctx *ctx, const hf_box *box, const float *cwt, float tau, int32_t *max_idx,
                               int64_t max_cap, int64_t *d_count, void *ws, size_t ws_bytes) {
    if (!ctx || !cwt || !d_count || max_cap < 0 || (max_cap > 0 && !max_idx)) return HF_ERR_ARG;
    if (tau != tau) return HF_ERR_ARG;
    hf_status s = check_box(box);
    if (s != HF_OK) return s;
    const MaximaLayout L = maxima_layout(box->n);
    s = check_ws(ws, ws_bytes, L.total);
    if (s != HF_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    char *w8 = static_cast<char *>(ws);
    auto *mask = reinterpret_cast<unsigned long long *>(w8 + L.mask);
    auto *counts = reinterpret_cast<uint32_t *>(w8 + L.counts);
    auto *offsets = reinterpret_cast<uint32_t *>(w8 + L.offsets);
    hipLaunchKernelGGL(maxima_mark_kernel, dim3(L.nchunks), dim3(MAX_BLOCK), 0, ctx->stream, cwt, box->n, tau, mask,
                       counts, ctx->d_status);
    hipLaunchKernelGGL(maxima_scan_kernel, dim3(1), dim3(1024), 0, ctx->stream, counts, L.nchunks, offsets, max_cap,
                       d_count, ctx->d_status);
    hipLaunchKernelGGL(maxima_write_kernel, dim3(L.nchunks), dim3(MAX_BLOCK), 0, ctx->stream, box->n, mask, offsets,
                       max_cap, max_idx);
    return launch_status();
}

extern "C" hf_status hf_segment(hf_ctx *ctx, const hf_box *box, const float *cwt, float tau, int32_t *cell_label,
                                void *ws, size_t ws_bytes) {
    if (!ctx || !cwt || !cell_label) return HF_ERR_ARG;
    if (tau != tau) return HF_ERR_ARG;
    hf_status s = check_box(box);
    if (s != HF_OK) return s;
    s = check_ws(ws, ws_bytes, segment_ws_bytes(*box));
    if (s != HF_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    const uint32_t cells = uint32_t(box->n) * box->n * box->n;
    const int rounds = rounds_for(cells);
    auto *flags = static_cast<uint32_t *>(ws);
    const int g = stride_grid(cells);
    hipLaunchKernelGGL(fill_flags_kernel, dim3((rounds + 2 + 255) / 256), dim3(256), 0, ctx->stream, flags,
                       rounds + 2);
    hipLaunchKernelGGL(parent_kernel, dim3(g), dim3(256), 0, ctx->stream, cwt, box->n, cell_label, ctx->d_status);
    for (int r = 0; r < rounds; ++r)
        hipLaunchKernelGGL(jump_kernel, dim3(g), dim3(256), 0, ctx->stream, cell_label, cells, flags, r);
    hipLaunchKernelGGL(finalize_kernel, dim3(g), dim3(256), 0, ctx->stream, cell_label, cwt, cells, tau);
    return launch_status();
}
