// Step 2 (Eq. (1)): cloud-in-cell deposit in 64-bit fixed point, and step 6:
// particle labels from the nearest node.
#include "hf_internal.h"

using namespace hf;

namespace {

constexpr int DEP_BLOCK = 256;

__global__ void fill_u64_kernel(unsigned long long *p, size_t count) {
    size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
    size_t stride = size_t(gridDim.x) * blockDim.x;
    for (; i < count; i += stride) p[i] = 0ull;
}

// Adds w to a cell; reports the add that carries the cell past 2^63 - 1.
__device__ __forceinline__ void cell_add(unsigned long long *rho, uint32_t idx, unsigned long long w,
                                         bool &overflow) {
    if (w == 0) return;
    unsigned long long old = atomicAdd(rho + idx, w);
    // every addend is below 2^61, so a sum crossing 2^63 is seen by exactly the
    // add that crosses it
    if (!(old >> 63) && ((old + w) >> 63)) overflow = true;
}

template <typename T>
__global__ void __launch_bounds__(DEP_BLOCK) deposit_atomic_kernel(const T *__restrict__ pos, int64_t np,
                                                                   FixedPoint<T> fp, int n,
                                                                   unsigned long long *rho, uint32_t *status) {
    const int64_t one = int64_t(1) << fp.bits;
    bool overflow = false, bad = false;
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < np; i += stride) {
        uint32_t qx, qy, qz;
        bool ok = fp.q(pos[3 * i + 0], qx);
        ok = fp.q(pos[3 * i + 1], qy) && ok;
        ok = fp.q(pos[3 * i + 2], qz) && ok;
        if (!ok) {
            bad = true;
            continue;
        }
        const uint32_t cx = qx >> fp.bits, cy = qy >> fp.bits, cz = qz >> fp.bits;
        const uint64_t fx = uint64_t(qx) & uint64_t(one - 1), fy = uint64_t(qy) & uint64_t(one - 1),
                       fz = uint64_t(qz) & uint64_t(one - 1);
        const uint64_t wx[2] = {uint64_t(one) - fx, fx};
        const uint64_t wy[2] = {uint64_t(one) - fy, fy};
        const uint64_t wz[2] = {uint64_t(one) - fz, fz};
        const uint32_t xs[2] = {cx, cx + 1 == uint32_t(n) ? 0u : cx + 1};
        const uint32_t ys[2] = {cy, cy + 1 == uint32_t(n) ? 0u : cy + 1};
        const uint32_t zs[2] = {cz, cz + 1 == uint32_t(n) ? 0u : cz + 1};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const uint64_t wzy = wz[a] * wy[b];
                const uint32_t row = (zs[a] * uint32_t(n) + ys[b]) * uint32_t(n);
                cell_add(rho, row + xs[0], wzy * wx[0], overflow);
                cell_add(rho, row + xs[1], wzy * wx[1], overflow);
            }
    }
    if (overflow) atomicOr(status, ST_OVERFLOW);
    if (bad) atomicOr(status, ST_INPUT);
}

template <typename T>
__global__ void __launch_bounds__(DEP_BLOCK) label_kernel(const T *__restrict__ pos, int64_t np, FixedPoint<T> fp,
                                                          int n, const int32_t *__restrict__ cell_label,
                                                          int32_t *__restrict__ out, uint32_t *status) {
    const uint32_t half = 1u << (fp.bits - 1);
    bool bad = false;
    constexpr int B = 4;  // particles per thread whose loads are issued together
    const int64_t step = int64_t(gridDim.x) * blockDim.x * B;
    for (int64_t i0 = blockIdx.x * int64_t(blockDim.x) * B + threadIdx.x; i0 < np; i0 += step) {
        T px[B], py[B], pz[B];
        int32_t lab[B];
        uint32_t cell[B];
        bool ok[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int64_t i = i0 + k * int64_t(blockDim.x);
            if (i < np) {
                px[k] = pos[3 * i + 0];
                py[k] = pos[3 * i + 1];
                pz[k] = pos[3 * i + 2];
            }
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int64_t i = i0 + k * int64_t(blockDim.x);
            uint32_t qx = 0, qy = 0, qz = 0;
            ok[k] = false;
            if (i < np) {
                ok[k] = fp.q(px[k], qx);
                ok[k] = fp.q(py[k], qy) && ok[k];
                ok[k] = fp.q(pz[k], qz) && ok[k];
                bad |= !ok[k];
            }
            uint32_t x = (qx + half) >> fp.bits, y = (qy + half) >> fp.bits, z = (qz + half) >> fp.bits;
            if (x == uint32_t(n)) x = 0;
            if (y == uint32_t(n)) y = 0;
            if (z == uint32_t(n)) z = 0;
            cell[k] = (z * uint32_t(n) + y) * uint32_t(n) + x;
        }
#pragma unroll
        for (int k = 0; k < B; ++k) lab[k] = ok[k] ? cell_label[cell[k]] : -1;
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int64_t i = i0 + k * int64_t(blockDim.x);
            if (i < np) out[i] = lab[k];
        }
    }
    if (bad) atomicOr(status, ST_INPUT);
}

int grid_for(int64_t work, int block, int cap) {
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return int(g);
}

}  // namespace

size_t hf::deposit_ws_bytes(const hf_box &box, int64_t np) {
    return deposit_tiled_supported(box, np) ? deposit_tiled_ws_bytes(box, np) : 0;
}

extern "C" hf_status hf_deposit(hf_ctx *ctx, const hf_box *box, const void *pos, hf_dtype dtype, int64_t np,
                                int64_t *rho, void *ws, size_t ws_bytes) {
    if (!ctx || !rho || np < 0 || (np > 0 && !pos)) return HF_ERR_ARG;
    if (dtype != HF_F32 && dtype != HF_F64) return HF_ERR_ARG;
    hf_status s = check_box_grid(box);
    if (s != HF_OK) return s;
    s = check_ws(ws, ws_bytes, deposit_ws_bytes(*box, np));
    if (s != HF_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    if (deposit_tiled_supported(*box, np)) return deposit_tiled(ctx, *box, pos, dtype, np, rho, ws);
    // direct form for grids the binned path does not cover: zero, then global atomics
    const size_t cells = size_t(box->n) * box->n * box->n;
    auto *grid = reinterpret_cast<unsigned long long *>(rho);
    HF_LAUNCH(ctx, K_ZERO_GRID, fill_u64_kernel, dim3(grid_for(int64_t(cells), 256, 8192)), dim3(256), 0, ctx->stream, grid,
                       cells);
    if (np > 0) {
        const int g = grid_for(np, DEP_BLOCK, 65536);
        if (dtype == HF_F32)
            HF_LAUNCH(ctx, K_DEP_ATOMIC, deposit_atomic_kernel<float>, dim3(g), dim3(DEP_BLOCK), 0, ctx->stream,
                               static_cast<const float *>(pos), np, make_fixed_point<float>(*box), box->n, grid,
                               ctx->d_status);
        else
            HF_LAUNCH(ctx, K_DEP_ATOMIC, deposit_atomic_kernel<double>, dim3(g), dim3(DEP_BLOCK), 0, ctx->stream,
                               static_cast<const double *>(pos), np, make_fixed_point<double>(*box), box->n, grid,
                               ctx->d_status);
    }
    return launch_status();
}

extern "C" hf_status hf_label(hf_ctx *ctx, const hf_box *box, const void *pos, hf_dtype dtype, int64_t np,
                              const int32_t *cell_label, int32_t *particle_label) {
    if (!ctx || !cell_label || np < 0 || (np > 0 && (!pos || !particle_label))) return HF_ERR_ARG;
    if (dtype != HF_F32 && dtype != HF_F64) return HF_ERR_ARG;
    hf_status s = check_box_grid(box);
    if (s != HF_OK) return s;
    if (np == 0) return HF_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    const int g = grid_for((np + 3) / 4, DEP_BLOCK, 65536);
    if (dtype == HF_F32)
        HF_LAUNCH(ctx, K_LABEL, label_kernel<float>, dim3(g), dim3(DEP_BLOCK), 0, ctx->stream,
                           static_cast<const float *>(pos), np, make_fixed_point<float>(*box), box->n, cell_label,
                           particle_label, ctx->d_status);
    else
        HF_LAUNCH(ctx, K_LABEL, label_kernel<double>, dim3(g), dim3(DEP_BLOCK), 0, ctx->stream,
                           static_cast<const double *>(pos), np, make_fixed_point<double>(*box), box->n, cell_label,
                           particle_label, ctx->d_status);
    return launch_status();
}
