// Group statistics and filters of one scale (Sec. 2, steps 5 and 7, with
// Table 1's dens_th and particle_th): the grid volume (cells) and particle
// number of every segmented group, the density and size test, and the labels
// of disposed groups set to -1.
#include "hf_internal.h"

using namespace hf;

namespace {

constexpr int GB = 256;  // threads per workgroup
constexpr int GPER = 4;  // elements per thread per sweep in the streaming passes

// The per-group counters are two n^3 uint32 arrays of the workspace indexed by
// the root's linear cell index, so a label addresses its group's counters
// directly.  Only the entries of the listed roots are cleared, counted and
// read; after the decision, cells[root] holds the keep flag (1 or 0).
struct GroupCounters {
    uint32_t *parts;
    uint32_t *cells;
};

// Adds one per lane whose label l is >= 0 into ctr[l], with one atomic per
// distinct label of the wavefront: labels of neighbouring cells mostly agree,
// so a wavefront of one grid row usually issues one or two atomics.  Every
// lane of the wavefront must call it (the loop is wavefront-uniform).
__device__ __forceinline__ void wave_count(uint32_t *ctr, int32_t l) {
    bool pending = l >= 0;
    const int lane = int(__lane_id());
    for (;;) {
        const unsigned long long m = __ballot(pending);
        if (m == 0) break;
        const int leader = __ffsll((long long)m) - 1;
        const int32_t ll = __shfl(l, leader, 64);
        const bool mine = pending && l == ll;
        const unsigned long long sm = __ballot(mine);
        if (lane == leader) atomicAdd(ctr + ll, uint32_t(__popcll(sm)));
        pending = pending && !mine;
    }
}

__global__ void __launch_bounds__(GB) groups_clear_kernel(const int32_t *__restrict__ roots, int64_t nroots,
                                                          int64_t ncells, GroupCounters g, uint32_t *status) {
    bool bad = false;
    for (int64_t i = blockIdx.x * int64_t(GB) + threadIdx.x; i < nroots; i += int64_t(gridDim.x) * GB) {
        const int32_t r = roots[i];
        if (r < 0 || r >= ncells) {
            bad = true;
            continue;
        }
        g.parts[r] = 0u;
        g.cells[r] = 0u;
    }
    if (bad) atomicOr(status, ST_INPUT);
}

// Step 5: the grid volume of every group, in cells.  Whole workgroups sweep
// GB * GPER consecutive cells at a time, so every wavefront takes part in
// every wave_count.
__global__ void __launch_bounds__(GB) groups_cells_kernel(const int32_t *__restrict__ cell_label, int64_t ncells,
                                                          uint32_t *__restrict__ cells, uint32_t *status) {
    bool bad = false;
    const int64_t sweep = int64_t(GB) * GPER;
    for (int64_t base = blockIdx.x * sweep; base < ncells; base += int64_t(gridDim.x) * sweep) {
        int32_t l[GPER];
#pragma unroll
        for (int k = 0; k < GPER; ++k) {
            const int64_t i = base + k * GB + threadIdx.x;
            l[k] = i < ncells ? cell_label[i] : -1;
        }
#pragma unroll
        for (int k = 0; k < GPER; ++k) {
            if (l[k] >= ncells || l[k] < -1) {
                bad = true;
                l[k] = -1;
            }
            wave_count(cells, l[k]);
        }
    }
    if (bad) atomicOr(status, ST_INPUT);
}

// Step 6 groups: the particle number of every group.  Particle labels come in
// input order, where neighbouring lanes rarely share a group, so every
// labelled particle adds with its own atomic.
__global__ void __launch_bounds__(GB) groups_particles_kernel(const int32_t *__restrict__ plabel, int64_t np,
                                                              int64_t ncells, uint32_t *__restrict__ parts,
                                                              uint32_t *status) {
    bool bad = false;
    const int64_t stride = int64_t(gridDim.x) * GB;
    for (int64_t i0 = blockIdx.x * int64_t(GB) + threadIdx.x; i0 < np; i0 += stride * GPER) {
        int32_t l[GPER];
#pragma unroll
        for (int k = 0; k < GPER; ++k) {
            const int64_t i = i0 + k * stride;
            l[k] = i < np ? plabel[i] : -1;
        }
#pragma unroll
        for (int k = 0; k < GPER; ++k) {
            if (l[k] >= ncells || l[k] < -1) bad = true;
            else if (l[k] >= 0) atomicAdd(parts + l[k], 1u);
        }
    }
    if (bad) atomicOr(status, ST_INPUT);
}

// Step 7 and Table 1: a group is kept if N_g n^3 >= dens_th V_g N_p (its density
// against dens_th times the box mean N_p / L^3, with V_g in cells of volume
// (L/n)^3) and N_g >= particle_th.  Decided in FP64 as
// double(N_g) * n^3 >= (dens_th * double(V_g)) * N_p (products only, so no
// contraction changes the rounding).
__global__ void __launch_bounds__(GB) groups_decide_kernel(const int32_t *__restrict__ roots, int64_t nroots,
                                                           int64_t ncells, GroupCounters g, double dens_th,
                                                           double np_total, int64_t particle_th,
                                                           uint32_t *__restrict__ out_parts,
                                                           uint32_t *__restrict__ out_cells,
                                                           uint8_t *__restrict__ out_keep) {
    for (int64_t i = blockIdx.x * int64_t(GB) + threadIdx.x; i < nroots; i += int64_t(gridDim.x) * GB) {
        const int32_t r = roots[i];
        if (r < 0 || r >= ncells) {  // reported by the clear pass
            out_parts[i] = 0u;
            out_cells[i] = 0u;
            out_keep[i] = 0;
            continue;
        }
        const uint32_t p = g.parts[r], c = g.cells[r];
        const double lhs = double(p) * double(ncells);
        const double rhs = (dens_th * double(c)) * np_total;
        const bool keep = int64_t(p) >= particle_th && lhs >= rhs;
        out_parts[i] = p;
        out_cells[i] = c;
        out_keep[i] = keep ? 1 : 0;
        g.cells[r] = keep ? 1u : 0u;
    }
}

// Labels of disposed groups become -1 (in place when out == in).  With no
// groups at all every label becomes -1.
__global__ void __launch_bounds__(GB) groups_filter_kernel(const int32_t *in, int32_t *out, int64_t count,
                                                           int64_t ncells, const uint32_t *__restrict__ keep,
                                                           int any_roots, uint32_t *status) {
    bool bad = false;
    const int64_t stride = int64_t(gridDim.x) * GB;
    for (int64_t i0 = blockIdx.x * int64_t(GB) + threadIdx.x; i0 < count; i0 += stride * GPER) {
        int32_t l[GPER];
#pragma unroll
        for (int k = 0; k < GPER; ++k) {
            const int64_t i = i0 + k * stride;
            l[k] = i < count ? in[i] : -1;
        }
#pragma unroll
        for (int k = 0; k < GPER; ++k) {
            const int64_t i = i0 + k * stride;
            if (i >= count) continue;
            int32_t v = -1;
            if (l[k] >= ncells || l[k] < -1) bad = true;
            else if (l[k] >= 0 && any_roots && keep[l[k]]) v = l[k];
            out[i] = v;
        }
    }
    if (bad) atomicOr(status, ST_INPUT);
}

unsigned grid_of(const hf_ctx *ctx, int64_t work, int64_t per_block) {
    const int64_t want = (work + per_block - 1) / per_block;
    const int64_t cap = int64_t(ctx->cus) * 32;
    return unsigned(want < 1 ? 1 : (want > cap ? cap : want));
}

}  // namespace

size_t hf::groups_ws_bytes(const hf_box &box) {
    const size_t cells = size_t(box.n) * size_t(box.n) * size_t(box.n);
    return 2 * align_up(cells * sizeof(uint32_t));
}

extern "C" hf_status hf_groups(hf_ctx *ctx, const hf_box *box, int64_t np, const int32_t *roots, int64_t nroots,
                               const int32_t *cell_label, const int32_t *particle_label, double dens_th,
                               int64_t particle_th, uint32_t *group_particles, uint32_t *group_cells,
                               uint8_t *group_keep, int32_t *cell_label_out, int32_t *particle_label_out, void *ws,
                               size_t ws_bytes) {
    if (!ctx || !cell_label) return HF_ERR_ARG;
    hf_status s = check_box(box);
    if (s != HF_OK) return s;
    const int64_t ncells = int64_t(box->n) * box->n * box->n;
    if (np < 0 || np > int64_t(UINT32_MAX) || nroots < 0 || nroots > ncells) return HF_ERR_ARG;
    if (!(dens_th >= 0.0) || !(dens_th < 1e300) || particle_th < 0) return HF_ERR_ARG;
    if (np > 0 && !particle_label) return HF_ERR_ARG;
    if (nroots > 0 && (!roots || !group_particles || !group_cells || !group_keep)) return HF_ERR_ARG;
    s = check_ws(ws, ws_bytes, groups_ws_bytes(*box));
    if (s != HF_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    const hipStream_t st = ctx->stream;
    unsigned char *base = static_cast<unsigned char *>(ws);
    GroupCounters g{reinterpret_cast<uint32_t *>(base),
                    reinterpret_cast<uint32_t *>(base + align_up(size_t(ncells) * sizeof(uint32_t)))};
    if (nroots > 0) {
        HF_LAUNCH(ctx, K_GROUP_CLEAR, groups_clear_kernel, dim3(grid_of(ctx, nroots, GB)), dim3(GB), 0, st, roots,
                  nroots, ncells, g, ctx->d_status);
        HF_LAUNCH(ctx, K_GROUP_CELLS, groups_cells_kernel, dim3(grid_of(ctx, ncells, GB * GPER)), dim3(GB), 0, st,
                  cell_label, ncells, g.cells, ctx->d_status);
        if (np > 0)
            HF_LAUNCH(ctx, K_GROUP_PARTICLES, groups_particles_kernel, dim3(grid_of(ctx, np, GB * GPER)), dim3(GB), 0,
                      st, particle_label, np, ncells, g.parts, ctx->d_status);
        HF_LAUNCH(ctx, K_GROUP_DECIDE, groups_decide_kernel, dim3(grid_of(ctx, nroots, GB)), dim3(GB), 0, st, roots,
                  nroots, ncells, g, dens_th, double(np), particle_th, group_particles, group_cells, group_keep);
    }
    const int any = nroots > 0 ? 1 : 0;
    if (cell_label_out)
        HF_LAUNCH(ctx, K_GROUP_FILTER, groups_filter_kernel, dim3(grid_of(ctx, ncells, GB * GPER)), dim3(GB), 0, st,
                  cell_label, cell_label_out, ncells, ncells, g.cells, any, ctx->d_status);
    if (particle_label_out && np > 0)
        HF_LAUNCH(ctx, K_GROUP_FILTER, groups_filter_kernel, dim3(grid_of(ctx, np, GB * GPER)), dim3(GB), 0, st,
                  particle_label, particle_label_out, np, ncells, g.cells, any, ctx->d_status);
    return launch_status();
}
