// Group statistics and filters of one scale (Sec. 2, steps 5 and 7, with
// Table 1's dens_th and particle_th): the grid volume (cells) and particle
// number of every segmented group, the density and size test, and the labels
// of disposed groups set to -1.
#include "hf_internal.h"

using namespace hf;

namespace {

constexpr int GB = 256;  // threads per workgroup
constexpr int GPER = 4;  // elements per thread per sweep in the streaming passes

// Number of roots: min(*d_count, cap) when the count is on the device (the
// maxima list of the one-call pipeline), else cap.
__device__ __forceinline__ int64_t root_count(const int64_t *d_count, int64_t cap) {
    if (!d_count) return cap;
    const int64_t c = *d_count;
    return c < cap ? c : cap;
}

__global__ void __launch_bounds__(GB) groups_clear_kernel(const int32_t *__restrict__ roots, const int64_t *d_count,
                                                          int64_t cap, int64_t ncells, GroupCounters g,
                                                          uint32_t *status) {
    const int64_t nroots = root_count(d_count, cap);
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

// Step 5: the grid volume of every group, in cells.  One workgroup counts a
// contiguous range of GCHUNK cells (a few grid rows, a few hundred labels) in
// an LDS table and adds it to the counters once.  With MASKED the same count
// runs over `count` labels of particles in the deposit's tile order (spatially
// coherent, like cells), skipping those whose mask byte is nonzero.
constexpr int GCHUNK = 16384;
constexpr int CELL_HT = 1024;

template <bool MASKED>
__global__ void __launch_bounds__(GB) groups_tally_kernel(const int32_t *__restrict__ label,
                                                          const uint8_t *__restrict__ mask, int64_t count,
                                                          int64_t ncells, uint32_t *__restrict__ cells,
                                                          uint32_t *status) {
    __shared__ int32_t hkey[CELL_HT];
    __shared__ uint32_t hcnt[CELL_HT];
    lds_tally_init<CELL_HT>(hkey, hcnt);
    __syncthreads();
    bool bad = false;
    const int64_t c0 = int64_t(blockIdx.x) * GCHUNK;
    const int64_t c1 = c0 + GCHUNK < count ? c0 + GCHUNK : count;
    for (int64_t base = c0; base < c1; base += int64_t(GB) * GPER) {
        int32_t l[GPER];
#pragma unroll
        for (int k = 0; k < GPER; ++k) {
            const int64_t i = base + k * GB + threadIdx.x;
            l[k] = i < c1 ? label[i] : -1;
            if (MASKED && i < c1 && mask[i]) l[k] = -1;
        }
#pragma unroll
        for (int k = 0; k < GPER; ++k) {
            if (l[k] >= ncells || l[k] < -1) {
                bad = true;
                l[k] = -1;
            }
            lds_tally_wave<CELL_HT>(hkey, hcnt, cells, l[k]);
        }
    }
    __syncthreads();
    lds_tally_flush<CELL_HT>(hkey, hcnt, cells);
    if (bad) atomicOr(status, ST_INPUT);
}

// Step 5 by runs: each thread takes CELL_RUN consecutive cells of a row (one
// vector load per four) and adds each run of equal labels to the LDS table
// once, so a basin a few cells wide costs one insert per run instead of one
// per cell.  With MASKED, the same over particle labels in the deposit's tile
// order, skipping those whose mask byte is nonzero.  Both arrays 16-byte
// aligned.
constexpr int CELL_RUN = 16;
static_assert(CELL_RUN == 16, "one 16-byte load of mask bytes per run of labels");

template <bool MASKED>
__global__ void __launch_bounds__(GB) groups_runs_kernel(const int32_t *__restrict__ cell_label,
                                                         const uint8_t *__restrict__ mask, int64_t count,
                                                         int64_t ncells, uint32_t *__restrict__ cells,
                                                         uint32_t *status) {
    __shared__ int32_t hkey[CELL_HT];
    __shared__ uint32_t hcnt[CELL_HT];
    lds_tally_init<CELL_HT>(hkey, hcnt);
    __syncthreads();
    bool bad = false;
    const int64_t c0 = int64_t(blockIdx.x) * GCHUNK;
    const int64_t c1 = c0 + GCHUNK < count ? c0 + GCHUNK : count;
    for (int64_t b = c0 + int64_t(threadIdx.x) * CELL_RUN; b < c1; b += int64_t(GB) * CELL_RUN) {
        int32_t v[CELL_RUN];
        if (b + CELL_RUN <= c1) {
            const int4 *p = reinterpret_cast<const int4 *>(cell_label + b);
            uint32_t mw[CELL_RUN / 4] = {};  // the CELL_RUN mask bytes, four per word
            if (MASKED) {
                const uint4 m = *reinterpret_cast<const uint4 *>(mask + b);
                mw[0] = m.x;
                mw[1] = m.y;
                mw[2] = m.z;
                mw[3] = m.w;
            }
#pragma unroll
            for (int q = 0; q < CELL_RUN / 4; ++q) {
                const int4 w = p[q];
                v[4 * q] = w.x;
                v[4 * q + 1] = w.y;
                v[4 * q + 2] = w.z;
                v[4 * q + 3] = w.w;
                if (MASKED) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if ((mw[q] >> (8 * e)) & 0xffu) v[4 * q + e] = -1;
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < CELL_RUN; ++q) {
                v[q] = b + q < c1 ? cell_label[b + q] : -1;
                if (MASKED && b + q < c1 && mask[b + q]) v[q] = -1;
            }
        }
        int32_t run = -1;
        uint32_t len = 0;
#pragma unroll
        for (int q = 0; q < CELL_RUN; ++q) {
            int32_t l = v[q];
            if (l >= ncells || l < -1) {
                bad = true;
                l = -1;
            }
            if (l != run) {
                if (run >= 0) lds_tally_add<CELL_HT>(hkey, hcnt, cells, run, len);
                run = l;
                len = 0;
            }
            ++len;
        }
        if (run >= 0) lds_tally_add<CELL_HT>(hkey, hcnt, cells, run, len);
    }
    __syncthreads();
    lds_tally_flush<CELL_HT>(hkey, hcnt, cells);
    if (bad) atomicOr(status, ST_INPUT);
}

// Step 6 groups from labels in input order, where neighbouring lanes rarely
// share a group: every labelled particle adds with its own atomic.  With
// skip, particles whose skip entry is >= 0 (claimed by an earlier scale of the
// identification loop) are not counted.
__global__ void __launch_bounds__(GB) groups_particles_kernel(const int32_t *__restrict__ plabel,
                                                              const int32_t *__restrict__ skip, int64_t np,
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
            if (skip && i < np && skip[i] >= 0) l[k] = -1;
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
__global__ void __launch_bounds__(GB) groups_decide_kernel(const int32_t *__restrict__ roots, const int64_t *d_count,
                                                           int64_t cap, int64_t ncells, GroupCounters g,
                                                           double dens_th, double np_total, int64_t particle_th,
                                                           const uint8_t *__restrict__ root_ok,
                                                           uint32_t *__restrict__ out_parts,
                                                           uint32_t *__restrict__ out_cells,
                                                           uint8_t *__restrict__ out_keep) {
    const int64_t nroots = root_count(d_count, cap);
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
        const bool keep = int64_t(p) >= particle_th && lhs >= rhs && (!root_ok || root_ok[i]);
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

// Step 4's correction of one grid maximum (App. B), in FP64 on the FP32
// field: per axis, with the maximum B and its neighbours A (larger) and C
// (smaller), l1 = A - C and l2 = B - C, the quadratic through them peaks
// l1^2 / (16 l2 - 8 l1) above B and l1 / (2 (2 l2 - l1)) cells towards A.  A
// flat axis (l2 = 0) adds nothing.  The value takes the three corrections in
// the order x, y, z; l1bar and l2bar are the means over the axes (for the
// cube-size term).  Every operation is rounded as written (no contraction).
struct PeakFit {
    double shift[3];  // cells, (x, y, z)
    double value;
    double l1bar, l2bar;
    bool nan;
};

__device__ PeakFit peak_fit(const float *__restrict__ c, uint32_t un, const uint32_t g[3], uint32_t r) {
    PeakFit f;
    const double b = double(c[r]);
    f.nan = b != b;
    f.value = b;
    double l1s[3], l2s[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        uint32_t up[3] = {g[0], g[1], g[2]}, dn[3] = {g[0], g[1], g[2]};
        up[ax] = (g[ax] + 1) % un;
        dn[ax] = (g[ax] + un - 1) % un;
        const double cu = double(c[(up[2] * un + up[1]) * un + up[0]]);
        const double cd = double(c[(dn[2] * un + dn[1]) * un + dn[0]]);
        f.nan |= (cu != cu) || (cd != cd);
        const double a = cu > cd ? cu : cd, low = cu > cd ? cd : cu;
        const double l1 = __dsub_rn(a, low), l2 = __dsub_rn(b, low);
        double corr = 0.0, shift = 0.0;
        if (l2 != 0.0) {
            corr = __ddiv_rn(__dmul_rn(l1, l1), __dsub_rn(__dmul_rn(16.0, l2), __dmul_rn(8.0, l1)));
            shift = __ddiv_rn(l1, __dmul_rn(2.0, __dsub_rn(__dmul_rn(2.0, l2), l1)));
            if (!(cu >= cd)) shift = -shift;
        }
        f.value = __dadd_rn(f.value, corr);
        f.shift[ax] = shift;
        l1s[ax] = l1;
        l2s[ax] = l2;
    }
    f.l1bar = __ddiv_rn(__dadd_rn(__dadd_rn(l1s[0], l1s[1]), l1s[2]), 3.0);
    f.l2bar = __ddiv_rn(__dadd_rn(__dadd_rn(l2s[0], l2s[1]), l2s[2]), 3.0);
    return f;
}

// Step 8: maximum i of one scale (field c_scale on an n2^3 grid) is kept if
// its value, corrected for the grid (step 4, App. B), strictly exceeds the
// adjacent smaller scale's field (n1^3 grid over the same box) at every grid
// point near the same physical position.  The correction is the per-axis
// quadratic top plus App. B's cube-size term with the 3/5 factor removed,
// (5/16)(2 l2bar - l1bar)(1 - (n2/n1)^2), which vanishes on one grid.  "Near"
// is the smaller grid's node nearest the corrected position (half a cell
// rounds up), ((g + shift) n1) / n2 in its cells, and its 26 periodic
// neighbours.  c_smaller null stands for the all-zero grid (the
// identification loop's last scale).  One thread per maximum; a NaN is
// reported.
__global__ void __launch_bounds__(GB) cross_scale_kernel(const int32_t *__restrict__ roots, const int64_t *d_count,
                                                         int64_t cap, int n2, const float *__restrict__ c_scale,
                                                         int n1, const float *__restrict__ c_smaller,
                                                         uint8_t *__restrict__ pass, uint32_t *status) {
    const int64_t nroots = root_count(d_count, cap);
    bool bad = false;
    const uint32_t un = uint32_t(n2), ncells = un * un * un, um = uint32_t(n1);
    const double r = __ddiv_rn(double(n2), double(n1));
    const double shrink = __dsub_rn(1.0, __dmul_rn(r, r));
    for (int64_t i = blockIdx.x * int64_t(GB) + threadIdx.x; i < nroots; i += int64_t(gridDim.x) * GB) {
        const int32_t root = roots[i];
        if (root < 0 || uint32_t(root) >= ncells) {
            bad = true;
            pass[i] = 0;
            continue;
        }
        const uint32_t g[3] = {uint32_t(root) % un, (uint32_t(root) / un) % un, uint32_t(root) / (un * un)};
        const PeakFit f = peak_fit(c_scale, un, g, uint32_t(root));
        bad |= f.nan;
        const double term = __dmul_rn(__dmul_rn(0.3125, __dsub_rn(__dmul_rn(2.0, f.l2bar), f.l1bar)), shrink);
        const double v = __dadd_rn(f.value, term);
        uint32_t node[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const double u = __ddiv_rn(__dmul_rn(__dadd_rn(double(g[ax]), f.shift[ax]), double(n1)), double(n2));
            int64_t k = int64_t(floor(__dadd_rn(u, 0.5))) % int64_t(n1);
            if (k < 0) k += n1;
            node[ax] = uint32_t(k);
        }
        bool above = !f.nan;
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const uint32_t gz = (node[2] + um + dz) % um, gy = (node[1] + um + dy) % um,
                                   gx = (node[0] + um + dx) % um;
                    const float u = c_smaller ? c_smaller[(gz * um + gy) * um + gx] : 0.0f;
                    bad |= u != u;
                    above = above && v > double(u);
                }
        pass[i] = above ? 1 : 0;
    }
    if (bad) atomicOr(status, ST_INPUT);
}

// The identification loop's per-particle bookkeeping: halo_scale[p] is the
// scale that claimed particle p (-1 while none has), halo_root[p] (may be
// null) the root of its group there.
__global__ void __launch_bounds__(GB) claim_init_kernel(int32_t *__restrict__ halo_scale,
                                                        int32_t *__restrict__ halo_root, int64_t np) {
    for (int64_t i = blockIdx.x * int64_t(GB) + threadIdx.x; i < np; i += int64_t(gridDim.x) * GB) {
        halo_scale[i] = -1;
        if (halo_root) halo_root[i] = -1;
    }
}

// One pass per scale after the decision: a particle keeps its label iff no
// earlier scale claimed it and its group is kept (else -1), and a kept
// label claims the particle for this scale (halo_root may be null).
__global__ void __launch_bounds__(GB) claim_filter_kernel(int32_t *__restrict__ label,
                                                          int32_t *__restrict__ halo_scale,
                                                          int32_t *__restrict__ halo_root, int64_t np,
                                                          int64_t ncells, const uint32_t *__restrict__ keep,
                                                          int any_roots, int32_t scale, uint32_t *status) {
    bool bad = false;
    const int64_t stride = int64_t(gridDim.x) * GB;
    for (int64_t i0 = blockIdx.x * int64_t(GB) + threadIdx.x; i0 < np; i0 += stride * GPER) {
        int32_t l[GPER], hs[GPER];
#pragma unroll
        for (int k = 0; k < GPER; ++k) {
            const int64_t i = i0 + k * stride;
            l[k] = i < np ? label[i] : -1;
            hs[k] = i < np ? halo_scale[i] : -1;
        }
#pragma unroll
        for (int k = 0; k < GPER; ++k) {
            const int64_t i = i0 + k * stride;
            if (i >= np) continue;
            int32_t v = -1;
            if (l[k] >= ncells || l[k] < -1) bad = true;
            else if (hs[k] < 0 && l[k] >= 0 && any_roots && keep[l[k]]) v = l[k];
            label[i] = v;
            if (v >= 0) {
                halo_scale[i] = scale;
                if (halo_root) halo_root[i] = v;
            }
        }
    }
    if (bad) atomicOr(status, ST_INPUT);
}

// Step 4's correction of grid maxima (App. B): each maximum's corrected
// position (wrapped into [0, L)) and value, from peak_fit.
__global__ void __launch_bounds__(GB) peaks_kernel(const int32_t *__restrict__ roots, int64_t nroots, int n,
                                                   double dx, double box_len, const float *__restrict__ c,
                                                   double *__restrict__ pos, double *__restrict__ value,
                                                   uint32_t *status) {
    bool bad = false;
    const uint32_t un = uint32_t(n), ncells = un * un * un;
    for (int64_t i = blockIdx.x * int64_t(GB) + threadIdx.x; i < nroots; i += int64_t(gridDim.x) * GB) {
        const int32_t r = roots[i];
        if (r < 0 || uint32_t(r) >= ncells) {
            bad = true;
            continue;
        }
        const uint32_t g[3] = {uint32_t(r) % un, (uint32_t(r) / un) % un, uint32_t(r) / (un * un)};
        const PeakFit f = peak_fit(c, un, g, uint32_t(r));
        bad |= f.nan;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            double p = __dmul_rn(__dadd_rn(double(g[ax]), f.shift[ax]), dx);
            p = fmod(p, box_len);
            if (p < 0.0) p = __dadd_rn(p, box_len);
            pos[3 * i + ax] = p;
        }
        value[i] = f.value;
    }
    if (bad) atomicOr(status, ST_INPUT);
}

// ---------------------------------------------------------------------------
// hf_groups on labels in input order, where neighbouring particles rarely
// share a group.  The particle labels are first partitioned by label >> shift
// into GP_BUCKETS ranges of cell indices (a histogram, a scan and a scatter
// staged in LDS, one run per bucket and workgroup); a chunk of the partitioned
// labels then holds a few thousand distinct roots at most, and is counted in
// an LDS table (lds_tally), each root's count added to its counter once per
// chunk.  The keep flags of the decision go to a bitmap of one bit per cell
// (n^3 / 8 bytes) and a summary of one bit per 512 cells (one line of the
// bitmap; 256 KB at 1024^3, which stays in the L2): the label filters read the
// summary first, and the bitmap only for labels whose 512-cell block holds a
// kept root, so the particles' scattered lookups mostly stay in the cache.
// The counts are exact integer sums, so the order the atomics resolve in
// changes nothing.
// ---------------------------------------------------------------------------
constexpr int GP_BUCKETS = 256;
constexpr int GP_THREADS = 1024;
constexpr int GP_PER = 8;
constexpr int GP_CHUNK = GP_THREADS * GP_PER;  // labels per scatter workgroup
constexpr int GP_HCHUNK = 8 * GP_CHUNK;        // labels per histogram workgroup
constexpr int GP_CCHUNK = 32 * GP_CHUNK;       // partitioned labels per counting workgroup (few flushes per root)
constexpr int GP_HT = 8192;                    // LDS tally slots of the counting pass

struct GroupPart {
    uint32_t *count;   // [GP_BUCKETS + 1]: labels per bucket, then the total at [GP_BUCKETS]
    uint32_t *cursor;  // [GP_BUCKETS]
    int32_t *sorted;   // [np]
    uint32_t *bits;    // keep bitmap, one bit per cell, then its summary
    int64_t words;     // of the bitmap and its summary together
    uint32_t *summary;  // [swords]: one bit per 2^blog cells, set where the block holds a kept root
    int64_t swords;
    int blog;
    int shift;
};

constexpr int GP_BLOCK_LOG = 9;  // fewest cells per summary bit (log 2): 512, one 64-byte line of the bitmap
constexpr int GP_SUMMARY_LOG = 20;  // most summary bits (log 2): 128 KB, to sit in one workgroup's LDS

__device__ __forceinline__ bool gp_label_ok(int32_t l, int64_t ncells, bool &bad) {
    if (l >= ncells || l < -1) {
        bad = true;
        return false;
    }
    return l >= 0;
}

__global__ void __launch_bounds__(512) gp_hist_kernel(const int32_t *__restrict__ label, int64_t np, int64_t ncells,
                                                      int shift, uint32_t *__restrict__ count, uint32_t *status) {
    __shared__ uint32_t h[GP_BUCKETS];
    for (int b = threadIdx.x; b < GP_BUCKETS; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    bool bad = false;
    const int64_t c0 = int64_t(blockIdx.x) * GP_HCHUNK;
    const int64_t c1 = c0 + GP_HCHUNK < np ? c0 + GP_HCHUNK : np;
    for (int64_t i0 = c0 + threadIdx.x; i0 < c1; i0 += int64_t(blockDim.x) * 8) {
        int32_t l[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t i = i0 + int64_t(k) * blockDim.x;
            l[k] = i < c1 ? label[i] : -1;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (gp_label_ok(l[k], ncells, bad)) atomicAdd(&h[uint32_t(l[k]) >> shift], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < GP_BUCKETS; b += blockDim.x)
        if (h[b]) atomicAdd(&count[b], h[b]);
    if (bad) atomicOr(status, ST_INPUT);
}

// cursor = exclusive scan of the bucket counts; count[GP_BUCKETS] = the total.
__global__ void __launch_bounds__(GP_BUCKETS) gp_scan_kernel(uint32_t *__restrict__ count,
                                                             uint32_t *__restrict__ cursor) {
    __shared__ uint32_t tot[GP_BUCKETS / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint32_t x = count[t];
    uint32_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) tot[wave] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < GP_BUCKETS / 64; ++w) {
        before += w < wave ? tot[w] : 0u;
        all += tot[w];
    }
    cursor[t] = before + inc - x;
    if (t == 0) count[GP_BUCKETS] = all;
}

__global__ void __launch_bounds__(GP_THREADS) gp_scatter_kernel(const int32_t *__restrict__ label, int64_t np,
                                                                int64_t ncells, int shift, uint32_t *cursor,
                                                                int32_t *__restrict__ sorted) {
    __shared__ int32_t stage[GP_CHUNK];
    __shared__ uint32_t h[GP_BUCKETS], off[GP_BUCKETS], gbase[GP_BUCKETS], tot[GP_BUCKETS / 64];
    const int t = threadIdx.x;
    if (t < GP_BUCKETS) h[t] = 0u;
    __syncthreads();
    const int64_t c0 = int64_t(blockIdx.x) * GP_CHUNK;
    int32_t l[GP_PER];
    uint32_t rank[GP_PER];
    bool bad = false;  // reported by the histogram pass
#pragma unroll
    for (int k = 0; k < GP_PER; ++k) {
        const int64_t i = c0 + int64_t(k) * GP_THREADS + t;
        l[k] = i < np ? label[i] : -1;
        if (!gp_label_ok(l[k], ncells, bad)) l[k] = -1;
    }
#pragma unroll
    for (int k = 0; k < GP_PER; ++k)
        if (l[k] >= 0) rank[k] = atomicAdd(&h[uint32_t(l[k]) >> shift], 1u);
    __syncthreads();
    if (t < GP_BUCKETS) {  // exclusive scan of the chunk's bucket counts, and the runs' places
        const int lane = t & 63, wave = t >> 6;
        const uint32_t x = h[t];
        uint32_t inc = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (lane == 63) tot[wave] = inc;
        off[t] = inc - x;
        if (x) gbase[t] = atomicAdd(&cursor[t], x);
    }
    __syncthreads();
    if (t < GP_BUCKETS) {
        uint32_t before = 0;
        for (int w = 0; w < (t >> 6); ++w) before += tot[w];
        off[t] += before;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GP_PER; ++k)
        if (l[k] >= 0) stage[off[uint32_t(l[k]) >> shift] + rank[k]] = l[k];
    __syncthreads();
    const uint32_t total = off[GP_BUCKETS - 1] + h[GP_BUCKETS - 1];
    for (uint32_t s = t; s < total; s += GP_THREADS) {
        const int32_t v = stage[s];
        const uint32_t b = uint32_t(v) >> shift;
        sorted[gbase[b] + (s - off[b])] = v;
    }
}

__global__ void __launch_bounds__(GP_THREADS) gp_count_kernel(const int32_t *__restrict__ sorted,
                                                              const uint32_t *__restrict__ count,
                                                              uint32_t *__restrict__ parts) {
    __shared__ int32_t hkey[GP_HT];
    __shared__ uint32_t hcnt[GP_HT];
    const uint32_t total = count[GP_BUCKETS];
    const int64_t c0 = int64_t(blockIdx.x) * GP_CCHUNK;
    if (c0 >= int64_t(total)) return;  // the same for the whole workgroup
    lds_tally_init<GP_HT>(hkey, hcnt);
    __syncthreads();
    const int64_t c1 = c0 + GP_CCHUNK < int64_t(total) ? c0 + GP_CCHUNK : int64_t(total);
    for (int64_t b0 = c0; b0 < c1; b0 += int64_t(GP_THREADS) * 8) {  // the same trip count on every lane
        int32_t l[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t i = b0 + int64_t(k) * GP_THREADS + threadIdx.x;
            l[k] = i < c1 ? sorted[i] : -1;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) lds_tally_wave<GP_HT>(hkey, hcnt, parts, l[k]);
    }
    __syncthreads();
    lds_tally_flush<GP_HT>(hkey, hcnt, parts);
}

__global__ void __launch_bounds__(GB) gp_zero_kernel(uint32_t *__restrict__ w, int64_t count) {
    for (int64_t i = blockIdx.x * int64_t(GB) + threadIdx.x; i < count; i += int64_t(gridDim.x) * GB) w[i] = 0u;
}

// Bit r of the bitmap for every kept root r (decided in the same pass's keep flags).
__global__ void __launch_bounds__(GB) gp_bits_kernel(const int32_t *__restrict__ roots, int64_t nroots,
                                                     int64_t ncells, const uint8_t *__restrict__ keep,
                                                     uint32_t *__restrict__ bits, uint32_t *__restrict__ summary,
                                                     int blog) {
    for (int64_t i = blockIdx.x * int64_t(GB) + threadIdx.x; i < nroots; i += int64_t(gridDim.x) * GB) {
        const int32_t r = roots[i];
        if (r >= 0 && r < ncells && keep[i]) {
            const uint32_t u = uint32_t(r), blk = u >> blog;
            atomicOr(&bits[u >> 5], 1u << (u & 31u));
            atomicOr(&summary[blk >> 5], 1u << (blk & 31u));
        }
    }
}

// Labels stream through once (non-temporal, so the bitmap and its summary keep
// the cache); the lookups go in phases so every lane has all its loads of one
// kind in flight at once: the labels, then the summary words, then the bitmap
// words of those whose summary block (2^blog cells) holds a kept root.
__global__ void __launch_bounds__(GB) gp_filter_kernel(const int32_t *in, int32_t *out, int64_t count,
                                                       int64_t ncells, const uint32_t *__restrict__ bits,
                                                       const uint32_t *__restrict__ summary, int blog,
                                                       uint32_t *status) {
    constexpr int P = 2 * GPER;
    bool bad = false;
    const int64_t stride = int64_t(gridDim.x) * GB;
    for (int64_t i0 = blockIdx.x * int64_t(GB) + threadIdx.x; i0 < count; i0 += stride * P) {
        int32_t l[P];
        uint32_t w[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int64_t i = i0 + k * stride;
            l[k] = i < count ? __builtin_nontemporal_load(in + i) : -1;
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (!gp_label_ok(l[k], ncells, bad)) l[k] = -1;
            const uint32_t blk = uint32_t(l[k] < 0 ? 0 : l[k]) >> blog;
            w[k] = summary[blk >> 5] >> (blk & 31u);
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const uint32_t u = uint32_t(l[k]);
            w[k] = (l[k] >= 0 && (w[k] & 1u)) ? bits[u >> 5] >> (u & 31u) : 0u;
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int64_t i = i0 + k * stride;
            if (i < count) __builtin_nontemporal_store((w[k] & 1u) ? l[k] : -1, out + i);
        }
    }
    if (bad) atomicOr(status, ST_INPUT);
}

// The same filter for labels in no spatial order (particles in input order):
// there neighbouring lanes look up unrelated summary words, which the vector
// cache serves one line at a time, so each workgroup first copies the summary
// (at most 128 KB) into LDS and looks it up there.
constexpr int GP_FP = 16;  // labels per thread per sweep of the LDS filter
__global__ void __launch_bounds__(GP_THREADS) gp_filter_lds_kernel(const int32_t *in, int32_t *out, int64_t count,
                                                                   int64_t ncells, const uint32_t *__restrict__ bits,
                                                                   const uint32_t *__restrict__ summary,
                                                                   int swords, int blog, uint32_t *status) {
    extern __shared__ uint32_t gp_lsum[];
    for (int i = threadIdx.x; i < swords; i += GP_THREADS) gp_lsum[i] = summary[i];
    __syncthreads();
    bool bad = false;
    const int64_t stride = int64_t(gridDim.x) * GP_THREADS;
    for (int64_t i0 = blockIdx.x * int64_t(GP_THREADS) + threadIdx.x; i0 < count; i0 += stride * GP_FP) {
        int32_t l[GP_FP];
        uint32_t w[GP_FP];
#pragma unroll
        for (int k = 0; k < GP_FP; ++k) {
            const int64_t i = i0 + k * stride;
            l[k] = i < count ? __builtin_nontemporal_load(in + i) : -1;
        }
#pragma unroll
        for (int k = 0; k < GP_FP; ++k) {
            if (!gp_label_ok(l[k], ncells, bad)) l[k] = -1;
            const uint32_t blk = uint32_t(l[k] < 0 ? 0 : l[k]) >> blog;
            w[k] = gp_lsum[blk >> 5] >> (blk & 31u);
        }
#pragma unroll
        for (int k = 0; k < GP_FP; ++k) {
            const uint32_t u = uint32_t(l[k]);
            w[k] = (l[k] >= 0 && (w[k] & 1u)) ? bits[u >> 5] >> (u & 31u) : 0u;
        }
#pragma unroll
        for (int k = 0; k < GP_FP; ++k) {
            const int64_t i = i0 + k * stride;
            if (i < count) __builtin_nontemporal_store((w[k] & 1u) ? l[k] : -1, out + i);
        }
    }
    if (bad) atomicOr(status, ST_INPUT);
}

unsigned grid_of(const hf_ctx *ctx, int64_t work, int64_t per_block) {
    const int64_t want = (work + per_block - 1) / per_block;
    const int64_t cap = int64_t(ctx->cus) * 32;
    return unsigned(want < 1 ? 1 : (want > cap ? cap : want));
}

int64_t cells_of(const hf_box &box) { return int64_t(box.n) * box.n * box.n; }

// The partition scratch of hf_groups, after the counters.
size_t part_layout(const hf_box &box, int64_t np, size_t base, void *ws, GroupPart *out) {
    const int64_t ncells = cells_of(box);
    int bitsneeded = 0;
    while ((int64_t(1) << bitsneeded) < ncells) ++bitsneeded;
    const int blog = bitsneeded - GP_SUMMARY_LOG > GP_BLOCK_LOG ? bitsneeded - GP_SUMMARY_LOG : GP_BLOCK_LOG;
    const int64_t fine = (ncells + 31) / 32, coarse = ncells > 0 ? (((ncells - 1) >> blog) >> 5) + 1 : 1;
    const int64_t words = fine + coarse;
    size_t off = base;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    const size_t c = take(sizeof(uint32_t) * (GP_BUCKETS + 1));
    const size_t cur = take(sizeof(uint32_t) * GP_BUCKETS);
    const size_t so = take(sizeof(int32_t) * size_t(np > 0 ? np : 1));
    const size_t bi = take(sizeof(uint32_t) * size_t(words));
    if (out && ws) {
        char *w = static_cast<char *>(ws);
        out->count = reinterpret_cast<uint32_t *>(w + c);
        out->cursor = reinterpret_cast<uint32_t *>(w + cur);
        out->sorted = reinterpret_cast<int32_t *>(w + so);
        out->bits = reinterpret_cast<uint32_t *>(w + bi);
        out->summary = out->bits + fine;
        out->words = words;
        out->swords = coarse;
        out->blog = blog;
        out->shift = bitsneeded > 8 ? bitsneeded - 8 : 0;  // label >> shift < GP_BUCKETS
    }
    return off - base;
}

}  // namespace

size_t hf::groups_part_ws_bytes(const hf_box &box, int64_t np) {
    return part_layout(box, np, 0, nullptr, nullptr);
}

size_t hf::groups_ws_bytes(const hf_box &box) { return 2 * align_up(size_t(cells_of(box)) * sizeof(uint32_t)); }

GroupCounters hf::group_counters_at(const hf_box &box, void *region) {
    unsigned char *base = static_cast<unsigned char *>(region);
    return GroupCounters{reinterpret_cast<uint32_t *>(base),
                         reinterpret_cast<uint32_t *>(base + align_up(size_t(cells_of(box)) * sizeof(uint32_t)))};
}

hf_status hf::groups_count_cells(hf_ctx *ctx, const hf_box &box, const int32_t *roots, const int64_t *d_count,
                                 int64_t cap, const int32_t *cell_label, const GroupCounters &g) {
    const int64_t ncells = cells_of(box);
    if (cap <= 0) return HF_OK;
    HF_LAUNCH(ctx, K_GROUP_CLEAR, groups_clear_kernel, dim3(grid_of(ctx, cap, GB)), dim3(GB), 0, ctx->stream, roots,
              d_count, cap, ncells, g, ctx->d_status);
    const dim3 grid(unsigned((ncells + GCHUNK - 1) / GCHUNK));
    if (reinterpret_cast<uintptr_t>(cell_label) % sizeof(int4) == 0)
        HF_LAUNCH(ctx, K_GROUP_CELLS, groups_runs_kernel<false>, grid, dim3(GB), 0, ctx->stream, cell_label, nullptr,
                  ncells, ncells, g.cells, ctx->d_status);
    else  // rows not 16-byte aligned: one label per lane
        HF_LAUNCH(ctx, K_GROUP_CELLS, groups_tally_kernel<false>, grid, dim3(GB), 0, ctx->stream, cell_label, nullptr,
                  ncells, ncells, g.cells, ctx->d_status);
    return launch_status();
}

hf_status hf::groups_count_particles_tiled(hf_ctx *ctx, const hf_box &box, const int32_t *label, const uint8_t *mask,
                                           int64_t np, const GroupCounters &g) {
    if (np <= 0) return HF_OK;
    const dim3 grid(unsigned((np + GCHUNK - 1) / GCHUNK));
    const bool aligned = reinterpret_cast<uintptr_t>(label) % sizeof(int4) == 0 &&
                         reinterpret_cast<uintptr_t>(mask) % sizeof(int4) == 0;
    if (!mask && aligned)
        HF_LAUNCH(ctx, K_GROUP_PARTICLES, groups_runs_kernel<false>, grid, dim3(GB), 0, ctx->stream, label, nullptr,
                  np, cells_of(box), g.parts, ctx->d_status);
    else if (!mask)
        HF_LAUNCH(ctx, K_GROUP_PARTICLES, groups_tally_kernel<false>, grid, dim3(GB), 0, ctx->stream, label, nullptr,
                  np, cells_of(box), g.parts, ctx->d_status);
    else if (aligned)
        HF_LAUNCH(ctx, K_GROUP_PARTICLES, groups_runs_kernel<true>, grid, dim3(GB), 0, ctx->stream, label, mask, np,
                  cells_of(box), g.parts, ctx->d_status);
    else
        HF_LAUNCH(ctx, K_GROUP_PARTICLES, groups_tally_kernel<true>, grid, dim3(GB), 0, ctx->stream, label, mask, np,
                  cells_of(box), g.parts, ctx->d_status);
    return launch_status();
}

hf_status hf::groups_count_particles(hf_ctx *ctx, const hf_box &box, const int32_t *particle_label, int64_t np,
                                     const GroupCounters &g, const int32_t *skip) {
    if (np <= 0) return HF_OK;
    HF_LAUNCH(ctx, K_GROUP_PARTICLES, groups_particles_kernel, dim3(grid_of(ctx, np, GB * GPER)), dim3(GB), 0,
              ctx->stream, particle_label, skip, np, cells_of(box), g.parts, ctx->d_status);
    return launch_status();
}

hf_status hf::groups_decide(hf_ctx *ctx, const hf_box &box, const int32_t *roots, const int64_t *d_count, int64_t cap,
                            const GroupCounters &g, double dens_th, int64_t np, int64_t particle_th,
                            const uint8_t *root_ok, uint32_t *group_particles, uint32_t *group_cells,
                            uint8_t *group_keep) {
    if (cap <= 0) return HF_OK;
    HF_LAUNCH(ctx, K_GROUP_DECIDE, groups_decide_kernel, dim3(grid_of(ctx, cap, GB)), dim3(GB), 0, ctx->stream, roots,
              d_count, cap, cells_of(box), g, dens_th, double(np), particle_th, root_ok, group_particles, group_cells,
              group_keep);
    return launch_status();
}

hf_status hf::groups_filter(hf_ctx *ctx, const hf_box &box, const int32_t *in, int32_t *out, int64_t count,
                            const GroupCounters &g, bool any_roots) {
    if (count <= 0 || !out) return HF_OK;
    HF_LAUNCH(ctx, K_GROUP_FILTER, groups_filter_kernel, dim3(grid_of(ctx, count, GB * GPER)), dim3(GB), 0,
              ctx->stream, in, out, count, cells_of(box), g.cells, any_roots ? 1 : 0, ctx->d_status);
    return launch_status();
}

hf_status hf::cross_scale_dev(hf_ctx *ctx, const hf_box &box, const int32_t *roots, const int64_t *d_count,
                              int64_t cap, const float *c_scale, int n_smaller, const float *c_smaller,
                              uint8_t *pass) {
    if (cap <= 0) return HF_OK;
    HF_LAUNCH(ctx, K_GROUP_CROSS, cross_scale_kernel, dim3(grid_of(ctx, cap, GB)), dim3(GB), 0, ctx->stream, roots,
              d_count, cap, box.n, c_scale, n_smaller, c_smaller, pass, ctx->d_status);
    return launch_status();
}

hf_status hf::claim_init(hf_ctx *ctx, int32_t *halo_scale, int32_t *halo_root, int64_t np) {
    if (np <= 0) return HF_OK;
    HF_LAUNCH(ctx, K_CLAIM, claim_init_kernel, dim3(grid_of(ctx, np, GB * GPER)), dim3(GB), 0, ctx->stream,
              halo_scale, halo_root, np);
    return launch_status();
}

hf_status hf::claim_filter(hf_ctx *ctx, const hf_box &box, int32_t *label, int32_t *halo_scale, int32_t *halo_root,
                           int64_t np, const GroupCounters &g, bool any_roots, int32_t scale) {
    if (np <= 0) return HF_OK;
    HF_LAUNCH(ctx, K_CLAIM, claim_filter_kernel, dim3(grid_of(ctx, np, GB * GPER)), dim3(GB), 0, ctx->stream, label,
              halo_scale, halo_root, np, cells_of(box), g.cells, any_roots ? 1 : 0, scale, ctx->d_status);
    return launch_status();
}

extern "C" hf_status hf_peaks(hf_ctx *ctx, const hf_box *box, const float *cwt, const int32_t *roots, int64_t nroots,
                              double *pos, double *value) {
    if (!ctx) return HF_ERR_ARG;
    hf_status s = check_box_grid(box);
    if (s != HF_OK) return s;
    if (nroots < 0 || nroots > cells_of(*box)) return HF_ERR_ARG;
    if (nroots == 0) return HF_OK;
    if (!cwt || !roots || !pos || !value) return HF_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    HF_LAUNCH(ctx, K_PEAKS, peaks_kernel, dim3(grid_of(ctx, nroots, GB)), dim3(GB), 0, ctx->stream, roots, nroots,
              box->n, box->box_len / box->n, box->box_len, cwt, pos, value, ctx->d_status);
    return launch_status();
}

extern "C" hf_status hf_cross_scale(hf_ctx *ctx, const hf_box *box, const int32_t *roots, int64_t nroots,
                                    const float *cwt_scale, int32_t n_smaller, const float *cwt_smaller,
                                    uint8_t *pass) {
    if (!ctx) return HF_ERR_ARG;
    hf_status s = check_box_grid(box);
    if (s != HF_OK) return s;
    if (n_smaller < 1 || n_smaller > 1024) return HF_ERR_SIZE;
    if (nroots < 0 || nroots > cells_of(*box)) return HF_ERR_ARG;
    if (nroots == 0) return HF_OK;
    if (!roots || !cwt_scale || !cwt_smaller || !pass) return HF_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    HF_LAUNCH(ctx, K_GROUP_CROSS, cross_scale_kernel, dim3(grid_of(ctx, nroots, GB)), dim3(GB), 0, ctx->stream, roots,
              nullptr, nroots, box->n, cwt_scale, int(n_smaller), cwt_smaller, pass, ctx->d_status);
    return launch_status();
}

extern "C" hf_status hf_groups(hf_ctx *ctx, const hf_box *box, int64_t np, const int32_t *roots, int64_t nroots,
                               const int32_t *cell_label, const int32_t *particle_label, double dens_th,
                               int64_t particle_th, const uint8_t *root_ok, uint32_t *group_particles,
                               uint32_t *group_cells,
                               uint8_t *group_keep, int32_t *cell_label_out, int32_t *particle_label_out, void *ws,
                               size_t ws_bytes) {
    if (!ctx || !cell_label) return HF_ERR_ARG;
    hf_status s = check_box_grid(box);
    if (s != HF_OK) return s;
    const int64_t ncells = cells_of(*box);
    if (np < 0 || np > int64_t(UINT32_MAX) || nroots < 0 || nroots > ncells) return HF_ERR_ARG;
    if (!(dens_th >= 0.0) || !(dens_th < 1e300) || particle_th < 0) return HF_ERR_ARG;
    if (np > 0 && !particle_label) return HF_ERR_ARG;
    if (nroots > 0 && (!roots || !group_particles || !group_cells || !group_keep)) return HF_ERR_ARG;
    s = check_ws(ws, ws_bytes, groups_ws_bytes(*box));
    if (s != HF_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    const GroupCounters g = group_counters_at(*box, ws);
    // with room for the partition scratch (the size hf_workspace_size gives for
    // HF_STAGE_GROUPS alone), the particles are partitioned before they are
    // counted and the filters read a keep bitmap; else one global atomic per
    // labelled particle and the keep flags in the counters
    const size_t base = groups_ws_bytes(*box);
    GroupPart gp{};
    const bool part = ws_bytes >= base + groups_part_ws_bytes(*box, np);
    if (part) part_layout(*box, np, base, ws, &gp);
    hipStream_t st = ctx->stream;
    if (part) {
        HF_LAUNCH(ctx, K_GROUP_CLEAR, gp_zero_kernel, dim3(grid_of(ctx, gp.words, GB)), dim3(GB), 0, st, gp.bits,
                  gp.words);
        HF_LAUNCH(ctx, K_GROUP_CLEAR, gp_zero_kernel, dim3(1), dim3(GB), 0, st, gp.count, int64_t(GP_BUCKETS + 1));
    }
    if (nroots > 0) {
        s = groups_count_cells(ctx, *box, roots, nullptr, nroots, cell_label, g);
        if (s == HF_OK && part && np > 0) {
            HF_LAUNCH(ctx, K_GROUP_PARTICLES, gp_hist_kernel, dim3(unsigned((np + GP_HCHUNK - 1) / GP_HCHUNK)),
                      dim3(512), 0, st, particle_label, np, ncells, gp.shift, gp.count, ctx->d_status);
            HF_LAUNCH(ctx, K_GROUP_PARTICLES, gp_scan_kernel, dim3(1), dim3(GP_BUCKETS), 0, st, gp.count, gp.cursor);
            const dim3 chunks(unsigned((np + GP_CHUNK - 1) / GP_CHUNK));
            HF_LAUNCH(ctx, K_GROUP_PARTICLES, gp_scatter_kernel, chunks, dim3(GP_THREADS), 0, st, particle_label, np,
                      ncells, gp.shift, gp.cursor, gp.sorted);
            HF_LAUNCH(ctx, K_GROUP_PARTICLES, gp_count_kernel, dim3(unsigned((np + GP_CCHUNK - 1) / GP_CCHUNK)),
                      dim3(GP_THREADS), 0, st, gp.sorted, gp.count, g.parts);
            s = launch_status();
        } else if (s == HF_OK) {
            s = groups_count_particles(ctx, *box, particle_label, np, g);
        }
        if (s == HF_OK)
            s = groups_decide(ctx, *box, roots, nullptr, nroots, g, dens_th, np, particle_th, root_ok,
                              group_particles, group_cells, group_keep);
        if (s != HF_OK) return s;
        if (part)
            HF_LAUNCH(ctx, K_GROUP_DECIDE, gp_bits_kernel, dim3(grid_of(ctx, nroots, GB)), dim3(GB), 0, st, roots,
                      nroots, ncells, group_keep, gp.bits, gp.summary, gp.blog);
    }
    if (part) {
        if (cell_label_out)
            HF_LAUNCH(ctx, K_GROUP_FILTER, gp_filter_kernel, dim3(grid_of(ctx, ncells, GB * 2 * GPER)), dim3(GB), 0, st,
                      cell_label, cell_label_out, ncells, ncells, gp.bits, gp.summary, gp.blog, ctx->d_status);
        if (particle_label_out && np > 0) {
            const size_t lds = sizeof(uint32_t) * size_t(gp.swords);
            const void *f = reinterpret_cast<const void *>(&gp_filter_lds_kernel);
            const hf_status before = launch_status();  // the attribute call below may leave its own error
            if (before != HF_OK) return before;
            if (lds <= 65536 || hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) == hipSuccess) {
                const int64_t want = (np + int64_t(GP_THREADS) * GP_FP - 1) / (int64_t(GP_THREADS) * GP_FP);
                const unsigned grid = unsigned(want < int64_t(ctx->cus) * 2 ? want : int64_t(ctx->cus) * 2);
                HF_LAUNCH(ctx, K_GROUP_FILTER, gp_filter_lds_kernel, dim3(grid), dim3(GP_THREADS), lds, st,
                          particle_label, particle_label_out, np, ncells, gp.bits, gp.summary, int(gp.swords), gp.blog,
                          ctx->d_status);
            } else {
                (void)hipGetLastError();  // no room for the summary in LDS: look it up through the cache
                HF_LAUNCH(ctx, K_GROUP_FILTER, gp_filter_kernel, dim3(grid_of(ctx, np, GB * 2 * GPER)), dim3(GB), 0,
                          st, particle_label, particle_label_out, np, ncells, gp.bits, gp.summary, gp.blog,
                          ctx->d_status);
            }
        }
        return launch_status();
    }
    s = groups_filter(ctx, *box, cell_label, cell_label_out, ncells, g, nroots > 0);
    if (s == HF_OK) s = groups_filter(ctx, *box, particle_label, particle_label_out, np, g, nroots > 0);
    return s;
}
