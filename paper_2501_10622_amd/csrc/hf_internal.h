// Internal definitions shared by the HIP translation units of libhf.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "hf.h"

namespace hf {

// Kernels whose launches the optional per-context timer tracks.
enum KernelId {
    K_ZERO_GRID, K_DEPOSIT, K_LABEL,
    K_DEP_ATOMIC, K_DEP_PREP, K_DEP_L1_HIST, K_DEP_L1_SCATTER, K_DEP_L2_HIST, K_DEP_L2_SCATTER, K_DEP_FOLD,
    K_TABLES_1, K_TABLES_2, K_X_FWD, K_MASS, K_Y_FWD, K_Z_MUL, K_Y_INV, K_X_INV,
    K_MAX_MARK, K_MAX_COUNT, K_MAX_SCAN, K_MAX_WRITE,
    K_PARENT, K_FLAGS, K_JUMP, K_FINALIZE,
    K_LABEL_TILES, K_LABEL_LEVEL1, K_LABEL_INPUT,
    K_GROUP_CLEAR, K_GROUP_CELLS, K_GROUP_PARTICLES, K_GROUP_DECIDE, K_GROUP_FILTER, K_GROUP_CROSS, K_PEAKS,
    K_ST_X, K_ST_MASS, K_ST_Y, K_ST_Z, K_CLAIM, K_UNBIND,
    K_COUNT
};
const char *kernel_name(int id);

struct ProfRecord {
    int kid;
    hipEvent_t start, stop;
};

}  // namespace hf

struct hf_ctx {
    int device;
    int cus = 256;  // compute units of the device
    hipStream_t stream;
    uint32_t *d_status;  // device status block: [0] error bit mask
    uint32_t *h_status;  // pinned host mirror
    void *scratch = nullptr;  // this device's hf_find_halos_noalloc workspace
    // kernel timer (off unless hf_profile_enable): events around every launch
    bool prof = false;
    std::vector<hf::ProfRecord> pending;
    std::vector<hipEvent_t> pool;
    double ms[hf::K_COUNT] = {};
    int64_t launches[hf::K_COUNT] = {};
};

namespace hf {

hipEvent_t take_event(hf_ctx *c);

// Brackets the launches issued in its scope with timing events when the
// context's timer is on.
struct ProfScope {
    hf_ctx *c;
    int kid;
    hipEvent_t start = nullptr;
    ProfScope(hf_ctx *ctx, int id) : c(ctx), kid(id) {
        if (c->prof) {
            start = take_event(c);
            if (start) (void)hipEventRecord(start, c->stream);
        }
    }
    ~ProfScope() {
        if (c->prof && start) {
            hipEvent_t stop = take_event(c);
            if (stop) {
                (void)hipEventRecord(stop, c->stream);
                c->pending.push_back({kid, start, stop});
            }
        }
    }
};

// Launches a kernel on ctx->stream under the context's kernel timer.
#define HF_LAUNCH(ctx, kid, ...)                 \
    do {                                         \
        ::hf::ProfScope hf_prof_scope_(ctx, kid); \
        hipLaunchKernelGGL(__VA_ARGS__);         \
    } while (0)

// Device status bits (one per device-detected hf_status code).
constexpr uint32_t ST_OVERFLOW = 1u << HF_ERR_OVERFLOW;
constexpr uint32_t ST_CAPACITY = 1u << HF_ERR_CAPACITY;
constexpr uint32_t ST_INPUT = 1u << HF_ERR_INPUT;

constexpr size_t WS_ALIGN = 256;

inline size_t align_up(size_t x, size_t a = WS_ALIGN) { return (x + a - 1) / a * a; }

// n = 2^a 3^b, a >= 1, 8 <= n <= 1024.
inline bool supported_n(int n) {
    if (n < 8 || n > 1024 || (n & 1)) return false;
    int m = n;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    return m == 1;
}

inline hf_status check_box(const hf_box *box) {
    if (!box) return HF_ERR_ARG;
    if (!supported_n(box->n)) return HF_ERR_SIZE;
    if (box->frac_bits < 8 || box->frac_bits > 20) return HF_ERR_SIZE;
    if (!(box->box_len > 0.0) || !(box->box_len < 1e300)) return HF_ERR_ARG;
    return HF_OK;
}

// The stages that use no FFT (deposit, stencil transform, maxima,
// segmentation, labels, groups, peaks, cross-scale) take any 8 <= n <= 1024:
// the flowchart's per-scale grids N_g = Int(400 k_w + 150) are arbitrary
// integers.  Grids their tiled paths cannot cover take the direct ones.
inline hf_status check_box_grid(const hf_box *box) {
    if (!box) return HF_ERR_ARG;
    if (box->n < 8 || box->n > 1024) return HF_ERR_SIZE;
    if (box->frac_bits < 8 || box->frac_bits > 20) return HF_ERR_SIZE;
    if (!(box->box_len > 0.0) || !(box->box_len < 1e300)) return HF_ERR_ARG;
    return HF_OK;
}

// The one-call pipelines: the FFT transform needs n = 2^a 3^b, the stencil
// transform any grid; their stage sets (the stencil's workspace replaces the FFT's).
inline hf_status check_box_for(const hf_box *box, hf_kernel k) {
    return k == HF_KERNEL_STENCIL ? check_box_grid(box) : check_box(box);
}
inline int pipeline_stages(hf_kernel k) {
    return k == HF_KERNEL_STENCIL ? ((HF_STAGE_ALL & ~HF_STAGE_CWT) | HF_STAGE_STENCIL) : HF_STAGE_ALL;
}

inline hf_status check_ws(void *ws, size_t ws_bytes, size_t need) {
    if (need == 0) return HF_OK;
    if (!ws || ws_bytes < need) return HF_ERR_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % WS_ALIGN) return HF_ERR_WORKSPACE;
    return HF_OK;
}

inline hf_status launch_status() {
    return hipGetLastError() == hipSuccess ? HF_OK : HF_ERR_DEVICE;
}

// The binned deposit's particle order, kept for the label stage: the level-2
// records (tile order), the bucket and tile offsets, the number of records and,
// for both partition levels, where every element went.  Lives in a caller
// workspace region of particle_order_bytes(box, np).
struct ParticleOrder {
    uint64_t *rec2;
    uint32_t *start2;
    uint32_t *nrec;
    uint32_t *start1;       // [513] first record of each bucket
    uint32_t *chunk_first;  // [513] first level-2 scatter chunk of each bucket
    // where each level's scatter chunks put their elements (layout private to
    // the deposit's translation unit)
    alignas(8) unsigned char maps[2][32];
};
bool particle_order_supported(const hf_box &box, int64_t np);  // binned, more than one bucket
size_t particle_order_bytes(const hf_box &box, int64_t np);
ParticleOrder particle_order_at(const hf_box &box, void *base, int64_t np);

// Binned deposit (n % 16 == 0, B <= 17, np < 2^32).  With `order`, the level-2
// records and tile offsets go to the order region and the slot maps are
// written; the workspace is then deposit_tiled_ws_bytes(box, np, true).
bool deposit_tiled_supported(const hf_box &box, int64_t np);
size_t deposit_tiled_ws_bytes(const hf_box &box, int64_t np, bool keep_order = false);
hf_status deposit_tiled(hf_ctx *ctx, const hf_box &box, const void *pos, hf_dtype dtype, int64_t np, int64_t *rho,
                        void *ws, const ParticleOrder *order = nullptr);

// Step 6 through a kept particle order, with label_scratch_bytes(np) of
// scratch.  Same result as hf_label on the positions the order was built from.
size_t label_scratch_bytes(int64_t np);
hf_status label_from_order(hf_ctx *ctx, const hf_box &box, int64_t np, const ParticleOrder &order,
                           const int32_t *cell_label, int32_t *particle_label, void *scratch);

// Steps 4 and 5 in one pass over the field where the grid is tiled (n % 32 ==
// 0), else hf_maxima then hf_segment; workspace maxima_segment_ws_bytes(box).
size_t maxima_segment_ws_bytes(const hf_box &box);
hf_status maxima_segment(hf_ctx *ctx, const hf_box &box, const float *cwt, float tau, int32_t *max_idx,
                         int64_t max_cap, int64_t *d_count, int32_t *cell_label, void *ws, size_t ws_bytes);

// Group statistics (steps 5 and 7): per-root counters in two n^3 uint32 arrays
// indexed by the root's cell (only the listed roots' entries are touched);
// after the decision cells[root] holds the keep flag.  groups_ws_bytes(box).
struct GroupCounters {
    uint32_t *parts;
    uint32_t *cells;
};
GroupCounters group_counters_at(const hf_box &box, void *region);
// Clears the counters of roots[0, min(*d_count, cap)) (all cap with d_count
// null) and counts every group's cells.
hf_status groups_count_cells(hf_ctx *ctx, const hf_box &box, const int32_t *roots, const int64_t *d_count,
                             int64_t cap, const int32_t *cell_label, const GroupCounters &g);
// Counts particle labels in input order (one atomic per labelled particle).
hf_status groups_count_particles(hf_ctx *ctx, const hf_box &box, const int32_t *particle_label, int64_t np,
                                 const GroupCounters &g, const int32_t *skip = nullptr);
// The same count over labels in the deposit's tile order (LDS tables; entries
// whose mask byte is nonzero skipped; mask may be null).
hf_status groups_count_particles_tiled(hf_ctx *ctx, const hf_box &box, const int32_t *label, const uint8_t *mask,
                                       int64_t np, const GroupCounters &g);
// Decides every group and writes the per-group outputs; then, where given,
// the filtered cell labels.
hf_status groups_decide(hf_ctx *ctx, const hf_box &box, const int32_t *roots, const int64_t *d_count, int64_t cap,
                        const GroupCounters &g, double dens_th, int64_t np, int64_t particle_th,
                        const uint8_t *root_ok, uint32_t *group_particles, uint32_t *group_cells,
                        uint8_t *group_keep);
hf_status groups_filter(hf_ctx *ctx, const hf_box &box, const int32_t *in, int32_t *out, int64_t count,
                        const GroupCounters &g, bool any_roots);

// Where the pass back to input order also claims particles for a scale of the
// identification loop: a label l >= 0 sets halo_scale = scale and
// halo_root = l; with first, every particle is written (-1 and -1 where
// l < 0), so that the two arrays need no clearing before the first scale.
struct ClaimOut {
    int32_t *halo_scale;
    int32_t *halo_root;
    int32_t scale;
    int32_t first;
};
// The same loop's claim state in the deposit's tile order (cs, one byte per
// level-2 slot: 1 once an earlier scale claimed the particle, else 0), tested
// and advanced by the pass to level-1 order: a label survives only where cs
// is 0, its group is kept and the scale has maxima (any), and then claims its
// slot.  With first, cs is not read but written for every slot.
struct TileClaim {
    uint8_t *cs;
    int32_t first;
    int32_t any;
};

// Step 6 through a kept particle order in its two halves: the tile pass
// (counting each label's particles into parts when given) and the two passes
// back to input order (labels of groups whose keep flag is 0 become -1 when
// keep is given; the particles claimed when claim is given).
// label_from_order is the two in turn.
hf_status label_tiles(hf_ctx *ctx, const hf_box &box, int64_t np, const ParticleOrder &order,
                      const int32_t *cell_label, void *scratch, uint32_t *parts);
hf_status label_back(hf_ctx *ctx, const hf_box &box, int64_t np, const ParticleOrder &order,
                     int32_t *particle_label, void *scratch, const uint32_t *keep, const ClaimOut *claim = nullptr,
                     const TileClaim *tile_claim = nullptr);

// Workspace requirements of each stage (defined next to each stage).
size_t deposit_ws_bytes(const hf_box &box, int64_t np);
size_t cwt_ws_bytes(const hf_box &box);
size_t maxima_ws_bytes(const hf_box &box);
size_t segment_ws_bytes(const hf_box &box);
size_t groups_ws_bytes(const hf_box &box);
// hf_groups' partition scratch beyond the counters (labels partitioned by
// range, a keep bitmap), for the workspace hf_workspace_size gives for
// HF_STAGE_GROUPS alone.
size_t groups_part_ws_bytes(const hf_box &box, int64_t np);
// Step 8 with the maxima count on the device (cap = the list's capacity); the
// smaller scale's field is on an n_smaller^3 grid over the same box; c_smaller
// null compares with the all-zero grid.
hf_status cross_scale_dev(hf_ctx *ctx, const hf_box &box, const int32_t *roots, const int64_t *d_count, int64_t cap,
                          const float *c_scale, int n_smaller, const float *c_smaller, uint8_t *pass);
// The identification loop's particle bookkeeping (halo_scale / halo_root).
hf_status claim_init(hf_ctx *ctx, int32_t *halo_scale, int32_t *halo_root, int64_t np);
// After the decision: labels of claimed particles and of disposed groups
// become -1, and the kept ones claim their particles for `scale` (halo_root
// may be null).
hf_status claim_filter(hf_ctx *ctx, const hf_box &box, int32_t *label, int32_t *halo_scale, int32_t *halo_root,
                       int64_t np, const GroupCounters &g, bool any_roots, int32_t scale);
size_t stencil_ws_bytes(const hf_box &box);
// Steps 9-10 for the kept groups (keep[i]) of the roots: afterwards only the
// bound particles of the groups that pass keep their labels; bound_keep[i]
// receives the decision.  nroots is the list's capacity; with d_count the
// list holds min(*d_count, nroots) roots.  Workspace: unbind_ws_bytes(box, np,
// nroots).
size_t unbind_ws_bytes(const hf_box &box, int64_t np, int64_t nroots);
hf_status unbind_dev(hf_ctx *ctx, const hf_box &box, const void *pos, const void *vel, hf_dtype dtype, int64_t np,
                     const int32_t *roots, int64_t nroots, const uint8_t *keep, int32_t *label, double grav_mass,
                     int64_t particle_th, uint8_t *bound_keep, void *ws, const int64_t *d_count = nullptr);
// Particles that scale `scale` claimed and whose label is now -1 are free again.
hf_status unclaim(hf_ctx *ctx, const int32_t *label, int64_t np, int32_t scale, int32_t *halo_scale,
                  int32_t *halo_root);
// The stencil half-width of HF_KERNEL_STENCIL on an n^3 grid: Table 1's
// count Int(1.5/k_w + 5) is in cells of the flowchart's grid for the scale,
// N_g = Int(400 k_w + 150), where it spans 10-12 scale lengths; on n cells the
// same physical extent is ceil(count n / N_g) cells (the count itself when
// n = N_g).  -1 when that exceeds HF_STENCIL_MAX_HALF_WIDTH.  Each FP64 sum
// is its own statement, so the host compiler cannot fuse it into an FMA.
inline int32_t stencil_half_width(double kw, int n) {
    double c = 1.5 / kw;
    c = c + 5.0;
    double g = 400.0 * kw;
    g = g + 150.0;
    if (!(c < 1e9) || !(g < 1e9)) return -1;
    const int64_t count = int64_t(__builtin_floor(c)), ng = int64_t(__builtin_floor(g));
    const int64_t h = (count * n + ng - 1) / ng;
    return h <= HF_STENCIL_MAX_HALF_WIDTH ? int32_t(h) : -1;
}

// ---------------------------------------------------------------------------
// Exact 128-bit sums of non-negative int64 cell masses (the mean density of a
// grid is formed from the exact total).
// ---------------------------------------------------------------------------
struct Mass128 {
    unsigned long long lo, hi;
};

__device__ __forceinline__ void add128(unsigned long long &lo, unsigned long long &hi, unsigned long long v) {
    unsigned long long t = lo + v;
    hi += (t < lo);
    lo = t;
}

// Correctly rounded conversion of a 128-bit unsigned integer to double.
__device__ inline double u128_to_double(unsigned long long lo, unsigned long long hi) {
    if (hi == 0) {
        // split into 32-bit halves: both converts are exact, one rounding in the add
        return double(uint32_t(lo >> 32)) * 4294967296.0 + double(uint32_t(lo));
    }
    const int lz = __clzll(hi);
    const int sh = 64 - lz;  // bits to drop so the value fits 64 bits
    unsigned long long top = (hi << lz) | (lo >> sh);
    const unsigned long long dropped = lo & ((1ull << sh) - 1ull);
    top |= (dropped != 0);  // sticky bit keeps round-to-nearest correct
    const double t = double(uint32_t(top >> 32)) * 4294967296.0 + double(uint32_t(top));
    return ldexp(t, sh);
}

// ---------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// xcd_remap turns the hardware block index into a logical one such that every
// XCD walks one contiguous range of logical blocks, so neighbouring tiles (which
// share halo and partial lines) are handled by the same L2.  Bijective on [0, G).
// ---------------------------------------------------------------------------
constexpr uint32_t NUM_XCD = 8;

__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t G) {
    const uint32_t q = G / NUM_XCD, r = G % NUM_XCD;
    const uint32_t x = b % NUM_XCD, k = b / NUM_XCD;
    return x * q + (x < r ? x : r) + k;
}

// ---------------------------------------------------------------------------
// Counting labels per workgroup in an LDS hash table of HT (a power of two)
// slots of (label, count), keys -1 when empty, linear probing over at most
// TALLY_PROBES slots; a label that finds no slot there adds to ctr[label]
// directly (so a chunk with more labels than the table holds costs a global
// atomic per extra run, not a scan of the whole table per insert).  lds_tally_wave first
// merges the lanes that share the first pending lane's label with one ballot
// round (the commonest case: a run of one label), then adds the other lanes'
// labels one by one.  Every lane of the wavefront must call it; labels below 0
// are not counted.  After a barrier, lds_tally_flush adds the table to ctr.
// ---------------------------------------------------------------------------
constexpr int TALLY_PROBES = 32;

template <int HT>
__device__ __forceinline__ void lds_tally_add(int32_t *hkey, uint32_t *hcnt, uint32_t *ctr, int32_t l, uint32_t c) {
    static_assert((HT & (HT - 1)) == 0 && HT >= 2, "power-of-two table");
    constexpr int BITS = __builtin_ctz(unsigned(HT));
    uint32_t h = (uint32_t(l) * 2654435761u) >> (32 - BITS);  // Knuth's multiplicative hash, top bits
    constexpr int PROBES = HT < TALLY_PROBES ? HT : TALLY_PROBES;
    for (int probe = 0; probe < PROBES; ++probe) {
        int32_t k = hkey[h];
        if (k == -1) k = atomicCAS(hkey + h, -1, l);  // -1 back: this lane took the slot
        if (k == -1 || k == l) {
            atomicAdd(hcnt + h, c);
            return;
        }
        h = (h + 1) & uint32_t(HT - 1);
    }
    atomicAdd(ctr + l, c);
}

template <int HT>
__device__ __forceinline__ void lds_tally_wave(int32_t *hkey, uint32_t *hcnt, uint32_t *ctr, int32_t l) {
    const unsigned long long m = __ballot(l >= 0);
    if (m == 0) return;
    const int leader = __ffsll((long long)m) - 1;
    const int32_t ll = __shfl(l, leader, 64);
    const bool mine = l >= 0 && l == ll;
    const uint32_t c = uint32_t(__popcll(__ballot(mine)));
    if (int(__lane_id()) == leader) lds_tally_add<HT>(hkey, hcnt, ctr, ll, c);
    if (l >= 0 && !mine) lds_tally_add<HT>(hkey, hcnt, ctr, l, 1u);
}

template <int HT>
__device__ __forceinline__ void lds_tally_init(int32_t *hkey, uint32_t *hcnt) {
    for (int s = threadIdx.x; s < HT; s += blockDim.x) {
        hkey[s] = -1;
        hcnt[s] = 0u;
    }
}

template <int HT>
__device__ __forceinline__ void lds_tally_flush(const int32_t *hkey, const uint32_t *hcnt, uint32_t *ctr) {
    for (int s = threadIdx.x; s < HT; s += blockDim.x)
        if (hkey[s] >= 0 && hcnt[s]) atomicAdd(ctr + hkey[s], hcnt[s]);
}

// ---------------------------------------------------------------------------
// A value the compiler cannot see through: code that uses opaque(threadIdx.x)
// computes its index arithmetic where it stands instead of hoisting it out of
// loops and branches, where it would stay live (and spill) for the whole kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// ---------------------------------------------------------------------------
// Division of 32-bit unsigned integers by an invariant divisor d >= 1 with a
// multiply-high and shifts (Granlund & Montgomery, "Division by invariant
// integers using multiplication", 1994): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, x / d = (t + ((x - t) >> min(l,1))) >> max(l-1,0)
// where t = mulhi(m, x).  Exact for every 32-bit x.
// ---------------------------------------------------------------------------
struct FastDiv {
    uint32_t d = 1, m = 1;
    int s1 = 0, s2 = 0;
    FastDiv() = default;
    explicit FastDiv(uint32_t dd) : d(dd) {
        int l = 0;
        while ((uint64_t(1) << l) < d) ++l;
        m = uint32_t((((uint64_t(1) << l) - d) << 32) / d + 1);
        s1 = l < 1 ? l : 1;
        s2 = l > 1 ? l - 1 : 0;
    }
    __device__ __forceinline__ uint32_t div(uint32_t x) const {
        const uint32_t t = __umulhi(m, x);
        return (t + ((x - t) >> s1)) >> s2;
    }
    __device__ __forceinline__ uint32_t mod(uint32_t x) const { return x - div(x) * d; }
};

// ---------------------------------------------------------------------------
// Fixed-point particle coordinates, shared by the deposit and the labels so
// both stages see exactly the same q for a particle.
// ---------------------------------------------------------------------------
template <typename T>
struct FixedPoint {
    T scale;        // n 2^B / L rounded to T
    T period_t;     // n 2^B as T (exact: at most 10 significant bits)
    int64_t period; // n 2^B
    int bits;

    // q = floor(x * scale) mod n 2^B.  Returns false for a position the
    // deposit rejects (non-finite t or |t| >= 2^62).
    __device__ __forceinline__ bool q(T x, uint32_t &out) const {
        const T t = x * scale;  // single correctly rounded multiply in T
        if (t >= T(0) && t < period_t) {  // in the box: truncation is the floor
            out = static_cast<uint32_t>(t);
            return true;
        }
        if (!(t > T(-4.611686018427388e18) && t < T(4.611686018427388e18))) return false;
        int64_t fl = static_cast<int64_t>(floor(t)) % period;
        if (fl < 0) fl += period;
        out = uint32_t(fl);
        return true;
    }
};

template <typename T>
inline FixedPoint<T> make_fixed_point(const hf_box &box) {
    FixedPoint<T> fp;
    fp.bits = box.frac_bits;
    fp.period = int64_t(box.n) << box.frac_bits;
    fp.period_t = T(fp.period);
    fp.scale = T(double(box.n) * double(int64_t(1) << box.frac_bits) / box.box_len);
    return fp;
}

}  // namespace hf
