// Steps 9-10 (Sec. 2.3): the self-boundness check of the groups one scale
// keeps.  For each group, repeatedly: the centre of mass of its remaining
// particles (equal masses) and their mean velocity; every particle's radius;
// the spherical shell potential at each particle,
//   Phi_i = -G m [ (members at or inside (r_i, id_i)) / r_i + sum over the
//                  members outside of 1 / r_j ],
// and the particles whose speed relative to the mean exceeds the local escape
// speed sqrt(-2 Phi_i) leave; until none leaves.  A group that lost more than
// 40% of its particles (5 removed > 2 N), or keeps fewer than particle_th, is
// discarded.  Afterwards only the bound particles of the groups that pass keep
// their labels.
//
// Layout of the work: the members of every kept group are gathered into
// contiguous runs (counts, an exclusive scan, then one slot per member by an
// atomic cursor); each group's workgroup sorts its run by particle index, so
// the member order -- and with it every floating-point sum -- does not depend
// on the order the atomics resolved in.  The workgroup then iterates the
// rounds: FP64 reductions for the centre and mean velocity, each member's
// radius and speed, and the potential by a pass over all members in
// LDS-staged tiles (O(N^2) per round: groups hold tens to tens of thousands of
// particles, and the pass needs no sort by radius).  The ties of equal radii
// are broken by particle index, the order the definition uses.
#include <cmath>

#include "hf_internal.h"
#include "scan.h"

using namespace hf;

namespace {

constexpr int UB_THREADS = 256;
constexpr int UB_TILE = 1024;          // members per LDS tile of the potential pass
constexpr int UB_MPT = 4;              // members each thread takes per pass over the tiles
constexpr int UB_SORT_LDS = 8192;      // runs up to this many members are sorted in LDS
constexpr int SCAN_GROUPS = 2;         // scan tag of this use

struct UnbindLayout {
    size_t slot, cnt, start, cursor, partial, pid, rad, inv, spd, alive, total;
};

UnbindLayout unbind_layout(int n, int64_t np, int64_t nroots) {
    UnbindLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.slot = take(sizeof(uint32_t) * size_t(n) * size_t(n) * size_t(n));
    L.cnt = take(sizeof(uint32_t) * size_t(nroots > 0 ? nroots : 1));
    L.start = take(sizeof(uint32_t) * size_t(nroots + 1));
    L.cursor = take(sizeof(uint32_t) * size_t(nroots > 0 ? nroots : 1));
    L.partial = take(sizeof(uint64_t) * SCAN_MAX_GROUPS);
    L.pid = take(sizeof(int32_t) * size_t(np > 0 ? np : 1));
    L.rad = take(sizeof(double) * size_t(np > 0 ? np : 1));
    L.inv = take(sizeof(double) * size_t(np > 0 ? np : 1));
    L.spd = take(sizeof(double) * size_t(np > 0 ? np : 1));
    L.alive = take(sizeof(uint8_t) * size_t(np > 0 ? np : 1));
    L.total = off;
    return L;
}

// Number of roots: min(*d_count, cap) when the count is on the device, else cap.
__device__ __forceinline__ int64_t ub_roots(const int64_t *d_count, int64_t cap) {
    if (!d_count) return cap;
    const int64_t c = *d_count;
    return c < cap ? c : cap;
}

unsigned ub_grid(const hf_ctx *ctx, int64_t work) {
    const int64_t want = (work + UB_THREADS - 1) / UB_THREADS;
    const int64_t cap = int64_t(ctx->cus) * 32;
    return unsigned(want < 1 ? 1 : (want > cap ? cap : want));
}

// slot[root_i] = i for every root; cnt[i] = cursor[i] = 0 over the capacity.
__global__ void __launch_bounds__(UB_THREADS) ub_slots_kernel(const int32_t *__restrict__ roots,
                                                              const int64_t *d_count, int64_t cap, int64_t ncells,
                                                              uint32_t *__restrict__ slot, uint32_t *__restrict__ cnt,
                                                              uint32_t *__restrict__ cur, uint32_t *status) {
    const int64_t nroots = ub_roots(d_count, cap);
    bool bad = false;
    for (int64_t i = blockIdx.x * int64_t(UB_THREADS) + threadIdx.x; i < cap; i += int64_t(gridDim.x) * UB_THREADS) {
        cnt[i] = 0u;
        cur[i] = 0u;
        if (i >= nroots) continue;
        const int32_t r = roots[i];
        if (r < 0 || r >= ncells) {
            bad = true;
            continue;
        }
        slot[r] = uint32_t(i);
    }
    if (bad) atomicOr(status, ST_INPUT);
}

// The group of a label, or -1: a label must be one of the roots (else it is
// reported and dropped), and its group must be kept (else dropped).
__device__ __forceinline__ int64_t group_of(int32_t l, const int32_t *__restrict__ roots, int64_t nroots,
                                            int64_t ncells, const uint32_t *__restrict__ slot,
                                            const uint8_t *__restrict__ keep, bool &bad) {
    if (l < 0) return -1;
    if (l >= ncells) {
        bad = true;
        return -1;
    }
    const uint32_t i = slot[l];
    if (int64_t(i) >= nroots || roots[i] != l) {
        bad = true;
        return -1;
    }
    return keep[i] ? int64_t(i) : -1;
}

// Members per kept group; labels outside a kept group become -1.
__global__ void __launch_bounds__(UB_THREADS) ub_count_kernel(int32_t *__restrict__ label, int64_t np,
                                                              const int32_t *__restrict__ roots,
                                                              const int64_t *d_count, int64_t cap, int64_t ncells,
                                                              const uint32_t *__restrict__ slot,
                                                              const uint8_t *__restrict__ keep,
                                                              uint32_t *__restrict__ cnt, uint32_t *status) {
    const int64_t nroots = ub_roots(d_count, cap);
    bool bad = false;
    for (int64_t p = blockIdx.x * int64_t(UB_THREADS) + threadIdx.x; p < np; p += int64_t(gridDim.x) * UB_THREADS) {
        const int32_t l = label[p];
        if (l < 0) continue;
        const int64_t g = group_of(l, roots, nroots, ncells, slot, keep, bad);
        if (g < 0) label[p] = -1;
        else atomicAdd(cnt + g, 1u);
    }
    if (bad) atomicOr(status, ST_INPUT);
}

// One slot per member in its group's run (in the order the cursors give).
__global__ void __launch_bounds__(UB_THREADS) ub_gather_kernel(const int32_t *__restrict__ label, int64_t np,
                                                               const uint32_t *__restrict__ slot,
                                                               const uint32_t *__restrict__ start,
                                                               uint32_t *__restrict__ cur, int32_t *__restrict__ pid) {
    for (int64_t p = blockIdx.x * int64_t(UB_THREADS) + threadIdx.x; p < np; p += int64_t(gridDim.x) * UB_THREADS) {
        const int32_t l = label[p];
        if (l < 0) continue;  // every label left is a kept group's
        const uint32_t g = slot[l];
        const uint32_t k = atomicAdd(cur + g, 1u);
        pid[start[g] + k] = int32_t(p);
    }
}

// Sorts a[0..m) ascending by the workgroup: a bitonic network in its
// all-ascending form (each merge first compares an element with its mirror in
// the block, then half-cleaners), over the next power of two, with the places
// past m taken as +infinity.  Every comparator puts the smaller value at the
// lower place, so a real value never moves past m and those places are never
// read or written.  Runs of up to lds_cap entries are sorted in LDS.
__device__ void block_sort(int32_t *a, int m, int32_t *lds, int lds_cap) {
    int p2 = 1;
    while (p2 < m) p2 <<= 1;
    const bool in_lds = m <= lds_cap;
    int32_t *s = in_lds ? lds : a;
    if (in_lds) {
        for (int k = threadIdx.x; k < m; k += UB_THREADS) s[k] = a[k];
        __syncthreads();
    }
    auto cswap = [&](int lo, int hi) {
        if (hi >= m) return;  // hi is +infinity: nothing moves
        const int32_t x = s[lo], y = s[hi];
        if (x > y) {
            s[lo] = y;
            s[hi] = x;
        }
    };
    for (int size = 2; size <= p2; size <<= 1) {
        const int half = size >> 1;
        for (int t = threadIdx.x; t < p2 / 2; t += UB_THREADS) {
            const int q = t % half, b = (t / half) * size;
            cswap(b + q, b + size - 1 - q);
        }
        __syncthreads();
        for (int stride = half >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < p2 / 2; t += UB_THREADS) {
                const int lo = 2 * t - (t & (stride - 1));
                cswap(lo, lo + stride);
            }
            __syncthreads();
        }
    }
    if (in_lds) {
        for (int k = threadIdx.x; k < m; k += UB_THREADS) a[k] = s[k];
        __syncthreads();
    }
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v = __dadd_rn(v, __shfl_down(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < UB_THREADS / 64; ++w) t = __dadd_rn(t, red[w]);
    __syncthreads();
    return t;
}

// Minimum-image offset of a coordinate from the group's reference point.
__device__ __forceinline__ double unwrap(double d, double box_len) {
    const double half = __dmul_rn(0.5, box_len);
    if (d >= half) return __dsub_rn(d, box_len);
    if (d < -half) return __dadd_rn(d, box_len);
    return d;
}

// One workgroup per root: the kept groups' check, then their labels.
template <typename T>
__global__ void __launch_bounds__(UB_THREADS)
    ub_group_kernel(const T *__restrict__ pos, const T *__restrict__ vel, int32_t *__restrict__ label,
                    const int32_t *__restrict__ roots, const int64_t *d_count, const uint8_t *__restrict__ keep,
                    const uint32_t *__restrict__ start, int32_t *__restrict__ pid, double *__restrict__ rad,
                    double *__restrict__ inv, double *__restrict__ spd, uint8_t *__restrict__ alive, int n,
                    double box_len, double gm, int64_t particle_th, uint8_t *__restrict__ bound_keep) {
    __shared__ double red[UB_THREADS / 64];
    __shared__ double tr[UB_TILE];
    __shared__ double tinv[UB_TILE];
    __shared__ int32_t tid_[UB_TILE];
    __shared__ uint8_t tal[UB_TILE];
    __shared__ int32_t sort_lds[UB_SORT_LDS];
    __shared__ uint32_t s_count[2];
    const uint32_t g = blockIdx.x;
    if (int64_t(g) >= ub_roots(d_count, int64_t(gridDim.x))) return;  // past the list's count
    if (!keep[g]) {
        if (threadIdx.x == 0) bound_keep[g] = 0;
        return;
    }
    const uint32_t s0 = start[g];
    const int m0 = int(start[g + 1] - s0);
    int32_t *P = pid + s0;
    double *R = rad + s0, *I = inv + s0, *S = spd + s0;
    uint8_t *A = alive + s0;
    block_sort(P, m0, sort_lds, UB_SORT_LDS);
    const uint32_t un = uint32_t(n), r0 = uint32_t(roots[g]);
    const double dx = box_len / double(n);
    const double ref[3] = {__dmul_rn(double(r0 % un), dx), __dmul_rn(double((r0 / un) % un), dx),
                           __dmul_rn(double(r0 / (un * un)), dx)};
    for (int k = threadIdx.x; k < m0; k += UB_THREADS) A[k] = 1;
    __syncthreads();
    int m = m0;
    while (m > 0) {
        // centre of mass and mean velocity of the remaining members
        double sd[3] = {0.0, 0.0, 0.0}, sv[3] = {0.0, 0.0, 0.0};
        for (int k = threadIdx.x; k < m0; k += UB_THREADS) {
            if (!A[k]) continue;
            const int64_t p = P[k];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                sd[a] = __dadd_rn(sd[a], unwrap(__dsub_rn(double(pos[3 * p + a]), ref[a]), box_len));
                sv[a] = __dadd_rn(sv[a], double(vel[3 * p + a]));
            }
        }
        double c[3], u[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c[a] = __ddiv_rn(block_sum(sd[a], red), double(m));
            u[a] = __ddiv_rn(block_sum(sv[a], red), double(m));
        }
        // radius and speed^2 of every remaining member
        for (int k = threadIdx.x; k < m0; k += UB_THREADS) {
            if (!A[k]) continue;
            const int64_t p = P[k];
            double r2 = 0.0, s2 = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double e = __dsub_rn(unwrap(__dsub_rn(double(pos[3 * p + a]), ref[a]), box_len), c[a]);
                const double w = __dsub_rn(double(vel[3 * p + a]), u[a]);
                r2 = __dadd_rn(r2, __dmul_rn(e, e));
                s2 = __dadd_rn(s2, __dmul_rn(w, w));
            }
            const double r = __dsqrt_rn(r2);
            R[k] = r;
            I[k] = __ddiv_rn(1.0, r);  // each member's 1 / r, once per round (inf at r = 0)
            S[k] = s2;
        }
        if (threadIdx.x == 0) s_count[0] = 0u;
        __syncthreads();
        // the shell potential at each remaining member, over LDS tiles of all
        // members; a leaver is marked 2 (still counted this round)
        uint32_t leaving = 0;
        for (int i0 = 0; i0 < m0; i0 += UB_THREADS * UB_MPT) {
            bool mine[UB_MPT];
            double ri[UB_MPT], outer[UB_MPT];
            int32_t pi[UB_MPT];
            uint32_t inner[UB_MPT];
#pragma unroll
            for (int q = 0; q < UB_MPT; ++q) {
                const int i = i0 + q * UB_THREADS + int(threadIdx.x);
                mine[q] = i < m0 && A[i] != 0;
                ri[q] = mine[q] ? R[i] : 0.0;
                pi[q] = mine[q] ? P[i] : 0;
                inner[q] = 0;
                outer[q] = 0.0;
            }
            for (int base = 0; base < m0; base += UB_TILE) {
                const int tile = m0 - base < UB_TILE ? m0 - base : UB_TILE;
                __syncthreads();
                for (int k = threadIdx.x; k < tile; k += UB_THREADS) {
                    tal[k] = A[base + k] != 0;
                    tr[k] = R[base + k];
                    tinv[k] = I[base + k];
                    tid_[k] = P[base + k];
                }
                __syncthreads();
                for (int k = 0; k < tile; ++k) {
                    if (!tal[k]) continue;
                    const double rj = tr[k], ij = tinv[k];
                    const int32_t pj = tid_[k];
#pragma unroll
                    for (int q = 0; q < UB_MPT; ++q) {
                        // at or inside (r_i, i): a point mass at the centre; outside: its own shell
                        const bool in = rj < ri[q] || (rj == ri[q] && pj <= pi[q]);
                        inner[q] += in ? 1u : 0u;
                        if (!in) outer[q] = __dadd_rn(outer[q], ij);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < UB_MPT; ++q) {
                if (!mine[q]) continue;
                const int i = i0 + q * UB_THREADS + int(threadIdx.x);
                const double phi = -__dmul_rn(gm, __dadd_rn(__ddiv_rn(double(inner[q]), ri[q]), outer[q]));
                if (S[i] > __dmul_rn(-2.0, phi)) {
                    A[i] = 2;
                    ++leaving;
                }
            }
        }
        if (leaving) atomicAdd(&s_count[0], leaving);
        __syncthreads();
        const uint32_t left = s_count[0];
        if (left == 0) break;
        for (int k = threadIdx.x; k < m0; k += UB_THREADS)
            if (A[k] == 2) A[k] = 0;
        m -= int(left);
        __syncthreads();
    }
    const int removed = m0 - m;
    const bool ok = m > 0 && 5LL * removed <= 2LL * m0 && int64_t(m) >= particle_th;
    if (threadIdx.x == 0) bound_keep[g] = ok ? 1 : 0;
    for (int k = threadIdx.x; k < m0; k += UB_THREADS)
        if (!ok || !A[k]) label[P[k]] = -1;
}

// The identification loop: particles this scale claimed whose label the check
// removed are free again.
__global__ void __launch_bounds__(UB_THREADS) ub_unclaim_kernel(const int32_t *__restrict__ label, int64_t np,
                                                                int32_t scale, int32_t *__restrict__ halo_scale,
                                                                int32_t *__restrict__ halo_root) {
    for (int64_t p = blockIdx.x * int64_t(UB_THREADS) + threadIdx.x; p < np; p += int64_t(gridDim.x) * UB_THREADS) {
        if (halo_scale[p] == scale && label[p] < 0) {
            halo_scale[p] = -1;
            halo_root[p] = -1;
        }
    }
}

__global__ void __launch_bounds__(UB_THREADS) ub_clear_kernel(int32_t *__restrict__ label, int64_t np) {
    for (int64_t p = blockIdx.x * int64_t(UB_THREADS) + threadIdx.x; p < np; p += int64_t(gridDim.x) * UB_THREADS)
        label[p] = -1;
}

}  // namespace

size_t hf::unbind_ws_bytes(const hf_box &box, int64_t np, int64_t nroots) {
    return unbind_layout(box.n, np, nroots).total;
}

hf_status hf::unbind_dev(hf_ctx *ctx, const hf_box &box, const void *pos, const void *vel, hf_dtype dtype,
                         int64_t np, const int32_t *roots, int64_t nroots, const uint8_t *keep, int32_t *label,
                         double grav_mass, int64_t particle_th, uint8_t *bound_keep, void *ws,
                         const int64_t *d_count) {
    if (nroots <= 0) return HF_OK;
    const UnbindLayout L = unbind_layout(box.n, np, nroots);
    char *w = static_cast<char *>(ws);
    auto *slot = reinterpret_cast<uint32_t *>(w + L.slot);
    auto *cnt = reinterpret_cast<uint32_t *>(w + L.cnt);
    auto *start = reinterpret_cast<uint32_t *>(w + L.start);
    auto *cur = reinterpret_cast<uint32_t *>(w + L.cursor);
    auto *partial = reinterpret_cast<uint64_t *>(w + L.partial);
    auto *pid = reinterpret_cast<int32_t *>(w + L.pid);
    auto *rad = reinterpret_cast<double *>(w + L.rad);
    auto *inv = reinterpret_cast<double *>(w + L.inv);
    auto *spd = reinterpret_cast<double *>(w + L.spd);
    auto *alive = reinterpret_cast<uint8_t *>(w + L.alive);
    const int64_t ncells = int64_t(box.n) * box.n * box.n;
    hipStream_t st = ctx->stream;
    HF_LAUNCH(ctx, K_UNBIND, ub_slots_kernel, dim3(ub_grid(ctx, nroots)), dim3(UB_THREADS), 0, st, roots, d_count,
              nroots, ncells, slot, cnt, cur, ctx->d_status);
    if (np > 0)
        HF_LAUNCH(ctx, K_UNBIND, ub_count_kernel, dim3(ub_grid(ctx, np)), dim3(UB_THREADS), 0, st, label, np, roots,
                  d_count, nroots, ncells, slot, keep, cnt, ctx->d_status);
    const ScanJob sj = scan_job(cnt, nroots, partial, start);
    HF_LAUNCH(ctx, K_UNBIND, seg_reduce_kernel<SCAN_GROUPS>, dim3(scan_groups(sj)), dim3(SCAN_THREADS), 0, st, sj);
    HF_LAUNCH(ctx, K_UNBIND, seg_scan_kernel<SCAN_GROUPS>, dim3(scan_groups(sj)), dim3(SCAN_THREADS), 0, st, sj);
    if (np > 0)
        HF_LAUNCH(ctx, K_UNBIND, ub_gather_kernel, dim3(ub_grid(ctx, np)), dim3(UB_THREADS), 0, st, label, np, slot,
                  start, cur, pid);
    if (dtype == HF_F32)
        HF_LAUNCH(ctx, K_UNBIND, ub_group_kernel<float>, dim3(unsigned(nroots)), dim3(UB_THREADS), 0, st,
                  static_cast<const float *>(pos), static_cast<const float *>(vel), label, roots, d_count, keep,
                  start, pid, rad, inv, spd, alive, box.n, box.box_len, grav_mass, particle_th, bound_keep);
    else
        HF_LAUNCH(ctx, K_UNBIND, ub_group_kernel<double>, dim3(unsigned(nroots)), dim3(UB_THREADS), 0, st,
                  static_cast<const double *>(pos), static_cast<const double *>(vel), label, roots, d_count, keep,
                  start, pid, rad, inv, spd, alive, box.n, box.box_len, grav_mass, particle_th, bound_keep);
    return launch_status();
}

hf_status hf::unclaim(hf_ctx *ctx, const int32_t *label, int64_t np, int32_t scale, int32_t *halo_scale,
                      int32_t *halo_root) {
    if (np <= 0) return HF_OK;
    HF_LAUNCH(ctx, K_UNBIND, ub_unclaim_kernel, dim3(ub_grid(ctx, np)), dim3(UB_THREADS), 0, ctx->stream, label,
              np, scale, halo_scale, halo_root);
    return launch_status();
}

extern "C" hf_status hf_unbind_ws_size(const hf_box *box, int64_t np, int64_t nroots, size_t *bytes) {
    if (!bytes || np < 0 || nroots < 0) return HF_ERR_ARG;
    hf_status s = check_box_grid(box);
    if (s != HF_OK) return s;
    *bytes = unbind_ws_bytes(*box, np, nroots);
    return HF_OK;
}

extern "C" hf_status hf_unbind(hf_ctx *ctx, const hf_box *box, const void *pos, const void *vel, hf_dtype dtype,
                               int64_t np, const int32_t *roots, int64_t nroots, const uint8_t *group_keep,
                               int32_t *particle_label, double grav_mass, int64_t particle_th,
                               uint8_t *bound_keep, void *ws, size_t ws_bytes) {
    if (!ctx) return HF_ERR_ARG;
    hf_status s = check_box_grid(box);
    if (s != HF_OK) return s;
    const int64_t ncells = int64_t(box->n) * box->n * box->n;
    if (np < 0 || np > int64_t(INT32_MAX) || nroots < 0 || nroots > ncells) return HF_ERR_ARG;
    if (dtype != HF_F32 && dtype != HF_F64) return HF_ERR_ARG;
    if (!(grav_mass > 0.0) || !(grav_mass < 1e300) || particle_th < 0) return HF_ERR_ARG;
    if (np > 0 && (!pos || !vel || !particle_label)) return HF_ERR_ARG;
    if (nroots > 0 && (!roots || !group_keep || !bound_keep)) return HF_ERR_ARG;
    s = check_ws(ws, ws_bytes, unbind_ws_bytes(*box, np, nroots));
    if (s != HF_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    if (nroots == 0) {  // no group: every label goes
        if (np > 0)
            HF_LAUNCH(ctx, K_UNBIND, ub_clear_kernel, dim3(ub_grid(ctx, np)), dim3(UB_THREADS), 0, ctx->stream,
                      particle_label, np);
        return launch_status();
    }
    return unbind_dev(ctx, *box, pos, vel, dtype, np, roots, nroots, group_keep, particle_label, grav_mass,
                      particle_th, bound_keep, ws);
}
