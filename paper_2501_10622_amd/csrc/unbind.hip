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
// radius and speed, then the remaining members sorted by (radius, member
// position) -- chunks of UB_CHUNK sorted in LDS, then merged pairwise in
// global memory -- so that a member's inner count is its sorted position plus
// one and its outer sum a suffix sum of 1 / r over the sorted order, formed
// block by block from the outermost inward (O(N log N) per round).  Member
// positions follow particle indices, so equal radii are ordered by particle
// index, the order the definition uses.
#include <cmath>

#include "hf_internal.h"
#include "scan.h"

using namespace hf;

namespace {

constexpr int UB_THREADS = 256;
constexpr int UB_CHUNK = 4096;           // members sorted by radius per LDS pass
constexpr int UB_LDS_WORDS = 3 * UB_CHUNK;  // LDS sort buffer: radii (8 B) and member positions (4 B)
constexpr int UB_SORT_LDS = UB_LDS_WORDS;   // runs of up to this many particle indices are sorted in LDS
constexpr int SCAN_GROUPS = 2;         // scan tag of this use

struct UnbindLayout {
    size_t slot, cnt, start, cursor, partial, queue, pid, rad, ord, tmp, spd, alive, total;
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
    L.queue = take(2 * sizeof(uint32_t));
    L.pid = take(sizeof(int32_t) * size_t(np > 0 ? np : 1));
    L.rad = take(sizeof(double) * size_t(np > 0 ? np : 1));
    L.ord = take(sizeof(uint32_t) * size_t(np > 0 ? np : 1));
    L.tmp = take(sizeof(uint32_t) * size_t(np > 0 ? np : 1));
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

// slot[root_i] = i for every root; cnt[i] = cursor[i] = 0 over the capacity;
// the group kernel's two work counters to 0.
__global__ void __launch_bounds__(UB_THREADS) ub_slots_kernel(const int32_t *__restrict__ roots,
                                                              const int64_t *d_count, int64_t cap, int64_t ncells,
                                                              uint32_t *__restrict__ slot, uint32_t *__restrict__ cnt,
                                                              uint32_t *__restrict__ cur, uint32_t *__restrict__ queue,
                                                              uint32_t *status) {
    const int64_t nroots = ub_roots(d_count, cap);
    if (blockIdx.x == 0 && threadIdx.x < 2) queue[threadIdx.x] = 0u;  // the group kernel's work counters
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

// (R[x], x) < (R[y], y): radius first, then member position.
__device__ __forceinline__ bool by_radius(const double *R, uint32_t x, uint32_t y) {
    const double a = R[x], b = R[y];
    return a < b || (a == b && x < y);
}

// One merge of sorted runs a[0..na) and b[0..nb) into out by the workgroup:
// each thread finds where its share of the output starts on the merge path
// (a binary search), then merges its share in order.
__device__ void merge_runs(const uint32_t *a, int na, const uint32_t *b, int nb, uint32_t *out, const double *R) {
    const int total = na + nb;
    const int per = (total + UB_THREADS - 1) / UB_THREADS;
    const int o0 = int(threadIdx.x) * per;
    if (o0 >= total) return;
    const int o1 = o0 + per < total ? o0 + per : total;
    int lo = o0 - nb > 0 ? o0 - nb : 0, hi = o0 < na ? o0 : na;
    while (lo < hi) {  // how many of the first o0 outputs come from a
        const int i = (lo + hi) >> 1;
        if (by_radius(R, a[i], b[o0 - i - 1])) lo = i + 1;
        else hi = i;
    }
    int i = lo, j = o0 - lo;
    for (int o = o0; o < o1; ++o) {
        const bool from_a = j >= nb || (i < na && by_radius(R, a[i], b[j]));
        out[o] = from_a ? a[i++] : b[j++];
    }
}

// Sorts the member positions ord[0..m) by (R, position) with the workgroup:
// runs of UB_CHUNK in LDS (the all-ascending bitonic network over (radius,
// position) pairs, places past the run taken as +infinity), then pairwise
// merges between ord and tmp.  Returns the array that holds the result.
__device__ uint32_t *sort_by_radius(const double *R, uint32_t *ord, uint32_t *tmp, int m, double *skey,
                                    uint32_t *sidx) {
    for (int c0 = 0; c0 < m; c0 += UB_CHUNK) {
        const int len = m - c0 < UB_CHUNK ? m - c0 : UB_CHUNK;
        for (int k = threadIdx.x; k < len; k += UB_THREADS) {
            const uint32_t x = ord[c0 + k];
            sidx[k] = x;
            skey[k] = R[x];
        }
        __syncthreads();
        int p2 = 1;
        while (p2 < len) p2 <<= 1;
        auto cswap = [&](int lo, int hi) {
            if (hi >= len) return;  // hi is +infinity: nothing moves
            const double a = skey[lo], b = skey[hi];
            const uint32_t x = sidx[lo], y = sidx[hi];
            if (b < a || (b == a && y < x)) {
                skey[lo] = b;
                skey[hi] = a;
                sidx[lo] = y;
                sidx[hi] = x;
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
        for (int k = threadIdx.x; k < len; k += UB_THREADS) ord[c0 + k] = sidx[k];
        __syncthreads();
    }
    uint32_t *src = ord, *dst = tmp;
    for (int w = UB_CHUNK; w < m; w *= 2) {
        for (int a = 0; a < m; a += 2 * w) {
            const int na = m - a < w ? m - a : w;
            const int nb = m - a - na < w ? m - a - na : w;
            merge_runs(src + a, na, src + a + na, nb, dst + a, R);
        }
        __syncthreads();
        uint32_t *t = src;
        src = dst;
        dst = t;
    }
    return src;
}

// The check of kept group g (steps 9-10) by the whole workgroup: its members
// sorted by particle index, then the rounds, the decision and the labels.
template <typename T>
__device__ void check_group(uint32_t g, const T *__restrict__ pos, const T *__restrict__ vel,
                            int32_t *__restrict__ label, const int32_t *__restrict__ roots,
                            const uint32_t *__restrict__ start, int32_t *__restrict__ pid, double *__restrict__ rad,
                            uint32_t *__restrict__ ordb, uint32_t *__restrict__ tmpb, double *__restrict__ spd,
                            uint8_t *__restrict__ alive, int n, double box_len, double gm, int64_t particle_th,
                            uint8_t *__restrict__ bound_keep, double *red, double *lds, uint32_t *s_count) {
    const uint32_t s0 = start[g];
    const int m0 = int(start[g + 1] - s0);
    int32_t *P = pid + s0;
    double *R = rad + s0, *S = spd + s0;
    uint32_t *ord = ordb + s0, *tmp = tmpb + s0;
    uint8_t *A = alive + s0;
    double *skey = lds;                                          // [UB_CHUNK]
    uint32_t *sidx = reinterpret_cast<uint32_t *>(lds + UB_CHUNK);  // [UB_CHUNK]
    block_sort(P, m0, reinterpret_cast<int32_t *>(lds), UB_SORT_LDS);
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
            R[k] = __dsqrt_rn(r2);
            S[k] = s2;
        }
        // the remaining members' positions, in order
        {
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
            uint32_t base = 0;
            for (int k0 = 0; k0 < m0; k0 += UB_THREADS) {
                const int k = k0 + int(threadIdx.x);
                const bool live = k < m0 && A[k] != 0;
                const unsigned long long bits = __ballot(live);
                if (lane == 0) s_count[2 + wave] = uint32_t(__popcll(bits));
                __syncthreads();
                uint32_t before = base;
                for (int w = 0; w < wave; ++w) before += s_count[2 + w];
                if (live) ord[before + __popcll(bits & ((1ull << lane) - 1ull))] = uint32_t(k);
                for (int w = 0; w < UB_THREADS / 64; ++w) base += s_count[2 + w];
                __syncthreads();
            }
        }
        const uint32_t *srt = sort_by_radius(R, ord, tmp, m, skey, sidx);
        if (threadIdx.x == 0) s_count[0] = 0u;
        // the shell potential at each remaining member from its sorted position
        // p: (p + 1) / r inside, plus the suffix sum of 1 / r of the members
        // after it, formed block by block from the outermost inward; a leaver
        // is marked 2 (still counted this round)
        uint32_t leaving = 0;
        {
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
            double carry = 0.0;
            for (int b = ((m - 1) / UB_THREADS) * UB_THREADS; b >= 0; b -= UB_THREADS) {
                const int p = b + int(threadIdx.x);
                const uint32_t x = p < m ? srt[p] : 0u;
                const double r = p < m ? R[x] : 0.0;
                const double v = p < m ? __ddiv_rn(1.0, r) : 0.0;  // inf at r = 0
                double incl = v;  // sum over this lane and the later lanes of the wavefront
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const double y = __shfl_down(incl, off, 64);
                    if (lane + off < 64) incl = __dadd_rn(incl, y);
                }
                const double after = __shfl_down(incl, 1, 64);
                if (lane == 0) red[wave] = incl;
                __syncthreads();
                double later = lane < 63 ? after : 0.0;
                for (int w = wave + 1; w < UB_THREADS / 64; ++w) later = __dadd_rn(later, red[w]);
                const double outer = __dadd_rn(later, carry);
                for (int w = 0; w < UB_THREADS / 64; ++w) carry = __dadd_rn(carry, red[w]);
                __syncthreads();
                if (p < m) {
                    const double phi = -__dmul_rn(gm, __dadd_rn(__ddiv_rn(double(p + 1), r), outer));
                    if (S[x] > __dmul_rn(-2.0, phi)) {
                        A[x] = 2;
                        ++leaving;
                    }
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
    __syncthreads();  // the workgroup's LDS is free for the next group
}

// Persistent: each workgroup takes the next UB_BATCH roots from a work
// counter until the list's count is reached (a grid of one workgroup per root
// would be mostly workgroups with nothing to do: the capacity is far above the
// count, and most groups are not kept).  The batch's kept groups are checked
// one after the other, then their labels.  Two sweeps over the list, each with
// its own counter: first the groups of at least UB_BIG members, then the rest,
// so that the longest checks start first and the short ones fill in around
// them.
constexpr int UB_BATCH = 64;
constexpr uint32_t UB_BIG = 2048;

template <typename T>
__global__ void __launch_bounds__(UB_THREADS)
    ub_group_kernel(const T *__restrict__ pos, const T *__restrict__ vel, int32_t *__restrict__ label,
                    const int32_t *__restrict__ roots, const int64_t *d_count, int64_t cap,
                    const uint8_t *__restrict__ keep, const uint32_t *__restrict__ start, uint32_t *queue,
                    int32_t *__restrict__ pid, double *__restrict__ rad, uint32_t *__restrict__ ordb,
                    uint32_t *__restrict__ tmpb, double *__restrict__ spd, uint8_t *__restrict__ alive, int n, double box_len, double gm,
                    int64_t particle_th, uint8_t *__restrict__ bound_keep) {
    static_assert(UB_BATCH <= UB_THREADS, "one root per thread of a batch");
    __shared__ double red[UB_THREADS / 64];
    __shared__ double lds[UB_LDS_WORDS / 2];         // the sorts' LDS (radii and positions, or particle indices)
    __shared__ uint32_t s_count[2 + UB_THREADS / 64];  // leavers of a round, then per-wavefront counts
    __shared__ uint32_t s_next, s_nlist, s_list[UB_BATCH];
    const int64_t count = ub_roots(d_count, cap);
    for (int sweep = 0; sweep < 2;) {
        if (threadIdx.x == 0) {
            s_next = atomicAdd(queue + sweep, uint32_t(UB_BATCH));
            s_nlist = 0u;
        }
        __syncthreads();
        const uint32_t g0 = s_next;
        if (int64_t(g0) >= count) {
            ++sweep;
            __syncthreads();  // s_next is read before the next take
            continue;
        }
        if (threadIdx.x < UB_BATCH && int64_t(g0) + threadIdx.x < count) {
            const uint32_t g = g0 + threadIdx.x;
            if (!keep[g]) {
                if (sweep == 0) bound_keep[g] = 0;
            } else if ((start[g + 1] - start[g] >= UB_BIG) == (sweep == 0)) {
                s_list[atomicAdd(&s_nlist, 1u)] = g;  // the order of the checks does not matter
            }
        }
        __syncthreads();
        const uint32_t nl = s_nlist;
        for (uint32_t q = 0; q < nl; ++q)
            check_group(s_list[q], pos, vel, label, roots, start, pid, rad, ordb, tmpb, spd, alive, n, box_len, gm,
                        particle_th, bound_keep, red, lds, s_count);
        __syncthreads();  // the batch's list is read before the next take rewrites it
    }
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
    auto *ordb = reinterpret_cast<uint32_t *>(w + L.ord);
    auto *tmpb = reinterpret_cast<uint32_t *>(w + L.tmp);
    auto *spd = reinterpret_cast<double *>(w + L.spd);
    auto *alive = reinterpret_cast<uint8_t *>(w + L.alive);
    const int64_t ncells = int64_t(box.n) * box.n * box.n;
    hipStream_t st = ctx->stream;
    auto *queue = reinterpret_cast<uint32_t *>(w + L.queue);
    HF_LAUNCH(ctx, K_UNBIND, ub_slots_kernel, dim3(ub_grid(ctx, nroots)), dim3(UB_THREADS), 0, st, roots, d_count,
              nroots, ncells, slot, cnt, cur, queue, ctx->d_status);
    if (np > 0)
        HF_LAUNCH(ctx, K_UNBIND, ub_count_kernel, dim3(ub_grid(ctx, np)), dim3(UB_THREADS), 0, st, label, np, roots,
                  d_count, nroots, ncells, slot, keep, cnt, ctx->d_status);
    const ScanJob sj = scan_job(cnt, nroots, partial, start);
    HF_LAUNCH(ctx, K_UNBIND, seg_reduce_kernel<SCAN_GROUPS>, dim3(scan_groups(sj)), dim3(SCAN_THREADS), 0, st, sj);
    HF_LAUNCH(ctx, K_UNBIND, seg_scan_kernel<SCAN_GROUPS>, dim3(scan_groups(sj)), dim3(SCAN_THREADS), 0, st, sj);
    if (np > 0)
        HF_LAUNCH(ctx, K_UNBIND, ub_gather_kernel, dim3(ub_grid(ctx, np)), dim3(UB_THREADS), 0, st, label, np, slot,
                  start, cur, pid);
    // a few resident workgroups per CU take the groups from the work counter
    const int64_t wgs = int64_t(ctx->cus) * 4;
    const dim3 grid(unsigned(nroots < wgs ? nroots : wgs));
    if (dtype == HF_F32)
        HF_LAUNCH(ctx, K_UNBIND, ub_group_kernel<float>, grid, dim3(UB_THREADS), 0, st,
                  static_cast<const float *>(pos), static_cast<const float *>(vel), label, roots, d_count, nroots,
                  keep, start, queue, pid, rad, ordb, tmpb, spd, alive, box.n, box.box_len, grav_mass, particle_th,
                  bound_keep);
    else
        HF_LAUNCH(ctx, K_UNBIND, ub_group_kernel<double>, grid, dim3(UB_THREADS), 0, st,
                  static_cast<const double *>(pos), static_cast<const double *>(vel), label, roots, d_count, nroots,
                  keep, start, queue, pid, rad, ordb, tmpb, spd, alive, box.n, box.box_len, grav_mass, particle_th,
                  bound_keep);
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
