// Step 2 (Eq. (1)), binned form of the CIC deposit.
//
// Particles arrive in arbitrary order, so depositing straight into an n^3 grid
// of int64 means random read-modify-writes of whole HBM lines.  Instead:
//
//   L1  partition the particles by coarse bucket (<= 512 buckets of tiles),
//       records = the three fixed-point coordinates q (12 bytes);
//   L2  partition each bucket by tile (TX x 8 x 8 cells, TX = 64, 32 or 16),
//       records = cell-in-tile and fraction bits packed into 8 bytes;
//   ACC one workgroup per row of tiles along x takes the row's tiles in order:
//       each tile's particles' eight CIC weights are accumulated in LDS int64
//       over the tile plus its +x/+y/+z skirt ((TX+1) x 9 x 9 cells), the owned
//       cells written once, the y and z skirt faces to a side buffer, and the x
//       face carried in LDS into the next tile of the row;
//   FOLD each tile adds the y- and z-face sums of its lower neighbours to its
//       y = 0 and z = 0 cells (whole rows).
//
// Level-1 records are stored replica-major: the scatter chunks of one counter
// replica (all on one XCD) write only into that replica's region, where the
// replica's share of every bucket lies back to back, so a chunk's runs land in
// a few pages instead of one page per bucket across the whole array.  Every
// other index (the run maps, the level-2 chunks, step 6's level-1 labels) is
// the bucket-major index the records would have with the buckets contiguous;
// a per-(bucket, replica) table of segment starts converts it to the storage
// slot where the records are read.
//
// Tiles are long in x so that the fold's face accesses are mostly whole rows.
// Each partition pass is a histogram pass plus a scatter pass whose writes are
// staged in LDS so that each workgroup writes one contiguous run per bucket
// (per tile at level 2).  Every sum is an exact integer sum, so the grid does
// not depend on particle order or on the order the atomics resolve in.
//
// With a caller-provided ParticleOrder the level-2 records and the bucket and
// tile offsets outlive the deposit, together with every particle's level-1
// slot and every level-1 record's level-2 slot.  Step 6 then labels the
// records tile by tile from a copy of the tile's cell labels in LDS, and brings
// the labels back to input order through the two slot maps.  Because every
// scatter workgroup writes one run per destination, the slots a workgroup of
// those passes reads form one run per bucket (per tile), which it reads into
// LDS with consecutive lanes on consecutive slots.
#include "hf_internal.h"
#include "scan.h"

using namespace hf;

namespace {

constexpr int TYZ = 8;               // tile extent in y and z
constexpr int AYZ = TYZ + 1;          // accumulator extent in y and z (tile + skirt)
constexpr int MAX_TX = 64;            // tile extent in x: 64, 32 or 16
constexpr int MAX_ACC_CELLS = (MAX_TX + 1) * AYZ * AYZ;
constexpr int PART_THREADS = 1024;
constexpr int PART_PER = 8;
constexpr int CHUNK = PART_THREADS * PART_PER;                          // particles per scatter workgroup
constexpr int HIST_CHUNKS = 8;                                          // scatter chunks per histogram workgroup
constexpr int HCHUNK = CHUNK * HIST_CHUNKS;
constexpr int REPLICAS = 16;   // level-1 counters are replicated to spread atomic traffic
constexpr int MAX_DIGITS = 512;
constexpr int HIST_THREADS = 512;  // histogram workgroups stay at 512 threads
constexpr int ACC_THREADS = 512;
constexpr uint16_t NO_POS = 0xffffu;  // staging position of a particle whose position was rejected
constexpr int OFF_STRIDE = MAX_DIGITS + 2;  // per-chunk row of staging offsets (ndest + 1 used)

// Where one level's scatter chunks put their elements, kept for step 6: the
// position of every element in its chunk's destination-sorted staging order
// (element order; NO_POS if rejected), and per chunk the first slot of each
// destination's run and the staging offset of each destination
// (offset[ndest] = elements staged).  The destination of a staging position is
// not stored: the runs are in destination order, so the offsets give it.
struct RunMaps {
    uint16_t *pos;     // [elements]
    uint32_t *base;    // [chunks * MAX_DIGITS]
    uint16_t *offset;  // [chunks * OFF_STRIDE]
};

// Records one scatter chunk's run table (called by every thread after the
// chunk's offsets and run starts are known).
__device__ __forceinline__ void save_run_table(const RunMaps &m, int64_t chunk, int ndest, const uint32_t *h,
                                               const uint32_t *off, const uint32_t *gbase, uint32_t total) {
    for (int d = threadIdx.x; d < ndest; d += blockDim.x) {
        m.base[chunk * MAX_DIGITS + d] = h[d] ? gbase[d] : 0u;
        m.offset[chunk * OFF_STRIDE + d] = uint16_t(off[d]);
    }
    if (threadIdx.x == 0) m.offset[chunk * OFF_STRIDE + ndest] = uint16_t(total);
}

struct Geom {
    int n;              // grid cells per axis
    int tx;             // tile extent in x (y and z: TYZ); a power of two
    int ltx;            // log2(tx)
    int ntx, nty, ntz;  // tiles per axis
    int btx, bty, btz;  // tiles per bucket along each axis
    int nbx, nby, nbz;  // buckets per axis
    int nbuckets;       // nbx * nby * nbz
    int digits;         // btx * bty * btz tiles per bucket
    int ntiles;         // ntx * nty * ntz
    int skirt;          // side-buffer cells per tile (y and z faces): 17 tx
    int bits;           // fraction bits B
    FastDiv cbx, cby, cbz;  // cells per bucket along x, y, z
    FastDiv tbx, tby, tbz;  // tiles per bucket along x, y, z
};

struct Q3 {
    uint32_t x, y, z;
};

__device__ __forceinline__ int bucket_of(const Geom &g, uint32_t cx, uint32_t cy, uint32_t cz) {
    return int((g.cbz.div(cz) * g.nby + g.cby.div(cy)) * g.nbx + g.cbx.div(cx));
}

__device__ __forceinline__ int tile_in_bucket(const Geom &g, uint32_t cx, uint32_t cy, uint32_t cz) {
    const uint32_t ux = g.tbx.mod(cx >> g.ltx), uy = g.tby.mod(cy >> 3), uz = g.tbz.mod(cz >> 3);
    return int((uz * g.bty + uy) * g.btx + ux);
}

// Packed tile-local record: x field ((cell_x % tx) << B) | frac (6 + B bits),
// y and z fields ((cell % 8) << B) | frac (3 + B bits); 12 + 3B <= 63 bits.
__device__ __forceinline__ uint64_t pack_local(const Geom &g, const Q3 &q) {
    const uint32_t fm = (1u << g.bits) - 1u;
    const int sx = 6 + g.bits, sy = 3 + g.bits;
    const uint64_t lx = (uint64_t((q.x >> g.bits) & uint32_t(g.tx - 1)) << g.bits) | (q.x & fm);
    const uint64_t ly = (uint64_t((q.y >> g.bits) & (TYZ - 1)) << g.bits) | (q.y & fm);
    const uint64_t lz = (uint64_t((q.z >> g.bits) & (TYZ - 1)) << g.bits) | (q.z & fm);
    return lx | (ly << sx) | (lz << (sx + sy));
}

constexpr int LBATCH = 8;  // loads per thread issued together in the streaming passes

// Raw coordinates of particles i0 + k * stride (k < LBATCH) below end, all
// loads issued before any is used.
template <typename T>
struct RawBatch {
    T x[LBATCH], y[LBATCH], z[LBATCH];
};

template <typename T>
__device__ __forceinline__ void load_raw(const T *__restrict__ pos, int64_t i0, int64_t stride, int64_t end,
                                         RawBatch<T> &raw) {
#pragma unroll
    for (int k = 0; k < LBATCH; ++k) {
        const int64_t i = i0 + k * stride;
        if (i < end) {
            raw.x[k] = pos[3 * i + 0];
            raw.y[k] = pos[3 * i + 1];
            raw.z[k] = pos[3 * i + 2];
        }
    }
}

// q of the batch; valid[k] is false for indices past the end and for
// positions the deposit rejects (bad set).
template <typename T>
__device__ __forceinline__ void convert_raw(const RawBatch<T> &raw, int64_t i0, int64_t stride, int64_t end,
                                            const FixedPoint<T> &fp, Q3 (&q)[LBATCH], bool (&valid)[LBATCH],
                                            bool &bad) {
#pragma unroll
    for (int k = 0; k < LBATCH; ++k) {
        valid[k] = false;
        if (i0 + k * stride < end) {
            bool ok = fp.q(raw.x[k], q[k].x);
            ok = fp.q(raw.y[k], q[k].y) && ok;
            ok = fp.q(raw.z[k], q[k].z) && ok;
            valid[k] = ok;
            bad |= !ok;
        }
    }
}

template <typename T>
__device__ __forceinline__ void load_q_batch(const T *__restrict__ pos, int64_t i0, int64_t stride, int64_t end,
                                             const FixedPoint<T> &fp, Q3 (&q)[LBATCH], bool (&valid)[LBATCH],
                                             bool &bad) {
    RawBatch<T> raw;
    load_raw(pos, i0, stride, end, raw);
    convert_raw(raw, i0, stride, end, fp, q, valid, bad);
}

template <typename T>
__device__ __forceinline__ bool load_q(const T *__restrict__ pos, int64_t i, const FixedPoint<T> &fp, Q3 &q) {
    bool ok = fp.q(pos[3 * i + 0], q.x);
    ok = fp.q(pos[3 * i + 1], q.y) && ok;
    ok = fp.q(pos[3 * i + 2], q.z) && ok;
    return ok;
}

// In-place exclusive scan of s[0..count) (count <= 512) by the whole workgroup
// (at least 512 threads); returns the total.  Each wavefront scans 64 entries
// with shuffles, then the wavefront totals are scanned; tmp holds 8 partials.
__device__ uint32_t block_exclusive_scan(uint32_t *s, uint32_t *tmp, int count) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t x = (t < count) ? s[t] : 0u;
    uint32_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (t < MAX_DIGITS && lane == 63) tmp[wave] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < MAX_DIGITS / 64; ++w) {
        const uint32_t v = tmp[w];
        before += w < wave ? v : 0u;
        total += v;
    }
    if (t < count) s[t] = before + inc - x;
    __syncthreads();
    return total;
}

__global__ void zero_u32_kernel(uint32_t *p, int64_t count) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < count; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0u;
}

// Scatter chunk of logical block b, or -1 for a spare block.  Workgroups go
// round-robin to the XCDs, so a logical block b kept on XCD b % 8 (the
// hardware block index, or one plus multiples of a grid size divisible by 8);
// this mapping gives XCD x the chunks of the histogram workgroups h = x
// (mod 8), in order, so the level-1 counter replicas h % REPLICAS it advances
// are its own: every replica's record runs are written (and later read back in
// the same order) through one L2.  The logical blocks are
// [0, replica_grid(nchunks)).
__device__ __forceinline__ int64_t replica_chunk(uint32_t b, uint32_t nchunks) {
    const uint32_t x = b % NUM_XCD, k = b / NUM_XCD;
    const uint64_t c = uint64_t(HIST_CHUNKS) * (x + uint64_t(NUM_XCD) * (k / HIST_CHUNKS)) + k % HIST_CHUNKS;
    return c < nchunks ? int64_t(c) : -1;
}

__host__ __device__ inline unsigned replica_grid(unsigned nchunks) {
    const unsigned g = HIST_CHUNKS * NUM_XCD;
    return (nchunks + g - 1) / g * g;
}
static_assert(REPLICAS % NUM_XCD == 0, "replicas split evenly over the XCDs");

// ---------------------------------------------------------------- level 1
template <typename T>
__global__ void __launch_bounds__(HIST_THREADS) l1_hist_kernel(const T *__restrict__ pos, int64_t np,
                                                               FixedPoint<T> fp, Geom g, uint32_t *count1,
                                                               uint32_t *status) {
    __shared__ uint32_t h[MAX_DIGITS];
    for (int b = threadIdx.x; b < MAX_DIGITS; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    bool bad = false;
    const int64_t base = int64_t(blockIdx.x) * HCHUNK;
    const int64_t end = base + HCHUNK < np ? base + HCHUNK : np;
    for (int64_t i0 = base + threadIdx.x; i0 < end; i0 += HIST_THREADS * LBATCH) {
        Q3 q[LBATCH];
        bool ok[LBATCH];
        load_q_batch(pos, i0, HIST_THREADS, end, fp, q, ok, bad);
#pragma unroll
        for (int k = 0; k < LBATCH; ++k)
            if (ok[k]) atomicAdd(&h[bucket_of(g, q[k].x >> g.bits, q[k].y >> g.bits, q[k].z >> g.bits)], 1u);
    }
    __syncthreads();
    uint32_t *mine = count1 + (blockIdx.x % REPLICAS) * MAX_DIGITS;
    for (int b = threadIdx.x; b < g.nbuckets; b += blockDim.x)
        if (h[b]) atomicAdd(&mine[b], h[b]);
    if (bad) atomicOr(status, ST_INPUT);
}

// start1 = exclusive scan of the bucket totals; cursor1[r][b] = where replica r's
// share of bucket b starts; chunk_first / hchunk_first = exclusive scans of the
// number of level-2 scatter / histogram chunks per bucket.
__global__ void __launch_bounds__(MAX_DIGITS) l1_scan_kernel(const uint32_t *__restrict__ count1, int nbuckets,
                                                             uint32_t *start1, uint32_t *cursor1,
                                                             uint32_t *chunk_first, uint32_t *hchunk_first,
                                                             uint32_t *nrec_out) {
    __shared__ uint32_t s[MAX_DIGITS], c[MAX_DIGITS], hc[MAX_DIGITS], tmp[MAX_DIGITS];
    const int t = threadIdx.x;
    uint32_t cnt = 0;
    if (t < nbuckets)
        for (int r = 0; r < REPLICAS; ++r) cnt += count1[r * MAX_DIGITS + t];
    s[t] = cnt;
    c[t] = (cnt + CHUNK - 1) / CHUNK;
    hc[t] = (cnt + HCHUNK - 1) / HCHUNK;
    __syncthreads();
    const uint32_t total = block_exclusive_scan(s, tmp, nbuckets);
    const uint32_t chunks = block_exclusive_scan(c, tmp, nbuckets);
    const uint32_t hchunks = block_exclusive_scan(hc, tmp, nbuckets);
    if (t < nbuckets) {
        start1[t] = s[t];
        uint32_t run = s[t];
        for (int r = 0; r < REPLICAS; ++r) {
            cursor1[r * MAX_DIGITS + t] = run;
            run += count1[r * MAX_DIGITS + t];
        }
        chunk_first[t] = c[t];
        hchunk_first[t] = hc[t];
    }
    if (t == 0) {
        start1[nbuckets] = total;
        if (nrec_out) *nrec_out = total;
        chunk_first[nbuckets] = chunks;
        hchunk_first[nbuckets] = hchunks;
    }
}

// Storage of the replica-major level-1 records, one workgroup per replica r:
// seg_v[b][r] = the bucket-major index where replica r's share of bucket b
// starts (cursor1's initial value), seg_p[b][r] = the storage slot where it is
// kept (the records of the replicas before r, then r's shares of the buckets
// before b).
__global__ void __launch_bounds__(MAX_DIGITS) l1_segs_kernel(const uint32_t *__restrict__ count1, int nbuckets,
                                                             const uint32_t *__restrict__ cursor1,
                                                             uint32_t *__restrict__ seg_v,
                                                             uint32_t *__restrict__ seg_p) {
    __shared__ uint32_t s[MAX_DIGITS], tmp[MAX_DIGITS];
    const int r = blockIdx.x, t = threadIdx.x;
    uint32_t before = 0;
    if (t < nbuckets)
        for (int q = 0; q < r; ++q) before += count1[q * MAX_DIGITS + t];
    s[t] = before;
    __syncthreads();
    const uint32_t rbase = block_exclusive_scan(s, tmp, nbuckets);
    s[t] = t < nbuckets ? count1[r * MAX_DIGITS + t] : 0u;
    __syncthreads();
    block_exclusive_scan(s, tmp, nbuckets);
    if (t < nbuckets) {
        seg_v[t * REPLICAS + r] = cursor1[r * MAX_DIGITS + t];
        seg_p[t * REPLICAS + r] = rbase + s[t];
    }
}

// Storage slot of bucket-major level-1 index i of a bucket whose segment
// starts sv[] / sp[] (per replica, in LDS) are given: the last replica whose
// share starts at or before i holds it (an empty share starts where the next
// one does, so the last of equal starts is the one that holds i).
__device__ __forceinline__ uint32_t seg_slot(const uint32_t *sv, const uint32_t *sp, uint32_t i) {
    int r = 0;
#pragma unroll
    for (int step = REPLICAS / 2; step > 0; step >>= 1)
        if (sv[r + step] <= i) r += step;
    return sp[r] + (i - sv[r]);
}
static_assert((REPLICAS & (REPLICAS - 1)) == 0, "the segment search halves a power of two");

// The indices [lo, hi) of one level-2 chunk: usually within one replica's
// share, whose storage offset then serves every record without a search.
struct SegRange {
    bool single;
    uint32_t shift;  // storage slot - index inside that share
};

__device__ __forceinline__ SegRange seg_range(const uint32_t *sv, const uint32_t *sp, uint32_t lo, uint32_t hi) {
    int r = 0;
#pragma unroll
    for (int step = REPLICAS / 2; step > 0; step >>= 1)
        if (sv[r + step] <= lo) r += step;
    return {r == REPLICAS - 1 || sv[r + 1] >= hi, sp[r] - sv[r]};
}

__device__ __forceinline__ uint32_t seg_slot(const uint32_t *sv, const uint32_t *sp, const SegRange &g,
                                             uint32_t i) {
    return g.single ? i + g.shift : seg_slot(sv, sp, i);
}

// Persistent: workgroup w takes the logical blocks w, w + G, w + 2G, ... of
// the replica mapping (G = gridDim.x, a multiple of NUM_XCD, so they all stay
// on one XCD).  Software-pipelined over two sets of bucket counts, offsets and
// cursor bases: while chunk c is written out from LDS, the positions of chunk
// c + 1 are converted, counted and scanned and its cursor atomics issued, so
// their latency hides behind c's stores; c + 1 is then staged without waiting.
template <typename T>
__global__ void __launch_bounds__(PART_THREADS) l1_scatter_kernel(const T *__restrict__ pos, int64_t np,
                                                                  FixedPoint<T> fp, Geom g, uint32_t *cursor1,
                                                                  const uint32_t *__restrict__ seg_v,
                                                                  const uint32_t *__restrict__ seg_p,
                                                                  Q3 *__restrict__ rec1, RunMaps maps) {
    __shared__ Q3 stage[CHUNK];
    __shared__ uint16_t sbk[CHUNK];
    __shared__ uint32_t h[2][MAX_DIGITS], off[2][MAX_DIGITS], gbase[2][MAX_DIGITS], gshift[2][MAX_DIGITS],
        tmp[MAX_DIGITS];
    static_assert(PART_PER == LBATCH, "one batch per scatter chunk");
    const uint32_t nchunks = uint32_t((np + CHUNK - 1) / CHUNK);
    const uint32_t logical = replica_grid(nchunks);
    auto next_chunk = [&](uint32_t &L) -> int64_t {
        for (; L < logical; L += gridDim.x) {
            const int64_t c = replica_chunk(L, nchunks);
            if (c >= 0) return c;
        }
        return -1;
    };
    uint32_t L = blockIdx.x;
    int64_t chunk = next_chunk(L);
    if (chunk < 0) return;  // the same for the whole workgroup
    RawBatch<T> raw;
    Q3 q[PART_PER];
    int bk[PART_PER];
    uint32_t rank[PART_PER];
    for (int b = threadIdx.x; b < MAX_DIGITS; b += blockDim.x) {
        h[0][b] = 0u;
        h[1][b] = 0u;
    }
    load_raw(pos, chunk * CHUNK + threadIdx.x, PART_THREADS, np, raw);
    __syncthreads();
    // chunk c from raw into set j (h[j] zeroed): bucket and rank of every
    // element, offsets, and the cursor bases (returned into gbase[j] later)
    auto prepare = [&](int64_t c, int j) -> uint32_t {
        bool ok[PART_PER];
        bool bad = false;  // reported by the histogram pass
        convert_raw(raw, c * CHUNK + threadIdx.x, PART_THREADS, np, fp, q, ok, bad);
#pragma unroll
        for (int k = 0; k < PART_PER; ++k) {
            bk[k] = -1;
            if (ok[k]) {
                bk[k] = bucket_of(g, q[k].x >> g.bits, q[k].y >> g.bits, q[k].z >> g.bits);
                rank[k] = atomicAdd(&h[j][bk[k]], 1u);
            }
        }
        __syncthreads();
        for (int b = threadIdx.x; b < g.nbuckets; b += blockDim.x) off[j][b] = h[j][b];
        __syncthreads();
        const uint32_t total = block_exclusive_scan(off[j], tmp, g.nbuckets);
        // the histogram pass counted this chunk under replica (c / HIST_CHUNKS) % REPLICAS
        const int rep = int((c / HIST_CHUNKS) % REPLICAS);
        uint32_t *mine = cursor1 + rep * MAX_DIGITS;
        for (int b = threadIdx.x; b < g.nbuckets; b += blockDim.x)
            if (h[j][b]) {
                gbase[j][b] = atomicAdd(&mine[b], h[j][b]);
                gshift[j][b] = seg_p[b * REPLICAS + rep] - seg_v[b * REPLICAS + rep];  // index -> storage slot
            }
        return total;
    };
    uint32_t total = prepare(chunk, 0);
    int j = 0;
    for (;;) {
        L += gridDim.x;
        const int64_t nxt = next_chunk(L);
        const int64_t base = chunk * CHUNK;
#pragma unroll
        for (int k = 0; k < PART_PER; ++k)
            if (bk[k] >= 0) {
                const uint32_t s = off[j][bk[k]] + rank[k];
                stage[s] = q[k];
                sbk[s] = uint16_t(bk[k]);
            }
        if (maps.pos) {
#pragma unroll
            for (int k = 0; k < PART_PER; ++k) {
                const int64_t i = base + k * PART_THREADS + threadIdx.x;
                if (i < np) maps.pos[i] = bk[k] >= 0 ? uint16_t(off[j][bk[k]] + rank[k]) : NO_POS;
            }
        }
        __syncthreads();  // staged, and gbase[j] is in
        if (nxt >= 0) load_raw(pos, nxt * CHUNK + threadIdx.x, PART_THREADS, np, raw);
        for (uint32_t s = threadIdx.x; s < total; s += PART_THREADS) {
            const int b = sbk[s];
            rec1[gbase[j][b] + gshift[j][b] + (s - off[j][b])] = stage[s];
        }
        if (maps.pos) save_run_table(maps, chunk, g.nbuckets, h[j], off[j], gbase[j], total);
        if (nxt < 0) break;
        // set j ^ 1 was last read by the previous chunk's write-out, which every
        // thread finished before the barrier above
        for (int b = threadIdx.x; b < MAX_DIGITS; b += blockDim.x) h[j ^ 1][b] = 0u;
        __syncthreads();
        total = prepare(nxt, j ^ 1);
        chunk = nxt;
        j ^= 1;
    }
}

// ---------------------------------------------------------------- level 2
// Input of level 2: either the level-1 records (FROM_REC) or, with a single
// bucket, the particle positions themselves.
template <typename T, bool FROM_REC>
struct L2Input {
    const T *pos;
    int64_t np;
    FixedPoint<T> fp;
    const Q3 *rec1;
    const uint32_t *seg_v, *seg_p;  // per (bucket, replica): where the level-1 records are kept
    const uint32_t *start1;
    const uint32_t *chunk_first;  // per-bucket chunk prefix for this kernel's chunk size
    int nbuckets;
    int chunk;                    // records per workgroup
};

// Level-2 chunk of this workgroup: XCD-contiguous, so neighbouring chunks of
// a bucket (whose runs share lines) go through one L2.
__device__ __forceinline__ uint32_t l2_chunk_index() { return xcd_remap(blockIdx.x, gridDim.x); }

// Locates this workgroup's chunk: bucket b and the index range [lo, hi).
template <typename T, bool FROM_REC>
__device__ __forceinline__ bool l2_chunk(const L2Input<T, FROM_REC> &in, int &b, int64_t &lo, int64_t &hi) {
    const uint32_t w = l2_chunk_index();
    if (!FROM_REC) {
        b = 0;
        lo = int64_t(w) * in.chunk;
        hi = lo + in.chunk < in.np ? lo + in.chunk : in.np;
        return lo < in.np;
    }
    if (w >= in.chunk_first[in.nbuckets]) return false;
    int L = 0, R = in.nbuckets - 1;  // last b with chunk_first[b] <= w
    while (L < R) {
        const int m = (L + R + 1) >> 1;
        if (in.chunk_first[m] <= w) L = m;
        else R = m - 1;
    }
    b = L;
    lo = int64_t(in.start1[b]) + int64_t(w - in.chunk_first[b]) * in.chunk;
    const int64_t end = in.start1[b + 1];
    hi = lo + in.chunk < end ? lo + in.chunk : end;
    return true;
}

// The segment starts of bucket b into LDS (the caller synchronises).
template <typename T, bool FROM_REC>
__device__ __forceinline__ void l2_segments(const L2Input<T, FROM_REC> &in, int b, uint32_t *sv, uint32_t *sp) {
    if (!FROM_REC) return;
    for (int r = threadIdx.x; r < REPLICAS; r += blockDim.x) {
        sv[r] = in.seg_v[b * REPLICAS + r];
        sp[r] = in.seg_p[b * REPLICAS + r];
    }
}

template <typename T, bool FROM_REC>
__global__ void __launch_bounds__(HIST_THREADS) l2_hist_kernel(L2Input<T, FROM_REC> in, Geom g, uint32_t *count2,
                                                               uint32_t *status) {
    __shared__ uint32_t h[MAX_DIGITS], sv[REPLICAS], sp[REPLICAS];
    int b;
    int64_t lo, hi;
    if (!l2_chunk(in, b, lo, hi)) return;
    for (int d = threadIdx.x; d < MAX_DIGITS; d += blockDim.x) h[d] = 0u;
    l2_segments(in, b, sv, sp);
    __syncthreads();
    const SegRange sg = FROM_REC ? seg_range(sv, sp, uint32_t(lo), uint32_t(hi)) : SegRange{true, 0u};
    bool bad = false;
    for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += HIST_THREADS * LBATCH) {
        Q3 q[LBATCH];
        bool ok[LBATCH];
        if (FROM_REC) {
#pragma unroll
            for (int k = 0; k < LBATCH; ++k) {
                const int64_t i = i0 + k * HIST_THREADS;
                ok[k] = i < hi;
                if (ok[k]) q[k] = in.rec1[seg_slot(sv, sp, sg, uint32_t(i))];
            }
        } else {
            load_q_batch(in.pos, i0, HIST_THREADS, hi, in.fp, q, ok, bad);
        }
#pragma unroll
        for (int k = 0; k < LBATCH; ++k)
            if (ok[k]) atomicAdd(&h[tile_in_bucket(g, q[k].x >> g.bits, q[k].y >> g.bits, q[k].z >> g.bits)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < g.digits; d += blockDim.x)
        if (h[d]) atomicAdd(&count2[int64_t(b) * g.digits + d], h[d]);
    if (bad) atomicOr(status, ST_INPUT);
}


// maps (optional, FROM_REC only) records where every level-1 record went.
template <typename T, bool FROM_REC>
__global__ void __launch_bounds__(PART_THREADS) l2_scatter_kernel(L2Input<T, FROM_REC> in, Geom g,
                                                                  uint32_t *cursor2, uint64_t *__restrict__ rec2,
                                                                  RunMaps maps) {
    __shared__ uint64_t stage[CHUNK];
    __shared__ uint16_t sdig[CHUNK];
    __shared__ uint32_t h[MAX_DIGITS], off[MAX_DIGITS], gbase[MAX_DIGITS], tmp[MAX_DIGITS], sv[REPLICAS],
        sp[REPLICAS];
    int b;
    int64_t lo, hi;
    if (!l2_chunk(in, b, lo, hi)) return;
    for (int d = threadIdx.x; d < MAX_DIGITS; d += blockDim.x) h[d] = 0u;
    l2_segments(in, b, sv, sp);
    __syncthreads();
    const SegRange sg = FROM_REC ? seg_range(sv, sp, uint32_t(lo), uint32_t(hi)) : SegRange{true, 0u};
    uint64_t r[PART_PER];
    int dg[PART_PER];
    uint32_t rank[PART_PER];
    Q3 q[PART_PER];
    bool ok[PART_PER];
    if (FROM_REC) {
#pragma unroll
        for (int k = 0; k < PART_PER; ++k) {
            const int64_t i = lo + k * PART_THREADS + threadIdx.x;
            ok[k] = i < hi;
            if (ok[k]) q[k] = in.rec1[seg_slot(sv, sp, sg, uint32_t(i))];
        }
    } else {
        bool bad = false;  // reported by the histogram pass
        load_q_batch(in.pos, lo + threadIdx.x, PART_THREADS, hi, in.fp, q, ok, bad);
    }
#pragma unroll
    for (int k = 0; k < PART_PER; ++k) {
        dg[k] = -1;
        if (ok[k]) {
            dg[k] = tile_in_bucket(g, q[k].x >> g.bits, q[k].y >> g.bits, q[k].z >> g.bits);
            r[k] = pack_local(g, q[k]);
            rank[k] = atomicAdd(&h[dg[k]], 1u);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < g.digits; d += blockDim.x) off[d] = h[d];
    __syncthreads();
    const uint32_t total = block_exclusive_scan(off, tmp, g.digits);
    for (int d = threadIdx.x; d < g.digits; d += blockDim.x)
        if (h[d]) gbase[d] = atomicAdd(&cursor2[int64_t(b) * g.digits + d], h[d]);
#pragma unroll
    for (int k = 0; k < PART_PER; ++k)
        if (dg[k] >= 0) {
            const uint32_t s = off[dg[k]] + rank[k];
            stage[s] = r[k];
            sdig[s] = uint16_t(dg[k]);
        }
    __syncthreads();
    const bool keep = FROM_REC && maps.pos;
    for (uint32_t s = threadIdx.x; s < total; s += PART_THREADS) {
        const int d = sdig[s];
        rec2[gbase[d] + (s - off[d])] = stage[s];
    }
    if (keep) {
        save_run_table(maps, l2_chunk_index(), g.digits, h, off, gbase, total);
#pragma unroll
        for (int k = 0; k < PART_PER; ++k)
            if (dg[k] >= 0) maps.pos[lo + k * PART_THREADS + threadIdx.x] = uint16_t(off[dg[k]] + rank[k]);
    }
}

// ---------------------------------------------------------------- accumulate and fold
__device__ __forceinline__ void tile_coords(const Geom &g, int b, int d, int &tx, int &ty, int &tz) {
    const int bx = b % g.nbx, by = (b / g.nbx) % g.nby, bz = b / (g.nbx * g.nby);
    const int ux = d % g.btx, uy = (d / g.btx) % g.bty, uz = d / (g.btx * g.bty);
    tx = bx * g.btx + ux;
    ty = by * g.bty + uy;
    tz = bz * g.btz + uz;
}

// CHECKED: returning atomic that reports the add carrying a cell past 2^63 - 1.
template <bool CHECKED>
__device__ __forceinline__ void lds_add(unsigned long long *acc, int c, unsigned long long w, bool &overflow) {
    if (CHECKED) {
        if (w == 0) return;
        const unsigned long long old = atomicAdd(acc + c, w);
        if (!(old >> 63) && ((old + w) >> 63)) overflow = true;
    } else {
        atomicAdd(acc + c, w);
    }
}

constexpr int ACC_RB = 8;  // records per thread loaded together

// The records lo + threadIdx.x + k * ACC_THREADS (k < ACC_RB) below hi of a tile.
__device__ __forceinline__ void load_records(const uint64_t *__restrict__ rec2, uint32_t i0, uint32_t hi,
                                             uint64_t (&rr)[ACC_RB]) {
#pragma unroll
    for (int k = 0; k < ACC_RB; ++k) {
        const uint32_t i = i0 + k * ACC_THREADS;
        rr[k] = i < hi ? rec2[i] : 0ull;
    }
}

// Adds the CIC weights of records [lo, hi) of a tile into acc; rr holds the
// first batch (load_records at lo + threadIdx.x) on entry.
template <bool CHECKED>
__device__ __forceinline__ void accumulate(const uint64_t *__restrict__ rec2, uint32_t lo, uint32_t hi, int bits,
                                           int ax, unsigned long long *acc, bool &overflow,
                                           uint64_t (&rr)[ACC_RB]) {
    const int sx = 6 + bits, sy = 3 + bits;
    const uint64_t fmask = (1ull << bits) - 1ull;
    const uint64_t mx = (1ull << sx) - 1ull, my = (1ull << sy) - 1ull;
    const uint64_t one = 1ull << bits;
    const int plane = ax * AYZ;
    constexpr int RB = ACC_RB;
    for (uint32_t i0 = lo + threadIdx.x; i0 < hi; i0 += ACC_THREADS * RB) {
        if (i0 != lo + threadIdx.x) load_records(rec2, i0, hi, rr);
#pragma unroll
        for (int k = 0; k < RB; ++k) {
        if (i0 + k * ACC_THREADS >= hi) break;
        const uint64_t r = rr[k];
        const uint64_t qx = r & mx, qy = (r >> sx) & my, qz = (r >> (sx + sy)) & my;
        const int cx = int(qx >> bits), cy = int(qy >> bits), cz = int(qz >> bits);
        const uint64_t fx = qx & fmask, fy = qy & fmask, fz = qz & fmask;
        const uint64_t wx0 = one - fx, wy0 = one - fy, wz0 = one - fz;
        const int c0 = (cz * AYZ + cy) * ax + cx;
        const uint64_t w00 = wz0 * wy0, w01 = wz0 * fy, w10 = fz * wy0, w11 = fz * fy;
        lds_add<CHECKED>(acc, c0, w00 * wx0, overflow);
        lds_add<CHECKED>(acc, c0 + 1, w00 * fx, overflow);
        lds_add<CHECKED>(acc, c0 + ax, w01 * wx0, overflow);
        lds_add<CHECKED>(acc, c0 + ax + 1, w01 * fx, overflow);
        lds_add<CHECKED>(acc, c0 + plane, w10 * wx0, overflow);
        lds_add<CHECKED>(acc, c0 + plane + 1, w10 * fx, overflow);
        lds_add<CHECKED>(acc, c0 + plane + ax, w11 * wx0, overflow);
        lds_add<CHECKED>(acc, c0 + plane + ax + 1, w11 * fx, overflow);
        }
    }
}

// Skirt cells of a tile, in side-buffer order: the y face (y = 8, x < tx, z in
// [0, 8]), then the z face (z = 8, x < tx, y < 8).  The x face (x = tx) is not
// stored: it is carried to the next tile of the row in LDS.
__device__ __forceinline__ void skirt_cell(int tx, int s, int &x, int &y, int &z) {
    const int fy = tx * AYZ;
    if (s < fy) {
        x = s % tx;
        y = TYZ;
        z = s / tx;
    } else {
        const int j = s - fy;
        x = j % tx;
        y = j / tx;
        z = TYZ;
    }
}

// Level-2 slot (bucket, tile in bucket) of the tile at tile coordinates (tx, ty, tz).
__device__ __forceinline__ int tile_slot(const Geom &g, int tx, int ty, int tz) {
    const int bx = tx / g.btx, by = ty / g.bty, bz = tz / g.btz;
    const int ux = tx - bx * g.btx, uy = ty - by * g.bty, uz = tz - bz * g.btz;
    return ((bz * g.nby + by) * g.nbx + bx) * g.digits + (uz * g.bty + uy) * g.btx + ux;
}

// One workgroup per row of tiles along x (fixed tile y and z), the tiles in
// order: each tile's particles are accumulated in LDS over the tile plus its
// +x/+y/+z skirt; the owned cells go to the grid, the y and z faces to the
// side buffer, and the x face (x = tx, all y and z in [0, 8]) stays in LDS as
// the x = 0 plane of the next tile, so no x face is ever folded through memory.
// The last tile's x face belongs to the first tile of the row (periodic): it
// is added to that tile's cells and side-buffer entries at the end.
__global__ void __launch_bounds__(ACC_THREADS) tile_accum_kernel(const uint64_t *__restrict__ rec2,
                                                                 const uint32_t *__restrict__ start2, Geom g,
                                                                 unsigned long long *__restrict__ rho,
                                                                 unsigned long long *__restrict__ skirt,
                                                                 uint32_t *status) {
    __shared__ unsigned long long acc[MAX_ACC_CELLS];
    int ty, tz;
    if (g.btx == g.ntx) {
        // rows of a bucket are whole rows: bucket-major row order, so each row's
        // records are one run of the level-2 order and neighbouring workgroups
        // read neighbouring runs
        const int rows = g.bty * g.btz, b = int(blockIdx.x) / rows, r = int(blockIdx.x) % rows;
        ty = ((b / g.nbx) % g.nby) * g.bty + r % g.bty;
        tz = (b / (g.nbx * g.nby)) * g.btz + r / g.bty;
    } else {
        ty = int(blockIdx.x) % g.nty;
        tz = int(blockIdx.x) / g.nty;
    }
    const int ax = g.tx + 1;
    const int ncells = ax * AYZ * AYZ;
    const size_t n = size_t(g.n);
    const size_t gy0 = size_t(ty) * TYZ, gz0 = size_t(tz) * TYZ;
    const int owned = g.tx * TYZ * TYZ;
    constexpr int FACE = AYZ * AYZ;  // cells of the x face
    bool overflow = false;
    uint32_t prev = 0;  // particles of the previous tile, whose x face is carried in
    // each tile's first batch of records is loaded before the previous tile
    // is written out, so that its latency hides behind the stores
    uint32_t lo = start2[tile_slot(g, 0, ty, tz)], hi = start2[tile_slot(g, 0, ty, tz) + 1];
    uint64_t rr[ACC_RB];
    load_records(rec2, lo + threadIdx.x, hi, rr);
    for (int tx = 0; tx < g.ntx; ++tx) {
        unsigned long long carried = 0ull;
        if (tx > 0 && threadIdx.x < FACE) carried = acc[threadIdx.x * ax + g.tx];  // (z, y) = (k / 9, k % 9)
        __syncthreads();
        for (int c = threadIdx.x; c < ncells; c += ACC_THREADS) acc[c] = 0ull;
        __syncthreads();
        if (tx > 0 && threadIdx.x < FACE) acc[threadIdx.x * ax] = carried;
        __syncthreads();
        // fewer than 2^(63 - 3B) particles (with those carried in) cannot carry
        // any cell of this tile past 2^63 - 1
        if (uint64_t(hi - lo) + prev < (1ull << (63 - 3 * g.bits)))
            accumulate<false>(rec2, lo, hi, g.bits, ax, acc, overflow, rr);
        else
            accumulate<true>(rec2, lo, hi, g.bits, ax, acc, overflow, rr);
        prev = hi - lo;
        if (tx + 1 < g.ntx) {
            const int next = tile_slot(g, tx + 1, ty, tz);
            lo = start2[next];
            hi = start2[next + 1];
            load_records(rec2, lo + threadIdx.x, hi, rr);
        }
        __syncthreads();
        const size_t gx0 = size_t(tx) * g.tx;
        for (int c = threadIdx.x; c < owned; c += ACC_THREADS) {
            const int x = c & (g.tx - 1), y = (c >> g.ltx) & (TYZ - 1), z = c >> (g.ltx + 3);
            rho[((gz0 + z) * n + gy0 + y) * n + gx0 + x] = acc[(z * AYZ + y) * ax + x];
        }
        const size_t tglob = (size_t(tz) * g.nty + ty) * g.ntx + tx;
        for (int k = threadIdx.x; k < g.skirt; k += ACC_THREADS) {
            int x, y, z;
            skirt_cell(g.tx, k, x, y, z);
            skirt[tglob * g.skirt + k] = acc[(z * AYZ + y) * ax + x];
        }
    }
    // the last x face onto the row's first tile (x = 0 there): its owned cells
    // in the grid, its y = 8 and z = 8 cells in the side buffer, all written by
    // this workgroup above (the barrier's workgroup-scope ordering makes them
    // visible here; a device-scope fence would write the L2 back)
    __syncthreads();
    if (threadIdx.x < FACE) {
        const int y = threadIdx.x % AYZ, z = threadIdx.x / AYZ;
        const unsigned long long w = acc[threadIdx.x * ax + g.tx];
        unsigned long long *at;
        if (y < TYZ && z < TYZ) {
            at = rho + ((gz0 + z) * n + gy0 + y) * n;
        } else {
            const size_t t0 = (size_t(tz) * g.nty + ty) * g.ntx;
            at = skirt + t0 * g.skirt + (y == TYZ ? z * g.tx : g.tx * AYZ + y * g.tx);
        }
        const unsigned long long v = *at, t = v + w;
        // both parts are below 2^63 unless already reported; the sum must be too
        if (t < v || (t >> 63)) overflow = true;
        *at = t;
    }
    if (overflow) atomicOr(status, ST_OVERFLOW);
}

// One workgroup per tile: its y = 0 and z = 0 cells (the z = 0 plane, then the
// y = 0 row of each plane z = 1..7: 15 tx cells, all in whole rows) gather the
// y- and z-face sums that the lower neighbours in y and z computed for them
// (the x faces were carried along the rows already).
__global__ void __launch_bounds__(ACC_THREADS) skirt_fold_kernel(const unsigned long long *__restrict__ skirt, Geom g,
                                                                 unsigned long long *__restrict__ rho,
                                                                 uint32_t *status) {
    const int t = blockIdx.x;
    const int tx = t % g.ntx, ty = (t / g.ntx) % g.nty, tz = t / (g.ntx * g.nty);
    const size_t n = size_t(g.n);
    const size_t gx0 = size_t(tx) * g.tx, gy0 = size_t(ty) * TYZ, gz0 = size_t(tz) * TYZ;
    const int sy = ty == 0 ? g.nty - 1 : ty - 1, sz = tz == 0 ? g.ntz - 1 : tz - 1;
    const size_t below_y = (size_t(tz) * g.nty + sy) * g.ntx + tx;   // tile - y
    const size_t below_z = (size_t(sz) * g.nty + ty) * g.ntx + tx;   // tile - z
    const size_t below_yz = (size_t(sz) * g.nty + sy) * g.ntx + tx;  // tile - y - z
    const int yface = g.tx * AYZ;  // start of the z face in a tile's side-buffer entries
    bool overflow = false;
    const int nface = 15 * g.tx;
    for (int k = threadIdx.x; k < nface; k += ACC_THREADS) {
        int x, y, z;
        if (k < 8 * g.tx) {
            z = 0;
            y = k >> g.ltx;
            x = k & (g.tx - 1);
        } else {
            const int j = k - 8 * g.tx;
            z = 1 + (j >> g.ltx);
            y = 0;
            x = j & (g.tx - 1);
        }
        const size_t at = ((gz0 + z) * n + gy0 + y) * n + gx0 + x;
        const unsigned long long v = rho[at];
        unsigned long long lo = 0ull, hi = 0ull;
        auto add = [&](unsigned long long w) {
            const unsigned long long s = lo + w;
            hi += s < w;
            lo = s;
        };
        if (z == 0) add(skirt[below_z * g.skirt + yface + y * g.tx + x]);            // (x, y, 8) of tile - z
        if (y == 0) add(skirt[below_y * g.skirt + z * g.tx + x]);                    // (x, 8, z) of tile - y
        if (y == 0 && z == 0) add(skirt[below_yz * g.skirt + TYZ * g.tx + x]);       // (x, 8, 8) of tile - y - z
        // every part is below 2^63 unless already reported; the total must be too
        const unsigned long long s = lo + v;
        hi += s < v;
        if (hi != 0 || (s >> 63)) overflow = true;
        rho[at] = s;
    }
    if (overflow) atomicOr(status, ST_OVERFLOW);
}

// ---------------------------------------------------------------- step 6 through the particle order
// Pass 1, one workgroup per tile in level-2 order: the cell labels of the tile
// and its +x/+y/+z skirt go to LDS; record k takes the label of its nearest
// node, lab2[k].  A tile-local node is ((q_local + 2^(B-1)) >> B) per axis,
// at most one cell past the tile, which the skirt holds.
//
// With COUNT, each label's particles are also counted into parts[label] (the
// group statistics of steps 5 and 7): a tile's records carry a few dozen
// labels at most, counted in an LDS table and added to parts once per tile.
// The record loop then runs whole sweeps on every thread, so that all lanes
// take part in each wavefront step of the count.
template <bool COUNT>
__global__ void __launch_bounds__(ACC_THREADS) tile_label_kernel(const uint64_t *__restrict__ rec2,
                                                                 const uint32_t *__restrict__ start2, Geom g,
                                                                 const int32_t *__restrict__ cell_label,
                                                                 int32_t *__restrict__ lab2,
                                                                 uint32_t *__restrict__ parts) {
    __shared__ int32_t lab[MAX_ACC_CELLS];
    const int slot = int(xcd_remap(blockIdx.x, gridDim.x));  // neighbouring tiles share skirt lines
    const int b = slot / g.digits, d = slot % g.digits;
    int tx, ty, tz;
    tile_coords(g, b, d, tx, ty, tz);
    const int ax = g.tx + 1;
    const int ncells = ax * AYZ * AYZ;
    const uint32_t n = uint32_t(g.n);
    const uint32_t gx0 = uint32_t(tx) * g.tx, gy0 = uint32_t(ty) * TYZ, gz0 = uint32_t(tz) * TYZ;
    for (int c = threadIdx.x; c < ncells; c += ACC_THREADS) {
        const int x = c % ax, y = (c / ax) % AYZ, z = c / (ax * AYZ);
        uint32_t gx = gx0 + x, gy = gy0 + y, gz = gz0 + z;
        if (gx >= n) gx -= n;
        if (gy >= n) gy -= n;
        if (gz >= n) gz -= n;
        lab[c] = cell_label[(gz * n + gy) * n + gx];
    }
    __syncthreads();
    const int bits = g.bits, sx = 6 + bits, sy = 3 + bits;
    const uint64_t mx = (1ull << sx) - 1ull, my = (1ull << sy) - 1ull;
    const uint64_t half = 1ull << (bits - 1);
    const uint32_t lo = start2[slot], hi = start2[slot + 1];
    constexpr int RB = 8;
    auto node_label = [&](uint64_t r) {
        const int nx = int(((r & mx) + half) >> bits);
        const int ny = int((((r >> sx) & my) + half) >> bits);
        const int nz = int((((r >> (sx + sy)) & my) + half) >> bits);
        return lab[(nz * AYZ + ny) * ax + nx];
    };
    if constexpr (!COUNT) {
        for (uint32_t i0 = lo + threadIdx.x; i0 < hi; i0 += ACC_THREADS * RB) {
            uint64_t rr[RB];
#pragma unroll
            for (int k = 0; k < RB; ++k) {
                const uint32_t i = i0 + k * ACC_THREADS;
                rr[k] = i < hi ? rec2[i] : 0ull;
            }
#pragma unroll
            for (int k = 0; k < RB; ++k) {
                const uint32_t i = i0 + k * ACC_THREADS;
                if (i >= hi) break;
                lab2[i] = node_label(rr[k]);
            }
        }
    } else {
        constexpr int HT = 256;
        __shared__ int32_t hkey[HT];
        __shared__ uint32_t hcnt[HT];
        lds_tally_init<HT>(hkey, hcnt);
        __syncthreads();
        for (uint32_t b0 = lo; b0 < hi; b0 += ACC_THREADS * RB) {
            const uint32_t i0 = b0 + threadIdx.x;
            uint64_t rr[RB];
#pragma unroll
            for (int k = 0; k < RB; ++k) {
                const uint32_t i = i0 + k * ACC_THREADS;
                rr[k] = i < hi ? rec2[i] : 0ull;
            }
#pragma unroll
            for (int k = 0; k < RB; ++k) {
                const uint32_t i = i0 + k * ACC_THREADS;
                int32_t l = -1;
                if (i < hi) {
                    l = node_label(rr[k]);
                    lab2[i] = l;
                }
                lds_tally_wave<HT>(hkey, hcnt, parts, l);
            }
        }
        __syncthreads();
        lds_tally_flush<HT>(hkey, hcnt, parts);
    }
}

// Destination of the staging positions k * PART_THREADS + threadIdx.x of a
// chunk, from its run offsets: each nonempty run's first position is marked
// with its destination, and an inclusive max-scan over the positions carries
// every mark over its run (runs are in destination order).  mark holds CHUNK
// words and is free again on return.
__device__ void slot_dest(const uint16_t *off_s, int ndest, uint32_t *mark, uint16_t (&dd)[PART_PER]) {
    __shared__ uint32_t wmax[PART_THREADS / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int j = 0; j < PART_PER; ++j) mark[t * PART_PER + j] = 0u;
    __syncthreads();
    for (int d = t; d < ndest; d += PART_THREADS)
        if (off_s[d + 1] > off_s[d]) mark[off_s[d]] = uint32_t(d);
    __syncthreads();
    // this thread's PART_PER consecutive positions, then the threads before it
    uint32_t v[PART_PER], run = 0u;
#pragma unroll
    for (int j = 0; j < PART_PER; ++j) {
        run = max(run, mark[t * PART_PER + j]);
        v[j] = run;
    }
    uint32_t incl = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl = max(incl, y);
    }
    if (lane == 63) wmax[wave] = incl;
    const uint32_t prev = __shfl_up(incl, 1, 64);
    __syncthreads();
    uint32_t before = lane > 0 ? prev : 0u;
    for (int w = 0; w < wave; ++w) before = max(before, wmax[w]);
#pragma unroll
    for (int j = 0; j < PART_PER; ++j) mark[t * PART_PER + j] = max(v[j], before);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PART_PER; ++k) dd[k] = uint16_t(mark[k * PART_THREADS + t]);
    __syncthreads();
}

// One scatter chunk back to element order: dst[e] = src[slot of element e]
// for the chunk's elements [e0, e1).  The chunk's runs are read into LDS in
// staging order, consecutive lanes on consecutive slots of a run, so a
// wavefront touches a few lines instead of one line per lane; element e then
// takes the value at its staging position.  Rejected elements get -1.  With
// FILTER, a label l >= 0 whose keep[l] is 0 becomes -1 (the group filter of
// step 7; labels of a chunk's runs are few, so these reads stay in cache).
// With CLAIM, the elements' labels also claim them as ClaimOut describes;
// with TCLAIM, the source slots' claim state is tested and advanced as
// TileClaim describes (FILTER is then on).
template <bool FILTER, bool CLAIM = false, bool TCLAIM = false>
__device__ void chunk_gather(const RunMaps &m, int64_t chunk, int ndest, int64_t e0, int64_t e1,
                             const int32_t *__restrict__ src, int32_t *__restrict__ dst,
                             const uint32_t *__restrict__ keep, const ClaimOut &claim = ClaimOut{},
                             const TileClaim &tc = TileClaim{}) {
    __shared__ uint32_t base_s[MAX_DIGITS];
    __shared__ uint16_t off_s[OFF_STRIDE];
    __shared__ int32_t val[CHUNK];
    static_assert(CHUNK == PART_THREADS * PART_PER, "one staging position per thread and slot");
    for (int d = threadIdx.x; d < ndest; d += blockDim.x) base_s[d] = m.base[chunk * MAX_DIGITS + d];
    for (int d = threadIdx.x; d <= ndest; d += blockDim.x) off_s[d] = m.offset[chunk * OFF_STRIDE + d];
    uint16_t p[PART_PER], dd[PART_PER];
#pragma unroll
    for (int k = 0; k < PART_PER; ++k) {
        const int64_t e = e0 + k * PART_THREADS + threadIdx.x;
        p[k] = e < e1 ? m.pos[e] : NO_POS;
    }
    __syncthreads();
    slot_dest(off_s, ndest, reinterpret_cast<uint32_t *>(val), dd);
    const uint32_t total = off_s[ndest];
    int32_t v[PART_PER];
#pragma unroll
    for (int k = 0; k < PART_PER; ++k) {
        const uint32_t s = k * PART_THREADS + threadIdx.x;
        if (s < total) {
            const int d = dd[k];
            const uint32_t at = base_s[d] + (s - off_s[d]);
            v[k] = src[at];
            if (TCLAIM) {
                const bool open = tc.first || tc.cs[at] == 0;
                if (!open || !tc.any || (v[k] >= 0 && !keep[v[k]])) v[k] = -1;
                if (tc.first) tc.cs[at] = v[k] >= 0 ? 1 : 0;
                else if (v[k] >= 0) tc.cs[at] = 1;
            } else if (FILTER && v[k] >= 0 && !keep[v[k]]) {
                v[k] = -1;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < PART_PER; ++k) {
        const uint32_t s = k * PART_THREADS + threadIdx.x;
        if (s < total) val[s] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PART_PER; ++k) {
        const int64_t e = e0 + k * PART_THREADS + threadIdx.x;
        if (e >= e1) continue;
        const int32_t l = p[k] < total ? val[p[k]] : -1;
        dst[e] = l;
        if (CLAIM && (claim.first || l >= 0)) {
            claim.halo_scale[e] = l >= 0 ? claim.scale : -1;
            claim.halo_root[e] = l;
        }
    }
}

// Pass 2, level-1 order: lab1[j] = lab2[level-2 slot of record j], one
// workgroup per level-2 scatter chunk (CHUNK records of one bucket); with
// FILTER, labels of disposed groups (keep[label] == 0) become -1; with
// TCLAIM, also those of particles claimed before, and the rest claim theirs.
template <bool FILTER, bool TCLAIM>
__global__ void __launch_bounds__(PART_THREADS) to_level1_kernel(RunMaps m2, const uint32_t *__restrict__ start1,
                                                                 const uint32_t *__restrict__ chunk_first,
                                                                 int nbuckets, int digits,
                                                                 const int32_t *__restrict__ lab2,
                                                                 int32_t *__restrict__ lab1,
                                                                 const uint32_t *__restrict__ keep, TileClaim tc) {
    const uint32_t w = xcd_remap(blockIdx.x, gridDim.x);  // as the level-2 scatter placed them
    if (w >= chunk_first[nbuckets]) return;
    int L = 0, R = nbuckets - 1;  // last b with chunk_first[b] <= w
    while (L < R) {
        const int mid = (L + R + 1) >> 1;
        if (chunk_first[mid] <= w) L = mid;
        else R = mid - 1;
    }
    const int b = L;
    const int64_t lo = int64_t(start1[b]) + int64_t(w - chunk_first[b]) * CHUNK;
    const int64_t end = start1[b + 1];
    const int64_t hi = lo + CHUNK < end ? lo + CHUNK : end;
    chunk_gather<FILTER, false, TCLAIM>(m2, w, digits, lo, hi, lab2, lab1, keep, ClaimOut{}, tc);
}

// Pass 3, input order: particle i -> lab1[level-1 slot of i], one workgroup
// per level-1 scatter chunk; with CLAIM the labels also claim their particles.
template <bool CLAIM>
__global__ void __launch_bounds__(PART_THREADS) to_input_kernel(RunMaps m1, int64_t np, int nbuckets,
                                                                const int32_t *__restrict__ lab1,
                                                                int32_t *__restrict__ out, ClaimOut claim) {
    // the level-1 scatter's chunk order: each XCD reads the runs of the counter
    // replicas it wrote, in the order it wrote them, so runs sharing lines meet in one L2
    const int64_t chunk = replica_chunk(blockIdx.x, unsigned((np + CHUNK - 1) / CHUNK));
    if (chunk < 0) return;
    const int64_t e0 = chunk * CHUNK;
    const int64_t e1 = e0 + CHUNK < np ? e0 + CHUNK : np;
    chunk_gather<false, CLAIM>(m1, chunk, nbuckets, e0, e1, lab1, out, nullptr, claim);
}

// ---------------------------------------------------------------- host side
// Tile and bucket shape for an n^3 grid; false if the binned form cannot hold it
// (at most MAX_DIGITS tiles per bucket and MAX_DIGITS buckets).
bool make_geom(const hf_box &box, Geom &out) {
    Geom g{};
    g.n = box.n;
    g.bits = box.frac_bits;
    g.tx = box.n % 64 == 0 ? 64 : (box.n % 32 == 0 ? 32 : 16);
    g.ltx = g.tx == 64 ? 6 : (g.tx == 32 ? 5 : 4);
    if (box.n % g.tx != 0 || box.n % TYZ != 0) return false;
    g.ntx = box.n / g.tx;
    g.nty = g.ntz = box.n / TYZ;
    g.ntiles = g.ntx * g.nty * g.ntz;
    g.skirt = g.tx * AYZ + g.tx * TYZ;  // y and z faces
    // buckets of whole rows of tiles along x where that fits (the accumulation
    // walks each row in order), then the fewest buckets, then the most
    // cube-like bucket
    long best_nb = -1;
    double best_shape = 0.0;
    auto search = [&](int bx_from) {
        for (int bx = bx_from; bx <= g.ntx; ++bx) {
            if (g.ntx % bx) continue;
            for (int by = 1; by <= g.nty; ++by) {
                if (g.nty % by) continue;
                for (int bz = 1; bz <= g.ntz; ++bz) {
                    if (g.ntz % bz || long(bx) * by * bz > MAX_DIGITS) continue;
                    const long nb = long(g.ntx / bx) * (g.nty / by) * (g.ntz / bz);
                    if (nb > MAX_DIGITS) continue;
                    const double ex = double(bx) * g.tx, ey = double(by) * TYZ, ez = double(bz) * TYZ;
                    const double hi = ex > ey ? (ex > ez ? ex : ez) : (ey > ez ? ey : ez);
                    const double lo = ex < ey ? (ex < ez ? ex : ez) : (ey < ez ? ey : ez);
                    const double shape = hi / lo;
                    if (best_nb < 0 || nb < best_nb || (nb == best_nb && shape < best_shape)) {
                        best_nb = nb;
                        best_shape = shape;
                        g.btx = bx;
                        g.bty = by;
                        g.btz = bz;
                    }
                }
            }
        }
    };
    search(g.ntx);               // whole rows
    if (best_nb < 0) search(1);  // else any shape
    if (best_nb < 0) return false;
    g.nbx = g.ntx / g.btx;
    g.nby = g.nty / g.bty;
    g.nbz = g.ntz / g.btz;
    g.nbuckets = g.nbx * g.nby * g.nbz;
    g.digits = g.btx * g.bty * g.btz;
    g.cbx = FastDiv(uint32_t(g.btx * g.tx));
    g.cby = FastDiv(uint32_t(g.bty * TYZ));
    g.cbz = FastDiv(uint32_t(g.btz * TYZ));
    g.tbx = FastDiv(uint32_t(g.btx));
    g.tby = FastDiv(uint32_t(g.bty));
    g.tbz = FastDiv(uint32_t(g.btz));
    out = g;
    return true;
}

struct DepLayout {
    size_t count1, start1, cursor1, seg_v, seg_p, chunk_first, hchunk_first, count2, start2, cursor2, partial, rec1,
        rec2, skirt, pad, total;
};

// Grid the binned form runs on for an n^3 box: n itself when its tiles fit
// (n a multiple of 16), else the next multiple of 16 above n.  On the larger
// grid the particles (cells 0..n-1) fill the low corner, their upper CIC
// corners reach cell n at most, and a last pass folds the planes at n onto
// the planes at 0 along each axis and keeps the n^3 cells.
int padded_n(int n) { return n % 16 == 0 ? n : (n + 1 + 15) / 16 * 16; }

hf_box padded_box(const hf_box &box) {
    hf_box b = box;
    b.n = padded_n(box.n);
    return b;
}

// rho[x, y, z] of the n^3 grid = the sum over the cells of the padded grid
// (side np) that coincide with it periodically: x and x + n where x = 0, and
// the same in y and z.  Exact, with the 2^63 check.
__global__ void crop_fold_kernel(const unsigned long long *__restrict__ pad, int npad, int n,
                                 unsigned long long *__restrict__ rho, uint32_t *status) {
    const int64_t cells = int64_t(n) * n * n;
    const size_t sp = size_t(npad);
    bool overflow = false;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < cells; i += int64_t(gridDim.x) * blockDim.x) {
        const int x = int(i % n), y = int((i / n) % n), z = int(i / (int64_t(n) * n));
        unsigned long long lo = 0ull, hi = 0ull;
        for (int dz = 0; dz <= (z == 0); ++dz)
            for (int dy = 0; dy <= (y == 0); ++dy)
                for (int dx = 0; dx <= (x == 0); ++dx) {
                    const unsigned long long w =
                        pad[(size_t(z + dz * n) * sp + size_t(y + dy * n)) * sp + size_t(x + dx * n)];
                    const unsigned long long t = lo + w;
                    hi += t < w;
                    lo = t;
                }
        if (hi != 0 || (lo >> 63)) overflow = true;
        rho[i] = lo;
    }
    if (overflow) atomicOr(status, ST_OVERFLOW);
}

// Deposit workspace; with keep_order the level-2 records and the bucket and
// tile offsets live in the ParticleOrder region instead.
DepLayout dep_layout(const Geom &g, int64_t np, bool keep_order, bool padded = false) {
    DepLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.count1 = take(sizeof(uint32_t) * MAX_DIGITS * REPLICAS);
    L.count2 = take(sizeof(uint32_t) * size_t(g.ntiles));
    L.start1 = take(keep_order ? 0 : sizeof(uint32_t) * (MAX_DIGITS + 1));
    L.cursor1 = take(sizeof(uint32_t) * MAX_DIGITS * REPLICAS);
    L.seg_v = take(sizeof(uint32_t) * MAX_DIGITS * REPLICAS);
    L.seg_p = take(sizeof(uint32_t) * MAX_DIGITS * REPLICAS);
    L.chunk_first = take(keep_order ? 0 : sizeof(uint32_t) * (MAX_DIGITS + 1));
    L.hchunk_first = take(sizeof(uint32_t) * (MAX_DIGITS + 1));
    L.start2 = take(keep_order ? 0 : sizeof(uint32_t) * (size_t(g.ntiles) + 1));
    L.cursor2 = take(sizeof(uint32_t) * size_t(g.ntiles));
    L.partial = take(sizeof(uint64_t) * SCAN_MAX_GROUPS);
    L.rec1 = take(g.nbuckets > 1 ? sizeof(Q3) * size_t(np) : 0);
    L.rec2 = take(keep_order ? 0 : sizeof(uint64_t) * size_t(np));
    L.skirt = take(sizeof(unsigned long long) * size_t(g.skirt) * size_t(g.ntiles));
    L.pad = take(padded ? sizeof(unsigned long long) * size_t(g.n) * size_t(g.n) * size_t(g.n) : 0);
    L.total = off;
    return L;
}

// ParticleOrder region: rec2 [np] | start2 [ntiles + 1] | nrec | start1 [513] |
// chunk_first [513] | the run maps of both levels (about 12.5 bytes per
// particle in all).
struct OrderLayout {
    size_t rec2, start2, nrec, start1, chunk_first, total;
    size_t pos[2], base[2], offset[2];
};

OrderLayout order_layout(const Geom &g, int64_t np) {
    OrderLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.rec2 = take(sizeof(uint64_t) * size_t(np));
    L.start2 = take(sizeof(uint32_t) * (size_t(g.ntiles) + 1));
    L.nrec = take(sizeof(uint32_t));
    L.start1 = take(sizeof(uint32_t) * (MAX_DIGITS + 1));
    L.chunk_first = take(sizeof(uint32_t) * (MAX_DIGITS + 1));
    const size_t chunks1 = (size_t(np) + CHUNK - 1) / CHUNK;
    const size_t chunks[2] = {chunks1, chunks1 + size_t(g.nbuckets)};  // level 2: one partial chunk per bucket
    for (int l = 0; l < 2; ++l) {
        L.pos[l] = take(sizeof(uint16_t) * size_t(np));
        L.base[l] = take(sizeof(uint32_t) * chunks[l] * MAX_DIGITS);
        L.offset[l] = take(sizeof(uint16_t) * chunks[l] * OFF_STRIDE);
    }
    L.total = off;
    return L;
}

// Workgroups of the persistent level-1 scatter: as many as are resident at once
// (a multiple of NUM_XCD), but no more than the blocks of work.
unsigned resident_grid(const hf_ctx *ctx, const void *kernel, unsigned blocks) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, PART_THREADS, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    unsigned g = unsigned(per_cu) * unsigned(ctx->cus) / NUM_XCD * NUM_XCD;
    if (g < NUM_XCD) g = NUM_XCD;
    const unsigned need = (blocks + NUM_XCD - 1) / NUM_XCD * NUM_XCD;
    return g < need ? g : need;
}

template <typename T>
hf_status run_tiled(hf_ctx *ctx, const hf_box &box, const T *pos, int64_t np, unsigned long long *rho_out,
                    char *ws, const ParticleOrder *order) {
    Geom g;  // on the padded grid where n is not a multiple of 16; the fixed point is the box's own
    const bool padded = padded_n(box.n) != box.n;
    if (!make_geom(padded_box(box), g)) return HF_ERR_SIZE;
    if (order && (g.nbuckets < 2 || padded)) return HF_ERR_ARG;  // no level-1 records to keep
    const DepLayout L = dep_layout(g, np, order != nullptr, padded);
    auto *rho = padded ? reinterpret_cast<unsigned long long *>(ws + L.pad) : rho_out;
    auto *count1 = reinterpret_cast<uint32_t *>(ws + L.count1);
    auto *count2 = reinterpret_cast<uint32_t *>(ws + L.count2);
    auto *start1 = order ? order->start1 : reinterpret_cast<uint32_t *>(ws + L.start1);
    auto *cursor1 = reinterpret_cast<uint32_t *>(ws + L.cursor1);
    auto *seg_v = reinterpret_cast<uint32_t *>(ws + L.seg_v);
    auto *seg_p = reinterpret_cast<uint32_t *>(ws + L.seg_p);
    auto *chunk_first = order ? order->chunk_first : reinterpret_cast<uint32_t *>(ws + L.chunk_first);
    auto *hchunk_first = reinterpret_cast<uint32_t *>(ws + L.hchunk_first);
    auto *start2 = order ? order->start2 : reinterpret_cast<uint32_t *>(ws + L.start2);
    auto *cursor2 = reinterpret_cast<uint32_t *>(ws + L.cursor2);
    auto *partial = reinterpret_cast<uint64_t *>(ws + L.partial);
    // start2 / cursor2 = exclusive scan of the per-tile counts (bucket-major order)
    const ScanJob tile_scan = scan_job(count2, g.ntiles, partial, start2, cursor2);
    auto *rec1 = reinterpret_cast<Q3 *>(ws + L.rec1);
    auto *rec2 = order ? order->rec2 : reinterpret_cast<uint64_t *>(ws + L.rec2);
    auto *skirt = reinterpret_cast<unsigned long long *>(ws + L.skirt);
    RunMaps m1{}, m2{};
    if (order) {
        __builtin_memcpy(&m1, order->maps[0], sizeof(m1));
        __builtin_memcpy(&m2, order->maps[1], sizeof(m2));
    }
    uint32_t *nrec = order ? order->nrec : nullptr;
    hipStream_t st = ctx->stream;
    const FixedPoint<T> fp = make_fixed_point<T>(box);
    HF_LAUNCH(ctx, K_DEP_PREP, zero_u32_kernel, dim3(64), dim3(256), 0, st, count1, int64_t(MAX_DIGITS * REPLICAS));
    HF_LAUNCH(ctx, K_DEP_PREP, zero_u32_kernel, dim3(64), dim3(256), 0, st, count2, int64_t(g.ntiles));
    const unsigned part_blocks = unsigned((np + CHUNK - 1) / CHUNK);
    const unsigned hist_blocks = unsigned((np + HCHUNK - 1) / HCHUNK);
    if (g.nbuckets > 1) {
        if (hist_blocks)
            HF_LAUNCH(ctx, K_DEP_L1_HIST, l1_hist_kernel<T>, dim3(hist_blocks), dim3(HIST_THREADS), 0, st, pos, np,
                      fp, g, count1, ctx->d_status);
        HF_LAUNCH(ctx, K_DEP_PREP, l1_scan_kernel, dim3(1), dim3(MAX_DIGITS), 0, st, count1, g.nbuckets, start1,
                  cursor1, chunk_first, hchunk_first, nrec);
        HF_LAUNCH(ctx, K_DEP_PREP, l1_segs_kernel, dim3(REPLICAS), dim3(MAX_DIGITS), 0, st, count1, g.nbuckets,
                  cursor1, seg_v, seg_p);
        if (part_blocks)
            HF_LAUNCH(ctx, K_DEP_L1_SCATTER, l1_scatter_kernel<T>,
                      dim3(resident_grid(ctx, reinterpret_cast<const void *>(&l1_scatter_kernel<T>),
                                         replica_grid(part_blocks))),
                      dim3(PART_THREADS), 0, st, pos, np, fp, g, cursor1, seg_v, seg_p, rec1, m1);
        const L2Input<T, true> hin{pos, np, fp, rec1, seg_v, seg_p, start1, hchunk_first, g.nbuckets, HCHUNK};
        const L2Input<T, true> sin{pos, np, fp, rec1, seg_v, seg_p, start1, chunk_first, g.nbuckets, CHUNK};
        HF_LAUNCH(ctx, K_DEP_L2_HIST, (l2_hist_kernel<T, true>), dim3(hist_blocks + unsigned(g.nbuckets)),
                  dim3(HIST_THREADS), 0, st, hin, g, count2, ctx->d_status);
        HF_LAUNCH(ctx, K_DEP_PREP, seg_reduce_kernel<SCAN_TILES>, dim3(scan_groups(tile_scan)), dim3(SCAN_THREADS),
                  0, st, tile_scan);
        HF_LAUNCH(ctx, K_DEP_PREP, seg_scan_kernel<SCAN_TILES>, dim3(scan_groups(tile_scan)), dim3(SCAN_THREADS), 0,
                  st, tile_scan);
        HF_LAUNCH(ctx, K_DEP_L2_SCATTER, (l2_scatter_kernel<T, true>), dim3(part_blocks + unsigned(g.nbuckets)),
                  dim3(PART_THREADS), 0, st, sin, g, cursor2, rec2, m2);
    } else {
        const L2Input<T, false> hin{pos, np, fp, nullptr, nullptr, nullptr, nullptr, nullptr, 1, HCHUNK};
        const L2Input<T, false> sin{pos, np, fp, nullptr, nullptr, nullptr, nullptr, nullptr, 1, CHUNK};
        if (hist_blocks)
            HF_LAUNCH(ctx, K_DEP_L2_HIST, (l2_hist_kernel<T, false>), dim3(hist_blocks), dim3(HIST_THREADS), 0, st,
                      hin, g, count2, ctx->d_status);
        HF_LAUNCH(ctx, K_DEP_PREP, seg_reduce_kernel<SCAN_TILES>, dim3(scan_groups(tile_scan)), dim3(SCAN_THREADS),
                  0, st, tile_scan);
        HF_LAUNCH(ctx, K_DEP_PREP, seg_scan_kernel<SCAN_TILES>, dim3(scan_groups(tile_scan)), dim3(SCAN_THREADS), 0,
                  st, tile_scan);
        if (part_blocks)
            HF_LAUNCH(ctx, K_DEP_L2_SCATTER, (l2_scatter_kernel<T, false>), dim3(part_blocks), dim3(PART_THREADS),
                      0, st, sin, g, cursor2, rec2, RunMaps{});
    }
    HF_LAUNCH(ctx, K_DEPOSIT, tile_accum_kernel, dim3(g.nty * g.ntz), dim3(ACC_THREADS), 0, st, rec2, start2, g, rho,
              skirt, ctx->d_status);
    HF_LAUNCH(ctx, K_DEP_FOLD, skirt_fold_kernel, dim3(g.ntiles), dim3(ACC_THREADS), 0, st, skirt, g, rho,
              ctx->d_status);
    if (padded) {
        const int64_t cells = int64_t(box.n) * box.n * box.n;
        const int64_t want = (cells + 255) / 256, cap = int64_t(ctx->cus) * 16;
        HF_LAUNCH(ctx, K_DEP_FOLD, crop_fold_kernel, dim3(unsigned(want < cap ? want : cap)), dim3(256), 0, st, rho,
                  g.n, box.n, rho_out, ctx->d_status);
    }
    return launch_status();
}

}  // namespace

bool hf::deposit_tiled_supported(const hf_box &box, int64_t np) {
    // packed tile records hold 12 + 3B <= 63 bits; counts are uint32
    if (box.frac_bits > 17 || np >= (int64_t(1) << 32)) return false;
    Geom g;
    return make_geom(padded_box(box), g);
}

size_t hf::deposit_tiled_ws_bytes(const hf_box &box, int64_t np, bool keep_order) {
    Geom g;
    const bool padded = padded_n(box.n) != box.n;
    return make_geom(padded_box(box), g) ? dep_layout(g, np, keep_order, padded).total : 0;
}

hf_status hf::deposit_tiled(hf_ctx *ctx, const hf_box &box, const void *pos, hf_dtype dtype, int64_t np,
                            int64_t *rho, void *ws, const ParticleOrder *order) {
    auto *grid = reinterpret_cast<unsigned long long *>(rho);
    char *w = static_cast<char *>(ws);
    if (dtype == HF_F32) return run_tiled<float>(ctx, box, static_cast<const float *>(pos), np, grid, w, order);
    return run_tiled<double>(ctx, box, static_cast<const double *>(pos), np, grid, w, order);
}

bool hf::particle_order_supported(const hf_box &box, int64_t np) {
    Geom g;
    return np > 0 && deposit_tiled_supported(box, np) && make_geom(box, g) && g.nbuckets > 1;
}

size_t hf::particle_order_bytes(const hf_box &box, int64_t np) {
    Geom g;
    return make_geom(box, g) ? order_layout(g, np).total : 0;
}

hf::ParticleOrder hf::particle_order_at(const hf_box &box, void *base, int64_t np) {
    Geom g;
    ParticleOrder o{};
    if (!make_geom(box, g)) return o;
    const OrderLayout L = order_layout(g, np);
    char *p = static_cast<char *>(base);
    o.rec2 = reinterpret_cast<uint64_t *>(p + L.rec2);
    o.start2 = reinterpret_cast<uint32_t *>(p + L.start2);
    o.nrec = reinterpret_cast<uint32_t *>(p + L.nrec);
    o.start1 = reinterpret_cast<uint32_t *>(p + L.start1);
    o.chunk_first = reinterpret_cast<uint32_t *>(p + L.chunk_first);
    static_assert(sizeof(RunMaps) <= sizeof(o.maps[0]), "run maps fit the opaque slots");
    for (int l = 0; l < 2; ++l) {
        const RunMaps m{reinterpret_cast<uint16_t *>(p + L.pos[l]), reinterpret_cast<uint32_t *>(p + L.base[l]),
                        reinterpret_cast<uint16_t *>(p + L.offset[l])};
        __builtin_memcpy(o.maps[l], &m, sizeof(m));
    }
    return o;
}

size_t hf::label_scratch_bytes(int64_t np) { return 2 * align_up(sizeof(int32_t) * size_t(np)); }

hf_status hf::label_tiles(hf_ctx *ctx, const hf_box &box, int64_t np, const ParticleOrder &order,
                          const int32_t *cell_label, void *scratch, uint32_t *parts) {
    if (np <= 0) return HF_OK;
    Geom g;
    if (!make_geom(box, g)) return HF_ERR_SIZE;
    auto *lab2 = static_cast<int32_t *>(scratch);
    if (parts)
        HF_LAUNCH(ctx, K_LABEL_TILES, tile_label_kernel<true>, dim3(g.ntiles), dim3(ACC_THREADS), 0, ctx->stream,
                  order.rec2, order.start2, g, cell_label, lab2, parts);
    else
        HF_LAUNCH(ctx, K_LABEL_TILES, tile_label_kernel<false>, dim3(g.ntiles), dim3(ACC_THREADS), 0, ctx->stream,
                  order.rec2, order.start2, g, cell_label, lab2, nullptr);
    return launch_status();
}

hf_status hf::label_back(hf_ctx *ctx, const hf_box &box, int64_t np, const ParticleOrder &order,
                         int32_t *particle_label, void *scratch, const uint32_t *keep, const ClaimOut *claim,
                         const TileClaim *tile_claim) {
    if (np <= 0) return HF_OK;
    Geom g;
    if (!make_geom(box, g)) return HF_ERR_SIZE;
    auto *lab2 = static_cast<int32_t *>(scratch);
    auto *lab1 = reinterpret_cast<int32_t *>(static_cast<char *>(scratch) + align_up(sizeof(int32_t) * size_t(np)));
    const unsigned blocks = unsigned((np + CHUNK - 1) / CHUNK);
    // level-2 scatter chunks: at most one partial chunk per bucket beyond np / CHUNK
    RunMaps m1, m2;
    __builtin_memcpy(&m1, order.maps[0], sizeof(m1));
    __builtin_memcpy(&m2, order.maps[1], sizeof(m2));
    if (tile_claim && !keep) return HF_ERR_ARG;
    if (tile_claim)
        HF_LAUNCH(ctx, K_LABEL_LEVEL1, (to_level1_kernel<true, true>), dim3(blocks + unsigned(g.nbuckets)),
                  dim3(PART_THREADS), 0, ctx->stream, m2, order.start1, order.chunk_first, g.nbuckets, g.digits, lab2,
                  lab1, keep, *tile_claim);
    else if (keep)
        HF_LAUNCH(ctx, K_LABEL_LEVEL1, (to_level1_kernel<true, false>), dim3(blocks + unsigned(g.nbuckets)),
                  dim3(PART_THREADS), 0, ctx->stream, m2, order.start1, order.chunk_first, g.nbuckets, g.digits, lab2,
                  lab1, keep, TileClaim{});
    else
        HF_LAUNCH(ctx, K_LABEL_LEVEL1, (to_level1_kernel<false, false>), dim3(blocks + unsigned(g.nbuckets)),
                  dim3(PART_THREADS), 0, ctx->stream, m2, order.start1, order.chunk_first, g.nbuckets, g.digits, lab2,
                  lab1, nullptr, TileClaim{});
    if (claim)
        HF_LAUNCH(ctx, K_LABEL_INPUT, to_input_kernel<true>, dim3(replica_grid(blocks)), dim3(PART_THREADS), 0,
                  ctx->stream, m1, np, g.nbuckets, lab1, particle_label, *claim);
    else
        HF_LAUNCH(ctx, K_LABEL_INPUT, to_input_kernel<false>, dim3(replica_grid(blocks)), dim3(PART_THREADS), 0,
                  ctx->stream, m1, np, g.nbuckets, lab1, particle_label, ClaimOut{});
    return launch_status();
}

hf_status hf::label_from_order(hf_ctx *ctx, const hf_box &box, int64_t np, const ParticleOrder &order,
                               const int32_t *cell_label, int32_t *particle_label, void *scratch) {
    hf_status s = label_tiles(ctx, box, np, order, cell_label, scratch, nullptr);
    return s == HF_OK ? label_back(ctx, box, np, order, particle_label, scratch, nullptr) : s;
}
