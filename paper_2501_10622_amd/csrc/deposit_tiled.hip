// Step 2 (Eq. (1)), binned form of the CIC deposit for grids with n % 16 == 0.
//
// Particles arrive in arbitrary order, so depositing straight into an n^3 grid
// of int64 means random read-modify-writes of whole HBM lines.  Instead:
//
//   L1  partition the particles by coarse bucket (<= 512 buckets of bt^3
//       tiles), records = the three fixed-point coordinates q (12 bytes);
//   L2  partition each bucket by 16^3-cell tile, records = cell-in-tile and
//       fraction bits packed into 8 bytes;
//   ACC one workgroup per tile accumulates its particles' eight CIC weights in
//       LDS int64 over the tile plus its +x/+y/+z skirt (17^3 cells), writes
//       the 16^3 owned cells once and the 817 skirt sums to a side buffer;
//   FOLD each tile adds the skirt sums of its lower neighbours to its low faces.
//
// Each partition pass is a histogram pass plus a scatter pass whose writes are
// staged in LDS so that each workgroup writes one contiguous run per bucket.
// Every sum is an exact integer sum, so the grid does not depend on particle
// order or on the order the atomics resolve in.
#include "hf_internal.h"

using namespace hf;

namespace {

constexpr int TILE = 16;
constexpr int ACC_EDGE = TILE + 1;
constexpr int ACC_CELLS = ACC_EDGE * ACC_EDGE * ACC_EDGE;              // 4913
constexpr int FACE_X = ACC_EDGE * ACC_EDGE;                             // cells (16, y, z), y,z <= 16
constexpr int FACE_Y = TILE * ACC_EDGE;                                 // cells (x, 16, z), x < 16, z <= 16
constexpr int FACE_Z = TILE * TILE;                                     // cells (x, y, 16), x, y < 16
constexpr int SKIRT = FACE_X + FACE_Y + FACE_Z;                         // 817
constexpr int PART_THREADS = 1024;
constexpr int PART_PER = 8;
constexpr int CHUNK = PART_THREADS * PART_PER;                          // particles per partition workgroup
constexpr int MAX_DIGITS = 512;
constexpr int ACC_THREADS = 256;

struct Geom {
    int n;        // grid cells per axis
    int nt;       // tiles per axis
    int bt;       // tiles per bucket edge
    int nb;       // buckets per axis
    int bcell;    // cells per bucket edge
    int nbuckets; // nb^3
    int digits;   // bt^3 tiles per bucket
    int ntiles;   // nt^3
    int bits;     // fraction bits B
};

struct Q3 {
    uint32_t x, y, z;
};

__device__ __forceinline__ int bucket_of(const Geom &g, uint32_t cx, uint32_t cy, uint32_t cz) {
    const uint32_t bc = uint32_t(g.bcell);
    return int(((cz / bc) * g.nb + cy / bc) * g.nb + cx / bc);
}

__device__ __forceinline__ int tile_in_bucket(const Geom &g, uint32_t cx, uint32_t cy, uint32_t cz) {
    const uint32_t bt = uint32_t(g.bt);
    return int((((cz / TILE) % bt) * bt + (cy / TILE) % bt) * bt + (cx / TILE) % bt);
}

// Packed tile-local record: per axis ((cell % 16) << B) | fraction, 4 + B bits.
__device__ __forceinline__ uint64_t pack_local(const Geom &g, const Q3 &q) {
    const uint32_t fm = (1u << g.bits) - 1u;
    const int s = 4 + g.bits;
    const uint64_t lx = (uint64_t(((q.x >> g.bits) & 15u)) << g.bits) | (q.x & fm);
    const uint64_t ly = (uint64_t(((q.y >> g.bits) & 15u)) << g.bits) | (q.y & fm);
    const uint64_t lz = (uint64_t(((q.z >> g.bits) & 15u)) << g.bits) | (q.z & fm);
    return lx | (ly << s) | (lz << (2 * s));
}

template <typename T>
__device__ __forceinline__ bool load_q(const T *__restrict__ pos, int64_t i, const FixedPoint<T> &fp, Q3 &q) {
    int64_t a, b, c;
    bool ok = fp.q(pos[3 * i + 0], a);
    ok = fp.q(pos[3 * i + 1], b) && ok;
    ok = fp.q(pos[3 * i + 2], c) && ok;
    q.x = uint32_t(a);
    q.y = uint32_t(b);
    q.z = uint32_t(c);
    return ok;
}

// In-place exclusive scan of s[0..count) (count <= 512) by the whole workgroup;
// returns the total.  Hillis-Steele on a copy in `tmp`.
__device__ uint32_t block_exclusive_scan(uint32_t *s, uint32_t *tmp, int count) {
    const int t = threadIdx.x;
    if (t < MAX_DIGITS) tmp[t] = t < count ? s[t] : 0u;
    __syncthreads();
    for (int off = 1; off < MAX_DIGITS; off <<= 1) {
        uint32_t v = 0;
        if (t < MAX_DIGITS && t >= off) v = tmp[t - off];
        __syncthreads();
        if (t < MAX_DIGITS) tmp[t] += v;
        __syncthreads();
    }
    const uint32_t total = tmp[MAX_DIGITS - 1];
    if (t < count) s[t] = tmp[t] - s[t];
    __syncthreads();
    return total;
}

__global__ void zero_u32_kernel(uint32_t *p, int64_t count) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < count; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0u;
}

// ---------------------------------------------------------------- level 1
template <typename T>
__global__ void __launch_bounds__(PART_THREADS) l1_hist_kernel(const T *__restrict__ pos, int64_t np,
                                                               FixedPoint<T> fp, Geom g, uint32_t *count1,
                                                               uint32_t *status) {
    __shared__ uint32_t h[MAX_DIGITS];
    for (int b = threadIdx.x; b < MAX_DIGITS; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    bool bad = false;
    const int64_t base = int64_t(blockIdx.x) * CHUNK;
#pragma unroll
    for (int k = 0; k < PART_PER; ++k) {
        const int64_t i = base + k * PART_THREADS + threadIdx.x;
        if (i < np) {
            Q3 q;
            if (load_q(pos, i, fp, q))
                atomicAdd(&h[bucket_of(g, q.x >> g.bits, q.y >> g.bits, q.z >> g.bits)], 1u);
            else
                bad = true;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < g.nbuckets; b += blockDim.x)
        if (h[b]) atomicAdd(&count1[b], h[b]);
    if (bad) atomicOr(status, ST_INPUT);
}

// start1 / cursor1 = exclusive scan of the bucket counts; chunk_first = exclusive
// scan of the number of CHUNK-sized level-2 chunks per bucket.
__global__ void __launch_bounds__(MAX_DIGITS) l1_scan_kernel(const uint32_t *__restrict__ count1, int nbuckets,
                                                             uint32_t *start1, uint32_t *cursor1,
                                                             uint32_t *chunk_first) {
    __shared__ uint32_t s[MAX_DIGITS], c[MAX_DIGITS], tmp[MAX_DIGITS];
    const int t = threadIdx.x;
    const uint32_t cnt = t < nbuckets ? count1[t] : 0u;
    s[t] = cnt;
    c[t] = (cnt + CHUNK - 1) / CHUNK;
    __syncthreads();
    const uint32_t total = block_exclusive_scan(s, tmp, nbuckets);
    const uint32_t chunks = block_exclusive_scan(c, tmp, nbuckets);
    if (t < nbuckets) {
        start1[t] = s[t];
        cursor1[t] = s[t];
        chunk_first[t] = c[t];
    }
    if (t == 0) {
        start1[nbuckets] = total;
        chunk_first[nbuckets] = chunks;
    }
}

template <typename T>
__global__ void __launch_bounds__(PART_THREADS) l1_scatter_kernel(const T *__restrict__ pos, int64_t np,
                                                                  FixedPoint<T> fp, Geom g, uint32_t *cursor1,
                                                                  Q3 *__restrict__ rec1) {
    __shared__ Q3 stage[CHUNK];
    __shared__ uint32_t h[MAX_DIGITS], off[MAX_DIGITS], gbase[MAX_DIGITS], tmp[MAX_DIGITS];
    for (int b = threadIdx.x; b < MAX_DIGITS; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * CHUNK;
    Q3 q[PART_PER];
    int bk[PART_PER];
    uint32_t rank[PART_PER];
#pragma unroll
    for (int k = 0; k < PART_PER; ++k) {
        const int64_t i = base + k * PART_THREADS + threadIdx.x;
        bk[k] = -1;
        if (i < np && load_q(pos, i, fp, q[k])) {
            bk[k] = bucket_of(g, q[k].x >> g.bits, q[k].y >> g.bits, q[k].z >> g.bits);
            rank[k] = atomicAdd(&h[bk[k]], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < g.nbuckets; b += blockDim.x) off[b] = h[b];
    __syncthreads();
    const uint32_t total = block_exclusive_scan(off, tmp, g.nbuckets);
    for (int b = threadIdx.x; b < g.nbuckets; b += blockDim.x)
        if (h[b]) gbase[b] = atomicAdd(&cursor1[b], h[b]);
#pragma unroll
    for (int k = 0; k < PART_PER; ++k)
        if (bk[k] >= 0) stage[off[bk[k]] + rank[k]] = q[k];
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < total; s += PART_THREADS) {
        const Q3 r = stage[s];
        const int b = bucket_of(g, r.x >> g.bits, r.y >> g.bits, r.z >> g.bits);
        rec1[gbase[b] + (s - off[b])] = r;
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
    const uint32_t *start1;
    const uint32_t *chunk_first;
    int nbuckets;
};

// Locates this workgroup's chunk: bucket b and the index range [lo, hi).
template <typename T, bool FROM_REC>
__device__ __forceinline__ bool l2_chunk(const L2Input<T, FROM_REC> &in, int &b, int64_t &lo, int64_t &hi) {
    const uint32_t w = blockIdx.x;
    if (!FROM_REC) {
        b = 0;
        lo = int64_t(w) * CHUNK;
        hi = lo + CHUNK < in.np ? lo + CHUNK : in.np;
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
    lo = int64_t(in.start1[b]) + int64_t(w - in.chunk_first[b]) * CHUNK;
    const int64_t end = in.start1[b + 1];
    hi = lo + CHUNK < end ? lo + CHUNK : end;
    return true;
}

template <typename T, bool FROM_REC>
__device__ __forceinline__ bool l2_load(const L2Input<T, FROM_REC> &in, int64_t i, Q3 &q) {
    if (FROM_REC) {
        q = in.rec1[i];
        return true;
    }
    return load_q(in.pos, i, in.fp, q);
}

template <typename T, bool FROM_REC>
__global__ void __launch_bounds__(PART_THREADS) l2_hist_kernel(L2Input<T, FROM_REC> in, Geom g, uint32_t *count2,
                                                               uint32_t *status) {
    __shared__ uint32_t h[MAX_DIGITS];
    int b;
    int64_t lo, hi;
    if (!l2_chunk(in, b, lo, hi)) return;
    for (int d = threadIdx.x; d < MAX_DIGITS; d += blockDim.x) h[d] = 0u;
    __syncthreads();
    bool bad = false;
#pragma unroll
    for (int k = 0; k < PART_PER; ++k) {
        const int64_t i = lo + k * PART_THREADS + threadIdx.x;
        if (i < hi) {
            Q3 q;
            if (l2_load(in, i, q))
                atomicAdd(&h[tile_in_bucket(g, q.x >> g.bits, q.y >> g.bits, q.z >> g.bits)], 1u);
            else
                bad = true;
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < g.digits; d += blockDim.x)
        if (h[d]) atomicAdd(&count2[int64_t(b) * g.digits + d], h[d]);
    if (bad) atomicOr(status, ST_INPUT);
}

// start2 / cursor2 = exclusive scan of the per-tile counts (bucket-major order).
__global__ void __launch_bounds__(1024) l2_scan_kernel(const uint32_t *__restrict__ count2, int ntiles,
                                                       uint32_t *start2, uint32_t *cursor2) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int per = (ntiles + 1023) / 1024;
    const int lo = t * per, hi = min(ntiles, lo + per);
    uint32_t s = 0;
    for (int i = lo; i < hi; ++i) s += count2[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t > 0 ? part[t - 1] : 0u;
    for (int i = lo; i < hi; ++i) {
        start2[i] = run;
        cursor2[i] = run;
        run += count2[i];
    }
    if (t == 1023) start2[ntiles] = part[1023];
}

template <typename T, bool FROM_REC>
__global__ void __launch_bounds__(PART_THREADS) l2_scatter_kernel(L2Input<T, FROM_REC> in, Geom g,
                                                                  uint32_t *cursor2, uint64_t *__restrict__ rec2) {
    __shared__ uint64_t stage[CHUNK];
    __shared__ uint16_t sdig[CHUNK];
    __shared__ uint32_t h[MAX_DIGITS], off[MAX_DIGITS], gbase[MAX_DIGITS], tmp[MAX_DIGITS];
    int b;
    int64_t lo, hi;
    if (!l2_chunk(in, b, lo, hi)) return;
    for (int d = threadIdx.x; d < MAX_DIGITS; d += blockDim.x) h[d] = 0u;
    __syncthreads();
    uint64_t r[PART_PER];
    int dg[PART_PER];
    uint32_t rank[PART_PER];
#pragma unroll
    for (int k = 0; k < PART_PER; ++k) {
        const int64_t i = lo + k * PART_THREADS + threadIdx.x;
        dg[k] = -1;
        Q3 q;
        if (i < hi && l2_load(in, i, q)) {
            dg[k] = tile_in_bucket(g, q.x >> g.bits, q.y >> g.bits, q.z >> g.bits);
            r[k] = pack_local(g, q);
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
    for (uint32_t s = threadIdx.x; s < total; s += PART_THREADS) {
        const int d = sdig[s];
        rec2[gbase[d] + (s - off[d])] = stage[s];
    }
}

// ---------------------------------------------------------------- accumulate and fold
__device__ __forceinline__ void tile_coords(const Geom &g, int b, int d, int &tx, int &ty, int &tz) {
    const int bx = b % g.nb, by = (b / g.nb) % g.nb, bz = b / (g.nb * g.nb);
    const int ux = d % g.bt, uy = (d / g.bt) % g.bt, uz = d / (g.bt * g.bt);
    tx = bx * g.bt + ux;
    ty = by * g.bt + uy;
    tz = bz * g.bt + uz;
}

__device__ __forceinline__ void lds_add(unsigned long long *acc, int c, unsigned long long w, bool &overflow) {
    if (w == 0) return;
    const unsigned long long old = atomicAdd(acc + c, w);
    if (!(old >> 63) && ((old + w) >> 63)) overflow = true;
}

__device__ __forceinline__ void skirt_cell(int s, int &x, int &y, int &z) {
    if (s < FACE_X) {
        x = TILE;
        y = s % ACC_EDGE;
        z = s / ACC_EDGE;
    } else if (s < FACE_X + FACE_Y) {
        const int j = s - FACE_X;
        x = j % TILE;
        y = TILE;
        z = j / TILE;
    } else {
        const int j = s - FACE_X - FACE_Y;
        x = j % TILE;
        y = j / TILE;
        z = TILE;
    }
}

__device__ __forceinline__ int skirt_index(int x, int y, int z) {
    if (x == TILE) return z * ACC_EDGE + y;
    if (y == TILE) return FACE_X + z * TILE + x;
    return FACE_X + FACE_Y + y * TILE + x;
}

// One workgroup per tile, in level-2 (bucket, tile-in-bucket) order.
__global__ void __launch_bounds__(ACC_THREADS) tile_accum_kernel(const uint64_t *__restrict__ rec2,
                                                                 const uint32_t *__restrict__ start2, Geom g,
                                                                 unsigned long long *__restrict__ rho,
                                                                 unsigned long long *__restrict__ skirt,
                                                                 uint32_t *status) {
    __shared__ unsigned long long acc[ACC_CELLS];
    const int slot = blockIdx.x;
    const int b = slot / g.digits, d = slot % g.digits;
    int tx, ty, tz;
    tile_coords(g, b, d, tx, ty, tz);
    for (int c = threadIdx.x; c < ACC_CELLS; c += ACC_THREADS) acc[c] = 0ull;
    __syncthreads();
    const uint32_t lo = start2[slot], hi = start2[slot + 1];
    const int s = 4 + g.bits;
    const uint64_t fmask = (1ull << g.bits) - 1ull, lmask = (1ull << s) - 1ull;
    const uint64_t one = 1ull << g.bits;
    bool overflow = false;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += ACC_THREADS) {
        const uint64_t r = rec2[i];
        const uint64_t ax = r & lmask, ay = (r >> s) & lmask, az = (r >> (2 * s)) & lmask;
        const int cx = int(ax >> g.bits), cy = int(ay >> g.bits), cz = int(az >> g.bits);
        const uint64_t fx = ax & fmask, fy = ay & fmask, fz = az & fmask;
        const uint64_t wx0 = one - fx, wy0 = one - fy, wz0 = one - fz;
        const int c0 = (cz * ACC_EDGE + cy) * ACC_EDGE + cx;
        const uint64_t w00 = wz0 * wy0, w01 = wz0 * fy, w10 = fz * wy0, w11 = fz * fy;
        lds_add(acc, c0, w00 * wx0, overflow);
        lds_add(acc, c0 + 1, w00 * fx, overflow);
        lds_add(acc, c0 + ACC_EDGE, w01 * wx0, overflow);
        lds_add(acc, c0 + ACC_EDGE + 1, w01 * fx, overflow);
        lds_add(acc, c0 + ACC_EDGE * ACC_EDGE, w10 * wx0, overflow);
        lds_add(acc, c0 + ACC_EDGE * ACC_EDGE + 1, w10 * fx, overflow);
        lds_add(acc, c0 + ACC_EDGE * ACC_EDGE + ACC_EDGE, w11 * wx0, overflow);
        lds_add(acc, c0 + ACC_EDGE * ACC_EDGE + ACC_EDGE + 1, w11 * fx, overflow);
    }
    __syncthreads();
    const size_t n = size_t(g.n);
    for (int c = threadIdx.x; c < TILE * TILE * TILE; c += ACC_THREADS) {
        const int x = c % TILE, y = (c / TILE) % TILE, z = c / (TILE * TILE);
        rho[((size_t(tz) * TILE + z) * n + size_t(ty) * TILE + y) * n + size_t(tx) * TILE + x] =
            acc[(z * ACC_EDGE + y) * ACC_EDGE + x];
    }
    const size_t tglob = (size_t(tz) * g.nt + ty) * g.nt + tx;
    for (int k = threadIdx.x; k < SKIRT; k += ACC_THREADS) {
        int x, y, z;
        skirt_cell(k, x, y, z);
        skirt[tglob * SKIRT + k] = acc[(z * ACC_EDGE + y) * ACC_EDGE + x];
    }
    if (overflow) atomicOr(status, ST_OVERFLOW);
}

// One workgroup per tile: its low-face cells gather the skirt sums that lower
// neighbours computed for them.
__global__ void __launch_bounds__(ACC_THREADS) skirt_fold_kernel(const unsigned long long *__restrict__ skirt, Geom g,
                                                                 unsigned long long *__restrict__ rho,
                                                                 uint32_t *status) {
    const int t = blockIdx.x;
    const int tx = t % g.nt, ty = (t / g.nt) % g.nt, tz = t / (g.nt * g.nt);
    const size_t n = size_t(g.n);
    bool overflow = false;
    // the 16^3 - 15^3 = 721 cells with at least one local coordinate 0
    for (int c = threadIdx.x; c < TILE * TILE * TILE; c += ACC_THREADS) {
        const int x = c % TILE, y = (c / TILE) % TILE, z = c / (TILE * TILE);
        const int zmask = (x == 0 ? 1 : 0) | (y == 0 ? 2 : 0) | (z == 0 ? 4 : 0);
        if (!zmask) continue;
        const size_t idx = ((size_t(tz) * TILE + z) * n + size_t(ty) * TILE + y) * n + size_t(tx) * TILE + x;
        unsigned long long v = rho[idx];
        for (int dm = zmask; dm; dm = (dm - 1) & zmask) {  // nonzero subsets of the zero axes
            const int dx = dm & 1, dy = (dm >> 1) & 1, dz = (dm >> 2) & 1;
            const int sx = (tx - dx + g.nt) % g.nt, sy = (ty - dy + g.nt) % g.nt, sz = (tz - dz + g.nt) % g.nt;
            const size_t src = (size_t(sz) * g.nt + sy) * g.nt + sx;
            const unsigned long long w = skirt[src * SKIRT + skirt_index(x + TILE * dx, y + TILE * dy, z + TILE * dz)];
            const unsigned long long old = v;
            v += w;
            if (!(old >> 63) && (v >> 63)) overflow = true;
        }
        rho[idx] = v;
    }
    if (overflow) atomicOr(status, ST_OVERFLOW);
}

// ---------------------------------------------------------------- host side
Geom make_geom(const hf_box &box) {
    Geom g{};
    g.n = box.n;
    g.nt = box.n / TILE;
    g.bt = 1;
    for (int d = 8; d >= 1; --d)
        if (g.nt % d == 0) {
            g.bt = d;
            break;
        }
    g.nb = g.nt / g.bt;
    g.bcell = g.bt * TILE;
    g.nbuckets = g.nb * g.nb * g.nb;
    g.digits = g.bt * g.bt * g.bt;
    g.ntiles = g.nt * g.nt * g.nt;
    g.bits = box.frac_bits;
    return g;
}

struct DepLayout {
    size_t count1, start1, cursor1, chunk_first, count2, start2, cursor2, rec1, rec2, skirt, total;
};

DepLayout dep_layout(const Geom &g, int64_t np) {
    DepLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.count1 = take(sizeof(uint32_t) * MAX_DIGITS);
    L.count2 = take(sizeof(uint32_t) * size_t(g.ntiles));  // count1 and count2 are zeroed together
    L.start1 = take(sizeof(uint32_t) * (MAX_DIGITS + 1));
    L.cursor1 = take(sizeof(uint32_t) * MAX_DIGITS);
    L.chunk_first = take(sizeof(uint32_t) * (MAX_DIGITS + 1));
    L.start2 = take(sizeof(uint32_t) * (size_t(g.ntiles) + 1));
    L.cursor2 = take(sizeof(uint32_t) * size_t(g.ntiles));
    L.rec1 = take(g.nbuckets > 1 ? sizeof(Q3) * size_t(np) : 0);
    L.rec2 = take(sizeof(uint64_t) * size_t(np));
    L.skirt = take(sizeof(unsigned long long) * SKIRT * size_t(g.ntiles));
    L.total = off;
    return L;
}

template <typename T>
FixedPoint<T> fixed_point_of(const hf_box &box) {
    FixedPoint<T> fp;
    fp.bits = box.frac_bits;
    fp.period = int64_t(box.n) << box.frac_bits;
    fp.scale = T(double(box.n) * double(int64_t(1) << box.frac_bits) / box.box_len);
    return fp;
}

template <typename T>
hf_status run_tiled(hf_ctx *ctx, const hf_box &box, const T *pos, int64_t np, unsigned long long *rho,
                    char *ws) {
    const Geom g = make_geom(box);
    const DepLayout L = dep_layout(g, np);
    auto *count1 = reinterpret_cast<uint32_t *>(ws + L.count1);
    auto *count2 = reinterpret_cast<uint32_t *>(ws + L.count2);
    auto *start1 = reinterpret_cast<uint32_t *>(ws + L.start1);
    auto *cursor1 = reinterpret_cast<uint32_t *>(ws + L.cursor1);
    auto *chunk_first = reinterpret_cast<uint32_t *>(ws + L.chunk_first);
    auto *start2 = reinterpret_cast<uint32_t *>(ws + L.start2);
    auto *cursor2 = reinterpret_cast<uint32_t *>(ws + L.cursor2);
    auto *rec1 = reinterpret_cast<Q3 *>(ws + L.rec1);
    auto *rec2 = reinterpret_cast<uint64_t *>(ws + L.rec2);
    auto *skirt = reinterpret_cast<unsigned long long *>(ws + L.skirt);
    hipStream_t st = ctx->stream;
    const FixedPoint<T> fp = fixed_point_of<T>(box);
    const int64_t zero_count = int64_t((L.start1 - L.count1) / sizeof(uint32_t));
    HF_LAUNCH(ctx, K_DEP_PREP, zero_u32_kernel, dim3(64), dim3(256), 0, st, count1, zero_count);
    const unsigned part_blocks = unsigned((np + CHUNK - 1) / CHUNK);
    if (g.nbuckets > 1) {
        if (part_blocks)
            HF_LAUNCH(ctx, K_DEP_L1_HIST, l1_hist_kernel<T>, dim3(part_blocks), dim3(PART_THREADS), 0, st, pos, np,
                      fp, g, count1, ctx->d_status);
        HF_LAUNCH(ctx, K_DEP_PREP, l1_scan_kernel, dim3(1), dim3(MAX_DIGITS), 0, st, count1, g.nbuckets, start1,
                  cursor1, chunk_first);
        if (part_blocks)
            HF_LAUNCH(ctx, K_DEP_L1_SCATTER, l1_scatter_kernel<T>, dim3(part_blocks), dim3(PART_THREADS), 0, st, pos,
                      np, fp, g, cursor1, rec1);
        L2Input<T, true> in{pos, np, fp, rec1, start1, chunk_first, g.nbuckets};
        const unsigned l2_blocks = part_blocks + unsigned(g.nbuckets);
        HF_LAUNCH(ctx, K_DEP_L2_HIST, (l2_hist_kernel<T, true>), dim3(l2_blocks), dim3(PART_THREADS), 0, st, in, g,
                  count2, ctx->d_status);
        HF_LAUNCH(ctx, K_DEP_PREP, l2_scan_kernel, dim3(1), dim3(1024), 0, st, count2, g.ntiles, start2, cursor2);
        HF_LAUNCH(ctx, K_DEP_L2_SCATTER, (l2_scatter_kernel<T, true>), dim3(l2_blocks), dim3(PART_THREADS), 0, st,
                  in, g, cursor2, rec2);
    } else {
        L2Input<T, false> in{pos, np, fp, nullptr, nullptr, nullptr, 1};
        if (part_blocks)
            HF_LAUNCH(ctx, K_DEP_L2_HIST, (l2_hist_kernel<T, false>), dim3(part_blocks), dim3(PART_THREADS), 0, st,
                      in, g, count2, ctx->d_status);
        HF_LAUNCH(ctx, K_DEP_PREP, l2_scan_kernel, dim3(1), dim3(1024), 0, st, count2, g.ntiles, start2, cursor2);
        if (part_blocks)
            HF_LAUNCH(ctx, K_DEP_L2_SCATTER, (l2_scatter_kernel<T, false>), dim3(part_blocks), dim3(PART_THREADS),
                      0, st, in, g, cursor2, rec2);
    }
    HF_LAUNCH(ctx, K_DEPOSIT, tile_accum_kernel, dim3(g.ntiles), dim3(ACC_THREADS), 0, st, rec2, start2, g, rho,
              skirt, ctx->d_status);
    HF_LAUNCH(ctx, K_DEP_FOLD, skirt_fold_kernel, dim3(g.ntiles), dim3(ACC_THREADS), 0, st, skirt, g, rho,
              ctx->d_status);
    return launch_status();
}

}  // namespace

bool hf::deposit_tiled_supported(const hf_box &box, int64_t np) {
    // packed tile records hold 3 x (4 + B) <= 63 bits; counts are uint32; the
    // partition kernels hold at most MAX_DIGITS buckets (n = 432 and 864 would need 729)
    if (box.n % TILE != 0 || box.frac_bits > 17 || np >= (int64_t(1) << 32)) return false;
    return make_geom(box).nbuckets <= MAX_DIGITS;
}

size_t hf::deposit_tiled_ws_bytes(const hf_box &box, int64_t np) {
    return dep_layout(make_geom(box), np).total;
}

hf_status hf::deposit_tiled(hf_ctx *ctx, const hf_box &box, const void *pos, hf_dtype dtype, int64_t np,
                            int64_t *rho, void *ws) {
    auto *grid = reinterpret_cast<unsigned long long *>(rho);
    if (dtype == HF_F32) return run_tiled<float>(ctx, box, static_cast<const float *>(pos), np, grid, static_cast<char *>(ws));
    return run_tiled<double>(ctx, box, static_cast<const double *>(pos), np, grid, static_cast<char *>(ws));
}
