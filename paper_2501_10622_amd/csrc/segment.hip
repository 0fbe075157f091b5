// Step 4 (local maxima of the grid CWT) and step 5 (segmentation of the grid
// by its maxima, Sec. 2.3) on the FP32 CWT field.
//
// Order on cells: (value, linear index), larger value first, equal values by
// larger index, -0 equal to +0.  It is encoded as a 64-bit key whose integer
// order is that order: high word = order-preserving bits of the float, low
// word = index.  A cell's parent is the largest key of its 3x3x3 periodic
// neighbourhood (itself included); a cell is a maximum iff it is its own
// parent and its value exceeds tau.
//
// Tiled path: one workgroup per 32x16x16 tile holds the tile and
// a one-cell halo of the field in LDS, forms every cell's parent (the largest
// key of its 3x3x3 neighbourhood) and the maxima mask, and follows the parent
// chains inside the tile, so the parents never go to memory.
//  - maxima: a wavefront covers two 32-cell rows, so its ballot is two aligned
//    32-bit words of a linear-order bit mask; count / scan / write passes turn
//    the mask into the sorted index list (hf_maxima alone forms the maxima of
//    32x8x8 tiles separably, x then y then z).
//  - segmentation: parent chains are followed inside each 32x16x16 tile by
//    pointer doubling in LDS, so every cell ends at a root or at the first cell
//    its chain reaches outside the tile.  Such exit targets are always on a
//    tile boundary, so only the 2312 boundary cells of each tile (kept in a
//    compact array) take part in the global pointer-jumping rounds.  A root at or
//    below tau is written as -1 by its own tile, so the rounds carry the
//    threshold along and no later pass reads the field again.  A last pass,
//    one workgroup per tile, loads the resolved entries of the one-cell shell
//    around the tile (every exit target lies in it) into LDS and maps each
//    cell of the tile through them.
// Any n: where n is not a multiple of a tile's extent, the last tile along
// that axis is short (its cells past n are absent); a short tile's far-edge
// cells take the boundary ranks of a full tile's far edge.  The separable
// maxima pass of hf_maxima alone needs n % 32 == 0; other sizes use a direct
// per-cell pass with the same results.
#include "hf_internal.h"
#include "scan.h"

using namespace hf;

namespace {

// ------------------------------------------------------------------ keys
__device__ __forceinline__ uint32_t ordered_bits(float c, bool &nan) {
    uint32_t u = __float_as_uint(c);
    if ((u & 0x7fffffffu) > 0x7f800000u) nan = true;
    if (u == 0x80000000u) u = 0u;  // -0 -> +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ uint64_t cell_key(float c, uint32_t idx, bool &nan) {
    return (uint64_t(ordered_bits(c, nan)) << 32) | idx;
}

__device__ __forceinline__ uint32_t wrap(int v, int n) { return uint32_t(v < 0 ? v + n : (v >= n ? v - n : v)); }

__device__ __forceinline__ uint64_t kmax(uint64_t a, uint64_t b) { return a > b ? a : b; }

uint32_t host_ordered_bits(float c) {
    uint32_t u;
    static_assert(sizeof(u) == sizeof(c), "float is 32-bit");
    __builtin_memcpy(&u, &c, sizeof(u));
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ------------------------------------------------------------------ tile geometry
constexpr int TX = 32, TY = 8, TZ = 8;
constexpr int TCELLS = TX * TY * TZ;                          // 2048
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
constexpr int HCELLS = HX * HY * HZ;                          // 3400
constexpr int SEG_THREADS = 512;
constexpr int PER_THREAD = TCELLS / SEG_THREADS;              // 4

// Resolve tiles: chains are followed inside RX x RY x RZ tiles.
constexpr int RX = 32, RY = 16, RZ = 16;
constexpr int RCELLS = RX * RY * RZ;                          // 8192
constexpr int RHX = RX + 2, RHY = RY + 2, RHZ = RZ + 2;
constexpr int RHCELLS = RHX * RHY * RHZ;                      // 11016 (tile plus one-cell shell)
static_assert(2 * RHX * RHY + (RHZ - 2) * (2 * RHX + 2 * (RHY - 2)) == RHCELLS - RCELLS, "shell enumeration");
constexpr int NBND = 2 * RX * RY + (RZ - 2) * (2 * RX + 2 * (RY - 2));  // 2312 boundary cells per tile
constexpr int RES_THREADS = 1024;
constexpr int RES_PER = RCELLS / RES_THREADS;                 // 8

struct TileGrid {
    int n;
    int ntx, nty, ntz;  // tiles per axis
    FastDiv dn;         // division by n
};

__device__ __forceinline__ void cell_coords(const TileGrid &tg, uint32_t g, uint32_t &x, uint32_t &y, uint32_t &z) {
    const uint32_t q = tg.dn.div(g);
    x = g - q * uint32_t(tg.n);
    z = tg.dn.div(q);
    y = q - z * uint32_t(tg.n);
}

// Rank of local cell (x, y, z) among its resolve tile's boundary cells, or -1.
// Order: plane z = 0, planes 1..RZ-2 (row y = 0, then x = 0 / x = RX-1 of rows
// 1..RY-2, then row y = RY-1), plane z = RZ-1.
__device__ __forceinline__ int bnd_rank(int x, int y, int z) {
    if (z == 0) return y * RX + x;
    constexpr int MID = 2 * RX + 2 * (RY - 2);
    if (z == RZ - 1) return RX * RY + (RZ - 2) * MID + y * RX + x;
    const int base = RX * RY + (z - 1) * MID;
    if (y == 0) return base + x;
    if (y == RY - 1) return base + RX + 2 * (RY - 2) + x;
    if (x == 0) return base + RX + 2 * (y - 1);
    if (x == RX - 1) return base + RX + 2 * (y - 1) + 1;
    return -1;
}

// Extent along one axis of the resolve tile starting at `origin`: R, or less
// for the last tile where n is not a multiple of R.
__device__ __forceinline__ int tile_extent(int origin, int R, int n) { return n - origin < R ? n - origin : R; }

// Rank among its tile's boundary cells of local cell (x, y, z) of a tile of
// extents (wx, wy, wz), or -1: a coordinate on a short tile's far edge counts
// as the full tile's far edge, which keeps the ranks distinct.
__device__ __forceinline__ int bnd_rank_in(int x, int y, int z, int wx, int wy, int wz) {
    return bnd_rank(x == wx - 1 ? RX - 1 : x, y == wy - 1 ? RY - 1 : y, z == wz - 1 ? RZ - 1 : z);
}

// Where the compact boundary array keeps cell (x, y, z) (rg: the resolve-tile
// grid), or -1 if it is interior to its tile.  FULL: n is a multiple of every
// tile extent, so no tile is short.
template <bool FULL>
__device__ __forceinline__ int64_t bnd_slot_at(const TileGrid &rg, uint32_t x, uint32_t y, uint32_t z) {
    const int tx = int(x / RX), ty = int(y / RY), tz = int(z / RZ);
    const int lx = int(x) - tx * RX, ly = int(y) - ty * RY, lz = int(z) - tz * RZ;
    const int r = FULL ? bnd_rank(lx, ly, lz)
                       : bnd_rank_in(lx, ly, lz, tile_extent(tx * RX, RX, rg.n), tile_extent(ty * RY, RY, rg.n),
                                     tile_extent(tz * RZ, RZ, rg.n));
    if (r < 0) return -1;
    const int64_t tile = (int64_t(tz) * rg.nty + ty) * rg.ntx + tx;
    return tile * NBND + r;
}

template <bool FULL>
__device__ __forceinline__ int64_t bnd_slot(const TileGrid &rg, int32_t g) {
    uint32_t x, y, z;
    cell_coords(rg, uint32_t(g), x, y, z);
    return bnd_slot_at<FULL>(rg, x, y, z);
}

// Loads the keys of the tile at (x0, y0, z0) plus a one-cell periodic halo and
// leaves the parent key of local cell e = x + TX (y + TY z) in M[e].
__device__ void tile_parent_keys(const float *__restrict__ c, int n, int x0, int y0, int z0, uint64_t *K,
                                 uint64_t *M, bool &nan) {
    // all loads of the tile are issued before any is used (one batch per thread)
    constexpr int LOADS = (HCELLS + SEG_THREADS - 1) / SEG_THREADS;
    float v[LOADS];
    uint32_t jj[LOADS];
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
        const int e = threadIdx.x + i * SEG_THREADS;
        const int hx = e % HX, hy = (e / HX) % HY, hz = e / (HX * HY);
        const uint32_t gx = wrap(x0 + hx - 1, n), gy = wrap(y0 + hy - 1, n), gz = wrap(z0 + hz - 1, n);
        jj[i] = (gz * uint32_t(n) + gy) * uint32_t(n) + gx;
        if (e < HCELLS) v[i] = c[jj[i]];
    }
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
        const int e = threadIdx.x + i * SEG_THREADS;
        if (e < HCELLS) K[e] = cell_key(v[i], jj[i], nan);
    }
    __syncthreads();
    // x: M[hz][hy][x] over HZ x HY x TX
    for (int e = threadIdx.x; e < TX * HY * HZ; e += SEG_THREADS) {
        const int x = e % TX, r = e / TX;  // r = hz * HY + hy
        const uint64_t *k = K + r * HX + x;
        M[e] = kmax(kmax(k[0], k[1]), k[2]);
    }
    __syncthreads();
    // y: K[hz][y][x] over HZ x TY x TX
    for (int e = threadIdx.x; e < TX * TY * HZ; e += SEG_THREADS) {
        const int x = e % TX, y = (e / TX) % TY, hz = e / (TX * TY);
        const uint64_t *m = M + (hz * HY + y) * TX + x;
        K[e] = kmax(kmax(m[0], m[TX]), m[2 * TX]);
    }
    __syncthreads();
    // z: M[z][y][x] over TZ x TY x TX
    for (int e = threadIdx.x; e < TCELLS; e += SEG_THREADS) {
        const uint64_t *k = K + e;
        M[e] = kmax(kmax(k[0], k[TX * TY]), k[2 * TX * TY]);
    }
    __syncthreads();
}

__device__ __forceinline__ void tile_origin(const TileGrid &tg, int t, int &x0, int &y0, int &z0) {
    x0 = (t % tg.ntx) * TX;
    y0 = ((t / tg.ntx) % tg.nty) * TY;
    z0 = (t / (tg.ntx * tg.nty)) * TZ;
}

__device__ __forceinline__ void rtile_origin(const TileGrid &rg, int t, int &x0, int &y0, int &z0) {
    x0 = (t % rg.ntx) * RX;
    y0 = ((t / rg.ntx) % rg.nty) * RY;
    z0 = (t / (rg.ntx * rg.nty)) * RZ;
}

// Maxima bit mask of the tile from its parent keys M: bit (j % 32) of word
// j / 32 is set iff cell j is its own parent with a value above tau.
__device__ __forceinline__ void write_mask(const uint64_t *M, uint32_t n, int x0, int y0, int z0, uint32_t tau_ord,
                                           uint32_t *__restrict__ mask) {
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
        const int e = i * SEG_THREADS + threadIdx.x;  // a wavefront covers rows (y, z) and (y + 1, z)
        const int x = e % TX, y = (e / TX) % TY, z = e / (TX * TY);
        const uint32_t g = ((uint32_t(z0 + z) * n) + uint32_t(y0 + y)) * n + uint32_t(x0 + x);
        const uint64_t p = M[e];
        const bool is_max = uint32_t(p) == g && uint32_t(p >> 32) > tau_ord;
        const unsigned long long bits = __ballot(is_max);
        if ((threadIdx.x & 63) == 0) {
            mask[g >> 5] = uint32_t(bits);
            mask[(g + n) >> 5] = uint32_t(bits >> 32);  // next row of the tile
        }
    }
}

__global__ void __launch_bounds__(SEG_THREADS) max_tile_kernel(const float *__restrict__ c, TileGrid tg,
                                                               uint32_t tau_ord, uint32_t *__restrict__ mask,
                                                               uint32_t *status) {
    __shared__ uint64_t K[HCELLS];
    __shared__ uint64_t M[TX * HY * HZ];
    int x0, y0, z0;
    const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
    tile_origin(tg, int(tile), x0, y0, z0);
    bool nan = false;
    tile_parent_keys(c, tg.n, x0, y0, z0, K, M, nan);
    write_mask(M, uint32_t(tg.n), x0, y0, z0, tau_ord, mask);
    if (nan) atomicOr(status, ST_INPUT);
}

// Parents and the chains inside a resolve tile in one pass, one workgroup per
// RX x RY x RZ tile.  A cell's parent is the index of the largest key of its
// 3x3x3 neighbourhood, or -1 for a root (its own parent) at or below tau; with
// a mask the tile's maxima bits are written as well (the maxima are exactly
// the cells that are their own parent, above tau).
//
// The tile and a one-cell halo of the field sit in LDS as 32-bit
// order-preserving bits (the index half of a key is formed in registers).
// Each thread walks one z column: the largest key of each 3x3 halo plane
// around the column is formed once, and a cell's parent is the largest of the
// three plane maxima around it (about 10 LDS reads per cell).  The parents
// then replace the field in LDS as the tile's pointer array, where chains are
// followed by pointer doubling, so that on exit every cell holds its root (-1
// for a root at or below tau) or the first cell its chain reaches outside the
// tile; that goes to ptr and, for the tile's boundary cells, to bnd.  In LDS,
// loc[e] >= 0 points to local cell loc[e]; loc[e] < 0 is resolved to the
// value -2 - loc[e].
constexpr int PR_THREADS = RX * RY;          // one z column each
constexpr int PR_PER = RCELLS / PR_THREADS;  // RZ cells per thread
static_assert(RHCELLS >= RCELLS, "the pointer array fits where the field was");

template <bool FULL>
__global__ void __launch_bounds__(PR_THREADS) parent_resolve_kernel(const float *__restrict__ c, TileGrid rg,
                                                                    uint32_t tau_ord, int32_t *__restrict__ ptr,
                                                                    int32_t *__restrict__ bnd,
                                                                    uint32_t *__restrict__ mask, uint32_t *status) {
    __shared__ uint32_t V[RHCELLS];
    int32_t *loc = reinterpret_cast<int32_t *>(V);  // after the parents are formed
    int x0, y0, z0;
    const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
    rtile_origin(rg, int(tile), x0, y0, z0);
    const int n = rg.n;
    const uint32_t un = uint32_t(n);
    // a tile at the far end of an axis is short where n is not a multiple of
    // the tile: its cells past n are absent (never pointed to, never written)
    const int wx = FULL ? RX : tile_extent(x0, RX, n), wy = FULL ? RY : tile_extent(y0, RY, n),
              wz = FULL ? RZ : tile_extent(z0, RZ, n);
    const bool full = FULL || (wx == RX && wy == RY && wz == RZ);
    bool nan = false;
    {
        // all loads of the halo tile are issued before any is used
        constexpr int LOADS = (RHCELLS + PR_THREADS - 1) / PR_THREADS;
        float v[LOADS];
#pragma unroll
        for (int i = 0; i < LOADS; ++i) {
            const int e = threadIdx.x + i * PR_THREADS;
            const int hx = e % RHX, hy = (e / RHX) % RHY, hz = e / (RHX * RHY);
            if (e < RHCELLS)
                v[i] = c[(wrap(z0 + hz - 1, n) * un + wrap(y0 + hy - 1, n)) * un + wrap(x0 + hx - 1, n)];
        }
#pragma unroll
        for (int i = 0; i < LOADS; ++i) {
            const int e = threadIdx.x + i * PR_THREADS;
            if (e < RHCELLS) V[e] = ordered_bits(v[i], nan);
        }
    }
    __syncthreads();
    // the thread's column (x, y); a wavefront covers rows y and y + 1 of one z,
    // so its ballot is two aligned 32-bit words of the mask
    const int x = threadIdx.x % RX, y = threadIdx.x / RX;
    const int lane = threadIdx.x & 63;
    uint32_t gx[3], gyn[3];  // global x of the halo columns x - 1 .. x + 1, and (global y) * n of the rows
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        gx[d] = wrap(x0 + x + d - 1, n);
        gyn[d] = wrap(y0 + y + d - 1, n) * un;
    }
    // largest key of halo plane hz around the column
    auto plane_max = [&](int hz) {
        const uint32_t plane = wrap(z0 + hz - 1, n) * un * un;
        uint64_t best = 0;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const uint32_t row = plane + gyn[dy];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
                best = kmax(best, (uint64_t(V[(hz * RHY + y + dy) * RHX + x + dx]) << 32) | (row + gx[dx]));
        }
        return best;
    };
    int32_t l[PR_PER];
    // a tile whose halo does not wrap around the periodic box: there a cell's
    // neighbours, taken in (dz, dy, dx) order, come in increasing global index,
    // so the largest key is the last largest value met in that order (32-bit
    // compares and a neighbour code 0..26, no index per neighbour)
    const bool interior = FULL && x0 > 0 && x0 + RX < n && y0 > 0 && y0 + RY < n && z0 > 0 && z0 + RZ < n;
    if (interior) {
        auto plane_arg = [&](int hz, uint32_t &bv, uint32_t &bc) {
            bv = V[(hz * RHY + y) * RHX + x];
            bc = 0u;
#pragma unroll
            for (int k = 1; k < 9; ++k) {
                const uint32_t v = V[(hz * RHY + y + k / 3) * RHX + x + k % 3];
                const bool up = v >= bv;
                bv = up ? v : bv;
                bc = up ? uint32_t(k) : bc;
            }
        };
        uint32_t v0, c0, v1, c1;
        plane_arg(0, v0, c0);
        plane_arg(1, v1, c1);
        const uint32_t gb = (uint32_t(z0) * un + uint32_t(y0 + y)) * un + uint32_t(x0 + x);
#pragma unroll
        for (int z = 0; z < RZ; ++z) {
            uint32_t v2, c2;
            plane_arg(z + 2, v2, c2);
            uint32_t bv = v0, bc = c0;
            if (v1 >= bv) {
                bv = v1;
                bc = c1 + 9u;
            }
            if (v2 >= bv) {
                bv = v2;
                bc = c2 + 18u;
            }
            const uint32_t g = gb + uint32_t(z) * un * un;
            const bool self = bc == 13u;  // (dz, dy, dx) = (1, 1, 1)
            const bool high = bv > tau_ord;
            if (mask) {  // the wavefront's two rows are two aligned mask words
                const unsigned long long bits = __ballot(self && high);
                if (lane == 0) {
                    mask[g >> 5] = uint32_t(bits);
                    mask[(g + un) >> 5] = uint32_t(bits >> 32);
                }
            }
            const int lx = x + int(bc % 3u) - 1, ly = y + int((bc / 3u) % 3u) - 1, lz = z + int(bc / 9u) - 1;
            if (self)
                l[z] = high ? -2 - int32_t(g) : -1;
            else if (lx >= 0 && lx < RX && ly >= 0 && ly < RY && lz >= 0 && lz < RZ)
                l[z] = lx + RX * (ly + RY * lz);
            else
                l[z] = -2 - int32_t((uint32_t(z0 + lz) * un + uint32_t(y0 + ly)) * un + uint32_t(x0 + lx));
            v0 = v1;
            c0 = c1;
            v1 = v2;
            c1 = c2;
        }
    } else {
        uint64_t b0 = plane_max(0), b1 = plane_max(1);
#pragma unroll
        for (int z = 0; z < RZ; ++z) {
            const uint64_t b2 = plane_max(z + 2);
            const uint64_t best = kmax(kmax(b0, b1), b2);
            const bool real = x < wx && y < wy && z < wz;
            const uint32_t g = (uint32_t(z0 + z) * un + uint32_t(y0 + y)) * un + uint32_t(x0 + x);
            const uint32_t p = uint32_t(best);
            const bool high = uint32_t(best >> 32) > tau_ord;
            if (mask) {
                if (FULL) {  // the wavefront's two rows are two aligned mask words
                    const unsigned long long bits = __ballot(p == g && high);
                    if (lane == 0) {
                        mask[g >> 5] = uint32_t(bits);
                        mask[(g + un) >> 5] = uint32_t(bits >> 32);
                    }
                } else if (real && p == g && high) {  // rows straddle words: the mask was cleared first
                    atomicOr(&mask[g >> 5], 1u << (g & 31u));
                }
            }
            // local form: a root (above tau: itself; else -1) is resolved, so is
            // a parent outside the tile; a parent inside is followed
            l[z] = (p == g) ? (high ? -2 - int32_t(g) : -1) : -2 - int32_t(p);
            if (!real) l[z] = -1;  // absent
            if (real && p != g) {
                uint32_t px, py, pz;
                cell_coords(rg, p, px, py, pz);
                const int lx = int(px) - x0, ly = int(py) - y0, lz = int(pz) - z0;
                if (lx >= 0 && lx < RX && ly >= 0 && ly < RY && lz >= 0 && lz < RZ) l[z] = lx + RX * (ly + RY * lz);
            }
            b0 = b1;
            b1 = b2;
        }
    }
    if (nan) atomicOr(status, ST_INPUT);
    __syncthreads();  // every read of the field is done
#pragma unroll
    for (int z = 0; z < RZ; ++z) loc[threadIdx.x + z * PR_THREADS] = l[z];  // local cell x + RX (y + RY z)
    __syncthreads();
    // pointer doubling inside the tile (chains are at most RCELLS - 1 long)
    bool open = true;
    while (open) {
        int32_t nv[PR_PER];
        bool any = false;
#pragma unroll
        for (int i = 0; i < PR_PER; ++i) {
            const int32_t w = loc[i * PR_THREADS + threadIdx.x];
            nv[i] = w >= 0 ? loc[w] : w;
            any |= nv[i] >= 0;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PR_PER; ++i) loc[i * PR_THREADS + threadIdx.x] = nv[i];
        open = __syncthreads_or(any);
    }
    if (!full) {
        // a short tile leaves some of its boundary slots unused: they hold -1
        // (final), so that the jump rounds, which visit every slot, read no
        // stale entry
        for (int k = threadIdx.x; k < NBND; k += PR_THREADS) bnd[int64_t(tile) * NBND + k] = -1;
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < PR_PER; ++i) {
        const int e = i * PR_THREADS + threadIdx.x;  // (x, y) of this thread, z = i
        if (x >= wx || y >= wy || i >= wz) continue;
        const uint32_t g = ((uint32_t(z0 + i) * un) + uint32_t(y0 + y)) * un + uint32_t(x0 + x);
        const int32_t t = -2 - loc[e];
        ptr[g] = t;
        const int r = bnd_rank_in(x, y, i, wx, wy, wz);
        if (r >= 0) bnd[int64_t(tile) * NBND + r] = t;
    }
}

__global__ void zero_words_kernel(uint32_t *w, int64_t count) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < count; i += int64_t(gridDim.x) * blockDim.x)
        w[i] = 0u;
}

__global__ void fill_flags_kernel(uint32_t *flags, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) flags[i] = (i == 0) ? 1u : 0u;
}

// Pointer jumping over the boundary entries, in place.  Round 0 visits every
// entry; each workgroup appends to its own slice of a list (cap entries at
// blockIdx * cap, count in counts[blockIdx]) the entries that changed and now
// point at a boundary cell, whose own entry may still change: only those can
// change again (an entry that does not change points at a root, which is
// final).  Each later round visits its workgroup's slice of the previous
// round's list and writes the entries still active to the other list, so no
// global counter is shared and the lists shrink.  Round r runs only if round
// r - 1 left an entry active, so a fixed number of launches is enough.
constexpr int BATCH = 8;  // independent iterations per thread and pass, so their loads overlap

// Appends the entries k with `again` set to this workgroup's slice `mine`
// (one LDS reservation per wavefront).
__device__ __forceinline__ void append_active(bool again, uint32_t k, uint32_t *mine, uint32_t *lcount) {
    const int lane = threadIdx.x & 63;
    const unsigned long long bits = __ballot(again);
    if (bits) {
        const int leader = __ffsll(bits) - 1;
        uint32_t at = 0;
        if (lane == leader) at = atomicAdd(lcount, uint32_t(__popcll(bits)));
        at = __shfl(at, leader, 64);
        if (again) mine[at + __popcll(bits & ((1ull << lane) - 1ull))] = k;
    }
}

template <bool FULL>
__global__ void __launch_bounds__(256) bnd_jump_first_kernel(int32_t *__restrict__ bnd, int64_t count, TileGrid tg,
                                                             uint32_t *__restrict__ list, int64_t cap,
                                                             uint32_t *__restrict__ counts, uint32_t *flags) {
    __shared__ uint32_t lcount;
    if (threadIdx.x == 0) lcount = 0u;
    __syncthreads();
    uint32_t *mine = list + int64_t(blockIdx.x) * cap;
    const int64_t step = int64_t(gridDim.x) * blockDim.x * BATCH;
    for (int64_t k0 = blockIdx.x * int64_t(blockDim.x) * BATCH + threadIdx.x; k0 < count; k0 += step) {
        int32_t p[BATCH], q[BATCH];
        int64_t s[BATCH];
#pragma unroll
        for (int i = 0; i < BATCH; ++i) {
            const int64_t k = k0 + int64_t(i) * blockDim.x;
            p[i] = k < count ? bnd[k] : 0;
        }
#pragma unroll
        for (int i = 0; i < BATCH; ++i) {
            const int64_t k = k0 + int64_t(i) * blockDim.x;
            // -1 (a root at or below tau) and interior targets (roots) are final
            s[i] = k < count && p[i] >= 0 ? bnd_slot<FULL>(tg, p[i]) : -1;
            q[i] = s[i] >= 0 ? bnd[s[i]] : p[i];
        }
#pragma unroll
        for (int i = 0; i < BATCH; ++i) {
            const int64_t k = k0 + int64_t(i) * blockDim.x;
            bool again = false;
            if (k < count && q[i] != p[i]) {
                bnd[k] = q[i];
                again = q[i] >= 0 && bnd_slot<FULL>(tg, q[i]) >= 0;
            }
            append_active(again, uint32_t(k), mine, &lcount);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        counts[blockIdx.x] = lcount;
        if (lcount) flags[1] = 1u;
    }
}

// Round r >= 1: list_in / counts_in hold round r - 1's active entries, the
// entries still active after this round go to list_out / counts_out.
template <bool FULL>
__global__ void __launch_bounds__(256) bnd_jump_kernel(int32_t *__restrict__ bnd, const uint32_t *__restrict__ list_in,
                                                       const uint32_t *__restrict__ counts_in,
                                                       uint32_t *__restrict__ list_out,
                                                       uint32_t *__restrict__ counts_out, int64_t cap, TileGrid tg,
                                                       uint32_t *flags, int round) {
    if (flags[round] == 0u) return;
    __shared__ uint32_t lcount;
    if (threadIdx.x == 0) lcount = 0u;
    __syncthreads();
    const uint32_t *from = list_in + int64_t(blockIdx.x) * cap;
    uint32_t *mine = list_out + int64_t(blockIdx.x) * cap;
    const int64_t count = counts_in[blockIdx.x];
    for (int64_t j0 = threadIdx.x; j0 < count; j0 += int64_t(blockDim.x) * BATCH) {
        uint32_t k[BATCH];
        int32_t p[BATCH], q[BATCH];
#pragma unroll
        for (int i = 0; i < BATCH; ++i) {
            const int64_t j = j0 + int64_t(i) * blockDim.x;
            k[i] = j < count ? from[j] : 0u;
        }
#pragma unroll
        for (int i = 0; i < BATCH; ++i) {
            const int64_t j = j0 + int64_t(i) * blockDim.x;
            p[i] = j < count ? bnd[k[i]] : -1;
        }
#pragma unroll
        for (int i = 0; i < BATCH; ++i) {
            const int64_t sl = p[i] >= 0 ? bnd_slot<FULL>(tg, p[i]) : -1;
            q[i] = sl >= 0 ? bnd[sl] : p[i];
        }
#pragma unroll
        for (int i = 0; i < BATCH; ++i) {
            const int64_t j = j0 + int64_t(i) * blockDim.x;
            bool again = false;
            if (j < count && q[i] != p[i]) {
                bnd[k[i]] = q[i];
                again = q[i] >= 0 && bnd_slot<FULL>(tg, q[i]) >= 0;
            }
            append_active(again, k[i], mine, &lcount);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        counts_out[blockIdx.x] = lcount;
        if (lcount) flags[round + 1] = 1u;
    }
}

// One workgroup per resolve tile: the resolved boundary entries of the
// one-cell shell around the tile go to LDS (they belong to the neighbouring
// tiles; every exit target of the tile lies in the shell), then every cell of
// the tile maps its pointer: -1 stays -1, a target inside the tile is a root
// above tau, a target in the shell takes the shell's entry.
template <bool FULL>
__global__ void __launch_bounds__(RES_THREADS) seg_finalize_kernel(const int32_t *__restrict__ ptr,
                                                                   const int32_t *__restrict__ bnd, TileGrid rg,
                                                                   int32_t *__restrict__ label) {
    __shared__ int32_t shell[RHCELLS];
    int x0, y0, z0;
    const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
    rtile_origin(rg, int(tile), x0, y0, z0);
    const int n = rg.n;
    const uint32_t un = uint32_t(n);
    const int wx = FULL ? RX : tile_extent(x0, RX, n), wy = FULL ? RY : tile_extent(y0, RY, n),
              wz = FULL ? RZ : tile_extent(z0, RZ, n);
    // this tile's pointers and the shell's entries, all loads issued before any is used
    int32_t t[RES_PER];
#pragma unroll
    for (int i = 0; i < RES_PER; ++i) {
        const int e = i * RES_THREADS + threadIdx.x;
        const int x = e % RX, y = (e / RX) % RY, z = e / (RX * RY);
        t[i] = 0;
        if (x < wx && y < wy && z < wz) t[i] = ptr[((uint32_t(z0 + z) * un) + uint32_t(y0 + y)) * un + uint32_t(x0 + x)];
    }
    // the one-cell shell around the tile's (wx, wy, wz) cells, enumerated: the
    // two z planes, then per inner plane the two y rows and the two x ends of
    // the rows between them; shell cell (hx, hy, hz) sits at LDS place
    // (hz RHY + hy) RHX + hx, with the tile's cells at 1..wx, 1..wy, 1..wz
    const int ex = wx + 2, ey = wy + 2, ez = wz + 2;
    const int zplane = ex * ey, ring = 2 * ex + 2 * (ey - 2);
    const int nshell = 2 * zplane + (ez - 2) * ring;
    constexpr int LOADS = (RHCELLS - RCELLS + RES_THREADS - 1) / RES_THREADS;
    int32_t v[LOADS];
    int at[LOADS];
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
        const int k = threadIdx.x + i * RES_THREADS;
        at[i] = -1;
        if (k >= nshell) continue;
        int hx, hy, hz;
        if (k < 2 * zplane) {
            hz = k < zplane ? 0 : ez - 1;
            const int j = k % zplane;
            hy = j / ex;
            hx = j % ex;
        } else {
            const int j = k - 2 * zplane;
            hz = 1 + j / ring;
            const int r = j % ring;
            if (r < 2 * ex) {
                hy = r < ex ? 0 : ey - 1;
                hx = r % ex;
            } else {
                const int q = r - 2 * ex;
                hy = 1 + q / 2;
                hx = (q & 1) ? ex - 1 : 0;
            }
        }
        const uint32_t gx = wrap(x0 + hx - 1, n), gy = wrap(y0 + hy - 1, n), gz = wrap(z0 + hz - 1, n);
        v[i] = bnd[bnd_slot_at<FULL>(rg, gx, gy, gz)];  // on its tile's boundary
        at[i] = (hz * RHY + hy) * RHX + hx;
    }
#pragma unroll
    for (int i = 0; i < LOADS; ++i)
        if (at[i] >= 0) shell[at[i]] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RES_PER; ++i) {
        const int e = i * RES_THREADS + threadIdx.x;
        const int x = e % RX, y = (e / RX) % RY, z = e / (RX * RY);
        if (x >= wx || y >= wy || z >= wz) continue;
        const uint32_t g = ((uint32_t(z0 + z) * un) + uint32_t(y0 + y)) * un + uint32_t(x0 + x);
        int32_t r = t[i];
        if (r >= 0) {
            uint32_t px, py, pz;
            cell_coords(rg, uint32_t(r), px, py, pz);
            // shell coordinates of the target, periodic
            const int hx = int(wrap(int(px) - x0 + 1, n)), hy = int(wrap(int(py) - y0 + 1, n)),
                      hz = int(wrap(int(pz) - z0 + 1, n));
            const bool inside = hx >= 1 && hx <= wx && hy >= 1 && hy <= wy && hz >= 1 && hz <= wz;
            if (!inside) r = shell[(hz * RHY + hy) * RHX + hx];
        }
        label[g] = r;
    }
}

// ------------------------------------------------------------------ direct path (n % 32 != 0)
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
                best = kmax(best, cell_key(c[j], j, nan));
            }
        }
    }
    return best;
}

__global__ void __launch_bounds__(256) max_direct_kernel(const float *__restrict__ c, int n, float tau,
                                                         uint32_t *__restrict__ mask, uint32_t *status) {
    const uint32_t cells = uint32_t(n) * n * n;
    const uint32_t words = (cells + 31) / 32;
    bool nan = false;
    // one wavefront per 64 consecutive cells: two mask words
    for (uint32_t base = blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < cells;
         base += gridDim.x * blockDim.x) {
        const uint32_t j = base + (threadIdx.x & 63u);
        bool is_max = false;
        if (j < cells) {
            const int x = int(j % uint32_t(n)), y = int((j / uint32_t(n)) % uint32_t(n)),
                      z = int(j / (uint32_t(n) * n));
            const float v = c[j];
            is_max = (v > tau) && cell_key(v, j, nan) > neighbour_max(c, n, x, y, z, nan);
        }
        const unsigned long long bits = __ballot(is_max);
        if ((threadIdx.x & 63) == 0) {
            mask[base >> 5] = uint32_t(bits);
            if ((base >> 5) + 1 < words) mask[(base >> 5) + 1] = uint32_t(bits >> 32);
        }
    }
    if (nan) atomicOr(status, ST_INPUT);
}

// ------------------------------------------------------------------ mask -> sorted list
constexpr int LIST_CHUNK_WORDS = 128;  // 4096 cells per chunk

__global__ void __launch_bounds__(LIST_CHUNK_WORDS) mask_count_kernel(const uint32_t *__restrict__ mask,
                                                                      int64_t words, uint32_t *__restrict__ counts) {
    const int64_t w = int64_t(blockIdx.x) * LIST_CHUNK_WORDS + threadIdx.x;
    uint32_t v = w < words ? uint32_t(__popc(mask[w])) : 0u;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __shared__ uint32_t red[LIST_CHUNK_WORDS / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = red[0] + red[1];
}


__global__ void __launch_bounds__(LIST_CHUNK_WORDS) list_write_kernel(const uint32_t *__restrict__ mask,
                                                                      int64_t words,
                                                                      const uint32_t *__restrict__ offsets,
                                                                      int64_t cap, int32_t *__restrict__ out) {
    __shared__ uint32_t pre[LIST_CHUNK_WORDS];
    const int64_t w = int64_t(blockIdx.x) * LIST_CHUNK_WORDS + threadIdx.x;
    const uint32_t bits0 = w < words ? mask[w] : 0u;
    pre[threadIdx.x] = uint32_t(__popc(bits0));
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t r = 0;
        for (int i = 0; i < LIST_CHUNK_WORDS; ++i) {
            const uint32_t v = pre[i];
            pre[i] = r;
            r += v;
        }
    }
    __syncthreads();
    uint32_t bits = bits0;
    uint32_t r = offsets[blockIdx.x] + pre[threadIdx.x];
    while (bits) {
        const int b = __ffs(bits) - 1;
        bits &= bits - 1;
        if (int64_t(r) < cap) out[r] = int32_t(w * 32 + b);
        ++r;
    }
}

// ------------------------------------------------------------------ host side
bool tiled(int n) { return n % TX == 0; }  // TY, TZ, RY and RZ (8 or 16) divide every multiple of 32

TileGrid tile_grid(int n) { return TileGrid{n, n / TX, n / TY, n / TZ, FastDiv(uint32_t(n))}; }

// True where every resolve tile is whole (n a multiple of 32, hence of 16).
bool all_full(int n) { return n % RX == 0 && n % RY == 0 && n % RZ == 0; }

// Resolve tiles over any n: the last tile along an axis is short where n is
// not a multiple of the tile.
TileGrid resolve_grid(int n) {
    return TileGrid{n, (n + RX - 1) / RX, (n + RY - 1) / RY, (n + RZ - 1) / RZ, FastDiv(uint32_t(n))};
}

int rounds_for(uint64_t count) {
    int k = 0;
    while ((uint64_t(1) << k) < count) ++k;
    return k + 1;  // ceil(log2(longest chain)) rounds, plus one that sees no change
}

struct MaximaLayout {
    size_t mask, counts, offsets, partial, total;
    int64_t words;
    int nchunks;
};

MaximaLayout maxima_layout(int n) {
    MaximaLayout L{};
    const size_t cells = size_t(n) * n * n;
    L.words = int64_t((cells + 31) / 32);
    L.nchunks = int((L.words + LIST_CHUNK_WORDS - 1) / LIST_CHUNK_WORDS);
    size_t off = 0;
    L.mask = off;
    off = align_up(off + sizeof(uint32_t) * size_t(L.words + 2));
    L.counts = off;
    off = align_up(off + sizeof(uint32_t) * L.nchunks);
    L.offsets = off;
    off = align_up(off + sizeof(uint32_t) * (L.nchunks + 1));
    L.partial = off;
    off = align_up(off + sizeof(uint64_t) * SCAN_MAX_GROUPS);
    L.total = off;
    return L;
}

int stride_grid(int64_t work) {
    int64_t g = (work + 255) / 256;
    return int(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

int batched_grid(int64_t work) { return stride_grid((work + BATCH - 1) / BATCH); }

struct SegmentLayout {
    size_t flags, ptr, bnd, list[2], counts[2], total;
    int rounds;
    int64_t nbnd;
    int jump_grid;      // workgroups of every jump round
    int64_t list_cap;   // list entries per workgroup
};

SegmentLayout segment_layout(int n) {
    SegmentLayout L{};
    const uint64_t cells = uint64_t(n) * n * n;
    size_t off = 0;
    L.flags = off;
    {
        const TileGrid rg = resolve_grid(n);
        L.nbnd = int64_t(rg.ntx) * rg.nty * rg.ntz * NBND;
        L.rounds = rounds_for(uint64_t(L.nbnd));
        off = align_up(off + sizeof(uint32_t) * (L.rounds + 2));
        L.ptr = off;
        off = align_up(off + sizeof(int32_t) * cells);
        L.bnd = off;
        off = align_up(off + sizeof(int32_t) * size_t(L.nbnd));
        // every round-0 workgroup visits at most cap entries
        L.jump_grid = batched_grid(L.nbnd);
        const int64_t per_pass = int64_t(L.jump_grid) * 256 * BATCH;
        L.list_cap = (L.nbnd + per_pass - 1) / per_pass * 256 * BATCH;
        for (int b = 0; b < 2; ++b) {  // the active lists of even and odd rounds
            L.list[b] = off;
            off = align_up(off + sizeof(uint32_t) * size_t(L.list_cap) * size_t(L.jump_grid));
            L.counts[b] = off;
            off = align_up(off + sizeof(uint32_t) * size_t(L.jump_grid));
        }
    }
    L.total = off;
    return L;
}


}  // namespace

size_t hf::maxima_ws_bytes(const hf_box &box) { return maxima_layout(box.n).total; }

size_t hf::segment_ws_bytes(const hf_box &box) { return segment_layout(box.n).total; }

namespace {

// Count / scan / write passes: maxima bit mask (in the maxima workspace at w8)
// -> sorted index list and its length.
hf_status mask_to_list(hf_ctx *ctx, const MaximaLayout &L, char *w8, int32_t *max_idx, int64_t max_cap,
                       int64_t *d_count) {
    auto *mask = reinterpret_cast<uint32_t *>(w8 + L.mask);
    auto *counts = reinterpret_cast<uint32_t *>(w8 + L.counts);
    auto *offsets = reinterpret_cast<uint32_t *>(w8 + L.offsets);
    HF_LAUNCH(ctx, K_MAX_COUNT, mask_count_kernel, dim3(L.nchunks), dim3(LIST_CHUNK_WORDS), 0, ctx->stream, mask,
              L.words, counts);
    const ScanJob sj = scan_job(counts, L.nchunks, reinterpret_cast<uint64_t *>(w8 + L.partial), offsets, nullptr,
                                d_count, max_cap, ctx->d_status);
    HF_LAUNCH(ctx, K_MAX_SCAN, seg_reduce_kernel<SCAN_MAXIMA>, dim3(scan_groups(sj)), dim3(SCAN_THREADS), 0,
              ctx->stream, sj);
    HF_LAUNCH(ctx, K_MAX_SCAN, seg_scan_kernel<SCAN_MAXIMA>, dim3(scan_groups(sj)), dim3(SCAN_THREADS), 0, ctx->stream,
              sj);
    HF_LAUNCH(ctx, K_MAX_WRITE, list_write_kernel, dim3(L.nchunks), dim3(LIST_CHUNK_WORDS), 0, ctx->stream, mask,
              L.words, offsets, max_cap, max_idx);
    return launch_status();
}

// Parents (and the maxima mask when given) of a tiled grid, with the chains
// inside each resolve tile followed: ptr and bnd of the segmentation workspace.
hf_status launch_parent_resolve(hf_ctx *ctx, const SegmentLayout &L, char *w8, int n, const float *cwt, float tau,
                                uint32_t *mask) {
    const TileGrid tg = resolve_grid(n);
    const dim3 grid(tg.ntx * tg.nty * tg.ntz);
    auto *ptr = reinterpret_cast<int32_t *>(w8 + L.ptr);
    auto *bnd = reinterpret_cast<int32_t *>(w8 + L.bnd);
    if (all_full(n))
        HF_LAUNCH(ctx, K_PARENT, parent_resolve_kernel<true>, grid, dim3(PR_THREADS), 0, ctx->stream, cwt, tg,
                  host_ordered_bits(tau), ptr, bnd, mask, ctx->d_status);
    else
        HF_LAUNCH(ctx, K_PARENT, parent_resolve_kernel<false>, grid, dim3(PR_THREADS), 0, ctx->stream, cwt, tg,
                  host_ordered_bits(tau), ptr, bnd, mask, ctx->d_status);
    return launch_status();
}

// After launch_parent_resolve: pointer-jumping rounds over the boundary
// entries, and the final mapping through them.
hf_status segment_finish(hf_ctx *ctx, const SegmentLayout &L, char *w8, int n, int32_t *cell_label) {
    const TileGrid tg = resolve_grid(n);
    auto *flags = reinterpret_cast<uint32_t *>(w8 + L.flags);
    auto *ptr = reinterpret_cast<int32_t *>(w8 + L.ptr);
    auto *bnd = reinterpret_cast<int32_t *>(w8 + L.bnd);
    uint32_t *list[2], *counts[2];
    for (int b = 0; b < 2; ++b) {
        list[b] = reinterpret_cast<uint32_t *>(w8 + L.list[b]);
        counts[b] = reinterpret_cast<uint32_t *>(w8 + L.counts[b]);
    }
    const bool full = all_full(n);
    if (full)
        HF_LAUNCH(ctx, K_JUMP, bnd_jump_first_kernel<true>, dim3(L.jump_grid), dim3(256), 0, ctx->stream, bnd,
                  L.nbnd, tg, list[0], L.list_cap, counts[0], flags);
    else
        HF_LAUNCH(ctx, K_JUMP, bnd_jump_first_kernel<false>, dim3(L.jump_grid), dim3(256), 0, ctx->stream, bnd,
                  L.nbnd, tg, list[0], L.list_cap, counts[0], flags);
    for (int r = 1; r < L.rounds; ++r) {
        if (full)
            HF_LAUNCH(ctx, K_JUMP, bnd_jump_kernel<true>, dim3(L.jump_grid), dim3(256), 0, ctx->stream, bnd,
                      list[(r - 1) & 1], counts[(r - 1) & 1], list[r & 1], counts[r & 1], L.list_cap, tg, flags, r);
        else
            HF_LAUNCH(ctx, K_JUMP, bnd_jump_kernel<false>, dim3(L.jump_grid), dim3(256), 0, ctx->stream, bnd,
                      list[(r - 1) & 1], counts[(r - 1) & 1], list[r & 1], counts[r & 1], L.list_cap, tg, flags, r);
    }
    const dim3 grid(tg.ntx * tg.nty * tg.ntz);
    if (full)
        HF_LAUNCH(ctx, K_FINALIZE, seg_finalize_kernel<true>, grid, dim3(RES_THREADS), 0, ctx->stream, ptr, bnd, tg,
                  cell_label);
    else
        HF_LAUNCH(ctx, K_FINALIZE, seg_finalize_kernel<false>, grid, dim3(RES_THREADS), 0, ctx->stream, ptr, bnd, tg,
                  cell_label);
    return launch_status();
}

}  // namespace

size_t hf::maxima_segment_ws_bytes(const hf_box &box) {
    return segment_layout(box.n).total + maxima_layout(box.n).total;
}

// Steps 4 and 5 together: on tiled grids one pass over the field yields both
// the parents and the maxima mask.  Same results as hf_maxima then hf_segment.
hf_status hf::maxima_segment(hf_ctx *ctx, const hf_box &box, const float *cwt, float tau, int32_t *max_idx,
                             int64_t max_cap, int64_t *d_count, int32_t *cell_label, void *ws, size_t ws_bytes) {
    const int n = box.n;
    if (!ctx || !cwt || !d_count || !cell_label || max_cap < 0 || (max_cap > 0 && !max_idx) || tau != tau)
        return HF_ERR_ARG;
    const SegmentLayout SL = segment_layout(n);
    const MaximaLayout ML = maxima_layout(n);
    hf_status s = check_ws(ws, ws_bytes, SL.total + ML.total);
    if (s != HF_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    char *w8 = static_cast<char *>(ws);
    char *wm = w8 + SL.total;
    auto *flags = reinterpret_cast<uint32_t *>(w8 + SL.flags);
    HF_LAUNCH(ctx, K_FLAGS, fill_flags_kernel, dim3((SL.rounds + 2 + 255) / 256), dim3(256), 0, ctx->stream, flags,
              SL.rounds + 2);
    auto *mask = reinterpret_cast<uint32_t *>(wm + ML.mask);
    if (n % 32 != 0)  // rows straddle mask words: the maxima are set bit by bit into a cleared mask
        HF_LAUNCH(ctx, K_FLAGS, zero_words_kernel, dim3(stride_grid(ML.words)), dim3(256), 0, ctx->stream, mask,
                  ML.words);
    s = launch_parent_resolve(ctx, SL, w8, n, cwt, tau, mask);
    if (s != HF_OK) return s;
    s = mask_to_list(ctx, ML, wm, max_idx, max_cap, d_count);
    if (s != HF_OK) return s;
    return segment_finish(ctx, SL, w8, n, cell_label);
}

extern "C" hf_status hf_maxima(hf_ctx *ctx, const hf_box *box, const float *cwt, float tau, int32_t *max_idx,
                               int64_t max_cap, int64_t *d_count, void *ws, size_t ws_bytes) {
    if (!ctx || !cwt || !d_count || max_cap < 0 || (max_cap > 0 && !max_idx)) return HF_ERR_ARG;
    if (tau != tau) return HF_ERR_ARG;
    hf_status s = check_box_grid(box);
    if (s != HF_OK) return s;
    const MaximaLayout L = maxima_layout(box->n);
    s = check_ws(ws, ws_bytes, L.total);
    if (s != HF_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    char *w8 = static_cast<char *>(ws);
    auto *mask = reinterpret_cast<uint32_t *>(w8 + L.mask);
    const int n = box->n;
    if (tiled(n)) {
        const TileGrid tg = tile_grid(n);
        HF_LAUNCH(ctx, K_MAX_MARK, max_tile_kernel, dim3(tg.ntx * tg.nty * tg.ntz), dim3(SEG_THREADS), 0,
                  ctx->stream, cwt, tg, host_ordered_bits(tau), mask, ctx->d_status);
    } else {
        const int64_t cells = int64_t(n) * n * n;
        HF_LAUNCH(ctx, K_MAX_MARK, max_direct_kernel, dim3(stride_grid(cells)), dim3(256), 0, ctx->stream, cwt, n,
                  tau, mask, ctx->d_status);
    }
    return mask_to_list(ctx, L, w8, max_idx, max_cap, d_count);
}

extern "C" hf_status hf_segment(hf_ctx *ctx, const hf_box *box, const float *cwt, float tau, int32_t *cell_label,
                                void *ws, size_t ws_bytes) {
    if (!ctx || !cwt || !cell_label) return HF_ERR_ARG;
    if (tau != tau) return HF_ERR_ARG;
    hf_status s = check_box_grid(box);
    if (s != HF_OK) return s;
    const SegmentLayout L = segment_layout(box->n);
    s = check_ws(ws, ws_bytes, L.total);
    if (s != HF_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    char *w8 = static_cast<char *>(ws);
    auto *flags = reinterpret_cast<uint32_t *>(w8 + L.flags);
    const int n = box->n;
    HF_LAUNCH(ctx, K_FLAGS, fill_flags_kernel, dim3((L.rounds + 2 + 255) / 256), dim3(256), 0, ctx->stream, flags,
              L.rounds + 2);
    s = launch_parent_resolve(ctx, L, w8, n, cwt, tau, nullptr);
    if (s != HF_OK) return s;
    return segment_finish(ctx, L, w8, n, cell_label);
}
