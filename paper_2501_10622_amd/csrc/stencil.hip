// Step 3 by the paper's own discretisation (Sec. 2.1): the grid CWT as the
// superposition, around every grid point, of the wavelet of Eq. (4) sampled at
// the grid spacing on the cube of node offsets |d_i| <= h (h = Table 1's
// gdw_resolution by default), periodically wrapped on the box.
//
// On a cube of offsets the sampled wavelet is a sum of separable terms.  With
// u = (w dx d)^2 per axis, A(d) = exp(-u/4), B(d) = u A(d) and P = dx^3 w^1.5,
//   dx^3 Psi(w, d dx) = P [6 A_x A_y A_z - B_x A_y A_z - A_x B_y A_z - A_x A_y B_z],
// so the (2h+1)^3-point superposition equals seven one-dimensional periodic
// convolutions of 2h+1 taps, made in three streaming passes over the grid:
//   x pass:  fA = A * rho,  fB = B * rho                (cell-mass units)
//   y pass:  G = A * fA,    S = 6 G - A * fB - B * fA
//   z pass:  C = (P / mean) (A * S - B * G)
// Each pass reads its lines (plus h cells of halo at each end) into LDS, with
// several loads in flight per lane, and every output sums its taps in pairs
// d, -d.  The mean cell mass comes from the exact 128-bit total of rho, reduced
// in FP64 between the x and y passes.  (A fused x-y pass over 2D tiles, which
// keeps fA and fB in LDS, measured slower than the two passes.)
#include <cmath>

#include "hf_internal.h"

using namespace hf;

namespace {

constexpr int ST_THREADS = 256;
constexpr int ST_LANES = 64;          // x columns of a y- or z-pass tile (one wavefront row)
constexpr int ST_GROUPS = 8;          // wavefront rows of a y- or z-pass workgroup
constexpr int ST_AX_THREADS = ST_LANES * ST_GROUPS;
constexpr int ST_K = 8;               // outputs per thread along the pass axis
constexpr int ST_T = ST_GROUPS * ST_K;  // outputs along the pass axis per tile

__host__ __device__ inline int stencil_pad(int h) { return (h + ST_K - 1) / ST_K * ST_K; }

// An x-pass row buffer holds slots q = 0 .. n + 2 hp - 1 (input x = q - hp,
// periodic) as ST_K rows of blocks: slot q at (q mod ST_K) LB + q / ST_K + 1,
// so a lane that owns the outputs of one block reads every window element at
// an address one above its left neighbour's.  Block 0 and the last block are
// spare (read by window refills that no output uses), and LB = 8 mod 64 keeps
// the staging writes of 64 consecutive slots on 64 distinct banks.
__host__ __device__ inline int xrow_blocks(int n, int hp) {
    const int nb = (n + ST_K - 1) / ST_K + 2 * hp / ST_K + 2;
    return nb + (72 - nb % 64) % 64;
}

struct StencilLayout {
    size_t scalars, mass, g0, g1, g2, total;
    int64_t xblocks;
    int xrows;
};

StencilLayout stencil_layout(int n) {
    StencilLayout L{};
    // rows enough for about two output blocks per thread, and at most 64 KB of
    // row buffers at the widest stencil
    const int64_t rows = int64_t(n) * n;
    const int64_t lanes = (n + ST_K - 1) / ST_K;
    const int64_t row_floats = int64_t(ST_K) * xrow_blocks(n, stencil_pad(HF_STENCIL_MAX_HALF_WIDTH));
    int64_t per = (2 * ST_THREADS + lanes - 1) / lanes;
    if (per > 16384 / row_floats) per = 16384 / row_floats;
    L.xrows = int(per < 1 ? 1 : (per < rows ? per : rows));
    L.xblocks = (rows + L.xrows - 1) / L.xrows;
    const size_t grid = sizeof(float) * size_t(n) * size_t(n) * size_t(n);
    size_t off = 0;
    L.scalars = off;
    off = align_up(off + 2 * sizeof(double));
    L.mass = off;
    off = align_up(off + sizeof(Mass128) * size_t(L.xblocks));
    L.g0 = off;
    off = align_up(off + grid);
    L.g1 = off;
    off = align_up(off + grid);
    L.g2 = off;
    off = align_up(off + grid);
    L.total = off;
    return L;
}

// A(d) and B(d) for d = 0..h into LDS, in FP64 rounded once to FP32.
__device__ __forceinline__ void stencil_weights(float *wa, float *wb, int h, double wdx) {
    for (int d = threadIdx.x; d <= h; d += blockDim.x) {
        const double t = wdx * double(d);
        const double u = t * t;
        const double a = exp(-0.25 * u);
        wa[d] = float(a);
        wb[d] = float(u * a);
    }
}

__device__ __forceinline__ int wrap(int t, int n) {
    t %= n;
    return t < 0 ? t + n : t;
}

// wrap with a fast path for the common in-range index
__device__ __forceinline__ int wrapq(int t, int n) { return unsigned(t) < unsigned(n) ? t : wrap(t, n); }

constexpr int LOAD_BATCH = 4;  // rows whose loads are issued together before any is used

// Workgroup sum of the threads' 128-bit masses, in a fixed order, to *out.
__device__ __forceinline__ void block_mass(unsigned long long lo, unsigned long long hi, Mass128 *out) {
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long olo = __shfl_down(lo, off, 64);
        const unsigned long long ohi = __shfl_down(hi, off, 64);
        add128(lo, hi, olo);
        hi += ohi;
    }
    __shared__ unsigned long long red_lo[ST_THREADS / 64], red_hi[ST_THREADS / 64];
    if ((threadIdx.x & 63) == 0) {
        red_lo[threadIdx.x >> 6] = lo;
        red_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long L = 0, H = 0;
        for (int w = 0; w < ST_THREADS / 64; ++w) {
            add128(L, H, red_lo[w]);
            H += red_hi[w];
        }
        out->lo = L;
        out->hi = H;
    }
}

// x pass: xrows whole rows per workgroup; row r of the grid (r = z n + y) is
// read once with hp cells of periodic halo on either side into a row buffer
// (xrow_blocks).  Each thread then makes the ST_K outputs of one block of a
// row from two register windows that move one slot per tap, as the y and z
// passes do (taps past h weigh 0), and every output adds its taps in the
// order of a plain loop over d.
__global__ void __launch_bounds__(ST_THREADS)
    stencil_x_kernel(const int64_t *__restrict__ rho, float *__restrict__ fa, float *__restrict__ fb,
                     Mass128 *__restrict__ mass, int n, int h, int xrows, double wdx, uint32_t *status) {
    extern __shared__ float sm[];
    const int hp = stencil_pad(h);
    float *wa = sm, *wb = sm + (hp + 1);
    float *buf = sm + 2 * (hp + 1);
    const int LB = xrow_blocks(n, hp), RF = ST_K * LB;
    const int tid = threadIdx.x;
    const int W = n + 2 * hp;
    const int64_t nrows = int64_t(n) * n;
    const int64_t row0 = int64_t(blockIdx.x) * xrows;
    const int rows = int(nrows - row0 < xrows ? nrows - row0 : xrows);
    stencil_weights(wa, wb, h, wdx);
    for (int d = h + 1 + tid; d <= hp; d += ST_THREADS) wa[d] = wb[d] = 0.0f;
    unsigned long long lo = 0, hi = 0;
    bool neg = false;
    // the rows' slots as one run of rows * W, LOAD_BATCH loads in flight per thread
    const int slots = rows * W;
    for (int s0 = tid; s0 < slots; s0 += ST_THREADS * LOAD_BATCH) {
        int64_t v[LOAD_BATCH];
#pragma unroll
        for (int u = 0; u < LOAD_BATCH; ++u) {
            const int sl = s0 + u * ST_THREADS;
            v[u] = 0;
            if (sl < slots) {
                const int r = sl / W, q = sl - r * W;
                v[u] = rho[(row0 + r) * n + wrapq(q - hp, n)];
            }
        }
#pragma unroll
        for (int u = 0; u < LOAD_BATCH; ++u) {
            const int sl = s0 + u * ST_THREADS;
            if (sl < slots) {
                const int r = sl / W, q = sl - r * W;
                if (q >= hp && q < hp + n) {  // each cell counted once, from its own slot
                    neg |= v[u] < 0;
                    add128(lo, hi, static_cast<unsigned long long>(v[u]));
                }
                buf[r * RF + (q % ST_K) * LB + q / ST_K + 1] = float(v[u]);
            }
        }
    }
    if (neg) atomicOr(status, ST_INPUT);
    block_mass(lo, hi, mass + blockIdx.x);  // its barrier also publishes the row buffers
    const float a0 = wa[0];
    const int lanes = (n + ST_K - 1) / ST_K;
    for (int w = tid; w < rows * lanes; w += ST_THREADS) {
        const int r = w / lanes, l = w - r * lanes;
        // slot qb + j (qb = ST_K l + hp, j >= -ST_K) at ((j + ST_K) mod ST_K) LB + qk + (j + ST_K) / ST_K
        const float *row = buf + r * RF;
        const int qk = l + hp / ST_K;  // qb / ST_K
        float sa[ST_K], sb[ST_K];
#pragma unroll
        for (int k = 0; k < ST_K; ++k) {
            sa[k] = a0 * row[k * LB + qk + 1];
            sb[k] = 0.0f;  // B(0) = 0
        }
        if (hp > 0) {
            // windows for d = 1: up[j % ST_K] = slot qb + j (j = 1 .. ST_K),
            // lo[(j + ST_K) % ST_K] = slot qb + j (j = -1 .. ST_K - 2)
            float up[ST_K], dn[ST_K];
#pragma unroll
            for (int j = 1; j <= ST_K; ++j) up[j % ST_K] = row[(j % ST_K) * LB + qk + 1 + j / ST_K];
#pragma unroll
            for (int j = -1; j < ST_K - 1; ++j)
                dn[(j + ST_K) % ST_K] = row[((j + ST_K) % ST_K) * LB + qk + (j + ST_K) / ST_K];
            for (int b8 = 0; b8 < hp / ST_K; ++b8) {
#pragma unroll
                for (int s = 0; s < ST_K; ++s) {
                    const int d = b8 * ST_K + s + 1;
                    const float wad = wa[d], wbd = wb[d];
#pragma unroll
                    for (int k = 0; k < ST_K; ++k) {
                        const float v = up[(k + s + 1) % ST_K] + dn[(k - s - 1 + 2 * ST_K) % ST_K];
                        sa[k] = fmaf(wad, v, sa[k]);
                        sb[k] = fmaf(wbd, v, sb[k]);
                    }
                    // slot qb + d + ST_K into up, slot qb - d - 1 into dn
                    up[(s + 1) % ST_K] = row[((s + 1) % ST_K) * LB + qk + b8 + 2 + (s + 1) / ST_K];
                    dn[(2 * ST_K - s - 2) % ST_K] =
                        row[((2 * ST_K - s - 2) % ST_K) * LB + qk - b8 - (s == ST_K - 1 ? 1 : 0)];
                }
            }
        }
        float *oa = fa + (row0 + r) * n, *ob = fb + (row0 + r) * n;
#pragma unroll
        for (int k = 0; k < ST_K; ++k) {
            const int x = ST_K * l + k;
            if (x < n) {
                oa[x] = sa[k];
                ob[x] = sb[k];
            }
        }
    }
}

// Mean cell mass from the exact partial sums; scalars[0] = P / mean.
__global__ void __launch_bounds__(1024)
    stencil_mass_kernel(const Mass128 *__restrict__ mass, int64_t nparts, int n, double pref, double *scalars,
                        uint32_t *status) {
    __shared__ unsigned long long red_lo[16], red_hi[16];
    unsigned long long lo = 0, hi = 0;
    constexpr int U = 8;  // partial sums in flight per thread
    const int64_t step = int64_t(blockDim.x) * U;
    int64_t i0 = threadIdx.x;
    for (; i0 + (U - 1) * int64_t(blockDim.x) < nparts; i0 += step) {
        Mass128 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = mass[i0 + u * int64_t(blockDim.x)];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            add128(lo, hi, v[u].lo);
            hi += v[u].hi;
        }
    }
    for (int64_t i = i0; i < nparts; i += blockDim.x) {
        add128(lo, hi, mass[i].lo);
        hi += mass[i].hi;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long olo = __shfl_down(lo, off, 64);
        const unsigned long long ohi = __shfl_down(hi, off, 64);
        add128(lo, hi, olo);
        hi += ohi;
    }
    if ((threadIdx.x & 63) == 0) {
        red_lo[threadIdx.x >> 6] = lo;
        red_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long L = 0, H = 0;
        for (int w = 0; w < int(blockDim.x >> 6); ++w) {
            add128(L, H, red_lo[w]);
            H += red_hi[w];
        }
        const double cells = double(n) * double(n) * double(n);
        const double mbar = u128_to_double(L, H) / cells;
        if (!(mbar > 0.0)) {
            atomicOr(status, ST_INPUT);
            scalars[0] = 0.0;
        } else {
            scalars[0] = pref / mbar;
        }
        scalars[1] = mbar;
    }
}

// y (ZPASS false, axis stride n) and z (ZPASS true, axis stride n^2) passes.
// A tile is ST_LANES x columns by ST_T outputs along the axis at one value of
// the third coordinate; it reads ST_T + 2 hp lines of both inputs into LDS,
// hp = h rounded up to ST_K (taps past h weigh 0), with one spare line at each
// end that the last tap's window refill may read but no output uses.  Tiles that neighbour along
// the axis (and share halo lines) are consecutive logical blocks, which
// xcd_remap keeps on one XCD.
//
// Each thread makes ST_K consecutive outputs along the axis.  For tap d they
// need the inputs at k + d and k - d (k < ST_K): two windows of ST_K values per
// input, kept in registers, that move by one line per tap, so a tap costs two
// LDS reads per input instead of 2 ST_K.  The tap loop is unrolled by ST_K,
// which turns each window's rotation into fixed register names.  Every output
// adds its taps in the same order as a plain loop over d would.

template <bool ZPASS>
__global__ void __launch_bounds__(ST_AX_THREADS)
    stencil_axis_kernel(const float *__restrict__ in0, const float *__restrict__ in1, float *__restrict__ out0,
                        float *__restrict__ out1, const double *__restrict__ scalars, int n, int h, int tiles_x,
                        int tiles_t, double wdx) {
    extern __shared__ float sm[];
    const int hp = stencil_pad(h);
    const int R = ST_T + 2 * hp;  // lines read (the spare lines are not loaded)
    float *wa = sm, *wb = sm + (hp + 1);
    float *b0 = sm + 2 * (hp + 1) + ST_LANES;  // line -1 is spare, so is line R
    float *b1 = b0 + (R + 2) * ST_LANES;
    const uint32_t lt = xcd_remap(blockIdx.x, gridDim.x);
    const int tt = int(lt % uint32_t(tiles_t));
    const uint32_t rest = lt / uint32_t(tiles_t);
    const int tx = int(rest % uint32_t(tiles_x));
    const int o = int(rest / uint32_t(tiles_x));
    const int lane = threadIdx.x % ST_LANES, grp = threadIdx.x / ST_LANES;
    const int x = tx * ST_LANES + lane;
    const int t0 = tt * ST_T;
    const size_t sn = size_t(n);
    // element (x, t, o): y pass (z = o, y = t), z pass (z = t, y = o)
    auto at = [sn, x, o](int t) -> size_t {
        return ZPASS ? (size_t(t) * sn + size_t(o)) * sn + size_t(x) : (size_t(o) * sn + size_t(t)) * sn + size_t(x);
    };
    stencil_weights(wa, wb, h, wdx);
    for (int d = h + 1 + int(threadIdx.x); d <= hp; d += ST_AX_THREADS) wa[d] = wb[d] = 0.0f;
    if (x < n) {
        constexpr int UB = 4 * LOAD_BATCH;  // 2 UB loads in flight per lane
        for (int rb = grp; rb < R; rb += ST_GROUPS * UB) {
            float v0[UB], v1[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const int r = rb + u * ST_GROUPS;
                v0[u] = v1[u] = 0.0f;
                if (r < R) {
                    const size_t e = at(wrapq(t0 - hp + r, n));
                    v0[u] = in0[e];
                    v1[u] = in1[e];
                }
            }
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const int r = rb + u * ST_GROUPS;
                if (r < R) {
                    b0[r * ST_LANES + lane] = v0[u];
                    b1[r * ST_LANES + lane] = v1[u];
                }
            }
        }
    }
    __syncthreads();
    if (x >= n) return;
    const int k0 = grp * ST_K;
    // line j of these is the input at axis offset t0 + k0 + j
    const float *c0 = b0 + (k0 + hp) * ST_LANES + lane;
    const float *c1 = b1 + (k0 + hp) * ST_LANES + lane;
    const float a0 = wa[0];
    float acc0[ST_K], acc1[ST_K], acc2[ST_K];  // y: G, A*fB, B*fA;  z: A*S, B*G
#pragma unroll
    for (int k = 0; k < ST_K; ++k) {
        acc0[k] = ZPASS ? a0 * c1[k * ST_LANES] : a0 * c0[k * ST_LANES];
        acc1[k] = ZPASS ? 0.0f : a0 * c1[k * ST_LANES];
        acc2[k] = 0.0f;
    }
    if (hp > 0) {
        // windows for d = 1: up[j % ST_K] = line j (j = d .. d + ST_K - 1),
        // lo[j % ST_K] = line j (j = -d .. ST_K - 1 - d)
        float up0[ST_K], lo0[ST_K], up1[ST_K], lo1[ST_K];
#pragma unroll
        for (int j = 1; j <= ST_K; ++j) {
            up0[j % ST_K] = c0[j * ST_LANES];
            up1[j % ST_K] = c1[j * ST_LANES];
        }
#pragma unroll
        for (int j = -1; j < ST_K - 1; ++j) {
            lo0[(j + ST_K) % ST_K] = c0[j * ST_LANES];
            lo1[(j + ST_K) % ST_K] = c1[j * ST_LANES];
        }
        for (int d8 = 0; d8 < hp; d8 += ST_K) {
#pragma unroll
            for (int s = 0; s < ST_K; ++s) {
                const int d = d8 + s + 1;
                const float wad = wa[d], wbd = wb[d];
#pragma unroll
                for (int k = 0; k < ST_K; ++k) {
                    const float s0 = up0[(k + s + 1) % ST_K] + lo0[(k - s - 1 + 2 * ST_K) % ST_K];
                    const float s1 = up1[(k + s + 1) % ST_K] + lo1[(k - s - 1 + 2 * ST_K) % ST_K];
                    if (!ZPASS) {
                        acc0[k] = fmaf(wad, s0, acc0[k]);
                        acc1[k] = fmaf(wad, s1, acc1[k]);
                        acc2[k] = fmaf(wbd, s0, acc2[k]);
                    } else {
                        acc0[k] = fmaf(wad, s1, acc0[k]);
                        acc2[k] = fmaf(wbd, s0, acc2[k]);
                    }
                }
                // move both windows one line outwards (after the last tap this
                // reads a spare line or the neighbouring group's, unused)
                up0[(s + 1) % ST_K] = c0[(d + ST_K) * ST_LANES];
                up1[(s + 1) % ST_K] = c1[(d + ST_K) * ST_LANES];
                lo0[(ST_K - 2 - s + ST_K) % ST_K] = c0[(-d - 1) * ST_LANES];
                lo1[(ST_K - 2 - s + ST_K) % ST_K] = c1[(-d - 1) * ST_LANES];
            }
        }
    }
    const double factor = ZPASS ? scalars[0] : 0.0;
#pragma unroll
    for (int k = 0; k < ST_K; ++k) {
        const int t = t0 + k0 + k;
        if (t >= n) break;
        const size_t e = at(t);
        if (!ZPASS) {
            // in0 = fA, in1 = fB: G = A*fA, S = 6 G - A*fB - B*fA
            out0[e] = acc0[k];
            out1[e] = 6.0f * acc0[k] - acc1[k] - acc2[k];
        } else {
            // in0 = G, in1 = S: C = (P / mean) (A*S - B*G)
            out0[e] = float(double(acc0[k] - acc2[k]) * factor);
        }
    }
}

}  // namespace

size_t hf::stencil_ws_bytes(const hf_box &box) { return stencil_layout(box.n).total; }

extern "C" hf_status hf_stencil_half_width(double kw, int32_t n, int32_t *half_width) {
    if (!half_width || !(kw > 0.0) || !std::isfinite(kw) || n < 1 || n > 1024) return HF_ERR_ARG;
    const int32_t h = stencil_half_width(kw, n);
    if (h < 0) return HF_ERR_ARG;
    *half_width = h;
    return HF_OK;
}

extern "C" hf_status hf_cwt_stencil(hf_ctx *ctx, const hf_box *box, const int64_t *rho, double kw,
                                    int32_t half_width, float *cwt, void *ws, size_t ws_bytes) {
    if (!ctx || !rho || !cwt) return HF_ERR_ARG;
    if (!(kw > 0.0) || !std::isfinite(kw)) return HF_ERR_ARG;
    if (half_width < 0 || half_width > HF_STENCIL_MAX_HALF_WIDTH) return HF_ERR_ARG;
    hf_status s = check_box_grid(box);
    if (s != HF_OK) return s;
    const int n = box->n, h = half_width;
    const StencilLayout L = stencil_layout(n);
    s = check_ws(ws, ws_bytes, L.total);
    if (s != HF_OK) return s;
    const double dx = box->box_len / n;
    const double w = 1000.0 * kw / box->box_len;
    const double wdx = w * dx;
    const double pref = dx * dx * dx * std::pow(w, 1.5);
    if (!std::isfinite(wdx) || !(pref > 0.0) || !std::isfinite(pref)) return HF_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    char *b = static_cast<char *>(ws);
    double *scalars = reinterpret_cast<double *>(b + L.scalars);
    Mass128 *mass = reinterpret_cast<Mass128 *>(b + L.mass);
    float *g0 = reinterpret_cast<float *>(b + L.g0);
    float *g1 = reinterpret_cast<float *>(b + L.g1);
    float *g2 = reinterpret_cast<float *>(b + L.g2);
    const size_t x_shm =
        sizeof(float) * (2 * size_t(stencil_pad(h) + 1) + size_t(L.xrows) * ST_K * size_t(xrow_blocks(n, stencil_pad(h))));
    const size_t a_shm =
        sizeof(float) * (2 * size_t(stencil_pad(h) + 1) + ST_LANES + 2 * size_t(ST_T + 2 * stencil_pad(h) + 2) * ST_LANES);
    auto allow = [](const void *f, size_t bytes) {
        return bytes <= 65536 ||
               hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)) == hipSuccess;
    };
    if (!allow(reinterpret_cast<const void *>(&stencil_x_kernel), x_shm) ||
        !allow(reinterpret_cast<const void *>(&stencil_axis_kernel<false>), a_shm) ||
        !allow(reinterpret_cast<const void *>(&stencil_axis_kernel<true>), a_shm))
        return HF_ERR_DEVICE;
    const int tiles_x = (n + ST_LANES - 1) / ST_LANES;
    const int tiles_t = (n + ST_T - 1) / ST_T;
    const unsigned tiles = unsigned(tiles_x) * unsigned(tiles_t) * unsigned(n);
    hipStream_t st = ctx->stream;
    // x pass: fA -> g0, fB -> cwt (the output doubles as the x pass's second field)
    HF_LAUNCH(ctx, K_ST_X, stencil_x_kernel, dim3(unsigned(L.xblocks)), dim3(ST_THREADS), x_shm, st, rho, g0, cwt,
              mass, n, h, L.xrows, wdx, ctx->d_status);
    HF_LAUNCH(ctx, K_ST_MASS, stencil_mass_kernel, dim3(1), dim3(1024), 0, st, mass, L.xblocks, n, pref, scalars,
              ctx->d_status);
    // y pass: (fA, fB) -> (G -> g1, S -> g2)
    HF_LAUNCH(ctx, K_ST_Y, stencil_axis_kernel<false>, dim3(tiles), dim3(ST_AX_THREADS), a_shm, st, g0, cwt, g1, g2,
              scalars, n, h, tiles_x, tiles_t, wdx);
    // z pass: (G, S) -> C
    HF_LAUNCH(ctx, K_ST_Z, stencil_axis_kernel<true>, dim3(tiles), dim3(ST_AX_THREADS), a_shm, st, g1, g2, cwt, nullptr,
              scalars, n, h, tiles_x, tiles_t, wdx);
    return launch_status();
}
