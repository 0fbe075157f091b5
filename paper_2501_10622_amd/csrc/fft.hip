// Step 3 (Eqs. (2)-(4)): the grid CWT as a real 3D FFT, a multiply by the
// wavelet's DFT-domain multiplier, and an inverse FFT, all in FP32 with
// FP64 only for the mean density and for table generation.
//
// Data flow (n^3 grid, H = n/2 + 1, half spectrum S complex64 stored in tiles
// of YZ_TILE columns, see spec_tile):
//   x_fwd   : rows of int64 rho -> float, two real rows packed as one complex
//             row, complex FFT along x, split into two half-spectrum rows;
//             also the exact 128-bit mass of the rows.
//   mass    : sums the row masses, mean density in FP64 -> overall scale.
//   y_pass  : complex FFT along y on tiles of YZ_TILE columns (forward).
//   z_mul   : forward FFT along z, times the multiplier and the scale,
//             inverse FFT along z, in LDS (one HBM round trip).
//   y_pass  : inverse along y.
//   x_inv   : two half-spectrum rows -> one complex row, inverse FFT, the
//             real and imaginary parts are the two output rows.
// Every 1D transform is a Stockham autosort FFT over radices 16/8/4/3/2 on a
// tile of pencils in LDS (element x of pencil p at row x, column p); the
// y and z passes read their first stage straight from HBM into registers and
// write their last stage straight back, and the z pass turns from forward to
// inverse in registers.
#include <cmath>

#include "hf_internal.h"

using namespace hf;

namespace {

constexpr int MAX_STAGES = 12;
constexpr int MAX_ELEMS = 16;  // complex values per thread per stage
constexpr int YZ_LOG = 3;
constexpr int YZ_TILE = 1 << YZ_LOG;  // pencils per workgroup in the y and z passes

// The half spectrum in HBM, in tiles of YZ_TILE columns: element (kx, y, z) of
// an n^3 grid at spec_at(n, kx / YZ_TILE, z, y) + kx % YZ_TILE.  A tile is an
// [z][y][column] block whose z planes are n + 1 rows apart, and tiles are
// n (n + 1) + 1 rows apart.  A y-pass tile (YZ_TILE columns at one z) is one
// contiguous run of n * YZ_TILE elements, a z-pass tile's elements are
// (n + 1) YZ_TILE apart inside one tile, and the x passes move YZ_TILE-column
// blocks of consecutive rows.  The spare rows keep those strides off powers of
// two, which would put a workgroup's accesses on few HBM channels.  Columns
// H .. tiles * YZ_TILE - 1 and the spare rows are padding that no pass reads.
__host__ __device__ inline int spec_tiles(int n) { return (n / 2 + 1 + YZ_TILE - 1) / YZ_TILE; }

__host__ __device__ inline size_t spec_tile_rows(int n) { return size_t(n) * (n + 1) + 1; }

__device__ __forceinline__ size_t spec_at(int n, int tile, int z, int y) {
    return (size_t(tile) * spec_tile_rows(n) + size_t(z) * (n + 1) + size_t(y)) * YZ_TILE;
}



struct FftPlan {
    int n;
    int nst;
    int radix[MAX_STAGES];
    FastDiv ns[MAX_STAGES];  // product of the radices before each stage
    FastDiv dn, dh;          // division by n and by n/2 + 1
};

FftPlan make_plan(int n) {
    FftPlan p{};
    p.n = n;
    p.dn = FastDiv(uint32_t(n));
    p.dh = FastDiv(uint32_t(n / 2 + 1));
    int m = n;
    while (m % 3 == 0) {
        p.radix[p.nst++] = 3;
        m /= 3;
    }
    for (int r : {16, 8, 4, 2})
        while (m % r == 0) {
            p.radix[p.nst++] = r;
            m /= r;
        }
    int ns = 1;
    for (int s = 0; s < p.nst; ++s) {
        p.ns[s] = FastDiv(uint32_t(ns));
        ns *= p.radix[s];
    }
    return p;
}

// The same factors with the last one moved to the front: the inverse transform
// that follows a forward one in registers starts with the radix the forward
// one ended with.
FftPlan rotate_plan(const FftPlan &f) {
    FftPlan p = f;
    p.radix[0] = f.radix[f.nst - 1];
    for (int s = 1; s < f.nst; ++s) p.radix[s] = f.radix[s - 1];
    int ns = 1;
    for (int s = 0; s < p.nst; ++s) {
        p.ns[s] = FastDiv(uint32_t(ns));
        ns *= p.radix[s];
    }
    return p;
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2 &a, float2 &b) {
    float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2 &v0, float2 &v1, float2 &v2, float2 &v3) {
    float2 t0 = cadd(v0, v2), t1 = csub(v0, v2);
    float2 t2 = cadd(v1, v3), t3 = mul_mi<INV>(csub(v1, v3));
    v0 = cadd(t0, t2);
    v2 = csub(t0, t2);
    v1 = cadd(t1, t3);
    v3 = csub(t1, t3);
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
    if constexpr (R == 2) {
        dft2<INV>(v[0], v[1]);
    } else if constexpr (R == 4) {
        dft4<INV>(v[0], v[1], v[2], v[3]);
    } else if constexpr (R == 8) {
        // radix-8 as two radix-4 transforms of the even and odd inputs
        float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
        dft4<INV>(e0, e1, e2, e3);
        dft4<INV>(o0, o1, o2, o3);
        const float r = 0.70710678118654752440f;
        // o_s *= exp(-+ 2 pi i s / 8)
        o1 = INV ? make_float2(r * (o1.x - o1.y), r * (o1.x + o1.y)) : make_float2(r * (o1.x + o1.y), r * (o1.y - o1.x));
        o2 = mul_mi<INV>(o2);
        o3 = INV ? make_float2(-r * (o3.x + o3.y), r * (o3.x - o3.y)) : make_float2(r * (o3.y - o3.x), -r * (o3.x + o3.y));
        v[0] = cadd(e0, o0);
        v[4] = csub(e0, o0);
        v[1] = cadd(e1, o1);
        v[5] = csub(e1, o1);
        v[2] = cadd(e2, o2);
        v[6] = csub(e2, o2);
        v[3] = cadd(e3, o3);
        v[7] = csub(e3, o3);
    } else if constexpr (R == 16) {
        // 16 = 4 x 4: element 4 a + b; length-4 transforms over a, the twiddles
        // W16^(b c), length-4 transforms over b; output c + 4 d sits at 4 c + d
        dft4<INV>(v[0], v[4], v[8], v[12]);
        dft4<INV>(v[1], v[5], v[9], v[13]);
        dft4<INV>(v[2], v[6], v[10], v[14]);
        dft4<INV>(v[3], v[7], v[11], v[15]);
        const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f, h = 0.70710678118654752440f;
        const float sg = INV ? 1.f : -1.f;  // exp(-+ 2 pi i m / 16) = cos - + i sin
        v[5] = cmul(v[5], make_float2(c1, sg * s1));     // m = 1
        v[9] = cmul(v[9], make_float2(h, sg * h));       // m = 2
        v[13] = cmul(v[13], make_float2(s1, sg * c1));   // m = 3
        v[6] = cmul(v[6], make_float2(h, sg * h));       // m = 2
        v[10] = mul_mi<INV>(v[10]);                      // m = 4
        v[14] = cmul(v[14], make_float2(-h, sg * h));    // m = 6
        v[7] = cmul(v[7], make_float2(s1, sg * c1));     // m = 3
        v[11] = cmul(v[11], make_float2(-h, sg * h));    // m = 6
        v[15] = cmul(v[15], make_float2(-c1, -sg * s1)); // m = 9
        dft4<INV>(v[0], v[1], v[2], v[3]);
        dft4<INV>(v[4], v[5], v[6], v[7]);
        dft4<INV>(v[8], v[9], v[10], v[11]);
        dft4<INV>(v[12], v[13], v[14], v[15]);
        float2 t[16];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int d = 0; d < 4; ++d) t[c + 4 * d] = v[4 * c + d];
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = t[e];
    } else if constexpr (R == 3) {
        const float c = -0.5f;
        const float s = INV ? 0.86602540378443864676f : -0.86602540378443864676f;
        float2 t = cadd(v[1], v[2]);
        float2 d = csub(v[1], v[2]);
        float2 m = make_float2(v[0].x + c * t.x, v[0].y + c * t.y);
        float2 id = make_float2(-s * d.y, s * d.x);  // i s d
        v[0] = cadd(v[0], t);
        v[1] = cadd(m, id);
        v[2] = csub(m, id);
    }
}

// Stages whose inputs or outputs need not be in LDS.  Butterfly b = tid + i *
// nthreads of a radix-R stage belongs to pencil p = b & (P - 1) and takes the
// elements j + r n/R (j = b >> lp, r < R) through load(p, index); after the
// twiddles (k = j mod Ns) and the length-R transform, element (j - k) R + k +
// r Ns goes to store(p, index, value).  The first stage (Ns = 1) can read
// straight from HBM and the last one (k = j) write straight back, so a
// length-n transform touches LDS once per stage boundary.  In LDS, element x of
// pencil p sits at buf[x P + p].

// Each stage passes the thread index through opaque(), so the stage's index
// arithmetic is computed there and not hoisted to the kernel entry for every
// radix the kernel could run (which spills).
template <int R, bool INV, class Load, class Store>
__device__ __forceinline__ void stage_rs(int n, int lp, int Ns, const FastDiv &dns, const float2 *tw, int tid_,
                                         int nthreads, bool sync, Load &load, Store &store) {
    const int tid = opaque(tid_);
    constexpr int MAXB = (MAX_ELEMS + R - 1) / R;
    const int nbf = n / R;
    const int total = nbf << lp;
    const int pmask = (1 << lp) - 1;
    const int twstride = n / (Ns * R);
    float2 v[MAXB][R];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * nthreads;
        if (b < total) {
            const int p = b & pmask, j = b >> lp;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = load(p, j + r * nbf);
        }
    }
    if (Ns > 1) {
#pragma unroll
        for (int i = 0; i < MAXB; ++i) {
            const int b = tid + i * nthreads;
            if (b < total) {
                const int k = int(dns.mod(uint32_t(b >> lp)));
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw[r * k * twstride];
                    if (INV) w.y = -w.y;
                    v[i][r] = cmul(v[i][r], w);
                }
            }
        }
    }
    if (sync) __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * nthreads;
        if (b < total) {
            const int p = b & pmask, j = b >> lp;
            const int k = int(dns.mod(uint32_t(j)));
            dft<R, INV>(v[i]);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) store(p, base + r * Ns, v[i][r]);
        }
    }
}

template <bool INV, class Load, class Store>
__device__ __forceinline__ void stage_any(int R, int n, int lp, int Ns, const FastDiv &dns, const float2 *tw, int tid,
                                          int nthreads, bool sync, Load &load, Store &store) {
    switch (R) {
        case 16: stage_rs<16, INV>(n, lp, Ns, dns, tw, tid, nthreads, sync, load, store); break;
        case 8: stage_rs<8, INV>(n, lp, Ns, dns, tw, tid, nthreads, sync, load, store); break;
        case 4: stage_rs<4, INV>(n, lp, Ns, dns, tw, tid, nthreads, sync, load, store); break;
        case 2: stage_rs<2, INV>(n, lp, Ns, dns, tw, tid, nthreads, sync, load, store); break;
        default: stage_rs<3, INV>(n, lp, Ns, dns, tw, tid, nthreads, sync, load, store); break;
    }
}

// Stages [from, to) of plan pl on P = 1 << lp pencils held in buf (the LDS
// rows above): stage `from` reads through load, stage to - 1 writes through
// store, the others go from LDS to LDS, with a barrier after every stage but
// the last.  A stage that reads and writes LDS (in place) also waits between
// its reads and its writes; LOAD_LDS / STORE_LDS say whether load and store
// are LDS accesses.  Ns of stage s is the product of the radices before it.
template <bool INV, bool LOAD_LDS, bool STORE_LDS, class Load, class Store>
__device__ __forceinline__ void fft_pencils(float2 *buf, int lp, const FftPlan &pl, int from, int to, const float2 *tw, int tid,
                            int nthreads, Load &load, Store &store) {
    auto lload = [buf, lp](int p, int x) { return buf[(x << lp) + p]; };
    auto lstore = [buf, lp](int p, int x, float2 v) { buf[(x << lp) + p] = v; };
    int Ns = 1;
    for (int s = 0; s < from; ++s) Ns *= pl.radix[s];
    for (int s = from; s < to; ++s) {
        const bool first = s == from, last = s == to - 1;
        if (first && last)
            stage_any<INV>(pl.radix[s], pl.n, lp, Ns, pl.ns[s], tw, tid, nthreads, LOAD_LDS && STORE_LDS, load, store);
        else if (first)
            stage_any<INV>(pl.radix[s], pl.n, lp, Ns, pl.ns[s], tw, tid, nthreads, LOAD_LDS, load, lstore);
        else if (last)
            stage_any<INV>(pl.radix[s], pl.n, lp, Ns, pl.ns[s], tw, tid, nthreads, STORE_LDS, lload, store);
        else
            stage_any<INV>(pl.radix[s], pl.n, lp, Ns, pl.ns[s], tw, tid, nthreads, true, lload, lstore);
        if (!last) __syncthreads();
        Ns *= pl.radix[s];
    }
}

// The seam of the z pass: the last forward stage (Ns = n/R, so k = j and its
// outputs are elements j + r n/R), the multiplier, and the first inverse stage
// (Ns = 1, inputs j + r n/R, outputs j R + r), in registers.
template <int R, class Load, class Store, class Mul>
__device__ __forceinline__ void stage_seam(int n, int lp, const float2 *tw, int tid_, int nthreads, bool sync,
                                           Load &load, Store &store, Mul &mul) {
    const int tid = opaque(tid_);
    constexpr int MAXB = (MAX_ELEMS + R - 1) / R;
    const int nbf = n / R;
    const int total = nbf << lp;
    const int pmask = (1 << lp) - 1;
    float2 v[MAXB][R];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * nthreads;
        if (b < total) {
            const int p = b & pmask, j = b >> lp;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = load(p, j + r * nbf);
            if (nbf > 1) {  // twstride = 1, k = j
#pragma unroll
                for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], tw[r * j]);
            }
        }
    }
    if (sync) __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * nthreads;
        if (b < total) {
            const int p = b & pmask, j = b >> lp;
            dft<R, false>(v[i]);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float m = mul(p, j + r * nbf);
                v[i][r] = make_float2(v[i][r].x * m, v[i][r].y * m);
            }
            dft<R, true>(v[i]);
#pragma unroll
            for (int r = 0; r < R; ++r) store(p, j * R + r, v[i][r]);
        }
    }
}

template <class Load, class Store, class Mul>
__device__ __forceinline__ void seam_any(int R, int n, int lp, const float2 *tw, int tid, int nthreads, bool sync,
                                         Load &load, Store &store, Mul &mul) {
    switch (R) {
        case 16: stage_seam<16>(n, lp, tw, tid, nthreads, sync, load, store, mul); break;
        case 8: stage_seam<8>(n, lp, tw, tid, nthreads, sync, load, store, mul); break;
        case 4: stage_seam<4>(n, lp, tw, tid, nthreads, sync, load, store, mul); break;
        case 2: stage_seam<2>(n, lp, tw, tid, nthreads, sync, load, store, mul); break;
        default: stage_seam<3>(n, lp, tw, tid, nthreads, sync, load, store, mul); break;
    }
}

// Loads of a workgroup's tile are issued as one batch into registers before
// any is written to LDS, so each thread keeps all of its loads in flight
// (a load-store loop would wait for every load in turn).  Every launch keeps
// the elements per thread at or below MAX_ELEMS.
__device__ __forceinline__ void load_twiddles(float2 *tw_s, const float2 *tw_g, int n) {
    float2 t[MAX_ELEMS];
#pragma unroll
    for (int i = 0; i < MAX_ELEMS; ++i) {
        const int e = threadIdx.x + i * blockDim.x;
        if (e < n) t[i] = tw_g[e];
    }
#pragma unroll
    for (int i = 0; i < MAX_ELEMS; ++i) {
        const int e = threadIdx.x + i * blockDim.x;
        if (e < n) tw_s[e] = t[i];
    }
}

// ---------------------------------------------------------------------------
// Tables, generated in FP64 and stored as FP32.
// ---------------------------------------------------------------------------
// Per-job workspace layout (offsets from the job's workspace base).
struct CwtLayout {
    size_t scalars, tw, gtab, htab, ctab, btab, ptab, mass, spec, total;
    int lp_x, lp_xi;          // log2 of row pairs per forward / inverse x-pass workgroup
    int64_t xblocks, xblocks_i;
};

// Up to MAX_BATCH same-n transforms in one launch per pass; the job index is a
// grid dimension and job j's workspace starts at ws + j * stride.
constexpr int MAX_BATCH = HF_CWT_BATCH_MAX;
struct CwtJobs {
    const int64_t *rho[MAX_BATCH];
    float *cwt[MAX_BATCH];
    double box_len[MAX_BATCH];
    double w[MAX_BATCH];
    int images[MAX_BATCH];
    char *ws;
    size_t stride;
    int mode;  // hf_kernel
    int count;
    // every job transforms job 0's density (one grid, several scales): the
    // forward x and y passes run for job 0 only and each job's z pass reads
    // job 0's half spectrum (and its normalisation) into its own; job 0's own
    // z pass, in place, runs in a launch after the others
    int shared_forward;
    int job_base;  // the z pass's first job (its launch covers job_base .. job_base + grid jobs - 1)
};

struct JobView {
    double *scalars;
    float2 *tw;
    double *gtab, *htab, *ctab;
    float *btab, *ptab;
    Mass128 *mass;
    float2 *spec;
};

__device__ __forceinline__ JobView job_view(const CwtJobs &J, const CwtLayout &L, int j) {
    char *b = J.ws + size_t(j) * J.stride;
    JobView v;
    v.scalars = reinterpret_cast<double *>(b + L.scalars);
    v.tw = reinterpret_cast<float2 *>(b + L.tw);
    v.gtab = reinterpret_cast<double *>(b + L.gtab);
    v.htab = reinterpret_cast<double *>(b + L.htab);
    v.ctab = reinterpret_cast<double *>(b + L.ctab);
    v.btab = reinterpret_cast<float *>(b + L.btab);
    v.ptab = reinterpret_cast<float *>(b + L.ptab);
    v.mass = reinterpret_cast<Mass128 *>(b + L.mass);
    v.spec = reinterpret_cast<float2 *>(b + L.spec);
    return v;
}

// twiddles tw[m] = exp(-2 pi i m / n), the cosines ctab[m] = cos(2 pi m / n)
// in FP64 for stage 2; periodised 1D Gaussian factors of the
// sampled wavelet: G_j = sum_m g(x_j + m L), Hs_j = sum_m (x_j + m L)^2 g(...)
// with g(t) = exp(-w^2 t^2 / 4) and x_j the minimum-image offset of node j.
// Job = blockIdx.y.
__global__ void tables_stage1(CwtJobs J, CwtLayout L, int n) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int job = blockIdx.y;
    const JobView v = job_view(J, L, job);
    const double box_len = J.box_len[job], w = J.w[job];
    double s, c;
    sincospi(2.0 * double(j) / double(n), &s, &c);
    v.tw[j] = make_float2(float(c), float(-s));
    v.ctab[j] = cospi(2.0 * double(j) / double(n));  // the DFT cosines of stage 2, one per phase
    const double dx = box_len / n;
    const int jc = (j + n / 2) % n - n / 2;
    double G = 0.0, Hs = 0.0;
    for (int m = -J.images[job]; m <= J.images[job]; ++m) {
        const double x = jc * dx + m * box_len;
        const double g = exp(-0.25 * w * w * x * x);
        G += g;
        Hs += x * x * g;
    }
    v.gtab[j] = G;
    v.htab[j] = Hs;
}

// Separable multiplier: M(kx,ky,kz) = P_x B_y B_z + B_x P_y B_z + B_x B_y P_z.
//  sampled : B = DFT(G), A = DFT(Hs), P = (alpha/3) B + beta A with
//            alpha = 6 dx^3 w^1.5, beta = -dx^3 w^3.5 (Eq. (4) split into
//            6 g g g - w^2 (x^2 g g g + ...), periodised and transformed);
//  analytic: B = exp(-k^2/w^2), P = 32 pi^1.5 w^-3.5 k^2 B (the transform of Eq. (4)).
// One workgroup of TAB_THREADS per frequency k: thread t sums the terms
// j = t, t + TAB_THREADS, ... and the partial sums are added in a fixed order.
constexpr int TAB_THREADS = 256;

__global__ void __launch_bounds__(TAB_THREADS) tables_stage2(CwtJobs J, CwtLayout L, int n) {
    const int k = blockIdx.x;
    const int job = blockIdx.y;
    const JobView v = job_view(J, L, job);
    const double w = J.w[job], box_len = J.box_len[job];
    if (J.mode == HF_KERNEL_ANALYTIC) {
        if (threadIdx.x != 0) return;
        const int ks = k <= n / 2 ? k : k - n;
        const double kk = 2.0 * M_PI * ks / box_len;
        const double B = exp(-(kk * kk) / (w * w));
        const double beta = 32.0 * pow(M_PI, 1.5) * pow(w, -3.5);
        v.btab[k] = float(B);
        v.ptab[k] = float(beta * kk * kk * B);
        return;
    }
    double B = 0.0, A = 0.0;
    const int step = int((int64_t(TAB_THREADS) * k) % n);  // phase step between a thread's terms
    int ph = int((int64_t(threadIdx.x) * k) % n);
    for (int j = threadIdx.x; j < n; j += TAB_THREADS) {
        const double c = v.ctab[ph];
        B += v.gtab[j] * c;
        A += v.htab[j] * c;
        ph += step;
        if (ph >= n) ph -= n;
    }
    __shared__ double rb[TAB_THREADS], ra[TAB_THREADS];
    rb[threadIdx.x] = B;
    ra[threadIdx.x] = A;
    __syncthreads();
    for (int h = TAB_THREADS / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) {
            rb[threadIdx.x] += rb[threadIdx.x + h];
            ra[threadIdx.x] += ra[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    B = rb[0];
    A = ra[0];
    const double dx = box_len / n;
    const double dx3 = dx * dx * dx;
    const double alpha = 6.0 * dx3 * pow(w, 1.5);
    const double beta = -dx3 * pow(w, 3.5);
    v.btab[k] = float(B);
    v.ptab[k] = float(alpha / 3.0 * B + beta * A);
}

// ---------------------------------------------------------------------------
// x passes
// ---------------------------------------------------------------------------


// One workgroup = xp row pairs (rows 2q, 2q+1 of the n*n rows of x).
__global__ void fft_x_fwd_kernel(CwtJobs J, CwtLayout L, FftPlan pl, uint32_t *status) {
    extern __shared__ float2 smem[];
    const int job = blockIdx.y;
    const JobView jv = job_view(J, L, job);
    const int64_t *__restrict__ rho = J.rho[job];
    float2 *__restrict__ spec = jv.spec;
    const float2 *__restrict__ tw_g = jv.tw;
    Mass128 *__restrict__ mass = jv.mass;
    const int lp = L.lp_x;
    const int n = pl.n, H = n / 2 + 1;
    const int xp = 1 << lp;
    float2 *tw = smem;
    float2 *buf = smem + n;  // element x of pair p at buf[(x << lp) + p]
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t pairs = int64_t(n) * n / 2;
    const int64_t q0 = int64_t(blockIdx.x) * xp;
    load_twiddles(tw, tw_g, n);
    unsigned long long lo = 0, hi = 0;
    bool neg = false;
    {
        int64_t va[MAX_ELEMS], vb[MAX_ELEMS];
#pragma unroll
        for (int i = 0; i < MAX_ELEMS; ++i) {
            const int e = tid + i * nt;
            va[i] = 0;
            vb[i] = 0;
            if (e < xp * n) {
                const int p = int(pl.dn.div(uint32_t(e))), x = e - p * n;
                const int64_t q = q0 + p;
                if (q < pairs) {
                    va[i] = rho[(2 * q) * n + x];
                    vb[i] = rho[(2 * q + 1) * n + x];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < MAX_ELEMS; ++i) {
            const int e = tid + i * nt;
            if (e < xp * n) {
                const int p = int(pl.dn.div(uint32_t(e))), x = e - p * n;
                const int64_t a = va[i], b = vb[i];
                neg |= (a < 0) | (b < 0);
                add128(lo, hi, static_cast<unsigned long long>(a));
                add128(lo, hi, static_cast<unsigned long long>(b));
                buf[(x << lp) + p] = make_float2(float(a), float(b));
            }
        }
    }
    if (neg) atomicOr(status, ST_INPUT);
    // workgroup sum of the 128-bit masses (fixed order: deterministic)
    __shared__ unsigned long long red_lo[1024 / 64], red_hi[1024 / 64];
    {
        // wave reduction by shuffles
        for (int off = 32; off > 0; off >>= 1) {
            unsigned long long olo = __shfl_down(lo, off, 64);
            unsigned long long ohi = __shfl_down(hi, off, 64);
            add128(lo, hi, olo);
            hi += ohi;
        }
        const int wave = tid >> 6;
        if ((tid & 63) == 0) {
            red_lo[wave] = lo;
            red_hi[wave] = hi;
        }
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long L = 0, Hh = 0;
        for (int w = 0; w < (nt + 63) / 64; ++w) {
            add128(L, Hh, red_lo[w]);
            Hh += red_hi[w];
        }
        mass[blockIdx.x].lo = L;
        mass[blockIdx.x].hi = Hh;
    }
    auto lload = [buf, lp](int p, int x) { return buf[(x << lp) + p]; };
    auto lstore = [buf, lp](int p, int x, float2 v) { buf[(x << lp) + p] = v; };
    fft_pencils<false, true, true>(buf, lp, pl, 0, pl.nst, tw, tid, nt, lload, lstore);
    __syncthreads();
    // split Z = A + iB into the two real rows' spectra; a wavefront writes one
    // column tile of the workgroup's 2 xp consecutive rows
    const int rows = 2 * xp;
    const int ntile = spec_tiles(n);
    for (int e = tid; e < ntile * YZ_TILE * rows; e += nt) {
        const int c = e & (YZ_TILE - 1), r = (e >> YZ_LOG) % rows, tile = (e >> YZ_LOG) / rows;
        const int k = tile * YZ_TILE + c, p = r >> 1;
        const int64_t q = q0 + p;
        if (k >= H || q >= pairs) continue;
        const float2 zk = buf[(k << lp) + p];
        const float2 zm = buf[(((n - k) % n) << lp) + p];
        const float2 v = (r & 1) ? make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x))  // B, row 2q + 1
                                 : make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));  // A, row 2q
        const uint32_t row = uint32_t(2 * q + (r & 1)), z = pl.dn.div(row);
        spec[spec_at(n, tile, int(z), int(row - z * uint32_t(n))) + c] = v;
    }
}

__global__ void fft_x_inv_kernel(CwtJobs J, CwtLayout L, FftPlan pl) {
    extern __shared__ float2 smem[];
    const int job = blockIdx.y;
    const JobView jv = job_view(J, L, job);
    const float2 *__restrict__ spec = jv.spec;
    float *__restrict__ out = J.cwt[job];
    const float2 *__restrict__ tw_g = jv.tw;
    const int lp = L.lp_xi;
    const int n = pl.n, H = n / 2 + 1;
    const int xp = 1 << lp;
    float2 *tw = smem;
    float2 *buf = smem + n;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t pairs = int64_t(n) * n / 2;
    const int64_t q0 = int64_t(blockIdx.x) * xp;
    load_twiddles(tw, tw_g, n);
    // element e: column c of tile `tile` for pair p; a wavefront reads one column
    // tile of consecutive rows
    const int ntile = spec_tiles(n);
    const int span = ntile * YZ_TILE * xp;  // at most xp n, so MAX_ELEMS per thread suffice
    float2 va[MAX_ELEMS], vb[MAX_ELEMS];
#pragma unroll
    for (int i = 0; i < MAX_ELEMS; ++i) {
        const int e = tid + i * nt;
        va[i] = make_float2(0.f, 0.f);
        vb[i] = va[i];
        if (e < span) {
            const int c = e & (YZ_TILE - 1), p = (e >> YZ_LOG) % xp, tile = (e >> YZ_LOG) / xp;
            const int64_t q = q0 + p;
            if (tile * YZ_TILE + c < H && q < pairs) {
                // rows 2q and 2q + 1 share z (n is even)
                const uint32_t row = uint32_t(2 * q), z = pl.dn.div(row);
                const size_t at = spec_at(n, tile, int(z), int(row - z * uint32_t(n))) + c;
                va[i] = spec[at];
                vb[i] = spec[at + YZ_TILE];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < MAX_ELEMS; ++i) {
        const int e = tid + i * nt;
        if (e >= span) continue;
        const int c = e & (YZ_TILE - 1), p = (e >> YZ_LOG) % xp, tile = (e >> YZ_LOG) / xp;
        const int k = tile * YZ_TILE + c;
        if (k >= H) continue;
        const float2 A = va[i], B = vb[i];
        if (k == 0 || 2 * k == n) {
            // DC and Nyquist of a real row are real
            buf[(k << lp) + p] = make_float2(A.x, B.x);
        } else {
            buf[(k << lp) + p] = make_float2(A.x - B.y, A.y + B.x);
            buf[((n - k) << lp) + p] = make_float2(A.x + B.y, B.x - A.y);
        }
    }
    __syncthreads();
    auto lload = [buf, lp](int p, int x) { return buf[(x << lp) + p]; };
    auto lstore = [buf, lp](int p, int x, float2 v) { buf[(x << lp) + p] = v; };
    fft_pencils<true, true, true>(buf, lp, pl, 0, pl.nst, tw, tid, nt, lload, lstore);
    __syncthreads();
    for (int e = tid; e < xp * n; e += nt) {
        const int p = int(pl.dn.div(uint32_t(e))), x = e - p * n;
        const int64_t q = q0 + p;
        if (q >= pairs) continue;
        const float2 v = buf[(x << lp) + p];
        out[(2 * q) * n + x] = v.x;
        out[(2 * q + 1) * n + x] = v.y;
    }
}

// ---------------------------------------------------------------------------
// mean density and overall scale
// ---------------------------------------------------------------------------

__global__ void mass_kernel(CwtJobs J, CwtLayout L, int n, uint32_t *status) {
    const JobView jv = job_view(J, L, blockIdx.x);
    const Mass128 *__restrict__ mass = jv.mass;
    const int64_t nparts = L.xblocks;
    double *scalars = jv.scalars;
    __shared__ unsigned long long red_lo[16], red_hi[16];
    unsigned long long lo = 0, hi = 0;
    for (int64_t i = threadIdx.x; i < nparts; i += blockDim.x) {
        add128(lo, hi, mass[i].lo);
        hi += mass[i].hi;
    }
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long olo = __shfl_down(lo, off, 64);
        unsigned long long ohi = __shfl_down(hi, off, 64);
        add128(lo, hi, olo);
        hi += ohi;
    }
    if ((threadIdx.x & 63) == 0) {
        red_lo[threadIdx.x >> 6] = lo;
        red_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long L = 0, Hh = 0;
        for (int w = 0; w < int(blockDim.x >> 6); ++w) {
            add128(L, Hh, red_lo[w]);
            Hh += red_hi[w];
        }
        const double total = u128_to_double(L, Hh);
        const double cells = double(n) * double(n) * double(n);
        const double mbar = total / cells;  // mean cell mass, FP64
        if (!(mbar > 0.0)) {
            atomicOr(status, ST_INPUT);
            scalars[0] = 0.0;
        } else {
            // C = IDFT(DFT(rho) M) / (mbar n^3): the mean normalisation and the
            // inverse-transform 1/n^3 folded into one factor
            scalars[0] = 1.0 / (mbar * cells);
        }
        scalars[1] = mbar;
    }
}

// ---------------------------------------------------------------------------
// y and z passes on tiles of YZ_TILE columns of the half spectrum
// ---------------------------------------------------------------------------
// Logical block (x, y, job) of an (X, Y, jobs) grid, XCD-contiguous over the
// whole launch: x = column tile, y = row in the y pass; x = row, y = column
// tile in the z pass.
__device__ __forceinline__ void yz_tile(int &x, int &y, int &job) {
    const uint32_t X = gridDim.x, Y = gridDim.y;
    const uint32_t lt = xcd_remap(blockIdx.x + X * (blockIdx.y + Y * blockIdx.z), X * Y * gridDim.z);
    x = int(lt % X);
    y = int((lt / X) % Y);
    job = int(lt / (X * Y));
}

template <bool INV>
__global__ void fft_y_kernel(CwtJobs J, CwtLayout L, FftPlan pl) {
    extern __shared__ float2 smem[];
    int tile, zrow, job;
    yz_tile(tile, zrow, job);
    const JobView jv = job_view(J, L, job);
    float2 *__restrict__ spec = jv.spec;
    const int n = pl.n, H = n / 2 + 1;
    float2 *tw = smem;
    float2 *buf = smem + n;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int kx0 = tile * YZ_TILE;
    const int valid = min(YZ_TILE, H - kx0);
    float2 *col = spec + spec_at(n, tile, zrow, 0);  // element y of pencil p at col[y YZ_TILE + p]
    load_twiddles(tw, jv.tw, n);                      // first read after the first stage's barrier
    auto gload = [=](int p, int y) { return p < valid ? col[y * YZ_TILE + p] : make_float2(0.f, 0.f); };
    auto gstore = [=](int p, int y, float2 v) {
        if (p < valid) col[y * YZ_TILE + p] = v;
    };
    fft_pencils<INV, false, false>(buf, YZ_LOG, pl, 0, pl.nst, tw, tid, nt, gload, gstore);
}

// Forward z transform, multiplier, inverse z transform; pi is pl with its
// last radix moved to the front.
// The z pass walks its tiles ky-fastest (grid (n, tiles, jobs)): the tiles of
// rows ky and ky + 1 read the two halves of the same 128-byte lines, so they
// run together on one XCD and each line comes from HBM once.
__global__ void fft_z_mul_kernel(CwtJobs J, CwtLayout L, FftPlan pl, FftPlan pi) {
    extern __shared__ float2 smem[];
    int tile, yrow, job;
    yz_tile(yrow, tile, job);
    job += J.job_base;
    const JobView jv = job_view(J, L, job);
    const JobView src = J.shared_forward ? job_view(J, L, 0) : jv;  // forward spectrum and normalisation
    float2 *spec = jv.spec;  // the same memory as src.spec unless the forward transform is shared
    const float *__restrict__ tab_b = jv.btab;
    const float *__restrict__ tab_p = jv.ptab;
    const int n = pl.n, H = n / 2 + 1;
    float2 *tw = smem;
    float2 *buf = smem + n;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int kx0 = tile * YZ_TILE;
    const int ky = yrow;
    const int valid = min(YZ_TILE, H - kx0);
    const size_t zstride = size_t(n + 1) * YZ_TILE;
    float2 *col = spec + spec_at(n, tile, 0, ky);  // element z of pencil p at col[z zstride + p]
    const float2 *col_in = src.spec + spec_at(n, tile, 0, ky);  // the same place, or job 0's
    load_twiddles(tw, jv.tw, n);
    const float scale = float(src.scalars[0]);
    const float by = tab_b[ky], py = tab_p[ky];
    // the thread's pencil is the same in every stage (nthreads is a multiple of P)
    const int kx = min(kx0 + (tid & (YZ_TILE - 1)), H - 1);
    const float bx = tab_b[kx], px = tab_p[kx];
    const float cxy = (px * by + bx * py) * scale, bxy = bx * by * scale;
    auto gload = [=](int p, int z) { return p < valid ? col_in[size_t(z) * zstride + p] : make_float2(0.f, 0.f); };
    auto gstore = [=](int p, int z, float2 v) {
        if (p < valid) col[size_t(z) * zstride + p] = v;
    };
    auto mul = [=](int, int kz) { return cxy * tab_b[kz] + bxy * tab_p[kz]; };
    auto lload = [buf](int p, int x) { return buf[(x << YZ_LOG) + p]; };
    auto lstore = [buf](int p, int x, float2 v) { buf[(x << YZ_LOG) + p] = v; };
    const int last = pl.nst - 1;
    if (last == 0) {
        seam_any(pl.radix[0], n, YZ_LOG, tw, tid, nt, false, gload, gstore, mul);
        return;
    }
    fft_pencils<false, false, true>(buf, YZ_LOG, pl, 0, last, tw, tid, nt, gload, lstore);
    __syncthreads();
    seam_any(pl.radix[last], n, YZ_LOG, tw, tid, nt, true, lload, lstore, mul);
    __syncthreads();
    fft_pencils<true, true, false>(buf, YZ_LOG, pi, 1, pi.nst, tw, tid, nt, lload, gstore);
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
// log2 of the row pairs per x-pass workgroup: at most `elems` complex values,
// between 4 and 16 pairs.  More pairs make longer runs in each spectrum tile.
int x_log_pairs(int n, int elems) {
    int lp = 4;
    while (lp > 2 && (n << lp) > elems) --lp;
    return lp;
}

CwtLayout cwt_layout(int n) {
    CwtLayout L{};
    L.lp_x = x_log_pairs(n, 8192);
    L.lp_xi = x_log_pairs(n, 8192);
    const int64_t pairs = int64_t(n) * n / 2;
    L.xblocks = (pairs + (1 << L.lp_x) - 1) >> L.lp_x;
    L.xblocks_i = (pairs + (1 << L.lp_xi) - 1) >> L.lp_xi;
    size_t off = 0;
    L.scalars = off;
    off = align_up(off + 64);
    L.tw = off;
    off = align_up(off + sizeof(float2) * n);
    L.gtab = off;
    off = align_up(off + sizeof(double) * n);
    L.htab = off;
    off = align_up(off + sizeof(double) * n);
    L.ctab = off;
    off = align_up(off + sizeof(double) * n);
    L.btab = off;
    off = align_up(off + sizeof(float) * n);
    L.ptab = off;
    off = align_up(off + sizeof(float) * n);
    L.mass = off;
    off = align_up(off + sizeof(Mass128) * size_t(L.xblocks));
    L.spec = off;
    off = align_up(off + sizeof(float2) * size_t(spec_tiles(n)) * spec_tile_rows(n) * YZ_TILE);
    L.total = off;
    return L;
}

int threads_for(int elems) {
    int t = (elems + MAX_ELEMS - 1) / MAX_ELEMS;
    t = (t + 63) / 64 * 64;
    if (t < 64) t = 64;
    if (t > 1024) t = 1024;
    return t;
}

// Enqueues the whole transform for J.count same-n jobs (one launch per pass).
hf_status run_cwt(hf_ctx *ctx, int n, const CwtJobs &J) {
    const CwtLayout L = cwt_layout(n);
    hipStream_t st = ctx->stream;
    const unsigned jobs = unsigned(J.count);
    const int tb = 256, tg = (n + tb - 1) / tb;
    HF_LAUNCH(ctx, K_TABLES_1, tables_stage1, dim3(tg, jobs), dim3(tb), 0, st, J, L, n);
    HF_LAUNCH(ctx, K_TABLES_2, tables_stage2, dim3(n, jobs), dim3(TAB_THREADS), 0, st, J, L, n);

    const FftPlan pl = make_plan(n);
    const FftPlan pi = rotate_plan(pl);
    const int H = n / 2 + 1;
    const int tiles = (H + YZ_TILE - 1) / YZ_TILE;
    const int yz_threads = threads_for(n * YZ_TILE);
    const size_t yz_shm = sizeof(float2) * (size_t(n) + size_t(n) * YZ_TILE);
    const int x_threads = threads_for((1 << L.lp_x) * n);
    const size_t x_shm = sizeof(float2) * (size_t(n) + size_t(n) * (1 << L.lp_x));
    const int xi_threads = threads_for((1 << L.lp_xi) * n);
    const size_t xi_shm = sizeof(float2) * (size_t(n) + size_t(n) * (1 << L.lp_xi));
    // workgroups that need more than the default 64 KiB of dynamic LDS say so
    auto allow = [](const void *f, size_t bytes) {
        return bytes <= 65536 ||
               hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)) == hipSuccess;
    };
    if (!allow(reinterpret_cast<const void *>(&fft_y_kernel<false>), yz_shm) ||
        !allow(reinterpret_cast<const void *>(&fft_y_kernel<true>), yz_shm) ||
        !allow(reinterpret_cast<const void *>(&fft_z_mul_kernel), yz_shm) ||
        !allow(reinterpret_cast<const void *>(&fft_x_fwd_kernel), x_shm) ||
        !allow(reinterpret_cast<const void *>(&fft_x_inv_kernel), xi_shm))
        return HF_ERR_DEVICE;
    const unsigned fwd_jobs = J.shared_forward ? 1u : jobs;
    HF_LAUNCH(ctx, K_X_FWD, fft_x_fwd_kernel, dim3(unsigned(L.xblocks), fwd_jobs), dim3(x_threads), x_shm, st, J, L,
              pl, ctx->d_status);
    HF_LAUNCH(ctx, K_MASS, mass_kernel, dim3(fwd_jobs), dim3(1024), 0, st, J, L, n, ctx->d_status);
    HF_LAUNCH(ctx, K_Y_FWD, fft_y_kernel<false>, dim3(tiles, n, fwd_jobs), dim3(yz_threads), yz_shm, st, J, L, pl);
    if (J.shared_forward && jobs > 1) {
        // the other scales read job 0's forward spectrum before job 0 overwrites it
        CwtJobs Jr = J;
        Jr.job_base = 1;
        HF_LAUNCH(ctx, K_Z_MUL, fft_z_mul_kernel, dim3(n, tiles, jobs - 1), dim3(yz_threads), yz_shm, st, Jr, L, pl,
                  pi);
        HF_LAUNCH(ctx, K_Z_MUL, fft_z_mul_kernel, dim3(n, tiles, 1), dim3(yz_threads), yz_shm, st, J, L, pl, pi);
    } else {
        HF_LAUNCH(ctx, K_Z_MUL, fft_z_mul_kernel, dim3(n, tiles, jobs), dim3(yz_threads), yz_shm, st, J, L, pl, pi);
    }
    HF_LAUNCH(ctx, K_Y_INV, fft_y_kernel<true>, dim3(tiles, n, jobs), dim3(yz_threads), yz_shm, st, J, L, pl);
    HF_LAUNCH(ctx, K_X_INV, fft_x_inv_kernel, dim3(unsigned(L.xblocks_i), jobs), dim3(xi_threads), xi_shm, st, J, L,
              pl);
    return launch_status();
}

bool fill_job(CwtJobs &J, int j, const int64_t *rho, float *cwt, double box_len, double kw) {
    if (!rho || !cwt || !(kw > 0.0) || !std::isfinite(kw) || !(box_len > 0.0) || !(box_len < 1e300)) return false;
    J.rho[j] = rho;
    J.cwt[j] = cwt;
    J.box_len[j] = box_len;
    J.w[j] = 1000.0 * kw / box_len;  // step 1: k_w = w L / 1000
    // periodic images within w (I + 1/2) L >= 16, where the wavelet is < 1e-25 of its peak
    J.images[j] = std::max(1, int(std::ceil(16.0 / (J.w[j] * box_len) - 0.5)));
    return true;
}

}  // namespace

size_t hf::cwt_ws_bytes(const hf_box &box) { return cwt_layout(box.n).total; }

extern "C" hf_status hf_cwt(hf_ctx *ctx, const hf_box *box, const int64_t *rho, double kw, hf_kernel kernel,
                            float *cwt, void *ws, size_t ws_bytes) {
    if (!ctx || !rho || !cwt) return HF_ERR_ARG;
    if (kernel != HF_KERNEL_SAMPLED && kernel != HF_KERNEL_ANALYTIC && kernel != HF_KERNEL_STENCIL) return HF_ERR_ARG;
    if (!(kw > 0.0) || !std::isfinite(kw)) return HF_ERR_ARG;
    if (kernel == HF_KERNEL_STENCIL) {
        if (!box) return HF_ERR_ARG;
        const int32_t h = stencil_half_width(kw, box->n);  // Table 1's extent on this grid
        if (h < 0) return HF_ERR_ARG;
        return hf_cwt_stencil(ctx, box, rho, kw, h, cwt, ws, ws_bytes);
    }
    hf_status s = check_box(box);
    if (s != HF_OK) return s;
    const size_t need = cwt_layout(box->n).total;
    s = check_ws(ws, ws_bytes, need);
    if (s != HF_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    CwtJobs J{};
    if (!fill_job(J, 0, rho, cwt, box->box_len, kw)) return HF_ERR_ARG;
    J.ws = static_cast<char *>(ws);
    J.stride = need;
    J.mode = kernel;
    J.count = 1;
    return run_cwt(ctx, box->n, J);
}

extern "C" hf_status hf_cwt_scales(hf_ctx *ctx, const hf_box *box, const int64_t *rho, int32_t count,
                                   const double *kws, hf_kernel kernel, float *const *cwts, void *ws,
                                   size_t ws_bytes) {
    if (!ctx || !rho || !kws || !cwts || count < 1 || count > HF_CWT_BATCH_MAX) return HF_ERR_ARG;
    if (kernel != HF_KERNEL_SAMPLED && kernel != HF_KERNEL_ANALYTIC) return HF_ERR_ARG;
    hf_status s = check_box(box);
    if (s != HF_OK) return s;
    const size_t per = cwt_layout(box->n).total;
    s = check_ws(ws, ws_bytes, per * size_t(count));
    if (s != HF_OK) return s;
    CwtJobs J{};
    for (int j = 0; j < count; ++j)
        if (!fill_job(J, j, rho, cwts[j], box->box_len, kws[j])) return HF_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    J.ws = static_cast<char *>(ws);
    J.stride = per;
    J.mode = kernel;
    J.count = count;
    J.shared_forward = 1;
    return run_cwt(ctx, box->n, J);
}

extern "C" hf_status hf_cwt_batch_ws_size(int32_t n, int32_t count, size_t *bytes) {
    if (!bytes || count < 1 || count > HF_CWT_BATCH_MAX) return HF_ERR_ARG;
    if (!supported_n(n)) return HF_ERR_SIZE;
    *bytes = cwt_layout(n).total * size_t(count);
    return HF_OK;
}

extern "C" hf_status hf_cwt_batch(hf_ctx *ctx, int32_t n, int32_t count, const hf_cwt_item *items, hf_kernel kernel,
                                  void *ws, size_t ws_bytes) {
    if (!ctx || !items || count < 1 || count > HF_CWT_BATCH_MAX) return HF_ERR_ARG;
    if (kernel != HF_KERNEL_SAMPLED && kernel != HF_KERNEL_ANALYTIC) return HF_ERR_ARG;
    if (!supported_n(n)) return HF_ERR_SIZE;
    const size_t per = cwt_layout(n).total;
    hf_status s = check_ws(ws, ws_bytes, per * size_t(count));
    if (s != HF_OK) return s;
    CwtJobs J{};
    for (int j = 0; j < count; ++j)
        if (!fill_job(J, j, items[j].rho, items[j].cwt, items[j].box_len, items[j].kw)) return HF_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    J.ws = static_cast<char *>(ws);
    J.stride = per;
    J.mode = kernel;
    J.count = count;
    return run_cwt(ctx, n, J);
}
