/*
 * hf.h - C ABI of the MI355X (gfx950) CWT halo-finding path.
 *
 * The path is the data-parallel core of CWTHF (Li, Wang & He,
 * arXiv:2501.10622), Sec. 2, identification steps 2-10:
 *
 *   hf_deposit  step 2  cloud-in-cell mass on a periodic n^3 grid, Eq. (1)
 *   hf_cwt      step 3  grid CWT with the Mexican-hat wavelet, Eqs. (2)-(4)
 *               (hf_cwt_batch: several grids; hf_cwt_scales: several scales;
 *               hf_cwt_stencil: the truncated real-space stencil of Sec. 2.1)
 *   hf_maxima   step 4  local maxima of the grid CWT
 *   hf_segment  step 5  segmentation of the grid by the maxima (Sec. 2.3)
 *   hf_label    step 6  particles take the label of their segmented cell
 *   hf_groups   steps 5 and 7  grid volume, particle number and density filter
 *                       of every group (Table 1: dens_th, particle_th)
 *   hf_peaks    step 4  sub-cell position and value of each maximum (App. B)
 *   hf_cross_scale  step 8  maxima that are also maxima across scale
 *   hf_identify steps 2-8   the loop over scales, largest first, that claims
 *                       particles for halos (Sec. 2 and its flowchart)
 *   hf_identify_grids  the same loop with every scale on its own grid N_g,
 *                       with steps 9-10 when velocities are given
 *   hf_unbind   steps 9-10  the self-boundness check of one scale's groups
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every array argument is a DEVICE pointer on the context's device.  The
 *    caller allocates and owns all of them; no call keeps a pointer after it
 *    returns.  Calls are asynchronous: they enqueue kernels on the context's
 *    stream and return.
 *  - Grids are C-order [z][y][x]; cell (x, y, z) has linear index
 *    (z*n + y)*n + x (int32, so n <= 1024).
 *  - Positions are [np][3] rows (x, y, z) in the units of box_len, FP32 or
 *    FP64 (hf_dtype).  Positions outside [0, box_len) wrap periodically.
 *  - Supported n: n = 2^a 3^b with a >= 1, 8 <= n <= 1024 wherever the FFT
 *    transform runs (hf_cwt with SAMPLED or ANALYTIC, the batched and
 *    multi-scale transforms, the one-call pipelines with those kernels, and
 *    hf_workspace_size with HF_STAGE_CWT); any 8 <= n <= 1024 for the other
 *    stages and for the pipelines with HF_KERNEL_STENCIL (the flowchart's
 *    per-scale grids N_g are arbitrary integers).
 *    frac_bits (B, CIC fraction bits per axis) in [8, 20].
 *  - Workspaces are device buffers of at least hf_workspace_size() bytes,
 *    256-byte aligned.  One workspace may be reused by every stage in turn.
 *  - Argument errors are returned synchronously and nothing is enqueued.
 *    Errors found by kernels (overflow, capacity, bad input values) set a
 *    status word in the context; hf_sync() waits for the stream and returns
 *    (then clears) them.
 *  - One context per stream; a context must not be used from two host
 *    threads at once.
 */
#ifndef HF_H
#define HF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HF_OK = 0,
    HF_ERR_ARG = 1,       /* null pointer, bad enum, non-finite scale, bad count */
    HF_ERR_SIZE = 2,      /* n not supported (see above) or frac_bits out of range */
    HF_ERR_WORKSPACE = 3, /* workspace smaller than hf_workspace_size or misaligned */
    HF_ERR_OVERFLOW = 4,  /* device: a CIC cell exceeded 2^63 - 1 */
    HF_ERR_CAPACITY = 5,  /* device: more maxima than the list capacity */
    HF_ERR_DEVICE = 6,    /* HIP runtime failure */
    HF_ERR_INPUT = 7      /* device: non-finite/out-of-range position, NaN in a field,
                             negative or all-zero density grid */
} hf_status;

typedef enum { HF_F32 = 0, HF_F64 = 1 } hf_dtype;

/* Discretisation of the wavelet convolution (Eq. (2)).
 *  SAMPLED:  the wavelet of Eq. (4) sampled at the grid spacing and summed
 *            over periodic images (the paper's discretised convolution,
 *            Sec. 2.1), applied through its exact DFT.
 *  ANALYTIC: the continuum Fourier transform of Eq. (4),
 *            32 pi^1.5 w^-1.5 (k/w)^2 exp(-(k/w)^2), at the DFT wavenumbers.
 *  STENCIL:  the sampled wavelet truncated to a cube of half-width
 *            ceil(Int(1.5/k_w + 5) n / Int(400 k_w + 150)) cells: Table 1's
 *            gdw_resolution counts cells of the flowchart's grid for the
 *            scale, N_g = Int(400 k_w + 150), where it spans 10-12 scale
 *            lengths, and the same physical extent is kept on the n^3 grid
 *            (the count itself when n = N_g).  No images; applied in real
 *            space as hf_cwt_stencil does.  Taken by hf_cwt,
 *            hf_find_halos and hf_find_halos_filtered (half-widths up to
 *            HF_STENCIL_MAX_HALF_WIDTH, else HF_ERR_ARG); the batched and
 *            multi-scale calls, which share FFT passes, return HF_ERR_ARG. */
typedef enum { HF_KERNEL_SAMPLED = 0, HF_KERNEL_ANALYTIC = 1, HF_KERNEL_STENCIL = 2 } hf_kernel;

/* Periodic box: n^3 grid on a side of box_len (Mpc/h); node g sits at g*box_len/n. */
typedef struct {
    int32_t n;
    int32_t frac_bits;
    double box_len;
} hf_box;

/* Stage selectors for hf_workspace_size (bit mask: the result covers every
 * selected stage, so one buffer can serve them in turn).  HF_STAGE_LABEL
 * together with HF_STAGE_DEPOSIT adds, where the binned deposit applies (see
 * hf_find_halos), a region that carries the deposit's particle order to the
 * label step: about 13 bytes per particle plus 8 per particle of label scratch. */
enum { HF_STAGE_DEPOSIT = 1, HF_STAGE_CWT = 2, HF_STAGE_MAXIMA = 4, HF_STAGE_SEGMENT = 8, HF_STAGE_LABEL = 16,
       HF_STAGE_ALL = 31, HF_STAGE_GROUPS = 32 /* hf_groups; not part of HF_STAGE_ALL */,
       HF_STAGE_STENCIL = 64 /* hf_cwt_stencil; not part of HF_STAGE_ALL */ };

typedef struct hf_ctx hf_ctx;

/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the default stream).  Allocates a 256-byte device
 * status block and a pinned host mirror, freed by hf_destroy. */
hf_status hf_create(int device, void *hip_stream, hf_ctx **out);
hf_status hf_destroy(hf_ctx *ctx);
const char *hf_status_str(hf_status s);

/* Wait for the context's stream, then return (and clear) the first
 * device-detected error, highest code first: INPUT, OVERFLOW, CAPACITY. */
hf_status hf_sync(hf_ctx *ctx);

/* Bytes of workspace the selected stages need for this box and particle count. */
hf_status hf_workspace_size(const hf_box *box, int64_t np, int stage_mask, size_t *bytes);

/* Step 2, Eq. (1): cloud-in-cell deposit.
 *  pos [np][3] (dtype), rho [n][n][n] int64 (overwritten).
 *  Per axis, s = n 2^B / box_len is rounded once to the position dtype,
 *  t = x*s is one correctly rounded multiply in that dtype, q = floor(t) mod
 *  n 2^B, cell = q >> B, f = q & (2^B - 1); the lower node gets weight 2^B - f,
 *  the upper node (periodic) f.  Each of the 8 corners gets the product of its
 *  three weights (one particle = 2^3B).  Sums are exact int64 and independent
 *  of particle order.  A cell above 2^63 - 1 -> HF_ERR_OVERFLOW; a position
 *  with non-finite t or |t| >= 2^62 -> HF_ERR_INPUT (that particle is skipped).
 *  np == 0 gives an all-zero grid.  Workspace: HF_STAGE_DEPOSIT. */
hf_status hf_deposit(hf_ctx *ctx, const hf_box *box, const void *pos, hf_dtype dtype,
                     int64_t np, int64_t *rho, void *ws, size_t ws_bytes);

/* Step 3, Eqs. (2)-(4): grid CWT at scale k_w = w box_len / 1000 (step 1).
 *  rho [n][n][n] int64 (>= 0, not all zero); cwt [n][n][n] FP32 (overwritten).
 *  C_j = sum_g f_g K(x_j - x_g) with f = rho / mean(rho) (mean density units)
 *  and K the kernel selected by `kernel` (dx^3 Psi sampled, or the analytic
 *  transform), computed as a real 3D FFT, a multiply and an inverse FFT in FP32.
 *  The mean is formed from the exact integer total in FP64.  Negative or
 *  all-zero rho -> HF_ERR_INPUT.  Workspace: HF_STAGE_CWT (HF_STAGE_STENCIL
 *  with HF_KERNEL_STENCIL). */
hf_status hf_cwt(hf_ctx *ctx, const hf_box *box, const int64_t *rho, double kw, hf_kernel kernel,
                 float *cwt, void *ws, size_t ws_bytes);

/* Step 3 by the paper's own discretisation (Sec. 2.1, Eq. (2) last line):
 * every grid point adds its mass times the wavelet of Eq. (4), sampled at the
 * grid spacing on the cube of node offsets |d_i| <= half_width around it
 * (periodic; no wavelet images).  Table 1's gdw_resolution, Int(1.5/k_w + 5),
 * is the paper's half_width on its grid N_g = Int(400 k_w + 150); HF_KERNEL_STENCIL
 * keeps that extent on other grids.  A stencil wider than the box wraps onto
 * itself.
 *  rho [n][n][n] int64 (>= 0, not all zero); cwt [n][n][n] FP32 (overwritten).
 *  C_j = sum_{|d_i| <= h} S_d f_{j-d}, f = rho / mean(rho) as in hf_cwt and
 *  S_d = dx^3 Psi(w, |d| dx).  Computed in FP32 as seven one-dimensional
 *  convolutions in three passes (the cube stencil is a sum of four separable
 *  terms); weights and the mean in FP64.  0 <= half_width <=
 *  HF_STENCIL_MAX_HALF_WIDTH, else HF_ERR_ARG.  rho and cwt must not overlap
 *  each other or the workspace.  Negative or all-zero rho -> HF_ERR_INPUT.
 *  Workspace: HF_STAGE_STENCIL (three FP32 grids). */
#define HF_STENCIL_MAX_HALF_WIDTH 64
/* The half-width HF_KERNEL_STENCIL takes on an n^3 grid at scale kw (Table 1's
 * gdw_resolution kept at its extent on the flowchart's grid N_g, see
 * hf_kernel): ceil(Int(1.5/k_w + 5) n / Int(400 k_w + 150)).  Host only, no
 * context.  HF_ERR_ARG for a null out pointer, kw not finite and positive, n
 * outside [1, 1024], or a result above HF_STENCIL_MAX_HALF_WIDTH. */
hf_status hf_stencil_half_width(double kw, int32_t n, int32_t *half_width);
hf_status hf_cwt_stencil(hf_ctx *ctx, const hf_box *box, const int64_t *rho, double kw, int32_t half_width,
                         float *cwt, void *ws, size_t ws_bytes);

/* Step 4: local maxima.  Cell j is a maximum iff (C_j, j) beats all 26
 * periodic neighbours in the order "larger value, then larger index"
 * (-0 equals +0) and C_j > tau.  max_idx receives the maxima's linear indices
 * in increasing order (at most max_cap of them); *d_count (device int64)
 * receives the total number found.  More than max_cap -> HF_ERR_CAPACITY.
 * NaN in cwt -> HF_ERR_INPUT.  Workspace: HF_STAGE_MAXIMA. */
hf_status hf_maxima(hf_ctx *ctx, const hf_box *box, const float *cwt, float tau,
                    int32_t *max_idx, int64_t max_cap, int64_t *d_count, void *ws, size_t ws_bytes);

/* Step 5, Sec. 2.3: segmentation by steepest ascent.  Each cell's parent is
 * the largest of itself and its 26 neighbours in the order above; following
 * parents ends at a local maximum (the root).  cell_label [n][n][n] int32
 * receives the root's linear index if C_root > tau, else -1.  Roots above tau
 * are exactly the hf_maxima list.  NaN -> HF_ERR_INPUT.
 * Workspace: HF_STAGE_SEGMENT. */
hf_status hf_segment(hf_ctx *ctx, const hf_box *box, const float *cwt, float tau,
                     int32_t *cell_label, void *ws, size_t ws_bytes);

/* Step 6: particle labels.  Each particle's node is the one with its largest
 * CIC weight, ((q + 2^(B-1)) >> B) mod n per axis with q as in hf_deposit
 * (half a cell goes up); particle_label[i] = cell_label[node].  Positions
 * hf_deposit would reject get label -1 and set HF_ERR_INPUT. */
hf_status hf_label(hf_ctx *ctx, const hf_box *box, const void *pos, hf_dtype dtype, int64_t np,
                   const int32_t *cell_label, int32_t *particle_label);

/* Steps 5 and 7 with Table 1's thresholds: group statistics and filters.
 * A group is the set of cells and particles carrying one label (a root of the
 * segmentation).  For every root of roots[0..nroots) (the strictly increasing
 * hf_maxima list whose labels cell_label and particle_label carry):
 *   group_cells[i]      cells labelled roots[i] (the grid volume, step 5, in
 *                       cells of volume (box_len/n)^3),
 *   group_particles[i]  particles labelled roots[i] (the group's mass in
 *                       particles, which have equal mass),
 *   group_keep[i]       1 iff the group's density is at least dens_th times the
 *                       box's mean density np / box_len^3 (step 7; Table 1:
 *                       dens_th = 4) and it has at least particle_th particles
 *                       (Table 1: particle_th = 15) and, when root_ok is given
 *                       (device [nroots] flags, e.g. from hf_cross_scale),
 *                       root_ok[i] != 0; else 0.  The density test is decided
 *                       in FP64 as
 *                       double(P) * n^3 >= (dens_th * double(V)) * double(np).
 * cell_label_out [n^3] and particle_label_out [np] (either may be NULL, and
 * either may be the corresponding input) receive the labels with those of
 * disposed groups replaced by -1; with nroots == 0 every label becomes -1.
 * np is the number of particles in the box (all of them, labelled or not),
 * at most 2^32 - 1; particle_label may be NULL when np == 0.
 * Errors: HF_ERR_ARG for a null required pointer, np or nroots out of range,
 * a negative or non-finite dens_th or a negative particle_th; a label outside
 * [-1, n^3) or a root outside [0, n^3) sets HF_ERR_INPUT (the label is
 * treated as -1).  Labels >= 0 that are not among the roots give undefined
 * statistics for themselves (never a memory fault).
 * Workspace: HF_STAGE_GROUPS (8 bytes per cell; only the roots' entries are
 * touched).  The size hf_workspace_size reports for HF_STAGE_GROUPS alone
 * adds 4 bytes per particle and n^3/8 bytes, for a partitioned count and a
 * keep bitmap (much faster on labels in input order); a workspace of the
 * counters' size alone (np == 0 in the query) is accepted and counts with one
 * global atomic per labelled particle.  Either way the results are the same. */
hf_status hf_groups(hf_ctx *ctx, const hf_box *box, int64_t np, const int32_t *roots, int64_t nroots,
                    const int32_t *cell_label, const int32_t *particle_label, double dens_th,
                    int64_t particle_th, const uint8_t *root_ok, uint32_t *group_particles, uint32_t *group_cells,
                    uint8_t *group_keep, int32_t *cell_label_out, int32_t *particle_label_out, void *ws,
                    size_t ws_bytes);

/* Step 4's correction of the grid maxima for the finite grid (App. B).  For
 * each maximum roots[i] (device, e.g. hf_maxima's list) of the FP32 field cwt:
 * per axis, with the maximum B and its two periodic neighbours A (the larger)
 * and C (the smaller), l1 = A - C and l2 = B - C, the quadratic through them
 * peaks l1^2 / (16 l2 - 8 l1) above B and l1 / (2 (2 l2 - l1)) cells from B
 * towards A; a flat axis (l2 = 0) adds nothing.  value[i] = B plus the three
 * axes' corrections; pos[3 i + 0..2] = (x, y, z) of B plus the shifts, in
 * box_len units, wrapped into [0, box_len).  FP64, each operation rounded as
 * written (no contraction).  pos [nroots][3], value [nroots]: device doubles.
 * A NaN or a root outside [0, n^3) sets HF_ERR_INPUT.  The comparison of
 * maxima between grids of different spacing (the rest of App. B) does not
 * arise: every scale of a box uses one grid. */
hf_status hf_peaks(hf_ctx *ctx, const hf_box *box, const float *cwt, const int32_t *roots, int64_t nroots,
                   double *pos, double *value);

/* Step 8: cross-scale maxima, each maximum first corrected for the grid as
 * step 4 asks (App. B).  For maximum roots[i] of cwt_scale (n^3, the box's
 * grid): its value becomes the top of its per-axis quadratics (as hf_peaks)
 * plus App. B's cube-size term for the smaller scale's grid with the paper's
 * 3/5 factor removed, (5/16)(2 l2bar - l1bar)(1 - (n / n_smaller)^2), l1bar and
 * l2bar the means of l1 and l2 over the three axes (zero when
 * n_smaller == n).  pass[i] = 1 iff that value (FP64) strictly exceeds
 * cwt_smaller (n_smaller^3 FP32 over the same box: the CWT at the adjacent
 * smaller scale, the flowchart's current grid) at the node of that grid
 * nearest the corrected position, ((g + shift) n_smaller) / n in its cells
 * with half a cell rounding up, and at that node's 26 periodic neighbours.
 * roots [nroots] (device, e.g. hf_maxima's list at this scale), pass [nroots]
 * (device).  n_smaller in [1, 1024].  A NaN in either field or a root outside
 * [0, n^3) sets HF_ERR_INPUT.  The flags can go to hf_groups as root_ok
 * (groups without a cross-scale maximum are disposed of).  No workspace. */
hf_status hf_cross_scale(hf_ctx *ctx, const hf_box *box, const int32_t *roots, int64_t nroots,
                         const float *cwt_scale, int32_t n_smaller, const float *cwt_smaller, uint8_t *pass);

/* Batched step 3 for serving: `count` (1..HF_CWT_BATCH_MAX) transforms of the
 * same grid size n, each with its own box length and scale, enqueued as one
 * launch per pass (the job is a grid dimension).  items[] is a HOST array read
 * during the call; rho/cwt in each item are device pointers as in hf_cwt, and
 * each job gets exactly the result hf_cwt would give it alone.  The workspace
 * holds count per-job workspaces: hf_cwt_batch_ws_size(n, count, &bytes). */
#define HF_CWT_BATCH_MAX 32
typedef struct {
    const int64_t *rho;
    float *cwt;
    double box_len;
    double kw;
} hf_cwt_item;
hf_status hf_cwt_batch_ws_size(int32_t n, int32_t count, size_t *bytes);

/* Step 3 at `count` (1..HF_CWT_BATCH_MAX) scales of one density grid (the
 * identification loop of Sec. 2 visits one scale after another, step 1):
 * the forward transform of rho (x and y passes, and the mean density) is made
 * once, then each scale applies its multiplier (Eq. (4)) in its own z pass and
 * its own inverse transform.  kws[] and cwts[] are HOST arrays (cwts holds
 * device pointers to [n^3] FP32 outputs); cwts[s] receives exactly what hf_cwt
 * gives at kws[s].  Workspace: hf_cwt_batch_ws_size(n, count) (one half
 * spectrum and table set per scale). */
hf_status hf_cwt_scales(hf_ctx *ctx, const hf_box *box, const int64_t *rho, int32_t count, const double *kws,
                        hf_kernel kernel, float *const *cwts, void *ws, size_t ws_bytes);
hf_status hf_cwt_batch(hf_ctx *ctx, int32_t n, int32_t count, const hf_cwt_item *items, hf_kernel kernel,
                       void *ws, size_t ws_bytes);

/* Steps 2-6 for one box in a single call (no host synchronisation inside):
 * hf_deposit, hf_cwt, hf_maxima, hf_segment and hf_label in order on the
 * context's stream, all sharing one workspace of
 * hf_workspace_size(box, np, HF_STAGE_ALL) bytes (| HF_STAGE_STENCIL with
 * HF_KERNEL_STENCIL).  Where the deposit bins the
 * particles (n a multiple of 16 with more than 512 tiles of 16-64 x 8 x 8
 * cells, frac_bits <= 17, np < 2^32) the binned order is kept and step 6 runs
 * through it: records are labelled tile by tile and the labels brought back
 * to input order, with the same result as hf_label.  Device-detected errors are
 * reported by hf_sync as for the separate calls. */
typedef struct {
    const void *pos;         /* [np][3] positions */
    int64_t np;
    hf_dtype dtype;
    double kw;               /* scale k_w = w box_len / 1000 */
    hf_kernel kernel;
    float tau;               /* peak threshold (0 in the paper's reading) */
    int64_t *rho;            /* [n^3] int64 density */
    float *cwt;              /* [n^3] FP32 CWT */
    int32_t *max_idx;        /* [max_cap] sorted maxima */
    int64_t max_cap;
    int64_t *d_count;        /* device int64: number of maxima */
    int32_t *cell_label;     /* [n^3] */
    int32_t *particle_label; /* [np] */
} hf_job;
hf_status hf_find_halos(hf_ctx *ctx, const hf_box *box, const hf_job *job, void *ws, size_t ws_bytes);

/* hf_find_halos for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same steps and results, with no workspace argument.  Its workspace is a
 * static device array of HF_NOALLOC_SCRATCH_BYTES (64 MiB) per device, made
 * resident when the first context on that device is created and held until the
 * process ends; the call itself allocates nothing.  Enough for every box whose
 * hf_workspace_size(box, np, HF_STAGE_ALL) (plus HF_STAGE_STENCIL with that
 * transform) fits, e.g. n <= 128 with up to 2 n^3 particles; larger jobs get
 * HF_ERR_WORKSPACE before anything is enqueued.  Every call on a device
 * shares that device's array: calls that overlap on one device (two streams,
 * or two host threads) race and must be serialised by the caller.  The
 * array's contents persist between calls; the steps never read what they have
 * not written in the same call.  HF_ERR_DEVICE if the array's address could
 * not be resolved when the context was created. */
#define HF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
hf_status hf_find_halos_noalloc(hf_ctx *ctx, const hf_box *box, const hf_job *job);

/* Steps 2-6 as hf_find_halos, then steps 5 and 7 as hf_groups on its own
 * results (the roots are job->max_idx[0 .. min(*d_count, max_cap))):
 * job->cell_label keeps the segmentation, job->particle_label receives the
 * labels AFTER the filter (disposed groups -> -1), gf->group_* [max_cap] are
 * indexed like job->max_idx (entries past the count are not written), and
 * gf->cell_label_kept [n^3] (may be NULL) receives the filtered cell labels.
 * With the binned deposit each label's particles are counted in the deposit's
 * tile order and the filter is applied on the way back to input order.
 * job->np must be below 2^32.  Workspace:
 * hf_workspace_size(box, np, HF_STAGE_ALL | HF_STAGE_GROUPS) (| HF_STAGE_STENCIL
 * with HF_KERNEL_STENCIL). */
typedef struct {
    double dens_th;            /* Table 1: 4 */
    int64_t particle_th;       /* Table 1: 15 */
    uint32_t *group_particles; /* [max_cap] */
    uint32_t *group_cells;     /* [max_cap] */
    uint8_t *group_keep;       /* [max_cap] */
    int32_t *cell_label_kept;  /* [n^3] or NULL */
} hf_group_filter;
hf_status hf_find_halos_filtered(hf_ctx *ctx, const hf_box *box, const hf_job *job, const hf_group_filter *gf,
                                 void *ws, size_t ws_bytes);

/* Steps 2-6 of one box at `count` (1..HF_CWT_BATCH_MAX) scales, as the
 * identification loop of Sec. 2 visits scales one after another: one deposit
 * into rho, one forward transform shared by every scale (as hf_cwt_scales),
 * then per scale its inverse transform, maxima, segmentation and particle
 * labels (through the deposit's particle order where it bins, as
 * hf_find_halos).  Each scale's outputs equal those of hf_find_halos at its
 * k_w.  scales[] is a HOST array of device output pointers; pos, np, dtype,
 * kernel and tau as in hf_job.  Workspace: hf_find_halos_scales_ws_size. */
typedef struct {
    double kw;               /* scale k_w = w box_len / 1000 */
    float *cwt;              /* [n^3] FP32 CWT at this scale */
    int32_t *max_idx;        /* [max_cap] sorted maxima */
    int64_t max_cap;
    int64_t *d_count;        /* device int64: number of maxima */
    int32_t *cell_label;     /* [n^3] */
    int32_t *particle_label; /* [np] */
} hf_scale_job;
hf_status hf_find_halos_scales_ws_size(const hf_box *box, int64_t np, int32_t count, size_t *bytes);
hf_status hf_find_halos_scales(hf_ctx *ctx, const hf_box *box, const void *pos, hf_dtype dtype, int64_t np,
                               hf_kernel kernel, float tau, int64_t *rho, int32_t count, const hf_scale_job *scales,
                               void *ws, size_t ws_bytes);

/* Sec. 2's identification loop over scales (steps 2-8; the self-boundness
 * check of steps 9-10 is not made), as its flowchart runs it with a pair of
 * grids, on the box's one n^3 grid.  scales[0..count) in strictly increasing
 * k_w (largest scale length first).  Every scale's field, maxima, segmentation
 * and step-6 labels are made as hf_find_halos_scales makes them; then, scale
 * by scale: particles claimed by an earlier scale are given label -1; the
 * groups of the remaining particles are measured (steps 5 and 7, as hf_groups,
 * with the mean density of all np particles); a group is kept iff it passes
 * dens_th and particle_th and its maximum exceeds the next scale's field at
 * its cell and 26 neighbours (step 8; after the last scale, the zero grid);
 * the kept groups' particles are claimed.
 * On return:
 *  scales[j].particle_label [np]: the root of the kept group that claimed the
 *    particle at scale j, else -1 (so each particle is >= 0 at one scale at most);
 *  scales[j].cell_label: scale j's whole segmentation (unfiltered);
 *  groups[j]: per maximum of scale j (indexed like its max_idx) the particles
 *    still unclaimed in its group, its cells, and 1 iff it became a halo;
 *  halo_scale [np]: the scale index that claimed the particle, -1 for none;
 *  halo_root [np]: the root cell of that group, -1 for none.
 * scales[] and groups[] are HOST arrays of device pointers.
 * Workspace: hf_identify_ws_size (that of hf_find_halos_scales, the group
 * counters and one byte per maximum of the largest list). */
typedef struct {
    uint32_t *group_particles; /* [max_cap] */
    uint32_t *group_cells;     /* [max_cap] */
    uint8_t *group_keep;       /* [max_cap] */
} hf_identify_groups;
hf_status hf_identify_ws_size(const hf_box *box, int64_t np, int32_t count, const hf_scale_job *scales,
                              size_t *bytes);
hf_status hf_identify(hf_ctx *ctx, const hf_box *box, const void *pos, hf_dtype dtype, int64_t np, hf_kernel kernel,
                      float tau, int64_t *rho, int32_t count, const hf_scale_job *scales,
                      const hf_identify_groups *groups, double dens_th, int64_t particle_th, int32_t *halo_scale,
                      int32_t *halo_root, void *ws, size_t ws_bytes);

/* Sec. 2's identification loop on per-scale grids (step 1 and the flowchart:
 * each scale is gridded afresh, N_g = Int(400 k_w + 150) points per side).
 * Scale j (scales[] in increasing kw, so the largest scale length comes first)
 * deposits the np particles on its own n_j^3 grid (any 8 <= n_j <= 1024) into
 * rho, takes the grid CWT by the paper's truncated stencil (Sec. 2.1; as
 * hf_cwt_stencil with hf_stencil_half_width(kw, n_j), which is Table 1's
 * count when n_j = N_g), then its maxima (capacity max_cap) and segmentation.
 * Then, scale by scale, steps 6-8 as hf_identify does in input order: the
 * step-8 flags of the scale's maxima against the next scale's field on that
 * scale's own grid (hf_cross_scale, whose App. B cube-size term corrects for
 * the two grid spacings; after the last scale the zero grid of its own size),
 * the particles no earlier scale claimed take their cell's label, the groups'
 * cell and particle counts and the step-7/8 decision (hf_groups' test with n_j,
 * dens_th, particle_th), and the kept groups claim their particles.
 * With velocities vel [np][3] (km/s, the dtype of pos; NULL skips it) steps
 * 9 and 10 follow at every scale (hf_unbind with grav_mass = G m_p): the kept
 * groups' self-boundness check, bound_keep [max_cap] receiving its decision,
 * and only the bound particles of the groups that pass are claimed; the others
 * stay free for the later scales.
 * particle_label [np] receives the scale's filtered labels (-1 unless the
 * particle is claimed at this scale); halo_scale/halo_root [np] as hf_identify.
 * All pointers are device pointers.  Errors: HF_ERR_ARG for a null required
 * pointer, scales not in increasing kw, count outside 1..HF_CWT_BATCH_MAX, a
 * max_cap above n_j^3, a stencil half-width above HF_STENCIL_MAX_HALF_WIDTH,
 * np above 2^31 - 1, a non-positive grav_mass with velocities;
 * HF_ERR_SIZE for an n_j outside [8, 1024] or frac_bits outside [8, 20].
 * Workspace: hf_identify_grids_ws_size (the largest scale's stage workspace,
 * or the check's with velocities, its group counters and one byte per
 * maximum of the largest list). */
typedef struct {
    double kw;                 /* scale k_w = w box_len / 1000 */
    int32_t n;                 /* this scale's grid points per side */
    int64_t *rho;              /* [n^3] int64: CIC density on this grid */
    float *cwt;                /* [n^3] FP32 grid CWT */
    int32_t *max_idx;          /* [max_cap] sorted maxima */
    int64_t max_cap;
    int64_t *d_count;          /* device int64: number of maxima */
    int32_t *cell_label;       /* [n^3] */
    int32_t *particle_label;   /* [np] */
    uint32_t *group_particles; /* [max_cap] */
    uint32_t *group_cells;     /* [max_cap] */
    uint8_t *group_keep;       /* [max_cap] steps 7-8 */
    uint8_t *bound_keep;       /* [max_cap] steps 9-10 (with velocities; else unused, may be NULL) */
} hf_grid_scale;
hf_status hf_identify_grids_ws_size(double box_len, int32_t frac_bits, int64_t np, int32_t count,
                                    const hf_grid_scale *scales, int32_t with_velocities, size_t *bytes);
hf_status hf_identify_grids(hf_ctx *ctx, double box_len, int32_t frac_bits, const void *pos, const void *vel,
                            hf_dtype dtype, int64_t np, float tau, int32_t count, const hf_grid_scale *scales,
                            double dens_th, int64_t particle_th, double grav_mass, int32_t *halo_scale,
                            int32_t *halo_root, void *ws, size_t ws_bytes);

/* Steps 9-10 (Sec. 2.3): the self-boundness check of one scale's groups.  For
 * every root i with group_keep[i] != 0, its group is the particles whose
 * particle_label is roots[i] (n^3 grid of box; roots and labels as hf_groups);
 * repeatedly, with the remaining particles: their centre of mass (positions
 * unwrapped about the root's node by minimum image) and mean velocity, each
 * one's radius r, the spherical shell potential
 *   Phi_i = -grav_mass [ (particles at or inside (r_i, index i)) / r_i
 *                        + sum over those outside of 1 / r_j ]
 * and the particles with |v - mean|^2 > -2 Phi_i leave, until none leaves.
 * bound_keep[i] = 1 iff no more than 40% left (5 removed <= 2 N) and at least
 * max(1, particle_th) remain.  particle_label (in/out) keeps only the bound
 * particles of the groups with bound_keep set; every other label becomes -1.
 * pos, vel [np][3] in dtype (vel in km/s), grav_mass = G m_p in
 * (Mpc/h)(km/s)^2 (equal particle masses), all in FP64 arithmetic.  Readings:
 * peculiar velocities, no Hubble flow; a particle at r = 0 is bound.  Errors:
 * HF_ERR_ARG for a null required pointer, np outside [0, 2^31 - 1], nroots
 * outside [0, n^3], a non-positive grav_mass or a negative particle_th; a
 * label >= 0 that is not among the roots, or a root outside [0, n^3), sets
 * HF_ERR_INPUT (the label becomes -1).  Workspace: hf_unbind_ws_size (a slot
 * per cell, and 29 bytes per particle). */
hf_status hf_unbind_ws_size(const hf_box *box, int64_t np, int64_t nroots, size_t *bytes);
hf_status hf_unbind(hf_ctx *ctx, const hf_box *box, const void *pos, const void *vel, hf_dtype dtype, int64_t np,
                    const int32_t *roots, int64_t nroots, const uint8_t *group_keep, int32_t *particle_label,
                    double grav_mass, int64_t particle_th, uint8_t *bound_keep, void *ws, size_t ws_bytes);

/* Serving form of steps 2-6 for `count` (1..HF_CWT_BATCH_MAX) boxes of the same
 * grid size n: per-box deposits, ONE batched transform (hf_cwt_batch) for the
 * group, then per-box maxima, segmentation and labels, all on the context's
 * stream.  items[] is a host array read during the call.  Each item carries its
 * box length and its own workspace of hf_workspace_size(box, np,
 * HF_STAGE_DEPOSIT | HF_STAGE_MAXIMA | HF_STAGE_SEGMENT) bytes; cwt_ws holds
 * hf_cwt_batch_ws_size(n, count) bytes.  All jobs must use `kernel`.  Every box
 * gets exactly the results hf_find_halos would give it alone. */
typedef struct {
    hf_job job;
    double box_len;
    void *ws;
    size_t ws_bytes;
} hf_group_item;
hf_status hf_find_halos_group(hf_ctx *ctx, int32_t n, int32_t frac_bits, int32_t count,
                              const hf_group_item *items, hf_kernel kernel, void *cwt_ws, size_t cwt_ws_bytes);

/* Kernel timer (a tracing aid, not part of the method).  When enabled, every
 * kernel launch made through this context is bracketed by HIP events on its
 * stream.  hf_profile_read(ctx, i, ...) waits for the stream and returns the
 * name, accumulated milliseconds and launch count of kernel i, for
 * i in [0, count); an index past the end returns HF_ERR_ARG.  The name string
 * is static.  hf_profile_reset zeroes the totals. */
hf_status hf_profile_enable(hf_ctx *ctx, int enable);
hf_status hf_profile_reset(hf_ctx *ctx);
hf_status hf_profile_read(hf_ctx *ctx, int index, const char **name, double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* HF_H */
