// Steps 2-6 of one box in a single native call (Sec. 2, identification steps).
#include "hf_internal.h"

using namespace hf;

extern "C" hf_status hf_find_halos(hf_ctx *ctx, const hf_box *box, const hf_job *job, void *ws, size_t ws_bytes) {
    if (!ctx || !job) return HF_ERR_ARG;
    hf_status s = check_box_for(box, job->kernel);
    if (s != HF_OK) return s;
    size_t need = 0;
    s = hf_workspace_size(box, job->np, pipeline_stages(job->kernel), &need);
    if (s != HF_OK) return s;
    s = check_ws(ws, ws_bytes, need);
    if (s != HF_OK) return s;
    // argument checks of every stage run before anything is enqueued
    if (!job->rho || !job->cwt || !job->d_count || !job->cell_label || job->np < 0 || job->max_cap < 0 ||
        (job->max_cap > 0 && !job->max_idx) || (job->np > 0 && (!job->pos || !job->particle_label)) ||
        (job->dtype != HF_F32 && job->dtype != HF_F64) ||
        (job->kernel != HF_KERNEL_SAMPLED && job->kernel != HF_KERNEL_ANALYTIC && job->kernel != HF_KERNEL_STENCIL) ||
        !(job->kw > 0.0) || (job->kernel == HF_KERNEL_STENCIL && stencil_half_width(job->kw, box->n) < 0) ||
        job->tau != job->tau)
        return HF_ERR_ARG;
    // With the binned deposit the particle order it builds is kept (in front of
    // the workspace) and step 6 reuses it; every other stage gets the rest.
    const bool order = particle_order_supported(*box, job->np);
    char *sw = static_cast<char *>(ws);
    size_t sb = ws_bytes;
    ParticleOrder po{};
    if (order) {
        po = particle_order_at(*box, ws, job->np);
        sw += particle_order_bytes(*box, job->np);
        sb -= particle_order_bytes(*box, job->np);
        if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
        s = deposit_tiled(ctx, *box, job->pos, job->dtype, job->np, job->rho, sw, &po);
    } else {
        s = hf_deposit(ctx, box, job->pos, job->dtype, job->np, job->rho, sw, sb);
    }
    if (s != HF_OK) return s;
    s = hf_cwt(ctx, box, job->rho, job->kw, job->kernel, job->cwt, sw, sb);
    if (s != HF_OK) return s;
    s = maxima_segment(ctx, *box, job->cwt, job->tau, job->max_idx, job->max_cap, job->d_count, job->cell_label, sw,
                       sb);
    if (s != HF_OK) return s;
    if (order) return label_from_order(ctx, *box, job->np, po, job->cell_label, job->particle_label, sw);
    return hf_label(ctx, box, job->pos, job->dtype, job->np, job->cell_label, job->particle_label);
}

// Steps 2-6 as hf_find_halos, then the group statistics and filters of steps 5
// and 7.  Through the kept particle order, step 6 counts each label's particles
// in tile order and its pass back to input order drops the disposed groups;
// otherwise the labels are counted and filtered in input order.
extern "C" hf_status hf_find_halos_filtered(hf_ctx *ctx, const hf_box *box, const hf_job *job,
                                           const hf_group_filter *gf, void *ws, size_t ws_bytes) {
    if (!ctx || !job || !gf) return HF_ERR_ARG;
    hf_status s = check_box_for(box, job->kernel);
    if (s != HF_OK) return s;
    const int64_t ncells = int64_t(box->n) * box->n * box->n;
    if (!(gf->dens_th >= 0.0) || !(gf->dens_th < 1e300) || gf->particle_th < 0 || job->np > int64_t(UINT32_MAX))
        return HF_ERR_ARG;
    if (job->max_cap > 0 && (!gf->group_particles || !gf->group_cells || !gf->group_keep)) return HF_ERR_ARG;
    if (job->max_cap > ncells) return HF_ERR_ARG;
    size_t need = 0;
    s = hf_workspace_size(box, job->np, pipeline_stages(job->kernel) | HF_STAGE_GROUPS, &need);
    if (s != HF_OK) return s;
    s = check_ws(ws, ws_bytes, need);
    if (s != HF_OK) return s;
    if (!job->rho || !job->cwt || !job->d_count || !job->cell_label || job->np < 0 || job->max_cap < 0 ||
        (job->max_cap > 0 && !job->max_idx) || (job->np > 0 && (!job->pos || !job->particle_label)) ||
        (job->dtype != HF_F32 && job->dtype != HF_F64) ||
        (job->kernel != HF_KERNEL_SAMPLED && job->kernel != HF_KERNEL_ANALYTIC && job->kernel != HF_KERNEL_STENCIL) ||
        !(job->kw > 0.0) || (job->kernel == HF_KERNEL_STENCIL && stencil_half_width(job->kw, box->n) < 0) ||
        job->tau != job->tau)
        return HF_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    const bool order = particle_order_supported(*box, job->np);
    char *sw = static_cast<char *>(ws);
    size_t sb = ws_bytes;
    ParticleOrder po{};
    GroupCounters g{};
    if (order) {
        po = particle_order_at(*box, ws, job->np);
        sw += particle_order_bytes(*box, job->np);
        sb -= particle_order_bytes(*box, job->np);
        g = group_counters_at(*box, sw);
        sw += groups_ws_bytes(*box);
        sb -= groups_ws_bytes(*box);
        s = deposit_tiled(ctx, *box, job->pos, job->dtype, job->np, job->rho, sw, &po);
    } else {
        s = hf_deposit(ctx, box, job->pos, job->dtype, job->np, job->rho, sw, sb);
    }
    if (s != HF_OK) return s;
    s = hf_cwt(ctx, box, job->rho, job->kw, job->kernel, job->cwt, sw, sb);
    if (s != HF_OK) return s;
    s = maxima_segment(ctx, *box, job->cwt, job->tau, job->max_idx, job->max_cap, job->d_count, job->cell_label, sw,
                       sb);
    if (s != HF_OK) return s;
    const int64_t cap = job->max_cap;
    if (order) {
        s = groups_count_cells(ctx, *box, job->max_idx, job->d_count, cap, job->cell_label, g);
        if (s == HF_OK) s = label_tiles(ctx, *box, job->np, po, job->cell_label, sw, cap > 0 ? g.parts : nullptr);
        if (s == HF_OK)
            s = groups_decide(ctx, *box, job->max_idx, job->d_count, cap, g, gf->dens_th, job->np, gf->particle_th,
                              nullptr, gf->group_particles, gf->group_cells, gf->group_keep);
        if (s == HF_OK && cap > 0) s = label_back(ctx, *box, job->np, po, job->particle_label, sw, g.cells);
        if (s == HF_OK && cap == 0) {
            s = label_back(ctx, *box, job->np, po, job->particle_label, sw, nullptr);
            if (s == HF_OK) s = groups_filter(ctx, *box, job->particle_label, job->particle_label, job->np, g, false);
        }
    } else {
        // the shared region is free again once the segmentation is done
        g = group_counters_at(*box, sw);
        s = hf_label(ctx, box, job->pos, job->dtype, job->np, job->cell_label, job->particle_label);
        if (s == HF_OK) s = groups_count_cells(ctx, *box, job->max_idx, job->d_count, cap, job->cell_label, g);
        if (s == HF_OK && cap > 0) s = groups_count_particles(ctx, *box, job->particle_label, job->np, g);
        if (s == HF_OK)
            s = groups_decide(ctx, *box, job->max_idx, job->d_count, cap, g, gf->dens_th, job->np, gf->particle_th,
                              nullptr, gf->group_particles, gf->group_cells, gf->group_keep);
        if (s == HF_OK)
            s = groups_filter(ctx, *box, job->particle_label, job->particle_label, job->np, g, cap > 0);
    }
    if (s == HF_OK && gf->cell_label_kept)
        s = groups_filter(ctx, *box, job->cell_label, gf->cell_label_kept, ncells, g, cap > 0);
    return s;
}

// Steps 2-6 of one box at several scales: one deposit (and, where it bins,
// one kept particle order), one forward transform shared by every scale
// (hf_cwt_scales), then per scale the multiplier and inverse transform,
// maxima and segmentation, and the labels through the same particle order.
extern "C" hf_status hf_find_halos_scales_ws_size(const hf_box *box, int64_t np, int32_t count, size_t *bytes) {
    if (!bytes || np < 0 || count < 1 || count > HF_CWT_BATCH_MAX) return HF_ERR_ARG;
    hf_status s = check_box(box);
    if (s != HF_OK) return s;
    size_t all = 0, cw = 0;
    s = hf_workspace_size(box, np, HF_STAGE_ALL, &all);
    if (s == HF_OK) s = hf_cwt_batch_ws_size(box->n, count, &cw);
    if (s != HF_OK) return s;
    const size_t ord = particle_order_supported(*box, np) ? particle_order_bytes(*box, np) : 0;
    const size_t shared = all - ord;  // every stage's share, one transform included
    *bytes = ord + (shared > cw ? shared : cw);
    return HF_OK;
}

extern "C" hf_status hf_find_halos_scales(hf_ctx *ctx, const hf_box *box, const void *pos, hf_dtype dtype, int64_t np,
                                          hf_kernel kernel, float tau, int64_t *rho, int32_t count,
                                          const hf_scale_job *scales, void *ws, size_t ws_bytes) {
    if (!ctx || !rho || !scales || count < 1 || count > HF_CWT_BATCH_MAX || np < 0 || (np > 0 && !pos)) return HF_ERR_ARG;
    if ((dtype != HF_F32 && dtype != HF_F64) || (kernel != HF_KERNEL_SAMPLED && kernel != HF_KERNEL_ANALYTIC) ||
        tau != tau)
        return HF_ERR_ARG;
    hf_status s = check_box(box);
    if (s != HF_OK) return s;
    size_t need = 0;
    s = hf_find_halos_scales_ws_size(box, np, count, &need);
    if (s != HF_OK) return s;
    s = check_ws(ws, ws_bytes, need);
    if (s != HF_OK) return s;
    double kws[HF_CWT_BATCH_MAX];
    float *cwts[HF_CWT_BATCH_MAX];
    for (int j = 0; j < count; ++j) {
        const hf_scale_job &sj = scales[j];
        if (!sj.cwt || !sj.d_count || !sj.cell_label || sj.max_cap < 0 || (sj.max_cap > 0 && !sj.max_idx) ||
            (np > 0 && !sj.particle_label) || !(sj.kw > 0.0))
            return HF_ERR_ARG;
        kws[j] = sj.kw;
        cwts[j] = sj.cwt;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    const bool order = particle_order_supported(*box, np);
    char *sw = static_cast<char *>(ws);
    size_t sb = ws_bytes;
    ParticleOrder po{};
    if (order) {
        po = particle_order_at(*box, ws, np);
        sw += particle_order_bytes(*box, np);
        sb -= particle_order_bytes(*box, np);
        s = deposit_tiled(ctx, *box, pos, dtype, np, rho, sw, &po);
    } else {
        s = hf_deposit(ctx, box, pos, dtype, np, rho, sw, sb);
    }
    if (s != HF_OK) return s;
    s = hf_cwt_scales(ctx, box, rho, count, kws, kernel, cwts, sw, sb);
    for (int j = 0; j < count && s == HF_OK; ++j) {
        const hf_scale_job &sj = scales[j];
        s = maxima_segment(ctx, *box, sj.cwt, tau, sj.max_idx, sj.max_cap, sj.d_count, sj.cell_label, sw, sb);
        if (s != HF_OK) break;
        s = order ? label_from_order(ctx, *box, np, po, sj.cell_label, sj.particle_label, sw)
                  : hf_label(ctx, box, pos, dtype, np, sj.cell_label, sj.particle_label);
    }
    return s;
}

// Workspace of hf_identify: that of hf_find_halos_scales, then the group
// counters, one pass flag per maximum of the largest list and, where the
// deposit keeps its particle order, the claim state in that order.
namespace {
struct IdentifyLayout {
    size_t base, groups, pass, claim, total;
};

hf_status identify_layout(const hf_box *box, int64_t np, int32_t count, const hf_scale_job *scales,
                          IdentifyLayout &L) {
    if (!scales) return HF_ERR_ARG;
    hf_status s = hf_find_halos_scales_ws_size(box, np, count, &L.base);
    if (s != HF_OK) return s;
    int64_t cap = 0;
    for (int j = 0; j < count; ++j) {
        if (scales[j].max_cap < 0) return HF_ERR_ARG;
        cap = scales[j].max_cap > cap ? scales[j].max_cap : cap;
    }
    L.groups = align_up(L.base);
    L.pass = L.groups + groups_ws_bytes(*box);
    L.claim = L.pass + align_up(size_t(cap));
    const bool order = particle_order_supported(*box, np);
    L.total = L.claim + (order ? align_up(size_t(np)) : 0);  // one claim byte per particle, tile order
    return HF_OK;
}
}  // namespace

extern "C" hf_status hf_identify_ws_size(const hf_box *box, int64_t np, int32_t count, const hf_scale_job *scales,
                                        size_t *bytes) {
    if (!bytes) return HF_ERR_ARG;
    IdentifyLayout L{};
    hf_status s = identify_layout(box, np, count, scales, L);
    if (s == HF_OK) *bytes = L.total;
    return s;
}

// Sec. 2's identification loop at one grid: one deposit and one forward
// transform, every scale's field, maxima and segmentation, then scale by scale
// (largest first) the flowchart's pair of grids: the cross-scale flags of this
// scale's maxima against the next scale's field (the zero grid after the last),
// the groups' statistics over the particles not yet claimed, the step-7/8
// decision, and the filter of the labels with the claims of the kept groups'
// particles.  Where the deposit keeps its particle order, labels and counts
// run in that (tile) order, whose neighbouring particles share groups, and
// the filter and the claims ride on the two passes that bring each scale's
// labels back to input order (the claim state is kept in tile order for the
// counts; the first scale writes the claim arrays outright).
extern "C" hf_status hf_identify(hf_ctx *ctx, const hf_box *box, const void *pos, hf_dtype dtype, int64_t np,
                                 hf_kernel kernel, float tau, int64_t *rho, int32_t count, const hf_scale_job *scales,
                                 const hf_identify_groups *groups, double dens_th, int64_t particle_th,
                                 int32_t *halo_scale, int32_t *halo_root, void *ws, size_t ws_bytes) {
    if (!ctx || !rho || !scales || !groups || count < 1 || count > HF_CWT_BATCH_MAX) return HF_ERR_ARG;
    if (np < 0 || np > int64_t(UINT32_MAX) || (np > 0 && (!pos || !halo_scale || !halo_root))) return HF_ERR_ARG;
    if ((dtype != HF_F32 && dtype != HF_F64) || (kernel != HF_KERNEL_SAMPLED && kernel != HF_KERNEL_ANALYTIC) ||
        tau != tau)
        return HF_ERR_ARG;
    if (!(dens_th >= 0.0) || !(dens_th < 1e300) || particle_th < 0) return HF_ERR_ARG;
    double kws[HF_CWT_BATCH_MAX];
    float *cwts[HF_CWT_BATCH_MAX];
    for (int j = 0; j < count; ++j) {
        const hf_scale_job &sj = scales[j];
        if (j > 0 && !(sj.kw > scales[j - 1].kw)) return HF_ERR_ARG;  // largest scale first
        if (!sj.cwt || !sj.d_count || !sj.cell_label || sj.max_cap < 0 || (sj.max_cap > 0 && !sj.max_idx) ||
            (np > 0 && !sj.particle_label) || !(sj.kw > 0.0))
            return HF_ERR_ARG;
        if (sj.max_cap > 0 && (!groups[j].group_particles || !groups[j].group_cells || !groups[j].group_keep))
            return HF_ERR_ARG;
        kws[j] = sj.kw;
        cwts[j] = sj.cwt;
    }
    hf_status s = check_box(box);
    if (s != HF_OK) return s;
    IdentifyLayout L{};
    s = identify_layout(box, np, count, scales, L);
    if (s != HF_OK) return s;
    s = check_ws(ws, ws_bytes, L.total);
    if (s != HF_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    const bool order = particle_order_supported(*box, np);
    char *w0 = static_cast<char *>(ws);
    char *sw = w0;
    size_t sb = L.base;
    ParticleOrder po{};
    if (order) {
        po = particle_order_at(*box, ws, np);
        sw += particle_order_bytes(*box, np);
        sb -= particle_order_bytes(*box, np);
        s = deposit_tiled(ctx, *box, pos, dtype, np, rho, sw, &po);
    } else {
        s = hf_deposit(ctx, box, pos, dtype, np, rho, sw, sb);
    }
    if (s == HF_OK) s = hf_cwt_scales(ctx, box, rho, count, kws, kernel, cwts, sw, sb);
    for (int j = 0; j < count && s == HF_OK; ++j) {
        const hf_scale_job &sj = scales[j];
        s = maxima_segment(ctx, *box, sj.cwt, tau, sj.max_idx, sj.max_cap, sj.d_count, sj.cell_label, sw, sb);
    }
    if (s != HF_OK) return s;
    const GroupCounters g = group_counters_at(*box, w0 + L.groups);
    uint8_t *pass = reinterpret_cast<uint8_t *>(w0 + L.pass);
    // whether a particle is claimed: in tile order one byte per particle (the
    // masks of the counts and the claims there), else halo_scale itself
    uint8_t *cs8 = order ? reinterpret_cast<uint8_t *>(w0 + L.claim) : nullptr;
    int32_t *lab2 = reinterpret_cast<int32_t *>(sw);  // tile-order labels (label scratch)
    // in tile order the first scale writes both claim arrays outright (nothing
    // is claimed before it), so neither is cleared first
    if (!order) s = claim_init(ctx, halo_scale, halo_root, np);
    for (int j = 0; j < count && s == HF_OK; ++j) {
        const hf_scale_job &sj = scales[j];
        const hf_identify_groups &gj = groups[j];
        const float *next = j + 1 < count ? scales[j + 1].cwt : nullptr;
        int32_t *lab = order ? lab2 : sj.particle_label;
        s = cross_scale_dev(ctx, *box, sj.max_idx, sj.d_count, sj.max_cap, sj.cwt, box->n, next, pass);
        if (s == HF_OK)
            s = order ? label_tiles(ctx, *box, np, po, sj.cell_label, sw, nullptr)
                      : hf_label(ctx, box, pos, dtype, np, sj.cell_label, sj.particle_label);
        if (s == HF_OK) s = groups_count_cells(ctx, *box, sj.max_idx, sj.d_count, sj.max_cap, sj.cell_label, g);
        // particles already claimed are not counted
        if (s == HF_OK && sj.max_cap > 0)
            s = order ? groups_count_particles_tiled(ctx, *box, lab, j > 0 ? cs8 : nullptr, np, g)
                      : groups_count_particles(ctx, *box, lab, np, g, halo_scale);
        if (s == HF_OK)
            s = groups_decide(ctx, *box, sj.max_idx, sj.d_count, sj.max_cap, g, dens_th, np, particle_th, pass,
                              gj.group_particles, gj.group_cells, gj.group_keep);
        if (s == HF_OK && !order)
            s = claim_filter(ctx, *box, lab, halo_scale, halo_root, np, g, sj.max_cap > 0, j);
        if (s == HF_OK && order) {
            // the filter and the claims ride on the two passes back to input order
            const TileClaim tc{cs8, j == 0 ? 1 : 0, sj.max_cap > 0 ? 1 : 0};
            const ClaimOut claim{halo_scale, halo_root, j, j == 0 ? 1 : 0};
            s = label_back(ctx, *box, np, po, sj.particle_label, sw, g.cells, &claim, &tc);
        }
    }
    return s;
}

// Sec. 2's identification loop on per-scale grids (step 1 and the flowchart's
// N_g): every scale deposits the particles on its own grid and takes the
// paper's truncated-stencil transform there; then, largest scale first, the
// flowchart's pair of grids as in hf_identify, in input order, with the
// cross-scale check between the two scales' grids.
namespace {
struct GridsLayout {
    size_t shared, groups, pass, total;
};

hf_status grids_layout(double box_len, int32_t frac_bits, int64_t np, int32_t count, const hf_grid_scale *scales,
                       bool with_vel, GridsLayout &L) {
    if (!scales || count < 1 || count > HF_CWT_BATCH_MAX || np < 0) return HF_ERR_ARG;
    size_t shared = 0, groups = 0;
    int64_t cap = 0;
    for (int j = 0; j < count; ++j) {
        const hf_box b{scales[j].n, frac_bits, box_len};
        hf_status s = check_box_grid(&b);
        if (s != HF_OK) return s;
        if (scales[j].max_cap < 0) return HF_ERR_ARG;
        size_t need = 0;
        s = hf_workspace_size(&b, np, HF_STAGE_DEPOSIT | HF_STAGE_STENCIL | HF_STAGE_MAXIMA | HF_STAGE_SEGMENT,
                              &need);
        if (s != HF_OK) return s;
        shared = need > shared ? need : shared;
        if (with_vel) {  // steps 9-10 reuse the stage region once every scale's stages are done
            const size_t ub = unbind_ws_bytes(b, np, scales[j].max_cap);
            shared = ub > shared ? ub : shared;
        }
        groups = groups_ws_bytes(b) > groups ? groups_ws_bytes(b) : groups;
        cap = scales[j].max_cap > cap ? scales[j].max_cap : cap;
    }
    L.shared = 0;
    L.groups = align_up(shared);
    L.pass = L.groups + align_up(groups);
    L.total = L.pass + align_up(size_t(cap));
    return HF_OK;
}
}  // namespace

extern "C" hf_status hf_identify_grids_ws_size(double box_len, int32_t frac_bits, int64_t np, int32_t count,
                                              const hf_grid_scale *scales, int32_t with_velocities, size_t *bytes) {
    if (!bytes) return HF_ERR_ARG;
    GridsLayout L{};
    hf_status s = grids_layout(box_len, frac_bits, np, count, scales, with_velocities != 0, L);
    if (s == HF_OK) *bytes = L.total;
    return s;
}

extern "C" hf_status hf_identify_grids(hf_ctx *ctx, double box_len, int32_t frac_bits, const void *pos,
                                       const void *vel, hf_dtype dtype, int64_t np, float tau, int32_t count,
                                       const hf_grid_scale *scales, double dens_th, int64_t particle_th,
                                       double grav_mass, int32_t *halo_scale, int32_t *halo_root, void *ws,
                                       size_t ws_bytes) {
    if (!ctx || !scales || count < 1 || count > HF_CWT_BATCH_MAX) return HF_ERR_ARG;
    if (np < 0 || np > int64_t(INT32_MAX) || (np > 0 && (!pos || !halo_scale || !halo_root))) return HF_ERR_ARG;
    if ((dtype != HF_F32 && dtype != HF_F64) || tau != tau) return HF_ERR_ARG;
    if (!(dens_th >= 0.0) || !(dens_th < 1e300) || particle_th < 0) return HF_ERR_ARG;
    const bool with_vel = vel != nullptr;
    if (with_vel && (!(grav_mass > 0.0) || !(grav_mass < 1e300))) return HF_ERR_ARG;
    GridsLayout L{};
    hf_status s = grids_layout(box_len, frac_bits, np, count, scales, with_vel, L);
    if (s != HF_OK) return s;
    int32_t hw[HF_CWT_BATCH_MAX];
    for (int j = 0; j < count; ++j) {
        const hf_grid_scale &sj = scales[j];
        if (j > 0 && !(sj.kw > scales[j - 1].kw)) return HF_ERR_ARG;  // largest scale first
        if (!sj.rho || !sj.cwt || !sj.d_count || !sj.cell_label || (sj.max_cap > 0 && !sj.max_idx) ||
            (np > 0 && !sj.particle_label) || !(sj.kw > 0.0) || !(sj.kw < 1e300))
            return HF_ERR_ARG;
        if (sj.max_cap > int64_t(sj.n) * sj.n * sj.n) return HF_ERR_ARG;
        if (sj.max_cap > 0 && (!sj.group_particles || !sj.group_cells || !sj.group_keep)) return HF_ERR_ARG;
        if (with_vel && sj.max_cap > 0 && !sj.bound_keep) return HF_ERR_ARG;
        hw[j] = stencil_half_width(sj.kw, sj.n);
        if (hw[j] < 0) return HF_ERR_ARG;
    }
    s = check_ws(ws, ws_bytes, L.total);
    if (s != HF_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    char *w0 = static_cast<char *>(ws);
    const size_t sb = L.groups;  // the shared stage region
    // steps 2-5 of every scale on its own grid
    for (int j = 0; j < count && s == HF_OK; ++j) {
        const hf_grid_scale &sj = scales[j];
        const hf_box b{sj.n, frac_bits, box_len};
        s = hf_deposit(ctx, &b, pos, dtype, np, sj.rho, w0, sb);
        if (s == HF_OK) s = hf_cwt_stencil(ctx, &b, sj.rho, sj.kw, hw[j], sj.cwt, w0, sb);
        if (s == HF_OK)
            s = maxima_segment(ctx, b, sj.cwt, tau, sj.max_idx, sj.max_cap, sj.d_count, sj.cell_label, w0, sb);
    }
    if (s != HF_OK) return s;
    uint8_t *pass = reinterpret_cast<uint8_t *>(w0 + L.pass);
    s = claim_init(ctx, halo_scale, halo_root, np);
    for (int j = 0; j < count && s == HF_OK; ++j) {
        const hf_grid_scale &sj = scales[j];
        const hf_box b{sj.n, frac_bits, box_len};
        const GroupCounters g = group_counters_at(b, w0 + L.groups);
        const bool last = j + 1 == count;
        s = cross_scale_dev(ctx, b, sj.max_idx, sj.d_count, sj.max_cap, sj.cwt, last ? sj.n : scales[j + 1].n,
                            last ? nullptr : scales[j + 1].cwt, pass);
        if (s == HF_OK) s = hf_label(ctx, &b, pos, dtype, np, sj.cell_label, sj.particle_label);
        if (s == HF_OK) s = groups_count_cells(ctx, b, sj.max_idx, sj.d_count, sj.max_cap, sj.cell_label, g);
        if (s == HF_OK && sj.max_cap > 0) s = groups_count_particles(ctx, b, sj.particle_label, np, g, halo_scale);
        if (s == HF_OK)
            s = groups_decide(ctx, b, sj.max_idx, sj.d_count, sj.max_cap, g, dens_th, np, particle_th, pass,
                              sj.group_particles, sj.group_cells, sj.group_keep);
        if (s == HF_OK) s = claim_filter(ctx, b, sj.particle_label, halo_scale, halo_root, np, g, sj.max_cap > 0, j);
        // steps 9-10: the kept groups' self-boundness check; the particles it
        // removes (all of a discarded group's) are free again for later scales
        if (s == HF_OK && with_vel && sj.max_cap > 0) {
            s = unbind_dev(ctx, b, pos, vel, dtype, np, sj.max_idx, sj.max_cap, sj.group_keep, sj.particle_label,
                           grav_mass, particle_th, sj.bound_keep, w0, sj.d_count);
            if (s == HF_OK) s = unclaim(ctx, sj.particle_label, np, j, halo_scale, halo_root);
        }
    }
    return s;
}

// A group of same-n boxes: per-box deposits, one batched transform for all of
// them, then per-box maxima, segmentation and labels, in that order on the
// context's stream.
extern "C" hf_status hf_find_halos_group(hf_ctx *ctx, int32_t n, int32_t frac_bits, int32_t count,
                                         const hf_group_item *items, hf_kernel kernel, void *cwt_ws,
                                         size_t cwt_ws_bytes) {
    if (!ctx || !items || count < 1 || count > HF_CWT_BATCH_MAX) return HF_ERR_ARG;
    if (kernel != HF_KERNEL_SAMPLED && kernel != HF_KERNEL_ANALYTIC) return HF_ERR_ARG;
    hf_cwt_item cw[HF_CWT_BATCH_MAX];
    for (int j = 0; j < count; ++j) {
        const hf_job &job = items[j].job;
        const hf_box box{n, frac_bits, items[j].box_len};
        hf_status s = check_box(&box);
        if (s != HF_OK) return s;
        size_t need = 0;
        s = hf_workspace_size(&box, job.np, HF_STAGE_DEPOSIT | HF_STAGE_MAXIMA | HF_STAGE_SEGMENT, &need);
        if (s != HF_OK) return s;
        s = check_ws(items[j].ws, items[j].ws_bytes, need);
        if (s != HF_OK) return s;
        if (!job.rho || !job.cwt || !job.d_count || !job.cell_label || job.np < 0 || job.max_cap < 0 ||
            (job.max_cap > 0 && !job.max_idx) || (job.np > 0 && (!job.pos || !job.particle_label)) ||
            (job.dtype != HF_F32 && job.dtype != HF_F64) || job.kernel != kernel || !(job.kw > 0.0) ||
            job.tau != job.tau)
            return HF_ERR_ARG;
        cw[j] = hf_cwt_item{job.rho, job.cwt, items[j].box_len, job.kw};
    }
    size_t need = 0;
    hf_status s = hf_cwt_batch_ws_size(n, count, &need);
    if (s != HF_OK) return s;
    s = check_ws(cwt_ws, cwt_ws_bytes, need);
    if (s != HF_OK) return s;
    for (int j = 0; j < count; ++j) {
        const hf_job &job = items[j].job;
        const hf_box box{n, frac_bits, items[j].box_len};
        s = hf_deposit(ctx, &box, job.pos, job.dtype, job.np, job.rho, items[j].ws, items[j].ws_bytes);
        if (s != HF_OK) return s;
    }
    s = hf_cwt_batch(ctx, n, count, cw, kernel, cwt_ws, cwt_ws_bytes);
    if (s != HF_OK) return s;
    for (int j = 0; j < count; ++j) {
        const hf_job &job = items[j].job;
        const hf_box box{n, frac_bits, items[j].box_len};
        s = maxima_segment(ctx, box, job.cwt, job.tau, job.max_idx, job.max_cap, job.d_count, job.cell_label,
                           items[j].ws, items[j].ws_bytes);
        if (s != HF_OK) return s;
        s = hf_label(ctx, &box, job.pos, job.dtype, job.np, job.cell_label, job.particle_label);
        if (s != HF_OK) return s;
    }
    return HF_OK;
}
