// Context management, status reporting and workspace sizing of libhf.
#include "hf_internal.h"

#include <mutex>

using namespace hf;

namespace {

__global__ void clear_status_kernel(uint32_t *st) {
    if (threadIdx.x == 0) st[0] = 0u;
}

// The workspace of hf_find_halos_noalloc: one array per device, resident from
// the first context on that device until the process ends.  Host code never
// names it except through HIP_SYMBOL: its device address on each device comes
// from hipGetSymbolAddress (bind_scratch) and is kept in g_scratch.
__device__ __align__(256) unsigned char scratch[HF_NOALLOC_SCRATCH_BYTES];

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[SCRATCH_DEVICES] = {};

// Resolves the scratch array's address on `device`, which must be current.
// Once per device; a failure leaves it unresolved (hf_find_halos_noalloc then
// returns HF_ERR_DEVICE) and costs the other entry points nothing.
void *bind_scratch(int device) {
    if (device < 0 || device >= SCRATCH_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p) g_scratch[device] = p;
        else (void)hipGetLastError();
    }
    return g_scratch[device];
}

}  // namespace

const char *hf::kernel_name(int id) {
    static const char *names[K_COUNT] = {
        "zero_grid", "deposit", "label",
        "deposit_atomic", "deposit_prep", "deposit_l1_hist", "deposit_l1_scatter", "deposit_l2_hist",
        "deposit_l2_scatter", "deposit_fold",
        "tables_1", "tables_2", "fft_x_fwd", "mass", "fft_y_fwd", "fft_z_mul", "fft_y_inv", "fft_x_inv",
        "maxima_mark", "maxima_count", "maxima_scan", "maxima_write",
        "parent", "jump_flags", "jump", "finalize",
        "label_tiles", "label_level1", "label_input",
        "groups_clear", "groups_cells", "groups_particles", "groups_decide", "groups_filter", "cross_scale",
        "peaks", "stencil_x", "stencil_mass", "stencil_y", "stencil_z", "claim", "unbind",
    };
    return (id >= 0 && id < K_COUNT) ? names[id] : "?";
}

hipEvent_t hf::take_event(hf_ctx *c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Resolves recorded event pairs into the per-kernel totals.
static hf_status flush_profile(hf_ctx *c) {
    if (c->pending.empty()) return HF_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return HF_ERR_DEVICE;
    for (const ProfRecord &r : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
            c->ms[r.kid] += ms;
            c->launches[r.kid] += 1;
        }
        c->pool.push_back(r.start);
        c->pool.push_back(r.stop);
    }
    c->pending.clear();
    return HF_OK;
}

extern "C" hf_status hf_profile_enable(hf_ctx *ctx, int enable) {
    if (!ctx) return HF_ERR_ARG;
    ctx->prof = enable != 0;
    return HF_OK;
}

extern "C" hf_status hf_profile_reset(hf_ctx *ctx) {
    if (!ctx) return HF_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    hf_status s = flush_profile(ctx);
    for (int i = 0; i < K_COUNT; ++i) {
        ctx->ms[i] = 0.0;
        ctx->launches[i] = 0;
    }
    return s;
}

extern "C" hf_status hf_profile_read(hf_ctx *ctx, int index, const char **name, double *ms, int64_t *launches) {
    if (!ctx || !name || !ms || !launches) return HF_ERR_ARG;
    if (index < 0 || index >= K_COUNT) return HF_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    hf_status s = flush_profile(ctx);
    *name = kernel_name(index);
    *ms = ctx->ms[index];
    *launches = ctx->launches[index];
    return s;
}

extern "C" hf_status hf_create(int device, void *hip_stream, hf_ctx **out) {
    if (!out) return HF_ERR_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return HF_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return HF_ERR_DEVICE;
    hf_ctx *c = new hf_ctx{};
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->cus = cus;
    if (hipMalloc(&c->d_status, 256) != hipSuccess) {
        delete c;
        return HF_ERR_DEVICE;
    }
    if (hipHostMalloc(&c->h_status, 256, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(c->d_status);
        delete c;
        return HF_ERR_DEVICE;
    }
    c->h_status[0] = 0;
    c->scratch = bind_scratch(device);
    hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(64), 0, c->stream, c->d_status);
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipFree(c->d_status);
        (void)hipHostFree(c->h_status);
        delete c;
        return HF_ERR_DEVICE;
    }
    *out = c;
    return HF_OK;
}

extern "C" hf_status hf_destroy(hf_ctx *ctx) {
    if (!ctx) return HF_ERR_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (const ProfRecord &r : ctx->pending) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    (void)hipFree(ctx->d_status);
    (void)hipHostFree(ctx->h_status);
    delete ctx;
    return HF_OK;
}

extern "C" const char *hf_status_str(hf_status s) {
    switch (s) {
        case HF_OK: return "ok";
        case HF_ERR_ARG: return "invalid argument";
        case HF_ERR_SIZE: return "unsupported grid size or fraction bits";
        case HF_ERR_WORKSPACE: return "workspace too small or misaligned";
        case HF_ERR_OVERFLOW: return "CIC cell overflow (cell mass above 2^63-1)";
        case HF_ERR_CAPACITY: return "maxima list capacity exceeded";
        case HF_ERR_DEVICE: return "HIP runtime error";
        case HF_ERR_INPUT: return "invalid input values (non-finite position, NaN field, or empty/negative density)";
    }
    return "unknown status";
}

extern "C" hf_status hf_sync(hf_ctx *ctx) {
    if (!ctx) return HF_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return HF_ERR_DEVICE;
    if (hipMemcpyAsync(ctx->h_status, ctx->d_status, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream) !=
        hipSuccess)
        return HF_ERR_DEVICE;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return HF_ERR_DEVICE;
    uint32_t st = ctx->h_status[0];
    if (st == 0) return HF_OK;
    hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->d_status);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return HF_ERR_DEVICE;
    if (st & ST_INPUT) return HF_ERR_INPUT;
    if (st & ST_OVERFLOW) return HF_ERR_OVERFLOW;
    if (st & ST_CAPACITY) return HF_ERR_CAPACITY;
    return HF_ERR_DEVICE;
}

extern "C" hf_status hf_workspace_size(const hf_box *box, int64_t np, int stage_mask, size_t *bytes) {
    if (!bytes || np < 0) return HF_ERR_ARG;
    hf_status s = (stage_mask & HF_STAGE_CWT) ? check_box(box) : check_box_grid(box);
    if (s != HF_OK) return s;
    if (stage_mask & ~(HF_STAGE_ALL | HF_STAGE_GROUPS | HF_STAGE_STENCIL)) return HF_ERR_ARG;
    // deposit + label: the deposit's particle order is kept for the labels in
    // a region of its own in front of the part the stages share in turn
    const bool order = (stage_mask & HF_STAGE_DEPOSIT) && (stage_mask & HF_STAGE_LABEL) &&
                       particle_order_supported(*box, np);
    size_t need = 0;
    auto take = [&need](size_t b) { need = need > b ? need : b; };
    if (stage_mask & HF_STAGE_DEPOSIT) take(order ? deposit_tiled_ws_bytes(*box, np, true) : deposit_ws_bytes(*box, np));
    if (stage_mask & HF_STAGE_CWT) take(cwt_ws_bytes(*box));
    if (stage_mask & HF_STAGE_STENCIL) take(stencil_ws_bytes(*box));
    if (stage_mask & HF_STAGE_MAXIMA) take(maxima_ws_bytes(*box));
    if (stage_mask & HF_STAGE_SEGMENT) take(segment_ws_bytes(*box));
    if ((stage_mask & HF_STAGE_MAXIMA) && (stage_mask & HF_STAGE_SEGMENT)) take(maxima_segment_ws_bytes(*box));
    if (order) take(label_scratch_bytes(np));
    // the group counters live through step 6 when it runs through the kept
    // order (hf_find_halos_filtered): then they get a region of their own
    const bool groups_apart = order && (stage_mask & HF_STAGE_GROUPS);
    if ((stage_mask & HF_STAGE_GROUPS) && !groups_apart) take(groups_ws_bytes(*box));
    // hf_groups on its own (its stage alone): room for its partitioned count
    if (stage_mask == HF_STAGE_GROUPS) take(groups_ws_bytes(*box) + groups_part_ws_bytes(*box, np));
    *bytes = (order ? particle_order_bytes(*box, np) : 0) + (groups_apart ? groups_ws_bytes(*box) : 0) + need;
    return HF_OK;
}

// Steps 2-6 as hf_find_halos, with the device's scratch array as workspace.
extern "C" hf_status hf_find_halos_noalloc(hf_ctx *ctx, const hf_box *box, const hf_job *job) {
    if (!ctx || !job) return HF_ERR_ARG;
    hf_status s = check_box_for(box, job->kernel);
    if (s != HF_OK) return s;
    size_t need = 0;
    s = hf_workspace_size(box, job->np, pipeline_stages(job->kernel), &need);
    if (s != HF_OK) return s;
    if (need > HF_NOALLOC_SCRATCH_BYTES) return HF_ERR_WORKSPACE;
    if (!ctx->scratch) return HF_ERR_DEVICE;
    return hf_find_halos(ctx, box, job, ctx->scratch, HF_NOALLOC_SCRATCH_BYTES);
}
