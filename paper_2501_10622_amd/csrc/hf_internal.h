// Internal definitions shared by the HIP translation units of libhf.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "hf.h"

namespace hf {

// Kernels whose launches the optional per-context timer tracks.
enum KernelId {
    K_ZERO_GRID, K_DEPOSIT, K_LABEL,
    K_DEP_ATOMIC, K_DEP_PREP, K_DEP_L1_HIST, K_DEP_L1_SCATTER, K_DEP_L2_HIST, K_DEP_L2_SCATTER, K_DEP_FOLD,
    K_TABLES_1, K_TABLES_2, K_X_FWD, K_MASS, K_Y_FWD, K_Z_MUL, K_Y_INV, K_X_INV,
    K_MAX_MARK, K_MAX_COUNT, K_MAX_SCAN, K_MAX_WRITE,
    K_PARENT, K_FLAGS, K_JUMP, K_FINALIZE,
    K_COUNT
};
const char *kernel_name(int id);

struct ProfRecord {
    int kid;
    hipEvent_t start, stop;
};

}  // namespace hf

struct hf_ctx {
    int device;
    hipStream_t stream;
    uint32_t *d_status;  // device status block: [0] error bit mask
    uint32_t *h_status;  // pinned host mirror
    // kernel timer (off unless hf_profile_enable): events around every launch
    bool prof = false;
    std::vector<hf::ProfRecord> pending;
    std::vector<hipEvent_t> pool;
    double ms[hf::K_COUNT] = {};
    int64_t launches[hf::K_COUNT] = {};
};

namespace hf {

hipEvent_t take_event(hf_ctx *c);

// Brackets the launches issued in its scope with timing events when the
// context's timer is on.
struct ProfScope {
    hf_ctx *c;
    int kid;
    hipEvent_t start = nullptr;
    ProfScope(hf_ctx *ctx, int id) : c(ctx), kid(id) {
        if (c->prof) {
            start = take_event(c);
            if (start) (void)hipEventRecord(start, c->stream);
        }
    }
    ~ProfScope() {
        if (c->prof && start) {
            hipEvent_t stop = take_event(c);
            if (stop) {
                (void)hipEventRecord(stop, c->stream);
                c->pending.push_back({kid, start, stop});
            }
        }
    }
};

// Launches a kernel on ctx->stream under the context's kernel timer.
#define HF_LAUNCH(ctx, kid, ...)                 \
    do {                                         \
        ::hf::ProfScope hf_prof_scope_(ctx, kid); \
        hipLaunchKernelGGL(__VA_ARGS__);         \
    } while (0)

// Device status bits (one per device-detected hf_status code).
constexpr uint32_t ST_OVERFLOW = 1u << HF_ERR_OVERFLOW;
constexpr uint32_t ST_CAPACITY = 1u << HF_ERR_CAPACITY;
constexpr uint32_t ST_INPUT = 1u << HF_ERR_INPUT;

constexpr size_t WS_ALIGN = 256;

inline size_t align_up(size_t x, size_t a = WS_ALIGN) { return (x + a - 1) / a * a; }

// n = 2^a 3^b, a >= 1, 8 <= n <= 1024.
inline bool supported_n(int n) {
    if (n < 8 || n > 1024 || (n & 1)) return false;
    int m = n;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    return m == 1;
}

inline hf_status check_box(const hf_box *box) {
    if (!box) return HF_ERR_ARG;
    if (!supported_n(box->n)) return HF_ERR_SIZE;
    if (box->frac_bits < 8 || box->frac_bits > 20) return HF_ERR_SIZE;
    if (!(box->box_len > 0.0) || !(box->box_len < 1e300)) return HF_ERR_ARG;
    return HF_OK;
}

inline hf_status check_ws(void *ws, size_t ws_bytes, size_t need) {
    if (need == 0) return HF_OK;
    if (!ws || ws_bytes < need) return HF_ERR_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % WS_ALIGN) return HF_ERR_WORKSPACE;
    return HF_OK;
}

inline hf_status launch_status() {
    return hipGetLastError() == hipSuccess ? HF_OK : HF_ERR_DEVICE;
}

// Binned deposit (n % 16 == 0, B <= 17, np < 2^32).
bool deposit_tiled_supported(const hf_box &box, int64_t np);
size_t deposit_tiled_ws_bytes(const hf_box &box, int64_t np);
hf_status deposit_tiled(hf_ctx *ctx, const hf_box &box, const void *pos, hf_dtype dtype, int64_t np, int64_t *rho,
                        void *ws);

// Workspace requirements of each stage (defined next to each stage).
size_t deposit_ws_bytes(const hf_box &box, int64_t np);
size_t cwt_ws_bytes(const hf_box &box);
size_t maxima_ws_bytes(const hf_box &box);
size_t segment_ws_bytes(const hf_box &box);

// ---------------------------------------------------------------------------
// Fixed-point particle coordinates, shared by the deposit and the labels so
// both stages see exactly the same q for a particle.
// ---------------------------------------------------------------------------
template <typename T>
struct FixedPoint {
    T scale;        // n 2^B / L rounded to T
    int64_t period; // n 2^B
    int bits;

    // Returns false for a position the deposit rejects (non-finite t or |t| >= 2^62).
    __device__ __forceinline__ bool q(T x, int64_t &out) const {
        T t = x * scale;  // single correctly rounded multiply in T
        if (!(t > T(-4.611686018427388e18) && t < T(4.611686018427388e18))) return false;
        int64_t fl = static_cast<int64_t>(floor(t));
        if (fl < 0 || fl >= period) {
            fl %= period;
            if (fl < 0) fl += period;
        }
        out = fl;
        return true;
    }
};

}  // namespace hf
