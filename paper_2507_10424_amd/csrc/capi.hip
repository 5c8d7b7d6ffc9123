// C-ABI entry points of libldpc: argument checks, workspace sizing and the
// choice of kernel path.
#include <mutex>

#include "ldpc_internal.h"

// Device memory of ldpc_minsum_decode_noalloc: the workspace of its kernels.
// Each GPU the library runs on holds its own copy until the process ends.  In
// host code `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, once per device (scratch_on).
static __device__ __align__(256) unsigned char scratch[LDPC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {}; // device address of `scratch` per device, null until looked up

// The address of `scratch` on `device`, which must be the current device
// (looked up on the first call on that device), or null on failure.
void *scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}

int check_common(const ldpc_graph *g, const float *llr, int32_t B, int32_t L, uint8_t *bits, int32_t *iters) {
    if (!g || B < 0 || L < 0) return LDPC_EINVAL;
    if (B > 0 && (!llr || !bits || !iters)) return LDPC_EINVAL;
    return LDPC_OK;
}

// Path choice: forced by a flag, else the tuning record, else on-chip
// whenever the graph fits.
bool use_onchip(const ldpc_graph &g, uint32_t flags) {
    if (flags & LDPC_FORCE_ONCHIP) return true;
    if (flags & LDPC_FORCE_STREAM) return false;
    if (g.tuning.set && g.tuning.path == 2) return false;
    return ldpc::onchip_fits(g);
}

int decode(const ldpc_graph *g, const float *llr, int32_t B, int32_t L, uint32_t flags, const float *alpha,
           const float *beta, int32_t T, uint8_t *bits, float *post, int32_t *iters, uint8_t *ok, void *ws,
           size_t ws_bytes, hipStream_t stream) {
    int st = check_common(g, llr, B, L, bits, iters);
    if (st) return st;
    if ((flags & LDPC_FORCE_STREAM) && (flags & LDPC_FORCE_ONCHIP)) return LDPC_EINVAL;
    if (flags & ~ldpc::kKnownFlags) return LDPC_EINVAL;
    if (B == 0) return LDPC_OK;
    if (use_onchip(*g, flags)) {
        if (!ldpc::onchip_fits(*g)) return LDPC_EUNSUPPORTED;
        return ldpc::onchip_decode(*g, llr, B, L, flags, alpha, beta, T, bits, post, iters, ok, ws, ws_bytes, stream);
    }
    return ldpc::stream_decode(*g, llr, B, L, flags, alpha, beta, T, bits, post, iters, ok, ws, ws_bytes, stream);
}

} // namespace

extern "C" size_t ldpc_decode_workspace_bytes(const ldpc_graph *g, int32_t B, uint32_t flags) {
    if (!g || B <= 0) return 0;
    if (use_onchip(*g, flags)) return ldpc::onchip_workspace_bytes(*g, B);
    return ldpc::stream_workspace_bytes(*g, B);
}

extern "C" int ldpc_minsum_decode(const ldpc_graph *g, const float *llr_dev, int32_t B, int32_t max_iter,
                                  uint32_t flags, uint8_t *bits_dev, float *post_dev, int32_t *iters_dev,
                                  uint8_t *ok_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream) {
    return decode(g, llr_dev, B, max_iter, flags, nullptr, nullptr, 0, bits_dev, post_dev, iters_dev, ok_dev, ws_dev,
                  ws_bytes, stream);
}

extern "C" int ldpc_nms_decode(const ldpc_graph *g, const float *llr_dev, int32_t B, int32_t max_iter, uint32_t flags,
                               const float *alpha_dev, const float *beta_dev, int32_t T, uint8_t *bits_dev,
                               float *post_dev, int32_t *iters_dev, uint8_t *ok_dev, void *ws_dev, size_t ws_bytes,
                               hipStream_t stream) {
    if (!alpha_dev || !beta_dev || T < 1 || max_iter > T) return LDPC_EINVAL;
    return decode(g, llr_dev, B, max_iter, flags, alpha_dev, beta_dev, T, bits_dev, post_dev, iters_dev, ok_dev,
                  ws_dev, ws_bytes, stream);
}

extern "C" int ldpc_minsum_decode_noalloc(const ldpc_graph *g, const float *llr_dev, int32_t B, int32_t max_iter,
                                          uint32_t flags, uint8_t *bits_dev, float *post_dev, int32_t *iters_dev,
                                          uint8_t *ok_dev, hipStream_t stream) {
    int st = check_common(g, llr_dev, B, max_iter, bits_dev, iters_dev);
    if (st) return st;
    if ((flags & LDPC_FORCE_STREAM) && (flags & LDPC_FORCE_ONCHIP)) return LDPC_EINVAL;
    if (flags & ~ldpc::kKnownFlags) return LDPC_EINVAL;
    if (B == 0) return LDPC_OK;
    int device = -1;
    if (hipGetDevice(&device) != hipSuccess) return LDPC_EHIP;
    if (device != g->device) return LDPC_EINVAL;
    const size_t need = ldpc_decode_workspace_bytes(g, B, flags);
    if (need > LDPC_NOALLOC_SCRATCH_BYTES) return LDPC_EWORKSPACE;
    void *ws = scratch_on(device);
    if (!ws) return LDPC_EHIP;
    return decode(g, llr_dev, B, max_iter, flags, nullptr, nullptr, 0, bits_dev, post_dev, iters_dev, ok_dev, ws,
                  LDPC_NOALLOC_SCRATCH_BYTES, stream);
}

extern "C" size_t ldpc_dense_workspace_bytes(const ldpc_graph *g, int32_t B) {
    if (!g || B <= 0 || g->dense_h == nullptr) return 0;
    return ldpc::dense_workspace_bytes(*g, B);
}

extern "C" int ldpc_minsum_decode_dense(const ldpc_graph *g, const float *llr_dev, int32_t B, int32_t max_iter,
                                        uint32_t flags, uint8_t *bits_dev, float *post_dev, int32_t *iters_dev,
                                        uint8_t *ok_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream) {
    int st = check_common(g, llr_dev, B, max_iter, bits_dev, iters_dev);
    if (st) return st;
    const uint32_t allowed = LDPC_NO_EARLY_EXIT | LDPC_CHECK_PERIOD(0xff);
    if (flags & ~allowed) return LDPC_EINVAL;
    if (B == 0) return LDPC_OK;
    return ldpc::dense_decode(*g, llr_dev, B, max_iter, flags, bits_dev, post_dev, iters_dev, ok_dev, ws_dev,
                              ws_bytes, stream);
}

extern "C" size_t ldpc_multi_workspace_bytes(int32_t njobs) { return ldpc::onchip_multi_workspace_bytes(njobs); }

extern "C" int ldpc_minsum_decode_multi(const ldpc_job *jobs, int32_t njobs, int32_t max_iter, uint32_t flags,
                                        void *ws_dev, size_t ws_bytes, hipStream_t stream) {
    if (!jobs || njobs < 1 || max_iter < 0 || (flags & ~ldpc::kKnownFlags)) return LDPC_EINVAL;
    int device = -1;
    for (int32_t k = 0; k < njobs; ++k) {
        const ldpc_job &j = jobs[k];
        if (!j.g || j.B < 0 || (j.B > 0 && (!j.llr_dev || !j.bits_dev || !j.iters_dev))) return LDPC_EINVAL;
        if (device >= 0 && j.g->device != device) return LDPC_EINVAL;
        device = j.g->device;
    }
    if (njobs > LDPC_MAX_JOBS) return LDPC_EUNSUPPORTED;
    return ldpc::onchip_decode_multi(jobs, njobs, max_iter, flags, ws_dev, ws_bytes, stream);
}

extern "C" const char *ldpc_status_string(int status) {
    switch (status) {
    case LDPC_OK: return "ok";
    case LDPC_EINVAL: return "invalid argument";
    case LDPC_EBADH: return "parity matrix not 0/1, has a row of degree 1, or too many ones";
    case LDPC_ENOMEM: return "out of memory";
    case LDPC_EHIP: return "HIP call or kernel launch failed";
    case LDPC_EWORKSPACE: return "workspace missing or too small";
    case LDPC_EUNSUPPORTED: return "graph exceeds a limit of the requested kernel path";
    default: return "unknown status";
    }
}
