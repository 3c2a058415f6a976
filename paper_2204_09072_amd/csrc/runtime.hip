// Context lifecycle, errors and synchronisation.
#include <mutex>

#include "common.hpp"

namespace {

// Scratch of the allocation-free dust solve (tr_dust_equilibrium_noalloc): the guess
// network's starting temperature of every state, TR_NOALLOC_DUST_STATES floats (16 MiB).
// Each GPU the library runs on holds its own copy until the process ends.  Host code never
// uses this name as an address: the per-device address comes from hipGetSymbolAddress.
static __device__ __align__(256) float scratch[TR_NOALLOC_DUST_STATES];

std::mutex g_scratch_mu;
std::map<int, float *> g_scratch; // device -> address of that device's scratch

// the calling thread's current device is `device`
int lookup_scratch(int device, float **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch.find(device);
    if (it == g_scratch.end()) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TR_EHIP;
        it = g_scratch.emplace(device, static_cast<float *>(ptr)).first;
    }
    *out = it->second;
    return TR_OK;
}

} // namespace

int tr_fail(tr_ctx *ctx, int code, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

extern "C" int tr_ctx_create(tr_ctx **out, int device, void *stream) {
    if (!out) return TR_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return TR_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return TR_EHIP;
    tr_ctx *c = new tr_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete c; return TR_EHIP; }
    c->n_cu = prop.multiProcessorCount;
    // once per device, with the device current: the address of its allocation-free scratch
    if (lookup_scratch(device, &c->noalloc_guess) != TR_OK) { delete c; return TR_EHIP; }
    if (hipMalloc(&c->d_ctl, 64 * sizeof(int)) != hipSuccess) { delete c; return TR_ENOMEM; }
    if (hipMemset(c->d_ctl, 0, 64 * sizeof(int)) != hipSuccess) { hipFree(c->d_ctl); delete c; return TR_EHIP; }
    if (hipHostMalloc(&c->h_err, sizeof(int)) != hipSuccess) { hipFree(c->d_ctl); delete c; return TR_ENOMEM; }
    *out = c;
    return TR_OK;
}

extern "C" void tr_ctx_destroy(tr_ctx *c) {
    if (!c) return;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    for (auto &kv : c->tables) {
        hipFree(kv.second.table);
        hipFree(kv.second.dirs);
        hipFree(kv.second.alpha);
        hipFree(kv.second.near);
    }
    hipFree(c->d_ctl);
    hipFree(c->ws_guess);
    hipFree(c->ws_thick);
    hipHostFree(c->h_err);
    delete c;
}

extern "C" int tr_ctx_set_stream(tr_ctx *c, void *stream) {
    if (!c) return TR_EINVAL;
    c->stream = (hipStream_t)stream;
    return TR_OK;
}

extern "C" int tr_ctx_set_validation(tr_ctx *c, int on) {
    if (!c) return TR_EINVAL;
    c->validate = on ? 1 : 0;
    return TR_OK;
}

extern "C" const char *tr_last_error(const tr_ctx *c) { return c ? c->err.c_str() : "null context"; }

extern "C" int tr_sync(tr_ctx *c) {
    if (!c) return TR_EINVAL;
    TR_HIP(c, hipSetDevice(c->device));
    TR_HIP(c, hipMemcpyAsync(c->h_err, c->d_ctl + 16, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    TR_HIP(c, hipStreamSynchronize(c->stream));
    if (*c->h_err) {
        int e = *c->h_err;
        TR_HIP(c, hipMemsetAsync(c->d_ctl + 16, 0, sizeof(int), c->stream));
        TR_HIP(c, hipStreamSynchronize(c->stream));
        return tr_fail(c, TR_EOVERFLOW, "device walk stack overflow (flag %d)", e);
    }
    return TR_OK;
}
