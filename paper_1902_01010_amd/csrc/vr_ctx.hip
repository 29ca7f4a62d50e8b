// vr_ctx.hip -- context, workspace pool, errors and argument checks.
#include "vr_internal.h"

#include <algorithm>
#include <cstring>

namespace {
thread_local std::string g_create_err;
}

namespace vr {

static void timers_drain(vr_ctx* ctx);

int set_err(vr_ctx* ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf; else g_create_err = buf;
    return code;
}

void* ws(vr_ctx* ctx, int slot, size_t bytes) {
    if ((int)ctx->slots.size() < WS_NSLOTS) ctx->slots.resize(WS_NSLOTS);
    vr_buf& b = ctx->slots[slot];
    if (b.bytes >= bytes && b.ptr) return b.ptr;
    size_t want = bytes + bytes / 4 + 4096;
    size_t newheld = ctx->held - b.bytes + want;
    if (ctx->max_ws && newheld > ctx->max_ws) {
        want = bytes;
        newheld = ctx->held - b.bytes + want;
        if (newheld > ctx->max_ws) {
            set_err(ctx, VR_ERR_OUT_OF_MEMORY, "workspace cap of %zu bytes exceeded (%zu requested)",
                    ctx->max_ws, newheld);
            return nullptr;
        }
    }
    if (b.ptr) {
        (void)hipFree(b.ptr);
        ctx->held -= b.bytes;
        b.ptr = nullptr;
        b.bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        set_err(ctx, VR_ERR_OUT_OF_MEMORY, "hipMalloc of %zu workspace bytes failed", want);
        return nullptr;
    }
    b.ptr = p;
    b.bytes = want;
    ctx->held += want;
    return p;
}

hipEvent_t timer_event(vr_ctx* ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void timer_push(vr_ctx* ctx, const char* name, hipEvent_t e0, hipEvent_t e1, double work) {
    for (auto& t : ctx->timers)
        if (t.name == name) {
            t.pending.push_back(e0);
            t.pending.push_back(e1);
            t.pending_work.push_back(work);
            return;
        }
    vr_timer t;
    t.name = name;
    t.pending = {e0, e1};
    t.pending_work = {work};
    ctx->timers.push_back(t);
}

static void timers_drain(vr_ctx* ctx) {
    for (auto& t : ctx->timers) {
        for (size_t k = 0; k + 1 < t.pending.size(); k += 2) {
            float ms = 0.f;
            (void)hipEventSynchronize(t.pending[k + 1]);
            (void)hipEventElapsedTime(&ms, t.pending[k], t.pending[k + 1]);
            t.ms += ms;
            t.launches += 1;
            t.work += t.pending_work[k / 2];
            ctx->event_pool.push_back(t.pending[k]);
            ctx->event_pool.push_back(t.pending[k + 1]);
        }
        t.pending.clear();
        t.pending_work.clear();
    }
}

int check_particles(vr_ctx* ctx, const vr_particles* p, bool need_vel) {
    if (!p) return set_err(ctx, VR_ERR_INVALID_ARG, "particles is NULL");
    if (p->n < 0 || p->n >= (int64_t(1) << 31))
        return set_err(ctx, VR_ERR_INVALID_ARG, "n = %lld out of range [0, 2^31)", (long long)p->n);
    if (p->grid_bits < 1 || p->grid_bits > 21)
        return set_err(ctx, VR_ERR_INVALID_ARG, "grid_bits = %d not in 1..21", p->grid_bits);
    if (!(p->box > 0)) return set_err(ctx, VR_ERR_INVALID_ARG, "box must be positive");
    if (p->n > 0 && (!p->qx || !p->qy || !p->qz))
        return set_err(ctx, VR_ERR_INVALID_ARG, "NULL coordinate array");
    if (need_vel && p->n > 0 && (!p->vx || !p->vy || !p->vz))
        return set_err(ctx, VR_ERR_INVALID_ARG, "NULL velocity array");
    if (!p->mass && !(p->mass_value > 0))
        return set_err(ctx, VR_ERR_INVALID_ARG, "uniform mass_value must be positive");
    return VR_OK;
}

int check_hosts(vr_ctx* ctx, int32_t n_hosts, const int32_t* off, const int32_t* mem) {
    if (n_hosts < 0) return set_err(ctx, VR_ERR_INVALID_ARG, "n_hosts < 0");
    if (n_hosts > 0 && (!off || !mem)) return set_err(ctx, VR_ERR_INVALID_ARG, "NULL host arrays");
    return VR_OK;
}

int copy_to_host(vr_ctx* ctx, void* host, const void* dev, size_t bytes, hipStream_t s) {
    if (bytes == 0) return VR_OK;
    if (ctx->stage_bytes < bytes) {
        if (ctx->stage) VR_HIP(ctx, hipHostFree(ctx->stage));
        ctx->stage = nullptr;
        ctx->stage_bytes = 0;
        const size_t want = bytes + bytes / 4;
        VR_HIP(ctx, hipHostMalloc(&ctx->stage, want, hipHostMallocDefault));
        ctx->stage_bytes = want;
    }
    VR_HIP(ctx, hipMemcpyAsync(ctx->stage, dev, bytes, hipMemcpyDeviceToHost, s));
    VR_HIP(ctx, hipStreamSynchronize(s));
    std::memcpy(host, ctx->stage, bytes);
    return VR_OK;
}

void* upload_begin(vr_ctx* ctx, size_t bytes) {
    if (ctx->up_pending) {
        const hipError_t e = hipEventSynchronize(ctx->up_event);
        if (e != hipSuccess) {
            set_err(ctx, VR_ERR_HIP, "hipEventSynchronize: %s", hipGetErrorString(e));
            return nullptr;
        }
        ctx->up_pending = false;
    }
    if (ctx->up_bytes < bytes) {
        if (ctx->up) {
            const hipError_t e = hipHostFree(ctx->up);
            if (e != hipSuccess) {
                set_err(ctx, VR_ERR_HIP, "hipHostFree: %s", hipGetErrorString(e));
                return nullptr;
            }
        }
        ctx->up = nullptr;
        ctx->up_bytes = 0;
        const size_t want = std::max<size_t>(bytes + bytes / 4, 65536);
        const hipError_t e = hipHostMalloc(&ctx->up, want, hipHostMallocDefault);
        if (e != hipSuccess) {
            ctx->up = nullptr;
            set_err(ctx, VR_ERR_HIP, "hipHostMalloc: %s", hipGetErrorString(e));
            return nullptr;
        }
        ctx->up_bytes = want;
    }
    return ctx->up;
}

int upload_end(vr_ctx* ctx, hipStream_t s) {
    if (!ctx->up_event) VR_HIP(ctx, hipEventCreateWithFlags(&ctx->up_event, hipEventDisableTiming));
    VR_HIP(ctx, hipEventRecord(ctx->up_event, s));
    ctx->up_pending = true;
    return VR_OK;
}

int read_back(vr_ctx* ctx, const void* dev, void* host, size_t bytes, hipStream_t s) {
    return copy_to_host(ctx, host, dev, bytes, s);
}

}  // namespace vr

extern "C" {

int vr_create(vr_ctx** out, int device, size_t max_workspace_bytes) {
    if (!out) return vr::set_err(nullptr, VR_ERR_INVALID_ARG, "ctx pointer is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return vr::set_err(nullptr, VR_ERR_NO_DEVICE, "no HIP device visible");
    }
    if (device < 0 || device >= count)
        return vr::set_err(nullptr, VR_ERR_NO_DEVICE, "device %d not in [0, %d)", device, count);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return vr::set_err(nullptr, VR_ERR_NO_DEVICE, "cannot query device %d", device);
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return vr::set_err(nullptr, VR_ERR_UNSUPPORTED, "device %d is %s, libvr is built for gfx950",
                           device, prop.gcnArchName);
    if (hipSetDevice(device) != hipSuccess)
        return vr::set_err(nullptr, VR_ERR_HIP, "hipSetDevice(%d) failed", device);
    if (int rc = vr::noalloc_scratch_init(device)) return rc;
    vr_ctx* c = new vr_ctx();
    c->device = device;
    c->num_cus = prop.multiProcessorCount;
    c->max_ws = max_workspace_bytes;
    if (hipHostMalloc((void**)&c->pinned, 64 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return vr::set_err(nullptr, VR_ERR_HIP, "hipHostMalloc failed");
    }
    if (hipHostMalloc(&c->stage, 65536, hipHostMallocDefault) != hipSuccess) {
        (void)hipHostFree(c->pinned);
        delete c;
        return vr::set_err(nullptr, VR_ERR_HIP, "hipHostMalloc failed");
    }
    c->stage_bytes = 65536;
    c->slots.resize(vr::WS_NSLOTS);
    *out = c;
    return VR_OK;
}

void vr_destroy(vr_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    vr::timers_drain(ctx);
    vr::unbind_release(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy((hipStream_t)ctx->cap_stream);
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    for (auto& b : ctx->slots)
        if (b.ptr) (void)hipFree(b.ptr);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    if (ctx->up) (void)hipHostFree(ctx->up);
    if (ctx->up_event) (void)hipEventDestroy(ctx->up_event);
    if (ctx->knn_cand) (void)hipFree(ctx->knn_cand);
    delete ctx;
}

const char* vr_last_error(const vr_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int vr_sync(vr_ctx* ctx, void* stream) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    VR_HIP(ctx, hipSetDevice(ctx->device));
    VR_HIP(ctx, hipStreamSynchronize((hipStream_t)stream));
    VR_HIP(ctx, hipGetLastError());
    return VR_OK;
}

size_t vr_workspace_bytes(const vr_ctx* ctx) { return ctx ? ctx->held : 0; }

int vr_new_snapshot(vr_ctx* ctx) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    ctx->kd_pre_m = -1;  // the next KD build sorts its members afresh
    return VR_OK;
}

int vr_set_timing(vr_ctx* ctx, int enabled) {
    if (!ctx) return VR_ERR_INVALID_ARG;
    VR_HIP(ctx, hipSetDevice(ctx->device));
    vr::timers_drain(ctx);
    ctx->timers.clear();
    ctx->timing = enabled ? 1 : 0;
    if (enabled) {
        if (!ctx->knn_cand) VR_HIP(ctx, hipMalloc((void**)&ctx->knn_cand, sizeof(unsigned long long)));
        VR_HIP(ctx, hipMemset(ctx->knn_cand, 0, sizeof(unsigned long long)));
    }
    return VR_OK;
}

int vr_tune(vr_ctx* ctx, const char* knob, int value) {
    if (!ctx || !knob) return VR_ERR_INVALID_ARG;
    const std::string k = knob;
    if (k == "knn_leaf") {
        if (value < 16 || value > 256) return vr::set_err(ctx, VR_ERR_INVALID_ARG, "knn_leaf must be in 16..256");
        ctx->knn_leaf = value;
    } else if (k == "unbind_tile") {
        if (value < 64 || value > 4096 || (value & 63))
            return vr::set_err(ctx, VR_ERR_INVALID_ARG, "unbind_tile must be a multiple of 64 in 64..4096");
        ctx->tuned_tile = value;
    } else if (k == "unbind_jchunk") {
        if (value < 256 || value > 65536) return vr::set_err(ctx, VR_ERR_INVALID_ARG, "unbind_jchunk must be in 256..65536");
        ctx->unbind_jchunk = value;
    } else if (k == "xcd_chunk") {
        if (value < 0 || value > 4096) return vr::set_err(ctx, VR_ERR_INVALID_ARG, "xcd_chunk must be in 0..4096");
        ctx->xcd_chunk = value;
    } else if (k == "unbind_bpc") {
        if (value < 0 || value > 8) return vr::set_err(ctx, VR_ERR_INVALID_ARG, "unbind_bpc must be in 0..8");
        ctx->unbind_bpc = value;
    } else if (k == "unbind_wide") {
        if (value < 256 || value > (1 << 30))
            return vr::set_err(ctx, VR_ERR_INVALID_ARG, "unbind_wide must be in 256..2^30");
        ctx->unbind_wide = value;
    } else {
        return vr::set_err(ctx, VR_ERR_INVALID_ARG, "unknown knob '%s'", knob);
    }
    return VR_OK;
}

int vr_get_tune(const vr_ctx* ctx, const char* knob, int* value) {
    if (!ctx || !knob || !value) return VR_ERR_INVALID_ARG;
    const std::string k = knob;
    if (k == "knn_leaf") *value = ctx->knn_leaf;
    else if (k == "unbind_tile") *value = ctx->tuned_tile ? ctx->tuned_tile : 256;
    else if (k == "unbind_jchunk") *value = ctx->unbind_jchunk;
    else if (k == "unbind_bpc") *value = ctx->unbind_bpc;
    else if (k == "unbind_wide") *value = ctx->unbind_wide;
    else if (k == "xcd_chunk") *value = ctx->xcd_chunk;
    else return VR_ERR_INVALID_ARG;
    return VR_OK;
}

int vr_kernel_time(vr_ctx* ctx, const char* kernel, int64_t* launches, double* total_ms, double* work) {
    if (!ctx || !kernel || !launches || !total_ms || !work) return VR_ERR_INVALID_ARG;
    VR_HIP(ctx, hipSetDevice(ctx->device));
    vr::timers_drain(ctx);
    *launches = 0;
    *total_ms = 0.0;
    *work = 0.0;
    // "knn_candidates": the kNN launches and time, with the candidate
    // distances the searches evaluated as the work
    const bool cand = std::strcmp(kernel, "knn_candidates") == 0;
    for (auto& t : ctx->timers)
        if (t.name == (cand ? "knn" : kernel)) {
            *launches = t.launches;
            *total_ms = t.ms;
            *work = t.work;
        }
    if (cand) {
        *work = 0.0;
        if (ctx->knn_cand) {
            unsigned long long c = 0;
            VR_HIP(ctx, hipMemcpy(&c, ctx->knn_cand, sizeof c, hipMemcpyDeviceToHost));
            *work = (double)c;
        }
    }
    return VR_OK;
}

}  // extern "C"
