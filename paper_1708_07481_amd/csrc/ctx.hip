// Context, error reporting and version of the spectral-clustering library.
#include <dlfcn.h>
#include <link.h>
#include <string.h>

#include "sc_internal.h"

sc_status sc_fail(sc_ctx* ctx, sc_status st, const char* fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

extern "C" int sc_version(void) { return 10100; }

namespace {
struct HipLibScan {
    int count = 0;
    uintptr_t base[8] = {};
};

int count_hip_libs(struct dl_phdr_info* info, size_t, void* data) {
    HipLibScan* s = static_cast<HipLibScan*>(data);
    const char* name = info->dlpi_name;
    if (!name || !strstr(name, "libamdhip64")) return 0;
    // the same object can appear under two names (soname link and file):
    // count distinct load addresses
    for (int i = 0; i < s->count && i < 8; ++i)
        if (s->base[i] == static_cast<uintptr_t>(info->dlpi_addr)) return 0;
    if (s->count < 8) s->base[s->count] = static_cast<uintptr_t>(info->dlpi_addr);
    ++s->count;
    return 0;
}
}  // namespace

extern "C" sc_status sc_runtime_info(int* hip_runtime_version, int* hip_libs_mapped, char* path,
                                     size_t path_len) {
    if (hip_runtime_version) {
        int v = 0;
        if (hipRuntimeGetVersion(&v) != hipSuccess) return SC_E_HIP;
        *hip_runtime_version = v;
    }
    if (hip_libs_mapped) {
        HipLibScan s;
        dl_iterate_phdr(count_hip_libs, &s);
        *hip_libs_mapped = s.count;
    }
    if (path && path_len) {
        Dl_info di{};
        path[0] = 0;
        if (dladdr(reinterpret_cast<void*>(&hipGetDeviceCount), &di) && di.dli_fname) {
            strncpy(path, di.dli_fname, path_len - 1);
            path[path_len - 1] = 0;
        }
    }
    return SC_OK;
}

extern "C" sc_status sc_ctx_create(int device, void* hip_stream, sc_ctx** out) {
    if (!out) return SC_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SC_E_INVAL;
    int libs = 0;
    if (sc_runtime_info(nullptr, &libs, nullptr, 0) != SC_OK || libs > 1) return SC_E_HIP;
    sc_ctx* c = new sc_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return SC_E_HIP;
    }
    if (hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device) !=
            hipSuccess ||
        c->num_cu <= 0) {
        delete c;
        return SC_E_HIP;
    }
    c->stage_bytes = 1 << 16;
    if (hipHostMalloc(&c->stage, c->stage_bytes, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return SC_E_HIP;
    }
    *out = c;
    return SC_OK;
}

extern "C" sc_status sc_ctx_destroy(sc_ctx* ctx) {
    if (!ctx) return SC_E_INVAL;
    prof_drain(ctx, true);
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    delete ctx;
    return SC_OK;
}

static hipEvent_t ev_get(sc_ctx* ctx) {
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(sc_ctx* c, int k) : ctx(c), kind(k) {
    if (kind < 0 || !(ctx->prof_mask & (1u << kind))) return;
    a = ev_get(ctx);
    b = ev_get(ctx);
    if (a && b) (void)hipEventRecord(a, ctx->stream);
}

ProfScope::~ProfScope() {
    if (!a || !b) return;
    (void)hipEventRecord(b, ctx->stream);
    ctx->pending.push_back({kind, a, b});
}

void prof_drain(sc_ctx* ctx, bool sync) {
    if (ctx->pending.empty()) return;
    if (sync) (void)hipStreamSynchronize(ctx->stream);
    for (auto& p : ctx->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            ctx->prof_count[p.kind] += 1;
            ctx->prof_ms[p.kind] += ms;
        }
        ctx->pool.push_back(p.a);
        ctx->pool.push_back(p.b);
    }
    ctx->pending.clear();
}

extern "C" sc_status sc_ctx_set_profiling(sc_ctx* ctx, unsigned mask) {
    if (!ctx) return SC_E_INVAL;
    prof_drain(ctx, true);
    ctx->prof_mask = mask;
    return SC_OK;
}

extern "C" sc_status sc_ctx_profile(sc_ctx* ctx, int kind, int64_t* launches, double* total_ms) {
    if (!ctx || kind < 0 || kind >= SC_KIND_COUNT) return SC_E_INVAL;
    prof_drain(ctx, true);
    if (launches) *launches = ctx->prof_count[kind];
    if (total_ms) *total_ms = ctx->prof_ms[kind];
    return SC_OK;
}

extern "C" sc_status sc_ctx_profile_reset(sc_ctx* ctx) {
    if (!ctx) return SC_E_INVAL;
    prof_drain(ctx, true);
    for (int k = 0; k < SC_KIND_COUNT; ++k) {
        ctx->prof_count[k] = 0;
        ctx->prof_ms[k] = 0.0;
    }
    return SC_OK;
}

extern "C" const char* sc_last_error(const sc_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }
