// Context, error reporting and version of the spectral-clustering library.
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

extern "C" int sc_version(void) { return 10000; }

extern "C" sc_status sc_ctx_create(int device, void* hip_stream, sc_ctx** out) {
    if (!out) return SC_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SC_E_INVAL;
    sc_ctx* c = new sc_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(device) != hipSuccess) {
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
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    delete ctx;
    return SC_OK;
}

extern "C" const char* sc_last_error(const sc_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }
