// Graph symmetrisation W <- W + W' (Section II-A) and the normalised
// Laplacian values on W's pattern.
//
// graph_build: every directed edge e emits the keys (src*n + dst) at slot 2e
// and (dst*n + src) at slot 2e+1; a stable radix sort of (key, slot) orders
// the entries by (row, col) and, for equal keys, by slot; runs of equal keys
// merge into one stored entry whose weight is 1 (logical sum) or the sum of
// the run's weights in slot order (algebraic sum).
#include "sc_internal.h"

namespace {

constexpr int TH = 256;

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_emit(int64_t n, int64_t m, const int32_t* __restrict__ src,
                       const int32_t* __restrict__ dst, const double* __restrict__ w,
                       uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                       unsigned long long* loops, int* status) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const uint64_t sentinel = (uint64_t)n * (uint64_t)n;
    int32_t s = src[e], d = dst[e];
    bool bad = s < 0 || s >= n || d < 0 || d >= n;
    if (w) {
        double we = w[e];
        if (!(we >= 0.0) || !isfinite(we)) bad = true;
    }
    if (bad) atomicOr(status, DEV_BAD_INPUT);
    if (bad || s == d) {
        if (!bad) atomicAdd(loops, 1ull);
        keys[2 * e] = sentinel;
        keys[2 * e + 1] = sentinel;
    } else {
        keys[2 * e] = (uint64_t)s * (uint64_t)n + (uint64_t)d;
        keys[2 * e + 1] = (uint64_t)d * (uint64_t)n + (uint64_t)s;
    }
    vals[2 * e] = (uint32_t)(2 * e);
    vals[2 * e + 1] = (uint32_t)(2 * e + 1);
}

__global__ void k_mark(int64_t len, const uint64_t* __restrict__ keys, uint64_t sentinel,
                       uint64_t* __restrict__ flag) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= len) return;
    uint64_t k = keys[p];
    flag[p] = (k != sentinel && (p == 0 || keys[p - 1] != k)) ? 1 : 0;
}

__global__ void k_compact(int64_t n, int64_t len, const uint64_t* __restrict__ keys,
                          const uint32_t* __restrict__ vals, const uint64_t* __restrict__ incl,
                          const double* __restrict__ w, int algebraic, uint64_t sentinel,
                          int64_t* __restrict__ row_ptr, int32_t* __restrict__ col,
                          double* __restrict__ w_sym) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= len) return;
    uint64_t k = keys[p];
    if (k == sentinel) return;
    const bool start = (p == 0 || keys[p - 1] != k);
    const int64_t row = (int64_t)(k / (uint64_t)n);
    if (start) {
        const int64_t pos = (int64_t)incl[p] - 1;
        col[pos] = (int32_t)(k % (uint64_t)n);
        if (w_sym) {
            double acc = 1.0;
            if (algebraic) {
                acc = 0.0;
                for (int64_t q = p; q < len && keys[q] == k; ++q) acc += w[vals[q] >> 1];
            }
            w_sym[pos] = acc;
        }
        const int64_t prev_row = p > 0 ? (int64_t)(keys[p - 1] / (uint64_t)n) : -1;
        for (int64_t r = prev_row + 1; r <= row; ++r) row_ptr[r] = pos;
    }
    // last stored entry closes every remaining row
    if (p + 1 == len || keys[p + 1] == sentinel) {
        const int64_t nnz = (int64_t)incl[p];
        for (int64_t r = row + 1; r <= n; ++r) row_ptr[r] = nnz;
    }
}

__global__ void k_degree(int64_t n, const int64_t* __restrict__ row_ptr,
                         const double* __restrict__ w_sym, int algebraic,
                         double* __restrict__ degree) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t lo = row_ptr[i], hi = row_ptr[i + 1];
    double acc = 0.0;
    if (algebraic) {
        for (int64_t p = lo; p < hi; ++p) acc += w_sym[p];
    } else {
        acc = (double)(hi - lo);
    }
    degree[i] = acc;
}

__global__ void k_laplacian(int64_t n, const int64_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ col, const double* __restrict__ w_sym,
                            const double* __restrict__ degree, double* __restrict__ val64,
                            float* __restrict__ val32, double* __restrict__ dinv_sqrt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double di = degree[i];
    if (dinv_sqrt) dinv_sqrt[i] = di > 0.0 ? 1.0 / sqrt(di) : 0.0;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        const double dj = degree[col[p]];
        const double wp = w_sym ? w_sym[p] : 1.0;
        const double prod = di * dj;
        const double v = prod > 0.0 ? -(wp / sqrt(prod)) : 0.0;
        if (val64) val64[p] = v;
        if (val32) val32[p] = (float)v;
    }
}

// L = D - W (Section II-A): off-diagonal -w_p (exact), diagonal the degrees;
// diag32 is the FP32 copy of the diagonal for the FP32 product
__global__ void k_laplacian_comb(int64_t n, const int64_t* __restrict__ row_ptr,
                                 const double* __restrict__ w_sym, const double* __restrict__ degree,
                                 double* __restrict__ val64, float* __restrict__ val32,
                                 float* __restrict__ diag32) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (diag32) diag32[i] = (float)degree[i];
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        const double v = -(w_sym ? w_sym[p] : 1.0);
        if (val64) val64[p] = v;
        if (val32) val32[p] = (float)v;
    }
}

struct GraphWs {
    uint64_t *keys, *keys_alt, *flag, *radix_tmp, *scan_tmp;
    uint32_t *vals, *vals_alt;
    unsigned long long* loops;
    int* status;
};

size_t carve_graph(Carver& c, int64_t m, GraphWs& g) {
    const int64_t len = std::max<int64_t>(2 * m, 1);
    g.keys = c.take<uint64_t>(len);
    g.keys_alt = c.take<uint64_t>(len);
    g.flag = c.take<uint64_t>(len);
    g.vals = c.take<uint32_t>(len);
    g.vals_alt = c.take<uint32_t>(len);
    g.radix_tmp = c.take<uint64_t>(radix_tmp_elems(len));
    g.scan_tmp = c.take<uint64_t>(scan_u64_tmp_elems(len));
    g.loops = c.take<unsigned long long>(1);
    g.status = c.take<int>(1);
    return c.size();
}

}  // namespace

extern "C" sc_status sc_graph_build_workspace(sc_ctx* ctx, int64_t n, int64_t m, size_t* bytes) {
    if (!ctx || !bytes) return SC_E_INVAL;
    if (n <= 0 || m < 0 || m >= (int64_t(1) << 31))
        return sc_fail(ctx, SC_E_INVAL, "graph_build: need n > 0 and 0 <= m < 2^31");
    Carver c(nullptr);
    GraphWs g;
    *bytes = carve_graph(c, m, g);
    return SC_OK;
}

extern "C" sc_status sc_graph_build(sc_ctx* ctx, int64_t n, int64_t m, const int32_t* src,
                                    const int32_t* dst, const double* w, sc_sym_mode mode,
                                    int64_t* row_ptr, int32_t* col, double* w_sym, double* degree,
                                    int64_t* nnz_out, int64_t* self_loops, void* ws,
                                    size_t ws_bytes) {
    if (!ctx) return SC_E_INVAL;
    if (n <= 0 || m < 0 || m >= (int64_t(1) << 31) || n > (int64_t(1) << 31) - 1)
        return sc_fail(ctx, SC_E_INVAL, "graph_build: need 0 < n < 2^31 and 0 <= m < 2^31");
    if (!row_ptr || !degree || !nnz_out || (m > 0 && (!src || !dst || !col)) || !ws)
        return sc_fail(ctx, SC_E_INVAL, "graph_build: null pointer argument");
    if (mode != SC_SYM_LOGICAL && mode != SC_SYM_ALGEBRAIC)
        return sc_fail(ctx, SC_E_INVAL, "graph_build: unknown symmetrisation mode");
    const int algebraic = mode == SC_SYM_ALGEBRAIC;
    if (algebraic && (!w || !w_sym))
        return sc_fail(ctx, SC_E_INVAL, "graph_build: algebraic mode needs w and w_sym");
    Carver c(ws);
    GraphWs g;
    size_t need = carve_graph(c, m, g);
    if (ws_bytes < need)
        return sc_fail(ctx, SC_E_NOMEM, "graph_build: workspace %zu < %zu bytes", ws_bytes, need);
    SC_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int64_t len = 2 * m;
    ProfScope ps(ctx, SC_KIND_GRAPH);
    const uint64_t sentinel = (uint64_t)n * (uint64_t)n;

    SC_CHECK_HIP(ctx, hipMemsetAsync(g.loops, 0, sizeof(unsigned long long), st));
    SC_CHECK_HIP(ctx, hipMemsetAsync(g.status, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_fill_i64, dim3(ceil_div(n + 1, TH)), dim3(TH), 0, st, row_ptr, n + 1,
                       (int64_t)0);
    SC_CHECK_LAUNCH(ctx);
    if (m > 0) {
        hipLaunchKernelGGL(k_emit, dim3(ceil_div(m, TH)), dim3(TH), 0, st, n, m, src, dst,
                           algebraic ? w : nullptr, g.keys, g.vals, g.loops, g.status);
        SC_CHECK_LAUNCH(ctx);
        const int bits = ceil_log2_u64(sentinel + 1);
        SC_TRY(radix_sort_pairs(ctx, g.keys, g.vals, g.keys_alt, g.vals_alt, len, bits,
                                g.radix_tmp));
        hipLaunchKernelGGL(k_mark, dim3(ceil_div(len, TH)), dim3(TH), 0, st, len, g.keys, sentinel,
                           g.flag);
        SC_CHECK_LAUNCH(ctx);
        SC_TRY(scan_u64(ctx, g.flag, g.flag, len, 1, g.scan_tmp));
        hipLaunchKernelGGL(k_compact, dim3(ceil_div(len, TH)), dim3(TH), 0, st, n, len, g.keys,
                           g.vals, g.flag, w, algebraic, sentinel, row_ptr, col, w_sym);
        SC_CHECK_LAUNCH(ctx);
    }
    hipLaunchKernelGGL(k_degree, dim3(ceil_div(n, TH)), dim3(TH), 0, st, n, row_ptr, w_sym,
                       algebraic, degree);
    SC_CHECK_LAUNCH(ctx);
    int64_t* h = static_cast<int64_t*>(ctx->stage);
    SC_CHECK_HIP(ctx, hipMemcpyAsync(&h[0], row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SC_CHECK_HIP(ctx, hipMemcpyAsync(&h[1], g.loops, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SC_CHECK_HIP(ctx, hipMemcpyAsync(&h[2], g.status, sizeof(int), hipMemcpyDeviceToHost, st));
    SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
    if ((int)h[2] & DEV_BAD_INPUT)
        return sc_fail(ctx, SC_E_INVAL, "graph_build: vertex id outside [0, n) or invalid weight");
    *nnz_out = h[0];
    if (self_loops) *self_loops = h[1];
    return SC_OK;
}

extern "C" sc_status sc_laplacian_csr(sc_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                      const int32_t* col, const double* w_sym,
                                      const double* degree, double* val64, float* val32,
                                      double* dinv_sqrt) {
    if (!ctx) return SC_E_INVAL;
    if (n <= 0 || nnz < 0) return sc_fail(ctx, SC_E_INVAL, "laplacian_csr: need n > 0, nnz >= 0");
    if (!row_ptr || !degree || (nnz > 0 && !col))
        return sc_fail(ctx, SC_E_INVAL, "laplacian_csr: null pointer argument");
    SC_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_laplacian, dim3(ceil_div(n, TH)), dim3(TH), 0, ctx->stream, n, row_ptr,
                       col, w_sym, degree, val64, val32, dinv_sqrt);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}

extern "C" sc_status sc_laplacian_combinatorial(sc_ctx* ctx, int64_t n, int64_t nnz,
                                                const int64_t* row_ptr, const double* w_sym,
                                                const double* degree, double* val64, float* val32,
                                                float* diag32) {
    if (!ctx) return SC_E_INVAL;
    if (n <= 0 || nnz < 0)
        return sc_fail(ctx, SC_E_INVAL, "laplacian_combinatorial: need n > 0, nnz >= 0");
    if (!row_ptr || !degree) return sc_fail(ctx, SC_E_INVAL, "laplacian_combinatorial: null pointer argument");
    SC_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_laplacian_comb, dim3(ceil_div(n, TH)), dim3(TH), 0, ctx->stream, n, row_ptr,
                       w_sym, degree, val64, val32, diag32);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}
