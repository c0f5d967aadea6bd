// Warm start for a streaming stage that adds vertices (Section III: the
// previous graph's approximate eigenvectors start the solve for the current
// one; the rows of vertices the previous graph lacked must be filled in).
// Vertices 0 .. n_old-1 keep their rows; each new vertex takes the mean of the
// rows of its neighbours that already existed: the FP64 sum over its CSR row
// in ascending column order, from 0.0, divided by their count, rounded once to
// the block's type.  A new vertex without such a neighbour keeps a zero row.
// One wave per new vertex, lanes over the columns.
#include "sc_internal.h"

namespace {

constexpr int WF_TH = 256;
constexpr int WF_CPL = 4;        // columns per lane: k <= 256

template <class T>
__global__ void __launch_bounds__(WF_TH)
k_warm_fill(int64_t n, int64_t n_old, const int64_t* __restrict__ row_ptr,
            const int32_t* __restrict__ col, int k, T* __restrict__ X, int64_t ldx) {
    const int64_t i = n_old + (int64_t)blockIdx.x * (WF_TH / 64) + (threadIdx.x >> 6);
    if (i >= n) return;
    const int lane = threadIdx.x & 63;
    double acc[WF_CPL];
#pragma unroll
    for (int c = 0; c < WF_CPL; ++c) acc[c] = 0.0;
    int64_t cnt = 0;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        const int64_t j = col[p];
        if (j >= n_old) continue;                 // wave-uniform
        const T* xj = X + j * ldx;
#pragma unroll
        for (int c = 0; c < WF_CPL; ++c) {
            const int d = lane + 64 * c;
            if (d < k) acc[c] += (double)xj[d];
        }
        ++cnt;
    }
    T* xi = X + i * ldx;
#pragma unroll
    for (int c = 0; c < WF_CPL; ++c) {
        const int d = lane + 64 * c;
        if (d < k) xi[d] = cnt > 0 ? (T)(acc[c] / (double)cnt) : T(0);
    }
}

}  // namespace

extern "C" sc_status sc_warm_fill(sc_ctx* ctx, int64_t n, int64_t n_old, const int64_t* row_ptr,
                                  const int32_t* col, int k, void* X, int64_t ldx, int x_fp32) {
    if (!ctx) return SC_E_INVAL;
    if (n <= 0 || n_old < 0 || n_old > n || k <= 0 || k > 64 * WF_CPL || ldx < k)
        return sc_fail(ctx, SC_E_INVAL, "warm_fill: need 0 <= n_old <= n, 0 < k <= %d, ldx >= k",
                       64 * WF_CPL);
    if (!row_ptr || !X || !col) return sc_fail(ctx, SC_E_INVAL, "warm_fill: null pointer argument");
    if (n_old == n) return SC_OK;
    SC_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    const dim3 grid((unsigned)ceil_div(n - n_old, WF_TH / 64));
    if (x_fp32)
        hipLaunchKernelGGL((k_warm_fill<float>), grid, dim3(WF_TH), 0, ctx->stream, n, n_old, row_ptr,
                           col, k, static_cast<float*>(X), ldx);
    else
        hipLaunchKernelGGL((k_warm_fill<double>), grid, dim3(WF_TH), 0, ctx->stream, n, n_old, row_ptr,
                           col, k, static_cast<double*>(X), ldx);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}
