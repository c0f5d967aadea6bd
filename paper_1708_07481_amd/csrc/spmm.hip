// Y = L X with L = diag(a) + offdiag(val) in CSR form: the single product
// with the graph Laplacian per LOBPCG iteration (Section III).  a = 1 (no
// diagonal array) for the normalised Laplacian I - D^-1/2 W D^-1/2; a = the
// degrees for L = D - W (Section II-A), as the pre-computed diagonal of the
// paper's matrix-free product.
//
// A group of LPR lanes owns one row i; lane l of the group owns the columns
// j = l + LPR*c (c < NC).  Every lane starts from a_i x_ij (one rounded
// product; x_ij itself when a = 1) and walks row i in ascending column order
// with y = fma(v_p, x_{col_p, j}, y), so each output element is the exact
// sequential chain of the definition; the lanes of a group gather one
// contiguous row of X per stored entry.
#include "sc_internal.h"

namespace {

constexpr int TH = 256;

template <class T, int LPR, int NC>
__global__ void __launch_bounds__(TH) k_spmm(int64_t n, const int64_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col,
                                              const T* __restrict__ val,
                                              const T* __restrict__ diag, int k,
                                              const T* __restrict__ X, int64_t ldx,
                                              T* __restrict__ Y, int64_t ldy) {
    const int64_t row = ((int64_t)blockIdx.x * TH + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= n) return;
    const int64_t lo = row_ptr[row], hi = row_ptr[row + 1];
    const T a = diag ? diag[row] : T(1);
    T acc[NC];
    bool ok[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int j = lane + LPR * c;
        ok[c] = j < k;
        const T x = ok[c] ? X[row * ldx + j] : T(0);
        acc[c] = diag ? a * x : x;
    }
    int64_t p = lo;
    for (; p + 4 <= hi; p += 4) {
        int32_t cp[4];
        T vp[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            cp[u] = col[p + u];
            vp[u] = val[p + u];
        }
        T g[4][NC];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < NC; ++c)
                g[u][c] = ok[c] ? X[(int64_t)cp[u] * ldx + lane + LPR * c] : T(0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] = fma(vp[u], g[u][c], acc[c]);
    }
    for (; p < hi; ++p) {
        const int32_t cp = col[p];
        const T vp = val[p];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (ok[c]) acc[c] = fma(vp, X[(int64_t)cp * ldx + lane + LPR * c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (ok[c]) Y[row * ldy + lane + LPR * c] = acc[c];
}

template <class T, int LPR, int NC>
sc_status go(sc_ctx* ctx, int64_t n, const int64_t* rp, const int32_t* col, const T* val,
             const T* diag, int k, const T* X, int64_t ldx, T* Y, int64_t ldy) {
    const int64_t rows_per_block = TH / LPR;
    hipLaunchKernelGGL((k_spmm<T, LPR, NC>), dim3(ceil_div(n, rows_per_block)), dim3(TH), 0,
                       ctx->stream, n, rp, col, val, diag, k, X, ldx, Y, ldy);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}

}  // namespace

template <class T>
sc_status launch_spmm(sc_ctx* ctx, int64_t n, const int64_t* rp, const int32_t* col, const T* val,
                      const T* diag, int k, const T* X, int64_t ldx, T* Y, int64_t ldy) {
    if (n <= 0 || k <= 0) return SC_OK;
    if (k <= 8) return go<T, 8, 1>(ctx, n, rp, col, val, diag, k, X, ldx, Y, ldy);
    if (k <= 16) return go<T, 16, 1>(ctx, n, rp, col, val, diag, k, X, ldx, Y, ldy);
    if (k <= 32) return go<T, 32, 1>(ctx, n, rp, col, val, diag, k, X, ldx, Y, ldy);
    if (k <= 64) return go<T, 64, 1>(ctx, n, rp, col, val, diag, k, X, ldx, Y, ldy);
    if (k <= 128) return go<T, 64, 2>(ctx, n, rp, col, val, diag, k, X, ldx, Y, ldy);
    if (k <= 192) return go<T, 64, 3>(ctx, n, rp, col, val, diag, k, X, ldx, Y, ldy);
    if (k <= 256) return go<T, 64, 4>(ctx, n, rp, col, val, diag, k, X, ldx, Y, ldy);
    return sc_fail(ctx, SC_E_UNSUPPORTED, "spmm: k = %d > 256", k);
}

template sc_status launch_spmm<double>(sc_ctx*, int64_t, const int64_t*, const int32_t*,
                                       const double*, const double*, int, const double*, int64_t,
                                       double*, int64_t);
template sc_status launch_spmm<float>(sc_ctx*, int64_t, const int64_t*, const int32_t*,
                                      const float*, const float*, int, const float*, int64_t,
                                      float*, int64_t);

extern "C" sc_status sc_spmm_diag(sc_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                  const int32_t* col, const void* val, const void* diag, int fp64,
                                  int k, const void* X, int64_t ldx, void* Y, int64_t ldy) {
    if (!ctx) return SC_E_INVAL;
    if (n <= 0 || nnz < 0 || k <= 0 || ldx < k || ldy < k)
        return sc_fail(ctx, SC_E_INVAL, "spmm: need n > 0, k > 0, ldx >= k, ldy >= k");
    if (!row_ptr || !X || !Y || (nnz > 0 && (!col || !val)))
        return sc_fail(ctx, SC_E_INVAL, "spmm: null pointer argument");
    if (X == Y) return sc_fail(ctx, SC_E_INVAL, "spmm: X and Y must not alias");
    SC_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    ProfScope ps(ctx, SC_KIND_SPMM);
    if (fp64)
        return launch_spmm<double>(ctx, n, row_ptr, col, static_cast<const double*>(val),
                                   static_cast<const double*>(diag), k,
                                   static_cast<const double*>(X), ldx, static_cast<double*>(Y),
                                   ldy);
    return launch_spmm<float>(ctx, n, row_ptr, col, static_cast<const float*>(val),
                              static_cast<const float*>(diag), k, static_cast<const float*>(X), ldx,
                              static_cast<float*>(Y), ldy);
}

extern "C" sc_status sc_spmm(sc_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                             const int32_t* col, const void* val, int fp64, int k, const void* X,
                             int64_t ldx, void* Y, int64_t ldy) {
    return sc_spmm_diag(ctx, n, nnz, row_ptr, col, val, nullptr, fp64, k, X, ldx, Y, ldy);
}
