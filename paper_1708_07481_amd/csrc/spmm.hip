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
#include <hip/hip_bf16.h>

#include <type_traits>

#include "sc_internal.h"

namespace {

constexpr int TH = 256;

template <class T>
__device__ __forceinline__ T widen(T v) { return v; }
template <class T>
__device__ __forceinline__ T widen(_Float16 v) { return (T)(float)v; }
template <class T>
__device__ __forceinline__ T widen(__hip_bfloat16 v) { return (T)__bfloat162float(v); }

// TG: type of the gathered neighbour rows (T itself, or a 16-bit copy Xg of X
// widened to T on load); the row's own x_ij always comes from X.  order:
// optional row permutation (group g computes row order[g]), e.g. the rows in
// descending length so that the longest rows start first.
template <class T, class TG, int LPR, int NC>
__global__ void __launch_bounds__(TH) k_spmm(int64_t n, const int64_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col,
                                              const T* __restrict__ val,
                                              const T* __restrict__ diag, int k,
                                              const T* __restrict__ X, int64_t ldx,
                                              const TG* __restrict__ Xg, int64_t ldg,
                                              const int32_t* __restrict__ order,
                                              T* __restrict__ Y, int64_t ldy) {
    const int64_t grp = ((int64_t)blockIdx.x * TH + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (grp >= n) return;
    const int64_t row = order ? (int64_t)order[grp] : grp;
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
                g[u][c] = ok[c] ? widen<T>(Xg[(int64_t)cp[u] * ldg + lane + LPR * c]) : T(0);
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
            if (ok[c]) acc[c] = fma(vp, widen<T>(Xg[(int64_t)cp * ldg + lane + LPR * c]), acc[c]);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (ok[c]) Y[row * ldy + lane + LPR * c] = acc[c];
}

// Same product with 16-byte lane accesses (sc_spmm_ex's SC_GATHER_FP32_LANE16,
// for comparing access widths; the solver takes k_spmm): lane l of a group of LPR lanes owns
// the V = 16 / sizeof(T) adjacent columns j = V (l + LPR c) + e (c < NC,
// e < V), and every gathered neighbour row is read as NC 16-byte pieces per
// lane.  A wave then holds 64 / LPR rows and issues one load instruction per
// 1 KB of neighbour rows instead of one per 256 B.  Each output element is
// still a_i x_ij followed by the fma chain over the row in ascending column
// order, so the result is bit-identical to k_spmm.  Requires k = V LPR NC,
// ldx and ldy multiples of V and 16-byte aligned X and Y.
template <class T, int LPR, int NC>
__global__ void __launch_bounds__(TH) k_spmm_vec(int64_t n, const int64_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col,
                                                  const T* __restrict__ val,
                                                  const T* __restrict__ diag,
                                                  const T* __restrict__ X, int64_t ldx,
                                                  const int32_t* __restrict__ order,
                                                  T* __restrict__ Y, int64_t ldy) {
    constexpr int V = 16 / (int)sizeof(T);
    using vec = T __attribute__((ext_vector_type(V)));
    const int64_t grp = ((int64_t)blockIdx.x * TH + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (grp >= n) return;
    const int64_t row = order ? (int64_t)order[grp] : grp;
    const int64_t lo = row_ptr[row], hi = row_ptr[row + 1];
    const T a = diag ? diag[row] : T(1);
    vec acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const vec x = *reinterpret_cast<const vec*>(X + row * ldx + V * (lane + LPR * c));
#pragma unroll
        for (int e = 0; e < V; ++e) acc[c][e] = diag ? a * x[e] : x[e];
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
        vec g[4][NC];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < NC; ++c)
                g[u][c] = *reinterpret_cast<const vec*>(X + (int64_t)cp[u] * ldx +
                                                        V * (lane + LPR * c));
        // all 4 NC pieces in flight before the first use (the scheduler would
        // otherwise keep two or three, for fewer registers)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int e = 0; e < V; ++e) acc[c][e] = fma(vp[u], g[u][c][e], acc[c][e]);
    }
    for (; p < hi; ++p) {
        const int32_t cp = col[p];
        const T vp = val[p];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const vec g = *reinterpret_cast<const vec*>(X + (int64_t)cp * ldx + V * (lane + LPR * c));
#pragma unroll
            for (int e = 0; e < V; ++e) acc[c][e] = fma(vp, g[e], acc[c][e]);
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        *reinterpret_cast<vec*>(Y + row * ldy + V * (lane + LPR * c)) = acc[c];
}

template <class T, int LPR, int NC>
sc_status go_vec(sc_ctx* ctx, int64_t n, const int64_t* rp, const int32_t* col, const T* val,
                 const T* diag, const T* X, int64_t ldx, const int32_t* order, T* Y,
                 int64_t ldy) {
    const int64_t rows_per_block = TH / LPR;
    hipLaunchKernelGGL((k_spmm_vec<T, LPR, NC>), dim3(ceil_div(n, rows_per_block)), dim3(TH), 0,
                       ctx->stream, n, rp, col, val, diag, X, ldx, order, Y, ldy);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}

// The 16-byte layout when k splits into whole 16-byte pieces over 8 or 16
// lanes (at most 6 pieces per lane) and the rows are 16-byte aligned; returns
// false when it does not apply.
template <class T>
bool try_vec(sc_ctx* ctx, sc_status* st, int64_t n, const int64_t* rp, const int32_t* col,
             const T* val, const T* diag, int k, const T* X, int64_t ldx, const int32_t* order,
             T* Y, int64_t ldy) {
    constexpr int V = 16 / (int)sizeof(T);
    if (k % V || ldx % V || ldy % V || (reinterpret_cast<uintptr_t>(X) & 15) ||
        (reinterpret_cast<uintptr_t>(Y) & 15))
        return false;
    const int kv = k / V;
    int lpr = 0;
    if (kv % 8 == 0 && kv / 8 <= 6) lpr = 8;
    else if (kv % 16 == 0 && kv / 16 <= 6) lpr = 16;
    else return false;
    const int nc = kv / lpr;
#define SC_SPMM_VEC(L, C) \
    if (lpr == L && nc == C) { \
        *st = go_vec<T, L, C>(ctx, n, rp, col, val, diag, X, ldx, order, Y, ldy); \
        return true; \
    }
    SC_SPMM_VEC(8, 1) SC_SPMM_VEC(8, 2) SC_SPMM_VEC(8, 3)
    SC_SPMM_VEC(8, 4) SC_SPMM_VEC(8, 5) SC_SPMM_VEC(8, 6)
    SC_SPMM_VEC(16, 5)
#undef SC_SPMM_VEC
    return false;
}

// FP32 product with the neighbour rows from a 16-bit copy Xg, 16-byte lane
// reads: lane l of a group of LPR lanes owns the 8 adjacent columns
// j = 8 (l + LPR c) + e, reads them as one 16-byte piece of the copy per
// neighbour, widens each to FP32 and runs the same fma chain as k_spmm (the
// row's own x_ij from X in FP32), so the result is bit-identical to k_spmm
// with the same copy.  Requires k = 8 LPR NC, ldx a multiple of 4, ldg and ldy
// multiples of 8 (ldy of 4), and 16-byte aligned X, Xg and Y.
__device__ __forceinline__ float widen16(unsigned short u, _Float16*) {
    return (float)__builtin_bit_cast(_Float16, u);
}
__device__ __forceinline__ float widen16(unsigned short u, __hip_bfloat16*) {
    return __uint_as_float((unsigned)u << 16);
}

template <class TG, int LPR, int NC>
__global__ void __launch_bounds__(TH) k_spmm_vec16(int64_t n, const int64_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col,
                                                    const float* __restrict__ val,
                                                    const float* __restrict__ diag,
                                                    const float* __restrict__ X, int64_t ldx,
                                                    const TG* __restrict__ Xg, int64_t ldg,
                                                    const int32_t* __restrict__ order,
                                                    float* __restrict__ Y, int64_t ldy) {
    using h8 = unsigned short __attribute__((ext_vector_type(8)));
    using f4 = float __attribute__((ext_vector_type(4)));
    const int64_t grp = ((int64_t)blockIdx.x * TH + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (grp >= n) return;
    const int64_t row = order ? (int64_t)order[grp] : grp;
    const int64_t lo = row_ptr[row], hi = row_ptr[row + 1];
    const float a = diag ? diag[row] : 1.0f;
    const unsigned short* G = reinterpret_cast<const unsigned short*>(Xg);
    float acc[NC][8];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const float* xr = X + row * ldx + 8 * (lane + LPR * c);
        const f4 x0 = *reinterpret_cast<const f4*>(xr), x1 = *reinterpret_cast<const f4*>(xr + 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            acc[c][e] = diag ? a * x0[e] : x0[e];
            acc[c][e + 4] = diag ? a * x1[e] : x1[e];
        }
    }
    int64_t p = lo;
    for (; p + 4 <= hi; p += 4) {
        int32_t cp[4];
        float vp[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            cp[u] = col[p + u];
            vp[u] = val[p + u];
        }
        h8 g[4][NC];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < NC; ++c)
                g[u][c] = *reinterpret_cast<const h8*>(G + (int64_t)cp[u] * ldg + 8 * (lane + LPR * c));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    acc[c][e] = fma(vp[u], widen16(g[u][c][e], (TG*)nullptr), acc[c][e]);
    }
    for (; p < hi; ++p) {
        const int32_t cp = col[p];
        const float vp = val[p];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const h8 g = *reinterpret_cast<const h8*>(G + (int64_t)cp * ldg + 8 * (lane + LPR * c));
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[c][e] = fma(vp, widen16(g[e], (TG*)nullptr), acc[c][e]);
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        float* yr = Y + row * ldy + 8 * (lane + LPR * c);
        *reinterpret_cast<f4*>(yr) = f4{acc[c][0], acc[c][1], acc[c][2], acc[c][3]};
        *reinterpret_cast<f4*>(yr + 4) = f4{acc[c][4], acc[c][5], acc[c][6], acc[c][7]};
    }
}

// The 16-byte layout for a 16-bit gather copy when k = 32 NC (NC <= 6) and the
// strides and pointers are aligned; returns false when it does not apply.
template <class TG>
bool try_vec16(sc_ctx* ctx, sc_status* st, int64_t n, const int64_t* rp, const int32_t* col,
               const float* val, const float* diag, int k, const float* X, int64_t ldx,
               const TG* Xg, int64_t ldg, const int32_t* order, float* Y, int64_t ldy) {
    if (k % 32 || k / 32 > 6 || ldx % 4 || ldy % 4 || ldg % 8 ||
        ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Xg) |
          reinterpret_cast<uintptr_t>(Y)) & 15))
        return false;
    constexpr int LPR = 4;
    const int64_t grid = ceil_div(n, (int64_t)(TH / LPR));
#define SC_SPMM_V16(C)                                                                          \
    case C:                                                                                     \
        hipLaunchKernelGGL((k_spmm_vec16<TG, LPR, C>), dim3(grid), dim3(TH), 0, ctx->stream, n, \
                           rp, col, val, diag, X, ldx, Xg, ldg, order, Y, ldy);                 \
        break;
    switch (k / 32) {
        SC_SPMM_V16(1) SC_SPMM_V16(2) SC_SPMM_V16(3) SC_SPMM_V16(4) SC_SPMM_V16(5) SC_SPMM_V16(6)
    default: return false;
    }
#undef SC_SPMM_V16
    const hipError_t e = hipGetLastError();
    *st = e == hipSuccess ? SC_OK : sc_fail(ctx, SC_E_HIP, "spmm launch: %s", hipGetErrorString(e));
    return true;
}

template <class T, class TG, int LPR, int NC>
sc_status go(sc_ctx* ctx, int64_t n, const int64_t* rp, const int32_t* col, const T* val,
             const T* diag, int k, const T* X, int64_t ldx, const TG* Xg, int64_t ldg,
             const int32_t* order, T* Y, int64_t ldy) {
    const int64_t rows_per_block = TH / LPR;
    hipLaunchKernelGGL((k_spmm<T, TG, LPR, NC>), dim3(ceil_div(n, rows_per_block)), dim3(TH), 0,
                       ctx->stream, n, rp, col, val, diag, k, X, ldx, Xg, ldg, order, Y, ldy);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}

// vec_lanes: take the 16-byte lane layouts (k_spmm_vec, k_spmm_vec16) where
// they apply.
template <class T, class TG>
sc_status dispatch(sc_ctx* ctx, int64_t n, const int64_t* rp, const int32_t* col, const T* val,
                   const T* diag, int k, const T* X, int64_t ldx, const TG* Xg, int64_t ldg,
                   const int32_t* order, T* Y, int64_t ldy, bool vec_lanes = false) {
    if (n <= 0 || k <= 0) return SC_OK;
    if constexpr (std::is_same<T, float>::value && std::is_same<TG, float>::value) {
        sc_status st;
        if (vec_lanes && try_vec<T>(ctx, &st, n, rp, col, val, diag, k, X, ldx, order, Y, ldy))
            return st;
    } else if constexpr (std::is_same<T, float>::value) {
        sc_status st;
        if (vec_lanes &&
            try_vec16<TG>(ctx, &st, n, rp, col, val, diag, k, X, ldx, Xg, ldg, order, Y, ldy))
            return st;
    }
#define SC_SPMM_GO(L, C) go<T, TG, L, C>(ctx, n, rp, col, val, diag, k, X, ldx, Xg, ldg, order, Y, ldy)
    if (k <= 8) return SC_SPMM_GO(8, 1);
    if (k <= 16) return SC_SPMM_GO(16, 1);
    if (k <= 32) return SC_SPMM_GO(32, 1);
    if (k <= 64) return SC_SPMM_GO(64, 1);
    if (k <= 128) return SC_SPMM_GO(64, 2);
    if (k <= 192) return SC_SPMM_GO(64, 3);
    if (k <= 256) return SC_SPMM_GO(64, 4);
#undef SC_SPMM_GO
    return sc_fail(ctx, SC_E_UNSUPPORTED, "spmm: k = %d > 256", k);
}

}  // namespace

template <class T>
sc_status launch_spmm(sc_ctx* ctx, int64_t n, const int64_t* rp, const int32_t* col, const T* val,
                      const T* diag, int k, const T* X, int64_t ldx, T* Y, int64_t ldy,
                      const int32_t* order) {
    return dispatch<T, T>(ctx, n, rp, col, val, diag, k, X, ldx, X, ldx, order, Y, ldy);
}

template sc_status launch_spmm<double>(sc_ctx*, int64_t, const int64_t*, const int32_t*,
                                       const double*, const double*, int, const double*, int64_t,
                                       double*, int64_t, const int32_t*);
template sc_status launch_spmm<float>(sc_ctx*, int64_t, const int64_t*, const int32_t*,
                                      const float*, const float*, int, const float*, int64_t,
                                      float*, int64_t, const int32_t*);

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

extern "C" sc_status sc_spmm_ex(sc_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                const int32_t* col, const float* val, const float* diag, int k,
                                const float* X, int64_t ldx, const void* Xg, int64_t ldg,
                                int gather, const int32_t* order, float* Y, int64_t ldy) {
    if (!ctx) return SC_E_INVAL;
    if (n <= 0 || nnz < 0 || k <= 0 || ldx < k || ldy < k)
        return sc_fail(ctx, SC_E_INVAL, "spmm_ex: need n > 0, k > 0, ldx >= k, ldy >= k");
    if (!row_ptr || !X || !Y || (nnz > 0 && (!col || !val)))
        return sc_fail(ctx, SC_E_INVAL, "spmm_ex: null pointer argument");
    if (X == Y) return sc_fail(ctx, SC_E_INVAL, "spmm_ex: X and Y must not alias");
    if ((gather == SC_GATHER_FP16 || gather == SC_GATHER_BF16) && (!Xg || ldg < k))
        return sc_fail(ctx, SC_E_INVAL, "spmm_ex: a 16-bit gather copy needs Xg and ldg >= k");
    SC_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    ProfScope ps(ctx, SC_KIND_SPMM);
    switch (gather) {
    case SC_GATHER_FP32:
        return dispatch<float, float>(ctx, n, row_ptr, col, val, diag, k, X, ldx, X, ldx, order, Y,
                                      ldy);
    case SC_GATHER_FP32_LANE16:
        return dispatch<float, float>(ctx, n, row_ptr, col, val, diag, k, X, ldx, X, ldx, order, Y,
                                      ldy, true);
    case SC_GATHER_FP16:
        return dispatch<float, _Float16>(ctx, n, row_ptr, col, val, diag, k, X, ldx,
                                         static_cast<const _Float16*>(Xg), ldg, order, Y, ldy,
                                         true);
    case SC_GATHER_BF16:
        return dispatch<float, __hip_bfloat16>(ctx, n, row_ptr, col, val, diag, k, X, ldx,
                                               static_cast<const __hip_bfloat16*>(Xg), ldg, order,
                                               Y, ldy, true);
    default:
        return sc_fail(ctx, SC_E_INVAL, "spmm_ex: unknown gather type %d", gather);
    }
}

// ---------------------------------------------------------------------------
// Row order by length: the rows sorted by descending stored-entry count (stable,
// so equal lengths keep ascending row order), for sc_spmm_ex's `order`.
// ---------------------------------------------------------------------------
namespace {

__global__ void k_len_keys(int64_t n, const int64_t* __restrict__ row_ptr,
                           uint64_t* __restrict__ keys, uint32_t* __restrict__ rows) {
    const int64_t i = (int64_t)blockIdx.x * TH + threadIdx.x;
    if (i >= n) return;
    const int64_t len = row_ptr[i + 1] - row_ptr[i];
    keys[i] = 0xFFFFFFFFull - (uint64_t)min<int64_t>(len, 0xFFFFFFFFll);
    rows[i] = (uint32_t)i;
}

struct OrderWs {
    uint64_t *keys, *keys_alt, *tmp;
    uint32_t* rows_alt;
};

size_t carve_order(Carver& c, int64_t n, OrderWs& w) {
    w.keys = c.take<uint64_t>((size_t)n);
    w.keys_alt = c.take<uint64_t>((size_t)n);
    w.rows_alt = c.take<uint32_t>((size_t)n);
    w.tmp = c.take<uint64_t>(radix_tmp_elems(n));
    return c.size();
}

}  // namespace

size_t row_order_scratch_bytes(int64_t n) {
    Carver c(nullptr);
    OrderWs w;
    return carve_order(c, n, w);
}

sc_status row_order_by_length(sc_ctx* ctx, int64_t n, const int64_t* row_ptr, int32_t* order,
                              void* scratch) {
    Carver c(scratch);
    OrderWs w;
    carve_order(c, n, w);
    uint32_t* rows = reinterpret_cast<uint32_t*>(order);
    hipLaunchKernelGGL(k_len_keys, dim3((unsigned)ceil_div(n, TH)), dim3(TH), 0, ctx->stream, n,
                       row_ptr, w.keys, rows);
    SC_CHECK_LAUNCH(ctx);
    return radix_sort_pairs(ctx, w.keys, rows, w.keys_alt, w.rows_alt, n, 32, w.tmp);
}

extern "C" sc_status sc_row_order_workspace(sc_ctx* ctx, int64_t n, size_t* bytes) {
    if (!ctx || !bytes) return SC_E_INVAL;
    if (n <= 0 || n >= (int64_t(1) << 31)) return sc_fail(ctx, SC_E_INVAL, "row_order: need 0 < n < 2^31");
    *bytes = row_order_scratch_bytes(n);
    return SC_OK;
}

extern "C" sc_status sc_row_order(sc_ctx* ctx, int64_t n, const int64_t* row_ptr, int32_t* order,
                                  void* ws, size_t ws_bytes) {
    if (!ctx) return SC_E_INVAL;
    if (n <= 0 || n >= (int64_t(1) << 31)) return sc_fail(ctx, SC_E_INVAL, "row_order: need 0 < n < 2^31");
    if (!row_ptr || !order || !ws) return sc_fail(ctx, SC_E_INVAL, "row_order: null pointer argument");
    const size_t need = row_order_scratch_bytes(n);
    if (ws_bytes < need) return sc_fail(ctx, SC_E_NOMEM, "row_order: workspace %zu < %zu", ws_bytes, need);
    SC_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    return row_order_by_length(ctx, n, row_ptr, order, ws);
}
