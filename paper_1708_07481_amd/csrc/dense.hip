// Dense multivector kernels of the LOBPCG iteration: Gram products of
// tall-skinny blocks, Cholesky-QR factors of small Gram matrices, in-place
// right multiplications of row blocks, the fused block update and the
// residual with its column norms.
//
// Reductions over the n rows are split into row chunks whose FP64 partial
// results are summed in chunk order by a second kernel, so every result is
// deterministic (no floating-point atomics).
#include "sc_internal.h"

namespace {

// ---------------------------------------------------------------------------
// Gram products: G = A^T B over n rows; 64 x 64 output tiles, 256 threads,
// 4 x 4 outputs per thread, 16 rows staged in LDS per step.
// ---------------------------------------------------------------------------
constexpr int GT = 64;      // tile edge
constexpr int GR = 16;      // rows per LDS stage

template <class T, class ACC, bool TWO>
__global__ void __launch_bounds__(256)
k_gram_partial(int64_t n, int c, int64_t chunk_rows, const T* __restrict__ A, int64_t lda,
               const T* __restrict__ B1, int64_t ldb1, const T* __restrict__ B2, int64_t ldb2,
               double* __restrict__ partial, int tiles) {
    // upper tile (ti <= tj) from the linear block index
    int t = blockIdx.x, ti = 0;
    while (t >= tiles - ti) {
        t -= tiles - ti;
        ++ti;
    }
    const int tj = ti + t;
    const int chunk = blockIdx.y;
    const int64_t r0 = (int64_t)chunk * chunk_rows;
    const int64_t r1 = min<int64_t>(n, r0 + chunk_rows);
    __shared__ T As[GR][GT];
    __shared__ T Bs1[GR][GT];
    __shared__ T Bs2[TWO ? GR : 1][GT];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    ACC acc1[4][4], acc2[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            acc1[r][s] = ACC(0);
            acc2[r][s] = ACC(0);
        }
    const int ca = ti * GT, cb = tj * GT;
    for (int64_t row = r0; row < r1; row += GR) {
#pragma unroll
        for (int q = 0; q < (GR * GT) / 256; ++q) {
            const int e = q * 256 + threadIdx.x;
            const int rr = e / GT, cc = e % GT;
            const int64_t gr = row + rr;
            const bool in = gr < r1;
            As[rr][cc] = (in && ca + cc < c) ? A[gr * lda + ca + cc] : T(0);
            Bs1[rr][cc] = (in && cb + cc < c) ? B1[gr * ldb1 + cb + cc] : T(0);
            if (TWO) Bs2[rr][cc] = (in && cb + cc < c) ? B2[gr * ldb2 + cb + cc] : T(0);
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < GR; ++rr) {
            ACC a[4], b1[4], b2[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = (ACC)As[rr][ty * 4 + r];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                b1[s] = (ACC)Bs1[rr][tx * 4 + s];
                if (TWO) b2[s] = (ACC)Bs2[rr][tx * 4 + s];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    acc1[r][s] = fma(a[r], b1[s], acc1[r][s]);
                    if (TWO) acc2[r][s] = fma(a[r], b2[s], acc2[r][s]);
                }
        }
        __syncthreads();
    }
    const int64_t cc2 = (int64_t)c * c;
    double* p1 = partial + (int64_t)chunk * (TWO ? 2 : 1) * cc2;
    double* p2 = p1 + cc2;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int a = ca + ty * 4 + r, b = cb + tx * 4 + s;
            if (a < c && b < c) {
                p1[(int64_t)a * c + b] = (double)acc1[r][s];
                if (TWO) p2[(int64_t)a * c + b] = (double)acc2[r][s];
            }
        }
}

// sum the chunk partials in chunk order; upper entries, mirrored
__global__ void k_gram_reduce(int c, int chunks, int nout, const double* __restrict__ partial,
                              double* __restrict__ G1, double* __restrict__ G2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cc2 = (int64_t)c * c;
    if (e >= cc2) return;
    const int a = (int)(e / c), b = (int)(e % c);
    if (a > b) return;
    for (int g = 0; g < nout; ++g) {
        double s = 0.0;
        for (int q = 0; q < chunks; ++q) s += partial[((int64_t)q * nout + g) * cc2 + e];
        double* G = g ? G2 : G1;
        G[(int64_t)a * c + b] = s;
        G[(int64_t)b * c + a] = s;
    }
}

// ---------------------------------------------------------------------------
// Cholesky QR factor of a small Gram matrix (one workgroup).
// ---------------------------------------------------------------------------
constexpr int CQ_TH = 256;
constexpr int CQ_MAX = 256;

__global__ void __launch_bounds__(CQ_TH)
k_cholqr_factor(int c, const double* __restrict__ G, int* __restrict__ mask, double tol,
                double* __restrict__ T64, float* __restrict__ T32, double* __restrict__ scr,
                int drop_on_fail, int require_all, int* status, int* counter) {
    __shared__ int idx[CQ_MAX];
    __shared__ double d[CQ_MAX];
    __shared__ int m_s, fail_s;
    const int tid = threadIdx.x;
    if (tid == 0) {
        int m = 0, missing = 0;
        for (int j = 0; j < c; ++j) {
            const double g = G[(int64_t)j * c + j];
            if (mask[j] && isfinite(g) && g > 0.0) {
                idx[m] = j;
                d[m] = sqrt(g);
                ++m;
            } else {
                if (mask[j]) missing = 1;
                mask[j] = 0;
            }
        }
        m_s = m;
        fail_s = (require_all && missing) ? 1 : 0;
    }
    __syncthreads();
    const int m = m_s;
    double* Gs = scr;                    // m x m equilibrated Gram
    double* R = scr + (int64_t)m * m;    // m x m upper factor
    double* Ri = R + (int64_t)m * m;     // m x m inverse
    for (int e = tid; e < m * m; e += CQ_TH) {
        const int a = e / m, b = e % m;
        Gs[e] = G[(int64_t)idx[a] * c + idx[b]] / (d[a] * d[b]);
        R[e] = 0.0;
        Ri[e] = 0.0;
    }
    __syncthreads();
    for (int j = 0; j < m && !fail_s; ++j) {
        if (tid == 0) {
            double s = Gs[(int64_t)j * m + j];
            for (int l = 0; l < j; ++l) s = fma(-R[(int64_t)l * m + j], R[(int64_t)l * m + j], s);
            if (!isfinite(s) || !(s > tol * Gs[(int64_t)j * m + j]) || !(s > 0.0)) fail_s = 1;
            else R[(int64_t)j * m + j] = sqrt(s);
        }
        __syncthreads();
        if (fail_s) break;
        const double rjj = R[(int64_t)j * m + j];
        for (int b = j + 1 + tid; b < m; b += CQ_TH) {
            double t = Gs[(int64_t)j * m + b];
            for (int l = 0; l < j; ++l) t = fma(-R[(int64_t)l * m + j], R[(int64_t)l * m + b], t);
            R[(int64_t)j * m + b] = t / rjj;
        }
        __syncthreads();
    }
    if (fail_s) {
        for (int e = tid; e < c * c; e += CQ_TH) {
            T64[e] = 0.0;
            T32[e] = 0.0f;
        }
        if (tid == 0) {
            if (drop_on_fail) {
                for (int j = 0; j < c; ++j) mask[j] = 0;
                atomicOr(status, DEV_P_DROPPED);
                if (counter) atomicAdd(counter, 1);
            } else {
                atomicOr(status, DEV_BREAKDOWN);
            }
        }
        return;
    }
    // R^-1 by back substitution, one column per thread
    for (int j = tid; j < m; j += CQ_TH) {
        Ri[(int64_t)j * m + j] = 1.0 / R[(int64_t)j * m + j];
        for (int a = j - 1; a >= 0; --a) {
            double s = 0.0;
            for (int l = a + 1; l <= j; ++l) s = fma(R[(int64_t)a * m + l], Ri[(int64_t)l * m + j], s);
            Ri[(int64_t)a * m + j] = -s / R[(int64_t)a * m + a];
        }
    }
    __syncthreads();
    for (int e = tid; e < c * c; e += CQ_TH) {
        T64[e] = 0.0;
        T32[e] = 0.0f;
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += CQ_TH) {
        const int a = e / m, b = e % m;
        const double v = Ri[e] / d[a];
        T64[(int64_t)idx[a] * c + idx[b]] = v;
        T32[(int64_t)idx[a] * c + idx[b]] = (float)v;
    }
}

// ---------------------------------------------------------------------------
// In-place V <- V T for an n x c row block (T upper triangular, c x c).
// ---------------------------------------------------------------------------
template <class T>
struct Prec;
template <>
struct Prec<double> {
    static __device__ inline double coef(const double* c64, const float*, int64_t i) { return c64[i]; }
};
template <>
struct Prec<float> {
    static __device__ inline float coef(const double*, const float* c32, int64_t i) { return c32[i]; }
};

template <class T>
__global__ void __launch_bounds__(256)
k_apply_right(int64_t n, int c, int ROWS, T* __restrict__ V, int64_t ldv, T* __restrict__ V2,
              int64_t ldv2, const double* __restrict__ T64, const float* __restrict__ T32) {
    extern __shared__ unsigned char smem_raw[];
    T* Vs = reinterpret_cast<T*>(smem_raw);
    const int64_t r0 = (int64_t)blockIdx.x * ROWS;
    const int rows = (int)min<int64_t>(ROWS, n - r0);
    for (int pass = 0; pass < (V2 ? 2 : 1); ++pass) {
        T* M = pass ? V2 : V;
        const int64_t ld = pass ? ldv2 : ldv;
        for (int e = threadIdx.x; e < rows * c; e += 256) {
            const int r = e / c, j = e % c;
            Vs[e] = M[(r0 + r) * ld + j];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < rows * c; e += 256) {
            const int r = e / c, j = e % c;
            T acc = T(0);
            for (int a = 0; a <= j; ++a)
                acc = fma(Vs[r * c + a], Prec<T>::coef(T64, T32, (int64_t)a * c + j), acc);
            M[(r0 + r) * ld + j] = acc;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Block update on S = [X W P] (row stride ld, blocks of kp columns):
//   P <- [W P] C_WP,  X <- X C_X + P.   Row-local, so it runs in place.
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256)
k_block_update(int64_t n, int kp, int ROWS, T* __restrict__ S, int64_t ld,
               const double* __restrict__ C64, const float* __restrict__ C32) {
    extern __shared__ unsigned char smem_raw[];
    T* Ss = reinterpret_cast<T*>(smem_raw);
    const int K3 = 3 * kp;
    const int64_t r0 = (int64_t)blockIdx.x * ROWS;
    const int rows = (int)min<int64_t>(ROWS, n - r0);
    for (int e = threadIdx.x; e < rows * K3; e += 256) {
        const int r = e / K3, j = e % K3;
        Ss[e] = S[(r0 + r) * ld + j];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows * kp; e += 256) {
        const int r = e / kp, j = e % kp;
        const T* s = Ss + r * K3;
        T accP = T(0), accX = T(0);
        for (int l = kp; l < K3; ++l) accP = fma(s[l], Prec<T>::coef(C64, C32, (int64_t)l * kp + j), accP);
        for (int l = 0; l < kp; ++l) accX = fma(s[l], Prec<T>::coef(C64, C32, (int64_t)l * kp + j), accX);
        S[(r0 + r) * ld + j] = accX + accP;
        S[(r0 + r) * ld + 2 * kp + j] = accP;
    }
}

// ---------------------------------------------------------------------------
// Residual R = LX - X diag(theta) written into the W block, with per-block
// FP64 partial sums of R^2 and X^2 per column.
// ---------------------------------------------------------------------------
constexpr int RES_ROWS = 256;

template <class T>
__global__ void __launch_bounds__(256)
k_residual(int64_t n, int kp, int k, T* __restrict__ S, const T* __restrict__ LS, int64_t ld,
           const double* __restrict__ theta, double* __restrict__ partial) {
    const int64_t r0 = (int64_t)blockIdx.x * RES_ROWS;
    const int64_t r1 = min<int64_t>(n, r0 + RES_ROWS);
    for (int j = threadIdx.x; j < kp; j += 256) {
        double rr = 0.0, xx = 0.0;
        if (j < k) {
            const T th = (T)theta[j];
            for (int64_t i = r0; i < r1; ++i) {
                const T x = S[i * ld + j];
                const T r = fma(-th, x, LS[i * ld + j]);
                S[i * ld + kp + j] = r;
                rr = fma((double)r, (double)r, rr);
                xx = fma((double)x, (double)x, xx);
            }
        } else {
            for (int64_t i = r0; i < r1; ++i) S[i * ld + kp + j] = T(0);
        }
        partial[((int64_t)blockIdx.x * 2 + 0) * kp + j] = rr;
        partial[((int64_t)blockIdx.x * 2 + 1) * kp + j] = xx;
    }
}

__global__ void __launch_bounds__(256)
k_residual_finalize(int nblocks, int kp, int k, const double* __restrict__ partial, double lock_tol,
                    double* __restrict__ relres, double* __restrict__ hist_row, int* __restrict__ wmask,
                    int* status, double* out_max, int* out_all_locked) {
    __shared__ double mx[256];
    __shared__ int locked_all[256];
    double my_max = 0.0;
    int my_all = 1;
    for (int j = threadIdx.x; j < kp; j += 256) {
        double rr = 0.0, xx = 0.0;
        for (int b = 0; b < nblocks; ++b) {
            rr += partial[((int64_t)b * 2 + 0) * kp + j];
            xx += partial[((int64_t)b * 2 + 1) * kp + j];
        }
        if (j < k) {
            const double rel = sqrt(rr) / (2.0 * sqrt(xx));
            if (!isfinite(rel)) atomicOr(status, DEV_NUMERIC);
            relres[j] = rel;
            if (hist_row) hist_row[j] = rel;
            const int active = rel > lock_tol;
            wmask[j] = active;
            my_all &= !active;
            my_max = fmax(my_max, rel);
        } else {
            relres[j] = 0.0;
            wmask[j] = 0;
        }
    }
    mx[threadIdx.x] = my_max;
    locked_all[threadIdx.x] = my_all;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        int a = 1;
        for (int t = 0; t < 256; ++t) {
            m = fmax(m, mx[t]);
            a &= locked_all[t];
        }
        *out_max = m;
        *out_all_locked = a;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
GramPlan gram_plan(int64_t n, int c) {
    GramPlan p;
    p.n = n;
    p.c = c;
    p.tiles = (int)ceil_div(c, GT);
    const int upper = p.tiles * (p.tiles + 1) / 2;
    // enough workgroups to fill 256 CUs several times, each chunk >= 512 rows
    int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(2048, upper), ceil_div(n, 512)));
    p.chunks = std::min(chunks, 256);
    return p;
}

size_t gram_partial_elems(const GramPlan& p, int nout) {
    return (size_t)p.chunks * nout * (size_t)p.c * p.c;
}

template <class T>
sc_status launch_gram(sc_ctx* ctx, const GramPlan& p, const T* A, int64_t lda, const T* B1,
                      int64_t ldb1, const T* B2, int64_t ldb2, double* partial, double* G1,
                      double* G2, int bf16) {
    (void)bf16;
    const int upper = p.tiles * (p.tiles + 1) / 2;
    const int64_t chunk_rows = ceil_div(p.n, p.chunks);
    dim3 grid(upper, p.chunks);
    using ACC = T;
    if (B2)
        hipLaunchKernelGGL((k_gram_partial<T, ACC, true>), grid, dim3(256), 0, ctx->stream, p.n,
                           p.c, chunk_rows, A, lda, B1, ldb1, B2, ldb2, partial, p.tiles);
    else
        hipLaunchKernelGGL((k_gram_partial<T, ACC, false>), grid, dim3(256), 0, ctx->stream, p.n,
                           p.c, chunk_rows, A, lda, B1, ldb1, B1, ldb1, partial, p.tiles);
    SC_CHECK_LAUNCH(ctx);
    const int64_t cc2 = (int64_t)p.c * p.c;
    hipLaunchKernelGGL(k_gram_reduce, dim3(ceil_div(cc2, 256)), dim3(256), 0, ctx->stream, p.c,
                       p.chunks, B2 ? 2 : 1, partial, G1, G2);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}

template sc_status launch_gram<double>(sc_ctx*, const GramPlan&, const double*, int64_t,
                                       const double*, int64_t, const double*, int64_t, double*,
                                       double*, double*, int);
template sc_status launch_gram<float>(sc_ctx*, const GramPlan&, const float*, int64_t,
                                      const float*, int64_t, const float*, int64_t, double*,
                                      double*, double*, int);

sc_status launch_cholqr_factor(sc_ctx* ctx, int c, const double* G, int* mask, double tol,
                               double* T64, float* T32, double* scratch, int drop_on_fail,
                               int* status, int* counter) {
    if (c > CQ_MAX) return sc_fail(ctx, SC_E_UNSUPPORTED, "cholqr: %d columns > %d", c, CQ_MAX);
    hipLaunchKernelGGL(k_cholqr_factor, dim3(1), dim3(CQ_TH), 0, ctx->stream, c, G, mask, tol, T64,
                       T32, scratch, drop_on_fail, drop_on_fail ? 0 : 1, status, counter);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}

template <class T>
sc_status launch_apply_right(sc_ctx* ctx, int64_t n, int c, T* V, int64_t ldv, T* V2, int64_t ldv2,
                             const double* T64, const float* T32) {
    const int ROWS = (int)std::max<int64_t>(1, std::min<int64_t>(64, 65536 / ((int64_t)c * sizeof(T))));
    const size_t lds = (size_t)ROWS * c * sizeof(T);
    hipLaunchKernelGGL((k_apply_right<T>), dim3(ceil_div(n, ROWS)), dim3(256), lds, ctx->stream, n,
                       c, ROWS, V, ldv, V2, ldv2, T64, T32);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}
template sc_status launch_apply_right<double>(sc_ctx*, int64_t, int, double*, int64_t, double*,
                                              int64_t, const double*, const float*);
template sc_status launch_apply_right<float>(sc_ctx*, int64_t, int, float*, int64_t, float*,
                                             int64_t, const double*, const float*);

template <class T>
sc_status launch_block_update(sc_ctx* ctx, int64_t n, int kp, T* S, int64_t ld, const double* C64,
                              const float* C32) {
    const int ROWS =
        (int)std::max<int64_t>(1, std::min<int64_t>(32, 65536 / (3 * (int64_t)kp * sizeof(T))));
    const size_t lds = (size_t)ROWS * 3 * kp * sizeof(T);
    hipLaunchKernelGGL((k_block_update<T>), dim3(ceil_div(n, ROWS)), dim3(256), lds, ctx->stream,
                       n, kp, ROWS, S, ld, C64, C32);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}
template sc_status launch_block_update<double>(sc_ctx*, int64_t, int, double*, int64_t,
                                               const double*, const float*);
template sc_status launch_block_update<float>(sc_ctx*, int64_t, int, float*, int64_t, const double*,
                                              const float*);

template <class T>
sc_status launch_residual(sc_ctx* ctx, int64_t n, int kp, int k, T* S, const T* LS, int64_t ld,
                          const double* theta, double* partial, int* nblocks_out) {
    const int nb = (int)ceil_div(n, RES_ROWS);
    hipLaunchKernelGGL((k_residual<T>), dim3(nb), dim3(256), 0, ctx->stream, n, kp, k, S, LS, ld,
                       theta, partial);
    SC_CHECK_LAUNCH(ctx);
    *nblocks_out = nb;
    return SC_OK;
}
template sc_status launch_residual<double>(sc_ctx*, int64_t, int, int, double*, const double*,
                                           int64_t, const double*, double*, int*);
template sc_status launch_residual<float>(sc_ctx*, int64_t, int, int, float*, const float*, int64_t,
                                          const double*, double*, int*);

sc_status launch_residual_finalize(sc_ctx* ctx, int nblocks, int kp, int k, const double* partial,
                                   double lock_tol, double* relres, double* hist_row, int* wmask,
                                   int* status, double* out_max, int* out_all_locked) {
    hipLaunchKernelGGL(k_residual_finalize, dim3(1), dim3(256), 0, ctx->stream, nblocks, kp, k,
                       partial, lock_tol, relres, hist_row, wmask, status, out_max,
                       out_all_locked);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}
