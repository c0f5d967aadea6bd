// Cluster labels by QR with column pivoting of the eigenvector block
// (Section II-A: the multi-way partition is read off the approximate
// eigenvectors by a pivoted QR, the method of Damle, Minden & Ying).
//
// With X the n x k block (row i = vertex i):
//   1. Businger-Golub pivoting over the rows of X: res_i = ||x_i||^2; step s
//      takes p_s = argmax res_i over the rows not chosen (ties: lowest i),
//      a_t = q_t . x_{p_s} (t < s), r = x_{p_s} - sum_t a_t q_t (fma over t in
//      order), q_s = r / ||r||, and every row's residual is downdated,
//      res_i = fma(-c, c, res_i) with c = q_s . x_i.
//   2. Q = the orthogonal polar factor of B' (B = the pivot rows):
//      B B' = W diag(l) W', Q = B' W diag(1/sqrt l) W'.
//   3. label_i = argmax_j |(X Q)_ij| (ties: lowest j).
// Every dot product is the ordered fma chain over the coordinates, so the
// pivots are those of the definition bit for bit.  Each pivot step is one
// small kernel (argmax of the previous pass's block maxima, the Gram-Schmidt
// vector in LDS) and one coalesced pass over a dimension-major copy of X
// (c, the downdate and the next block maxima).
#include <cmath>

#include "sc_internal.h"

namespace {

constexpr int CP_TH = 256;
constexpr int CP_MAXK = 256;     // one thread per coordinate in the pivot kernel
constexpr int CP_DC = 16;        // dimensions per staged chunk of the transposing pass
constexpr int CP_JB = 32;        // clusters per pass of the labelling kernel
// a chosen squared residual at or below this fraction of the first pivot's
// (1e-5 relative in norm, far above the downdates' rounding noise of about
// 1e-15) means the block has rank below k
constexpr double CP_RANK_TOL = 1e-10;

struct Best {
    double v;
    int64_t i;
};

// a before b: larger value, then lower index
__device__ __forceinline__ bool cp_better(double av, int64_t ai, double bv, int64_t bi) {
    return av > bv || (av == bv && ai < bi);
}

// block argmax of (v, i) over CP_TH threads; thread 0 gets the result
__device__ Best cp_block_best(double v, int64_t i) {
    __shared__ double sv[CP_TH];
    __shared__ int64_t si[CP_TH];
    const int t = threadIdx.x;
    sv[t] = v;
    si[t] = i;
    __syncthreads();
    for (int o = CP_TH / 2; o > 0; o >>= 1) {
        if (t < o && cp_better(sv[t + o], si[t + o], sv[t], si[t])) {
            sv[t] = sv[t + o];
            si[t] = si[t + o];
        }
        __syncthreads();
    }
    return Best{sv[0], si[0]};
}

// dimension-major copy of X, squared row norms and the block maxima for the
// first pivot; rows staged through LDS in chunks of CP_DC coordinates
template <class TX>
__global__ void __launch_bounds__(CP_TH)
k_cpqr_prep(int64_t n, int k, const TX* __restrict__ X, int64_t ldx, TX* __restrict__ Xt,
            double* __restrict__ res, double* __restrict__ pval, int64_t* __restrict__ pidx,
            int* status) {
    __shared__ TX xs[CP_DC][CP_TH + 1];
    const int64_t row0 = (int64_t)blockIdx.x * CP_TH;
    const int t = threadIdx.x;
    const bool live = row0 + t < n;
    double s = 0.0;
    bool bad = false;
    for (int d0 = 0; d0 < k; d0 += CP_DC) {
        const int nd = min(CP_DC, k - d0);
        for (int q = t; q < CP_TH * CP_DC; q += CP_TH) {        // row-major reads
            const int r = q / CP_DC, dd = q % CP_DC;
            const int64_t i = row0 + r;
            xs[dd][r] = (i < n && dd < nd) ? X[i * ldx + d0 + dd] : TX(0);
        }
        __syncthreads();
        for (int dd = 0; dd < nd; ++dd) {
            const double x = (double)xs[dd][t];
            bad |= !isfinite(x);
            s = fma(x, x, s);
        }
        for (int q = t; q < CP_TH * CP_DC; q += CP_TH) {        // dimension-major writes
            const int dd = q / CP_TH, r = q % CP_TH;
            if (dd < nd && row0 + r < n) Xt[(int64_t)(d0 + dd) * n + row0 + r] = xs[dd][r];
        }
        __syncthreads();
    }
    if (live) res[row0 + t] = s;
    if (bad && live) atomicOr(status, DEV_NUMERIC);
    const Best b = cp_block_best(live ? s : -INFINITY, live ? row0 + t : INT64_MAX);
    if (t == 0) {
        pval[blockIdx.x] = b.v;
        pidx[blockIdx.x] = b.i;
    }
}

// pivot s: argmax of the block maxima, then q_s by Gram-Schmidt against
// q_0 .. q_{s-1} in the order of the definition.  One workgroup.
template <class TX>
__global__ void __launch_bounds__(CP_TH)
k_cpqr_pivot(int64_t n, int k, int s, const TX* __restrict__ X, int64_t ldx,
             const double* __restrict__ pval, const int64_t* __restrict__ pidx, int nparts,
             double* __restrict__ res, double* __restrict__ q, int32_t* __restrict__ pivots,
             double* __restrict__ floor_res, int* status) {
    __shared__ double xp[CP_MAXK], a[CP_MAXK], r[CP_MAXK];
    __shared__ double nr_s;
    __shared__ int64_t p_s;
    const int t = threadIdx.x;
    double bv = -INFINITY;
    int64_t bi = INT64_MAX;
    for (int j = t; j < nparts; j += CP_TH)
        if (cp_better(pval[j], pidx[j], bv, bi)) {
            bv = pval[j];
            bi = pidx[j];
        }
    const Best b = cp_block_best(bv, bi);
    if (t == 0) {
        int64_t p = b.i;
        const double fl = s == 0 ? 0.0 : *floor_res;
        if (!(b.v > fl) || p < 0 || p >= n) {                // rank below k
            atomicOr(status, DEV_BREAKDOWN);
            p = 0;
        }
        if (s == 0) *floor_res = b.v * CP_RANK_TOL;
        p_s = p;
        pivots[s] = (int32_t)p;
        res[p] = -INFINITY;                                 // never chosen again
    }
    __syncthreads();
    const int64_t p = p_s;
    if (t < k) xp[t] = (double)X[p * ldx + t];
    __syncthreads();
    if (t < s) {                                            // a_t = q_t . x_p
        const double* qt = q + (int64_t)t * k;
        double dot = 0.0;
        for (int d = 0; d < k; ++d) dot = fma(qt[d], xp[d], dot);
        a[t] = dot;
    }
    __syncthreads();
    if (t < k) {                                            // r_d = x_p,d - sum_t a_t q_t,d
        double v = xp[t];
        for (int u = 0; u < s; ++u) v = fma(-a[u], q[(int64_t)u * k + t], v);
        r[t] = v;
    }
    __syncthreads();
    if (t == 0) {
        double nr2 = 0.0;
        for (int d = 0; d < k; ++d) nr2 = fma(r[d], r[d], nr2);
        const double nr = sqrt(nr2);
        if (!(nr > 0.0)) atomicOr(status, DEV_BREAKDOWN);
        nr_s = nr > 0.0 ? nr : 1.0;
    }
    __syncthreads();
    if (t < k) q[(int64_t)s * k + t] = r[t] / nr_s;
}

// one pass per pivot: c = q_s . x_i, res_i = fma(-c, c, res_i), block maxima
template <class TT>
__global__ void __launch_bounds__(CP_TH)
k_cpqr_pass(int64_t n, int k, int s, const TT* __restrict__ Xt, const double* __restrict__ q,
            double* __restrict__ res, double* __restrict__ pval, int64_t* __restrict__ pidx) {
    __shared__ double qs[CP_MAXK];
    const int t = threadIdx.x;
    if (t < k) qs[t] = q[(int64_t)s * k + t];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * CP_TH + t;
    const bool live = i < n;
    const int64_t ii = live ? i : n - 1;
    double c = 0.0;
    constexpr int DU = 8;
    int d = 0;
    for (; d + DU <= k; d += DU) {
        TT x[DU];
#pragma unroll
        for (int u = 0; u < DU; ++u) x[u] = Xt[(int64_t)(d + u) * n + ii];
#pragma unroll
        for (int u = 0; u < DU; ++u) c = fma(qs[d + u], (double)x[u], c);
    }
    for (; d < k; ++d) c = fma(qs[d], (double)Xt[(int64_t)d * n + ii], c);
    double v = -INFINITY;
    if (live) {
        v = fma(-c, c, res[i]);
        res[i] = v;
    }
    const Best b = cp_block_best(v, live ? i : INT64_MAX);
    if (t == 0) {
        pval[blockIdx.x] = b.v;
        pidx[blockIdx.x] = b.i;
    }
}

// G = B B' with B the pivot rows
template <class TX>
__global__ void k_cpqr_gram(int k, const TX* __restrict__ X, int64_t ldx,
                            const int32_t* __restrict__ piv, double* __restrict__ G) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k * k) return;
    const int u = e / k, v = e % k;
    const TX* bu = X + (int64_t)piv[u] * ldx;
    const TX* bv = X + (int64_t)piv[v] * ldx;
    double t = 0.0;
    for (int d = 0; d < k; ++d) t = fma((double)bu[d], (double)bv[d], t);
    G[e] = t;
}

// M = W diag(1/sqrt l) W'
__global__ void k_cpqr_isqrt(int k, const double* __restrict__ W, const double* __restrict__ l,
                             double* __restrict__ M, int* status) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k * k) return;
    const int u = e / k, v = e % k;
    double t = 0.0;
    bool bad = false;
    for (int j = 0; j < k; ++j) {
        const double lj = l[j];
        bad |= !(lj > 0.0);
        const double f = 1.0 / sqrt(lj > 0.0 ? lj : 1.0);
        t = fma(W[(int64_t)u * k + j] * f, W[(int64_t)v * k + j], t);
    }
    M[e] = t;
    if (bad && e == 0) atomicOr(status, DEV_BREAKDOWN);
}

// Q = B' M, written to Q (k x k) and to a copy Qp with kpad columns (zeros
// beyond k) for the predicate-free labelling kernel
template <class TX>
__global__ void k_cpqr_polar(int k, int kpad, const TX* __restrict__ X, int64_t ldx,
                             const int32_t* __restrict__ piv, const double* __restrict__ M,
                             double* __restrict__ Q, double* __restrict__ Qp) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k * kpad) return;
    const int d = e / kpad, j = e % kpad;
    double t = 0.0;
    if (j < k) {
        for (int u = 0; u < k; ++u) t = fma((double)X[(int64_t)piv[u] * ldx + d], M[(int64_t)u * k + j], t);
        Q[(int64_t)d * k + j] = t;
    }
    Qp[(int64_t)d * kpad + j] = t;
}

// label_i = argmax_j |sum_d x_id Q_dj|; CP_JB clusters per pass over the row,
// Q entries as wave-uniform loads
template <class TT>
__global__ void __launch_bounds__(CP_TH)
k_cpqr_labels(int64_t n, int k, int kpad, const TT* __restrict__ Xt, const double* __restrict__ Qp,
              int32_t* __restrict__ labels) {
    const int64_t i = (int64_t)blockIdx.x * CP_TH + threadIdx.x;
    if (i >= n) return;
    double bv = -1.0;
    int bj = 0;
    for (int j0 = 0; j0 < kpad; j0 += CP_JB) {
        double acc[CP_JB];
#pragma unroll
        for (int u = 0; u < CP_JB; ++u) acc[u] = 0.0;
        for (int d = 0; d < k; ++d) {
            const double x = (double)Xt[(int64_t)d * n + i];
            const double* qr = Qp + (int64_t)d * kpad + j0;
#pragma unroll
            for (int u = 0; u < CP_JB; ++u) acc[u] = fma(x, qr[u], acc[u]);
        }
#pragma unroll
        for (int u = 0; u < CP_JB; ++u) {
            const double a = fabs(acc[u]);
            if (j0 + u < k && a > bv) {
                bv = a;
                bj = j0 + u;
            }
        }
    }
    labels[i] = bj;
}

// number of clusters from the gap in the ascending Ritz values (one thread):
// the first increment g_j (j >= 1) above 1e-8 of the spread theta_{k-1} -
// theta_0 (the rounding noise of equal eigenvalues) and above sig times the
// mean of the increments before it, else the largest increment; ratio = that
// increment over the median increment
__global__ void k_eigengap(int k, const double* __restrict__ theta, double sig,
                           int* __restrict__ count, double* __restrict__ ratio) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (k <= 1) {
        *count = k;
        *ratio = 0.0;
        return;
    }
    double g[CP_MAXK];
    for (int j = 0; j + 1 < k; ++j) g[j] = theta[j + 1] - theta[j];
    int jj = -1;
    const double tiny = 1e-8 * (theta[k - 1] - theta[0]);
    double sum = g[0];
    for (int j = 1; j + 1 < k; ++j) {
        if (g[j] > tiny && g[j] > sig * (sum / (double)j)) {
            jj = j;
            break;
        }
        sum += g[j];
    }
    if (jj < 0) {
        double gmax = -INFINITY;
        for (int j = 0; j + 1 < k; ++j)
            if (g[j] > gmax) {
                gmax = g[j];
                jj = j;
            }
    }
    const double gap = g[jj];
    for (int a = 1; a < k - 1; ++a) {            // insertion sort for the median
        const double v = g[a];
        int b = a - 1;
        while (b >= 0 && g[b] > v) {
            g[b + 1] = g[b];
            --b;
        }
        g[b + 1] = v;
    }
    const int m = k - 1;
    const double med = m % 2 ? g[m / 2] : 0.5 * (g[m / 2 - 1] + g[m / 2]);
    *count = jj + 1;
    *ratio = med > 0.0 ? gap / med : INFINITY;
}

int cp_kpad(int k) { return (int)ceil_div(k, CP_JB) * CP_JB; }

struct CpWs {
    void* Xt;
    double *res, *pval, *q, *G, *W, *l, *M, *Qp, *eig, *floor_res;
    int64_t* pidx;
    int* status;
};

size_t carve_cp(Carver& c, int64_t n, int k, int es, CpWs& w) {
    const int64_t nparts = ceil_div(n, CP_TH);
    w.Xt = c.take<char>((size_t)n * k * es);
    w.res = c.take<double>((size_t)n);
    w.pval = c.take<double>((size_t)nparts);
    w.pidx = c.take<int64_t>((size_t)nparts);
    w.q = c.take<double>((size_t)k * k);
    w.G = c.take<double>((size_t)k * k);
    w.W = c.take<double>((size_t)k * k);
    w.l = c.take<double>((size_t)k);
    w.M = c.take<double>((size_t)k * k);
    w.Qp = c.take<double>((size_t)k * cp_kpad(k));
    w.eig = c.take<double>(symeig_scratch_elems(k, k));
    w.floor_res = c.take<double>(1);
    w.status = c.take<int>(1);
    return c.size();
}

sc_status cp_validate(sc_ctx* ctx, int64_t n, int k, int64_t ldx) {
    if (n <= 0 || k <= 0 || k > CP_MAXK || k > n || ldx < k)
        return sc_fail(ctx, SC_E_INVAL, "cpqr: need 0 < k <= min(n, %d) and ldx >= k", CP_MAXK);
    if (n >= (int64_t(1) << 31)) return sc_fail(ctx, SC_E_UNSUPPORTED, "cpqr: n >= 2^31");
    return SC_OK;
}

template <class TX>
sc_status cp_run(sc_ctx* ctx, int64_t n, int k, const TX* X, int64_t ldx, int32_t* pivots,
                 int32_t* labels, double* Q, const CpWs& w) {
    hipStream_t st = ctx->stream;
    const int nparts = (int)ceil_div(n, CP_TH);
    TX* Xt = static_cast<TX*>(w.Xt);
    SC_CHECK_HIP(ctx, hipMemsetAsync(w.status, 0, sizeof(int), st));
    hipLaunchKernelGGL((k_cpqr_prep<TX>), dim3(nparts), dim3(CP_TH), 0, st, n, k, X, ldx, Xt, w.res,
                       w.pval, w.pidx, w.status);
    SC_CHECK_LAUNCH(ctx);
    for (int s = 0; s < k; ++s) {
        hipLaunchKernelGGL((k_cpqr_pivot<TX>), dim3(1), dim3(CP_TH), 0, st, n, k, s, X, ldx, w.pval,
                           w.pidx, nparts, w.res, w.q, pivots, w.floor_res, w.status);
        if (s + 1 < k)
            hipLaunchKernelGGL((k_cpqr_pass<TX>), dim3(nparts), dim3(CP_TH), 0, st, n, k, s, Xt, w.q,
                               w.res, w.pval, w.pidx);
    }
    SC_CHECK_LAUNCH(ctx);
    // the eigensolver below only sees a finite, full-rank pivot block
    int h = 0;
    SC_CHECK_HIP(ctx, hipMemcpyAsync(&h, w.status, sizeof h, hipMemcpyDeviceToHost, st));
    SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
    if (h & DEV_NUMERIC) return sc_fail(ctx, SC_E_NUMERIC, "cpqr: NaN or Inf in X");
    if (h & DEV_BREAKDOWN)
        return sc_fail(ctx, SC_E_BREAKDOWN, "cpqr: the block has rank below k (pivoted QR breakdown)");
    const unsigned gk = (unsigned)ceil_div((int64_t)k * k, CP_TH);
    hipLaunchKernelGGL((k_cpqr_gram<TX>), dim3(gk), dim3(CP_TH), 0, st, k, X, ldx, pivots, w.G);
    SC_CHECK_LAUNCH(ctx);
    SC_TRY(launch_symeig(ctx, k, k, w.G, w.l, w.W, w.eig));
    hipLaunchKernelGGL(k_cpqr_isqrt, dim3(gk), dim3(CP_TH), 0, st, k, w.W, w.l, w.M, w.status);
    const int kpad = cp_kpad(k);
    hipLaunchKernelGGL((k_cpqr_polar<TX>), dim3((unsigned)ceil_div((int64_t)k * kpad, CP_TH)),
                       dim3(CP_TH), 0, st, k, kpad, X, ldx, pivots, w.M, Q, w.Qp);
    hipLaunchKernelGGL((k_cpqr_labels<TX>), dim3(nparts), dim3(CP_TH), 0, st, n, k, kpad, Xt, w.Qp,
                       labels);
    SC_CHECK_LAUNCH(ctx);
    SC_CHECK_HIP(ctx, hipMemcpyAsync(&h, w.status, sizeof h, hipMemcpyDeviceToHost, st));
    SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
    if (h & DEV_NUMERIC) return sc_fail(ctx, SC_E_NUMERIC, "cpqr: NaN or Inf in X");
    if (h & DEV_BREAKDOWN)
        return sc_fail(ctx, SC_E_BREAKDOWN, "cpqr: the block has rank below k (pivoted QR breakdown)");
    return SC_OK;
}

}  // namespace

extern "C" sc_status sc_cpqr_workspace(sc_ctx* ctx, int64_t n, int k, int x_fp32, size_t* bytes) {
    if (!ctx || !bytes) return SC_E_INVAL;
    SC_TRY(cp_validate(ctx, n, k, k));
    Carver c(nullptr);
    CpWs w;
    *bytes = carve_cp(c, n, k, x_fp32 ? 4 : 8, w);
    return SC_OK;
}

extern "C" sc_status sc_cpqr_labels(sc_ctx* ctx, int64_t n, int k, const void* X, int64_t ldx,
                                    int x_fp32, int32_t* pivots, int32_t* labels, double* Q,
                                    void* ws, size_t ws_bytes) {
    if (!ctx) return SC_E_INVAL;
    SC_TRY(cp_validate(ctx, n, k, ldx));
    if (!X || !pivots || !labels || !Q || !ws)
        return sc_fail(ctx, SC_E_INVAL, "cpqr: null pointer argument");
    Carver c(ws);
    CpWs w;
    const size_t need = carve_cp(c, n, k, x_fp32 ? 4 : 8, w);
    if (ws_bytes < need) return sc_fail(ctx, SC_E_NOMEM, "cpqr: workspace %zu < %zu", ws_bytes, need);
    SC_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    ProfScope ps(ctx, SC_KIND_KMEANS);
    if (x_fp32)
        return cp_run<float>(ctx, n, k, static_cast<const float*>(X), ldx, pivots, labels, Q, w);
    return cp_run<double>(ctx, n, k, static_cast<const double*>(X), ldx, pivots, labels, Q, w);
}

extern "C" sc_status sc_eigengap(sc_ctx* ctx, int k, const double* theta, double sig, int* count,
                                 double* ratio) {
    if (!ctx) return SC_E_INVAL;
    if (k <= 0 || k > CP_MAXK || !(sig > 0.0))
        return sc_fail(ctx, SC_E_INVAL, "eigengap: need 0 < k <= %d and sig > 0", CP_MAXK);
    if (!theta || !count || !ratio) return sc_fail(ctx, SC_E_INVAL, "eigengap: null pointer argument");
    SC_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_eigengap, dim3(1), dim3(64), 0, ctx->stream, k, theta, sig, count, ratio);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}
