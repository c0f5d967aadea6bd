// k-means labelling of the row-normalised eigenvectors (Section II-A: the
// clusters are read off the approximate eigenvectors; k-means++ is the
// classic labelling the paper refers to).  All restarts run together.
//
// Exactness rules, so that labels do not depend on the launch shape:
//   - a squared distance is accumulated with fma in dimension order by one
//     thread;
//   - k-means++ draws use integer weights floor(D2 * 2^s) and an exact
//     integer prefix sum;
//   - a centroid is the sum of its members in ascending vertex order (a
//     stable radix sort by label gives the member lists), divided by the count;
//   - the restart with the least integer inertia wins (ties: lowest restart).
#include <cmath>
#include <cstring>
#include <vector>

#include "sc_internal.h"

namespace {

constexpr int TH = 256;

__device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

template <class TX>
__global__ void k_rownorm(int64_t n, int dim, const TX* __restrict__ X, int64_t ldx,
                          int normalize, double* __restrict__ Y, double* __restrict__ Yt,
                          unsigned long long* m2bits, int* status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const TX* x = X + i * ldx;
    double s = 0.0;
    bool bad = false;
    for (int d = 0; d < dim; ++d) {
        const double xd = (double)x[d];
        bad |= !isfinite(xd);
        s = fma(xd, xd, s);
    }
    if (bad) atomicOr(status, DEV_NUMERIC);
    const double nrm = sqrt(s);
    double s2 = 0.0;
    for (int d = 0; d < dim; ++d) {
        double y = (double)x[d];
        if (normalize) y = nrm > 0.0 ? y / nrm : 0.0;
        Y[i * dim + d] = y;
        Yt[(int64_t)d * n + i] = y;
        s2 = fma(y, y, s2);
    }
    // non-negative doubles order like their bit patterns
    atomicMax(m2bits, (unsigned long long)__double_as_longlong(s2));
}

__device__ inline double sqdist_t(int dim, int64_t n, const double* __restrict__ Yt, int64_t i,
                                  const double* __restrict__ c) {
    double acc = 0.0;
    for (int d = 0; d < dim; ++d) {
        const double diff = Yt[(int64_t)d * n + i] - c[d];
        acc = fma(diff, diff, acc);
    }
    return acc;
}

// centre j of every restart r from a chosen row (grid: R blocks)
__global__ void k_seed_pick(int64_t n, int dim, int K, int j, const double* __restrict__ Y,
                            const uint64_t* __restrict__ draws, const uint64_t* __restrict__ pref,
                            double* __restrict__ C) {
    __shared__ int64_t pick;
    const int r = blockIdx.x;
    if (threadIdx.x == 0) {
        const uint64_t u = draws[(int64_t)r * K + j];
        if (j == 0) {
            pick = (int64_t)mulhi64(u, (uint64_t)n);
        } else {
            const uint64_t* pr = pref + (int64_t)r * n;
            const uint64_t T = pr[n - 1];
            if (T == 0) {
                pick = (int64_t)mulhi64(u, (uint64_t)n);
            } else {
                const uint64_t t = mulhi64(u, T);
                int64_t lo = 0, hi = n - 1;          // first i with prefix_i > t
                while (lo < hi) {
                    const int64_t mid = lo + (hi - lo) / 2;
                    if (pr[mid] > t) hi = mid;
                    else lo = mid + 1;
                }
                pick = lo;
            }
        }
    }
    __syncthreads();
    double* c = C + ((int64_t)r * K + j) * dim;
    for (int d = threadIdx.x; d < dim; d += blockDim.x) c[d] = Y[pick * dim + d];
}

// D2 <- dist(y_i, c_j) (j == 0) or min(D2, dist(y_i, c_j)); then integer weights
__global__ void k_seed_d2(int64_t n, int dim, int K, int j, int R, const double* __restrict__ Yt,
                          const double* __restrict__ C, double* __restrict__ D2,
                          uint64_t* __restrict__ wq, int shift) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * R) return;
    const int r = (int)(e / n);
    const int64_t i = e % n;
    const double dd = sqdist_t(dim, n, Yt, i, C + ((int64_t)r * K + j) * dim);
    double v = D2[e];
    if (j == 0 || dd < v) v = dd;
    D2[e] = v;
    wq[e] = (uint64_t)floor(ldexp(v, shift));
}

// nearest centroid (ties to the lowest index) for every (restart, point)
__global__ void k_assign(int64_t n, int dim, int K, int R, const double* __restrict__ Yt,
                         const double* __restrict__ C, const int* __restrict__ active,
                         const int32_t* __restrict__ old_lab, int32_t* __restrict__ lab,
                         double* __restrict__ D2, int* __restrict__ changed, int count_changes) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * R) return;
    const int r = (int)(e / n);
    if (!active[r]) return;
    const int64_t i = e % n;
    const double* Cr = C + (int64_t)r * K * dim;
    double best = 0.0;
    int bj = 0;
    constexpr int JB = 8;
    for (int j0 = 0; j0 < K; j0 += JB) {
        double acc[JB];
#pragma unroll
        for (int u = 0; u < JB; ++u) acc[u] = 0.0;
        for (int d = 0; d < dim; ++d) {
            const double y = Yt[(int64_t)d * n + i];
#pragma unroll
            for (int u = 0; u < JB; ++u) {
                if (j0 + u < K) {
                    const double diff = y - Cr[(int64_t)(j0 + u) * dim + d];
                    acc[u] = fma(diff, diff, acc[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < JB; ++u) {
            const int j = j0 + u;
            if (j < K && (j == 0 || acc[u] < best)) {
                best = acc[u];
                bj = j;
            }
        }
    }
    lab[e] = bj;
    D2[e] = best;
    if (count_changes && old_lab[e] != bj) atomicAdd(&changed[r], 1);
}

__global__ void k_label_keys(int64_t n, int K, int R, const int32_t* __restrict__ lab,
                             const int* __restrict__ active, uint64_t* __restrict__ keys,
                             uint32_t* __restrict__ vals, int* __restrict__ counts) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * R) return;
    const int r = (int)(e / n);
    const int64_t key = (int64_t)r * K + lab[e];
    keys[e] = (uint64_t)key;
    vals[e] = (uint32_t)(e % n);
    (void)active;
    atomicAdd(&counts[key], 1);   // every restart: offsets index the whole sorted list
}

__global__ void k_counts_scan(int total, const int* __restrict__ counts, int64_t* __restrict__ off) {
    // one thread: total = R*K is small
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t s = 0;
        for (int q = 0; q < total; ++q) {
            off[q] = s;
            s += counts[q];
        }
        off[total] = s;
    }
}

// centroid (r, j), dimension d: members in ascending vertex order
__global__ void k_centroids(int dim, int K, int R, const double* __restrict__ Y,
                            const uint32_t* __restrict__ members, const int* __restrict__ counts,
                            const int64_t* __restrict__ off, const int* __restrict__ active,
                            int64_t n, double* __restrict__ C) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)R * K * dim) return;
    const int d = (int)(e % dim);
    const int64_t rj = e / dim;
    const int r = (int)(rj / K);
    if (!active[r]) return;
    const int cnt = counts[rj];
    if (cnt == 0) return;
    // the sorted list holds all restarts back to back
    const uint32_t* mem = members + off[rj];
    double s = 0.0;
    for (int p = 0; p < cnt; ++p) s += Y[(int64_t)mem[p] * dim + d];
    C[e] = s / (double)cnt;
}

__global__ void k_inertia(int64_t n, int R, const double* __restrict__ D2, int shift,
                          unsigned long long* __restrict__ q) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * R) return;
    const int r = (int)(e / n);
    atomicAdd(&q[r], (unsigned long long)floor(ldexp(D2[e], shift)));
}

// FP64 inertia of restart r: fixed-shape tree (block sums in order)
__global__ void k_sum_rows(int64_t n, const double* __restrict__ D2, double* __restrict__ part) {
    __shared__ double sm[TH];
    const int64_t base = (int64_t)blockIdx.x * TH * 16;
    double s = 0.0;
    for (int u = 0; u < 16; ++u) {
        const int64_t i = base + (int64_t)u * TH + threadIdx.x;
        if (i < n) s += D2[i];
    }
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int o = TH / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void k_sum_final(int nb, const double* __restrict__ part, double* out) {
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[b];
        *out = s;
    }
}

__global__ void k_zero_i32(int* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

struct KmWs {
    double *Y, *Yt, *D2, *C, *part, *inertia;
    uint64_t *wq, *scan_tmp, *keys, *keys_alt, *radix_tmp;
    uint32_t *vals, *vals_alt;
    int32_t *lab, *lab2;
    int *changed, *active, *counts, *status;
    int64_t* off;
    unsigned long long *m2, *q;
};

size_t carve_km(Carver& c, int64_t n, int dim, int K, int R, KmWs& w) {
    const int64_t nr = n * R;
    w.Y = c.take<double>((size_t)n * dim);
    w.Yt = c.take<double>((size_t)n * dim);
    w.D2 = c.take<double>(nr);
    w.C = c.take<double>((size_t)R * K * dim);
    w.part = c.take<double>(ceil_div(n, TH * 16) + 1);
    w.inertia = c.take<double>(1);
    w.wq = c.take<uint64_t>(nr);
    w.scan_tmp = c.take<uint64_t>(scan_u64_batched_tmp_elems(n, R));
    w.keys = c.take<uint64_t>(nr);
    w.keys_alt = c.take<uint64_t>(nr);
    w.vals = c.take<uint32_t>(nr);
    w.vals_alt = c.take<uint32_t>(nr);
    w.radix_tmp = c.take<uint64_t>(radix_tmp_elems(nr));
    w.lab = c.take<int32_t>(nr);
    w.lab2 = c.take<int32_t>(nr);
    w.changed = c.take<int>(R);
    w.active = c.take<int>(R);
    w.counts = c.take<int>((size_t)R * K);
    w.status = c.take<int>(1);
    w.off = c.take<int64_t>((size_t)R * K + 1);
    w.m2 = c.take<unsigned long long>(1);
    w.q = c.take<unsigned long long>(R);
    return c.size();
}

sc_status km_validate(sc_ctx* ctx, int64_t n, int dim, const sc_kmeans_opts* o) {
    if (!o) return sc_fail(ctx, SC_E_INVAL, "kmeans: opts is NULL");
    if (n <= 0 || dim <= 0) return sc_fail(ctx, SC_E_INVAL, "kmeans: need n > 0 and dim > 0");
    if (n >= (int64_t(1) << 32)) return sc_fail(ctx, SC_E_UNSUPPORTED, "kmeans: n >= 2^32");
    if (o->n_clusters < 1 || o->n_clusters > n || o->n_clusters > 1024)
        return sc_fail(ctx, SC_E_INVAL, "kmeans: need 1 <= K <= min(n, 1024)");
    if (o->restarts < 1 || o->max_iter < 0)
        return sc_fail(ctx, SC_E_INVAL, "kmeans: need restarts >= 1 and max_iter >= 0");
    return SC_OK;
}

}  // namespace

extern "C" sc_status sc_kmeans_workspace(sc_ctx* ctx, int64_t n, int dim,
                                         const sc_kmeans_opts* opts, size_t* bytes) {
    if (!ctx || !bytes) return SC_E_INVAL;
    SC_TRY(km_validate(ctx, n, dim, opts));
    Carver c(nullptr);
    KmWs w;
    *bytes = carve_km(c, n, dim, opts->n_clusters, opts->restarts, w);
    return SC_OK;
}

extern "C" sc_status sc_kmeans_assign(sc_ctx* ctx, int64_t n, int dim, const void* X,
                                      int64_t ldx, const sc_kmeans_opts* opts,
                                      const uint64_t* draws, const double* init_centroids,
                                      int32_t* labels, double* centroids, double* inertia,
                                      uint64_t* inertia_q, int* best_restart, void* ws,
                                      size_t ws_bytes) {
    if (!ctx) return SC_E_INVAL;
    SC_TRY(km_validate(ctx, n, dim, opts));
    if (ldx < dim) return sc_fail(ctx, SC_E_INVAL, "kmeans: need ldx >= dim");
    if (!X || !labels || !centroids || !ws || (!init_centroids && !draws))
        return sc_fail(ctx, SC_E_INVAL, "kmeans: null pointer argument");
    if (init_centroids && opts->restarts != 1)
        return sc_fail(ctx, SC_E_INVAL, "kmeans: init_centroids needs restarts == 1");
    const int K = opts->n_clusters, R = opts->restarts;
    Carver c(ws);
    KmWs w;
    const size_t need = carve_km(c, n, dim, K, R, w);
    if (ws_bytes < need) return sc_fail(ctx, SC_E_NOMEM, "kmeans: workspace %zu < %zu", ws_bytes, need);
    SC_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int64_t nr = n * R;
    const dim3 gnr(ceil_div(nr, TH));

    SC_CHECK_HIP(ctx, hipMemsetAsync(w.m2, 0, sizeof(unsigned long long), st));
    SC_CHECK_HIP(ctx, hipMemsetAsync(w.status, 0, sizeof(int), st));
    ProfScope ps(ctx, SC_KIND_KMEANS);
    if (opts->x_fp32)
        hipLaunchKernelGGL((k_rownorm<float>), dim3(ceil_div(n, TH)), dim3(TH), 0, st, n, dim,
                           static_cast<const float*>(X), ldx, opts->normalize_rows, w.Y, w.Yt, w.m2,
                           w.status);
    else
        hipLaunchKernelGGL((k_rownorm<double>), dim3(ceil_div(n, TH)), dim3(TH), 0, st, n, dim,
                           static_cast<const double*>(X), ldx, opts->normalize_rows, w.Y, w.Yt,
                           w.m2, w.status);
    SC_CHECK_LAUNCH(ctx);
    char* h = static_cast<char*>(ctx->stage);
    SC_CHECK_HIP(ctx, hipMemcpyAsync(h, w.m2, 8, hipMemcpyDeviceToHost, st));
    SC_CHECK_HIP(ctx, hipMemcpyAsync(h + 8, w.status, 4, hipMemcpyDeviceToHost, st));
    SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
    int stv;
    memcpy(&stv, h + 8, 4);
    if (stv & DEV_NUMERIC) return sc_fail(ctx, SC_E_NUMERIC, "kmeans: NaN or Inf in X");
    double m2;
    memcpy(&m2, h, 8);
    int e = 0;
    (void)std::frexp(4.0 * m2, &e);
    if (m2 == 0.0) e = 0;
    const int shift = 61 - ceil_log2_u64((uint64_t)n) - e;

    // all restarts active
    std::vector<int> act_h(R, 1);
    SC_CHECK_HIP(ctx, hipMemcpyAsync(w.active, act_h.data(), R * sizeof(int), hipMemcpyHostToDevice, st));
    if (init_centroids) {
        SC_CHECK_HIP(ctx, hipMemcpyAsync(w.C, init_centroids, (size_t)K * dim * sizeof(double),
                                         hipMemcpyDeviceToDevice, st));
    } else {
        for (int j = 0; j < K; ++j) {
            hipLaunchKernelGGL(k_seed_pick, dim3(R), dim3(TH), 0, st, n, dim, K, j, w.Y, draws,
                               w.wq, w.C);
            SC_CHECK_LAUNCH(ctx);
            if (j + 1 < K) {
                hipLaunchKernelGGL(k_seed_d2, gnr, dim3(TH), 0, st, n, dim, K, j, R, w.Yt, w.C, w.D2,
                                   w.wq, shift);
                SC_CHECK_LAUNCH(ctx);
                SC_TRY(scan_u64_batched(ctx, w.wq, w.wq, n, R, w.scan_tmp));
            }
        }
    }
    // Lloyd
    hipLaunchKernelGGL(k_assign, gnr, dim3(TH), 0, st, n, dim, K, R, w.Yt, w.C, w.active, w.lab,
                       w.lab, w.D2, w.changed, 0);
    SC_CHECK_LAUNCH(ctx);
    const int bits = ceil_log2_u64((uint64_t)R * K);
    int32_t* cur = w.lab;
    int32_t* nxt = w.lab2;
    int n_active = R;
    for (int it = 1; it <= opts->max_iter && n_active > 0; ++it) {
        hipLaunchKernelGGL(k_zero_i32, dim3(ceil_div((int64_t)R * K, TH)), dim3(TH), 0, st, w.counts,
                           (int64_t)R * K);
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(TH), 0, st, w.changed, (int64_t)R);
        hipLaunchKernelGGL(k_label_keys, gnr, dim3(TH), 0, st, n, K, R, cur, w.active, w.keys,
                           w.vals, w.counts);
        SC_CHECK_LAUNCH(ctx);
        SC_TRY(radix_sort_pairs(ctx, w.keys, w.vals, w.keys_alt, w.vals_alt, nr, bits, w.radix_tmp));
        hipLaunchKernelGGL(k_counts_scan, dim3(1), dim3(64), 0, st, R * K, w.counts, w.off);
        hipLaunchKernelGGL(k_centroids, dim3(ceil_div((int64_t)R * K * dim, TH)), dim3(TH), 0, st,
                           dim, K, R, w.Y, w.vals, w.counts, w.off, w.active, n, w.C);
        hipLaunchKernelGGL(k_assign, gnr, dim3(TH), 0, st, n, dim, K, R, w.Yt, w.C, w.active, cur,
                           nxt, w.D2, w.changed, 1);
        SC_CHECK_LAUNCH(ctx);
        // inactive restarts keep their labels in `cur`; carry them into `nxt`
        std::vector<int> ch(R);
        SC_CHECK_HIP(ctx, hipMemcpyAsync(ch.data(), w.changed, R * sizeof(int), hipMemcpyDeviceToHost, st));
        SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
        for (int r = 0; r < R; ++r) {
            if (!act_h[r]) {
                SC_CHECK_HIP(ctx, hipMemcpyAsync(nxt + (int64_t)r * n, cur + (int64_t)r * n,
                                                 n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
            } else if (ch[r] == 0) {
                act_h[r] = 0;
                --n_active;
            }
        }
        std::swap(cur, nxt);
        SC_CHECK_HIP(ctx, hipMemcpyAsync(w.active, act_h.data(), R * sizeof(int),
                                         hipMemcpyHostToDevice, st));
        SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
    }
    // choose the restart
    SC_CHECK_HIP(ctx, hipMemsetAsync(w.q, 0, R * sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_inertia, gnr, dim3(TH), 0, st, n, R, w.D2, shift, w.q);
    SC_CHECK_LAUNCH(ctx);
    std::vector<unsigned long long> qh(R);
    SC_CHECK_HIP(ctx, hipMemcpyAsync(qh.data(), w.q, R * sizeof(unsigned long long),
                                     hipMemcpyDeviceToHost, st));
    SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
    int best = 0;
    for (int r = 1; r < R; ++r)
        if (qh[r] < qh[best]) best = r;
    SC_CHECK_HIP(ctx, hipMemcpyAsync(labels, cur + (int64_t)best * n, n * sizeof(int32_t),
                                     hipMemcpyDeviceToDevice, st));
    SC_CHECK_HIP(ctx, hipMemcpyAsync(centroids, w.C + (int64_t)best * K * dim,
                                     (size_t)K * dim * sizeof(double), hipMemcpyDeviceToDevice, st));
    const int nb = (int)ceil_div(n, TH * 16);
    hipLaunchKernelGGL(k_sum_rows, dim3(nb), dim3(TH), 0, st, n, w.D2 + (int64_t)best * n, w.part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(64), 0, st, nb, w.part, w.inertia);
    SC_CHECK_LAUNCH(ctx);
    double inert = 0.0;
    SC_CHECK_HIP(ctx, hipMemcpyAsync(h, w.inertia, 8, hipMemcpyDeviceToHost, st));
    SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
    memcpy(&inert, h, 8);
    if (inertia) *inertia = inert;
    if (inertia_q) *inertia_q = qh[best];
    if (best_restart) *best_restart = best;
    return SC_OK;
}
