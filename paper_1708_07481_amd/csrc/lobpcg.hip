// Block LOBPCG without preconditioning for the smallest k eigenpairs of the
// normalised graph Laplacian (Section II-B: one product with L per
// iteration; Section III: random or warm-start initial block, no
// preconditioner).  The host loop enqueues the kernels of dense.hip, spmm.hip
// and rr.hip and synchronises once per iteration for the convergence test.
//
// Workspace layout: S = [X W P] and LS = [LX LW LP], each n x 3kp row-major
// (kp = k rounded up to a multiple of 4; pad columns stay zero), the Gram
// matrices, the small factors, and the per-iteration residual history.  With
// soft locking the active W columns are moved to the front of the W block;
// the rest of the block is then skipped by the products that span the basis.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sc_internal.h"

namespace {

__global__ void k_fill_bytes(uint32_t* p, int64_t words) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride) p[i] = 0u;
}

// mask[0..c) = (j < ones) for `c` columns
__global__ void k_set_mask(int* mask, int c, int ones) {
    for (int j = threadIdx.x; j < c; j += blockDim.x) mask[j] = j < ones ? 1 : 0;
}

// Soft locking (Sec. IV): the active W columns (mask[j], j < k) listed in
// ascending order, and the mask rewritten for the compacted block (its first
// `count` columns active).  One workgroup.
__global__ void k_wlist(int k, int kp, int* __restrict__ mask, int* __restrict__ list) {
    __shared__ int flags[256];
    for (int j = threadIdx.x; j < kp; j += blockDim.x) flags[j] = j < k ? mask[j] : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = 0;
        for (int j = 0; j < kp; ++j)
            if (flags[j]) list[m++] = j;
        for (int j = 0; j < kp; ++j) flags[j] = j < m;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kp; j += blockDim.x) mask[j] = flags[j];
}

// W[i][j] <- W[i][list[j]] for j < count, in place: one wave per row reads all
// of its row's active entries, then writes them (list[j] >= j).
template <class T>
__global__ void __launch_bounds__(256)
k_compact_w(int64_t n, int count, T* __restrict__ W, int64_t ld, const int* __restrict__ list) {
    constexpr int PER = 4;                           // up to 256 columns per row
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    T* row = W + i * ld;
    T v[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int j = lane + 64 * t;
        v[t] = j < count ? row[list[j]] : T(0);
    }
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int j = lane + 64 * t;
        if (j < count) row[j] = v[t];
    }
}

template <class Tin, class T>
__global__ void k_load_block(int64_t n, int k, int kp, const Tin* __restrict__ X0, int64_t ldx,
                             T* __restrict__ S, int64_t ld, int* status) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * kp) return;
    const int64_t i = e / kp;
    const int j = (int)(e % kp);
    T v = T(0);
    if (j < k) {
        const Tin x = X0[i * ldx + j];
        if (!isfinite((double)x)) atomicOr(status, DEV_NUMERIC);
        v = (T)x;
    }
    S[i * ld + j] = v;
}

// bound[0] = 2 max_i |d_i|, Gershgorin's bound on ||D - W|| when d_i is the
// row sum of W (one workgroup; max is exact in any order)
template <class T>
__global__ void __launch_bounds__(1024) k_diag_bound(int64_t n, const T* __restrict__ d,
                                                     double* __restrict__ bound) {
    __shared__ double sm[1024];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) m = fmax(m, fabs((double)d[i]));
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) bound[0] = 2.0 * sm[0];
}

template <class T>
__global__ void k_store_block(int64_t n, int k, const T* __restrict__ S, int64_t ld,
                              T* __restrict__ X, int64_t ldx) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * (int64_t)k) return;
    const int64_t i = e / k;
    const int j = (int)(e % k);
    X[i * ldx + j] = S[i * ld + j];
}

}  // namespace

struct sc_lobpcg_state {
    // problem
    int64_t n = 0, nnz = 0;
    const int64_t* row_ptr = nullptr;
    const int32_t* col = nullptr;
    const void* val = nullptr;
    const void* diag = nullptr;     // diagonal of L (nullptr: unit, normalised Laplacian)
    int k = 0, kp = 0, K3 = 0, maxit = 0;
    double tol = 0, lock_tol = 0, chol_tol = 0;
    double op_norm = 2.0;           // bound on ||L|| scaling the relative residual
    int k_conv = 0;                 // columns covered by the stopping test
    sc_precision prec = SC_PREC_FP64;
    int64_t ldx = 0;
    // workspace views
    void* S = nullptr;
    void* LS = nullptr;
    double *GA, *GB, *Gpart, *Gw, *Gwpart, *T64, *C64, *theta, *relres, *res_part, *cq_scr,
        *rr_scr, *hist, *out_max;
    float *T32, *C32;
    // status block (8 ints): [0] flags, [1] P drops, [2] all columns locked,
    // [3] W columns dropped as dependent, [4] Gram recomputations with FP64
    // accumulation, [5] Gram-precision probe flag of the current iteration,
    // [6] inconsistent-iterate flag of the last residual
    int *act, *status, *pdrops, *all_locked, *wdrops, *gram_fallbacks, *gflag, *restart_flag;
    int* gram_queue;                // work counters of the persistent Gram launches
    int* wlist;                     // active W columns, compacted to the front of W
    int kw = 0;                     // W columns active in the next iteration
    int32_t* row_order;             // rows longest first, for the SpMM's row groups
    void* order_scr;                // scratch of the sort that makes it
    GramPlan plan3{}, plan3x{}, plank{};
    int res_blocks = 0;
    // progress
    int t = 0;
    int has_p = 0;
    int converged = 0;
    int done = 0;
    int need_restart = 0;
    int restarts = 0;
    double max_relres = 0.0;
    // asynchronous iteration: convergence flags land in `readback` (pinned
    // host memory of this solve); `ready` is recorded after the copy
    char* readback = nullptr;
    hipEvent_t ready = nullptr;
    int in_flight = 0;
    ~sc_lobpcg_state() {
        if (ready) (void)hipEventDestroy(ready);
        if (readback) (void)hipHostFree(readback);
    }
};

static size_t carve(Carver& c, int64_t n, int k, int maxit, sc_precision prec, sc_lobpcg_state& s) {
    const int kp = (k + 3) / 4 * 4;
    const int K3 = 3 * kp;
    const size_t es = prec == SC_PREC_FP64 ? 8 : 4;
    s.kp = kp;
    s.K3 = K3;
    s.S = c.take<char>((size_t)n * K3 * es);
    s.LS = c.take<char>((size_t)n * K3 * es);
    s.plan3 = gram_plan(n, K3, (int)es);
    s.plan3x = gram_plan(n, K3, 8);          // FP32 data widened to FP64 (fallback)
    s.plank = gram_plan(n, kp, (int)es);
    s.GA = c.take<double>((size_t)K3 * K3);
    s.GB = c.take<double>((size_t)K3 * K3);
    s.Gpart = c.take<double>(std::max(gram_partial_elems(s.plan3, 2),
                                      gram_partial_elems(s.plan3x, 2)));
    s.Gw = c.take<double>((size_t)kp * kp);
    s.Gwpart = c.take<double>(gram_partial_elems(s.plank, 1));
    s.T64 = c.take<double>((size_t)kp * kp);
    s.T32 = c.take<float>((size_t)kp * kp);
    s.C64 = c.take<double>((size_t)K3 * kp);
    s.C32 = c.take<float>((size_t)K3 * kp);
    s.theta = c.take<double>(kp);
    s.relres = c.take<double>(kp);
    s.res_blocks = (int)ceil_div(n, 256);
    s.res_part = c.take<double>((size_t)s.res_blocks * 2 * kp);
    s.cq_scr = c.take<double>(3 * (size_t)kp * kp);
    s.rr_scr = c.take<double>(rr_scratch_elems(K3, k));
    s.hist = c.take<double>((size_t)(maxit + 1) * kp);
    s.out_max = c.take<double>(1);
    s.act = c.take<int>(K3);
    s.status = c.take<int>(8);
    s.pdrops = s.status + 1;
    s.all_locked = s.status + 2;
    s.wdrops = s.status + 3;
    s.gram_fallbacks = s.status + 4;
    s.gflag = s.status + 5;
    s.restart_flag = s.status + 6;
    s.gram_queue = c.take<int>(2);
    s.wlist = c.take<int>(kp);
    s.plan3.queue = s.plan3x.queue = s.plank.queue = s.gram_queue;
    s.row_order = c.take<int32_t>((size_t)n);
    s.order_scr = c.take<char>(row_order_scratch_bytes(n));
    return c.size();
}

static sc_status validate(sc_ctx* ctx, int64_t n, int64_t nnz, const sc_lobpcg_opts* o) {
    if (!o) return sc_fail(ctx, SC_E_INVAL, "lobpcg: opts is NULL");
    if (n <= 0 || nnz < 0) return sc_fail(ctx, SC_E_INVAL, "lobpcg: need n > 0 and nnz >= 0");
    if (o->k < 1) return sc_fail(ctx, SC_E_INVAL, "lobpcg: need k >= 1");
    if (o->k > 256) return sc_fail(ctx, SC_E_UNSUPPORTED, "lobpcg: k = %d > 256", o->k);
    if (3 * (int64_t)o->k > n) return sc_fail(ctx, SC_E_INVAL, "lobpcg: need 3k <= n");
    if (o->maxit < 0) return sc_fail(ctx, SC_E_INVAL, "lobpcg: need maxit >= 0");
    if (o->ldx < o->k) return sc_fail(ctx, SC_E_INVAL, "lobpcg: need ldx >= k");
    if (!(o->tol >= 0.0)) return sc_fail(ctx, SC_E_INVAL, "lobpcg: need tol >= 0");
    if (o->prec != SC_PREC_FP64 && o->prec != SC_PREC_FP32 && o->prec != SC_PREC_FP32_BF16GRAM)
        return sc_fail(ctx, SC_E_INVAL, "lobpcg: unknown precision");
    return SC_OK;
}

extern "C" sc_status sc_lobpcg_workspace(sc_ctx* ctx, int64_t n, int64_t nnz,
                                         const sc_lobpcg_opts* opts, size_t* bytes) {
    if (!ctx || !bytes) return SC_E_INVAL;
    SC_TRY(validate(ctx, n, nnz, opts));
    Carver c(nullptr);
    sc_lobpcg_state s;
    *bytes = carve(c, n, opts->k, opts->maxit, opts->prec, s);
    return SC_OK;
}

namespace {

// Relative pivot floors for the Cholesky factor of a basis Gram matrix
// computed from BF16-rounded inputs (eight BF16 unit roundoffs, 2^-8 each)
// or with FP32 accumulation (about fifty times the accumulated FP32 rounding
// of a row chunk).  Below them a pivot is not resolved by the Gram matrix's
// own rounding error.
constexpr double BF16_PIVOT_TOL = 1.0 / 32.0;
constexpr double FP32_PIVOT_TOL = 1e-4;

template <class T>
struct Solver {
    static T* S(sc_lobpcg_state* s) { return static_cast<T*>(s->S); }
    static T* LS(sc_lobpcg_state* s) { return static_cast<T*>(s->LS); }
    static const T* val(sc_lobpcg_state* s) { return static_cast<const T*>(s->val); }
    static const T* diag(sc_lobpcg_state* s) { return static_cast<const T*>(s->diag); }

    // Gram plan for a basis (or block) narrower than the one the state was
    // sized for: same persistent work counter, partials within the buffer
    static GramPlan narrow_plan(const sc_lobpcg_state* s, const GramPlan& full, int c, int bytes) {
        if (c == full.c) return full;
        GramPlan p = gram_plan(s->n, c, bytes);
        p.queue = full.queue;
        return p;
    }

    // W/X/P block CholQR with mask act[off..off + c) on the c columns at
    // column offset `off` (c = kp, or the active W columns after compaction)
    static sc_status cholqr(sc_ctx* ctx, sc_lobpcg_state* s, int off, int with_L, int mode,
                            int* counter, int c = 0) {
        const int64_t ld = s->K3;
        if (c <= 0) c = s->kp;
        T* V = S(s) + off;
        ProfScope ps(ctx, SC_KIND_CHOLQR);
        SC_TRY(launch_gram<T>(ctx, narrow_plan(s, s->plank, c, (int)sizeof(T)), V, ld, V, ld,
                              nullptr, 0, s->Gwpart, s->Gw, nullptr, GRAM_NATIVE));
        SC_TRY(launch_cholqr_factor(ctx, c, s->Gw, s->act + off, s->chol_tol, s->T64, s->T32,
                                    s->cq_scr, mode, s->status, counter));
        SC_TRY(launch_apply_right<T>(ctx, s->n, c, V, ld, with_L ? LS(s) + off : nullptr, ld,
                                     s->T64, s->T32));
        return SC_OK;
    }

    // G_A = S'LS, G_B = S'S, Rayleigh-Ritz, block update.
    // FP64: Gram in FP64, the Rayleigh-Ritz rules of the plain method.
    // FP32 / FP32_BF16GRAM: the Gram matrices come from FP32 (or BF16-rounded)
    // data with FP32 accumulation; the set-up first probes S'S with a pivot
    // floor matched to that rounding.  Where the basis is too ill-conditioned
    // for it, S'LS and S'S of this iteration are recomputed from the same data
    // widened to FP64 (exact products, FP64 accumulation) and the ordinary
    // set-up (P-drop rule, dependent W columns left out) runs on those.  The
    // recomputation is predicated on a device flag: no host round trip.
    // kw: W columns in use (kp, or the active ones after compaction; the
    // columns [kp + kw, 2kp) are then left out of the Gram products and the
    // block update, and are inactive in the Rayleigh-Ritz step)
    static sc_status rr_and_update(sc_ctx* ctx, sc_lobpcg_state* s, int kw) {
        const int64_t ld = s->K3;
        const int c = s->K3;
        GramPlan p3 = s->plan3, p3x = s->plan3x;
        p3.gap_lo = p3x.gap_lo = s->kp + kw;
        p3.gap_hi = p3x.gap_hi = 2 * s->kp;
        if (s->prec == SC_PREC_FP64) {
            {
                ProfScope ps(ctx, SC_KIND_GRAM);
                SC_TRY(launch_gram<T>(ctx, p3, S(s), ld, LS(s), ld, S(s), ld, s->Gpart, s->GA, s->GB,
                                      GRAM_NATIVE));
            }
            ProfScope ps(ctx, SC_KIND_RR);
            SC_TRY(launch_rayleigh_ritz(ctx, c, s->kp, s->k, s->GA, s->GB, s->act, s->chol_tol,
                                        s->C64, s->C32, s->theta, s->rr_scr, s->status, s->pdrops,
                                        nullptr));
        } else {
            const int bf16 = s->prec == SC_PREC_FP32_BF16GRAM;
            {
                ProfScope ps(ctx, SC_KIND_GRAM);
                SC_TRY(launch_gram<T>(ctx, p3, S(s), ld, LS(s), ld, S(s), ld, s->Gpart, s->GA, s->GB,
                                      bf16 ? GRAM_BF16 : GRAM_NATIVE));
            }
            {
                ProfScope ps(ctx, SC_KIND_RR);
                SC_TRY(launch_rr_setup(ctx, c, s->kp, s->k, s->GA, s->GB, s->act,
                                       bf16 ? BF16_PIVOT_TOL : FP32_PIVOT_TOL, s->rr_scr, s->status,
                                       s->pdrops, nullptr, s->gflag, s->gram_fallbacks, nullptr));
            }
            {
                ProfScope ps(ctx, SC_KIND_GRAM_FP64ACC);
                SC_TRY(launch_gram<T>(ctx, p3x, S(s), ld, LS(s), ld, S(s), ld, s->Gpart, s->GA,
                                      s->GB, GRAM_F32_EXACT, s->gflag));
            }
            ProfScope ps(ctx, SC_KIND_RR);
            SC_TRY(launch_rr_setup(ctx, c, s->kp, s->k, s->GA, s->GB, s->act, s->chol_tol,
                                   s->rr_scr, s->status, s->pdrops, s->gflag, nullptr, nullptr,
                                   s->wdrops));
            SC_TRY(launch_rr_solve(ctx, c, s->kp, s->k, s->C64, s->C32, s->theta, s->rr_scr,
                                   s->status));
        }
        ProfScope ps(ctx, SC_KIND_UPDATE);
        SC_TRY(launch_block_update<T>(ctx, s->n, s->kp, kw, S(s), ld, s->C64, s->C32));
        SC_TRY(launch_block_update<T>(ctx, s->n, s->kp, kw, LS(s), ld, s->C64, s->C32));
        return SC_OK;
    }

    // residual of the current iterate, history row t, W mask, and the copy of
    // the convergence flags to the solve's pinned readback buffer
    static sc_status residual_enqueue(sc_ctx* ctx, sc_lobpcg_state* s) {
        int nb = 0;
        {
            ProfScope ps(ctx, SC_KIND_RESIDUAL);
            SC_TRY(launch_residual<T>(ctx, s->n, s->kp, s->k, s->kp, S(s), LS(s), s->K3,
                                      s->theta, s->res_part, &nb));
            SC_TRY(launch_residual_finalize(ctx, nb, s->kp, s->k, s->k_conv, s->res_part, s->op_norm,
                                            s->lock_tol,
                                            s->relres, s->hist + (int64_t)s->t * s->kp,
                                            s->act + s->kp, s->status, s->out_max,
                                            s->all_locked, s->theta,
                                            s->prec == SC_PREC_FP64 ? nullptr : s->restart_flag,
                                            s->status + 7));
        }
        char* h = s->readback;
        SC_CHECK_HIP(ctx, hipMemcpyAsync(h, s->status, 8 * sizeof(int), hipMemcpyDeviceToHost,
                                         ctx->stream));
        SC_CHECK_HIP(ctx, hipMemcpyAsync(h + 32, s->out_max, sizeof(double), hipMemcpyDeviceToHost,
                                         ctx->stream));
        SC_CHECK_HIP(ctx, hipEventRecord(s->ready, ctx->stream));
        s->in_flight = 1;
        return SC_OK;
    }

    // the readback has landed: convergence test and error flags
    static sc_status residual_process(sc_ctx* ctx, sc_lobpcg_state* s) {
        s->in_flight = 0;
        prof_drain(ctx, false);
        const char* h = s->readback;
        int st[8];
        memcpy(st, h, sizeof st);
        if (st[0] & DEV_BREAKDOWN)
            return sc_fail(ctx, SC_E_BREAKDOWN,
                           "lobpcg: Cholesky QR breakdown (rank-deficient X or W block) at "
                           "iteration %d", s->t);
        if (st[0] & DEV_BREAKDOWN_RR)
            return sc_fail(ctx, SC_E_BREAKDOWN,
                           "lobpcg: Rayleigh-Ritz breakdown (basis Gram matrix not positive "
                           "definite without P) at iteration %d", s->t);
        if (st[0] & DEV_SYNC_TIMEOUT)
            return sc_fail(ctx, SC_E_HIP, "lobpcg: a grid-barrier wait timed out");
        if (st[0] & DEV_NUMERIC)
            return sc_fail(ctx, SC_E_NUMERIC, "lobpcg: NaN or Inf in a residual");
        double mx;
        memcpy(&mx, h + 32, sizeof(double));
        s->max_relres = mx;
        // reduced precision: an inconsistent iterate (LX drifted from L X) is
        // never reported as converged; the next iteration restarts from X
        s->need_restart = s->prec != SC_PREC_FP64 && st[6] != 0;
        s->kw = st[7];
        s->converged = !s->need_restart && ((mx <= s->tol) || st[2]);
        s->done = s->converged || s->t >= s->maxit;
        return SC_OK;
    }

    static sc_status residual(sc_ctx* ctx, sc_lobpcg_state* s) {
        SC_TRY(residual_enqueue(ctx, s));
        SC_CHECK_HIP(ctx, hipEventSynchronize(s->ready));
        return residual_process(ctx, s);
    }

    static sc_status begin(sc_ctx* ctx, sc_lobpcg_state* s, const void* X0) {
        hipStream_t st = ctx->stream;
        const int64_t ld = s->K3;
        const int64_t words = (int64_t)s->n * s->K3 * (int64_t)sizeof(T) / 4;
        hipLaunchKernelGGL(k_fill_bytes, dim3(2048), dim3(256), 0, st, (uint32_t*)s->S, words);
        hipLaunchKernelGGL(k_fill_bytes, dim3(2048), dim3(256), 0, st, (uint32_t*)s->LS, words);
        hipLaunchKernelGGL(k_fill_bytes, dim3(1), dim3(64), 0, st, (uint32_t*)s->status, (int64_t)8);
        hipLaunchKernelGGL(k_fill_bytes, dim3(1), dim3(64), 0, st, (uint32_t*)s->gram_queue,
                           (int64_t)2);
        SC_CHECK_LAUNCH(ctx);
        // the SpMM's row groups take the rows longest first, so that the long
        // rows of high-degree vertices do not trail each launch
        SC_TRY(row_order_by_length(ctx, s->n, s->row_ptr, s->row_order, s->order_scr));
        hipLaunchKernelGGL((k_load_block<T, T>), dim3(ceil_div(s->n * s->kp, 256)), dim3(256), 0, st,
                           s->n, s->k, s->kp, static_cast<const T*>(X0), s->ldx, S(s), ld, s->status);
        SC_CHECK_LAUNCH(ctx);
        {
            const bool bound = s->diag && s->op_norm <= 0.0;
            if (bound) {
                hipLaunchKernelGGL((k_diag_bound<T>), dim3(1), dim3(1024), 0, st, s->n, diag(s),
                                   s->out_max);
                SC_CHECK_LAUNCH(ctx);
            }
            char* h = static_cast<char*>(ctx->stage);
            SC_CHECK_HIP(ctx, hipMemcpyAsync(h, s->status, sizeof(int), hipMemcpyDeviceToHost, st));
            if (bound)
                SC_CHECK_HIP(ctx, hipMemcpyAsync(h + 8, s->out_max, sizeof(double),
                                                 hipMemcpyDeviceToHost, st));
            SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
            int flags;
            memcpy(&flags, h, sizeof flags);
            if (flags & DEV_NUMERIC) return sc_fail(ctx, SC_E_NUMERIC, "lobpcg: NaN or Inf in X0");
            if (bound) {
                memcpy(&s->op_norm, h + 8, sizeof(double));
                if (!(s->op_norm > 0.0) || !std::isfinite(s->op_norm))
                    return sc_fail(ctx, SC_E_NUMERIC, "lobpcg: the diagonal has no positive finite entry");
            }
        }
        // X <- CholQR2(X0)
        for (int rep = 0; rep < 2; ++rep) {
            hipLaunchKernelGGL(k_set_mask, dim3(1), dim3(256), 0, st, s->act, s->kp, s->k);
            SC_TRY(cholqr(ctx, s, 0, 0, CQ_REQUIRE_ALL, nullptr));
        }
        {
            ProfScope ps(ctx, SC_KIND_SPMM);
            SC_TRY(launch_spmm<T>(ctx, s->n, s->row_ptr, s->col, val(s), diag(s), s->k, S(s), ld, LS(s), ld,
                                  s->row_order));
        }
        // Rayleigh-Ritz on span(X) alone
        hipLaunchKernelGGL(k_set_mask, dim3(1), dim3(256), 0, st, s->act, s->K3, s->k);
        SC_CHECK_LAUNCH(ctx);
        SC_TRY(rr_and_update(ctx, s, s->kp));
        s->t = 0;
        s->has_p = 0;
        SC_TRY(residual(ctx, s));
        return SC_OK;
    }

    static sc_status step(sc_ctx* ctx, sc_lobpcg_state* s) {
        SC_TRY(step_enqueue(ctx, s));
        SC_CHECK_HIP(ctx, hipEventSynchronize(s->ready));
        return residual_process(ctx, s);
    }

    // explicit restart: X <- CholQR2(X), LX = L X (a fresh product instead of
    // the recurrence), Rayleigh-Ritz on span(X) alone, P emptied
    static sc_status restart_enqueue(sc_ctx* ctx, sc_lobpcg_state* s) {
        hipStream_t st = ctx->stream;
        const int64_t ld = s->K3;
        s->need_restart = 0;
        s->restarts += 1;
        for (int rep = 0; rep < 2; ++rep) {
            hipLaunchKernelGGL(k_set_mask, dim3(1), dim3(256), 0, st, s->act, s->kp, s->k);
            SC_TRY(cholqr(ctx, s, 0, 0, CQ_REQUIRE_ALL, nullptr));
        }
        {
            ProfScope ps(ctx, SC_KIND_SPMM);
            SC_TRY(launch_spmm<T>(ctx, s->n, s->row_ptr, s->col, val(s), diag(s), s->k, S(s), ld, LS(s), ld,
                                  s->row_order));
        }
        hipLaunchKernelGGL(k_set_mask, dim3(1), dim3(256), 0, st, s->act, s->K3, s->k);
        SC_CHECK_LAUNCH(ctx);
        SC_TRY(rr_and_update(ctx, s, s->kp));
        s->has_p = 0;
        s->t += 1;
        return residual_enqueue(ctx, s);
    }

    // one iteration enqueued on the context's stream, ending with the readback
    static sc_status step_enqueue(sc_ctx* ctx, sc_lobpcg_state* s) {
        if (s->need_restart) return restart_enqueue(ctx, s);
        hipStream_t st = ctx->stream;
        const int64_t ld = s->K3;
        const int kp = s->kp;
        // X stays fully active; the W mask was set by the residual step.
        // Soft locking (Sec. IV): when columns have left W, the active ones
        // move to the front of the W block, and the W products, the basis
        // Gram matrices and the block update run without the rest.
        const int woff = kp;
        const int kw = std::max(0, std::min(s->kw, s->k));
        hipLaunchKernelGGL(k_set_mask, dim3(1), dim3(256), 0, st, s->act, kp, s->k);
        SC_CHECK_LAUNCH(ctx);
        if (kw < s->k) {
            hipLaunchKernelGGL(k_wlist, dim3(1), dim3(256), 0, st, s->k, kp, s->act + woff,
                               s->wlist);
            if (kw > 0)
                hipLaunchKernelGGL((k_compact_w<T>), dim3((unsigned)ceil_div(s->n, 4)), dim3(256),
                                   0, st, s->n, kw, S(s) + woff, ld, s->wlist);
            SC_CHECK_LAUNCH(ctx);
        }
        const int wc = kw < s->k ? kw : kp;          // W columns in use
        if (wc > 0) {
            // a rank-deficient residual block: an error in FP64 (the plain
            // method), dependent columns left out in the reduced-precision modes
            if (s->prec == SC_PREC_FP64)
                SC_TRY(cholqr(ctx, s, woff, 0, CQ_REQUIRE_ALL, nullptr, wc));
            else
                SC_TRY(cholqr(ctx, s, woff, 0, CQ_DROP_DEPENDENT, s->wdrops, wc));
            ProfScope ps(ctx, SC_KIND_SPMM);
            SC_TRY(launch_spmm<T>(ctx, s->n, s->row_ptr, s->col, val(s), diag(s),
                                  kw < s->k ? kw : s->k, S(s) + woff, ld, LS(s) + woff, ld,
                                  s->row_order));
        }
        hipLaunchKernelGGL(k_set_mask, dim3(1), dim3(256), 0, st, s->act + 2 * kp, kp,
                           s->has_p ? s->k : 0);
        SC_CHECK_LAUNCH(ctx);
        if (s->has_p) SC_TRY(cholqr(ctx, s, 2 * kp, 1, CQ_DROP_ALL, s->pdrops));
        SC_TRY(rr_and_update(ctx, s, wc));
        s->has_p = 1;
        s->t += 1;
        return residual_enqueue(ctx, s);
    }

    static sc_status finish(sc_ctx* ctx, sc_lobpcg_state* s, void* X_out, double* theta,
                            double* relres_hist, sc_lobpcg_info* info) {
        hipStream_t st = ctx->stream;
        if (X_out) {
            hipLaunchKernelGGL((k_store_block<T>), dim3(ceil_div(s->n * s->k, 256)), dim3(256), 0,
                               st, s->n, s->k, S(s), s->K3, static_cast<T*>(X_out), s->ldx);
            SC_CHECK_LAUNCH(ctx);
        }
        if (theta)
            SC_CHECK_HIP(ctx, hipMemcpyAsync(theta, s->theta, s->k * sizeof(double),
                                             hipMemcpyDeviceToDevice, st));
        const int rows = s->t + 1;
        std::vector<double> h((size_t)rows * s->kp);
        SC_CHECK_HIP(ctx, hipMemcpyAsync(h.data(), s->hist, h.size() * sizeof(double),
                                         hipMemcpyDeviceToHost, st));
        int cnt[8];
        SC_CHECK_HIP(ctx, hipMemcpyAsync(cnt, s->status, sizeof cnt, hipMemcpyDeviceToHost, st));
        SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
        if (relres_hist)
            for (int r = 0; r < rows; ++r)
                for (int j = 0; j < s->k; ++j) relres_hist[(int64_t)r * s->k + j] = h[(size_t)r * s->kp + j];
        if (info) {
            info->iterations = s->t;
            info->converged = s->converged;
            info->p_drops = cnt[1];
            int locked = 0;
            for (int j = 0; j < s->k; ++j) locked += h[(size_t)s->t * s->kp + j] <= s->lock_tol;
            info->locked_cols = locked;
            info->max_relres = s->max_relres;
            info->w_drops = cnt[3];
            info->gram_fallbacks = cnt[4];
            info->restarts = s->restarts;
        }
        return SC_OK;
    }
};

sc_status dispatch_begin(sc_ctx* ctx, sc_lobpcg_state* s, const void* X0) {
    return s->prec == SC_PREC_FP64 ? Solver<double>::begin(ctx, s, X0)
                                   : Solver<float>::begin(ctx, s, X0);
}
sc_status dispatch_step(sc_ctx* ctx, sc_lobpcg_state* s) {
    return s->prec == SC_PREC_FP64 ? Solver<double>::step(ctx, s) : Solver<float>::step(ctx, s);
}
sc_status dispatch_step_enqueue(sc_ctx* ctx, sc_lobpcg_state* s) {
    return s->prec == SC_PREC_FP64 ? Solver<double>::step_enqueue(ctx, s)
                                   : Solver<float>::step_enqueue(ctx, s);
}
sc_status dispatch_process(sc_ctx* ctx, sc_lobpcg_state* s) {
    return s->prec == SC_PREC_FP64 ? Solver<double>::residual_process(ctx, s)
                                   : Solver<float>::residual_process(ctx, s);
}
sc_status dispatch_finish(sc_ctx* ctx, sc_lobpcg_state* s, void* X_out, double* theta,
                          double* relres_hist, sc_lobpcg_info* info) {
    return s->prec == SC_PREC_FP64 ? Solver<double>::finish(ctx, s, X_out, theta, relres_hist, info)
                                   : Solver<float>::finish(ctx, s, X_out, theta, relres_hist, info);
}

}  // namespace

extern "C" sc_status sc_lobpcg_begin(sc_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                     const int32_t* col, const void* val,
                                     const sc_lobpcg_opts* opts, const void* X0, void* ws,
                                     size_t ws_bytes, sc_lobpcg_state** state, int* done) {
    if (!ctx || !state) return SC_E_INVAL;
    *state = nullptr;
    SC_TRY(validate(ctx, n, nnz, opts));
    if (!row_ptr || !X0 || !ws || (nnz > 0 && (!col || !val)))
        return sc_fail(ctx, SC_E_INVAL, "lobpcg: null pointer argument");
    sc_lobpcg_state* s = new sc_lobpcg_state();
    Carver c(ws);
    const size_t need = carve(c, n, opts->k, opts->maxit, opts->prec, *s);
    if (ws_bytes < need) {
        delete s;
        return sc_fail(ctx, SC_E_NOMEM, "lobpcg: workspace %zu < %zu bytes", ws_bytes, need);
    }
    s->n = n;
    s->nnz = nnz;
    s->row_ptr = row_ptr;
    s->col = col;
    s->val = val;
    s->diag = opts->diag;
    // with a diagonal (L = D - W) and no bound given, begin() computes
    // 2 max |d_i| on the device
    s->op_norm = opts->op_norm > 0 ? opts->op_norm : (opts->diag ? 0.0 : 2.0);
    s->k_conv = (opts->k_conv > 0 && opts->k_conv < opts->k) ? opts->k_conv : opts->k;
    s->k = opts->k;
    s->maxit = opts->maxit;
    s->tol = opts->tol;
    s->prec = opts->prec;
    s->ldx = opts->ldx;
    const bool f64 = opts->prec == SC_PREC_FP64;
    s->lock_tol = opts->lock_tol > 0 ? opts->lock_tol : (f64 ? 1e-13 : 1e-6);
    s->chol_tol = opts->chol_tol > 0 ? opts->chol_tol : (f64 ? 1e-14 : 1e-6);
    sc_status st = hipSetDevice(ctx->device) == hipSuccess ? SC_OK : SC_E_HIP;
    if (st == SC_OK && (hipHostMalloc((void**)&s->readback, 64, hipHostMallocDefault) != hipSuccess ||
                        hipEventCreateWithFlags(&s->ready, hipEventDisableTiming) != hipSuccess))
        st = sc_fail(ctx, SC_E_HIP, "lobpcg: cannot create the readback buffer or event");
    if (st == SC_OK) st = dispatch_begin(ctx, s, X0);
    if (st != SC_OK) {
        delete s;
        return st;
    }
    *state = s;
    if (done) *done = s->done;
    return SC_OK;
}

extern "C" sc_status sc_lobpcg_step(sc_ctx* ctx, sc_lobpcg_state* s, int* done) {
    if (!ctx || !s) return SC_E_INVAL;
    if (s->in_flight) {
        SC_CHECK_HIP(ctx, hipEventSynchronize(s->ready));
        SC_TRY(dispatch_process(ctx, s));
    } else if (!s->done) {
        SC_TRY(dispatch_step(ctx, s));
    }
    if (done) *done = s->done;
    return SC_OK;
}

extern "C" sc_status sc_lobpcg_step_async(sc_ctx* ctx, sc_lobpcg_state* s) {
    if (!ctx || !s) return SC_E_INVAL;
    if (s->in_flight) return sc_fail(ctx, SC_E_INVAL, "lobpcg: an iteration is already in flight");
    if (s->done) return SC_OK;
    return dispatch_step_enqueue(ctx, s);
}

extern "C" sc_status sc_lobpcg_step_poll(sc_ctx* ctx, sc_lobpcg_state* s, int* ready, int* done) {
    if (!ctx || !s) return SC_E_INVAL;
    int rdy = 1;
    if (s->in_flight) {
        const hipError_t q = hipEventQuery(s->ready);
        if (q == hipErrorNotReady) {
            rdy = 0;
        } else if (q != hipSuccess) {
            return sc_fail(ctx, SC_E_HIP, "lobpcg: hipEventQuery failed: %s", hipGetErrorString(q));
        } else {
            SC_TRY(dispatch_process(ctx, s));
        }
    }
    if (ready) *ready = rdy;
    if (done) *done = s->done;
    return SC_OK;
}

extern "C" sc_status sc_lobpcg_end(sc_ctx* ctx, sc_lobpcg_state* s, void* X_out, double* theta,
                                   double* relres_hist, sc_lobpcg_info* info) {
    if (!ctx || !s) return SC_E_INVAL;
    if (s->in_flight) (void)hipEventSynchronize(s->ready);
    sc_status st = dispatch_finish(ctx, s, X_out, theta, relres_hist, info);
    delete s;
    return st;
}

extern "C" sc_status sc_lobpcg_solve(sc_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                     const int32_t* col, const void* val,
                                     const sc_lobpcg_opts* opts, const void* X0, void* X_out,
                                     double* theta, double* relres_hist, sc_lobpcg_info* info,
                                     void* ws, size_t ws_bytes) {
    sc_lobpcg_state* s = nullptr;
    int done = 0;
    SC_TRY(sc_lobpcg_begin(ctx, n, nnz, row_ptr, col, val, opts, X0, ws, ws_bytes, &s, &done));
    while (!done) {
        sc_status st = sc_lobpcg_step(ctx, s, &done);
        if (st != SC_OK) {
            delete s;
            return st;
        }
    }
    return sc_lobpcg_end(ctx, s, X_out, theta, relres_hist, info);
}
