// Internal declarations of the gfx950 spectral-clustering library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include <string>
#include <vector>

#include "../../include/spectral.h"

struct sc_ctx {
    int device = 0;
    int num_cu = 0;                 // compute units of the device (persistent launches)
    hipStream_t stream = nullptr;
    std::string err;
    // pinned host staging area for the small device-to-host reads of the
    // convergence tests (hipHostMalloc'ed once per context)
    void* stage = nullptr;
    size_t stage_bytes = 0;
    // kernel timing (HIP events on `stream` around launches of the kinds in prof_mask)
    unsigned prof_mask = 0;
    struct Pending {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    int64_t prof_count[SC_KIND_COUNT] = {};
    double prof_ms[SC_KIND_COUNT] = {};
};

// Accumulate the durations of completed timed launches (the caller has
// synchronised the stream, or calls with sync = true).
void prof_drain(sc_ctx* ctx, bool sync);

// Times everything enqueued on ctx->stream during its lifetime when the kind
// is enabled.
struct ProfScope {
    sc_ctx* ctx;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(sc_ctx* c, int k);
    ~ProfScope();
};

sc_status sc_fail(sc_ctx* ctx, sc_status st, const char* fmt, ...);

#define SC_CHECK_HIP(ctx, call)                                                         \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return sc_fail((ctx), SC_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define SC_CHECK_LAUNCH(ctx) SC_CHECK_HIP(ctx, hipGetLastError())

#define SC_TRY(expr)                     \
    do {                                 \
        sc_status s_ = (expr);           \
        if (s_ != SC_OK) return s_;      \
    } while (0)

// Device status word bits (set with atomicOr by kernels, read by the host).
enum : int {
    DEV_BAD_INPUT = 1,      // id out of range / invalid weight
    DEV_NUMERIC = 2,        // NaN or Inf
    DEV_BREAKDOWN = 4,      // unrecoverable Cholesky failure
    DEV_P_DROPPED = 8,      // P dropped in this iteration (informational)
    DEV_BREAKDOWN_RR = 16,  // basis Gram matrix of the Rayleigh-Ritz step not positive definite
    DEV_SYNC_TIMEOUT = 32,  // a grid-barrier wait of a cooperative kernel exceeded its bound
};

// Bump allocator over a caller-provided workspace.  With base == nullptr it
// only measures.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t size() const { return (off + 255) & ~size_t(255); }
};

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline int ceil_log2_u64(uint64_t v) {
    int e = 0;
    while (e < 64 && (uint64_t(1) << e) < v) ++e;
    return e;
}

// ---------------------------------------------------------------------------
// Wave-wide FP64 sum through DPP moves (quad permutes, row mirrors, row
// broadcasts), which stay in the vector ALU instead of going through the LDS
// crossbar like a shuffle does.  The total ends in lane 63 and is returned to
// every lane.  All 64 lanes must be active.  The order of the additions is
// fixed (lanes pairwise within quads, then half-rows, rows, and the four rows
// in sequence), so the result is deterministic.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ inline double sc_dpp_move(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, ROW_MASK, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ inline double sc_wave_sum(double v) {
    v += sc_dpp_move<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v += sc_dpp_move<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    v += sc_dpp_move<0x141, 0xF>(v);   // row_half_mirror
    v += sc_dpp_move<0x140, 0xF>(v);   // row_mirror
    v += sc_dpp_move<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v += sc_dpp_move<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    const long long u = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readlane((int)u, 63);
    const unsigned hi = __builtin_amdgcn_readlane((int)(u >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// ---------------------------------------------------------------------------
// Device-wide primitives (scan.hip, radix.hip)
// ---------------------------------------------------------------------------
// Exclusive (inclusive = 0) or inclusive scan of n uint64 values, in place
// allowed.  tmp needs scan_u64_tmp_elems(n) elements.
size_t scan_u64_tmp_elems(int64_t n);
sc_status scan_u64(sc_ctx* ctx, const uint64_t* in, uint64_t* out, int64_t n, int inclusive,
                   uint64_t* tmp);
// Batched inclusive (exclusive) scan: `batch` independent rows of length n
// (row stride n), in place allowed.
sc_status scan_u64_batched(sc_ctx* ctx, const uint64_t* in, uint64_t* out, int64_t n, int batch,
                           uint64_t* tmp);
sc_status scan_u64_batched_exclusive(sc_ctx* ctx, const uint64_t* in, uint64_t* out, int64_t n,
                                     int batch, uint64_t* tmp);
size_t scan_u64_batched_tmp_elems(int64_t n, int batch);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of key.
// Buffers: keys/vals (in/out), keys_alt/vals_alt (same size, scratch),
// tmp: radix_tmp_elems(n) uint64.  Result ends in keys/vals.
size_t radix_tmp_elems(int64_t n);
sc_status radix_sort_pairs(sc_ctx* ctx, uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                           uint32_t* vals_alt, int64_t n, int bits, uint64_t* tmp);

// ---------------------------------------------------------------------------
// Kernels used by the LOBPCG driver (spmm.hip, dense.hip, rr.hip)
// ---------------------------------------------------------------------------
// order: optional row permutation for the row groups (rows longest first:
// row_order_by_length); the arithmetic of every row is unchanged.
template <class T>
sc_status launch_spmm(sc_ctx* ctx, int64_t n, const int64_t* row_ptr, const int32_t* col,
                      const T* val, const T* diag, int k, const T* X, int64_t ldx, T* Y,
                      int64_t ldy, const int32_t* order = nullptr);
// order[0 .. n) = the rows by descending length, stable; `scratch` needs
// row_order_scratch_bytes(n) bytes (256-byte aligned)
size_t row_order_scratch_bytes(int64_t n);
sc_status row_order_by_length(sc_ctx* ctx, int64_t n, const int64_t* row_ptr, int32_t* order,
                              void* scratch);

// Gram products G1 = A^T B1 (and G2 = A^T B2 when B2 != nullptr), ca x cb,
// upper triangle computed, mirrored; FP64 results.  A/B1/B2 are n x c blocks
// of T with row strides.  bf16 != 0 (T = float only) rounds the inputs to
// BF16 and accumulates in FP32 on the matrix cores.
struct GramPlan {
    int64_t n;
    int c;              // columns of A and B (square Gram)
    int chunks;         // row chunks (split-K)
    int64_t chunk_rows; // rows per chunk (multiple of 32)
    int bt;             // workgroup output tile edge
    int tiles;          // tiles per side
    // two zeroed ints of device memory owned by the caller: the FP32 kernels
    // run as persistent workgroups that take (tile pair, chunk) items from
    // this counter, and the last workgroup out zeroes both again, so launches
    // on one stream can share them (nullptr: the unstaged FP32 kernel)
    int* queue = nullptr;
    // columns [gap_lo, gap_hi) are not used (their results are never read):
    // MFMA sub-tiles wholly inside skip their products
    int gap_lo = 0, gap_hi = 0;
};
// Gram precision for FP32 data: native FP32 MFMA, BF16-rounded inputs, or
// widened to FP64 (exact products, FP64 accumulation).  FP64 data always
// accumulates in FP64.
enum { GRAM_NATIVE = 0, GRAM_BF16 = 1, GRAM_F32_EXACT = 2 };
// plan for `accum_bytes` = 8 (FP64 accumulation: FP64 data or GRAM_F32_EXACT)
// or 4 (GRAM_NATIVE / GRAM_BF16 on FP32 data)
GramPlan gram_plan(int64_t n, int c, int accum_bytes);
size_t gram_partial_elems(const GramPlan& p, int nout);
// G1 = A'B1 (and G2 = A'B2), split over row chunks; with `pred` non-null the
// launches do nothing when *pred == 0.
template <class T>
sc_status launch_gram(sc_ctx* ctx, const GramPlan& p, const T* A, int64_t lda, const T* B1,
                      int64_t ldb1, const T* B2, int64_t ldb2, double* partial, double* G1,
                      double* G2, int gmode, const int* pred = nullptr);

// Small-matrix Cholesky QR factor: from the c x c FP64 Gram G and the
// active-column mask, T = D^-1 R^-1 (zero rows/cols for inactive columns).
// On a failing pivot, by mode:
//   CQ_REQUIRE_ALL     status |= BREAKDOWN (also when an active column is zero);
//   CQ_DROP_ALL        T = 0, mask = 0, status |= P_DROPPED, counter[0]++;
//   CQ_DROP_DEPENDENT  the failing column leaves the mask (counter[0]++) and
//                      the factorisation is redone without it.
enum { CQ_REQUIRE_ALL = 0, CQ_DROP_ALL = 1, CQ_DROP_DEPENDENT = 2 };
sc_status launch_cholqr_factor(sc_ctx* ctx, int c, const double* G, int* mask, double tol,
                               double* T64, float* T32, double* scratch, int mode,
                               int* status, int* counter);
// V <- V T (and V2 <- V2 T) on n x c row blocks, in place.
template <class T>
sc_status launch_apply_right(sc_ctx* ctx, int64_t n, int c, T* V, int64_t ldv, T* V2,
                             int64_t ldv2, const double* T64, const float* T32);
// Block update on S = [X W P] (n x 3kp, row stride ld): P <- [W P] C_WP,
// X <- X C_X + P.  kw: W columns in use (the first kw of the W block; the rest
// of the block and their rows of C are skipped).
template <class T>
sc_status launch_block_update(sc_ctx* ctx, int64_t n, int kp, int kw, T* S, int64_t ld,
                              const double* C64, const float* C32);
// Residual R = LX - X diag(theta) into columns [woff, woff + kp) of S;
// per-block partial sums of R^2, X^2.
template <class T>
sc_status launch_residual(sc_ctx* ctx, int64_t n, int kp, int k, int woff, T* S, const T* LS,
                          int64_t ld, const double* theta, double* partial, int* nblocks_out);
// Finalise: column totals of the block partials (in place), then relres,
// history row, W mask, flags; out[0] = max relres, out_flags[0] = all columns
// locked.  relres_j = ||r_j|| / (op_norm ||x_j||), op_norm >= ||L|| (2 for the
// normalised Laplacian).  With out_restart non-null it is set to 1 when the
// iterate is inconsistent (a Ritz value outside [0, op_norm] by more than
// op_norm * 5e-4, or relres > 1, impossible when LX = L X), else 0.
// out_wcount[0] = the number of W columns left active (relres > lock_tol).
sc_status launch_residual_finalize(sc_ctx* ctx, int nblocks, int kp, int k, int k_conv,
                                   double* partial, double op_norm, double lock_tol, double* relres,
                                   double* hist_row, int* wmask, int* status, double* out_max,
                                   int* out_all_locked, const double* theta, int* out_restart,
                                   int* out_wcount);

// Rayleigh-Ritz (FP64) on the active columns: C (K3 x kp), theta (kp).
// Split in two: the set-up (active set, Cholesky of G_B with the P-drop
// rule, reduced G_A) and the solve (reduced eigenproblem, C, theta).
//   pred   (device int or null): the set-up does nothing when *pred == 0;
//   probe  (device int or null): probing set-up, tolerance `tol` without the
//          P-drop rule; on a failing pivot it sets *probe = 1 (and
//          probe_counter[0]++) and leaves m = 0, else *probe = 0;
//   wcounter (device int or null): when the factorisation fails without P,
//          the failing W column leaves the basis (wcounter[0]++) and the
//          factorisation is redone, instead of a breakdown.
size_t rr_scratch_elems(int K3, int k);
sc_status launch_rr_setup(sc_ctx* ctx, int K3, int kp, int k, const double* GA, const double* GB,
                          int* act, double tol, double* scratch, int* status, int* counter,
                          const int* pred, int* probe, int* probe_counter, int* wcounter);
sc_status launch_rr_solve(sc_ctx* ctx, int K3, int kp, int k, double* C64, float* C32,
                          double* theta, double* scratch, int* status);
sc_status launch_rayleigh_ritz(sc_ctx* ctx, int K3, int kp, int k, const double* GA,
                               const double* GB, int* act, double tol, double* C64, float* C32,
                               double* theta, double* scratch, int* status, int* counter,
                               int* wcounter);
sc_status launch_symeig(sc_ctx* ctx, int m, int k, const double* A, double* w, double* V,
                        double* scratch);
size_t symeig_scratch_elems(int m, int k);
