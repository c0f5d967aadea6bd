/*
 * spectral.h -- C ABI of the MI355X (gfx950) spectral-clustering library.
 *
 * The library implements the hot path of spectral clustering by LOBPCG as
 * described in "Preconditioned Spectral Clustering for Stochastic Block
 * Partition Streaming Graph Challenge" (Zhuzhunashvili & Knyazev):
 *   1. symmetrise the directed adjacency, W <- W + W'        (Section II-A)
 *   2. form the normalised graph Laplacian I - D^-1/2 W D^-1/2
 *      (Section II-A defines the Laplacian from W and its row sums D; the
 *      normalised form is used here)
 *   3. compute its smallest k eigenpairs with block LOBPCG without
 *      preconditioning, from a random or warm-start block X0
 *      (Section II-B, Section III)
 *   4. label the vertices by k-means on the row-normalised eigenvectors
 *      (Section II-A).
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers (memory owned by the caller)
 *     unless the comment says "host".  The library never allocates device
 *     memory; each call that needs scratch takes a caller-provided workspace
 *     `ws` of at least the size returned by the matching *_workspace query,
 *     aligned to 256 bytes.
 *   - Work is enqueued on the stream given to sc_ctx_create.  Calls that
 *     return host values synchronise that stream; their comments say so.
 *   - Multivectors (n x k blocks) are row-major with a row stride `ld`
 *     (elements) >= k: the k values of one vertex are contiguous.
 *   - Every call returns an sc_status; on failure sc_last_error(ctx) holds a
 *     message.  Arguments are validated on the host before any launch.
 *   - One context per host thread; calls on one context are not reentrant.
 */
#ifndef SPECTRAL_H
#define SPECTRAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SC_OK = 0,
    SC_E_INVAL = -1,        /* invalid argument (sizes, ids out of range, null pointers) */
    SC_E_NOMEM = -2,        /* workspace smaller than the query returned */
    SC_E_HIP = -3,          /* HIP runtime error */
    SC_E_BREAKDOWN = -4,    /* Cholesky breakdown that the rules below cannot recover */
    SC_E_NUMERIC = -5,      /* NaN / Inf in an input block or a residual norm */
    SC_E_UNSUPPORTED = -6   /* size outside what the kernels support (e.g. k > 256) */
} sc_status;

/* Symmetrisation of Section II-A: "+" is a logical or (unweighted graph) or
 * an algebraic sum of non-negative weights. */
typedef enum { SC_SYM_LOGICAL = 0, SC_SYM_ALGEBRAIC = 1 } sc_sym_mode;

/* Arithmetic of the LOBPCG multivectors.  FP64: everything in FP64.
 * FP32: Laplacian values, SpMM, multivectors, block updates and Gram
 * products in FP32 (Gram partial sums promoted to FP64); every Cholesky and
 * the Rayleigh-Ritz eigenproblem in FP64 (the paper's single-precision
 * variant, Section IV).  FP32_BF16GRAM: as FP32 but the Gram products of the
 * Rayleigh-Ritz step read their inputs rounded to BF16 (round to nearest
 * even) and accumulate in FP32 on the matrix cores. */
typedef enum { SC_PREC_FP64 = 0, SC_PREC_FP32 = 1, SC_PREC_FP32_BF16GRAM = 2 } sc_precision;

typedef struct sc_ctx sc_ctx;

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  Host memory only.  Fails with
 * SC_E_HIP when more than one HIP runtime is mapped into the process (see
 * sc_runtime_info). */
sc_status sc_ctx_create(int device, void* hip_stream, sc_ctx** out);
/* Synchronises the context's stream, then frees its events and pinned host
 * buffer.  Call it while the HIP runtime is alive, i.e. before the program
 * starts its exit: not from process-exit handlers or finalisers. */
sc_status sc_ctx_destroy(sc_ctx* ctx);
/* Text of the last error on this context ("" if none).  Host string owned by ctx. */
const char* sc_last_error(const sc_ctx* ctx);
/* Library ABI version (major * 10000 + minor * 100 + patch). */
int sc_version(void);
/* The HIP runtime this process runs the library on (host outputs, any may be
 * NULL): hipRuntimeGetVersion's value, the number of distinct libamdhip64
 * objects mapped into the process (1 when the library shares the runtime of
 * the program that loaded it; 2 means two runtimes, which must not happen),
 * and the file path of the one that resolves the library's HIP calls,
 * truncated to path_len - 1 bytes.  Needs no device and no context. */
sc_status sc_runtime_info(int* hip_runtime_version, int* hip_libs_mapped, char* path,
                          size_t path_len);

/* ------------------------------------------------------------------------
 * Graph construction: W <- W + W' (Section II-A).
 * ------------------------------------------------------------------------ */
sc_status sc_graph_build_workspace(sc_ctx* ctx, int64_t n, int64_t m, size_t* bytes);

/*
 * Directed COO (src[e] -> dst[e], e < m; ids in [0, n)) to the CSR of the
 * symmetric matrix W + W'.  Edge e contributes (src,dst) and (dst,src); self
 * loops are dropped and counted.  Repeated (row,col) entries are merged:
 * SC_SYM_LOGICAL gives weight 1; SC_SYM_ALGEBRAIC sums the weights in the
 * order edge 0 forward, edge 0 backward, edge 1 forward, ...  Columns are
 * strictly ascending in every row.  degree[i] = sum of row i in ascending
 * column order (the diagonal matrix D of Section II-A).
 *   src, dst     int32 [m] (device)
 *   w            float64 [m] (device) or NULL for unit weights; weights must
 *                be finite and >= 0 (SC_SYM_ALGEBRAIC only)
 *   row_ptr      int64 [n+1] (device, out)
 *   col          int32 [2m] capacity (device, out); first nnz entries valid
 *   w_sym        float64 [2m] capacity (device, out) or NULL
 *   degree       float64 [n] (device, out)
 *   nnz_out      host, out: number of stored entries (synchronises)
 *   self_loops   host, out, may be NULL
 * Errors: SC_E_INVAL for n <= 0, m < 0, m >= 2^31, an id outside [0,n) or
 * an invalid weight (detected on the device, reported after the sync).
 */
sc_status sc_graph_build(sc_ctx* ctx, int64_t n, int64_t m, const int32_t* src,
                         const int32_t* dst, const double* w, sc_sym_mode mode,
                         int64_t* row_ptr, int32_t* col, double* w_sym, double* degree,
                         int64_t* nnz_out, int64_t* self_loops, void* ws, size_t ws_bytes);

/* ------------------------------------------------------------------------
 * Normalised Laplacian L = I - D^-1/2 W D^-1/2 on W's pattern.
 * ------------------------------------------------------------------------ */
/*
 * val[p] = -(w_p / sqrt(d_i d_j)) for the entry p = (i, j) of W (0 when
 * d_i d_j == 0); the unit diagonal is implicit and not stored.
 * dinv_sqrt[i] = 1 / sqrt(d_i), or 0 for an isolated vertex (whose row of L
 * is then the unit row).  One rounded quotient per entry keeps L bitwise
 * symmetric.
 *   row_ptr, col, degree  from sc_graph_build (device)
 *   w_sym    float64 [nnz] or NULL (unit weights)
 *   val64    float64 [nnz] (out) or NULL
 *   val32    float32 [nnz] (out) or NULL: val64 rounded to nearest
 *   dinv_sqrt float64 [n] (out) or NULL
 * No synchronisation.
 */
sc_status sc_laplacian_csr(sc_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                           const int32_t* col, const double* w_sym, const double* degree,
                           double* val64, float* val32, double* dinv_sqrt);

/*
 * The graph Laplacian L = D - W as Section II-A introduces it (Section III
 * applies it matrix-free with the degrees as pre-computed diagonal), on the
 * pattern of sc_graph_build: val_p = -w_p (exact; -1 for unit weights), and
 * the diagonal d_i, which is `degree` itself for FP64 products.
 *   row_ptr, degree  from sc_graph_build (device)
 *   w_sym    float64 [nnz] or NULL (unit weights)
 *   val64    float64 [nnz] (out) or NULL
 *   val32    float32 [nnz] (out) or NULL: val64 rounded to nearest
 *   diag32   float32 [n] (out) or NULL: the degrees rounded to nearest, the
 *            diagonal of FP32 products
 * Pass the diagonal to sc_spmm_diag / sc_lobpcg_opts.diag; with
 * sc_lobpcg_opts.op_norm = 0 the solver bounds ||D - W|| by 2 max_i d_i
 * (Gershgorin), computed on the device.
 * No synchronisation.
 */
sc_status sc_laplacian_combinatorial(sc_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                                     const double* w_sym, const double* degree, double* val64,
                                     float* val32, float* diag32);

/*
 * Y = L X: the one multiplication by the graph Laplacian per LOBPCG
 * iteration (Section III).  For every row i and column j < k,
 *   y_ij = x_ij, then over row i in ascending column order
 *   y_ij = fma(val_p, x_{col_p, j}, y_ij).
 * fp64 != 0: val, X, Y are float64; else float32.  X and Y must not alias.
 * ldx, ldy >= k.  No synchronisation.
 */
sc_status sc_spmm(sc_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                  const int32_t* col, const void* val, int fp64, int k, const void* X,
                  int64_t ldx, void* Y, int64_t ldy);

/*
 * Y = L X with an explicit diagonal a (L = D - W: a = the degrees):
 *   y_ij = a_i x_ij (one rounded product), then over row i in ascending
 *   column order y_ij = fma(val_p, x_{col_p, j}, y_ij).
 * diag: n entries of the product's type (float64 if fp64 else float32), device,
 * or NULL for the unit diagonal (then identical to sc_spmm).  Other arguments
 * as sc_spmm.  No synchronisation.
 */
sc_status sc_spmm_diag(sc_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                       const int32_t* col, const void* val, const void* diag, int fp64, int k,
                       const void* X, int64_t ldx, void* Y, int64_t ldy);

/* ------------------------------------------------------------------------
 * LOBPCG without preconditioning for the k smallest eigenpairs of L.
 * ------------------------------------------------------------------------ */
typedef struct {
    int k;                 /* block size = number of eigenpairs, 1 <= k <= 256, 3k <= n */
    int maxit;             /* iterations (products L W) at most, >= 0 */
    double tol;            /* stop when max_j relres_j <= tol (0: run maxit iterations) */
    sc_precision prec;
    int64_t ldx;           /* row stride of X0 / X_out, >= k */
    double lock_tol;       /* columns with relres_j <= lock_tol leave the W block
                              (0 = default: 1e-13 in FP64, 1e-6 otherwise) */
    double chol_tol;       /* relative pivot floor of every Cholesky
                              (0 = default: 1e-14 in FP64, 1e-6 otherwise) */
    const void* diag;      /* diagonal of L, n entries (float64 in FP64 mode, else
                              float32), device; NULL = unit diagonal, i.e. the
                              normalised Laplacian I - D^-1/2 W D^-1/2 */
    double op_norm;        /* upper bound of ||L|| in relres_j = ||r_j|| / (op_norm
                              ||x_j||); 0 = default: 2 (the normalised Laplacian's
                              bound) without diag, 2 max_i |diag_i| (Gershgorin,
                              computed on the device) with diag */
    int k_conv;            /* the stopping test (and info.max_relres) covers columns
                              0 .. k_conv-1 only (0 = all k): a block wider than the
                              wanted pairs, as Section IV runs l slightly above k */
} sc_lobpcg_opts;

typedef struct {
    int iterations;        /* Rayleigh-Ritz updates after the initial one */
    int converged;         /* 1 if max relres <= tol (or every column locked) */
    int p_drops;           /* iterations in which the P block was dropped */
    int locked_cols;       /* W columns excluded in the last iteration */
    double max_relres;     /* of the returned block */
    int w_drops;           /* W columns left out as numerically dependent
                              (reduced-precision modes; always 0 in FP64) */
    int gram_fallbacks;    /* iterations whose Gram matrices were recomputed with
                              FP64 accumulation (reduced-precision modes) */
    int restarts;          /* explicit restarts (reduced-precision modes) */
} sc_lobpcg_info;

sc_status sc_lobpcg_workspace(sc_ctx* ctx, int64_t n, int64_t nnz, const sc_lobpcg_opts* opts,
                              size_t* bytes);

/*
 * Block LOBPCG (Knyazev 2001) with T = I for the smallest k eigenpairs of
 * L = diag(a) + offdiag(val): a = 1 (opts.diag NULL, the normalised
 * Laplacian) or a = opts.diag (L = D - W).  Iteration, with S = [X W P] and
 * LS = L S (N = opts.op_norm, 2 by default):
 *   init: X <- CholQR2(X0); LX = L X; Rayleigh-Ritz on span(X);
 *   each iteration: R = LX - X diag(theta); relres_j = ||R_j|| / (N ||x_j||);
 *     stop if max relres <= tol; W <- CholQR(R without locked columns);
 *     LW = L W; P, LP <- CholQR(P) (P dropped for this iteration if that
 *     Cholesky fails); Gram matrices S'LS and S'S (3k x 3k); Rayleigh-Ritz in
 *     FP64 (Cholesky of S'S; on failure P is dropped and the step redone);
 *     P <- [W P] C_WP, X <- X C_X + P (and the same for LX, LP).
 * Soft locking (Sec. IV, opts.lock_tol): a column whose relres is at or below
 * lock_tol leaves W; the active W columns are moved to the front of the W
 * block, and the W products, the Gram matrices and the block update skip the
 * rest of it (the Rayleigh-Ritz step sees those columns as inactive).
 * Every CholQR equilibrates the columns before the Cholesky.
 * Reduced precision (FP32, FP32_BF16GRAM): a W column whose CholQR pivot
 * fails, or whose pivot in the Cholesky of S'S fails once P is out, is left
 * out of the basis for that iteration (info.w_drops) instead of ending the
 * solve.  The Gram matrices S'LS, S'S of an iteration are computed with
 * FP32 accumulation (FP32_BF16GRAM: from BF16-rounded inputs) and S'S is
 * first factored with a relative pivot floor matched to that rounding (1e-4
 * for FP32, 2^-5 for BF16); where it fails, both are recomputed from the
 * FP32 data widened to FP64 (exact products, FP64 accumulation) and the
 * ordinary Rayleigh-Ritz runs on those (info.gram_fallbacks).  An iterate
 * whose Ritz values leave [0, N] by more than N * 5e-4, or with a relres above 1
 * (impossible while LX = L X holds), shows that the recurrence for LX has
 * drifted: it is not accepted as converged, and the next iteration restarts
 * explicitly (X <- CholQR2(X), LX = L X, Rayleigh-Ritz on span(X), P
 * emptied; info.restarts).  It counts as an iteration.
 *   val     float64 [nnz] (prec FP64) or float32 [nnz] (other precisions)
 *   X0      n x ldx start block (float64 for FP64, float32 otherwise); must
 *           have full column rank and finite entries
 *   X_out   n x ldx result (may alias X0)
 *   theta   float64 [k] (device, out): Ritz values, ascending
 *   relres_hist  host float64 [(maxit+1) * k] or NULL: relres of every
 *           iterate (row t after t iterations)
 *   info    host, out
 * Synchronises once per iteration (convergence test).
 * Errors: SC_E_INVAL (sizes), SC_E_UNSUPPORTED (k > 256), SC_E_NUMERIC (NaN
 * or Inf in X0 or a residual), SC_E_BREAKDOWN (rank-deficient X0; in FP64
 * also a rank-deficient W, or S'S not positive definite even without P).
 * On SC_E_BREAKDOWN X_out is not written.
 */
sc_status sc_lobpcg_solve(sc_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                          const int32_t* col, const void* val, const sc_lobpcg_opts* opts,
                          const void* X0, void* X_out, double* theta, double* relres_hist,
                          sc_lobpcg_info* info, void* ws, size_t ws_bytes);

/* Step API: the same solver (Section II-B) advanced one iteration per call,
 * so that a scheduler can interleave several solves (continuous batching of
 * the streaming stages of Section III, each warm-started from the previous
 * stage's eigenvectors).  The iterates live in the workspace; the same
 * buffers must be passed to every call.
 *   begin: validates, runs the initial CholQR2 / SpMM / Rayleigh-Ritz and the
 *          first residual; *done = 1 if already converged.  Synchronises.
 *   step:  one iteration; *done = 1 when converged or maxit reached.
 *          Synchronises (convergence test).
 *   end:   writes X_out, theta and info.  Synchronises. */
typedef struct sc_lobpcg_state sc_lobpcg_state;
/* step_async: enqueues one iteration (and the copy of its convergence flags
 *          to pinned host memory owned by the state) without waiting; at most
 *          one iteration per state is in flight.
 * step_poll: non-blocking; *ready = 0 while the enqueued iteration runs;
 *          once it has finished, processes its flags (errors are reported
 *          here) and sets *ready = 1 and *done.
 * Several states, each on its own context and stream, can be in flight at
 * once: their kernels overlap on the device. */
sc_status sc_lobpcg_begin(sc_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                          const int32_t* col, const void* val, const sc_lobpcg_opts* opts,
                          const void* X0, void* ws, size_t ws_bytes, sc_lobpcg_state** state,
                          int* done);
sc_status sc_lobpcg_step(sc_ctx* ctx, sc_lobpcg_state* state, int* done);
sc_status sc_lobpcg_step_async(sc_ctx* ctx, sc_lobpcg_state* state);
sc_status sc_lobpcg_step_poll(sc_ctx* ctx, sc_lobpcg_state* state, int* ready, int* done);
sc_status sc_lobpcg_end(sc_ctx* ctx, sc_lobpcg_state* state, void* X_out, double* theta,
                        double* relres_hist, sc_lobpcg_info* info);

/*
 * FP32 product Y = L X (as sc_spmm_diag, FP32) with two options for the
 * measurements of the product's memory traffic:
 *   gather  SC_GATHER_FP32: neighbour rows from X itself (the result is then
 *           bit-identical to sc_spmm_diag); SC_GATHER_FP16 / SC_GATHER_BF16:
 *           neighbour rows from Xg, a 16-bit copy of X (row stride ldg >= k,
 *           _Float16 or bfloat16), widened to FP32 on load; a row's own x_ij
 *           always comes from X.  Half the gathered bytes, at the copy's
 *           precision; where k is a multiple of 32 (at most 192) and the
 *           strides and pointers allow, every lane reads 16-byte pieces (8
 *           entries) of the copy.  SC_GATHER_FP32_LANE16: as SC_GATHER_FP32
 *           but, where k splits into 16-byte pieces over 8 or 16 lanes, every
 *           lane reads 16-byte pieces of the neighbour rows instead of 4-byte
 *           elements (the same fma chains, a bit-identical result; kept to
 *           compare the two access widths).
 *   order   NULL, or an int32 permutation of the n rows: the row groups of the
 *           launch take the rows in that order (sc_row_order gives the rows
 *           longest first, so long rows do not trail the launch).  The
 *           arithmetic of every row is unchanged.
 * No synchronisation.
 */
typedef enum {
    SC_GATHER_FP32 = 0,
    SC_GATHER_FP16 = 1,
    SC_GATHER_BF16 = 2,
    SC_GATHER_FP32_LANE16 = 3
} sc_gather;
sc_status sc_spmm_ex(sc_ctx* ctx, int64_t n, int64_t nnz, const int64_t* row_ptr,
                     const int32_t* col, const float* val, const float* diag, int k,
                     const float* X, int64_t ldx, const void* Xg, int64_t ldg, int gather,
                     const int32_t* order, float* Y, int64_t ldy);
/* order[0 .. n) = the rows by descending stored-entry count (row_ptr[i+1] -
 * row_ptr[i]), stable (equal lengths in ascending row order); a stable LSD
 * radix sort in the caller's workspace (sc_row_order_workspace bytes).
 * Requires n < 2^31.  No synchronisation. */
sc_status sc_row_order_workspace(sc_ctx* ctx, int64_t n, size_t* bytes);
sc_status sc_row_order(sc_ctx* ctx, int64_t n, const int64_t* row_ptr, int32_t* order, void* ws,
                       size_t ws_bytes);

/* ------------------------------------------------------------------------
 * Random start block (Section III: LOBPCG starts from random vectors,
 * Gaussian or uniform on [-1, 1], when no previous eigenvectors exist).
 * ------------------------------------------------------------------------ */
typedef enum { SC_RAND_NORMAL = 0, SC_RAND_UNIFORM = 1, SC_RAND_RAW = 2 } sc_rand_dist;
/*
 * Fills a rows x cols block (row stride ld >= cols elements, device memory
 * owned by the caller) from the counter-based Philox4x64-10 generator
 * (Salmon et al., SC'11) keyed by (seed, stream): word t of the stream is
 * word t mod 4 of the generator at counter t / 4 + 1, and element
 * e = row * cols + col uses
 *   SC_RAND_RAW      word e itself (out is uint64; prec ignored);
 *   SC_RAND_UNIFORM  (word e >> 11) * 2^-52 - 1, exact in [-1, 1);
 *   SC_RAND_NORMAL   Box-Muller on words 2p, 2p+1 (p = e / 2):
 *                    u1 = ((w >> 11) + 1) 2^-53, u2 = (w' >> 11) 2^-53,
 *                    r = sqrt(-2 ln u1), r cos(2 pi u2) for even e,
 *                    r sin(2 pi u2) for odd e (device log / sin / cos).
 * out is float64 for SC_PREC_FP64, float32 (rounded to nearest) otherwise.
 * Deterministic and independent of the launch shape.  Asynchronous on the
 * context's stream.  Errors: SC_E_INVAL (sizes, unknown dist or precision,
 * NULL out with rows > 0).
 */
sc_status sc_randn(sc_ctx* ctx, int64_t rows, int cols, int64_t ld, uint64_t seed,
                   uint64_t stream, int dist, void* out, sc_precision prec);

/* ------------------------------------------------------------------------
 * k-means on the row-normalised eigenvectors (Section II-A labels).
 * ------------------------------------------------------------------------ */
typedef struct {
    int n_clusters;        /* K, 1 <= K <= min(n, 1024) */
    int restarts;          /* k-means++ seedings, >= 1 */
    int max_iter;          /* Lloyd updates per restart, >= 0 */
    int normalize_rows;    /* 1: y_i = x_i / ||x_i|| (zero rows stay zero) */
    int x_fp32;            /* 1: X is float32 (widened to float64 on load), 0: float64 */
    int scan;              /* Lloyd scans of the points whose bounds fail:
                              SC_KM_SCAN_AUTO: pruned (Elkan) scans while the lists are long,
                              full scans once they are short;
                              SC_KM_SCAN_PRUNED: pruned scans whenever a list is long enough
                              to be ordered by label; SC_KM_SCAN_FULL: full scans only.
                              All three give identical results. */
} sc_kmeans_opts;
enum { SC_KM_SCAN_AUTO = 0, SC_KM_SCAN_PRUNED = 1, SC_KM_SCAN_FULL = 2 };

sc_status sc_kmeans_workspace(sc_ctx* ctx, int64_t n, int dim, const sc_kmeans_opts* opts,
                              size_t* bytes);

/*
 * Labels from k-means with k-means++ seeding (Arthur & Vassilvitskii) and
 * Lloyd iterations, the best of `restarts` runs.
 *   seeding: c_0 = y[mulhi64(u_0, n)]; for j >= 1 integer weights
 *     w_i = floor(D2_i * 2^s) (s = 61 - ceil(log2 n) - e, 2^e > 4 max ||y||^2),
 *     T = sum w, t = mulhi64(u_j, T), c_j = y[min i : prefix_i > t]
 *     (T = 0: y[mulhi64(u_j, n)]), D2_i <- min(D2_i, |y_i - c_j|^2);
 *   Lloyd: assign to the nearest centroid (squared distance accumulated with
 *     fma in dimension order, ties to the lowest index); each centroid
 *     coordinate is one FP64 sum from 0.0 over the members in ascending
 *     vertex order, divided by the member count (empty clusters keep theirs);
 *     stop when no label changes or after max_iter updates;
 *   best restart: least sum_i floor(mind_i * 2^s), ties to the lowest.
 *   X        float64 (or float32 when opts->x_fp32) n x ldx (device)
 *   draws    uint64 [restarts * K] uniform words (device), unused when
 *            init_centroids != NULL
 *   init_centroids float64 [K * dim] (device) or NULL; requires restarts = 1
 *   labels   int32 [n] (out); centroids float64 [K * dim] (out)
 *   inertia  host out (sum of squared distances, FP64), inertia_q host out
 *            (integer inertia), best_restart host out, lloyd_iterations host
 *            out (centroid updates of the slowest restart); each may be NULL.
 * Synchronises once per Lloyd iteration.
 */
sc_status sc_kmeans_assign(sc_ctx* ctx, int64_t n, int dim, const void* X, int64_t ldx,
                           const sc_kmeans_opts* opts, const uint64_t* draws,
                           const double* init_centroids, int32_t* labels, double* centroids,
                           double* inertia, uint64_t* inertia_q, int* best_restart,
                           int* lloyd_iterations, void* ws, size_t ws_bytes);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * k-means as sc_kmeans_assign, same arguments and results bit for bit, with
 * its scratch in a fixed 64 MiB device array of the library instead of a
 * caller workspace.  It calls no hipMalloc / hipFree and allocates no host
 * memory (at most 64 restarts; kernel timing must be off).  Each GPU holds
 * one copy of the array until the process ends, and every call on that GPU
 * uses it: calls that overlap on one GPU (other threads or streams) race and
 * must be serialised by the caller.  Nothing in it needs to start at zero.
 * Errors: as sc_kmeans_assign, plus SC_E_UNSUPPORTED when the problem needs
 * more than the fixed scratch (sc_kmeans_workspace > 64 MiB) or more than 64
 * restarts.
 */
sc_status sc_kmeans_assign_static(sc_ctx* ctx, int64_t n, int dim, const void* X, int64_t ldx,
                                  const sc_kmeans_opts* opts, const uint64_t* draws,
                                  const double* init_centroids, int32_t* labels,
                                  double* centroids, double* inertia, uint64_t* inertia_q,
                                  int* best_restart, int* lloyd_iterations);

/* ------------------------------------------------------------------------
 * Kernel timing on the context's stream (HIP events around every launch of
 * the selected kinds).  Used to report per-kernel durations and roofline
 * fractions; off by default.  Reading the totals synchronises the stream.
 * ------------------------------------------------------------------------ */
typedef enum {
    SC_KIND_SPMM = 0, SC_KIND_GRAM = 1, SC_KIND_RR = 2, SC_KIND_UPDATE = 3,
    SC_KIND_CHOLQR = 4, SC_KIND_RESIDUAL = 5, SC_KIND_GRAPH = 6, SC_KIND_KMEANS = 7,
    SC_KIND_GRAM_FP64ACC = 8,   /* the reduced-precision modes' FP64-accumulated Gram
                                   recomputation (a predicated launch: about 10 us when
                                   not needed) */
    SC_KIND_COUNT = 9
} sc_kernel_kind;
/* mask: bit (1 << kind) enables timing of that kind; 0 disables all. */
sc_status sc_ctx_set_profiling(sc_ctx* ctx, unsigned mask);
/* Launch count and summed duration (ms) of `kind` since the last reset. */
sc_status sc_ctx_profile(sc_ctx* ctx, int kind, int64_t* launches, double* total_ms);
sc_status sc_ctx_profile_reset(sc_ctx* ctx);

/* ------------------------------------------------------------------------
 * Warm start for a streaming stage that adds vertices (Section III: the
 * previous graph's eigenvectors start the next solve; the entries of the new
 * vertices must be filled in).  X: n x k start block (ldx >= k, float64, or
 * float32 with x_fp32 != 0), device, in place, whose rows 0 .. n_old-1 hold the
 * previous stage's block (old vertices keep their ids and come first).  Each
 * row i >= n_old becomes the mean of the rows of its neighbours j < n_old in
 * the current CSR (row_ptr, col from sc_graph_build): FP64 sum in ascending
 * column order from 0.0, divided by the count, rounded once to X's type; a new
 * vertex without such a neighbour gets a zero row.  1 <= k <= 256.  No
 * synchronisation.
 * ------------------------------------------------------------------------ */
sc_status sc_warm_fill(sc_ctx* ctx, int64_t n, int64_t n_old, const int64_t* row_ptr,
                       const int32_t* col, int k, void* X, int64_t ldx, int x_fp32);

/* ------------------------------------------------------------------------
 * Cluster labels by QR with column pivoting of the eigenvector block
 * (Section II-A: the paper reads its multi-way partition off the approximate
 * eigenvectors with a pivoted QR, the method of Damle, Minden & Ying).
 * X: n x k (ldx >= k, float64, or float32 with x_fp32 != 0), device, rows =
 * vertices; 1 <= k <= min(n, 256), n < 2^31.
 *   1. pivots: Businger-Golub over the rows of X.  res_i = ||x_i||^2; step s
 *      takes p_s = argmax res_i over rows not yet chosen (ties: lowest i),
 *      a_t = q_t . x_{p_s} (t < s), r = x_{p_s} - sum_t a_t q_t, q_s =
 *      r / ||r||, then res_i = fma(-c, c, res_i) with c = q_s . x_i; every dot
 *      product is the ordered fma chain over the coordinates;
 *   2. Q = orthogonal polar factor of B' (B = pivot rows): B B' = W diag(l) W',
 *      Q = B' W diag(1/sqrt l) W';
 *   3. labels_i = argmax_j |(X Q)_ij| (ties: lowest j).
 * pivots int32 [k], labels int32 [n], Q float64 k x k row-major (Q[d*k+j]),
 * all device outputs.  Synchronises.  A block of rank below k (a chosen
 * squared residual at or below 1e-10 of the first pivot's, i.e. 1e-5 relative
 * in norm, or an eigenvalue of B B' that is not positive) is SC_E_BREAKDOWN;
 * NaN or Inf in X is SC_E_NUMERIC.
 * ------------------------------------------------------------------------ */
sc_status sc_cpqr_workspace(sc_ctx* ctx, int64_t n, int k, int x_fp32, size_t* bytes);

/*
 * Number of clusters from the gap in the smallest eigenvalues (Section II-A:
 * the count of eigenvalues below the first significantly large increment).
 * theta float64 [k] ascending (device, e.g. the Ritz values of a solve with
 * k above the expected count), 1 <= k <= 256.  With g_j = theta_{j+1} -
 * theta_j, the gap is the first j >= 1 with g_j > 1e-8 (theta_{k-1} - theta_0)
 * and g_j > sig * mean(g_0 .. g_{j-1}) (sig > 0, e.g. 10), else the largest
 * g_j (first of equals);
 * count (int32, device, out) = j + 1 (1 when k == 1); ratio (float64, device,
 * out) = g_j / median(g), large for a clear gap.  No synchronisation.
 */
sc_status sc_eigengap(sc_ctx* ctx, int k, const double* theta, double sig, int* count,
                      double* ratio);
sc_status sc_cpqr_labels(sc_ctx* ctx, int64_t n, int k, const void* X, int64_t ldx, int x_fp32,
                         int32_t* pivots, int32_t* labels, double* Q, void* ws, size_t ws_bytes);

/* ------------------------------------------------------------------------
 * Dense FP64 symmetric eigensolver used inside the Rayleigh-Ritz step,
 * exposed for testing: the k smallest eigenpairs of the m x m symmetric A
 * (row-major, device).  w float64 [k] ascending, V float64 m x k row-major
 * (device, out).  m <= 1024.
 * ------------------------------------------------------------------------ */
sc_status sc_symeig_workspace(sc_ctx* ctx, int m, int k, size_t* bytes);
sc_status sc_symeig(sc_ctx* ctx, int m, int k, const double* A, double* w, double* V,
                    void* ws, size_t ws_bytes);

#ifdef __cplusplus
}
#endif
#endif /* SPECTRAL_H */
