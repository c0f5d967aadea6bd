/*
 * Plain FP64 CPU oracle for the spectral-clustering path of
 * "Preconditioned Spectral Clustering for Stochastic Block Partition
 * Streaming Graph Challenge" (Zhuzhunashvili & Knyazev).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  It shares no code with
 * the GPU library and must never be called from the product path; only the
 * tests, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Conventions
 *   - every multivector is stored column-major inside the oracle
 *     (column j of V is V[j*n .. j*n+n-1]); the Python wrapper converts;
 *   - every inner product / accumulation is a sequential sum in index order
 *     with fused multiply-add, no blocking, no reordering;
 *   - OpenMP (when enabled) only distributes independent outputs (rows, or
 *     matrix entries); the arithmetic of every output is unchanged, so the
 *     results do not depend on the thread count;
 *   - built with -O2 -ffp-contract=off and no fast-math.
 *
 * Contents
 *   orc_graph_build   symmetrisation W + W' (Section II-A): logical sum for
 *                     unweighted graphs, algebraic sum for weighted ones
 *   orc_laplacian     normalised Laplacian I - D^-1/2 W D^-1/2 of W's pattern
 *   orc_laplacian_combinatorial
 *                     the graph Laplacian L = D - W as Section II-A introduces it
 *                     (off-diagonal -w, diagonal the degrees)
 *   orc_spmm          Y = L X, the one matrix product per iteration (Section III)
 *   orc_gram, orc_cholesky, orc_symeig (cyclic Jacobi)  dense helpers
 *   orc_lobpcg        block LOBPCG without preconditioning (Section II-B,
 *                     Section III; Knyazev 2001 with explicit Gram basis)
 *   orc_kmeans        row normalisation + k-means++ seeding + Lloyd
 *                     (Section II-A names k-means++ as the classic labelling)
 *   orc_cpqr_labels   labels by QR with column pivoting of the eigenvector
 *                     block (Section II-A's own labelling)
 *   orc_eigengap      number of clusters from the gap in the eigenvalues
 *   orc_warm_fill     start rows of the vertices a streaming stage adds
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORC_OK 0
#define ORC_E_INVAL (-1)
#define ORC_E_NOMEM (-2)
#define ORC_E_BREAKDOWN (-4)
#define ORC_E_NUMERIC (-5)

/* Wall-clock seconds (timing of the CPU baseline only; no arithmetic uses it). */
static double orc_now(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* Progress lines on stderr when the environment sets ORC_TRACE (long runs). */
static int orc_trace(void) {
    static int v = -1;
    if (v < 0) v = getenv("ORC_TRACE") != NULL;
    return v;
}

/* ------------------------------------------------------------------------ */
/* Graph symmetrisation (Section II-A).                                      */
/* ------------------------------------------------------------------------ */

typedef struct { int32_t col; int64_t slot; double w; } orc_entry;

static int entry_cmp(const void* a, const void* b) {
    const orc_entry* x = (const orc_entry*)a;
    const orc_entry* y = (const orc_entry*)b;
    if (x->col != y->col) return x->col < y->col ? -1 : 1;
    if (x->slot != y->slot) return x->slot < y->slot ? -1 : 1;
    return 0;
}

/*
 * Directed COO (src[e] -> dst[e], weight w[e] or 1 when w == NULL) to the CSR
 * of the symmetric W + W'.  Edge e contributes (src,dst) and (dst,src); self
 * loops are dropped and counted.  Entries of one (row,col) are merged: the
 * logical sum gives weight 1, the algebraic sum adds the weights in the order
 * edge 0 forward, edge 0 backward, edge 1 forward, ...  Columns ascend in
 * every row.  degree[i] = sum of row i of W in ascending column order.
 * col / w_sym need room for 2m entries; w_sym may be NULL.
 */
int orc_graph_build(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                    const double* w, int algebraic, int64_t* row_ptr, int32_t* col,
                    double* w_sym, double* degree, int64_t* nnz_out, int64_t* self_loops_out) {
    if (n <= 0 || m < 0) return ORC_E_INVAL;
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return ORC_E_INVAL;
        if (w && (!(w[e] >= 0.0) || !isfinite(w[e]))) return ORC_E_INVAL;
    }
    int64_t* count = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    orc_entry* ent = (orc_entry*)malloc(sizeof(orc_entry) * (size_t)(2 * m + 1));
    if (!count || !ent) { free(count); free(ent); return ORC_E_NOMEM; }
    int64_t loops = 0;
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] == dst[e]) { ++loops; continue; }
        count[src[e] + 1]++;
        count[dst[e] + 1]++;
    }
    for (int64_t i = 0; i < n; ++i) count[i + 1] += count[i];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!fill) { free(count); free(ent); return ORC_E_NOMEM; }
    for (int64_t i = 0; i < n; ++i) fill[i] = count[i];
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] == dst[e]) continue;
        double we = w ? w[e] : 1.0;
        orc_entry a = {dst[e], 2 * e, we};
        orc_entry b = {src[e], 2 * e + 1, we};
        ent[fill[src[e]]++] = a;
        ent[fill[dst[e]]++] = b;
    }
    int64_t nnz = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t lo = count[i], hi = count[i + 1];
        qsort(ent + lo, (size_t)(hi - lo), sizeof(orc_entry), entry_cmp);
        double deg = 0.0;
        for (int64_t p = lo; p < hi;) {
            int64_t q = p;
            double acc = 0.0;
            while (q < hi && ent[q].col == ent[p].col) { acc += ent[q].w; ++q; }
            double val = algebraic ? acc : 1.0;
            col[nnz] = ent[p].col;
            if (w_sym) w_sym[nnz] = val;
            deg += val;
            ++nnz;
            p = q;
        }
        degree[i] = deg;
        row_ptr[i + 1] = nnz;
    }
    *nnz_out = nnz;
    if (self_loops_out) *self_loops_out = loops;
    free(count); free(ent); free(fill);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Normalised Laplacian L = I - D^-1/2 W D^-1/2 (values of the off-diagonal  */
/* pattern; the unit diagonal is implicit).                                  */
/* ------------------------------------------------------------------------ */
int orc_laplacian(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* w_sym,
                  const double* degree, double* val, double* dinv_sqrt) {
    if (n <= 0) return ORC_E_INVAL;
    for (int64_t i = 0; i < n; ++i) {
        double di = degree[i];
        dinv_sqrt[i] = di > 0.0 ? 1.0 / sqrt(di) : 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            double dj = degree[col[p]];
            double wp = w_sym ? w_sym[p] : 1.0;
            double prod = di * dj;
            val[p] = prod > 0.0 ? -(wp / sqrt(prod)) : 0.0;
        }
    }
    return ORC_OK;
}

/*
 * The graph Laplacian L = D - W (Section II-A; the diagonal entries are the
 * vertex degrees, as the pre-computed diagonal of the matrix-free product in
 * Section III).  Off-diagonal value -w_p, exact.
 */
int orc_laplacian_combinatorial(int64_t n, const int64_t* row_ptr, const int32_t* col,
                                const double* w_sym, double* val) {
    if (n <= 0) return ORC_E_INVAL;
    (void)col;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) val[p] = -(w_sym ? w_sym[p] : 1.0);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Y = L X with L = diag(a) + offdiag(val): y_ij = a_i x_ij (one rounded     */
/* product; a_i = 1, i.e. y_ij = x_ij, when diag is NULL: the normalised     */
/* Laplacian), then, over row i in ascending column order,                   */
/* y_ij = fma(v_p, x_{col_p j}, y_ij).                                        */
/* Row-major entry point (ld = row stride) used directly by the tests.       */
/* ------------------------------------------------------------------------ */
void orc_spmm_rowmajor(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                       const double* diag, int k, const double* X, int64_t ldx, double* Y,
                       int64_t ldy) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        for (int j = 0; j < k; ++j) {
            double acc = diag ? diag[i] * X[i * ldx + j] : X[i * ldx + j];
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                acc = fma(val[p], X[(int64_t)col[p] * ldx + j], acc);
            Y[i * ldy + j] = acc;
        }
    }
}

/* Column-major variant used inside the oracle's LOBPCG (same arithmetic). */
static void spmm_cm(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                    const double* diag, int k, const double* X, double* Y) {
    for (int j = 0; j < k; ++j) {
        const double* x = X + (int64_t)j * n;
        double* y = Y + (int64_t)j * n;
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n; ++i) {
            double acc = diag ? diag[i] * x[i] : x[i];
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) acc = fma(val[p], x[col[p]], acc);
            y[i] = acc;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Dense helpers.  Small matrices are row-major: A[r*ld + c].                */
/* ------------------------------------------------------------------------ */

static double dot_cm(int64_t n, const double* a, const double* b) {
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc = fma(a[i], b[i], acc);
    return acc;
}

/* G = A^T B for column-major n x ca and n x cb multivectors; when sym != 0
 * (A == B or the caller wants A^T B symmetrised) only the upper triangle is
 * formed and mirrored. */
static void gram_cm(int64_t n, int ca, const double* A, int cb, const double* B, double* G, int sym) {
    int64_t pairs = (int64_t)ca * cb;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < pairs; ++t) {
        int a = (int)(t / cb), b = (int)(t % cb);
        if (sym && b < a) continue;
        G[(int64_t)a * cb + b] = dot_cm(n, A + (int64_t)a * n, B + (int64_t)b * n);
    }
    if (sym)
        for (int a = 0; a < ca; ++a)
            for (int b = 0; b < a; ++b) G[(int64_t)a * cb + b] = G[(int64_t)b * cb + a];
}

void orc_gram(int64_t n, int ca, const double* A, int cb, const double* B, double* G, int sym) {
    gram_cm(n, ca, A, cb, B, G, sym);
}

/*
 * Upper Cholesky G = R^T R of an m x m symmetric matrix (row-major, ld m).
 * Fails (returns 0) when a pivot is not finite or is not larger than
 * tol * G_jj, i.e. when the column is numerically in the span of the previous
 * ones.  R's strictly lower part is set to zero.
 */
static int cholesky_upper(int m, const double* G, double* R, double tol) {
    memset(R, 0, sizeof(double) * (size_t)m * (size_t)m);
    for (int j = 0; j < m; ++j) {
        double s = G[(int64_t)j * m + j];
        for (int l = 0; l < j; ++l) s = fma(-R[(int64_t)l * m + j], R[(int64_t)l * m + j], s);
        if (!isfinite(s) || !(s > tol * G[(int64_t)j * m + j]) || !(s > 0.0)) return 0;
        double rjj = sqrt(s);
        R[(int64_t)j * m + j] = rjj;
        for (int b = j + 1; b < m; ++b) {
            double t = G[(int64_t)j * m + b];
            for (int l = 0; l < j; ++l) t = fma(-R[(int64_t)l * m + j], R[(int64_t)l * m + b], t);
            R[(int64_t)j * m + b] = t / rjj;
        }
    }
    return 1;
}

int orc_cholesky(int m, const double* G, double* R, double tol) {
    return cholesky_upper(m, G, R, tol) ? ORC_OK : ORC_E_BREAKDOWN;
}

/* Inverse of an upper-triangular m x m matrix by back substitution. */
static void upper_inverse(int m, const double* R, double* Ri) {
    memset(Ri, 0, sizeof(double) * (size_t)m * (size_t)m);
    for (int j = 0; j < m; ++j) {
        Ri[(int64_t)j * m + j] = 1.0 / R[(int64_t)j * m + j];
        for (int a = j - 1; a >= 0; --a) {
            double s = 0.0;
            for (int l = a + 1; l <= j; ++l) s = fma(R[(int64_t)a * m + l], Ri[(int64_t)l * m + j], s);
            Ri[(int64_t)a * m + j] = -s / R[(int64_t)a * m + a];
        }
    }
}

/*
 * Symmetric eigendecomposition by the cyclic Jacobi method (Golub & Van Loan,
 * Matrix Computations, sym.schur2 rotations swept row by row).  A is m x m
 * row-major and symmetric; on return w holds the eigenvalues in ascending
 * order and V (row-major, m x m) the matching eigenvectors in its columns.
 * Sweeps stop when the off-diagonal Frobenius mass is below 1e-30 of the
 * total, or after 100 sweeps.
 */
int orc_symeig(int m, const double* A_in, double* w, double* V) {
    double* A = (double*)malloc(sizeof(double) * (size_t)m * (size_t)m);
    double* U = (double*)malloc(sizeof(double) * (size_t)m * (size_t)m);
    int* ord = (int*)malloc(sizeof(int) * (size_t)m);
    if (!A || !U || !ord) { free(A); free(U); free(ord); return ORC_E_NOMEM; }
    memcpy(A, A_in, sizeof(double) * (size_t)m * (size_t)m);
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) U[(int64_t)r * m + c] = (r == c) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int r = 0; r < m; ++r)
            for (int c = 0; c < m; ++c) {
                double a = A[(int64_t)r * m + c];
                tot += a * a;
                if (r != c) off += a * a;
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < m - 1; ++p) {
            for (int q = p + 1; q < m; ++q) {
                double apq = A[(int64_t)p * m + q];
                if (apq == 0.0) continue;
                double app = A[(int64_t)p * m + p], aqq = A[(int64_t)q * m + q];
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                /* A <- J^T A J with J the rotation in the (p,q) plane */
                for (int r = 0; r < m; ++r) {
                    double arp = A[(int64_t)r * m + p], arq = A[(int64_t)r * m + q];
                    A[(int64_t)r * m + p] = c * arp - s * arq;
                    A[(int64_t)r * m + q] = s * arp + c * arq;
                }
                for (int r = 0; r < m; ++r) {
                    double apr = A[(int64_t)p * m + r], aqr = A[(int64_t)q * m + r];
                    A[(int64_t)p * m + r] = c * apr - s * aqr;
                    A[(int64_t)q * m + r] = s * apr + c * aqr;
                }
                A[(int64_t)p * m + q] = 0.0;
                A[(int64_t)q * m + p] = 0.0;
                for (int r = 0; r < m; ++r) {
                    double urp = U[(int64_t)r * m + p], urq = U[(int64_t)r * m + q];
                    U[(int64_t)r * m + p] = c * urp - s * urq;
                    U[(int64_t)r * m + q] = s * urp + c * urq;
                }
            }
        }
    }
    /* ascending order, ties by original index (insertion sort, stable) */
    for (int i = 0; i < m; ++i) ord[i] = i;
    for (int i = 1; i < m; ++i) {
        int v = ord[i], j = i - 1;
        while (j >= 0 && A[(int64_t)ord[j] * m + ord[j]] > A[(int64_t)v * m + v]) { ord[j + 1] = ord[j]; --j; }
        ord[j + 1] = v;
    }
    for (int i = 0; i < m; ++i) {
        w[i] = A[(int64_t)ord[i] * m + ord[i]];
        for (int r = 0; r < m; ++r) V[(int64_t)r * m + i] = U[(int64_t)r * m + ord[i]];
    }
    free(A); free(U); free(ord);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* LOBPCG without preconditioning (Section II-B: the block method, one       */
/* product with L per iteration; Section III: no preconditioner, random or   */
/* warm start X0).                                                           */
/* ------------------------------------------------------------------------ */

/*
 * Cholesky QR with column equilibration of the n x k column-major block V
 * restricted to the columns with act[j] != 0:
 *   G = V^T V;  columns with G_jj == 0 (or not finite) become inactive;
 *   d_j = sqrt(G_jj);  Ghat = D^-1 G D^-1;  Ghat = R^T R (upper);
 *   T = D^-1 R^-1;  V <- V T  (inactive columns become exactly zero).
 * When V2 != NULL the same T is applied to V2 (the block L V).
 * Returns 1 on success, 0 on Cholesky failure (V, V2 untouched).
 */
static int cholqr_masked(int64_t n, int k, double* V, double* V2, int* act, double tol) {
    double* G = (double*)malloc(sizeof(double) * (size_t)k * k);
    int* idx = (int*)malloc(sizeof(int) * (size_t)k);
    gram_cm(n, k, V, k, V, G, 1);
    int m = 0;
    for (int j = 0; j < k; ++j) {
        double g = G[(int64_t)j * k + j];
        if (act[j] && isfinite(g) && g > 0.0) idx[m++] = j;
        else act[j] = 0;
    }
    double* Gs = (double*)malloc(sizeof(double) * (size_t)(m ? m : 1) * (m ? m : 1));
    double* R = (double*)malloc(sizeof(double) * (size_t)(m ? m : 1) * (m ? m : 1));
    double* Ri = (double*)malloc(sizeof(double) * (size_t)(m ? m : 1) * (m ? m : 1));
    double* d = (double*)malloc(sizeof(double) * (size_t)(m ? m : 1));
    int ok = 1;
    for (int a = 0; a < m; ++a) d[a] = sqrt(G[(int64_t)idx[a] * k + idx[a]]);
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b)
            Gs[(int64_t)a * m + b] = G[(int64_t)idx[a] * k + idx[b]] / (d[a] * d[b]);
    if (m > 0 && !cholesky_upper(m, Gs, R, tol)) ok = 0;
    if (ok) {
        upper_inverse(m, R, Ri);
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) Ri[(int64_t)a * m + b] /= d[a];
        /* V <- V T, column j of the result = sum_{a<=j} V_a T_aj in index order */
        for (int pass = 0; pass < (V2 ? 2 : 1); ++pass) {
            double* B = pass ? V2 : V;
            double* out = (double*)calloc((size_t)n * (size_t)k, sizeof(double));
            for (int jb = 0; jb < m; ++jb) {
                double* y = out + (int64_t)idx[jb] * n;
                for (int a = 0; a <= jb; ++a) {
                    const double* x = B + (int64_t)idx[a] * n;
                    double t = Ri[(int64_t)a * m + jb];
#pragma omp parallel for schedule(static)
                    for (int64_t i = 0; i < n; ++i) y[i] = fma(x[i], t, y[i]);
                }
            }
            memcpy(B, out, sizeof(double) * (size_t)n * (size_t)k);
            free(out);
        }
    }
    free(G); free(idx); free(Gs); free(R); free(Ri); free(d);
    return ok;
}

/*
 * Rayleigh-Ritz on the active columns of S = [X W P] (3k columns):
 *   B = G_B[act,act] = U^T U (upper Cholesky; on failure with P active, P is
 *   dropped and B is rebuilt; a second failure is a breakdown);
 *   M = U^-T A U^-1 with A = G_A[act,act], symmetrised (M + M^T)/2;
 *   M = Q Theta Q^T (ascending);  C_act = U^-1 Q[:, :k];  theta = Theta[:k].
 * C is 3k x k row-major; rows of inactive columns are zero.
 */
static int rayleigh_ritz(int k, const double* GA, const double* GB, int* act3, double* C,
                         double* theta, int* p_dropped, double tol) {
    int K3 = 3 * k;
    int* idx = (int*)malloc(sizeof(int) * (size_t)K3);
    double* B = (double*)malloc(sizeof(double) * (size_t)K3 * K3);
    double* U = (double*)malloc(sizeof(double) * (size_t)K3 * K3);
    double* Ui = (double*)malloc(sizeof(double) * (size_t)K3 * K3);
    double* T = (double*)malloc(sizeof(double) * (size_t)K3 * K3);
    double* M = (double*)malloc(sizeof(double) * (size_t)K3 * K3);
    double* Q = (double*)malloc(sizeof(double) * (size_t)K3 * K3);
    double* w = (double*)malloc(sizeof(double) * (size_t)K3);
    int status = ORC_OK, m = 0;
    *p_dropped = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        m = 0;
        for (int j = 0; j < K3; ++j) if (act3[j]) idx[m++] = j;
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) B[(int64_t)a * m + b] = GB[(int64_t)idx[a] * K3 + idx[b]];
        if (cholesky_upper(m, B, U, tol)) break;
        int has_p = 0;
        for (int j = 2 * k; j < K3; ++j) has_p |= act3[j];
        if (!has_p || attempt == 1) { status = ORC_E_BREAKDOWN; goto done; }
        for (int j = 2 * k; j < K3; ++j) act3[j] = 0;
        *p_dropped = 1;
    }
    upper_inverse(m, U, Ui);
    /* T = A U^-1 */
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            double s = 0.0;
            for (int l = 0; l <= b; ++l) s = fma(GA[(int64_t)idx[a] * K3 + idx[l]], Ui[(int64_t)l * m + b], s);
            T[(int64_t)a * m + b] = s;
        }
    /* M = U^-T T */
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            double s = 0.0;
            for (int l = 0; l <= a; ++l) s = fma(Ui[(int64_t)l * m + a], T[(int64_t)l * m + b], s);
            M[(int64_t)a * m + b] = s;
        }
    for (int a = 0; a < m; ++a)
        for (int b = a + 1; b < m; ++b) {
            double s = 0.5 * (M[(int64_t)a * m + b] + M[(int64_t)b * m + a]);
            M[(int64_t)a * m + b] = s;
            M[(int64_t)b * m + a] = s;
        }
    status = orc_symeig(m, M, w, Q);
    if (status != ORC_OK) goto done;
    memset(C, 0, sizeof(double) * (size_t)K3 * k);
    for (int a = 0; a < m; ++a)
        for (int j = 0; j < k; ++j) {
            double s = 0.0;
            for (int l = a; l < m; ++l) s = fma(Ui[(int64_t)a * m + l], Q[(int64_t)l * m + j], s);
            C[(int64_t)idx[a] * k + j] = s;
        }
    for (int j = 0; j < k; ++j) theta[j] = w[j];
done:
    free(idx); free(B); free(U); free(Ui); free(T); free(M); free(Q); free(w);
    return status;
}

typedef struct {
    int k;
    int maxit;
    double tol;        /* converged when max_j relres_j <= tol */
    double lock_tol;   /* columns with relres_j <= lock_tol leave the W block */
    double chol_tol;   /* relative pivot floor of every Cholesky */
    double op_norm;    /* upper bound of ||L|| scaling the relative residual (0: 2) */
    int k_conv;        /* the convergence test covers columns 0 .. k_conv-1 (0: all k);
                          a block wider than the wanted pairs (Section IV: l > k) */
} orc_lobpcg_opts;

typedef struct {
    int iterations;    /* Rayleigh-Ritz updates after the initial one (= SpMMs of W) */
    int converged;
    int p_drops;
    int locked_cols;   /* W columns left out in the last iteration */
    double max_relres; /* of the returned X */
    double seconds_setup;  /* wall time of CholQR2(X0), L X, the first Rayleigh-Ritz step
                              and residual */
    double seconds_iters;  /* wall time of the iterations after it */
} orc_lobpcg_info;

/*
 * Smallest-k eigenpairs of L = diag(a) + offdiag(val) by block LOBPCG with
 * T = I: the normalised Laplacian (diag NULL, a = 1) or L = D - W (diag the
 * degrees).  X0 and X_out are row-major n x k (ld k).  relres_hist (optional)
 * receives (iterations+1) rows of k relative residuals
 *   relres_j = ||L x_j - theta_j x_j|| / (N ||x_j||),  N = op_norm >= ||L||
 * (N = 2 for the normalised Laplacian; 2 max_i d_i bounds D - W, Gershgorin);
 * theta_hist (optional) receives the Ritz values after every RR step
 * (iterations+1 rows).  Both need room for (maxit+1)*k doubles.
 */
int orc_lobpcg(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
               const double* diag, const orc_lobpcg_opts* o, const double* X0, double* X_out, double* theta,
               double* relres_hist, double* theta_hist, orc_lobpcg_info* info) {
    int k = o->k, K3 = 3 * o->k;
    const double opn = o->op_norm > 0.0 ? o->op_norm : 2.0;
    if (n <= 0 || k < 1 || (int64_t)K3 > n || o->maxit < 0) return ORC_E_INVAL;
    for (int64_t i = 0; i < n * k; ++i) if (!isfinite(X0[i])) return ORC_E_NUMERIC;
    size_t blk = (size_t)n * (size_t)k;
    double* S = (double*)calloc(3 * blk, sizeof(double));   /* [X W P] column-major */
    double* LS = (double*)calloc(3 * blk, sizeof(double));  /* [LX LW LP] */
    double* GA = (double*)malloc(sizeof(double) * (size_t)K3 * K3);
    double* GB = (double*)malloc(sizeof(double) * (size_t)K3 * K3);
    double* C = (double*)malloc(sizeof(double) * (size_t)K3 * k);
    double* Xn = (double*)malloc(sizeof(double) * blk);
    double* LXn = (double*)malloc(sizeof(double) * blk);
    double* rho = (double*)malloc(sizeof(double) * (size_t)k);
    double* relres = (double*)malloc(sizeof(double) * (size_t)k);
    int* act3 = (int*)malloc(sizeof(int) * (size_t)K3);
    if (!S || !LS || !GA || !GB || !C || !Xn || !LXn || !rho || !relres || !act3) return ORC_E_NOMEM;
    double *X = S, *W = S + blk, *P = S + 2 * blk;
    double *LX = LS, *LW = LS + blk, *LP = LS + 2 * blk;
    int status = ORC_OK, p_dropped = 0;
    orc_lobpcg_info inf = {0, 0, 0, 0, 0.0, 0.0, 0.0};
    const double t_start = orc_now();
    double t_mark = t_start;

    for (int64_t i = 0; i < n; ++i)
        for (int j = 0; j < k; ++j) X[(int64_t)j * n + i] = X0[i * k + j];
    /* X <- CholQR2(X0) */
    for (int rep = 0; rep < 2; ++rep) {
        for (int j = 0; j < k; ++j) act3[j] = 1;
        if (!cholqr_masked(n, k, X, NULL, act3, o->chol_tol)) { status = ORC_E_BREAKDOWN; goto out; }
        for (int j = 0; j < k; ++j) if (!act3[j]) { status = ORC_E_BREAKDOWN; goto out; }
    }
    spmm_cm(n, row_ptr, col, val, diag, k, X, LX);

    /* Rayleigh-Ritz on span(X) alone; then the main loop */
    int has_p = 0;
    for (int t = 0;; ++t) {
        for (int j = 0; j < K3; ++j) act3[j] = 0;
        if (t == 0) {
            for (int j = 0; j < k; ++j) act3[j] = 1;
        } else {
            /* residual R = LX - X theta stored in W, its norms, relres */
            for (int j = 0; j < k; ++j) act3[j] = 1;
            int any_w = 0;
            for (int j = 0; j < k; ++j) {
                int wj = relres[j] > o->lock_tol;
                act3[k + j] = wj;
                any_w |= wj;
                if (!wj) {
                    double* wc = W + (int64_t)j * n;
                    for (int64_t i = 0; i < n; ++i) wc[i] = 0.0;
                }
            }
            inf.locked_cols = 0;
            for (int j = 0; j < k; ++j) inf.locked_cols += !act3[k + j];
            (void)any_w;
            if (!cholqr_masked(n, k, W, NULL, act3 + k, o->chol_tol)) { status = ORC_E_BREAKDOWN; goto out; }
            spmm_cm(n, row_ptr, col, val, diag, k, W, LW);
            if (has_p) {
                for (int j = 0; j < k; ++j) act3[2 * k + j] = 1;
                if (!cholqr_masked(n, k, P, LP, act3 + 2 * k, o->chol_tol)) {
                    for (int j = 0; j < k; ++j) act3[2 * k + j] = 0;
                    memset(P, 0, sizeof(double) * blk);
                    memset(LP, 0, sizeof(double) * blk);
                    inf.p_drops++;
                }
            }
        }
        gram_cm(n, K3, S, K3, LS, GA, 1);
        gram_cm(n, K3, S, K3, S, GB, 1);
        if (orc_trace())
            fprintf(stderr, "[oracle lobpcg] t=%d Gram products done (%.1f s)\n", t, orc_now() - t_mark);
        status = rayleigh_ritz(k, GA, GB, act3, C, theta, &p_dropped, o->chol_tol);
        if (status != ORC_OK) goto out;
        if (p_dropped) inf.p_drops++;
        if (theta_hist) for (int j = 0; j < k; ++j) theta_hist[(int64_t)t * k + j] = theta[j];
        /* P <- [W P] C_WP, LP <- [LW LP] C_WP, X <- X C_X + P, LX <- LX C_X + LP */
        for (int pass = 0; pass < 2; ++pass) {
            double* Sb = pass ? LS : S;
            double* Pn = pass ? LP : P;
            double* Xb = pass ? LX : X;
            double* out = pass ? LXn : Xn;
            double* tmpP = (double*)calloc(blk, sizeof(double));
            for (int j = 0; j < k; ++j) {
                double* y = tmpP + (int64_t)j * n;
                for (int l = k; l < K3; ++l) {
                    double c = C[(int64_t)l * k + j];
                    const double* x = Sb + (int64_t)l * n;
#pragma omp parallel for schedule(static)
                    for (int64_t i = 0; i < n; ++i) y[i] = fma(x[i], c, y[i]);
                }
                double* z = out + (int64_t)j * n;
                for (int64_t i = 0; i < n; ++i) z[i] = 0.0;
                for (int l = 0; l < k; ++l) {
                    double c = C[(int64_t)l * k + j];
                    const double* x = Xb + (int64_t)l * n;
#pragma omp parallel for schedule(static)
                    for (int64_t i = 0; i < n; ++i) z[i] = fma(x[i], c, z[i]);
                }
                for (int64_t i = 0; i < n; ++i) z[i] = z[i] + y[i];
            }
            memcpy(Xb, out, sizeof(double) * blk);
            memcpy(Pn, tmpP, sizeof(double) * blk);
            free(tmpP);
        }
        if (t > 0) has_p = 1;
        inf.iterations = t;

        /* residual of the new iterate */
        for (int j = 0; j < k; ++j) {
            const double* x = X + (int64_t)j * n;
            const double* lx = LX + (int64_t)j * n;
            double* r = W + (int64_t)j * n;
            double th = theta[j];
            double rr = 0.0, xx = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                double ri = fma(-th, x[i], lx[i]);
                r[i] = ri;
                rr = fma(ri, ri, rr);
                xx = fma(x[i], x[i], xx);
            }
            rho[j] = sqrt(rr);
            relres[j] = rho[j] / (opn * sqrt(xx));
        }
        double mx = 0.0;
        int all_locked = 1;
        const int kc = (o->k_conv > 0 && o->k_conv < k) ? o->k_conv : k;
        for (int j = 0; j < k; ++j) {
            if (!isfinite(relres[j])) { status = ORC_E_NUMERIC; goto out; }
            if (j < kc && relres[j] > mx) mx = relres[j];
            if (relres[j] > o->lock_tol) all_locked = 0;
        }
        if (relres_hist) for (int j = 0; j < k; ++j) relres_hist[(int64_t)t * k + j] = relres[j];
        inf.max_relres = mx;
        {
            const double now = orc_now();
            if (t == 0) inf.seconds_setup = now - t_start;
            else inf.seconds_iters = now - t_start - inf.seconds_setup;
            if (orc_trace())
                fprintf(stderr, "[oracle lobpcg] n=%lld k=%d t=%d max relres %.3e (%.1f s)\n",
                        (long long)n, k, t, mx, now - t_mark);
            t_mark = now;
        }
        if (mx <= o->tol || all_locked) { inf.converged = 1; break; }
        if (t == o->maxit) break;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int j = 0; j < k; ++j) X_out[i * k + j] = X[(int64_t)j * n + i];
out:
    if (info) *info = inf;
    free(S); free(LS); free(GA); free(GB); free(C); free(Xn); free(LXn); free(rho); free(relres); free(act3);
    return status;
}

/* ------------------------------------------------------------------------ */
/* k-means on the row-normalised eigenvectors (Section II-A: the labels come */
/* from the approximate eigenvectors; k-means++ seeding, Arthur &            */
/* Vassilvitskii 2007, followed by Lloyd iterations).                        */
/* ------------------------------------------------------------------------ */

static uint64_t mulhi64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

static int ceil_log2_u64(uint64_t v) {
    int e = 0;
    while (((uint64_t)1 << e) < v) ++e;
    return e;
}

/* squared distance, fma-accumulated in dimension order */
static double sqdist(int dim, const double* y, const double* c) {
    double acc = 0.0;
    for (int d = 0; d < dim; ++d) {
        double diff = y[d] - c[d];
        acc = fma(diff, diff, acc);
    }
    return acc;
}

/*
 * Exact integer weight of a squared distance: floor(D2 * 2^shift), shift
 * chosen so that n weights of at most 2^(61 - ceil(log2 n)) sum below 2^62.
 */
static uint64_t qweight(double d2, int shift) {
    return (uint64_t)floor(ldexp(d2, shift));
}

/*
 * Row normalisation then k-means with `restarts` k-means++ seedings and up to
 * max_iter Lloyd updates each.  draws[r*K + j] are uniform 64-bit words.
 *   normalise: y_i = x_i / ||x_i|| (IEEE division), zero rows stay zero;
 *   seeding:   c_0 = y[mulhi(u_0, n)]; then with integer weights
 *              w_i = floor(D2_i 2^s), T = sum w, t = mulhi(u_j, T),
 *              c_j = y[min i : prefix_i > t] (T == 0: y[mulhi(u_j, n)]);
 *   Lloyd:     assign (argmin, ties to the lowest cluster), update centroids
 *              (each dimension is one FP64 sum from 0.0 over the members in
 *              ascending vertex order, divided by the member count; an empty
 *              cluster keeps its centroid), stop when no label changes;
 *   choice:    restart with the least integer inertia sum_i floor(mind_i 2^s),
 *              ties to the lowest restart.
 * timing (optional, [4]): wall seconds of the row normalisation, of the
 * seedings with their first assignments, of the Lloyd updates, and the number
 * of Lloyd updates, all restarts together.
 * If init_centroids != NULL it replaces the seeding (restarts must be 1).
 */
int orc_kmeans(int64_t n, int dim, const double* X, int64_t ldx, int K, int restarts, int max_iter,
               const uint64_t* draws, const double* init_centroids, int normalize,
               int32_t* labels, double* centroids, double* inertia, uint64_t* inertia_q,
               int* best_restart, int* lloyd_iters, double* timing) {
    if (n <= 0 || dim <= 0 || K <= 0 || K > n || restarts <= 0 || max_iter < 0 || ldx < dim)
        return ORC_E_INVAL;
    if (init_centroids && restarts != 1) return ORC_E_INVAL;
    double* Y = (double*)malloc(sizeof(double) * (size_t)n * dim);
    double* Cc = (double*)malloc(sizeof(double) * (size_t)K * dim);
    double* D2 = (double*)malloc(sizeof(double) * (size_t)n);
    uint64_t* pref = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    int32_t* lab = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* nl = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)K);
    if (!Y || !Cc || !D2 || !pref || !lab || !nl || !cnt) return ORC_E_NOMEM;
    double t_norm = orc_now(), t_seed = 0.0, t_lloyd = 0.0, n_lloyd = 0.0;
    double m2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double* x = X + i * ldx;
        double* y = Y + i * dim;
        for (int d = 0; d < dim; ++d) if (!isfinite(x[d])) return ORC_E_NUMERIC;
        if (normalize) {
            double s = 0.0;
            for (int d = 0; d < dim; ++d) s = fma(x[d], x[d], s);
            double nrm = sqrt(s);
            for (int d = 0; d < dim; ++d) y[d] = nrm > 0.0 ? x[d] / nrm : 0.0;
        } else {
            for (int d = 0; d < dim; ++d) y[d] = x[d];
        }
        double s2 = 0.0;
        for (int d = 0; d < dim; ++d) s2 = fma(y[d], y[d], s2);
        if (s2 > m2) m2 = s2;
    }
    /* every distance is at most 4 max ||y||^2 = 2^e (up to rounding) */
    int e;
    (void)frexp(4.0 * m2, &e);
    if (m2 == 0.0) e = 0;
    int shift = 61 - ceil_log2_u64((uint64_t)n) - e;
    t_norm = orc_now() - t_norm;
    uint64_t best_q = UINT64_MAX;
    int best_r = -1, best_iters = 0;
    for (int r = 0; r < restarts; ++r) {
        const uint64_t* u = draws ? draws + (int64_t)r * K : NULL;
        const double t_r0 = orc_now();
        if (init_centroids) {
            memcpy(Cc, init_centroids, sizeof(double) * (size_t)K * dim);
        } else {
            int64_t c0 = (int64_t)mulhi64(u[0], (uint64_t)n);
            memcpy(Cc, Y + c0 * dim, sizeof(double) * (size_t)dim);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) D2[i] = sqdist(dim, Y + i * dim, Cc);
            for (int j = 1; j < K; ++j) {
                uint64_t T = 0;
                for (int64_t i = 0; i < n; ++i) { T += qweight(D2[i], shift); pref[i] = T; }
                int64_t pick;
                if (T == 0) {
                    pick = (int64_t)mulhi64(u[j], (uint64_t)n);
                } else {
                    uint64_t t = mulhi64(u[j], T);
                    int64_t lo = 0, hi = n - 1;     /* first i with pref[i] > t */
                    while (lo < hi) {
                        int64_t mid = lo + (hi - lo) / 2;
                        if (pref[mid] > t) hi = mid; else lo = mid + 1;
                    }
                    pick = lo;
                }
                memcpy(Cc + (int64_t)j * dim, Y + pick * dim, sizeof(double) * (size_t)dim);
#pragma omp parallel for schedule(static)
                for (int64_t i = 0; i < n; ++i) {
                    double dd = sqdist(dim, Y + i * dim, Cc + (int64_t)j * dim);
                    if (dd < D2[i]) D2[i] = dd;
                }
            }
        }
        /* Lloyd */
        int iters = 0;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double best = sqdist(dim, Y + i * dim, Cc);
            int bj = 0;
            for (int j = 1; j < K; ++j) {
                double dd = sqdist(dim, Y + i * dim, Cc + (int64_t)j * dim);
                if (dd < best) { best = dd; bj = j; }
            }
            lab[i] = bj;
            D2[i] = best;
        }
        const double t_r1 = orc_now();
        t_seed += t_r1 - t_r0;
        for (int it = 1; it <= max_iter; ++it) {
            for (int j = 0; j < K; ++j) cnt[j] = 0;
            for (int64_t i = 0; i < n; ++i) cnt[lab[i]]++;
            for (int j = 0; j < K; ++j) {
                if (cnt[j] == 0) continue;
                double* c = Cc + (int64_t)j * dim;
                for (int d = 0; d < dim; ++d) c[d] = 0.0;
            }
            for (int64_t i = 0; i < n; ++i) {
                double* c = Cc + (int64_t)lab[i] * dim;
                const double* y = Y + i * dim;
                for (int d = 0; d < dim; ++d) c[d] += y[d];
            }
            for (int j = 0; j < K; ++j) {
                if (cnt[j] == 0) continue;
                double* c = Cc + (int64_t)j * dim;
                for (int d = 0; d < dim; ++d) c[d] = c[d] / (double)cnt[j];
            }
            int64_t changed = 0;
#pragma omp parallel for schedule(static) reduction(+ : changed)
            for (int64_t i = 0; i < n; ++i) {
                double best = sqdist(dim, Y + i * dim, Cc);
                int bj = 0;
                for (int j = 1; j < K; ++j) {
                    double dd = sqdist(dim, Y + i * dim, Cc + (int64_t)j * dim);
                    if (dd < best) { best = dd; bj = j; }
                }
                changed += (bj != lab[i]);
                nl[i] = bj;
                D2[i] = best;
            }
            memcpy(lab, nl, sizeof(int32_t) * (size_t)n);
            iters = it;
            if (changed == 0) break;
        }
        t_lloyd += orc_now() - t_r1;
        n_lloyd += iters;
        if (orc_trace())
            fprintf(stderr, "[oracle kmeans] restart %d: seeding %.1f s, %d Lloyd updates %.1f s\n",
                    r, t_r1 - t_r0, iters, orc_now() - t_r1);
        uint64_t q = 0;
        for (int64_t i = 0; i < n; ++i) q += qweight(D2[i], shift);
        if (q < best_q || best_r < 0) {
            best_q = q;
            best_r = r;
            best_iters = iters;
            memcpy(labels, lab, sizeof(int32_t) * (size_t)n);
            memcpy(centroids, Cc, sizeof(double) * (size_t)K * dim);
            double s = 0.0;
            for (int64_t i = 0; i < n; ++i) s += D2[i];
            *inertia = s;
        }
    }
    if (inertia_q) *inertia_q = best_q;
    if (best_restart) *best_restart = best_r;
    if (lloyd_iters) *lloyd_iters = best_iters;
    if (timing) {
        timing[0] = t_norm;
        timing[1] = t_seed;
        timing[2] = t_lloyd;
        timing[3] = n_lloyd;
    }
    free(Y); free(Cc); free(D2); free(pref); free(lab); free(nl); free(cnt);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Cluster labels by QR with column pivoting of X' (Section II-A: the        */
/* multi-way partition is read off the approximate eigenvectors by a pivoted */
/* QR; Damle, Minden & Ying, the method it cites).                           */
/* ------------------------------------------------------------------------ */

/*
 * X: n x k row-major (row i holds vertex i's k coordinates), row stride ldx.
 * 1. Businger-Golub pivoting over the columns of X' (the rows of X):
 *      res_i = ||x_i||^2 (fma over the coordinates in order);
 *      step s: p_s = argmax of res_i over the rows not chosen yet (ties: lowest i);
 *        a_t = q_t . x_{p_s} for t < s (fma over the coordinates in order);
 *        r_d = x_{p_s, d}, then r_d = fma(-a_t, q_{t,d}, r_d) for t = 0 .. s-1;
 *        q_s = r / ||r|| (ordered fma sum, IEEE sqrt and division);
 *        every row: c = q_s . x_i (fma in order), res_i = fma(-c, c, res_i).
 *      A chosen residual at or below CPQR_RANK_TOL times the first pivot's
 *      (1e-5 relative in norm, far above the downdates' rounding noise of about
 *      1e-15) is a breakdown: the block has rank below k.
 * 2. B = the pivot rows (k x k, row s = x_{p_s}).  The orthogonal polar factor
 *    of B' is Q = B' (B B')^-1/2; with B B' = W diag(l) W' (cyclic Jacobi),
 *    M = W diag(1/sqrt(l)) W' and Q = B' M (fma sums in index order).
 * 3. label_i = argmax_j |(X Q)_ij| (fma over the coordinates in order; ties:
 *    lowest j).
 * pivots [k], labels [n] and Q (k x k row-major, Q[d*k + j]) are outputs.
 */
#define CPQR_RANK_TOL 1e-10
int orc_cpqr_labels(int64_t n, int k, const double* X, int64_t ldx, int32_t* pivots,
                    int32_t* labels, double* Qout) {
    double floor_res = 0.0;
    if (n <= 0 || k <= 0 || k > n || ldx < k) return ORC_E_INVAL;
    int status = ORC_OK;
    double* res = (double*)malloc(sizeof(double) * (size_t)n);
    char* chosen = (char*)calloc((size_t)n, 1);
    double* q = (double*)malloc(sizeof(double) * (size_t)k * k);     /* q_t rows */
    double* a = (double*)malloc(sizeof(double) * (size_t)k);
    double* r = (double*)malloc(sizeof(double) * (size_t)k);
    double* B = (double*)malloc(sizeof(double) * (size_t)k * k);
    double* G = (double*)malloc(sizeof(double) * (size_t)k * k);
    double* W = (double*)malloc(sizeof(double) * (size_t)k * k);
    double* l = (double*)malloc(sizeof(double) * (size_t)k);
    double* M = (double*)malloc(sizeof(double) * (size_t)k * k);
    if (!res || !chosen || !q || !a || !r || !B || !G || !W || !l || !M) { status = ORC_E_NOMEM; goto out; }
    for (int64_t i = 0; i < n; ++i) {
        const double* x = X + i * ldx;
        double t = 0.0;
        for (int d = 0; d < k; ++d) {
            if (!isfinite(x[d])) { status = ORC_E_NUMERIC; goto out; }
            t = fma(x[d], x[d], t);
        }
        res[i] = t;
    }
    for (int st = 0; st < k; ++st) {
        int64_t p = -1;
        double best = 0.0;
        for (int64_t i = 0; i < n; ++i)
            if (!chosen[i] && (p < 0 || res[i] > best)) { p = i; best = res[i]; }
        if (!(best > floor_res)) { status = ORC_E_BREAKDOWN; goto out; }
        if (st == 0) floor_res = best * CPQR_RANK_TOL;
        chosen[p] = 1;
        pivots[st] = (int32_t)p;
        const double* xp = X + p * ldx;
        for (int t = 0; t < st; ++t) {
            double dot = 0.0;
            for (int d = 0; d < k; ++d) dot = fma(q[(int64_t)t * k + d], xp[d], dot);
            a[t] = dot;
        }
        for (int d = 0; d < k; ++d) {
            double v = xp[d];
            for (int t = 0; t < st; ++t) v = fma(-a[t], q[(int64_t)t * k + d], v);
            r[d] = v;
        }
        double nr2 = 0.0;
        for (int d = 0; d < k; ++d) nr2 = fma(r[d], r[d], nr2);
        const double nr = sqrt(nr2);
        if (!(nr > 0.0)) { status = ORC_E_BREAKDOWN; goto out; }
        for (int d = 0; d < k; ++d) q[(int64_t)st * k + d] = r[d] / nr;
        const double* qs = q + (int64_t)st * k;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            const double* x = X + i * ldx;
            double c = 0.0;
            for (int d = 0; d < k; ++d) c = fma(qs[d], x[d], c);
            res[i] = fma(-c, c, res[i]);
        }
    }
    for (int s2 = 0; s2 < k; ++s2)
        memcpy(B + (int64_t)s2 * k, X + (int64_t)pivots[s2] * ldx, sizeof(double) * (size_t)k);
    for (int u = 0; u < k; ++u)
        for (int v = 0; v < k; ++v) {
            double t = 0.0;
            for (int d = 0; d < k; ++d) t = fma(B[(int64_t)u * k + d], B[(int64_t)v * k + d], t);
            G[(int64_t)u * k + v] = t;
        }
    status = orc_symeig(k, G, l, W);
    if (status != ORC_OK) goto out;
    for (int j = 0; j < k; ++j) {
        if (!(l[j] > 0.0)) { status = ORC_E_BREAKDOWN; goto out; }
        l[j] = 1.0 / sqrt(l[j]);
    }
    for (int u = 0; u < k; ++u)
        for (int v = 0; v < k; ++v) {
            double t = 0.0;
            for (int j = 0; j < k; ++j) t = fma(W[(int64_t)u * k + j] * l[j], W[(int64_t)v * k + j], t);
            M[(int64_t)u * k + v] = t;
        }
    for (int d = 0; d < k; ++d)
        for (int j = 0; j < k; ++j) {
            double t = 0.0;
            for (int u = 0; u < k; ++u) t = fma(B[(int64_t)u * k + d], M[(int64_t)u * k + j], t);
            Qout[(int64_t)d * k + j] = t;
        }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double* x = X + i * ldx;
        int bj = 0;
        double bv = -1.0;
        for (int j = 0; j < k; ++j) {
            double z = 0.0;
            for (int d = 0; d < k; ++d) z = fma(x[d], Qout[(int64_t)d * k + j], z);
            if (fabs(z) > bv) { bv = fabs(z); bj = j; }
        }
        labels[i] = bj;
    }
out:
    free(res); free(chosen); free(q); free(a); free(r); free(B); free(G); free(W); free(l); free(M);
    return status;
}

/*
 * Number of clusters from the gap in the smallest eigenvalues (Section II-A:
 * the first significantly large increment; the count of eigenvalues below it).
 * theta ascending.  Increments g_j = theta_{j+1} - theta_j, j = 0 .. k-2; the
 * gap is the first j >= 1 with g_j > 1e-8 (theta_{k-1} - theta_0) (above the
 * rounding noise of eigenvalues that are equal in exact arithmetic) and
 * g_j > sig * (g_0 + .. + g_{j-1}) / j (significantly larger than the
 * increments before it); if none, the largest
 * increment (the first of equals).  The count is j + 1; k == 1 gives 1.
 * *ratio (optional) = g_j / the median increment, a confidence figure.
 */
int orc_eigengap(int k, const double* theta, double sig, double* ratio) {
    if (k <= 1) { if (ratio) *ratio = 0.0; return k; }
    int jj = -1;
    const double tiny = 1e-8 * (theta[k - 1] - theta[0]);
    double sum = theta[1] - theta[0];
    for (int j = 1; j + 1 < k; ++j) {
        const double g = theta[j + 1] - theta[j];
        if (g > tiny && g > sig * (sum / (double)j)) { jj = j; break; }
        sum += g;
    }
    if (jj < 0) {
        double gmax = -INFINITY;
        for (int j = 0; j + 1 < k; ++j) {
            const double g = theta[j + 1] - theta[j];
            if (g > gmax) { gmax = g; jj = j; }
        }
    }
    if (ratio) {
        /* median increment (insertion sort of a copy) */
        double* g = (double*)malloc(sizeof(double) * (size_t)(k - 1));
        if (g) {
            for (int j = 0; j + 1 < k; ++j) g[j] = theta[j + 1] - theta[j];
            for (int a = 1; a < k - 1; ++a) {
                double v = g[a];
                int b = a - 1;
                while (b >= 0 && g[b] > v) { g[b + 1] = g[b]; --b; }
                g[b + 1] = v;
            }
            const double med = (k - 1) % 2 ? g[(k - 1) / 2] : 0.5 * (g[(k - 1) / 2 - 1] + g[(k - 1) / 2]);
            *ratio = med > 0.0 ? (theta[jj + 1] - theta[jj]) / med : INFINITY;
            free(g);
        } else {
            *ratio = 0.0;
        }
    }
    return jj + 1;
}

/*
 * Warm start for a stage that adds vertices (Section III: the approximate
 * eigenvectors of the previous graph start the solve for the next; the
 * entries of vertices the previous graph lacked must be filled in).  Vertices
 * 0 .. n_old-1 keep their rows of X; each new vertex i >= n_old gets the mean
 * of the rows of its neighbours j < n_old in the current graph: the sum in
 * FP64 over the row's entries in ascending column order, starting from 0.0,
 * divided by their count (IEEE division).  A new vertex with no old
 * neighbour keeps a zero row.  X row-major n x k, row stride ldx, in place.
 */
void orc_warm_fill(int64_t n, int64_t n_old, const int64_t* row_ptr, const int32_t* col, int k,
                   double* X, int64_t ldx) {
    for (int64_t i = n_old; i < n; ++i) {
        double* xi = X + i * ldx;
        int64_t cnt = 0;
        for (int d = 0; d < k; ++d) xi[d] = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            const int64_t j = col[p];
            if (j >= n_old) continue;
            const double* xj = X + j * ldx;
            for (int d = 0; d < k; ++d) xi[d] += xj[d];
            ++cnt;
        }
        if (cnt > 0)
            for (int d = 0; d < k; ++d) xi[d] = xi[d] / (double)cnt;
    }
}

/* Row normalisation alone (exposed for the tests). */
void orc_row_normalize(int64_t n, int dim, const double* X, int64_t ldx, double* Y) {
    for (int64_t i = 0; i < n; ++i) {
        const double* x = X + i * ldx;
        double s = 0.0;
        for (int d = 0; d < dim; ++d) s = fma(x[d], x[d], s);
        double nrm = sqrt(s);
        for (int d = 0; d < dim; ++d) Y[i * dim + d] = nrm > 0.0 ? x[d] / nrm : 0.0;
    }
}
