// Rayleigh-Ritz step of LOBPCG in FP64 on one workgroup, and the dense
// symmetric eigensolver it uses (exposed as sc_symeig for testing).
//
// Given the Gram matrices G_A = S'LS and G_B = S'S of the basis S = [X W P]
// and the mask of active columns:
//   B = G_B[act,act] = U'U (Cholesky; on failure with P active, P leaves the
//   basis and the factorisation is redone; a second failure is a breakdown);
//   M = U^-T G_A[act,act] U^-1, symmetrised;
//   M = Q diag(lambda) Q' for the k smallest eigenvalues:
//     Householder reduction to tridiagonal form, bisection with Sturm counts
//     for the k smallest eigenvalues, inverse iteration with a pivoted
//     tridiagonal LU for their eigenvectors (vectors of tightly clustered
//     eigenvalues are re-orthogonalised by modified Gram-Schmidt), and the
//     Householder reflectors applied back;
//   C = U^-1 Q (scattered to the rows of the active columns), theta = lambda.
// The matrices live in a global scratch area (L2 resident at these sizes).
#include <float.h>

#include "chol.h"
#include "sc_internal.h"

namespace {

constexpr int NT = 1024;
constexpr int NWAVE = NT / 64;
constexpr int MAXM = 1024;

__device__ inline double block_sum(double v, double* red) {
    v = sc_wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < NWAVE; ++w) s += red[w];
        red[NWAVE] = s;
    }
    __syncthreads();
    const double r = red[NWAVE];
    __syncthreads();
    return r;
}

__device__ inline double block_max(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = red[0];
        for (int w = 1; w < NWAVE; ++w) s = fmax(s, red[w]);
        red[NWAVE] = s;
    }
    __syncthreads();
    const double r = red[NWAVE];
    __syncthreads();
    return r;
}

__device__ inline uint64_t mix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Householder reduction of the symmetric m x m matrix A (row-major, both
// triangles kept current) to tridiagonal form: diagonal d, off-diagonal e.
// Reflector j (acting on rows j+1..m-1) is I - tau_j v v' with v_0 = 1 and
// v_r (r >= 1) stored in A[j][j+1+r].
__device__ void tridiagonalize(int m, double* A, double* d, double* e, double* tau, double* v,
                               double* p, double* red, double* sh) {
    const int tid = threadIdx.x;
    for (int j = 0; j + 2 < m; ++j) {
        const int len = m - j - 1;
        const double* x = A + (int64_t)j * m + j + 1;   // row j right of the diagonal
        double part = 0.0;
        for (int r = 1 + tid; r < len; r += NT) part = fma(x[r], x[r], part);
        const double sigma = block_sum(part, red);
        if (tid == 0) {
            const double x0 = x[0];
            d[j] = A[(int64_t)j * m + j];
            if (sigma == 0.0) {
                tau[j] = 0.0;
                e[j] = x0;
                sh[0] = 1.0;
            } else {
                const double mu = sqrt(x0 * x0 + sigma);
                const double v0 = x0 <= 0.0 ? x0 - mu : -sigma / (x0 + mu);
                tau[j] = 2.0 * v0 * v0 / (sigma + v0 * v0);
                e[j] = mu;
                sh[0] = v0;
            }
        }
        __syncthreads();
        const double tj = tau[j];
        if (tj == 0.0) {
            __syncthreads();
            continue;
        }
        const double v0 = sh[0];
        for (int r = tid; r < len; r += NT) v[r] = r == 0 ? 1.0 : x[r] / v0;
        __syncthreads();
        // p = tau A22 v, read column-wise (A22 symmetric) for coalescing
        const double* A22 = A + (int64_t)(j + 1) * m + (j + 1);
        for (int r = tid; r < len; r += NT) {
            double s = 0.0;
            for (int c = 0; c < len; ++c) s = fma(A22[(int64_t)c * m + r], v[c], s);
            p[r] = tj * s;
        }
        __syncthreads();
        part = 0.0;
        for (int r = tid; r < len; r += NT) part = fma(p[r], v[r], part);
        const double K = 0.5 * tj * block_sum(part, red);
        for (int r = tid; r < len; r += NT) p[r] = p[r] - K * v[r];   // p <- w
        __syncthreads();
        double* B22 = A + (int64_t)(j + 1) * m + (j + 1);
        for (int64_t q = tid; q < (int64_t)len * len; q += NT) {
            const int r = (int)(q / len), c = (int)(q % len);
            B22[(int64_t)r * m + c] -= v[r] * p[c] + p[r] * v[c];
        }
        __syncthreads();
        // keep the reflector in row j (no longer read by later steps)
        double* xs = A + (int64_t)j * m + j + 1;
        for (int r = 1 + tid; r < len; r += NT) xs[r] = v[r];
        __syncthreads();
    }
    if (tid == 0) {
        if (m >= 2) {
            d[m - 2] = A[(int64_t)(m - 2) * m + (m - 2)];
            e[m - 2] = A[(int64_t)(m - 2) * m + (m - 1)];
            tau[m - 2] = 0.0;
        }
        d[m - 1] = A[(int64_t)(m - 1) * m + (m - 1)];
        if (m >= 1) tau[m - 1] = 0.0;
    }
    __syncthreads();
}

// number of eigenvalues of the tridiagonal (d, e) smaller than x
__device__ inline int sturm_count(int m, const double* d, const double* e, double x, double pivmin) {
    int c = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
    for (int i = 1; i < m; ++i) {
        q = (d[i] - x) - e[i - 1] * e[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++c;
    }
    return c;
}

// ---------------------------------------------------------------------------
// Eigenpairs of the symmetric tridiagonal T = (d, e) for its k smallest
// eigenvalues, in four launches:
//   k_tri_params  Gershgorin interval, scale and pivot floor;
//   k_tri_bisect  one wave per eigenvalue: 64-way multisection with Sturm
//                 counts (lane l evaluates the count at the l-th interior
//                 point; the bracket keeps count(lo) <= i < count(hi));
//   k_tri_invit   one thread per eigenvector: inverse iteration with a
//                 pivoted LU of T - shift I (3 steps from a fixed
//                 pseudo-random start); coincident eigenvalues get shifts
//                 pulled apart by 10 eps ||T||;
//   k_tri_bcgs    vectors of eigenvalues closer than 1e-4 ||T|| are
//                 re-orthogonalised by block Gram-Schmidt (twice, Cholesky
//                 QR within blocks of eight).
// Layout of the tridiagonal block `tri` (doubles): d[MAXM], e[MAXM],
// tau[MAXM], params[8].
// ---------------------------------------------------------------------------
constexpr int TRI_PARAMS = 3 * MAXM;

__global__ void __launch_bounds__(NT) k_tri_params(const int* __restrict__ info, double* __restrict__ tri) {
    __shared__ double red[NWAVE + 1];
    const int m = info[0];
    if (m == 0) return;
    const double* d = tri;
    const double* e = tri + MAXM;
    double lo_l = DBL_MAX, hi_l = -DBL_MAX, nrm_l = 0.0, emax_l = 0.0;
    for (int i = threadIdx.x; i < m; i += NT) {
        const double el = i > 0 ? fabs(e[i - 1]) : 0.0;
        const double er = i + 1 < m ? fabs(e[i]) : 0.0;
        lo_l = fmin(lo_l, d[i] - el - er);
        hi_l = fmax(hi_l, d[i] + el + er);
        nrm_l = fmax(nrm_l, fabs(d[i]) + el + er);
        if (i + 1 < m) emax_l = fmax(emax_l, e[i] * e[i]);
    }
    const double gl = -block_max(-lo_l, red);
    const double gu = block_max(hi_l, red);
    const double tnorm = fmax(block_max(nrm_l, red), DBL_MIN);
    const double emax2 = block_max(emax_l, red);
    if (threadIdx.x == 0) {
        const double pivmin = DBL_MIN * fmax(1.0, emax2);
        double* P = tri + TRI_PARAMS;
        P[0] = gl - 2.0 * DBL_EPSILON * tnorm - 2.0 * pivmin;
        P[1] = gu + 2.0 * DBL_EPSILON * tnorm + 2.0 * pivmin;
        P[2] = tnorm;
        P[3] = pivmin;
    }
}

__global__ void __launch_bounds__(256)
k_tri_bisect(int k, const int* __restrict__ info, const double* __restrict__ tri,
             double* __restrict__ w) {
    const int m = info[0];
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (m == 0 || i >= k) return;
    const double* d = tri;
    const double* e = tri + MAXM;
    const double* P = tri + TRI_PARAMS;
    double lo = P[0], hi = P[1];
    const double tnorm = P[2], pivmin = P[3];
    for (int it = 0; it < 24; ++it) {
        if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + 1e-18 * tnorm) break;
        const double x = lo + (hi - lo) * ((double)(lane + 1) / 65.0);
        const bool le = (x > lo && x < hi) ? sturm_count(m, d, e, x, pivmin) <= i : (x <= lo);
        const unsigned long long mask = __ballot(le);
        // first lane whose point has more than i eigenvalues below it
        const unsigned long long gt = ~mask;
        const int t = gt ? __ffsll((long long)gt) - 1 : 64;
        const double xl = __shfl(x, t > 0 ? t - 1 : 0, 64);
        const double xh = __shfl(x, t < 64 ? t : 63, 64);
        const double nlo = t > 0 ? xl : lo;
        const double nhi = t < 64 ? xh : hi;
        if (nlo == lo && nhi == hi) break;
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) w[i] = 0.5 * (lo + hi);
}

// one thread per eigenvector, IV_T eigenvectors per workgroup.  The LU
// factors live in global memory laid out [q][eigenvector] (a workgroup's
// threads touch consecutive addresses); the iterate z lives in LDS during the
// sweeps and is written to V once at the end, so the sweeps issue no global
// stores and their loads of the (read-only) factors never wait for stores.
// Factorisation and sweeps are serial recurrences whose loads do not depend
// on the recurrence: they are issued IV_B steps ahead.
constexpr int IV_B = 8;
constexpr int IV_T = 16;
__global__ void __launch_bounds__(IV_T)
k_tri_invit(int k, const int* __restrict__ info, const double* __restrict__ tri,
            const double* __restrict__ w, double* __restrict__ V, int ldv, double* __restrict__ lu) {
    __shared__ double zs[MAXM * IV_T];
    const int m = info[0];
    const int i = blockIdx.x * IV_T + threadIdx.x;
    if (m == 0 || i >= k) return;
    const double* d = tri;
    const double* e = tri + MAXM;
    const double tnorm = tri[TRI_PARAMS + 2];
    const double eps = DBL_EPSILON;
    const double tiny = eps * tnorm;
    // shift: coincident eigenvalues pulled apart (sequential over lower indices)
    const double sep = 10.0 * eps * tnorm;
    double lam = w[0];
    for (int q = 1; q <= i; ++q) {
        const double s = w[q];
        lam = (s - lam < sep) ? lam + sep : s;
    }
    double* U0 = lu;
    double* U1 = U0 + (int64_t)MAXM * k;
    double* U2 = U1 + (int64_t)MAXM * k;
    double* Lm = U2 + (int64_t)MAXM * k;
    double* SW = Lm + (int64_t)MAXM * k;
#define AT(arr, q) arr[(int64_t)(q) * k + i]
#define ZS(q) zs[(q) * IV_T + threadIdx.x]
    // LU with partial pivoting of T - lam I (rows q, q + 1 per step); the
    // factors of a block are stored after the next block's loads
    const int nq = m - 1;                        // steps
    double r0 = d[0] - lam, r1 = (m > 1 ? e[0] : 0.0) + 0.0;
    {
        double sub[IV_B], a1[IV_B], b1[IV_B];
        double f0[IV_B], f1[IV_B], f2[IV_B], fl[IV_B], fs[IV_B];
        auto load = [&](int q0) {
#pragma unroll
            for (int t = 0; t < IV_B; ++t) {
                const int q = min(q0 + t, nq - 1);
                sub[t] = e[q];
                a1[t] = d[q + 1] - lam;
                b1[t] = q + 2 < m ? e[q + 1] : 0.0;
            }
        };
        if (nq > 0) load(0);
        for (int q0 = 0; q0 < nq; q0 += IV_B) {
            const int nb = min(IV_B, nq - q0);
#pragma unroll
            for (int t = 0; t < IV_B; ++t) {
                if (t < nb) {
                    // keep row q (no interchange) or swap in row q + 1
                    const bool keep = fabs(r0) >= fabs(sub[t]);
                    const double p0 = (keep && r0 == 0.0) ? tiny : r0;
                    const double l = keep ? sub[t] / p0 : p0 / sub[t];
                    f0[t] = keep ? p0 : sub[t];
                    f1[t] = keep ? r1 : a1[t];
                    f2[t] = keep ? 0.0 : b1[t];
                    fl[t] = l;
                    fs[t] = keep ? 0.0 : 1.0;
                    const double n0 = keep ? a1[t] - l * r1 : r1 - l * a1[t];
                    const double n1 = keep ? b1[t] : -l * b1[t];
                    r0 = n0;
                    r1 = n1;
                }
            }
            if (q0 + IV_B < nq) load(q0 + IV_B);
#pragma unroll
            for (int t = 0; t < IV_B; ++t) {
                if (t < nb) {
                    const int q = q0 + t;
                    AT(U0, q) = f0[t]; AT(U1, q) = f1[t]; AT(U2, q) = f2[t]; AT(Lm, q) = fl[t];
                    AT(SW, q) = fs[t];
                }
            }
        }
    }
    if (r0 == 0.0) r0 = tiny;
    AT(U0, m - 1) = r0;
    // the last row has no superdiagonal entries; they are still read (times
    // zero) by the back substitution, so they must not hold stale NaN / Inf
    AT(U1, m - 1) = 0.0;
    AT(U2, m - 1) = 0.0;
    for (int r = 0; r < m; ++r)
        ZS(r) = (double)(mix64(((uint64_t)i << 32) ^ (uint64_t)r) >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    double inv = 1.0;
    for (int itn = 0; itn < 3; ++itn) {
        // forward sweep (row interchanges and L)
        double rc = ZS(0) * inv;
        {
            double l[IV_B], sw[IV_B];
            auto load = [&](int q0) {
#pragma unroll
                for (int t = 0; t < IV_B; ++t) {
                    const int q = min(q0 + t, nq - 1);
                    l[t] = AT(Lm, q);
                    sw[t] = AT(SW, q);
                }
            };
            if (nq > 0) load(0);
            for (int q0 = 0; q0 < nq; q0 += IV_B) {
                const int nb = min(IV_B, nq - q0);
                double nxt[IV_B], lc[IV_B], swc[IV_B];
#pragma unroll
                for (int t = 0; t < IV_B; ++t) {
                    nxt[t] = t < nb ? ZS(q0 + t + 1) * inv : 0.0;
                    lc[t] = l[t];
                    swc[t] = sw[t];
                }
                if (q0 + IV_B < nq) load(q0 + IV_B);
#pragma unroll
                for (int t = 0; t < IV_B; ++t) {
                    if (t < nb) {
                        const bool swp = swc[t] != 0.0;
                        ZS(q0 + t) = swp ? nxt[t] : rc;
                        rc = swp ? rc - lc[t] * nxt[t] : nxt[t] - lc[t] * rc;
                    }
                }
            }
        }
        ZS(m - 1) = rc;
        // back substitution; the last two solution values stay in registers
        double z1 = 0.0, z2 = 0.0, nn = 0.0;
        {
            double u0[IV_B], u1[IV_B], u2[IV_B];
            auto load = [&](int q1) {
#pragma unroll
                for (int t = 0; t < IV_B; ++t) {
                    const int q = max(q1 - t, 0);
                    u0[t] = AT(U0, q);
                    u1[t] = AT(U1, q);
                    u2[t] = AT(U2, q);
                }
            };
            load(m - 1);
            for (int q1 = m - 1; q1 >= 0; q1 -= IV_B) {
                const int nb = min(IV_B, q1 + 1);
                double zc[IV_B], a0[IV_B], a1v[IV_B], a2[IV_B];
#pragma unroll
                for (int t = 0; t < IV_B; ++t) {
                    zc[t] = t < nb ? ZS(q1 - t) : 0.0;
                    a0[t] = u0[t];
                    a1v[t] = u1[t];
                    a2[t] = u2[t];
                }
                if (q1 - IV_B >= 0) load(q1 - IV_B);
#pragma unroll
                for (int t = 0; t < IV_B; ++t) {
                    if (t < nb) {
                        double sacc = zc[t];
                        sacc -= a1v[t] * z1;
                        sacc -= a2[t] * z2;
                        const double zq = sacc / a0[t];
                        ZS(q1 - t) = zq;
                        nn = fma(zq, zq, nn);
                        z2 = z1;
                        z1 = zq;
                    }
                }
            }
        }
        // the normalisation is applied where z is next read
        inv = 1.0 / sqrt(nn);
    }
    double* z = V + i;      // column i, row stride ldv
    for (int r = 0; r < m; ++r) z[(int64_t)r * ldv] = ZS(r) * inv;
#undef ZS
#undef AT
}

// Vectors of a cluster are orthonormalised in index order; vector q is
// projected against all earlier members at once (classical Gram-Schmidt,
// applied twice) and normalised.  Clusters are independent: workgroup g takes
// clusters g, g + gridDim, ...  A cluster is first copied to the scratch Wt
// with each vector contiguous (V itself is row-major, one row per entry), so
// every dot product and update reads consecutive addresses; it is copied back
// at the end.  The vector being orthogonalised is held in LDS; each wave
// forms four dot products per sweep over the rows, and the update keeps four
// independent partial sums, so the loads of the earlier members overlap.
// Wt holds >= k * m doubles (vector q at Wt + q m).
// Clusters of close eigenvalues: their inverse-iteration vectors are made
// orthonormal by block classical Gram-Schmidt with reorthogonalisation
// (BCGS2): blocks of BCG_B vectors, each projected twice against the
// cluster's earlier vectors (in chunks of BCG_PC, the coefficients of a chunk
// from the block as the previous chunk left it) and orthonormalised after each
// projection by Cholesky QR of its BCG_B x BCG_B Gram matrix.  Every earlier
// vector is read once per block and pass instead of once per vector, which is
// what bounds this one-workgroup kernel.  A block whose Gram matrix is not
// safely positive definite (pivot below 1e-14 of the largest diagonal entry)
// is orthonormalised vector by vector instead (Gram-Schmidt, twice).
constexpr int BCG_B = 8;
constexpr int BCG_PC = 128;

__global__ void __launch_bounds__(NT)
k_tri_bcgs(int k, const int* __restrict__ info, const double* __restrict__ tri,
           const double* __restrict__ w, double* __restrict__ V, int ldv, double* __restrict__ Wt) {
    __shared__ double red[NWAVE + 1];
    __shared__ double blk[BCG_B][MAXM];
    __shared__ double cf[BCG_PC][BCG_B];
    __shared__ double G[BCG_B][BCG_B], Li[BCG_B][BCG_B];
    __shared__ int fail;
    const int m = info[0];
    if (m == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double ctol = 1e-4 * tri[TRI_PARAMS + 2];
    int cl = 0;
    for (int c0 = 0; c0 < k; ++cl) {
        int c1 = c0 + 1;
        while (c1 < k && w[c1] - w[c1 - 1] <= ctol) ++c1;
        if (c1 - c0 > 1 && cl % gridDim.x == blockIdx.x) {
            const int cs = c1 - c0;
            for (int e = tid; e < cs * m; e += NT) {
                const int r = e / cs, q = c0 + e % cs;      // consecutive threads: one row of V
                Wt[(int64_t)q * m + r] = V[(int64_t)r * ldv + q];
            }
            __syncthreads();
            for (int b0 = c0; b0 < c1; b0 += BCG_B) {
                const int nb = min(BCG_B, c1 - b0);
                for (int e = tid; e < BCG_B * m; e += NT) {
                    const int u = e / m, r = e % m;
                    blk[u][r] = u < nb ? Wt[(int64_t)(b0 + u) * m + r] : 0.0;
                }
                __syncthreads();
                for (int rep = 0; rep < 2; ++rep) {
                    // projection against the cluster's earlier vectors
                    for (int p0 = c0; p0 < b0; p0 += BCG_PC) {
                        const int np = min(BCG_PC, b0 - p0);
                        for (int pi = wave; pi < np; pi += NWAVE) {
                            const double* q = Wt + (int64_t)(p0 + pi) * m;
                            double part[BCG_B];
#pragma unroll
                            for (int u = 0; u < BCG_B; ++u) part[u] = 0.0;
                            for (int r = lane; r < m; r += 64) {
                                const double qv = q[r];
#pragma unroll
                                for (int u = 0; u < BCG_B; ++u) part[u] = fma(qv, blk[u][r], part[u]);
                            }
#pragma unroll
                            for (int u = 0; u < BCG_B; ++u) {
                                const double t = sc_wave_sum(part[u]);
                                if (lane == 0) cf[pi][u] = t;
                            }
                        }
                        __syncthreads();
                        for (int r = tid; r < m; r += NT) {
                            double acc[BCG_B];
#pragma unroll
                            for (int u = 0; u < BCG_B; ++u) acc[u] = 0.0;
                            for (int pi = 0; pi < np; ++pi) {
                                const double qv = Wt[(int64_t)(p0 + pi) * m + r];
#pragma unroll
                                for (int u = 0; u < BCG_B; ++u) acc[u] = fma(cf[pi][u], qv, acc[u]);
                            }
#pragma unroll
                            for (int u = 0; u < BCG_B; ++u)
                                if (u < nb) blk[u][r] -= acc[u];
                        }
                        __syncthreads();
                    }
                    // Gram matrix of the block: one wave per (u, v) pair, u <= v
                    for (int pr = wave; pr < BCG_B * BCG_B; pr += NWAVE) {
                        const int u = pr / BCG_B, v = pr % BCG_B;
                        if (u > v || v >= nb) continue;                  // wave-uniform
                        double part = 0.0;
                        for (int r = lane; r < m; r += 64) part = fma(blk[u][r], blk[v][r], part);
                        const double t = sc_wave_sum(part);
                        if (lane == 0) {
                            G[u][v] = t;
                            G[v][u] = t;
                        }
                    }
                    __syncthreads();
                    if (tid == 0) {
                        // G = L L', Li = L^-1 (nb x nb)
                        double gmax = 0.0;
                        for (int u = 0; u < nb; ++u) gmax = fmax(gmax, G[u][u]);
                        int bad = !(gmax > 0.0) || !isfinite(gmax);
                        for (int j = 0; j < nb && !bad; ++j) {
                            double d = G[j][j];
                            for (int t = 0; t < j; ++t) d -= G[j][t] * G[j][t];
                            if (!(d > 1e-14 * gmax)) {
                                bad = 1;
                                break;
                            }
                            const double ljj = sqrt(d);
                            G[j][j] = ljj;
                            for (int i = j + 1; i < nb; ++i) {
                                double x = G[i][j];
                                for (int t = 0; t < j; ++t) x -= G[i][t] * G[j][t];
                                G[i][j] = x / ljj;
                            }
                        }
                        if (!bad)
                            for (int c = 0; c < nb; ++c)
                                for (int i = 0; i < nb; ++i) {
                                    if (i < c) {
                                        Li[i][c] = 0.0;
                                        continue;
                                    }
                                    double x = i == c ? 1.0 : 0.0;
                                    for (int t = c; t < i; ++t) x -= G[i][t] * Li[t][c];
                                    Li[i][c] = x / G[i][i];
                                }
                        fail = bad;
                    }
                    __syncthreads();
                    if (!fail) {
                        // Q = V R^-1 with R = L': q_u = sum_{t <= u} Li[u][t] v_t
                        for (int r = tid; r < m; r += NT) {
                            double x[BCG_B], y[BCG_B];
#pragma unroll
                            for (int u = 0; u < BCG_B; ++u) x[u] = blk[u][r];
#pragma unroll
                            for (int u = 0; u < BCG_B; ++u) {
                                double a = 0.0;
#pragma unroll
                                for (int t = 0; t < BCG_B; ++t)
                                    if (t <= u) a = fma(Li[u][t], x[t], a);
                                y[u] = a;
                            }
#pragma unroll
                            for (int u = 0; u < BCG_B; ++u)
                                if (u < nb) blk[u][r] = y[u];
                        }
                        __syncthreads();
                    } else {
                        // vector by vector: Gram-Schmidt against the block's earlier
                        // members, twice, then normalisation
                        for (int u = 0; u < nb; ++u) {
                            for (int pass = 0; pass < 2; ++pass)
                                for (int t = 0; t < u; ++t) {
                                    double part = 0.0;
                                    for (int r = tid; r < m; r += NT) part = fma(blk[t][r], blk[u][r], part);
                                    const double d = block_sum(part, red);
                                    for (int r = tid; r < m; r += NT) blk[u][r] = fma(-d, blk[t][r], blk[u][r]);
                                    __syncthreads();
                                }
                            double part = 0.0;
                            for (int r = tid; r < m; r += NT) part = fma(blk[u][r], blk[u][r], part);
                            const double nrm = sqrt(block_sum(part, red));
                            const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
                            for (int r = tid; r < m; r += NT) blk[u][r] *= inv;
                            __syncthreads();
                        }
                    }
                }
                for (int e = tid; e < nb * m; e += NT) {
                    const int u = e / m, r = e % m;
                    Wt[(int64_t)(b0 + u) * m + r] = blk[u][r];
                }
                __syncthreads();
            }
            for (int e = tid; e < cs * m; e += NT) {
                const int r = e / cs, q = c0 + e % cs;
                V[(int64_t)r * ldv + q] = Wt[(int64_t)q * m + r];
            }
            __syncthreads();
        }
        c0 = c1;
    }
}

// --- Rayleigh-Ritz, step 1 (one workgroup): active set, Cholesky of the
// basis Gram matrix (P dropped and retried once on failure), and the
// reduced G_A gathered to a dense m x m block.  info[0] = m (0 on breakdown),
// info[1..m] = the active column indices.
__global__ void __launch_bounds__(NT)
k_rr_setup(int K3, int kp, const double* __restrict__ GA, const double* __restrict__ GB,
           int* __restrict__ act, double tol, double* __restrict__ U, double* __restrict__ Am,
           int* __restrict__ info, int* status, int* counter, const int* __restrict__ pred,
           int* __restrict__ probe, int* __restrict__ probe_counter, int* __restrict__ wcounter) {
    __shared__ int idx[MAXM], actl[MAXM];
    __shared__ int m_s, fail_s, fail_at, has_p;
    __shared__ CholLds L;
    if (pred && *pred == 0) return;
    const int tid = threadIdx.x;
    int m = 0;
    // each failed attempt removes P, or (with wcounter) one dependent W column
    for (int attempt = 0; attempt < K3 + 2; ++attempt) {
        // active columns: flags read in parallel, listed from LDS by one thread
        for (int j = tid; j < K3; j += NT) actl[j] = act[j];
        __syncthreads();
        if (tid == 0) {
            int mm = 0;
            for (int j = 0; j < K3; ++j)
                if (actl[j]) idx[mm++] = j;
            m_s = mm;
            fail_s = 0;
            fail_at = -1;
        }
        __syncthreads();
        m = m_s;
        for (int q = tid; q < m * m; q += NT) {         // m <= MAXM: 32-bit indices
            const int a = q / m, b = q - a * m;
            U[q] = GB[(int64_t)idx[a] * K3 + idx[b]];
        }
        __syncthreads();
        // B = U'U in place (upper triangle), blocked
        const int fa = chol_blocked<NT>(m, U, tol, L);
        if (tid == 0) {
            fail_s = fa >= 0;
            fail_at = fa;
        }
        __syncthreads();
        if (!fail_s) break;
        if (probe) {
            // the basis Gram matrix is too ill-conditioned for its precision
            if (tid == 0) {
                *probe = 1;
                if (probe_counter) atomicAdd(probe_counter, 1);
                info[0] = 0;
            }
            return;
        }
        if (tid == 0) {
            has_p = 0;
            for (int j = 2 * kp; j < K3; ++j) has_p |= act[j];
        }
        __syncthreads();
        if (has_p) {
            for (int j = 2 * kp + tid; j < K3; j += NT) act[j] = 0;
            if (tid == 0) {
                atomicOr(status, DEV_P_DROPPED);
                if (counter) atomicAdd(counter, 1);
            }
            __syncthreads();
            continue;
        }
        const int col = fail_at >= 0 ? idx[fail_at] : -1;
        if (wcounter && col >= kp && col < 2 * kp) {
            // W column numerically inside the span of the earlier basis vectors
            if (tid == 0) {
                act[col] = 0;
                atomicAdd(wcounter, 1);
            }
            __syncthreads();
            continue;
        }
        if (tid == 0) {
            atomicOr(status, DEV_BREAKDOWN_RR);
            info[0] = 0;
        }
        return;
    }
    for (int q = tid; q < m * m; q += NT) {
        const int a = q / m, b = q - a * m;
        Am[q] = GA[(int64_t)idx[a] * K3 + idx[b]];
    }
    if (tid == 0) {
        info[0] = m;
        if (probe) *probe = 0;
    }
    for (int j = tid; j < m; j += NT) info[1 + j] = idx[j];
}

// --- dense FP64 products on many workgroups: C = op(A) B with op(A) = A or
// A', all row-major m x m (N = m or k columns); m is read from info[0].
// 64 x 64 output tiles, 4 x 4 per thread, K staged in LDS by 16.
__global__ void __launch_bounds__(256)
k_gemm64(const int* __restrict__ info, int n_fixed, int transA, const double* __restrict__ A,
         const double* __restrict__ B, double* __restrict__ C) {
    const int m = info[0];
    const int N = n_fixed > 0 ? n_fixed : m;
    const int row0 = blockIdx.y * 64, col0 = blockIdx.x * 64;
    if (row0 >= m || col0 >= N) return;
    __shared__ double As[16][65];
    __shared__ double Bs[16][64];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < m; k0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e / 64, r = e % 64;
            const int gr = row0 + r, gk = k0 + kk;
            double v = 0.0;
            if (gr < m && gk < m) v = transA ? A[(int64_t)gk * m + gr] : A[(int64_t)gr * m + gk];
            As[kk][r] = v;
            const int gc = col0 + r;
            Bs[kk][r] = (gk < m && gc < N) ? B[(int64_t)gk * N + gc] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx + 16 * c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gr = row0 + ty * 4 + r;
        if (gr >= m) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int gc = col0 + tx + 16 * c;
            if (gc < N) C[(int64_t)gr * N + gc] = acc[r][c];
        }
    }
}

// --- step 2: U^-1 (upper triangular), one wave per row i: the row x' of U^-1
// solves x' U = e_i', a forward sweep over c = i .. m-1 with x_c = b_c / U(c, c)
// and b_l -= x_c U(c, l) for l > c.  Lane l holds entries l, l + 64, ...; each
// step reads one contiguous row of U and broadcasts b_c from its lane, with no
// cross-lane reductions.  U was written by another workgroup (often another
// XCD), so rows are loaded INV_G steps ahead.
constexpr int INV_G = 4;

__device__ inline double rr_readlane(double v, int lane) {
    const uint64_t u = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// INV_SLOTS * 64 >= m: the launch picks the smallest of 8 and 16
template <int INV_SLOTS>
__global__ void __launch_bounds__(256)
k_rr_inv(const int* __restrict__ info, const double* __restrict__ U, double* __restrict__ Ui) {
    const int m = info[0];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + wave;
    if (i >= m) return;
    double x[INV_SLOTS], u[INV_G][INV_SLOTS], un[INV_G][INV_SLOTS];
    auto load = [&](double (&dst)[INV_G][INV_SLOTS], int c0) {
#pragma unroll
        for (int g = 0; g < INV_G; ++g)
#pragma unroll
            for (int t = 0; t < INV_SLOTS; ++t) {
                const int l = lane + 64 * t, c = c0 + g;
                dst[g][t] = (c < m && l < m) ? U[(int64_t)c * m + l] : 0.0;
            }
    };
#pragma unroll
    for (int t = 0; t < INV_SLOTS; ++t) x[t] = lane + 64 * t == i ? 1.0 : 0.0;
    load(u, i);
    for (int c0 = i; c0 < m; c0 += INV_G) {
        if (c0 + INV_G < m) load(un, c0 + INV_G);
#pragma unroll
        for (int g = 0; g < INV_G; ++g) {
            const int c = c0 + g;
            if (c >= m) break;
            const int tc = c >> 6, lc = c & 63;
            double bsrc = x[0], dsrc = u[g][0];
#pragma unroll
            for (int t = 1; t < INV_SLOTS; ++t)
                if (t == tc) {
                    bsrc = x[t];
                    dsrc = u[g][t];
                }
            const double xc = rr_readlane(bsrc, lc) / rr_readlane(dsrc, lc);
#pragma unroll
            for (int t = 0; t < INV_SLOTS; ++t) {
                const int l = lane + 64 * t;
                if (l == c) x[t] = xc;
                else if (l > c) x[t] -= xc * u[g][t];
            }
        }
#pragma unroll
        for (int g = 0; g < INV_G; ++g)
#pragma unroll
            for (int t = 0; t < INV_SLOTS; ++t) u[g][t] = un[g][t];
    }
#pragma unroll
    for (int t = 0; t < INV_SLOTS; ++t) {
        const int l = lane + 64 * t;
        if (l < m) Ui[(int64_t)i * m + l] = l >= i ? x[t] : 0.0;
    }
}

// --- step 3a (one workgroup): symmetrise M and reduce it to tridiagonal form
__global__ void __launch_bounds__(NT)
k_rr_tridiag(const int* __restrict__ info, double* __restrict__ M, double* __restrict__ dtau) {
    __shared__ double red[NWAVE + 1];
    __shared__ double sh[4];
    __shared__ double vs[MAXM], ps[MAXM];
    const int m = info[0];
    if (m == 0) return;
    for (int64_t q = threadIdx.x; q < (int64_t)m * m; q += NT) {
        const int a = (int)(q / m), b = (int)(q % m);
        if (a < b) {
            const double s = 0.5 * (M[(int64_t)a * m + b] + M[(int64_t)b * m + a]);
            M[(int64_t)a * m + b] = s;
            M[(int64_t)b * m + a] = s;
        }
    }
    __syncthreads();
    double* d = dtau;
    double* e = d + MAXM;
    double* tau = e + MAXM;
    tridiagonalize(m, M, d, e, tau, vs, ps, red, sh);
}

// --- step 3a on many workgroups (cooperative launch): the same Householder
// reduction, with the symmetric product p = tau A22 v and the rank-2 update
// spread over every wave of the grid (one wave per row, lanes along the row)
// and two grid barriers per column.  Every workgroup computes the reflector
// redundantly from the same row, so all take identical control flow.
constexpr int TD_NT = 256;
constexpr int TD_WAVES = TD_NT / 64;
constexpr int TD_GRID = 32;
static_assert(MAXM % TD_NT == 0, "the exchange loads take MAXM / TD_NT values per thread");
constexpr int TDL_GRID = 32;    // workgroups of the LDS-resident reduction
constexpr int TDL_RG = 4;       // rows per wave whose dot products run together
// bound on the spin of one barrier wait (each spin sleeps ~128 clocks); a
// wait that reaches it raises DEV_SYNC_TIMEOUT and the kernel runs to its end
constexpr unsigned long long TD_SPIN_LIMIT = 1ull << 26;

__device__ inline double wave_sum(double v) { return sc_wave_sum(v); }

__device__ inline double block_sum_td(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < TD_WAVES; ++w) s += red[w];
    __syncthreads();
    return s;
}

// grid barrier: bar[0] counts the arrivals of the whole launch (zero at
// launch); barrier number g (from 1) is passed once bar[0] reaches
// g * gridDim.x, so the last arrival's own increment releases every
// workgroup.  Thread 0 publishes the workgroup's writes with an agent-scope
// release fence before arriving and acquires the others' after the wait.
__device__ inline void grid_sync(unsigned* bar, unsigned& gen, int* status) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned target = (gen + 1u) * gridDim.x;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > TD_SPIN_LIMIT) {
                atomicOr(status, DEV_SYNC_TIMEOUT);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        gen = gen + 1u;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(TD_NT)
k_tridiag_coop(const int* __restrict__ info, double* __restrict__ M, double* __restrict__ dtau,
               double* __restrict__ P, unsigned* __restrict__ bar, int* status) {
    __shared__ double vs[MAXM], ws[MAXM];
    __shared__ double red[TD_WAVES];
    const int m = info[0];
    if (m == 0) return;
    unsigned gen = 0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gw = blockIdx.x * TD_WAVES + wave, GW = gridDim.x * TD_WAVES;
    // symmetrise; the pair (a, b), a < b, belongs to the wave of row a
    for (int a = gw; a < m; a += GW)
        for (int b = a + 1 + lane; b < m; b += 64) {
            const double sv = 0.5 * (M[(int64_t)a * m + b] + M[(int64_t)b * m + a]);
            M[(int64_t)a * m + b] = sv;
            M[(int64_t)b * m + a] = sv;
        }
    grid_sync(bar, gen, status);
    double* d = dtau;
    double* e = d + MAXM;
    double* tau = e + MAXM;
    for (int j = 0; j + 2 < m; ++j) {
        const int len = m - j - 1;
        const double* x = M + (int64_t)j * m + j + 1;
        double part = 0.0;
        for (int r = 1 + threadIdx.x; r < len; r += TD_NT) part = fma(x[r], x[r], part);
        const double sigma = block_sum_td(part, red);
        const double x0 = x[0];
        double tj, v0, ej;
        if (sigma == 0.0) {
            tj = 0.0;
            ej = x0;
            v0 = 1.0;
        } else {
            const double mu = sqrt(x0 * x0 + sigma);
            v0 = x0 <= 0.0 ? x0 - mu : -sigma / (x0 + mu);
            tj = 2.0 * v0 * v0 / (sigma + v0 * v0);
            ej = mu;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            d[j] = M[(int64_t)j * m + j];
            e[j] = ej;
            tau[j] = tj;
        }
        if (tj == 0.0) continue;          // same decision in every workgroup
        for (int r = threadIdx.x; r < len; r += TD_NT) vs[r] = r == 0 ? 1.0 : x[r] / v0;
        __syncthreads();
        for (int r = gw; r < len; r += GW) {
            const double* row = M + (int64_t)(j + 1 + r) * m + (j + 1);
            double sacc = 0.0;
            for (int c = lane; c < len; c += 64) sacc = fma(row[c], vs[c], sacc);
            sacc = wave_sum(sacc);
            if (lane == 0) P[r] = tj * sacc;
        }
        grid_sync(bar, gen, status);
        part = 0.0;
        for (int r = threadIdx.x; r < len; r += TD_NT) {
            const double pr = P[r];
            ws[r] = pr;
            part = fma(pr, vs[r], part);
        }
        const double K = 0.5 * tj * block_sum_td(part, red);
        for (int r = threadIdx.x; r < len; r += TD_NT) ws[r] = ws[r] - K * vs[r];
        __syncthreads();
        for (int r = gw; r < len; r += GW) {
            double* row = M + (int64_t)(j + 1 + r) * m + (j + 1);
            const double vr = vs[r], wr = ws[r];
            for (int c = lane; c < len; c += 64) row[c] -= vr * ws[c] + wr * vs[c];
        }
        // the reflector is kept in row j (not read again by the reduction)
        if (blockIdx.x == 0)
            for (int r = 1 + threadIdx.x; r < len; r += TD_NT) M[(int64_t)j * m + j + 1 + r] = vs[r];
        grid_sync(bar, gen, status);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (m >= 2) {
            d[m - 2] = M[(int64_t)(m - 2) * m + (m - 2)];
            e[m - 2] = M[(int64_t)(m - 2) * m + (m - 1)];
            tau[m - 2] = 0.0;
        }
        d[m - 1] = M[(int64_t)(m - 1) * m + (m - 1)];
        tau[m - 1] = 0.0;
    }
}

// The same reduction with every workgroup's rows resident in LDS and one grid
// barrier per column.  Row R belongs to workgroup R mod G (slot R / G), so
// the trailing block stays spread over all workgroups.  Every workgroup keeps
// the whole current column j (= row j, by symmetry) and computes the
// reflector from it.  At step j each workgroup
//   1. forms P_R = tau_j (A_R,trailing . v) for its rows and publishes P_R and
//      its rows' entries of column j + 1 (before this step's update);
//   2. after the barrier reads all of P and of column j + 1, forms
//      w = P - (tau_j / 2)(P . v) v, updates column j + 1 itself (it is the
//      next step's column) and applies A -= v w' + w v' to its own rows.
// The arithmetic of every element is that of the two-barrier kernel above.
// The exchange buffer X holds two sets (steps alternate) of P and column
// values, 4 * MAXM doubles; a set is rewritten only after the barrier that
// follows its last reader.
__global__ void __launch_bounds__(TD_NT)
k_tridiag_lds(const int* __restrict__ info, int m_max, double* __restrict__ M,
              double* __restrict__ dtau, double* __restrict__ X, unsigned* __restrict__ bar,
              int* status) {
    extern __shared__ double lds[];
    const int m = info[0];
    if (m == 0) return;
    const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slots = (m_max + G - 1) / G;
    double* A = lds;                              // slots x m_max (own rows)
    double* col = A + (int64_t)slots * m_max;     // current column, by row index
    double* vs = col + m_max;                     // reflector, by trailing index
    double* ws = vs + m_max;
    __shared__ double red[TD_WAVES];
    unsigned gen = 0;
    // own rows and column 0, symmetrised
    for (int s = 0; s * G + g < m; ++s) {
        const int R = s * G + g;
        for (int c = tid; c < m; c += TD_NT)
            A[(int64_t)s * m_max + c] = 0.5 * (M[(int64_t)R * m + c] + M[(int64_t)c * m + R]);
    }
    for (int R = tid; R < m; R += TD_NT) col[R] = 0.5 * (M[(int64_t)R * m] + M[R]);
    __syncthreads();
    double* d = dtau;
    double* e = d + MAXM;
    double* tau = e + MAXM;
    for (int j = 0; j + 2 < m; ++j) {
        const int len = m - j - 1;
        const double* x = col + j + 1;
        double part = 0.0;
        for (int r = 1 + tid; r < len; r += TD_NT) part = fma(x[r], x[r], part);
        const double sigma = block_sum_td(part, red);
        const double x0 = x[0];
        double tj, v0, ej;
        if (sigma == 0.0) {
            tj = 0.0;
            ej = x0;
            v0 = 1.0;
        } else {
            const double mu = sqrt(x0 * x0 + sigma);
            v0 = x0 <= 0.0 ? x0 - mu : -sigma / (x0 + mu);
            tj = 2.0 * v0 * v0 / (sigma + v0 * v0);
            ej = mu;
        }
        if (g == 0 && tid == 0) {
            d[j] = col[j];
            e[j] = ej;
            tau[j] = tj;
        }
        for (int r = tid; r < len; r += TD_NT) vs[r] = r == 0 ? 1.0 : x[r] / v0;
        __syncthreads();
        double* Pb = X + (int64_t)(j & 1) * 2 * MAXM;
        double* Cb = Pb + MAXM;
        // 1. own rows of the trailing block: P and the column j + 1 entries;
        //    a wave takes TDL_RG of its rows at once so their reductions overlap
        const int s0 = (j + 1 - g + G - 1) / G;   // first slot with R >= j + 1
        for (int s = s0 + wave; s * G + g < m; s += TDL_RG * TD_WAVES) {
            double sacc[TDL_RG];
            const double* row[TDL_RG];
            bool ok[TDL_RG];
#pragma unroll
            for (int q = 0; q < TDL_RG; ++q) {
                const int sq = s + q * TD_WAVES;
                ok[q] = sq * G + g < m;
                row[q] = A + (int64_t)(ok[q] ? sq : s) * m_max + (j + 1);
                sacc[q] = 0.0;
            }
            if (tj != 0.0) {
                for (int c = lane; c < len; c += 64) {
                    const double v = vs[c];
#pragma unroll
                    for (int q = 0; q < TDL_RG; ++q) sacc[q] = fma(row[q][c], v, sacc[q]);
                }
#pragma unroll
                for (int q = 0; q < TDL_RG; ++q) sacc[q] = sc_wave_sum(sacc[q]);
            }
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < TDL_RG; ++q) {
                    if (!ok[q]) continue;
                    const int R = (s + q * TD_WAVES) * G + g;
                    Pb[R] = tj * sacc[q];
                    Cb[R] = row[q][0];
                }
            }
        }
        grid_sync(bar, gen, status);
        // 2. w, the next column, and the update of the own rows.  All of a
        //    thread's loads of P and of the column are issued before any is
        //    used, so the exchange costs one memory latency.
        double pv[MAXM / TD_NT], cv[MAXM / TD_NT];
#pragma unroll
        for (int q = 0; q < MAXM / TD_NT; ++q) {
            const int r = tid + q * TD_NT;
            pv[q] = r < len ? Pb[j + 1 + r] : 0.0;
            cv[q] = r < len ? Cb[j + 1 + r] : 0.0;
        }
        part = 0.0;
#pragma unroll
        for (int q = 0; q < MAXM / TD_NT; ++q) {
            const int r = tid + q * TD_NT;
            if (r < len) {
                ws[r] = pv[q];
                col[j + 1 + r] = cv[q];
                part = fma(pv[q], vs[r], part);
            }
        }
        const double Kc = 0.5 * tj * block_sum_td(part, red);
        for (int r = tid; r < len; r += TD_NT) ws[r] = ws[r] - Kc * vs[r];
        __syncthreads();
        if (tj != 0.0)
            for (int r = tid; r < len; r += TD_NT)
                col[j + 1 + r] = col[j + 1 + r] - (vs[r] * ws[0] + ws[r] * vs[0]);
        if (tj != 0.0) {
            for (int s = s0 + wave; s * G + g < m; s += TD_WAVES) {
                const int r = s * G + g - (j + 1);
                double* row = A + (int64_t)s * m_max + (j + 1);
                const double vr = vs[r], wr = ws[r];
                for (int c = lane; c < len; c += 64) row[c] -= vr * ws[c] + wr * vs[c];
            }
            // the reflector is kept in row j (not read again by the reduction)
            if (g == 0)
                for (int r = 1 + tid; r < len; r += TD_NT) M[(int64_t)j * m + j + 1 + r] = vs[r];
        }
        __syncthreads();
    }
    if (g == 0 && tid == 0) {
        if (m >= 2) {
            d[m - 2] = col[m - 2];
            e[m - 2] = col[m - 1];
            tau[m - 2] = 0.0;
        }
        tau[m - 1] = 0.0;
    }
    // the last diagonal entry from its owner's row
    if (g == (m - 1) % G && tid == 0) d[m - 1] = A[(int64_t)((m - 1) / G) * m_max + (m - 1)];
}

size_t tridiag_lds_bytes(int m_max, int G) {
    const int slots = (m_max + G - 1) / G;
    return ((size_t)slots * m_max + 3 * (size_t)m_max) * sizeof(double);
}

__global__ void k_zero_u32(unsigned* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

__global__ void k_set_info(int* info, int m) {
    if (threadIdx.x == 0) info[0] = m;
}

__global__ void k_copy_f64(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// --- step 3c: Householder back-transform of the k eigenvectors, one wave each
// BK_W columns per workgroup, one per wave, held in registers (lane l owns
// entries l, l + 64, ...).  The reflectors are staged in LDS BK_NB at a time
// by the whole workgroup, so each is read from global memory once per
// workgroup, in bulk, instead of once per column and step.
constexpr int BK_NB = 8;
constexpr int BK_W = 16;
template <int SL>
__global__ void __launch_bounds__(BK_W * 64)
k_rr_back(int k, const int* __restrict__ info, const double* __restrict__ M,
          const double* __restrict__ dtau, double* __restrict__ Q) {
    __shared__ double refl[BK_NB][MAXM];
    __shared__ double tl[BK_NB];
    const int m = info[0];
    if (m == 0) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * BK_W + wave;
    const bool live = i < k;
    const double* tau = dtau + 2 * MAXM;
    double x[SL];
#pragma unroll
    for (int t = 0; t < SL; ++t) {
        const int e = lane + 64 * t;
        x[t] = (live && e < m) ? Q[(int64_t)e * k + i] : 0.0;
    }
    for (int jb = m - 3; jb >= 0; jb -= BK_NB) {
        __syncthreads();
        for (int q = 0; q < BK_NB; ++q) {
            const int j = jb - q;
            if (j < 0) break;
            const int len = m - j - 1;
            for (int r = threadIdx.x; r < len; r += BK_W * 64)
                refl[q][r] = r == 0 ? 1.0 : M[(int64_t)j * m + j + 1 + r];
            if (threadIdx.x == 0) tl[q] = tau[j];
        }
        __syncthreads();
        if (!live) continue;
        for (int q = 0; q < BK_NB; ++q) {
            const int j = jb - q;
            if (j < 0) break;
            const double tj = tl[q];
            if (tj == 0.0) continue;
            double part = 0.0;
#pragma unroll
            for (int t = 0; t < SL; ++t) {
                const int e = lane + 64 * t;
                if (e > j && e < m) part = fma(refl[q][e - j - 1], x[t], part);
            }
            const double sc = tj * sc_wave_sum(part);
#pragma unroll
            for (int t = 0; t < SL; ++t) {
                const int e = lane + 64 * t;
                if (e > j && e < m) x[t] -= sc * refl[q][e - j - 1];
            }
        }
    }
    if (!live) return;
#pragma unroll
    for (int t = 0; t < SL; ++t) {
        const int e = lane + 64 * t;
        if (e < m) Q[(int64_t)e * k + i] = x[t];
    }
}

// reduction to tridiagonal form: a cooperative kernel when the matrix is
// large enough to feed many workgroups (m_max >= 128), else one workgroup.
// `P` holds >= 4 MAXM doubles, `bar` two unsigned ints (zeroed before the launch).
static sc_status tridiagonalize_launch(sc_ctx* ctx, int m_max, const int* info, double* M,
                                       double* tri, double* P, unsigned* bar, int* status) {
    hipStream_t st = ctx->stream;
    if (m_max >= 128) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, bar, 2);
        // rows resident in LDS when they fit, else the two-barrier kernel
        const size_t lds = tridiag_lds_bytes(m_max, TDL_GRID);
        int lds_max = 0;
        if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) !=
            hipSuccess)
            lds_max = 0;
        if (lds + 1024 <= (size_t)lds_max &&
            hipFuncSetAttribute((const void*)k_tridiag_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) == hipSuccess) {
            void* args[] = {(void*)&info, (void*)&m_max, (void*)&M, (void*)&tri, (void*)&P,
                            (void*)&bar, (void*)&status};
            const hipError_t e = hipLaunchCooperativeKernel((const void*)k_tridiag_lds, dim3(TDL_GRID),
                                                            dim3(TD_NT), args, (unsigned)lds, st);
            if (e == hipSuccess) return SC_OK;
        }
        (void)hipGetLastError();
        void* args[] = {(void*)&info, (void*)&M, (void*)&tri, (void*)&P, (void*)&bar, (void*)&status};
        const hipError_t e = hipLaunchCooperativeKernel((const void*)k_tridiag_coop, dim3(TD_GRID),
                                                        dim3(TD_NT), args, 0, st);
        if (e == hipSuccess) return SC_OK;
        (void)hipGetLastError();
    }
    hipLaunchKernelGGL(k_rr_tridiag, dim3(1), dim3(NT), 0, st, info, M, tri);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}

// tridiagonalised M (in `M`, reflectors inside) + tri block -> k smallest
// eigenpairs (w, and V = m x k eigenvectors of M)
static void eig_pipeline(hipStream_t st, int m_max, int k, const int* info, const double* M,
                         double* tri, double* w, double* V, double* lu) {
    hipLaunchKernelGGL(k_tri_params, dim3(1), dim3(NT), 0, st, info, tri);
    hipLaunchKernelGGL(k_tri_bisect, dim3((unsigned)ceil_div(k, 4)), dim3(256), 0, st, k, info, tri, w);
    hipLaunchKernelGGL(k_tri_invit, dim3((unsigned)ceil_div(k, IV_T)), dim3(IV_T), 0, st, k, info,
                       tri, w, V, k, lu);
    // the inverse-iteration LU arrays (5 MAXM k doubles) are free again: cluster scratch
    hipLaunchKernelGGL(k_tri_bcgs, dim3(32), dim3(NT), 0, st, k, info, tri, w, V, k, lu);
    if (m_max <= 512)
        hipLaunchKernelGGL((k_rr_back<8>), dim3((unsigned)ceil_div(k, BK_W)), dim3(BK_W * 64), 0, st, k,
                           info, M, tri, V);
    else
        hipLaunchKernelGGL((k_rr_back<MAXM / 64>), dim3((unsigned)ceil_div(k, BK_W)), dim3(BK_W * 64),
                           0, st, k, info, M, tri, V);
}

// --- step 5: scatter C_act (m x k) to the rows of the active columns (the
// other rows were zeroed by k_rr_zero)
__global__ void k_rr_zero(int K3, int kp, int k, double* __restrict__ C64, float* __restrict__ C32,
                          double* __restrict__ theta) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (int64_t)K3 * kp) {
        C64[e] = 0.0;
        C32[e] = 0.0f;
    }
    if (e < kp && e >= k) theta[e] = 0.0;
}

__global__ void k_rr_scatter(int k, int kp, const int* __restrict__ info,
                             const double* __restrict__ Cq, double* __restrict__ C64,
                             float* __restrict__ C32) {
    const int m = info[0];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * k) return;
    const int a = (int)(e / k), i = (int)(e % k);
    const int row = info[1 + a];
    const double v = Cq[(int64_t)a * k + i];
    C64[(int64_t)row * kp + i] = v;
    C32[(int64_t)row * kp + i] = (float)v;
}

}  // namespace

size_t symeig_scratch_elems(int m, int k) {
    // matrix copy, d/e/tau/params, info, LU arrays
    return (size_t)m * m + 3 * (size_t)MAXM + 8 + (MAXM + 64) / 2 + 5 * (size_t)MAXM * k + 64;
}

size_t rr_scratch_elems(int K3, int k) {
    // U, Ui, Am, Tm (K3^2 each), Q and Cq (K3 x k), d/e/tau/params, info, LU arrays
    return 4 * (size_t)K3 * K3 + 2 * (size_t)K3 * k + 3 * (size_t)MAXM + 8 + (MAXM + 64) / 2 +
           5 * (size_t)MAXM * k + 64;
}

struct RrScratch {
    double *U, *Ui, *Am, *Tm, *Q, *Cq, *dtau, *ews;
    int* info;
    unsigned* bar;                            // grid-barrier words (in the tail slack)
    RrScratch(double* scratch, int K3, int k) {
        const size_t sq = (size_t)K3 * K3;
        U = scratch;
        Ui = U + sq;
        Am = Ui + sq;
        Tm = Am + sq;                         // A U^-1
        Q = Tm + sq;                          // m x k
        Cq = Q + (size_t)K3 * k;              // m x k
        dtau = Cq + (size_t)K3 * k;           // d, e, tau (3 x MAXM) + params
        info = reinterpret_cast<int*>(dtau + 3 * MAXM + 8);
        ews = dtau + 3 * MAXM + 8 + (MAXM + 64) / 2;   // inverse-iteration LU arrays
        bar = reinterpret_cast<unsigned*>(ews + 5 * (size_t)MAXM * k);
    }
};

sc_status launch_rr_setup(sc_ctx* ctx, int K3, int kp, int k, const double* GA, const double* GB,
                          int* act, double tol, double* scratch, int* status, int* counter,
                          const int* pred, int* probe, int* probe_counter, int* wcounter) {
    if (K3 > MAXM) return sc_fail(ctx, SC_E_UNSUPPORTED, "rayleigh_ritz: basis %d > %d", K3, MAXM);
    RrScratch w(scratch, K3, k);
    hipLaunchKernelGGL(k_rr_setup, dim3(1), dim3(NT), 0, ctx->stream, K3, kp, GA, GB, act, tol, w.U,
                       w.Am, w.info, status, counter, pred, probe, probe_counter, wcounter);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}

sc_status launch_rr_solve(sc_ctx* ctx, int K3, int kp, int k, double* C64, float* C32,
                          double* theta, double* scratch, int* status) {
    if (K3 > MAXM) return sc_fail(ctx, SC_E_UNSUPPORTED, "rayleigh_ritz: basis %d > %d", K3, MAXM);
    RrScratch w(scratch, K3, k);
    hipStream_t st = ctx->stream;
    if (K3 <= 512)
        hipLaunchKernelGGL((k_rr_inv<8>), dim3((unsigned)ceil_div(K3, 4)), dim3(256), 0, st, w.info,
                           w.U, w.Ui);
    else
        hipLaunchKernelGGL((k_rr_inv<MAXM / 64>), dim3((unsigned)ceil_div(K3, 4)), dim3(256), 0, st,
                           w.info, w.U, w.Ui);
    const dim3 gsq((unsigned)ceil_div(K3, 64), (unsigned)ceil_div(K3, 64));
    hipLaunchKernelGGL(k_gemm64, gsq, dim3(256), 0, st, w.info, 0, 0, w.Am, w.Ui, w.Tm);  // Tm = A U^-1
    hipLaunchKernelGGL(k_gemm64, gsq, dim3(256), 0, st, w.info, 0, 1, w.Ui, w.Tm, w.U);   // M = U^-T Tm
    SC_TRY(tridiagonalize_launch(ctx, K3, w.info, w.U, w.dtau, w.Tm, w.bar, status));   // Tm is free here
    eig_pipeline(st, K3, k, w.info, w.U, w.dtau, theta, w.Q, w.ews);
    const dim3 gk((unsigned)ceil_div(k, 64), (unsigned)ceil_div(K3, 64));
    hipLaunchKernelGGL(k_gemm64, gk, dim3(256), 0, st, w.info, k, 0, w.Ui, w.Q, w.Cq);    // C = U^-1 Q
    hipLaunchKernelGGL(k_rr_zero, dim3((unsigned)ceil_div((int64_t)K3 * kp, 256)), dim3(256), 0, st,
                       K3, kp, k, C64, C32, theta);
    hipLaunchKernelGGL(k_rr_scatter, dim3((unsigned)ceil_div((int64_t)K3 * k, 256)), dim3(256), 0,
                       st, k, kp, w.info, w.Cq, C64, C32);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}

sc_status launch_rayleigh_ritz(sc_ctx* ctx, int K3, int kp, int k, const double* GA,
                               const double* GB, int* act, double tol, double* C64, float* C32,
                               double* theta, double* scratch, int* status, int* counter,
                               int* wcounter) {
    SC_TRY(launch_rr_setup(ctx, K3, kp, k, GA, GB, act, tol, scratch, status, counter, nullptr,
                           nullptr, nullptr, wcounter));
    return launch_rr_solve(ctx, K3, kp, k, C64, C32, theta, scratch, status);
}

sc_status launch_symeig(sc_ctx* ctx, int m, int k, const double* A, double* w, double* V,
                        double* scratch) {
    if (m > MAXM) return sc_fail(ctx, SC_E_UNSUPPORTED, "symeig: m = %d > %d", m, MAXM);
    hipStream_t st = ctx->stream;
    double* M = scratch;
    double* tri = M + (size_t)m * m;
    int* info = reinterpret_cast<int*>(tri + 3 * MAXM + 8);
    double* lu = tri + 3 * MAXM + 8 + (MAXM + 64) / 2;
    unsigned* bar = reinterpret_cast<unsigned*>(lu + 5 * (size_t)MAXM * k);
    int* flags = reinterpret_cast<int*>(bar + 2);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, bar, 4);
    hipLaunchKernelGGL(k_copy_f64, dim3((unsigned)ceil_div((int64_t)m * m, 256)), dim3(256), 0, st,
                       (int64_t)m * m, A, M);
    hipLaunchKernelGGL(k_set_info, dim3(1), dim3(64), 0, st, info, m);
    SC_TRY(tridiagonalize_launch(ctx, m, info, M, tri, lu, bar, flags));
    eig_pipeline(st, m, k, info, M, tri, w, V, lu);
    SC_CHECK_LAUNCH(ctx);
    int h = 0;
    SC_CHECK_HIP(ctx, hipMemcpyAsync(&h, flags, sizeof h, hipMemcpyDeviceToHost, st));
    SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
    if (h & DEV_SYNC_TIMEOUT) return sc_fail(ctx, SC_E_HIP, "symeig: grid barrier wait timed out");
    return SC_OK;
}

extern "C" sc_status sc_symeig_workspace(sc_ctx* ctx, int m, int k, size_t* bytes) {
    if (!ctx || !bytes) return SC_E_INVAL;
    if (m <= 0 || k <= 0 || k > m || m > MAXM)
        return sc_fail(ctx, SC_E_INVAL, "symeig: need 0 < k <= m <= %d", MAXM);
    *bytes = symeig_scratch_elems(m, k) * sizeof(double) + 256;
    return SC_OK;
}

extern "C" sc_status sc_symeig(sc_ctx* ctx, int m, int k, const double* A, double* w, double* V,
                               void* ws, size_t ws_bytes) {
    if (!ctx) return SC_E_INVAL;
    size_t need = 0;
    SC_TRY(sc_symeig_workspace(ctx, m, k, &need));
    if (!A || !w || !V || !ws) return sc_fail(ctx, SC_E_INVAL, "symeig: null pointer argument");
    if (ws_bytes < need) return sc_fail(ctx, SC_E_NOMEM, "symeig: workspace too small");
    SC_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    return launch_symeig(ctx, m, k, A, w, V, static_cast<double*>(ws));
}
