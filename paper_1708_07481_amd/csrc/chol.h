// Cholesky factorisation of a small symmetric positive definite matrix by
// one workgroup, blocked for bandwidth: B = R'R with R upper triangular,
// computed in place in the upper triangle of a row-major m x m array U in
// global memory (the strict lower triangle is not read).
//
// Right-looking with panels of CHOL_NB rows:
//   1. the CHOL_NB x CHOL_NB diagonal block is factored in LDS (pivot test
//      s_j > tol * diag0_j against the matrix's original diagonal);
//   2. the panel rows right of the block are solved, R_pp' X = A_p,rest, one
//      thread per column (the column's panel entries loaded before the
//      substitution starts), and kept in LDS;
//   3. the trailing upper triangle is updated, A -= X'X: a wave takes four
//      rows and up to 256 columns from the first upper one, each lane four
//      columns 64 apart, so that a wave's LDS reads of X are one broadcast
//      (the rows) and consecutive words (the columns), free of bank conflicts.
// Each trailing element is read and written once per panel (instead of once
// per column in the unblocked form).  Every element takes the same sequence
// of operations whatever the workgroup size.
#pragma once

#include <hip/hip_runtime.h>

constexpr int CHOL_NB = 16;
constexpr int CHOL_MAXM = 1024;

struct CholLds {
    double panel[CHOL_NB][CHOL_MAXM];     // rows of the current panel, trailing columns
    double blk[CHOL_NB][CHOL_NB + 1];     // diagonal block
    double diag0[CHOL_MAXM];              // original diagonal (pivot reference)
    int fail_at;
};

// Returns -1 on success, else the index of the first failing pivot (the
// factor is then incomplete).  All threads of the workgroup must call it.
template <int NTH>
__device__ inline int chol_blocked(int m, double* __restrict__ U, double tol, CholLds& L) {
    const int tid = threadIdx.x;
    for (int j = tid; j < m; j += NTH) L.diag0[j] = U[(int64_t)j * m + j];
    if (tid == 0) L.fail_at = -1;
    __syncthreads();
    for (int p0 = 0; p0 < m; p0 += CHOL_NB) {
        const int nb = min(CHOL_NB, m - p0);
        const int q0 = p0 + nb;
        const int len = m - q0;
        // 1. diagonal block into LDS and factored there (tiny: thread 0 takes
        //    the pivots, the block's threads the row updates)
        for (int e = tid; e < nb * nb; e += NTH) {
            const int a = e / nb, b = e % nb;
            L.blk[a][b] = U[(int64_t)(p0 + a) * m + p0 + b];
        }
        __syncthreads();
        for (int jj = 0; jj < nb; ++jj) {
            if (tid == 0) {
                const double s = L.blk[jj][jj];
                if (!isfinite(s) || !(s > tol * L.diag0[p0 + jj]) || !(s > 0.0))
                    L.fail_at = p0 + jj;
                else
                    L.blk[jj][jj] = sqrt(s);
            }
            __syncthreads();
            if (L.fail_at >= 0) return L.fail_at;
            const double rjj = L.blk[jj][jj];
            for (int b = jj + 1 + tid; b < nb; b += NTH) L.blk[jj][b] /= rjj;
            __syncthreads();
            const int rem = nb - jj - 1;
            for (int e = tid; e < rem * rem; e += NTH) {
                const int a = jj + 1 + e / rem, b = jj + 1 + e % rem;
                if (b >= a) L.blk[a][b] -= L.blk[jj][a] * L.blk[jj][b];
            }
            __syncthreads();
        }
        for (int e = tid; e < nb * nb; e += NTH) {
            const int a = e / nb, b = e % nb;
            if (b >= a) U[(int64_t)(p0 + a) * m + p0 + b] = L.blk[a][b];
        }
        // 2. panel solve: column c of the rows p0..q0-1, forward substitution
        for (int c = tid; c < len; c += NTH) {
            double x[CHOL_NB];                    // the loaded entries, then the solution
#pragma unroll
            for (int i = 0; i < CHOL_NB; ++i) x[i] = i < nb ? U[(int64_t)(p0 + i) * m + q0 + c] : 0.0;
#pragma unroll
            for (int i = 0; i < CHOL_NB; ++i) {
                if (i < nb) {
                    double s = x[i];
                    for (int l = 0; l < i; ++l) s -= L.blk[l][i] * x[l];
                    x[i] = s / L.blk[i][i];
                    U[(int64_t)(p0 + i) * m + q0 + c] = x[i];
                    L.panel[i][c] = x[i];
                }
            }
        }
        __syncthreads();
        // 3. trailing update of the upper triangle: rows a0..a0+3 of a wave,
        //    columns a0 + 256 cb + lane + 64 c of a lane (clamped reads, masked
        //    writes)
        const int wave = tid >> 6, lane = tid & 63;
        for (int ta = wave; 4 * ta < len; ta += NTH / 64) {
            const int a0 = 4 * ta;
            double* __restrict__ Ur = U + (int64_t)(q0 + a0) * m + q0;
            for (int cb = 0; a0 + 256 * cb < len; ++cb) {
                int bc[4];
                bool okc[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int b = a0 + 256 * cb + lane + 64 * c;
                    okc[c] = b < len;
                    bc[c] = okc[c] ? b : len - 1;
                }
                double acc[4][4] = {};
                for (int i = 0; i < nb; ++i) {
                    double xa[4], xb[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) xa[r] = L.panel[i][min(a0 + r, len - 1)];
#pragma unroll
                    for (int c = 0; c < 4; ++c) xb[c] = L.panel[i][bc[c]];
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int c = 0; c < 4; ++c) acc[r][c] = fma(xa[r], xb[c], acc[r][c]);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (a0 + r >= len) break;
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (okc[c] && bc[c] >= a0 + r) Ur[(int64_t)r * m + bc[c]] -= acc[r][c];
                }
            }
        }
        __syncthreads();
    }
    return -1;
}

// In-place inverse of the upper triangular factor into Ri (row-major m x m,
// zero below the diagonal), one wave per column with the column in LDS.
// `col` holds (NTH / 64) x CHOL_MAXM doubles.
template <int NTH>
__device__ inline void tri_inv_upper(int m, const double* __restrict__ R, double* __restrict__ Ri,
                                     double* col) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double* cj = col + wave * CHOL_MAXM;
    for (int j = wave; j < m; j += NTH / 64) {
        if (lane == 0) cj[j] = 1.0 / R[(int64_t)j * m + j];
        __builtin_amdgcn_wave_barrier();
        for (int a = j - 1; a >= 0; --a) {
            double part = 0.0;
            for (int l = a + 1 + lane; l <= j; l += 64) part = fma(R[(int64_t)a * m + l], cj[l], part);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
            if (lane == 0) cj[a] = -part / R[(int64_t)a * m + a];
            __builtin_amdgcn_wave_barrier();
        }
        for (int a = lane; a < m; a += 64) Ri[(int64_t)a * m + j] = a <= j ? cj[a] : 0.0;
        __builtin_amdgcn_wave_barrier();
    }
}
