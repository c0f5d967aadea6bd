// Dense multivector kernels of the LOBPCG iteration: Gram products of
// tall-skinny blocks, Cholesky-QR factors of small Gram matrices, in-place
// right multiplications of row blocks, the fused block update and the
// residual with its column norms.
//
// Reductions over the n rows are split into row chunks whose FP64 partial
// results are summed in chunk order by a second kernel, so every result is
// deterministic (no floating-point atomics).
#include "chol.h"
#include "sc_internal.h"
#include <type_traits>

namespace {

// ---------------------------------------------------------------------------
// Gram products on the matrix cores.  Each of the four waves of a workgroup
// owns a (16 WT) x (16 WT) block of the output (the workgroup a 2x2 arrangement
// of them) and accumulates WT x WT MFMA 16x16 tiles for both outputs while
// walking its row chunk KR rows at a time.  Operand lanes (16x16xK MFMA):
// lane l supplies column (l % 16) of its 16-wide column strip at rows
// r0 + KR/4 * (l / 16) + t; the accumulator's element v of lane l is output
// row 4 (l / 16) + v (FP32, BF16) or (l / 16) + 4 v (FP64), column l % 16.
//   float : v_mfma_f32_16x16x4_f32   (FP32 in, FP32 accumulate)
//   double: v_mfma_f64_16x16x4_f64   (FP64 in, FP64 accumulate)
//   bf16  : v_mfma_f32_16x16x32_bf16 (FP32 in, rounded to BF16 (RNE), FP32 accumulate)
//   f32x64: v_mfma_f64_16x16x4_f64   (FP32 in, widened: exact products, FP64 accumulate)
// ---------------------------------------------------------------------------
typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef __bf16 mf_bf8 __attribute__((ext_vector_type(8)));

__device__ inline __bf16 to_bf16_rne(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
}

struct MfF32 {
    using in_t = float;
    using acc_t = mf_f4;
    using frag_t = float;
    static constexpr int KR = 4;
    static constexpr int WT = 5;
    __device__ static int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
    __device__ static frag_t load(const float* __restrict__ M, int64_t ld, int64_t r0, int64_t r1,
                                  int col, int c, int lane) {
        const int64_t r = r0 + (lane >> 4);
        return (r < r1 && col < c) ? M[r * ld + col] : 0.0f;
    }
    // fragment from an LDS tile T[k][col] (row stride ls)
    __device__ static frag_t lds(const float* T, int ls, int k, int col, int lane) {
        return T[(k + (lane >> 4)) * ls + col];
    }
    __device__ static acc_t mma(frag_t a, frag_t b, acc_t acc) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
};
struct MfF64 {
    using in_t = double;
    using acc_t = mf_d4;
    using frag_t = double;
    static constexpr int KR = 4;
    static constexpr int WT = 2;
    __device__ static int out_row(int lane, int v) { return (lane >> 4) + 4 * v; }
    __device__ static frag_t load(const double* __restrict__ M, int64_t ld, int64_t r0, int64_t r1,
                                  int col, int c, int lane) {
        const int64_t r = r0 + (lane >> 4);
        return (r < r1 && col < c) ? M[r * ld + col] : 0.0;
    }
    __device__ static acc_t mma(frag_t a, frag_t b, acc_t acc) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
};
struct MfF32x64 {
    using in_t = float;
    using acc_t = mf_d4;
    using frag_t = double;
    static constexpr int KR = 4;
    static constexpr int WT = 2;
    __device__ static int out_row(int lane, int v) { return (lane >> 4) + 4 * v; }
    __device__ static frag_t load(const float* __restrict__ M, int64_t ld, int64_t r0, int64_t r1,
                                  int col, int c, int lane) {
        const int64_t r = r0 + (lane >> 4);
        return (r < r1 && col < c) ? (double)M[r * ld + col] : 0.0;
    }
    __device__ static frag_t lds(const float* T, int ls, int k, int col, int lane) {
        return (double)T[(k + (lane >> 4)) * ls + col];
    }
    __device__ static acc_t mma(frag_t a, frag_t b, acc_t acc) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
};
struct MfBF16 {
    using in_t = float;
    using acc_t = mf_f4;
    using frag_t = mf_bf8;
    static constexpr int KR = 32;
    static constexpr int WT = 5;
    __device__ static int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
    __device__ static frag_t load(const float* __restrict__ M, int64_t ld, int64_t r0, int64_t r1,
                                  int col, int c, int lane) {
        frag_t f;
        const int64_t rb = r0 + 8 * (lane >> 4);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int64_t r = rb + t;
            f[t] = to_bf16_rne((r < r1 && col < c) ? M[r * ld + col] : 0.0f);
        }
        return f;
    }
    __device__ static frag_t lds(const float* T, int ls, int k, int col, int lane) {
        frag_t f;
        const int kb = k + 8 * (lane >> 4);
#pragma unroll
        for (int t = 0; t < 8; ++t) f[t] = to_bf16_rne(T[(kb + t) * ls + col]);
        return f;
    }
    __device__ static acc_t mma(frag_t a, frag_t b, acc_t acc) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
};

template <class MF, bool TWO>
__global__ void __launch_bounds__(256)
k_gram_mfma(int64_t n, int c, int64_t chunk_rows, const typename MF::in_t* __restrict__ A, int64_t lda,
            const typename MF::in_t* __restrict__ B1, int64_t ldb1,
            const typename MF::in_t* __restrict__ B2, int64_t ldb2, double* __restrict__ partial,
            int tiles, const int* __restrict__ pred) {
    if (pred && *pred == 0) return;
    constexpr int WT = MF::WT;
    constexpr int WTILE = 16 * WT;          // wave tile edge
    constexpr int BT = 2 * WTILE;           // workgroup tile edge
    int t = blockIdx.x, ti = 0;
    while (t >= tiles - ti) {
        t -= tiles - ti;
        ++ti;
    }
    const int tj = ti + t;
    const int chunk = blockIdx.y;
    const int64_t r0 = (int64_t)chunk * chunk_rows;
    const int64_t r1 = min<int64_t>(n, r0 + chunk_rows);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ca = ti * BT + (wave >> 1) * WTILE;      // this wave's output rows (columns of A)
    const int cb = tj * BT + (wave & 1) * WTILE;       // this wave's output cols (columns of B)
    using acc_t = typename MF::acc_t;
    acc_t acc1[WT][WT], acc2[WT][WT];
#pragma unroll
    for (int p = 0; p < WT; ++p)
#pragma unroll
        for (int q = 0; q < WT; ++q) {
            acc1[p][q] = acc_t{0, 0, 0, 0};
            acc2[p][q] = acc_t{0, 0, 0, 0};
        }
    const int lc = lane & 15;
    for (int64_t row = r0; row < r1; row += MF::KR) {
        typename MF::frag_t fa[WT], fb1[WT], fb2[WT];
#pragma unroll
        for (int p = 0; p < WT; ++p) fa[p] = MF::load(A, lda, row, r1, ca + 16 * p + lc, c, lane);
#pragma unroll
        for (int q = 0; q < WT; ++q) {
            fb1[q] = MF::load(B1, ldb1, row, r1, cb + 16 * q + lc, c, lane);
            if (TWO) fb2[q] = MF::load(B2, ldb2, row, r1, cb + 16 * q + lc, c, lane);
        }
#pragma unroll
        for (int p = 0; p < WT; ++p)
#pragma unroll
            for (int q = 0; q < WT; ++q) {
                acc1[p][q] = MF::mma(fa[p], fb1[q], acc1[p][q]);
                if (TWO) acc2[p][q] = MF::mma(fa[p], fb2[q], acc2[p][q]);
            }
    }
    const int64_t cc2 = (int64_t)c * c;
    double* p1 = partial + (int64_t)chunk * (TWO ? 2 : 1) * cc2;
    double* p2 = p1 + cc2;
#pragma unroll
    for (int p = 0; p < WT; ++p)
#pragma unroll
        for (int q = 0; q < WT; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = ca + 16 * p + MF::out_row(lane, v);
                const int b = cb + 16 * q + lc;
                if (a < c && b < c) {
                    p1[(int64_t)a * c + b] = (double)acc1[p][q][v];
                    if (TWO) p2[(int64_t)a * c + b] = (double)acc2[p][q][v];
                }
            }
}

// The same products for FP32 data with the operand tiles staged through LDS:
// per chunk of GL_KC rows, the A columns [ca, ca + BT) and the B columns
// [cb, cb + BT) are loaded with 16-byte coalesced loads into registers one
// chunk ahead (rows beyond the chunk or columns beyond c as zeros), stored to
// LDS, and the waves read their MFMA fragments from LDS.  Rows are padded to BT + 16 floats (bank spread of the 4-row fragment
// reads).  Needs 16-byte aligned operands and row strides.
constexpr int GL_KC = 32;

template <int BT>
struct GramStage {
    static constexpr int LS = BT + 16;
    static constexpr int V4 = BT / 4;                      // float4 per staged row
    static constexpr int PER = GL_KC * V4 / 256;            // float4 per thread
    float4 v[PER];
    // global -> registers (issued ahead of the compute on the previous chunk)
    __device__ void load(const float* __restrict__ M, int64_t ld, int64_t row, int64_t r1, int col0,
                         int c) {
        if (row + GL_KC <= r1 && col0 + BT <= c) {
            // a whole chunk inside the matrix: plain loads, no per-element tests
            // (the issue slots between the matrix-core instructions stay free)
            const float* base = M + row * ld + col0;
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int q = threadIdx.x + 256 * u;
                const int rr = q / V4, cc = 4 * (q % V4);
                v[u] = *reinterpret_cast<const float4*>(base + rr * ld + cc);
            }
            return;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = threadIdx.x + 256 * u;
            const int rr = q / V4, cc = 4 * (q % V4);
            const int64_t r = row + rr;
            const int col = col0 + cc;
            float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < r1) {
                const float* src = M + r * ld + col;
                if (col + 3 < c) {
                    x = *reinterpret_cast<const float4*>(src);
                } else {
                    if (col < c) x.x = src[0];
                    if (col + 1 < c) x.y = src[1];
                    if (col + 2 < c) x.z = src[2];
                }
            }
            v[u] = x;
        }
    }
    // registers -> LDS tile T[rr][cc] (LS and cc are multiples of 4)
    __device__ void store(float* T) const {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = threadIdx.x + 256 * u;
            const int rr = q / V4, cc = 4 * (q % V4);
            *reinterpret_cast<float4*>(T + rr * LS + cc) = v[u];
        }
    }
};

// One wave's piece of a workgroup tile: the MFMA sub-tiles [pa0, pa0 + NP) x
// [qb0, qb0 + NQ) of the tile's (BT/16) x (BT/16) grid, with TRI keeping only
// q >= p (a piece on the diagonal of a diagonal tile).  All four waves of the
// workgroup run this loop with the same row range, so they meet at the same
// barriers whatever their pieces.  B1s or B2s may alias As (the same columns of
// the same matrix): the caller then skips staging them.
template <class MF, bool TWO, int NP, int NQ, bool TRI, bool PART>
__device__ __forceinline__ void gram_piece(int64_t r0, int64_t r1, int c, int ca, int cb,
                                           const float* __restrict__ A, int64_t lda,
                                           const float* __restrict__ B1, int64_t ldb1,
                                           const float* __restrict__ B2, int64_t ldb2,
                                           float* As, float* B1s, float* B2s, bool ld1, bool ld2,
                                           int pa0, int qb0, double* p1, double* p2, int gap_lo,
                                           int gap_hi) {
    constexpr int BT = 32 * MF::WT;
    constexpr int LS = BT + 16;
    const int lane = threadIdx.x & 63, lc = lane & 15;
    // PART: MFMA sub-tiles wholly past column c, or wholly inside the unused
    // columns [gap_lo, gap_hi), are skipped (their results are never read)
    bool pok[NP], qok[NQ];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int s0 = ca + 16 * (pa0 + p);
        pok[p] = !PART || (s0 < c && !(s0 >= gap_lo && s0 + 16 <= gap_hi));
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int s0 = cb + 16 * (qb0 + q);
        qok[q] = !PART || (s0 < c && !(s0 >= gap_lo && s0 + 16 <= gap_hi));
    }
    using acc_t = typename MF::acc_t;
    acc_t acc1[NP][NQ], acc2[NP][NQ];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            acc1[p][q] = acc_t{0, 0, 0, 0};
            acc2[p][q] = acc_t{0, 0, 0, 0};
        }
    GramStage<BT> ga, gb1, gb2;
    if (r0 < r1) {
        ga.load(A, lda, r0, r1, ca, c);
        if (ld1) gb1.load(B1, ldb1, r0, r1, cb, c);
        if (TWO && ld2) gb2.load(B2, ldb2, r0, r1, cb, c);
    }
    for (int64_t row = r0; row < r1; row += GL_KC) {
        __syncthreads();
        ga.store(As);
        if (ld1) gb1.store(B1s);
        if (TWO && ld2) gb2.store(B2s);
        __syncthreads();
        if (row + GL_KC < r1) {                 // next chunk in flight during this one's MFMAs
            ga.load(A, lda, row + GL_KC, r1, ca, c);
            if (ld1) gb1.load(B1, ldb1, row + GL_KC, r1, cb, c);
            if (TWO && ld2) gb2.load(B2, ldb2, row + GL_KC, r1, cb, c);
        }
#pragma unroll 2
        for (int k = 0; k < GL_KC; k += MF::KR) {
            typename MF::frag_t fa[NP], fb1[NQ], fb2[NQ];
#pragma unroll
            for (int p = 0; p < NP; ++p) fa[p] = MF::lds(As, LS, k, 16 * (pa0 + p) + lc, lane);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                fb1[q] = MF::lds(B1s, LS, k, 16 * (qb0 + q) + lc, lane);
                if (TWO) fb2[q] = MF::lds(B2s, LS, k, 16 * (qb0 + q) + lc, lane);
            }
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    if (TRI && q < p) continue;
                    if (PART && !(pok[p] && qok[q])) continue;
                    acc1[p][q] = MF::mma(fa[p], fb1[q], acc1[p][q]);
                    if (TWO) acc2[p][q] = MF::mma(fa[p], fb2[q], acc2[p][q]);
                }
        }
    }
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (TRI && q < p) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = ca + 16 * (pa0 + p) + MF::out_row(lane, v);
                const int b = cb + 16 * (qb0 + q) + lc;
                if (a < c && b < c) {
                    p1[(int64_t)a * c + b] = (double)acc1[p][q][v];
                    if (TWO) p2[(int64_t)a * c + b] = (double)acc2[p][q][v];
                }
            }
        }
}

// one (tile pair, row chunk) item of the FP32 Gram kernel
template <class MF, bool TWO, bool PART>
__device__ __forceinline__ void gram_tile(int64_t n, int c, int64_t chunk_rows,
                                          const float* __restrict__ A, int64_t lda,
                                          const float* __restrict__ B1, int64_t ldb1,
                                          const float* __restrict__ B2, int64_t ldb2,
                                          double* __restrict__ partial, int ti, int tj, int chunk,
                                          float* As, float* B1s, float* B2s, int gap_lo,
                                          int gap_hi) {
    constexpr int WT = MF::WT;
    constexpr int BT = 32 * WT;
    const int64_t r0 = (int64_t)chunk * chunk_rows;
    const int64_t r1 = min<int64_t>(n, r0 + chunk_rows);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int ca = ti * BT, cb = tj * BT;
    const int64_t cc2 = (int64_t)c * c;
    double* p1 = partial + (int64_t)chunk * (TWO ? 2 : 1) * cc2;
    double* p2 = p1 + cc2;
    if (ti != tj) {
        gram_piece<MF, TWO, WT, WT, false, PART>(r0, r1, c, ca, cb, A, lda, B1, ldb1, B2, ldb2, As, B1s,
                                           B2s, true, true, (wave >> 1) * WT, (wave & 1) * WT, p1,
                                           p2, gap_lo, gap_hi);
        return;
    }
    const bool same1 = B1 == A && ldb1 == lda;
    const bool same2 = TWO && B2 == A && ldb2 == lda;
    float* b1s = same1 ? As : B1s;
    float* b2s = same2 ? As : B2s;
    constexpr int QA = (WT + 1) / 2, QB = WT / 2;
    switch (wave) {
    case 0:
        gram_piece<MF, TWO, WT, WT, true, PART>(r0, r1, c, ca, cb, A, lda, B1, ldb1, B2, ldb2, As, b1s,
                                          b2s, !same1, !same2, 0, 0, p1, p2, gap_lo, gap_hi);
        break;
    case 1:
        gram_piece<MF, TWO, WT, WT, true, PART>(r0, r1, c, ca, cb, A, lda, B1, ldb1, B2, ldb2, As, b1s,
                                          b2s, !same1, !same2, WT, WT, p1, p2, gap_lo,
                                                gap_hi);
        break;
    case 2:
        gram_piece<MF, TWO, WT, QA, false, PART>(r0, r1, c, ca, cb, A, lda, B1, ldb1, B2, ldb2, As, b1s,
                                           b2s, !same1, !same2, 0, WT, p1, p2, gap_lo,
                                                 gap_hi);
        break;
    default:
        gram_piece<MF, TWO, WT, QB, false, PART>(r0, r1, c, ca, cb, A, lda, B1, ldb1, B2, ldb2, As, b1s,
                                           b2s, !same1, !same2, 0, WT + QA, p1, p2,
                                                 gap_lo, gap_hi);
        break;
    }
}

// Only the upper triangle of a Gram product is reduced and mirrored, so a
// diagonal tile (ti == tj) needs only its MFMA sub-tiles with q >= p: 55 of
// 100 for WT = 5.  Off the diagonal each wave owns a WT x WT quarter; on it the
// four waves split the upper sub-tiles into two diagonal triangles and the
// off-diagonal quarter cut in two column strips (15, 15, 15 and 10 sub-tiles
// for WT = 5), so the tile's barrier-to-barrier time follows the largest piece.
// On a diagonal tile a B operand that is the A matrix itself (S'S, V'V) is the
// A tile already in LDS and is not staged again.
//
// PERSIST: as many workgroups as fit on the device at once (one per CU here)
// take (tile pair, chunk) items from a counter.  Measured per workgroup,
// one-item-per-workgroup launches left a CU idle about 120 us between items
// and spread 5 to 8 items over the CUs, 17 % of the kernel's time.  The BF16
// instantiation stays one item per workgroup: its loop would spill.
// Item -> (tile pair, chunk): the off-diagonal (longer) items first, so the
// last items to finish are short.
__device__ __forceinline__ void gram_item(int item, int tiles, int chunks, int& ti, int& tj,
                                          int& chunk) {
    const int noff = tiles * (tiles - 1) / 2;
    if (item < noff * chunks) {
        int m = item % noff;
        chunk = item / noff;
        ti = 0;
        while (m >= tiles - 1 - ti) {           // off-diagonal pairs of row ti: tj > ti
            m -= tiles - 1 - ti;
            ++ti;
        }
        tj = ti + 1 + m;
    } else {
        const int j = item - noff * chunks;
        ti = tj = j % tiles;
        chunk = j / tiles;
    }
}

template <class MF, bool TWO, bool PERSIST, bool PART>
__global__ void __launch_bounds__(256)
k_gram_lds(int64_t n, int c, int64_t chunk_rows, const float* __restrict__ A, int64_t lda,
           const float* __restrict__ B1, int64_t ldb1, const float* __restrict__ B2, int64_t ldb2,
           double* __restrict__ partial, int tiles, int chunks, int* __restrict__ queue,
           int gap_lo, int gap_hi, const int* __restrict__ pred) {
    if (pred && *pred == 0) return;
    constexpr int WT = MF::WT;
    constexpr int BT = 32 * WT;
    constexpr int LS = BT + 16;
    __shared__ __attribute__((aligned(16))) float As[GL_KC * LS];
    __shared__ __attribute__((aligned(16))) float B1s[GL_KC * LS];
    __shared__ __attribute__((aligned(16))) float B2s[TWO ? GL_KC * LS : 4];
    const int upper = tiles * (tiles + 1) / 2;
    const int items = upper * chunks;
    if (!PERSIST) {                             // one item per workgroup
        int ti, tj, chunk;
        gram_item((int)blockIdx.x, tiles, chunks, ti, tj, chunk);
        gram_tile<MF, TWO, PART>(n, c, chunk_rows, A, lda, B1, ldb1, B2, ldb2, partial, ti, tj, chunk,
                                 As, B1s, B2s, gap_lo, gap_hi);
        return;
    }
    __shared__ int item_s;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(&queue[0], 1);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= items) break;
        int ti, tj, chunk;
        gram_item(item, tiles, chunks, ti, tj, chunk);
        // a tile wholly inside the unused columns: nothing of the pair is read
        if (PART && ((ti * BT >= gap_lo && (ti + 1) * BT <= gap_hi) ||
                     (tj * BT >= gap_lo && (tj + 1) * BT <= gap_hi)))
            continue;
        // only the items that reach past column c or into the unused columns
        // take the sub-tile tests; the others run the unconditional code
        const bool part_item =
            PART && ((tj + 1) * BT > c || (ti * BT < gap_hi && (ti + 1) * BT > gap_lo) ||
                     (tj * BT < gap_hi && (tj + 1) * BT > gap_lo));
        if (part_item)
            gram_tile<MF, TWO, true>(n, c, chunk_rows, A, lda, B1, ldb1, B2, ldb2, partial, ti, tj,
                                     chunk, As, B1s, B2s, gap_lo, gap_hi);
        else
            gram_tile<MF, TWO, false>(n, c, chunk_rows, A, lda, B1, ldb1, B2, ldb2, partial, ti, tj,
                                      chunk, As, B1s, B2s, gap_lo, gap_hi);
    }
    if (threadIdx.x == 0 && atomicAdd(&queue[1], 1) == (int)gridDim.x - 1) {   // PERSIST only
        atomicExch(&queue[0], 0);               // last one out: ready for the next launch
        atomicExch(&queue[1], 0);
    }
}

// sum the chunk partials in chunk order; upper entries, mirrored
__global__ void k_gram_reduce(int c, int chunks, int nout, const double* __restrict__ partial,
                              double* __restrict__ G1, double* __restrict__ G2,
                              const int* __restrict__ pred) {
    if (pred && *pred == 0) return;
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
constexpr int CQ_TH = 1024;
// Ritz values further than this (relative to op_norm / 2, i.e. absolute for the
// normalised Laplacian's [0, 2]) outside [0, op_norm] mark an inconsistent iterate
constexpr double RESTART_THETA_SLACK = 1e-3;
constexpr int CQ_MAX = 256;

__global__ void __launch_bounds__(CQ_TH)
k_cholqr_factor(int c, const double* __restrict__ G, int* __restrict__ mask, double tol,
                double* __restrict__ T64, float* __restrict__ T32, double* __restrict__ scr,
                int mode, int* status, int* counter) {
    __shared__ int idx[CQ_MAX];
    __shared__ double d[CQ_MAX];
    __shared__ int m_s, fail_s, fail_at;
    __shared__ CholLds L;
    const int tid = threadIdx.x;
    int m = 0;
    double* R = scr;                     // m x m equilibrated Gram, factored in place
    double* Ri = nullptr;                // m x m inverse
    // CQ_DROP_DEPENDENT removes one failing column per pass and refactors
    for (int pass = 0; pass <= c; ++pass) {
        if (tid == 0) {
            int mm = 0, missing = 0;
            for (int j = 0; j < c; ++j) {
                const double g = G[(int64_t)j * c + j];
                if (mask[j] && isfinite(g) && g > 0.0) {
                    idx[mm] = j;
                    d[mm] = sqrt(g);
                    ++mm;
                } else {
                    if (mask[j]) missing = 1;
                    mask[j] = 0;
                }
            }
            m_s = mm;
            fail_s = (mode == CQ_REQUIRE_ALL && missing) ? 1 : 0;
            fail_at = -1;
        }
        __syncthreads();
        m = m_s;
        Ri = R + (int64_t)m * m;
        if (fail_s) break;
        for (int e = tid; e < m * m; e += CQ_TH) {
            const int a = e / m, b = e % m;
            R[e] = G[(int64_t)idx[a] * c + idx[b]] / (d[a] * d[b]);
        }
        __syncthreads();
        const int fa = chol_blocked<CQ_TH>(m, R, tol, L);
        if (tid == 0) {
            fail_s = fa >= 0;
            fail_at = fa;
        }
        __syncthreads();
        if (!fail_s || mode != CQ_DROP_DEPENDENT) break;
        // the failing column is (numerically) in the span of the earlier ones
        if (tid == 0) {
            mask[idx[fail_at]] = 0;
            if (counter) atomicAdd(counter, 1);
        }
        __syncthreads();
    }
    if (fail_s) {
        for (int e = tid; e < c * c; e += CQ_TH) {
            T64[e] = 0.0;
            T32[e] = 0.0f;
        }
        if (tid == 0) {
            if (mode == CQ_DROP_ALL) {
                for (int j = 0; j < c; ++j) mask[j] = 0;
                atomicOr(status, DEV_P_DROPPED);
                if (counter) atomicAdd(counter, 1);
            } else {
                atomicOr(status, DEV_BREAKDOWN);
            }
        }
        return;
    }
    // R^-1, one wave per column (columns in LDS, reusing the panel buffer)
    tri_inv_upper<CQ_TH>(m, R, Ri, &L.panel[0][0]);
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

// The same factor with the equilibrated Gram matrix resident in LDS (packed
// upper triangle, element (a, b) at P[ro[a] + b]), for up to CQL_MAXM columns,
// same modes, pivot test and outputs as k_cholqr_factor:
//   - the active columns are flagged in parallel and listed by one thread
//     from LDS;
//   - blocked right-looking Cholesky with panels of CQL_NB rows: wave 0
//     factors the diagonal block, one thread per column solves the panel
//     rows (kept also in Xp), and the trailing triangle takes the rank-CQL_NB
//     update, four rows per wave and lane-consecutive columns; three
//     barriers per panel;
//   - R^-1 one wave per column j by a column sweep of R x = e_j: for
//     a = j .. 0, x_a = b_a / R(a, a) (b_a broadcast from its lane, the
//     reciprocal precomputed), then b_l -= R(l, a) x_a on the lanes' rows l < a.
constexpr int CQL_MAXM = 176;
constexpr int CQL_NB = 16;
constexpr int CQL_SLOTS = (CQL_MAXM + 63) / 64;
__device__ inline int cql_off(int a, int m) { return a * m - (a * (a - 1)) / 2; }

__device__ inline double cql_readlane(double v, int lane) {
    const uint64_t u = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__global__ void __launch_bounds__(CQ_TH)
k_cholqr_factor_lds(int c, const double* __restrict__ G, int* __restrict__ mask, double tol,
                    double* __restrict__ T64, float* __restrict__ T32, int mode, int* status,
                    int* counter) {
    __shared__ double P[CQL_MAXM * (CQL_MAXM + 1) / 2];
    __shared__ double Xp[CQL_NB][CQL_MAXM];
    __shared__ double d[CQL_MAXM], diag0[CQL_MAXM], gd[CQL_MAXM];
    __shared__ int idx[CQL_MAXM], ok[CQL_MAXM], ro[CQL_MAXM];
    __shared__ int m_s, fail_s, fail_at;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    constexpr int NW = CQ_TH / 64;
    int m = 0;
    for (int pass = 0; pass <= c; ++pass) {
        for (int j = tid; j < c; j += CQ_TH) {
            const double g = G[(int64_t)j * c + j];
            ok[j] = mask[j] ? ((isfinite(g) && g > 0.0) ? 1 : 2) : 0;
            gd[j] = g;
        }
        __syncthreads();
        if (tid == 0) {
            int mm = 0, missing = 0;
            for (int j = 0; j < c; ++j) {
                if (ok[j] == 1) {
                    idx[mm] = j;
                    d[mm] = sqrt(gd[j]);
                    ++mm;
                } else if (ok[j] == 2) {
                    missing = 1;
                    mask[j] = 0;
                }
            }
            m_s = mm;
            fail_s = (mode == CQ_REQUIRE_ALL && missing) ? 1 : 0;
            fail_at = -1;
        }
        __syncthreads();
        m = m_s;
        if (fail_s) break;
        for (int a = tid; a < m; a += CQ_TH) ro[a] = cql_off(a, m) - a;
        for (int a = wave; a < m; a += NW) {
            const int o = cql_off(a, m) - a;
            for (int b = a + lane; b < m; b += 64) {
                const double v = G[(int64_t)idx[a] * c + idx[b]] / (d[a] * d[b]);
                P[o + b] = v;
                if (b == a) diag0[a] = v;
            }
        }
        __syncthreads();
        for (int p0 = 0; p0 < m; p0 += CQL_NB) {
            const int nb = min(CQL_NB, m - p0);
            const int q0 = p0 + nb;
            const int len = m - q0;
            // 1. diagonal block, by wave 0
            if (wave == 0) {
                for (int jj = 0; jj < nb; ++jj) {
                    const int j = p0 + jj;
                    const int oj = ro[j];
                    const double sj = P[oj + j];
                    if (!isfinite(sj) || !(sj > tol * diag0[j]) || !(sj > 0.0)) {
                        if (lane == 0) fail_at = j;
                        break;
                    }
                    const double rjj = sqrt(sj);
                    if (j + 1 + lane < q0) P[oj + j + 1 + lane] /= rjj;
                    __builtin_amdgcn_wave_barrier();
                    if (lane == 0) P[oj + j] = rjj;
                    const int L = q0 - j - 1;
                    for (int e = lane; e < L * L; e += 64) {
                        const int a = j + 1 + e / L, b = j + 1 + e % L;
                        if (b >= a) P[ro[a] + b] -= P[oj + a] * P[oj + b];
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
            __syncthreads();
            if (fail_at >= 0) break;
            // 2. panel rows right of the block: R_pp' X = A_p,rest, one thread per column
            for (int cc = q0 + tid; cc < m; cc += CQ_TH) {
                double x[CQL_NB];
#pragma unroll
                for (int i = 0; i < CQL_NB; ++i) {
                    if (i < nb) {
                        const int ri = ro[p0 + i];
                        double sv = P[ri + cc];
                        for (int l = 0; l < i; ++l) sv -= P[ro[p0 + l] + p0 + i] * x[l];
                        x[i] = sv / P[ri + p0 + i];
                        P[ri + cc] = x[i];
                        Xp[i][cc] = x[i];
                    }
                }
            }
            __syncthreads();
            // 3. trailing upper triangle: a wave takes rows a0..a0+3, a lane the
            //    columns a0 + lane + 64 c, so that a wave's reads of Xp are one
            //    broadcast (the rows) and consecutive words (the columns), and
            //    its updates of P consecutive words; clamped reads, masked writes
            for (int ta = wave; 4 * ta < len; ta += NW) {
                const int a0 = q0 + 4 * ta;
                int bc[CQL_SLOTS];
                bool okc[CQL_SLOTS];
#pragma unroll
                for (int c = 0; c < CQL_SLOTS; ++c) {
                    const int b = a0 + lane + 64 * c;
                    okc[c] = b < m;
                    bc[c] = okc[c] ? b : m - 1;
                }
                double acc[4][CQL_SLOTS] = {};
                for (int i = 0; i < nb; ++i) {
                    double xa[4], xb[CQL_SLOTS];
#pragma unroll
                    for (int r = 0; r < 4; ++r) xa[r] = Xp[i][min(a0 + r, m - 1)];
#pragma unroll
                    for (int c = 0; c < CQL_SLOTS; ++c) xb[c] = Xp[i][bc[c]];
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int c = 0; c < CQL_SLOTS; ++c) acc[r][c] = fma(xa[r], xb[c], acc[r][c]);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int aa = a0 + r;
                    if (aa >= m) break;
                    const int o = ro[aa];
#pragma unroll
                    for (int c = 0; c < CQL_SLOTS; ++c)
                        if (okc[c] && bc[c] >= aa) P[o + bc[c]] -= acc[r][c];
                }
            }
            __syncthreads();
        }
        if (tid == 0) fail_s = fail_at >= 0;
        __syncthreads();
        if (!fail_s || mode != CQ_DROP_DEPENDENT) break;
        // the failing column is (numerically) in the span of the earlier ones
        if (tid == 0) {
            mask[idx[fail_at]] = 0;
            if (counter) atomicAdd(counter, 1);
        }
        __syncthreads();
    }
    for (int e = tid; e < c * c; e += CQ_TH) {
        T64[e] = 0.0;
        T32[e] = 0.0f;
    }
    if (fail_s) {
        if (tid == 0) {
            if (mode == CQ_DROP_ALL) {
                for (int j = 0; j < c; ++j) mask[j] = 0;
                atomicOr(status, DEV_P_DROPPED);
                if (counter) atomicAdd(counter, 1);
            } else {
                atomicOr(status, DEV_BREAKDOWN);
            }
        }
        return;
    }
    for (int a = tid; a < m; a += CQ_TH) gd[a] = 1.0 / P[ro[a] + a];     // reciprocals of R(a, a)
    __syncthreads();
    // R^-1 by column sweeps; lane l holds rows l, l + 64, ...
    int rol[CQL_SLOTS];
#pragma unroll
    for (int t = 0; t < CQL_SLOTS; ++t) {
        const int l = lane + 64 * t;
        rol[t] = l < m ? ro[l] : 0;
    }
    for (int j = wave; j < m; j += NW) {
        double x[CQL_SLOTS];
#pragma unroll
        for (int t = 0; t < CQL_SLOTS; ++t) x[t] = (lane + 64 * t == j) ? 1.0 : 0.0;
        for (int a = j; a >= 0; --a) {
            const int ta = a >> 6, la = a & 63;
            double xa_src = x[0];
#pragma unroll
            for (int t = 1; t < CQL_SLOTS; ++t)
                if (t == ta) xa_src = x[t];
            const double xa = cql_readlane(xa_src, la) * gd[a];
#pragma unroll
            for (int t = 0; t < CQL_SLOTS; ++t) {
                const int l = lane + 64 * t;
                if (l == a) x[t] = xa;
                else if (l < a) x[t] -= P[rol[t] + a] * xa;
            }
        }
#pragma unroll
        for (int t = 0; t < CQL_SLOTS; ++t) {
            const int l = lane + 64 * t;
            if (l <= j) {
                const double v = x[t] / d[l];
                T64[(int64_t)idx[l] * c + idx[j]] = v;
                T32[(int64_t)idx[l] * c + idx[j]] = (float)v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Row-block products with a small matrix, in place.  For every row of V:
//   acc1[j] = sum_{l in [a0,a1)} V[row][l] M[l][j]
//   acc2[j] = sum_{l in [b0,b1)} V[row][l] M[l][j]       (empty range: 0)
//   V[row][o1 + j] = acc1 + acc2,   V[row][o2 + j] = acc2 (when o2 >= 0)
// for j < nout.  A workgroup owns BM whole rows, so every read of a row
// precedes every write to it.  K is staged through LDS in chunks of 32; each
// thread keeps RPT rows x NC columns of accumulators (columns tx + 16 c).
// This serves the block update (P <- [W P] C_WP, X <- X C_X + P) and the
// right multiplication by the Cholesky-QR factor (V <- V T).
// ---------------------------------------------------------------------------
template <class T>
struct Prec;
template <>
struct Prec<double> {
    static __host__ __device__ inline const double* pick(const double* c64, const float*) { return c64; }
};
template <>
struct Prec<float> {
    static __host__ __device__ inline const float* pick(const double*, const float* c32) { return c32; }
};

constexpr int RG_BK = 32;

template <class T, int RPT, int NC>
__device__ inline void rowgemm_section(const T* __restrict__ V, int64_t ld, int64_t r0, int64_t n,
                                       int lo, int hi, const T* __restrict__ M, int ldm, int nout,
                                       T (*Vs)[16 * RPT + 1], T (*Ms)[16 * NC], T (&acc)[RPT][NC]) {
    constexpr int BM = 16 * RPT;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    for (int l0 = lo; l0 < hi; l0 += RG_BK) {
        const int kc = min(RG_BK, hi - l0);
        __syncthreads();
        for (int e = threadIdx.x; e < BM * RG_BK; e += 256) {
            const int row = e / RG_BK, kk = e % RG_BK;
            Vs[kk][row] = (r0 + row < n && kk < kc) ? V[(r0 + row) * ld + l0 + kk] : T(0);
        }
        for (int e = threadIdx.x; e < RG_BK * 16 * NC; e += 256) {
            const int kk = e / (16 * NC), j = e % (16 * NC);
            Ms[kk][j] = (kk < kc && j < nout) ? M[(int64_t)(l0 + kk) * ldm + j] : T(0);
        }
        __syncthreads();
        for (int kk = 0; kk < kc; ++kk) {
            T v[RPT], m[NC];
#pragma unroll
            for (int r = 0; r < RPT; ++r) v[r] = Vs[kk][ty * RPT + r];
#pragma unroll
            for (int c = 0; c < NC; ++c) m[c] = Ms[kk][tx + 16 * c];
#pragma unroll
            for (int r = 0; r < RPT; ++r)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[r][c] = fma(v[r], m[c], acc[r][c]);
        }
    }
}

template <class T, int RPT, int NC>
__global__ void __launch_bounds__(256)
k_rowgemm(int64_t n, T* __restrict__ V, int64_t ld, int a0, int a1, int b0, int b1, int b2,
          int b3, const T* __restrict__ M, int ldm, int nout, int o1, int o2) {
    constexpr int BM = 16 * RPT;
    __shared__ T Vs[RG_BK][BM + 1];
    __shared__ T Ms[RG_BK][16 * NC];
    const int64_t r0 = (int64_t)blockIdx.x * BM;
    T acc1[RPT][NC], acc2[RPT][NC];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            acc1[r][c] = T(0);
            acc2[r][c] = T(0);
        }
    rowgemm_section<T, RPT, NC>(V, ld, r0, n, a0, a1, M, ldm, nout, Vs, Ms, acc1);
    rowgemm_section<T, RPT, NC>(V, ld, r0, n, b0, b1, M, ldm, nout, Vs, Ms, acc2);
    rowgemm_section<T, RPT, NC>(V, ld, r0, n, b2, b3, M, ldm, nout, Vs, Ms, acc2);
    __syncthreads();
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int64_t row = r0 + ty * RPT + r;
        if (row >= n) continue;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int j = tx + 16 * c;
            if (j >= nout) continue;
            V[row * ld + o1 + j] = acc1[r][c] + acc2[r][c];
            if (o2 >= 0) V[row * ld + o2 + j] = acc2[r][c];
        }
    }
}

// ---------------------------------------------------------------------------
// Residual R = LX - X diag(theta) written into the W block, with per-block
// FP64 partial sums of R^2 and X^2 per column.
// ---------------------------------------------------------------------------
constexpr int RES_ROWS = 256;

template <class T>
__global__ void __launch_bounds__(256)
k_residual(int64_t n, int kp, int k, int woff, T* __restrict__ S, const T* __restrict__ LS,
           int64_t ld, const double* __restrict__ theta, double* __restrict__ partial) {
    const int64_t r0 = (int64_t)blockIdx.x * RES_ROWS;
    const int64_t r1 = min<int64_t>(n, r0 + RES_ROWS);
    for (int j = threadIdx.x; j < kp; j += 256) {
        double rr = 0.0, xx = 0.0;
        if (j < k) {
            const T th = (T)theta[j];
            for (int64_t i = r0; i < r1; ++i) {
                const T x = S[i * ld + j];
                const T r = fma(-th, x, LS[i * ld + j]);
                S[i * ld + woff + j] = r;
                rr = fma((double)r, (double)r, rr);
                xx = fma((double)x, (double)x, xx);
            }
        } else {
            for (int64_t i = r0; i < r1; ++i) S[i * ld + woff + j] = T(0);
        }
        partial[((int64_t)blockIdx.x * 2 + 0) * kp + j] = rr;
        partial[((int64_t)blockIdx.x * 2 + 1) * kp + j] = xx;
    }
}

// The same residual with 16-byte accesses: a thread takes V = 16 / sizeof(T)
// adjacent columns of every RS-th row of the block (G = kp / V column groups,
// RS = 256 / G row lanes); each column's FP64 sums are then added over the
// row lanes in lane order.  For kp a multiple of V with kp / V <= 256, and
// strides, the W offset and both pointers multiples of 16 bytes.
template <class T>
__global__ void __launch_bounds__(256)
k_residual_vec(int64_t n, int kp, int k, int woff, T* __restrict__ S, const T* __restrict__ LS,
               int64_t ld, const double* __restrict__ theta, double* __restrict__ partial) {
    constexpr int V = 16 / (int)sizeof(T);
    using VT = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    __shared__ double red[2][256 * V];
    const int G = kp / V, RS = 256 / G;
    const int g = (int)threadIdx.x % G, sl = (int)threadIdx.x / G;
    const int64_t r0 = (int64_t)blockIdx.x * RES_ROWS;
    const int64_t r1 = min<int64_t>(n, r0 + RES_ROWS);
    double rr[V], xx[V];
    T th[V];
    bool on[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int j = g * V + v;
        on[v] = j < k;
        th[v] = on[v] ? (T)theta[j] : T(0);
        rr[v] = 0.0;
        xx[v] = 0.0;
    }
    if (sl < RS) {
#pragma unroll 4
        for (int64_t i = r0 + sl; i < r1; i += RS) {
            const VT xv = *reinterpret_cast<const VT*>(S + i * ld + g * V);
            const VT lv = *reinterpret_cast<const VT*>(LS + i * ld + g * V);
            const T* x = reinterpret_cast<const T*>(&xv);
            const T* l = reinterpret_cast<const T*>(&lv);
            VT rv;
            T* r = reinterpret_cast<T*>(&rv);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                r[v] = on[v] ? fma(-th[v], x[v], l[v]) : T(0);
                rr[v] = fma((double)r[v], (double)r[v], rr[v]);
                if (on[v]) xx[v] = fma((double)x[v], (double)x[v], xx[v]);
            }
            *reinterpret_cast<VT*>(S + i * ld + woff + g * V) = rv;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            red[0][sl * kp + g * V + v] = rr[v];
            red[1][sl * kp + g * V + v] = xx[v];
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kp; j += 256) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < RS; ++q) {
            a += red[0][q * kp + j];
            b += red[1][q * kp + j];
        }
        partial[((int64_t)blockIdx.x * 2 + 0) * kp + j] = a;
        partial[((int64_t)blockIdx.x * 2 + 1) * kp + j] = b;
    }
}

// per-column totals of the block partials, in place into block 0's slots:
// workgroup (j, t) sums partial[b][t][j] over the blocks b (fixed tree order)
__global__ void __launch_bounds__(256)
k_residual_colsum(int nblocks, int kp, double* __restrict__ partial) {
    __shared__ double red[256];
    const int j = blockIdx.x, t = blockIdx.y;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += partial[((int64_t)b * 2 + t) * kp + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)t * kp + j] = red[0];
}

__global__ void __launch_bounds__(256)
k_residual_finalize(int nblocks, int kp, int k, int k_conv, const double* __restrict__ partial,
                    double op_norm,
                    double lock_tol,
                    double* __restrict__ relres, double* __restrict__ hist_row, int* __restrict__ wmask,
                    int* status, double* out_max, int* out_all_locked,
                    const double* __restrict__ theta, int* __restrict__ out_restart,
                    int* __restrict__ out_wcount) {
    __shared__ double mx[256];
    __shared__ int locked_all[256];
    __shared__ int bad[256];
    __shared__ int nact[256];
    double my_max = 0.0;
    int my_all = 1;
    int my_bad = 0;
    int my_act = 0;
    for (int j = threadIdx.x; j < kp; j += 256) {
        double rr = 0.0, xx = 0.0;
        for (int b = 0; b < nblocks; ++b) {
            rr += partial[((int64_t)b * 2 + 0) * kp + j];
            xx += partial[((int64_t)b * 2 + 1) * kp + j];
        }
        if (j < k) {
            const double rel = sqrt(rr) / (op_norm * sqrt(xx));
            if (!isfinite(rel)) atomicOr(status, DEV_NUMERIC);
            relres[j] = rel;
            if (hist_row) hist_row[j] = rel;
            const int active = rel > lock_tol;
            wmask[j] = active;
            // a consistent iterate has theta in [0, op_norm] (spectrum of L)
            // and ||Lx - theta x|| <= op_norm ||x||, i.e. relres <= 1
            if (out_restart) {
                const double th = theta[j];
                const double slack = RESTART_THETA_SLACK * 0.5 * op_norm;
                if (!(th >= -slack && th <= op_norm + slack) || rel > 1.0) my_bad = 1;
            }
            my_all &= !active;
            my_act += active;
            if (j < k_conv) my_max = fmax(my_max, rel);
        } else {
            relres[j] = 0.0;
            wmask[j] = 0;
        }
    }
    mx[threadIdx.x] = my_max;
    locked_all[threadIdx.x] = my_all;
    bad[threadIdx.x] = my_bad;
    nact[threadIdx.x] = my_act;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        int a = 1, b = 0, w = 0;
        for (int t = 0; t < 256; ++t) {
            m = fmax(m, mx[t]);
            a &= locked_all[t];
            b |= bad[t];
            w += nact[t];
        }
        *out_max = m;
        *out_all_locked = a;
        if (out_restart) *out_restart = b;
        if (out_wcount) *out_wcount = w;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
GramPlan gram_plan(int64_t n, int c, int gmode_bytes) {
    GramPlan p;
    p.n = n;
    p.c = c;
    // workgroup tile edge: 160 (FP32 / BF16 matrix-core path: 2 x 2 waves of
    // 5 x 5 MFMA tiles, so k = 160 and 3k = 480 need no padding), 64 (FP64
    // accumulation: FP64 data, or FP32 data widened)
    p.bt = gmode_bytes == 8 ? 64 : 160;
    p.tiles = (int)ceil_div(c, p.bt);
    const int upper = p.tiles * (p.tiles + 1) / 2;
    // enough workgroups to fill 256 CUs several times, each chunk >= 512 rows
    int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(2048, upper), ceil_div(n, 512)));
    p.chunks = std::min(chunks, 256);
    // chunk boundaries on multiples of 32 rows (the BF16 MFMA step)
    p.chunk_rows = ceil_div(ceil_div(n, p.chunks), 32) * 32;
    p.chunks = (int)ceil_div(n, p.chunk_rows);
    return p;
}

size_t gram_partial_elems(const GramPlan& p, int nout) {
    return (size_t)p.chunks * nout * (size_t)p.c * p.c;
}

static bool aligned16(const void* ptr, int64_t ld, size_t es) {
    return ptr == nullptr || (((uintptr_t)ptr % 16) == 0 && ((size_t)ld * es) % 16 == 0);
}

// workgroups of a persistent FP32 Gram launch: as many as are resident at once
// (occupancy of the instantiation x compute units), at most one per item
template <class MF, bool TWO>
static unsigned gram_grid(sc_ctx* ctx, unsigned items) {
    static int per_cu = -1;                  // one value per kernel instantiation
    if (per_cu < 0) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &b, reinterpret_cast<const void*>(k_gram_lds<MF, TWO, true, false>), 256, 0) !=
                hipSuccess ||
            b < 1)
            b = 1;
        per_cu = b;
    }
    return std::min<unsigned>(items, (unsigned)(per_cu * ctx->num_cu));
}

template <class MF>
static void gram_go(sc_ctx* ctx, const GramPlan& p, const typename MF::in_t* A, int64_t lda,
                    const typename MF::in_t* B1, int64_t ldb1, const typename MF::in_t* B2,
                    int64_t ldb2, double* partial, const int* pred) {
    const int upper = p.tiles * (p.tiles + 1) / 2;
    dim3 grid(upper, p.chunks);
    if constexpr (sizeof(typename MF::in_t) == 4) {
        constexpr size_t es = sizeof(float);
        if (p.queue && aligned16(A, lda, es) && aligned16(B1, ldb1, es) && aligned16(B2, ldb2, es)) {
            const unsigned items = (unsigned)(upper * p.chunks);
            constexpr bool PS = !std::is_same<MF, MfBF16>::value;
            unsigned g2 = items, g1 = items;
            if constexpr (PS) {
                g2 = gram_grid<MF, true>(ctx, items);
                g1 = gram_grid<MF, false>(ctx, items);
            }
            // (the BF16 instantiation with skipping would spill: it computes the
            // zero sub-tiles instead)
            const bool part = PS && (p.c % p.bt != 0 || p.gap_hi > p.gap_lo);
            if (B2) {
                if (part)
                    hipLaunchKernelGGL((k_gram_lds<MF, true, PS, PS>), dim3(g2), dim3(256), 0,
                                       ctx->stream, p.n, p.c, p.chunk_rows, A, lda, B1, ldb1, B2,
                                       ldb2, partial, p.tiles, p.chunks, p.queue, p.gap_lo,
                                       p.gap_hi, pred);
                else
                    hipLaunchKernelGGL((k_gram_lds<MF, true, PS, false>), dim3(g2), dim3(256), 0,
                                       ctx->stream, p.n, p.c, p.chunk_rows, A, lda, B1, ldb1, B2,
                                       ldb2, partial, p.tiles, p.chunks, p.queue, p.gap_lo,
                                       p.gap_hi, pred);
            } else {
                if (part)
                    hipLaunchKernelGGL((k_gram_lds<MF, false, PS, PS>), dim3(g1), dim3(256), 0,
                                       ctx->stream, p.n, p.c, p.chunk_rows, A, lda, B1, ldb1, B1,
                                       ldb1, partial, p.tiles, p.chunks, p.queue, p.gap_lo,
                                       p.gap_hi, pred);
                else
                    hipLaunchKernelGGL((k_gram_lds<MF, false, PS, false>), dim3(g1), dim3(256), 0,
                                       ctx->stream, p.n, p.c, p.chunk_rows, A, lda, B1, ldb1, B1,
                                       ldb1, partial, p.tiles, p.chunks, p.queue, p.gap_lo,
                                       p.gap_hi, pred);
            }
            return;
        }
    }
    if (B2)
        hipLaunchKernelGGL((k_gram_mfma<MF, true>), grid, dim3(256), 0, ctx->stream, p.n, p.c,
                           p.chunk_rows, A, lda, B1, ldb1, B2, ldb2, partial, p.tiles, pred);
    else
        hipLaunchKernelGGL((k_gram_mfma<MF, false>), grid, dim3(256), 0, ctx->stream, p.n, p.c,
                           p.chunk_rows, A, lda, B1, ldb1, B1, ldb1, partial, p.tiles, pred);
}

template <class T>
sc_status launch_gram(sc_ctx* ctx, const GramPlan& p, const T* A, int64_t lda, const T* B1,
                      int64_t ldb1, const T* B2, int64_t ldb2, double* partial, double* G1,
                      double* G2, int gmode, const int* pred) {
    if constexpr (sizeof(T) == 8) {
        gram_go<MfF64>(ctx, p, A, lda, B1, ldb1, B2, ldb2, partial, pred);
    } else {
        const int bt = gmode == GRAM_F32_EXACT ? 64 : 160;
        if (p.bt != bt) return sc_fail(ctx, SC_E_INVAL, "gram: plan tile %d, kernel tile %d", p.bt, bt);
        if (gmode == GRAM_BF16)
            gram_go<MfBF16>(ctx, p, A, lda, B1, ldb1, B2, ldb2, partial, pred);
        else if (gmode == GRAM_F32_EXACT)
            gram_go<MfF32x64>(ctx, p, A, lda, B1, ldb1, B2, ldb2, partial, pred);
        else
            gram_go<MfF32>(ctx, p, A, lda, B1, ldb1, B2, ldb2, partial, pred);
    }
    SC_CHECK_LAUNCH(ctx);
    const int64_t cc2 = (int64_t)p.c * p.c;
    hipLaunchKernelGGL(k_gram_reduce, dim3(ceil_div(cc2, 256)), dim3(256), 0, ctx->stream, p.c,
                       p.chunks, B2 ? 2 : 1, partial, G1, G2, pred);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}

template sc_status launch_gram<double>(sc_ctx*, const GramPlan&, const double*, int64_t,
                                       const double*, int64_t, const double*, int64_t, double*,
                                       double*, double*, int, const int*);
template sc_status launch_gram<float>(sc_ctx*, const GramPlan&, const float*, int64_t,
                                      const float*, int64_t, const float*, int64_t, double*,
                                      double*, double*, int, const int*);

sc_status launch_cholqr_factor(sc_ctx* ctx, int c, const double* G, int* mask, double tol,
                               double* T64, float* T32, double* scratch, int mode,
                               int* status, int* counter) {
    if (c > CQ_MAX) return sc_fail(ctx, SC_E_UNSUPPORTED, "cholqr: %d columns > %d", c, CQ_MAX);
    if (c <= CQL_MAXM)
        hipLaunchKernelGGL(k_cholqr_factor_lds, dim3(1), dim3(CQ_TH), 0, ctx->stream, c, G, mask, tol,
                           T64, T32, mode, status, counter);
    else
        hipLaunchKernelGGL(k_cholqr_factor, dim3(1), dim3(CQ_TH), 0, ctx->stream, c, G, mask, tol,
                           T64, T32, scratch, mode, status, counter);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}

// FP32 row-block products on the matrix cores: the same contract as
// k_rowgemm (sections [a0,a1) and [b0,b1) of each row times rows of M, in
// place), as a tall GEMM with v_mfma_f32_16x16x4_f32.  A workgroup owns
// RG_BM rows; each of its four waves 16 * RG_WR rows and all NC 16-column
// output tiles.  K is staged through LDS in chunks of RG_KC: the V chunk with
// 16-byte loads (row stride RG_KC + 2 floats, so the 16-row fragment reads
// fall in distinct banks) and the matching rows of M.  Section b is reduced
// first: its sum alone goes to the o2 columns (which must not overlap
// [a0, a1)); section a is then added and the total goes to the o1 columns.
constexpr int RG_WR = 2;
constexpr int RG_BM = 4 * 16 * RG_WR;
// K chunk width and waves per SIMD: the 160-column block update (NC = 10)
// takes 16-wide chunks, which fit it in 144 registers and so three
// workgroups per CU (2.7 % faster than two at 32-wide chunks); the
// triangular apply keeps 32-wide chunks (16 costs it 5 %), and the other
// widths already fit three workgroups or cannot.
template <int NC, bool TRI>
constexpr int rg_kc() { return (NC == 10 && !TRI) ? 16 : 32; }
template <int NC, bool TRI>
constexpr int rg_waves() { return (NC == 10 && !TRI) ? 3 : 1; }

template <int NC, bool TRI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(rg_waves<NC, TRI>())))
k_rowgemm_mfma(int64_t n, float* __restrict__ V, int64_t ld, int a0, int a1, int b0, int b1,
               int b2, int b3, const float* __restrict__ M, int ldm, int nout, int o1, int o2) {
    constexpr int RG_KC = rg_kc<NC, TRI>();
    constexpr int VS = RG_KC + 2;
    constexpr int MS = 16 * NC + ((NC % 2 == 0) ? 16 : 0);
    __shared__ __attribute__((aligned(16))) float Vs[RG_BM * VS];
    __shared__ __attribute__((aligned(16))) float Ms[RG_KC * MS];
    const int64_t row0 = (int64_t)blockIdx.x * RG_BM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr0 = wave * 16 * RG_WR;
    const int l16 = lane & 15, lk = lane >> 4;
    mf_f4 acc[RG_WR][NC];
#pragma unroll
    for (int w = 0; w < RG_WR; ++w)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[w][j] = mf_f4{0.f, 0.f, 0.f, 0.f};
    // staging registers: the next chunk's V tile (float4) and M rows, loaded
    // while the current chunk is on the matrix cores
    constexpr int PV = RG_BM * (RG_KC / 4) / 256;
    constexpr int PM = (RG_KC * 4 * NC + 255) / 256;     // float4 of M per thread
    float4 rv[PV];
    float4 rm[PM];
    auto load = [&](int kc, int kn) {
        // whole tiles take plain loads, with no per-element tests
        const bool whole = kn == RG_KC && row0 + RG_BM <= n && nout == 16 * NC;
#pragma unroll
        for (int u = 0; u < PV; ++u) {
            const int q = tid + 256 * u;
            const int r = q / (RG_KC / 4), c4 = 4 * (q % (RG_KC / 4));
            const int64_t row = row0 + r;
            const float* src = V + row * ld + kc + c4;
            float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
            if (whole) {
                x = *reinterpret_cast<const float4*>(src);
            } else if (row < n) {
                if (c4 + 3 < kn) {
                    x = *reinterpret_cast<const float4*>(src);
                } else {
                    if (c4 < kn) x.x = src[0];
                    if (c4 + 1 < kn) x.y = src[1];
                    if (c4 + 2 < kn) x.z = src[2];
                }
            }
            rv[u] = x;
        }
        // rows of M by 16-byte loads when they are whole and aligned
        const bool m4 = whole && ldm % 4 == 0 && ((uintptr_t)M % 16) == 0;
#pragma unroll
        for (int u = 0; u < PM; ++u) {
            const int q = tid + 256 * u;
            const int k = q / (4 * NC), j = 4 * (q % (4 * NC));
            const float* src = M + (int64_t)(kc + k) * ldm + j;
            float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
            if (q < RG_KC * 4 * NC) {
                if (m4) {
                    x = *reinterpret_cast<const float4*>(src);
                } else if (k < kn) {
                    if (j < nout) x.x = src[0];
                    if (j + 1 < nout) x.y = src[1];
                    if (j + 2 < nout) x.z = src[2];
                    if (j + 3 < nout) x.w = src[3];
                }
            }
            rm[u] = x;
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int u = 0; u < PV; ++u) {
            const int q = tid + 256 * u;
            const int r = q / (RG_KC / 4), c4 = 4 * (q % (RG_KC / 4));
            float* dst = Vs + r * VS + c4;
            *reinterpret_cast<float2*>(dst) = make_float2(rv[u].x, rv[u].y);
            *reinterpret_cast<float2*>(dst + 2) = make_float2(rv[u].z, rv[u].w);
        }
#pragma unroll
        for (int u = 0; u < PM; ++u) {
            const int q = tid + 256 * u;
            if (q < RG_KC * 4 * NC)
                *reinterpret_cast<float4*>(Ms + (q / (4 * NC)) * MS + 4 * (q % (4 * NC))) = rm[u];
        }
    };
    auto section = [&](int lo, int hi) {
        if (lo < hi) load(lo, min(RG_KC, hi - lo));
        for (int kc = lo; kc < hi; kc += RG_KC) {
            __syncthreads();
            stage();
            __syncthreads();
            if (kc + RG_KC < hi) load(kc + RG_KC, min(RG_KC, hi - kc - RG_KC));
#pragma unroll 2
            for (int kk = 0; kk < RG_KC; kk += 4) {
                float af[RG_WR], bf[NC];
#pragma unroll
                for (int w = 0; w < RG_WR; ++w) af[w] = Vs[(wr0 + 16 * w + l16) * VS + kk + lk];
#pragma unroll
                for (int j = 0; j < NC; ++j) bf[j] = Ms[(kk + lk) * MS + 16 * j + l16];
#pragma unroll
                for (int w = 0; w < RG_WR; ++w)
#pragma unroll
                    for (int j = 0; j < NC; ++j)
                        acc[w][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[w], bf[j], acc[w][j], 0, 0, 0);
            }
        }
    };
    // M upper triangular (M[k][j] = 0 for k > j, the Cholesky-QR factor): the
    // MFMA over rows k .. k + 3 of M reaches only the output tiles j with
    // 16 j + 15 >= k, so tiles left of (k / 16) are skipped.  Chunks and k
    // steps are unrolled, which makes each step's first tile a constant.
    // Skipped products are exact zeros, so the sums are unchanged.
    auto section_tri = [&](int hi) {
        if (hi > 0) load(0, min(RG_KC, hi));
#pragma unroll
        for (int i = 0; i < (16 * NC + RG_KC - 1) / RG_KC; ++i) {
            const int kc = i * RG_KC;
            if (kc >= hi) break;
            __syncthreads();
            stage();
            __syncthreads();
            if (kc + RG_KC < hi) load(kc + RG_KC, min(RG_KC, hi - kc - RG_KC));
#pragma unroll
            for (int kk = 0; kk < RG_KC; kk += 4) {
                const int j0 = (kc + kk) / 16;
                float af[RG_WR], bf[NC];
#pragma unroll
                for (int w = 0; w < RG_WR; ++w) af[w] = Vs[(wr0 + 16 * w + l16) * VS + kk + lk];
#pragma unroll
                for (int j = 0; j < NC; ++j)
                    if (j >= j0) bf[j] = Ms[(kk + lk) * MS + 16 * j + l16];
#pragma unroll
                for (int w = 0; w < RG_WR; ++w)
#pragma unroll
                    for (int j = 0; j < NC; ++j)
                        if (j >= j0)
                            acc[w][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[w], bf[j], acc[w][j], 0, 0, 0);
            }
        }
    };
    auto store = [&](int o) {
#pragma unroll
        for (int w = 0; w < RG_WR; ++w)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = row0 + wr0 + 16 * w + 4 * lk + v;
                if (row >= n) continue;
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    const int col = 16 * j + l16;
                    if (col < nout) V[row * ld + o + col] = acc[w][j][v];
                }
            }
    };
    if (TRI) {                                   // a0 = 0, no second section
        section_tri(a1);
        store(o1);
        return;
    }
    if (b1 > b0 || b3 > b2) {
        if (b1 > b0) section(b0, b1);
        if (b3 > b2) section(b2, b3);
        if (o2 >= 0) store(o2);
    }
    section(a0, a1);
    store(o1);
}

template <int NC>
static void rowgemm_mfma_go(sc_ctx* ctx, int64_t n, float* V, int64_t ld, int a0, int a1, int b0,
                            int b1, int b2, int b3, const float* M, int ldm, int nout, int o1,
                            int o2, bool tri) {
    if (tri)
        hipLaunchKernelGGL((k_rowgemm_mfma<NC, true>), dim3((unsigned)ceil_div(n, RG_BM)),
                           dim3(256), 0, ctx->stream, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm,
                           nout, o1, o2);
    else
        hipLaunchKernelGGL((k_rowgemm_mfma<NC, false>), dim3((unsigned)ceil_div(n, RG_BM)),
                           dim3(256), 0, ctx->stream, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm,
                           nout, o1, o2);
}

template <class T, int NC>
static void rowgemm_go(sc_ctx* ctx, int64_t n, T* V, int64_t ld, int a0, int a1, int b0, int b1,
                       int b2, int b3, const T* M, int ldm, int nout, int o1, int o2) {
    constexpr int RPT = sizeof(T) == 8 ? 2 : 4;
    constexpr int BM = 16 * RPT;
    hipLaunchKernelGGL((k_rowgemm<T, RPT, NC>), dim3((unsigned)ceil_div(n, BM)), dim3(256), 0,
                       ctx->stream, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2);
}

// Section b is [b0, b1) followed by [b2, b3) (either may be empty).
// tri: M is upper triangular with a0 = 0 and an empty section b (the
// matrix-core path then skips the all-zero products)
template <class T>
static sc_status rowgemm(sc_ctx* ctx, int64_t n, T* V, int64_t ld, int a0, int a1, int b0, int b1,
                         int b2, int b3, const T* M, int ldm, int nout, int o1, int o2,
                         bool tri = false) {
    if (tri && (a0 != 0 || b1 > b0 || b3 > b2))
        return sc_fail(ctx, SC_E_INVAL, "rowgemm: triangular factor with sections [%d,%d) [%d,%d)",
                       a0, a1, b0, b1);
    const int nc = (nout + 15) / 16;
    if constexpr (sizeof(T) == 4) {
        // matrix-core path: 16-byte aligned rows and section starts
        if (((uintptr_t)V % 16) == 0 && ld % 4 == 0 && a0 % 4 == 0 && b0 % 4 == 0 &&
            b2 % 4 == 0 && nout <= 256) {
            switch (nc <= 4 ? nc : nc <= 6 ? 6 : nc <= 8 ? 8 : nc <= 10 ? 10 : nc <= 12 ? 12 : 16) {
                case 1: rowgemm_mfma_go<1>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2, tri); break;
                case 2: rowgemm_mfma_go<2>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2, tri); break;
                case 3: rowgemm_mfma_go<3>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2, tri); break;
                case 4: rowgemm_mfma_go<4>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2, tri); break;
                case 6: rowgemm_mfma_go<6>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2, tri); break;
                case 8: rowgemm_mfma_go<8>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2, tri); break;
                case 10: rowgemm_mfma_go<10>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2, tri); break;
                case 12: rowgemm_mfma_go<12>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2, tri); break;
                default: rowgemm_mfma_go<16>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2, tri); break;
            }
            SC_CHECK_LAUNCH(ctx);
            return SC_OK;
        }
    }
    switch (nc <= 4 ? nc : nc <= 6 ? 6 : nc <= 8 ? 8 : nc <= 10 ? 10 : nc <= 12 ? 12 : 16) {
        case 1: rowgemm_go<T, 1>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2); break;
        case 2: rowgemm_go<T, 2>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2); break;
        case 3: rowgemm_go<T, 3>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2); break;
        case 4: rowgemm_go<T, 4>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2); break;
        case 6: rowgemm_go<T, 6>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2); break;
        case 8: rowgemm_go<T, 8>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2); break;
        case 10: rowgemm_go<T, 10>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2); break;
        case 12: rowgemm_go<T, 12>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2); break;
        default:
            if (nout > 256) return sc_fail(ctx, SC_E_UNSUPPORTED, "rowgemm: %d columns > 256", nout);
            rowgemm_go<T, 16>(ctx, n, V, ld, a0, a1, b0, b1, b2, b3, M, ldm, nout, o1, o2);
            break;
    }
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}

template <class T>
sc_status launch_apply_right(sc_ctx* ctx, int64_t n, int c, T* V, int64_t ldv, T* V2, int64_t ldv2,
                             const double* T64, const float* T32) {
    const T* M = Prec<T>::pick(T64, T32);
    SC_TRY(rowgemm<T>(ctx, n, V, ldv, 0, c, 0, 0, 0, 0, M, c, c, 0, -1, true));
    if (V2) SC_TRY(rowgemm<T>(ctx, n, V2, ldv2, 0, c, 0, 0, 0, 0, M, c, c, 0, -1, true));
    return SC_OK;
}
template sc_status launch_apply_right<double>(sc_ctx*, int64_t, int, double*, int64_t, double*,
                                              int64_t, const double*, const float*);
template sc_status launch_apply_right<float>(sc_ctx*, int64_t, int, float*, int64_t, float*,
                                             int64_t, const double*, const float*);

template <class T>
sc_status launch_block_update(sc_ctx* ctx, int64_t n, int kp, int kw, T* S, int64_t ld,
                              const double* C64, const float* C32) {
    const T* M = Prec<T>::pick(C64, C32);
    // [W P] C_WP: the W columns in use, then P (the unused W columns' rows of
    // C are zero)
    return rowgemm<T>(ctx, n, S, ld, 0, kp, kp, kp + kw, 2 * kp, 3 * kp, M, kp, kp, 0, 2 * kp);
}
template sc_status launch_block_update<double>(sc_ctx*, int64_t, int, int, double*, int64_t,
                                               const double*, const float*);
template sc_status launch_block_update<float>(sc_ctx*, int64_t, int, int, float*, int64_t, const double*,
                                              const float*);

template <class T>
sc_status launch_residual(sc_ctx* ctx, int64_t n, int kp, int k, int woff, T* S, const T* LS,
                          int64_t ld, const double* theta, double* partial, int* nblocks_out) {
    const int nb = (int)ceil_div(n, RES_ROWS);
    constexpr int V = 16 / (int)sizeof(T);
    const bool vec = kp % V == 0 && kp / V <= 256 && ld % V == 0 && woff % V == 0 &&
                     (uintptr_t)S % 16 == 0 && (uintptr_t)LS % 16 == 0;
    if (vec)
        hipLaunchKernelGGL((k_residual_vec<T>), dim3(nb), dim3(256), 0, ctx->stream, n, kp, k, woff, S,
                           LS, ld, theta, partial);
    else
        hipLaunchKernelGGL((k_residual<T>), dim3(nb), dim3(256), 0, ctx->stream, n, kp, k, woff, S, LS,
                           ld, theta, partial);
    SC_CHECK_LAUNCH(ctx);
    *nblocks_out = nb;
    return SC_OK;
}
template sc_status launch_residual<double>(sc_ctx*, int64_t, int, int, int, double*, const double*,
                                           int64_t, const double*, double*, int*);
template sc_status launch_residual<float>(sc_ctx*, int64_t, int, int, int, float*, const float*,
                                          int64_t, const double*, double*, int*);

sc_status launch_residual_finalize(sc_ctx* ctx, int nblocks, int kp, int k, int k_conv,
                                   double* partial, double op_norm, double lock_tol, double* relres,
                                   double* hist_row, int* wmask, int* status, double* out_max,
                                   int* out_all_locked, const double* theta, int* out_restart,
                                   int* out_wcount) {
    if (nblocks > 1) {
        hipLaunchKernelGGL(k_residual_colsum, dim3(kp, 2), dim3(256), 0, ctx->stream, nblocks, kp,
                           partial);
        nblocks = 1;
    }
    hipLaunchKernelGGL(k_residual_finalize, dim3(1), dim3(256), 0, ctx->stream, nblocks, kp, k,
                       k_conv, partial, op_norm, lock_tol, relres, hist_row, wmask, status, out_max,
                       out_all_locked, theta, out_restart, out_wcount);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}
