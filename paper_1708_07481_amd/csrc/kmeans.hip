// k-means labelling of the row-normalised eigenvectors (Section II-A: the
// clusters are read off the approximate eigenvectors; k-means++ is the
// classic labelling the paper refers to).  All restarts run together.
//
// Exactness rules, so that labels do not depend on the launch shape:
//   - a squared distance is accumulated with fma in dimension order by one
//     lane (the same chain for every point/centroid pair, wherever computed);
//   - k-means++ draws use integer weights floor(D2 * 2^s) and an exact
//     integer prefix sum;
//   - a centroid is the sum of its members in ascending vertex order (a
//     stable counting sort by label gives the member lists), divided by the count;
//   - the restart with the least integer inertia wins (ties: lowest restart).
// Lloyd iterations skip points whose assignment provably cannot change
// (Hamerly's bounds: an upper bound on the distance to the assigned centre
// and a lower bound on the distance to every other centre, both moved by the
// centre displacements).  The bounds are inflated by a relative margin far
// above the rounding error of the distance chain, so a skipped point's
// computed argmin is exactly the one a full scan would give.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "sc_internal.h"

namespace {

constexpr int TH = 256;
constexpr double BOUND_MARGIN = 1e-12;   // relative inflation of every bound
constexpr double BOUND_TINY = 1e-150;    // absolute slack for zero distances
// The Hamerly bounds are formed in FP64 and stored in FP32 rounded outward
// (upper bounds up, lower bounds down), so a stored bound is never tighter
// than the FP64 one; a bound only decides which points are scanned, and the
// labels come from exact distances.

__device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }
__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// The normalised rows y_i = x_i / ||x_i|| are read in two layouts: row-major
// (Lloyd scans, centroid sums, seeding picks) and dimension-major (the
// point-per-lane seeding and final distances).  FP64 input: both are
// materialised as FP64.  FP32 input: the row-major FP64 copy serves the
// centroid sums only; the Lloyd scans and seeding picks read the caller's X
// itself and the dimension-major copy is a transposed FP32 X (half the bytes of
// every pass), with the divisor b_i of each row (its norm, or 1.0 for a zero
// row or without normalisation) and r_i = RN(1/b_i); the kernels redo the
// quotient in registers, with the same bits as the IEEE division:
// q0 = x r is within 1.5 ulp of x/b, one fma residual correction brings it
// within 1 ulp, and a second one rounds correctly (Markstein's theorem: with r
// within half an ulp of 1/b and q within one ulp of x/b, the residual
// x - b q is exact and RN(q + (x - b q) r) = RN(x/b)).  Five FP64 operations
// instead of a division's eleven.  A -0.0 may come out as +0.0, which no
// squared difference can tell apart.
struct YDiv {
    double b, r;
};
__device__ __forceinline__ double ycoord(double v, YDiv) { return v; }
__device__ __forceinline__ double ycoord(float v, YDiv dv) {
    const double x = v;
    const double q0 = x * dv.r;
    const double q1 = fma(fma(-q0, dv.b, x), dv.r, q0);
    return fma(fma(-q1, dv.b, x), dv.r, q1);
}
template <class TT>
__device__ __forceinline__ YDiv ydiv_of(const YDiv* dv, int64_t i) {
    return sizeof(TT) == 4 ? dv[i] : YDiv{1.0, 1.0};
}

// A workgroup takes TH rows; the rows are staged through LDS in chunks of RN_DC
// dimensions (coalesced loads and stores), while each thread accumulates its
// own row's sum of squares in dimension order.  The chunks are read twice:
// once for the norm, once for the quotients.
constexpr int RN_DC = 16;
template <class TX>
__global__ void __launch_bounds__(TH)
k_rownorm(int64_t n, int dim, const TX* __restrict__ X, int64_t ldx, int normalize,
          double* __restrict__ Y, TX* __restrict__ Yt, YDiv* __restrict__ dv,
          unsigned long long* m2bits, int* status) {
    constexpr bool RAW = sizeof(TX) == 4;    // the dimension-major copy holds x, not y
    __shared__ double xs[RN_DC][TH + 1];
    const int64_t row0 = (int64_t)blockIdx.x * TH;
    const int t = threadIdx.x;
    const bool live = row0 + t < n;
    double s = 0.0;
    bool bad = false;
    for (int pass = 0; pass < 2; ++pass) {
        const double nrm = sqrt(s);
        if (RAW && pass == 1 && live) {
            const double b = (normalize && nrm > 0.0) ? nrm : 1.0;
            dv[row0 + t] = YDiv{b, 1.0 / b};
        }
        double s2 = 0.0;
        for (int d0 = 0; d0 < dim; d0 += RN_DC) {
            const int nd = min(RN_DC, dim - d0);
            for (int q = t; q < TH * RN_DC; q += TH) {
                const int r = q / RN_DC, dd = q % RN_DC;
                const int64_t i = row0 + r;
                xs[dd][r] = (i < n && dd < nd) ? (double)X[i * ldx + d0 + dd] : 0.0;
            }
            __syncthreads();
            if (pass == 0) {
                for (int dd = 0; dd < nd; ++dd) {
                    const double xd = xs[dd][t];
                    bad |= !isfinite(xd);
                    s = fma(xd, xd, s);
                }
            } else {
                if (RAW) {
                    for (int q = t; q < TH * RN_DC; q += TH) { // dimension-major: rows fastest
                        const int dd = q / TH, r = q % TH;
                        if (dd < nd && row0 + r < n) Yt[(int64_t)(d0 + dd) * n + row0 + r] = (TX)xs[dd][r];
                    }
                    __syncthreads();
                }
                for (int dd = 0; dd < nd; ++dd) {
                    double y = xs[dd][t];
                    if (normalize) y = nrm > 0.0 ? y / nrm : 0.0;
                    xs[dd][t] = y;
                    s2 = fma(y, y, s2);
                }
                __syncthreads();
                if (!RAW)
                    for (int q = t; q < TH * RN_DC; q += TH) { // dimension-major: rows fastest
                        const int dd = q / TH, r = q % TH;
                        if (dd < nd && row0 + r < n) Yt[(int64_t)(d0 + dd) * n + row0 + r] = (TX)xs[dd][r];
                    }
                if (Y)
                    for (int q = t; q < TH * RN_DC; q += TH) { // row-major: dimensions fastest
                        const int r = q / RN_DC, dd = q % RN_DC;
                        if (dd < nd && row0 + r < n) Y[(row0 + r) * dim + d0 + dd] = xs[dd][r];
                    }
            }
            __syncthreads();
        }
        if (pass == 1) {
            // non-negative doubles order like their bit patterns: wave maximum,
            // one atomic per wave
            unsigned long long b = live ? (unsigned long long)__double_as_longlong(s2) : 0ull;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const unsigned long long u = __shfl_xor(b, o, 64);
                b = u > b ? u : b;
            }
            if ((t & 63) == 0) atomicMax(m2bits, b);
        }
    }
    if (bad && live) atomicOr(status, DEV_NUMERIC);
}

// Seeding weights w_i = floor(D2_i 2^shift) are summed per tile of SEED_TILE
// consecutive points by the distance kernel (tsum[r][tile]).  The pick of
// centre j finds c_j = y[min i : prefix_i > t], t = mulhi64(u, T), T = sum w,
// in two levels: the tile whose inclusive prefix first exceeds t, then the
// point inside it (weights recomputed from D2); all sums are exact integers.
// Grid: R blocks of PICK_NT threads.
constexpr int SEED_TILE = 64;
constexpr int PICK_NT = 1024;
template <class TT>
__global__ void __launch_bounds__(PICK_NT)
k_seed_pick(int64_t n, int dim, int K, int j, int Rpad, const TT* __restrict__ Y, int64_t ldy,
            const YDiv* __restrict__ dv, const uint64_t* __restrict__ draws, const uint64_t* __restrict__ tsum,
            const double* __restrict__ D2, int shift, double* __restrict__ C,
            double* __restrict__ ccur) {
    __shared__ uint64_t part[PICK_NT];
    __shared__ uint64_t wtot[PICK_NT / 64];
    __shared__ int64_t pick;
    __shared__ int64_t tile_s;
    __shared__ uint64_t base_s;
    __shared__ int owner_s;
    const int r = blockIdx.x, tid = threadIdx.x;
    const uint64_t u = draws[(int64_t)r * K + j];
    if (tid == 0) pick = (int64_t)mulhi64(u, (uint64_t)n);
    if (j > 0) {
        const int64_t ntiles = (n + SEED_TILE - 1) / SEED_TILE;
        const uint64_t* ts = tsum + (int64_t)r * ntiles;
        const int64_t per = (ntiles + PICK_NT - 1) / PICK_NT;
        // thread tid's sum covers the tiles [tid per, (tid + 1) per); a wave's 64
        // ranges are one contiguous run of tiles, which its lanes read coalesced
        // and add into the owners' slots (integer sums: any order gives the same)
        part[tid] = 0;
        __syncthreads();
        {
            const int wave = tid >> 6, lane = tid & 63;
            const int64_t w0 = min((int64_t)wave * 64 * per, ntiles), w1 = min(w0 + 64 * per, ntiles);
            for (int64_t q = w0 + lane; q < w1; q += 64) atomicAdd(&part[(uint32_t)q / (uint32_t)per], ts[q]);
        }
        __syncthreads();
        const uint64_t mine = part[tid];
        // inclusive scan of the per-thread sums: within waves by shuffles, then
        // the totals of the earlier waves
        {
            const int wave = tid >> 6, lane = tid & 63;
            uint64_t incl = mine;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint64_t x = __shfl_up(incl, o);
                if (lane >= o) incl += x;
            }
            if (lane == 63) wtot[wave] = incl;
            __syncthreads();
            for (int w = 0; w < wave; ++w) incl += wtot[w];
            part[tid] = incl;
        }
        __syncthreads();
        const uint64_t T = part[PICK_NT - 1];
        if (T > 0) {
            const uint64_t t = mulhi64(u, T);
            const uint64_t lo = part[tid] - mine;            // prefix before this thread's tiles
            if (lo <= t && t < part[tid]) owner_s = tid;     // exactly one thread's range holds t
            __syncthreads();
            // the owner's tiles, 64 at a time by wave 0: the first whose inclusive
            // prefix exceeds t, and the prefix before it
            if (tid < 64) {
                const int ow = owner_s;
                const int64_t a0 = min((int64_t)ow * per, ntiles), a1 = min(a0 + per, ntiles);
                uint64_t acc = ow > 0 ? part[ow - 1] : 0;     // prefix before the owner's tiles
                for (int64_t c0 = a0; c0 < a1; c0 += 64) {
                    const int64_t q = c0 + tid;
                    const uint64_t w = q < a1 ? ts[q] : 0;
                    uint64_t incl = w;
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const uint64_t x = __shfl_up(incl, o);
                        if (tid >= o) incl += x;
                    }
                    const unsigned long long m = __ballot(q < a1 && t < acc + incl);
                    if (m) {
                        const int f = __ffsll((long long)m) - 1;
                        const uint64_t before = __shfl(incl - w, f);
                        if (tid == 0) {
                            tile_s = c0 + f;
                            base_s = acc + before;
                        }
                        break;
                    }
                    acc += __shfl(incl, 63);
                }
            }
            __syncthreads();
            if (tid < 64) {
                const int64_t i = tile_s * SEED_TILE + tid;
                uint64_t wv = i < n ? (uint64_t)floor(ldexp(D2[(int64_t)r * n + i], shift)) : 0;
                uint64_t incl = wv;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint64_t x = __shfl_up(incl, o);
                    if (tid >= o) incl += x;
                }
                const bool hit = i < n && base_s + incl > t;
                const unsigned long long m = __ballot(hit);
                if (tid == 0) pick = tile_s * SEED_TILE + (__ffsll((long long)m) - 1);
            }
        }
    }
    __syncthreads();
    const int64_t pk = pick;
    double* c = C + ((int64_t)r * K + j) * dim;
    const YDiv dp = ydiv_of<TT>(dv, pk);
    for (int d = tid; d < dim; d += PICK_NT) {
        const double v = ycoord(Y[pk * ldy + d], dp);
        c[d] = v;
        ccur[(int64_t)d * Rpad + r] = v;      // this round's centres, dimension-major
    }
}


// For every point and every restart: D2 <- dist(y_i, c_j) (j == 0) or
// min(D2, dist(y_i, c_j)); then the integer weights.  One pass over Y serves
// up to RB restarts.
constexpr int RB = 16;
// the accumulator width a seeding pass uses for R restarts
inline int seed_width(int R) {
    return R <= 1 ? 1 : R <= 2 ? 2 : R <= 4 ? 4 : R <= 8 ? 8 : R <= 10 ? 10 : R <= 12 ? 12 : RB;
}
// Row stride of the dimension-major centres: a whole number of passes, and no
// wider, so that the rows a pass reads through the scalar cache stay compact
// (160 dimensions x 10 restarts: 12.8 KB rather than 20 KB at stride 16).
inline int seed_stride(int R) { return R <= RB ? seed_width(R) : (R + RB - 1) / RB * RB; }
// WB restarts per pass over the points (WB <= RB; the launch picks the
// smallest width covering the restarts, so no accumulator is wasted)
template <int WB, class TT>
__global__ void __launch_bounds__(TH)
k_seed_d2(int64_t n, int dim, int R, int Rpad, int j, const TT* __restrict__ Yt,
          const YDiv* __restrict__ dv, const double* __restrict__ ccur, double* __restrict__ D2,
          uint64_t* __restrict__ tsum, int shift, int32_t* __restrict__ lab,
          float* __restrict__ secf) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i0 < n;
    const int64_t i = live ? i0 : n - 1;
    const YDiv dvi = ydiv_of<TT>(dv, i);
    const int64_t ntiles = (n + SEED_TILE - 1) / SEED_TILE;
    const int64_t tile = i0 / SEED_TILE;    // a wave is one tile
    for (int r0 = 0; r0 < R; r0 += WB) {
        double acc[WB];
#pragma unroll
        for (int q = 0; q < WB; ++q) acc[q] = 0.0;
        // all WB accumulators, no predicates: ccur is zero beyond restart R, and
        // those lanes' sums are never stored (wide uniform loads, pipelined)
        constexpr int DU = 8;                 // coordinates loaded ahead of their use
        int d = 0;
        for (; d + DU <= dim; d += DU) {
            TT y[DU];
#pragma unroll
            for (int u = 0; u < DU; ++u) y[u] = Yt[(int64_t)(d + u) * n + i];
#pragma unroll
            for (int u = 0; u < DU; ++u) {
                const double* cd = ccur + (int64_t)(d + u) * Rpad + r0;   // wave-uniform, contiguous
                const double yu = ycoord(y[u], dvi);
#pragma unroll
                for (int q = 0; q < WB; ++q) {
                    const double diff = yu - cd[q];
                    acc[q] = fma(diff, diff, acc[q]);
                }
            }
        }
        for (; d < dim; ++d) {
            const double y = ycoord(Yt[(int64_t)d * n + i], dvi);
            const double* cd = ccur + (int64_t)d * Rpad + r0;
#pragma unroll
            for (int q = 0; q < WB; ++q) {
                const double diff = y - cd[q];
                acc[q] = fma(diff, diff, acc[q]);
            }
        }
        // D2 = least distance so far (the seeding weights, stored only when it
        // changes); lab = its centre; secf = a lower bound of the second least
        // distance (rounded down to FP32).  After the last centre they give the
        // first assignment (ties to the lowest centre) and its Hamerly bounds.
#pragma unroll
        for (int q = 0; q < WB; ++q) {
            if (r0 + q < R) {
                const int64_t e = (int64_t)(r0 + q) * n + i;
                const double a = acc[q];
                double v = 0.0;
                if (live) {
                    if (j == 0) {
                        v = a;
                        secf[e] = INFINITY;
                        lab[e] = 0;
                        D2[e] = v;
                    } else {
                        v = D2[e];
                        if (a < v) {
                            secf[e] = __double2float_rd(v);
                            v = a;
                            lab[e] = j;
                            D2[e] = v;
                        } else if (a < (double)secf[e]) {
                            secf[e] = __double2float_rd(a);
                        }
                    }
                }
                // the tile's weight sum
                uint64_t ws = live ? (uint64_t)floor(ldexp(v, shift)) : 0;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) ws += __shfl_xor(ws, o);
                if ((threadIdx.x & 63) == 0 && tile < ntiles) tsum[(int64_t)(r0 + q) * ntiles + tile] = ws;
            }
        }
    }
}

// first assignment from the seeding's distances: Hamerly bounds from the
// least distance (D2) and the lower bound of the second least (secf)
__global__ void k_first_bounds(int64_t nr, const double* __restrict__ D2, float* __restrict__ ub,
                               const float* __restrict__ secf, float* __restrict__ lb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nr) return;
    ub[e] = __double2float_ru(sqrt(D2[e]) * (1.0 + BOUND_MARGIN) + BOUND_TINY);
    const double s = secf[e];
    lb[e] = isinf(s) ? INFINITY : __double2float_rd(sqrt(s) * (1.0 - BOUND_MARGIN) - BOUND_TINY);
}

// Ct[r][d][j] = C[r][j][d] for j < K; columns K <= j < Kpad hold +inf, a
// centre no point is ever nearest (or second nearest) to
__global__ void k_transpose_centroids(int R, int K, int Kpad, int dim, const double* __restrict__ C,
                                      double* __restrict__ Ct) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)R * Kpad * dim) return;
    const int j = (int)(e % Kpad);
    const int64_t rd = e / Kpad;
    const int d = (int)(rd % dim);
    const int r = (int)(rd / dim);
    Ct[e] = j < K ? C[((int64_t)r * K + j) * dim + d] : INFINITY;
}

__global__ void k_fill_lists(int64_t n, int R, uint32_t* __restrict__ pts, int* __restrict__ cnt) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n * R) pts[e] = (uint32_t)(e % n);
    if (e < R) cnt[e] = (int)n;
}

// Nearest and second-nearest centre for the listed points of restart r
// (blockIdx.y).  64 points per workgroup; their coordinates are staged in
// LDS in chunks of 32 dimensions; each of the four waves scans its own range
// of JB centres per pass, with the centre coordinates read as wave-uniform
// (scalar) loads from the transposed centroid table.  Every distance is the
// full fma chain over the dimensions in order.
template <int JB, class TT>
__global__ void __launch_bounds__(TH)
k_assign_list(int64_t n, int dim, int K, int Kpad, const TT* __restrict__ Y, int64_t ldy,
              const YDiv* __restrict__ dv, const double* __restrict__ Ct, const uint32_t* __restrict__ pts,
              const int* __restrict__ cnt, const int* __restrict__ active,
              int32_t* __restrict__ lab, float* __restrict__ ub, float* __restrict__ lb,
              int* __restrict__ changed, int* __restrict__ dirty, int first) {
    constexpr int DC = 32;
    __shared__ double ys[DC][65];   // padded row: fewer LDS bank conflicts on the transposing store
    __shared__ uint32_t pid[64];
    __shared__ YDiv pdv[64];
    __shared__ double wbest[4][64], wsec[4][64];
    __shared__ int wj[4][64];
    const int r = blockIdx.y;
    if (!active[r]) return;
    const int c = cnt[r];
    const int q0 = blockIdx.x * 64;
    if (q0 >= c) return;
    const int np = min(64, c - q0);
    const int lane = threadIdx.x & 63;
    const int wave = uniform(threadIdx.x >> 6);
    if (threadIdx.x < 64) {
        const uint32_t i = pts[(int64_t)r * n + q0 + min((int)threadIdx.x, np - 1)];
        pid[threadIdx.x] = i;
        pdv[threadIdx.x] = ydiv_of<TT>(dv, i);
    }
    double best = INFINITY, second = INFINITY;
    int bj = K;
    const int passes = Kpad / (4 * JB);
    const double* Ctr = Ct + (int64_t)r * dim * Kpad;
    for (int pass = 0; pass < passes; ++pass) {
        const int cb = uniform(pass * 4 * JB + wave * JB);
        double acc[JB];
#pragma unroll
        for (int u = 0; u < JB; ++u) acc[u] = 0.0;
        for (int d0 = 0; d0 < dim; d0 += DC) {
            __syncthreads();
            for (int q = threadIdx.x; q < 64 * DC; q += TH) {
                const int p = q / DC, dd = q % DC;
                ys[dd][p] = d0 + dd < dim ? ycoord(Y[(int64_t)pid[p] * ldy + d0 + dd], pdv[p]) : 0.0;
            }
            __syncthreads();
            if (cb < K) {
                const int nd = min(DC, dim - d0);
                for (int dd = 0; dd < nd; ++dd) {
                    const double y = ys[dd][lane];
                    const double* crow = Ctr + (int64_t)(d0 + dd) * Kpad + cb;
                    constexpr int G = JB < 8 ? JB : 8;
#pragma unroll
                    for (int u0 = 0; u0 < JB; u0 += G) {
                        double cv[G];
#pragma unroll
                        for (int q = 0; q < G; ++q) cv[q] = crow[u0 + q];
#pragma unroll
                        for (int q = 0; q < G; ++q) {
                            const double diff = y - cv[q];
                            acc[u0 + q] = fma(diff, diff, acc[u0 + q]);
                        }
                    }
                }
            }
        }
        if (cb < K) {
#pragma unroll
            for (int u = 0; u < JB; ++u) {
                if (cb + u < K) {
                    const double v = acc[u];
                    if (v < best) {
                        second = best;
                        best = v;
                        bj = cb + u;
                    } else if (v < second) {
                        second = v;
                    }
                }
            }
        }
    }
    wbest[wave][lane] = best;
    wsec[wave][lane] = second;
    wj[wave][lane] = bj;
    __syncthreads();
    if (threadIdx.x < 64 && lane < np) {
        double b = INFINITY, s = INFINITY;
        int j = K;
        for (int w = 0; w < 4; ++w) {
            const double v = wbest[w][lane], sv = wsec[w][lane];
            const int jw = wj[w][lane];
            if (jw >= K) continue;
            if (v < b || (v == b && jw < j)) {
                s = fmin(fmin(s, b), sv);
                b = v;
                j = jw;
            } else {
                s = fmin(s, v);
            }
        }
        const int64_t e = (int64_t)r * n + pid[lane];
        if (!first) {
            const int old = lab[e];
            if (old != j) {
                atomicAdd(&changed[r], 1);
                dirty[(int64_t)r * K + old] = 1;    // both member lists changed
                dirty[(int64_t)r * K + j] = 1;
            }
        }
        lab[e] = j;
        ub[e] = __double2float_ru(sqrt(b) * (1.0 + BOUND_MARGIN) + BOUND_TINY);
        lb[e] = isinf(s) ? INFINITY : __double2float_rd(sqrt(s) * (1.0 - BOUND_MARGIN) - BOUND_TINY);
    }
}

constexpr int PR_DC = 8;                // dimensions per staged chunk: 64 B of a row
template <class TT>
constexpr int pr_dc() { return PR_DC * 8 / (int)sizeof(TT); }
constexpr int PR_KMAX = 1024;
constexpr int PR_KMAX_HS = PR_KMAX;
constexpr int PR_WIDE = 16;
constexpr int PR_LIST_MIN = 2048;       // shorter lists go to the full scan whole
// the pruned path runs when (points listed over all restarts) x K reaches this
constexpr int64_t PR_WORK_MIN = 32000000;

// Half the separation of every centre pair, h(a, j) <= ||c_a - c_j|| / 2
// (deflated by the bound margin; 0 for j = a), from the transposed centroid
// table.  Elkan's lemma: a point with ||y - c_a|| <= u < h(a, j) is strictly
// nearer to c_a than to c_j.  Each centre's row is stored sorted ascending
// (ties by index): hsv[r][a][t] the t-th least value, hsi[r][a][t] its centre.
// One workgroup per (centre a, restart r).
__global__ void __launch_bounds__(TH)
k_half_sep(int K, int Kpad, int dim, const double* __restrict__ Ct, const int* __restrict__ active,
           double* __restrict__ hsv, uint16_t* __restrict__ hsi) {
    __shared__ double hv[PR_KMAX_HS];
    const int r = blockIdx.y, a = blockIdx.x;
    if (!active[r]) return;
    const double* ct = Ct + (int64_t)r * dim * Kpad;
    for (int j = threadIdx.x; j < K; j += TH) {
        double s = 0.0;
        for (int d = 0; d < dim; ++d) {
            const double t = ct[(int64_t)d * Kpad + a] - ct[(int64_t)d * Kpad + j];
            s = fma(t, t, s);
        }
        hv[j] = a == j ? 0.0 : 0.5 * sqrt(s) * (1.0 - BOUND_MARGIN) - BOUND_TINY;
    }
    __syncthreads();
    const int64_t row = ((int64_t)r * K + a) * K;
    for (int j = threadIdx.x; j < K; j += TH) {
        const double v = hv[j];
        int rank = 0;
        for (int l = 0; l < K; ++l) {
            const double w = hv[l];
            rank += w < v || (w == v && l < j);
        }
        hsv[row + rank] = v;
        hsi[row + rank] = (uint16_t)j;
    }
}

// Lloyd scan of the listed points with Elkan pruning.  Each wave owns 64
// consecutive list entries; the list is ordered by current label, so a
// wave's points share one or a few labels.
//   1. The exact distance to the assigned centre a gives a tight bound u.
//   2. A centre j with u < h(a, j) cannot be nearer than c_a.  A point that
//      cannot rule out more than PR_WIDE centres is "wide" and is handed to
//      the full scan (appended to the list fl), and so is every point of a
//      list shorter than PR_LIST_MIN.  The rest are "narrow": their candidates are
//      the head of their centre's sorted row, merged into a wave bitmap.
//   3. The wave scans the union of the narrow points' candidates, in
//      ascending order, JB at a time.
// Rows are staged in LDS PR_DC dimensions at a time (the next chunk is loaded
// into registers while the current one is used); centre coordinates come from
// the transposed table.  Every distance is the full fma chain in dimension
// order, and a ruled-out centre is strictly farther than c_a, so the argmin
// (lowest index on ties) equals a full scan's.  The new lower bound covers the
// centres nobody scanned by the triangle inequality,
// ||y - c_j|| >= 2 h(a, j) - ||y - c_a||.
template <class TT, int DC>
__device__ inline void pr_load(TT (&v)[DC], const TT* __restrict__ Y, int64_t ldy,
                               const uint32_t* pidw, int dim, int d0, int lane) {
#pragma unroll
    for (int t = 0; t < DC; ++t) {
        const int q = t * 64 + lane;
        const int p = q / DC, dd = q % DC;
        v[t] = d0 + dd < dim ? Y[(int64_t)pidw[p] * ldy + d0 + dd] : (TT)0;
    }
}

template <class TT, int DC>
__device__ inline void pr_store(TT (*ys)[65], const TT (&v)[DC], int lane) {
#pragma unroll
    for (int t = 0; t < DC; ++t) {
        const int q = t * 64 + lane;
        ys[q % DC][q / DC] = v[t];
    }
}

template <int JB, class TT>
__global__ void __launch_bounds__(TH)
k_assign_pruned(int64_t n, int dim, int K, int Kpad, const TT* __restrict__ Y, int64_t ldy,
                const YDiv* __restrict__ dv, const double* __restrict__ Ct, const double* __restrict__ C,
                const double* __restrict__ hsv, const uint16_t* __restrict__ hsi,
                const uint32_t* __restrict__ pts,
                const int* __restrict__ cnt, const int* __restrict__ active,
                int32_t* __restrict__ lab, float* __restrict__ ub, float* __restrict__ lb,
                int* __restrict__ changed, int* __restrict__ dirty, uint32_t* __restrict__ fl,
                int* __restrict__ fcnt) {
    constexpr int NW = TH / 64;
    constexpr int DC = pr_dc<TT>();
    __shared__ TT ys[NW][DC][65];      // raw values; each lane forms its own point's y
    __shared__ uint32_t pid[NW][64];
    __shared__ uint16_t cand[NW][PR_KMAX];
    __shared__ uint32_t bits[NW][PR_KMAX / 32];
    const int r = blockIdx.y;
    if (!active[r]) return;
    const int c = cnt[r];
    const int wave = uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int q0 = (blockIdx.x * NW + wave) * 64;
    if (q0 >= c) return;                    // wave-uniform; no workgroup barrier below
    const int np = min(64, c - q0);
    const bool live = lane < np;
    const uint32_t i = pts[(int64_t)r * n + q0 + min(lane, np - 1)];
    const int64_t e = (int64_t)r * n + i;
    const uint64_t lanes_below = (1ull << lane) - 1ull;
    if (c < PR_LIST_MIN) {
        // short list: every point goes to the full scan
        const unsigned long long mask = __ballot(live);
        int base = 0;
        if (lane == 0) base = atomicAdd(&fcnt[r], (int)__popcll(mask));
        base = __shfl(base, 0);
        if (live) fl[(int64_t)r * n + base + __popcll(mask & lanes_below)] = i;
        return;
    }
    const int nwords = (K + 31) / 32;
    pid[wave][lane] = i;
    if (lane < nwords) bits[wave][lane] = 0u;
    const int a = lab[e];
    const YDiv mdv = ydiv_of<TT>(dv, i);
    const double* Ctr = Ct + (int64_t)r * dim * Kpad;
    const double* Cr = C + (int64_t)r * K * dim;
    __builtin_amdgcn_wave_barrier();
    // 1. exact distance to the assigned centre
    double own = 0.0;
    {
        const double* ca = Ctr + a;
        TT v[DC];
        double cv[DC];
        pr_load(v, Y, ldy, pid[wave], dim, 0, lane);
#pragma unroll
        for (int dd = 0; dd < DC; ++dd) cv[dd] = dd < dim ? ca[(int64_t)dd * Kpad] : 0.0;
        for (int d0 = 0; d0 < dim; d0 += DC) {
            pr_store(ys[wave], v, lane);
            double cc[DC];
#pragma unroll
            for (int dd = 0; dd < DC; ++dd) cc[dd] = cv[dd];
            if (d0 + DC < dim) {
                pr_load(v, Y, ldy, pid[wave], dim, d0 + DC, lane);
#pragma unroll
                for (int dd = 0; dd < DC; ++dd)
                    cv[dd] = d0 + DC + dd < dim ? ca[(int64_t)(d0 + DC + dd) * Kpad] : 0.0;
            }
            __builtin_amdgcn_wave_barrier();
            const int nd = min(DC, dim - d0);
#pragma unroll
            for (int dd = 0; dd < DC; ++dd) {
                if (dd < nd) {
                    const double diff = ycoord(ys[wave][dd][lane], mdv) - cc[dd];
                    own = fma(diff, diff, own);
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    const double u = sqrt(own) * (1.0 + BOUND_MARGIN) + BOUND_TINY;
    const int64_t row = ((int64_t)r * K + a) * K;
    // 2. wide: the PR_WIDE-th smallest half-separation (0-based) is not above u
    const bool wide = live && K > PR_WIDE && !(u < hsv[row + PR_WIDE]);
    const bool narrow = live && !wide;
    {
        const unsigned long long mask = __ballot(wide);
        if (mask) {
            int base = 0;
            if (lane == 0) base = atomicAdd(&fcnt[r], (int)__popcll(mask));
            base = __shfl(base, 0);
            if (wide) fl[(int64_t)r * n + base + __popcll(mask & lanes_below)] = i;
        }
    }
    // a narrow point's candidates: the head of its sorted row (own centre aside)
    int nkeep = 0;
    if (narrow) {
        while (nkeep < K && !(u < hsv[row + nkeep])) {
            const int j = hsi[row + nkeep];
            if (j != a) atomicOr(&bits[wave][j >> 5], 1u << (j & 31));
            ++nkeep;
        }
    }
    __builtin_amdgcn_wave_barrier();
    // the union as an ascending list: lane l expands word l
    int m = 0;
    {
        const uint32_t wbits = lane < nwords ? bits[wave][lane] : 0u;
        const int pc = __popc(wbits);
        int incl = pc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        m = __shfl(incl, 63);
        int off = incl - pc;
        uint32_t b = wbits;
        while (b) {
            const int bit = __ffs(b) - 1;
            cand[wave][off++] = (uint16_t)(lane * 32 + bit);
            b &= b - 1u;
        }
    }
    // least half-separation over the centres nobody scans
    double hmin = INFINITY;
    if (narrow) {
        for (int t = nkeep; t < K; ++t) {
            const int j = hsi[row + t];
            if (j == a || ((bits[wave][j >> 5] >> (j & 31)) & 1u)) continue;
            hmin = hsv[row + t];
            break;
        }
    }
    __builtin_amdgcn_wave_barrier();
    // 3. scan of the candidates
    double best = own, second = INFINITY;
    int bj = a;
    for (int g0 = 0; g0 < m; g0 += JB) {
        int cj[JB];
#pragma unroll
        for (int u2 = 0; u2 < JB; ++u2) cj[u2] = uniform(cand[wave][min(g0 + u2, m - 1)]);
        double acc[JB];
#pragma unroll
        for (int u2 = 0; u2 < JB; ++u2) acc[u2] = 0.0;
        TT v[DC];
        pr_load(v, Y, ldy, pid[wave], dim, 0, lane);
        for (int d0 = 0; d0 < dim; d0 += DC) {
            pr_store(ys[wave], v, lane);
            if (d0 + DC < dim) pr_load(v, Y, ldy, pid[wave], dim, d0 + DC, lane);
            __builtin_amdgcn_wave_barrier();
            const int nd = min(DC, dim - d0);
#pragma unroll
            for (int dd = 0; dd < DC; ++dd) {
                if (dd < nd) {
                    const double y = ycoord(ys[wave][dd][lane], mdv);
#pragma unroll
                    for (int u2 = 0; u2 < JB; ++u2) {
                        // centre-major rows: a candidate's coordinates are contiguous
                        const double diff = y - Cr[(int64_t)cj[u2] * dim + d0 + dd];
                        acc[u2] = fma(diff, diff, acc[u2]);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int u2 = 0; u2 < JB; ++u2) {
            if (g0 + u2 < m) {
                const double v2 = acc[u2];
                const int j = cj[u2];
                if (v2 < best || (v2 == best && j < bj)) {
                    second = best;
                    best = v2;
                    bj = j;
                } else if (v2 < second) {
                    second = v2;
                }
            }
        }
    }
    const bool moved = narrow && bj != a;
    const unsigned long long mv = __ballot(moved);
    if (mv && lane == 0) atomicAdd(&changed[r], (int)__popcll(mv));
    if (!narrow) return;
    if (moved) {
        dirty[(int64_t)r * K + a] = 1;          // both member lists changed
        dirty[(int64_t)r * K + bj] = 1;
    }
    lab[e] = bj;
    ub[e] = __double2float_ru(sqrt(best) * (1.0 + BOUND_MARGIN) + BOUND_TINY);
    double l = isinf(second) ? INFINITY : sqrt(second) * (1.0 - BOUND_MARGIN) - BOUND_TINY;
    if (hmin < INFINITY) l = fmin(l, (2.0 * hmin - u) * (1.0 - BOUND_MARGIN) - BOUND_TINY);
    lb[e] = __double2float_rd(l);
}

// centre displacements: delta[r][j] = ||c_new - c_old|| (inflated); a centre
// whose member list did not change kept its coordinates, so its displacement
// is 0.  One wave per centre, lanes along the dimensions (the order of the sum
// does not matter: the value only moves bounds, with the bound margin).
__global__ void __launch_bounds__(TH)
k_delta(int K, int R, int dim, const double* __restrict__ C, const double* __restrict__ Cold,
        const int* __restrict__ active, const int* __restrict__ dirty, double* __restrict__ delta) {
    const int64_t rj = (int64_t)blockIdx.x * (TH / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (rj >= (int64_t)R * K || !active[rj / K]) return;
    if (!dirty[rj]) {
        if (lane == 0) delta[rj] = 0.0;
        return;
    }
    const double* cn = C + rj * dim;
    const double* co = Cold + rj * dim;
    double s = 0.0;
    for (int d = lane; d < dim; d += 64) {
        const double t = cn[d] - co[d];
        s = fma(t, t, s);
    }
    s = sc_wave_sum(s);
    if (lane == 0) delta[rj] = sqrt(s) * (1.0 + BOUND_MARGIN) + BOUND_TINY;
}

// per restart the largest displacement (with its centre) and the second
// largest; one wave per restart
__global__ void __launch_bounds__(64)
k_delta_max(int K, const int* __restrict__ active, const double* __restrict__ delta,
            double* __restrict__ dinfo) {
    const int r = blockIdx.x, lane = threadIdx.x;
    if (!active[r]) return;
    double m1 = 0.0, m2 = 0.0;
    int a1 = -1;
    for (int j = lane; j < K; j += 64) {
        const double dj = delta[(int64_t)r * K + j];
        if (dj > m1) {
            m2 = m1;
            m1 = dj;
            a1 = j;
        } else if (dj > m2) {
            m2 = dj;
        }
    }
    // combine the lanes in order (lane 0 first), as a serial scan would
    __shared__ double sm1[64], sm2[64];
    __shared__ int sa[64];
    sm1[lane] = m1;
    sm2[lane] = m2;
    sa[lane] = a1;
    __syncthreads();
    if (lane == 0) {
        double b1 = 0.0, b2 = 0.0;
        int arg = -1;
        for (int t = 0; t < 64; ++t) {
            if (sm1[t] > b1) {
                b2 = fmax(b1, sm2[t]);
                b1 = sm1[t];
                arg = sa[t];
            } else {
                b2 = fmax(b2, sm1[t]);
            }
        }
        dinfo[3 * r + 0] = b1;
        dinfo[3 * r + 1] = (double)arg;
        dinfo[3 * r + 2] = b2;
    }
}

// move the bounds by the displacements; list the points that need a scan.
// Grid: x over tiles of TH * PPT points, y over restarts; the tile's list
// entries are reserved with a single atomic (the counters are per restart,
// so per-wave atomics would serialise on a handful of addresses).
constexpr int PPT = 8;
__global__ void __launch_bounds__(TH)
k_bounds(int64_t n, int K, const int32_t* __restrict__ lab, float* __restrict__ ub,
         float* __restrict__ lb, const double* __restrict__ delta, const double* __restrict__ dinfo,
         const int* __restrict__ active, uint32_t* __restrict__ pts, int* __restrict__ cnt) {
    __shared__ int wtot[TH / 64];
    __shared__ int base_s;
    const int r = blockIdx.y;
    if (!active[r]) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double dmax0 = dinfo[3 * r + 0], dmax1 = dinfo[3 * r + 2];
    const int amax = (int)dinfo[3 * r + 1];
    unsigned long long masks[PPT];
    int mine = 0;
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
        const int64_t i = ((int64_t)blockIdx.x * PPT + u) * TH + threadIdx.x;
        bool need = false;
        if (i < n) {
            const int64_t e = (int64_t)r * n + i;
            const int a = lab[e];
            const double dmax = a == amax ? dmax1 : dmax0;
            const double uu = (ub[e] + delta[(int64_t)r * K + a]) * (1.0 + BOUND_MARGIN);
            const double ll = (lb[e] - dmax) * (1.0 - BOUND_MARGIN) - BOUND_TINY;
            ub[e] = __double2float_ru(uu);
            lb[e] = __double2float_rd(ll);
            need = !(uu < ll);
        }
        masks[u] = __ballot(need);
        mine += __popcll(masks[u]);
    }
    if (lane == 0) wtot[wave] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int q = 0; q < TH / 64; ++q) t += wtot[q];
        base_s = t ? atomicAdd(&cnt[r], t) : 0;
    }
    __syncthreads();
    int off = base_s;
    for (int q = 0; q < wave; ++q) off += wtot[q];
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
        const unsigned long long mask = masks[u];
        if ((mask >> lane) & 1ull) {
            const int64_t i = ((int64_t)blockIdx.x * PPT + u) * TH + threadIdx.x;
            pts[(int64_t)r * n + off + __popcll(mask & ((1ull << lane) - 1ull))] = (uint32_t)i;
        }
        off += __popcll(mask);
    }
}

// Member lists: a stable counting sort of each active restart's points by
// label (ascending vertex order within a label).  Tiles of LS_TILE points:
// per-tile label histograms (label-major, tile-minor), one exclusive scan per
// restart, then every tile is ordered by label in LDS with stable two-bit
// splits (two label bits per pass) and scattered to its offsets.  The scan also gives the
// segment of every label directly.
constexpr int LS_ITEMS = 8;
constexpr int LS_TILE = TH * LS_ITEMS;

// Exclusive scan over the workgroup of four 16-bit counters packed in a
// 64-bit word (each field's block total stays below 2^16: a tile holds
// LS_TILE points); *total = the block's sums.
static_assert(2 * LS_TILE < 65536, "16-bit digit counters plus digit bases");
__device__ inline uint64_t ls_block_excl_scan4(uint64_t v, uint64_t* total, uint64_t* wsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t acc = 0;
        for (int w = 0; w < TH / 64; ++w) {
            const uint64_t t = wsum[w];
            wsum[w] = acc;
            acc += t;
        }
        wsum[TH / 64] = acc;
    }
    __syncthreads();
    const uint64_t r = x - v + wsum[wave];
    *total = wsum[TH / 64];
    __syncthreads();
    return r;
}

// The same sort serves the scan lists: with `list` given, restart r sorts its
// first counts[r] entries list[r n + q] by lab[r n + list[r n + q]]; without,
// it sorts its points 0 .. n - 1.  grid (tiles, R)
__global__ void __launch_bounds__(TH)
k_lab_hist(int64_t n, int K, const int* __restrict__ active, const int32_t* __restrict__ lab,
           const uint32_t* __restrict__ list, const int* __restrict__ counts,
           uint64_t* __restrict__ hist, int ntiles) {
    __shared__ uint32_t h[PR_KMAX];
    const int r = blockIdx.y;
    if (!active[r]) return;
    for (int b = threadIdx.x; b < K; b += TH) h[b] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * LS_TILE;
    const int64_t c = list ? counts[r] : n;
    const int32_t* lr = lab + (int64_t)r * n;
    const uint32_t* li = list ? list + (int64_t)r * n : nullptr;
#pragma unroll
    for (int t = 0; t < LS_ITEMS; ++t) {
        const int64_t idx = base + (int64_t)t * TH + threadIdx.x;
        if (idx < c) atomicAdd(&h[lr[li ? li[idx] : idx]], 1u);
    }
    __syncthreads();
    uint64_t* hr = hist + (int64_t)r * K * ntiles;
    for (int b = threadIdx.x; b < K; b += TH) hr[(int64_t)b * ntiles + blockIdx.x] = h[b];
}

// label segments from the scanned histogram: seg[2 (r K + b)] / seg[2 (r K + b) + 1]
// = first / one past the last position of label b in restart r's list
__global__ void k_lab_segments(int64_t n, int K, int R, const int* __restrict__ active,
                               const uint64_t* __restrict__ off, int ntiles,
                               int64_t* __restrict__ seg) {
    const int64_t rj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (rj >= (int64_t)R * K) return;
    const int r = (int)(rj / K), b = (int)(rj % K);
    if (!active[r]) return;
    const uint64_t* o = off + (int64_t)r * K * ntiles;
    const int64_t start = (int64_t)o[(int64_t)b * ntiles];
    const int64_t end = b + 1 < K ? (int64_t)o[(int64_t)(b + 1) * ntiles] : n;
    seg[2 * rj] = (int64_t)r * n + start;
    seg[2 * rj + 1] = (int64_t)r * n + end;
}

// grid (tiles, R); vals[r n + position] = vertex
__global__ void __launch_bounds__(TH)
k_lab_scatter(int64_t n, int K, int nbits, const int* __restrict__ active,
              const int32_t* __restrict__ lab, const uint32_t* __restrict__ list,
              const int* __restrict__ counts, const uint64_t* __restrict__ off, int ntiles,
              uint32_t* __restrict__ vals) {
    __shared__ uint16_t kb[2][LS_TILE];
    __shared__ uint32_t vb[2][LS_TILE];
    __shared__ uint64_t wsum[TH / 64 + 1];
    __shared__ uint32_t lstart[PR_KMAX];
    const int r = blockIdx.y;
    if (!active[r]) return;
    const int64_t base = (int64_t)blockIdx.x * LS_TILE;
    const int64_t c = list ? counts[r] : n;
    if (base >= c) return;
    const int cnt = (int)min<int64_t>(LS_TILE, c - base);
    const int32_t* lr = lab + (int64_t)r * n;
    const uint32_t* li = list ? list + (int64_t)r * n : nullptr;
    // padding carries the largest key and stays behind every real point
    const uint16_t pad = (uint16_t)((1u << nbits) - 1u);
#pragma unroll
    for (int t = 0; t < LS_ITEMS; ++t) {
        const int p = t * TH + threadIdx.x;
        const uint32_t v = p < cnt ? (li ? li[base + p] : (uint32_t)(base + p)) : 0u;
        kb[0][p] = p < cnt ? (uint16_t)lr[v] : pad;
        vb[0][p] = v;
    }
    __syncthreads();
    // stable LSD radix sort of the tile in shared memory, two key bits per
    // pass: a digit's items go to its base (the tile's items with smaller
    // digits) plus the items with the same digit before them (earlier
    // threads, then earlier items of the same thread)
    int cur = 0;
    for (int bit = 0; bit < nbits; bit += 2) {
        const uint32_t dmask = bit + 1 < nbits ? 3u : 1u;
        uint16_t k[LS_ITEMS];
        uint32_t v[LS_ITEMS];
        uint64_t cnt4 = 0;
#pragma unroll
        for (int t = 0; t < LS_ITEMS; ++t) {
            k[t] = kb[cur][threadIdx.x * LS_ITEMS + t];
            v[t] = vb[cur][threadIdx.x * LS_ITEMS + t];
            cnt4 += 1ull << (16 * ((k[t] >> bit) & dmask));
        }
        uint64_t tot;
        uint64_t pos = ls_block_excl_scan4(cnt4, &tot, wsum);
        // digit bases, packed like the counters: field d = sum of totals below d
        const uint64_t base = (tot << 16) + (tot << 32) + (tot << 48);
        pos += base;
#pragma unroll
        for (int t = 0; t < LS_ITEMS; ++t) {
            const int sh = 16 * (int)((k[t] >> bit) & dmask);
            const uint32_t np = (uint32_t)((pos >> sh) & 0xFFFFu);
            pos += 1ull << sh;
            kb[cur ^ 1][np] = k[t];
            vb[cur ^ 1][np] = v[t];
        }
        cur ^= 1;
        __syncthreads();
    }
    // first sorted position of every label present in the tile
#pragma unroll
    for (int t = 0; t < LS_ITEMS; ++t) {
        const int p = threadIdx.x * LS_ITEMS + t;
        if (p < cnt) {
            const uint16_t key = kb[cur][p];
            if (p == 0 || kb[cur][p - 1] != key) lstart[key] = p;
        }
    }
    __syncthreads();
    const uint64_t* o = off + (int64_t)r * K * ntiles;
    uint32_t* vr = vals + (int64_t)r * n;
#pragma unroll
    for (int t = 0; t < LS_ITEMS; ++t) {
        const int p = t * TH + threadIdx.x;
        if (p < cnt) {
            const uint16_t key = kb[cur][p];
            vr[o[(int64_t)key * ntiles + blockIdx.x] + (p - (int)lstart[key])] = vb[cur][p];
        }
    }
}

// Centroid update.  Dimension d of centroid (r, j) is one FP64 chain: from
// 0.0, y_id of every member i of cluster j added in ascending vertex order
// (the stable sort by label keeps vertex order within a label), then divided
// by the member count.  A wave owns one cluster and 64 consecutive
// dimensions (lane = dimension): the member ids and their row divisors are
// wave-uniform scalar loads, a member's coordinates are one contiguous read
// across the lanes, and the loads of U members are issued ahead of their
// additions.  Only clusters whose member list changed since their last update
// are summed again (an unchanged list gives a bitwise identical sum); an empty
// cluster keeps its centroid.
__device__ inline bool km_needs_update(int64_t rj, int K, const int* active, const int* dirty,
                                       const int64_t* seg) {
    return active[rj / K] && dirty[rj] && seg[2 * rj + 1] > seg[2 * rj];
}

// One workgroup per (cluster, 64-coordinate slab): wave 0 runs the chains
// (lane = coordinate) and waves 1 .. PW gather member rows for it.  A
// single wave doing both issues about ten instructions per member (id
// read-out, address, load, addition), and a wave issues at most one
// instruction every four cycles; split this way the chain costs a shared-
// memory read and an addition per member, while the gathers of the next
// batches run on the other waves.  The rows are the FP64 copy of y (row
// stride dim).  Batches of CP_B members pass through a two-slot ring in
// shared memory; step u stores batch u into the ring, requests the rows of
// batch u + CP_S (each gathering wave keeps CP_S batches in flight in
// registers) and adds batch u - 1; a barrier closes every step.
//
// Member ids reach the gathering waves through shared memory too, in chunks
// of CP_CH batches: wave 0 stores chunk c one step before its first batch is
// requested and then loads chunk c + 1 into registers, where it has CP_CH
// steps to arrive.  A wave's vector loads complete in issue order, so an id
// load among a gathering wave's row loads would make every row load issued
// before it complete first and cap the rows in flight; this way the
// gathering waves load rows only.  Positions past the last member are
// clamped to it and never stored.
// s_waitcnt immediate (gfx9 layout) for vmcnt(0) with expcnt and lgkmcnt left free
constexpr int KM_WAIT_VM0 = (0x7 << 4) | (0xF << 8);
constexpr int CP_M = 15;                   // members per gathering wave and batch
constexpr int CP_S = 4;                    // batches in flight per gathering wave
constexpr int CP_CH = 16;                  // batches per id chunk
static_assert(CP_S * CP_M <= 63, "rows in flight beyond the vector load counter");
static_assert(CP_CH > CP_S, "chunk 0 holds the ids the gathering waves start with");
// PW gathering waves: 3 (three workgroups per CU, for the first Lloyd
// iterations, when every cluster is summed again and the launch streams the
// whole row copy), or 7 (one workgroup per CU with 420 rows in flight, for the
// late iterations, when a few long chains on a few CUs set the time)
template <int PW>
struct CentroidShape {
    static constexpr int B = PW * CP_M;            // members per batch
    static constexpr int CI = CP_CH * B;           // ids per chunk
    static constexpr int NL = (CI + 63) / 64;      // id loads per lane and chunk
    static constexpr int NT = 64 * (PW + 1);
};
// Workgroup order of a centroid launch: the (restart, cluster) pairs that
// need an update, longest member list first, then the others (which exit at
// once).  The longest chains set a launch's length, and workgroups start in
// index order as slots free up, so the longest ones should start first
// (longest processing time first).  One workgroup buckets the pairs by the
// leading three bits of their member count (four buckets per power of two,
// so a bucket's counts lie within a factor of 1.25) and lays the buckets out
// in descending order; within a bucket the order is that of the atomic
// position grabs.  The order only decides when a workgroup starts: every
// cluster's sum is the same whatever it is.
constexpr int CO_TH = 1024;
constexpr int CO_NB = 4 * 64;
__device__ inline int centroid_bucket(int64_t c) {
    if (c <= 0) return 0;
    const int e = 63 - __clzll((unsigned long long)c);              // leading one
    const int sub = e >= 2 ? (int)((c >> (e - 2)) & 3) : (int)((c << (2 - e)) & 3);
    return 4 * e + sub + 1 < CO_NB ? 4 * e + sub + 1 : CO_NB - 1;
}
__global__ void __launch_bounds__(CO_TH)
k_centroid_order(int K, int RK, const int* __restrict__ active, const int* __restrict__ dirty,
                 const int64_t* __restrict__ seg, int* __restrict__ order) {
    __shared__ int hist[CO_NB], start[CO_NB];
    for (int b = threadIdx.x; b < CO_NB; b += CO_TH) hist[b] = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < RK; j += CO_TH) {
        const int64_t c = km_needs_update(j, K, active, dirty, seg) ? seg[2 * j + 1] - seg[2 * j] : 0;
        atomicAdd(&hist[centroid_bucket(c)], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int b = CO_NB - 1; b >= 0; --b) {
            start[b] = acc;
            acc += hist[b];
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < RK; j += CO_TH) {
        const int64_t c = km_needs_update(j, K, active, dirty, seg) ? seg[2 * j + 1] - seg[2 * j] : 0;
        order[atomicAdd(&start[centroid_bucket(c)], 1)] = j;
    }
}

template <int PW>
__global__ void __launch_bounds__(CentroidShape<PW>::NT)
k_centroid_sum(int dim, int K, int R, const double* __restrict__ Y,
               const uint32_t* __restrict__ members, const int64_t* __restrict__ seg,
               const int* __restrict__ active, const int* __restrict__ dirty,
               const int* __restrict__ order, double* __restrict__ C) {
    constexpr int CP_B = CentroidShape<PW>::B;
    constexpr int CP_CI = CentroidShape<PW>::CI;
    constexpr int CP_NL = CentroidShape<PW>::NL;
    __shared__ double ring[2][CP_B][64];
    __shared__ int idbuf[2][CP_CI];
    const int wps = (dim + 63) / 64;
    const int64_t slot = blockIdx.x / wps;
    if (slot >= (int64_t)R * K) return;
    const int64_t rj = order[slot];
    if (!km_needs_update(rj, K, active, dirty, seg)) return;
    const int wave = uniform((int)(threadIdx.x >> 6)), lane = (int)(threadIdx.x & 63);
    const int d = (int)(blockIdx.x - slot * wps) * 64 + lane;
    const int dd = d < dim ? d : dim - 1;
    const int64_t lo = seg[2 * rj];
    const int64_t cnt = seg[2 * rj + 1] - lo;       // >= 1
    const uint32_t* mem = members + lo;
    const double* Yd = Y + dd;
    const int64_t nb = (cnt + CP_B - 1) / CP_B;
    const int pw = wave - 1;                         // gathering wave index
    // the ids of gathering wave pw's share of batch b, from the chunk buffer
    auto ids = [&](int64_t b, int* out) {
        const int* ir = &idbuf[(b / CP_CH) & 1][(int)(b % CP_CH) * CP_B + pw * CP_M];
#pragma unroll
        for (int q = 0; q < CP_M; ++q) out[q] = uniform(ir[q]);
    };
    auto rows = [&](const int* id, double* v) {
#pragma unroll
        for (int q = 0; q < CP_M; ++q) v[q] = Yd[(int64_t)(uint32_t)id[q] * dim];
    };
    auto chunk_load = [&](int64_t c, int* r) {
#pragma unroll
        for (int l = 0; l < CP_NL; ++l)
            r[l] = (int)mem[min<int64_t>(c * CP_CI + l * 64 + lane, cnt - 1)];
    };
    auto chunk_store = [&](int64_t c, const int* r) {
#pragma unroll
        for (int l = 0; l < CP_NL; ++l)
            if (l * 64 + lane < CP_CI) idbuf[c & 1][l * 64 + lane] = r[l];
    };
    // The two roles run separate loops with the same barrier per step, so the
    // compiler sees the gathering waves' loads as one uninterrupted stream and
    // waits only for the batch a step stores.  Both run whole groups of CP_S
    // steps (steps past nb store and add nothing), so the unrolled body has no
    // exits in it.
    if (wave > 0) {
        double v[CP_S][CP_M];
        __syncthreads();                             // chunk 0 published
        // steps -CP_S .. -1 only request the first batches (the pipeline fill
        // is the loop itself, so no loads are pending on entry)
        for (int64_t u0 = -CP_S; u0 <= nb; u0 += CP_S) {
#pragma unroll
            for (int j = 0; j < CP_S; ++j) {
                const int64_t u = u0 + j;            // store batch u, request batch u + CP_S
                if (u >= 0 && u < nb) {
#pragma unroll
                    for (int q = 0; q < CP_M; ++q) ring[u & 1][pw * CP_M + q][lane] = v[j][q];
                }
                int idc[CP_M];
                ids(u + CP_S, idc);
                rows(idc, v[j]);
                __syncthreads();
            }
        }
        // drain the requests past the last batch here: the compiler joins this
        // path with wave 0's before the exit, and loads it believes pending
        // there would add waits to wave 0's loop
        __builtin_amdgcn_s_waitcnt(KM_WAIT_VM0);
    } else {
        int idr[CP_NL];                              // the next chunk's ids, in flight
        chunk_load(0, idr);
        chunk_store(0, idr);
        chunk_load(1, idr);
        __syncthreads();
        double s = 0.0;
        for (int64_t u0 = -CP_S; u0 <= nb; u0 += CP_S) {
#pragma unroll
            for (int j = 0; j < CP_S; ++j) {
                const int64_t u = u0 + j;            // add batch u - 1
                if ((u + CP_S + 1) % CP_CH == 0) {   // chunk c is first requested at step u + 1
                    const int64_t c = (u + CP_S + 1) / CP_CH;
                    chunk_store(c, idr);
                    chunk_load(c + 1, idr);
                }
                if (u > 0 && u <= nb) {
                    const int64_t b = u - 1;
                    const double* rb = &ring[b & 1][0][lane];
                    if (b + 1 < nb) {
                        // a full batch, CP_M reads issued ahead of their additions
#pragma unroll
                        for (int g = 0; g < PW; ++g) {
                            double x[CP_M];
#pragma unroll
                            for (int q = 0; q < CP_M; ++q) x[q] = rb[(g * CP_M + q) * 64];
#pragma unroll
                            for (int q = 0; q < CP_M; ++q) s += x[q];
                        }
                    } else {
                        const int m = (int)(cnt - b * CP_B);
#pragma unroll
                        for (int q = 0; q < CP_B; ++q)
                            if (q < m) s += rb[q * 64];
                    }
                }
                __syncthreads();
            }
        }
        if (d < dim) C[rj * dim + d] = s / (double)cnt;
    }
}

// exact squared distance of every point to its assigned centre, reading the
// transposed centroid table Ct[r][d][Kpad] (a dimension's centres share a few
// cache lines, so the per-lane gathers by label stay in L1)
template <int WB, class TT>
__global__ void __launch_bounds__(TH)
k_final_d2(int64_t n, int dim, int K, int Kpad, int R, const TT* __restrict__ Yt,
           const YDiv* __restrict__ dv, const double* __restrict__ Ct,
           const int32_t* __restrict__ lab, double* __restrict__ D2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const YDiv dvi = ydiv_of<TT>(dv, i);
    // one pass over the point's coordinates serves up to WB restarts; lanes of
    // restarts >= R repeat restart R - 1 and are not stored (no predicates)
    for (int r0 = 0; r0 < R; r0 += WB) {
        const double* c[WB];
        double acc[WB];
#pragma unroll
        for (int q = 0; q < WB; ++q) {
            const int r = min(r0 + q, R - 1);
            c[q] = Ct + (int64_t)r * dim * Kpad + lab[(int64_t)r * n + i];
            acc[q] = 0.0;
        }
        for (int d = 0; d < dim; ++d) {
            const double y = ycoord(Yt[(int64_t)d * n + i], dvi);
#pragma unroll
            for (int q = 0; q < WB; ++q) {
                const double diff = y - c[q][(int64_t)d * Kpad];
                acc[q] = fma(diff, diff, acc[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < WB; ++q)
            if (r0 + q < R) D2[(int64_t)(r0 + q) * n + i] = acc[q];
    }
}

// integer inertia per restart: block sums (exact) then one atomic per block
// of INERTIA_PPT * TH points
constexpr int INERTIA_PPT = 16;
__global__ void __launch_bounds__(TH)
k_inertia(int64_t n, const double* __restrict__ D2, int shift, unsigned long long* __restrict__ q) {
    __shared__ unsigned long long sm[TH];
    const int r = blockIdx.y;
    unsigned long long v = 0;
    for (int u = 0; u < INERTIA_PPT; ++u) {
        const int64_t i = ((int64_t)blockIdx.x * INERTIA_PPT + u) * TH + threadIdx.x;
        if (i < n) v += (unsigned long long)floor(ldexp(D2[(int64_t)r * n + i], shift));
    }
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int o = TH / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&q[r], sm[0]);
}

// FP64 inertia of one restart: fixed-shape tree (block sums in order)
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

__global__ void k_zero_i64(int64_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_zero_i32(int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_fill_i32(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// centres per wave and pass: the smallest supported width covering K in one
// pass (four waves), else 64 with several passes; Kpad = passes * 4 * JB
int assign_width(int K) {
    const int need = (K + 3) / 4;
    const int widths[] = {2, 8, 16, 24, 32, 40, 48, 56, 64};
    for (int wdt : widths)
        if (wdt >= need) return wdt;
    return 64;
}
int assign_kpad(int K) {
    const int jb = assign_width(K);
    return (int)ceil_div(K, 4 * jb) * 4 * jb;
}

struct KmWs {
    double *Y, *D2, *C, *Cold, *Ct, *delta, *dinfo, *part, *inertia;
    float *ub, *lb;      // Hamerly bounds, stored in FP32 rounded outward
    uint64_t *tsum, *lhist, *lscan_tmp;
    uint32_t *vals, *pts, *fl;
    int32_t* lab;
    int *changed, *active, *cnt, *fcnt, *status, *dirty, *order;
    int64_t* seg;
    double *ccur, *hsv;
    float* secf;
    uint16_t* hsi;
    void* Yt;        // dimension-major copy: FP64 y, or FP32 x with the divisors dv
    YDiv* dv;
    bool yt32;       // FP32 input: Ysrc is the caller's X (row stride ldy), Yt and dv as above
    const void* Ysrc;
    int64_t ldy;
    int Rpad;
    unsigned long long *m2, *q;
};

size_t carve_km(Carver& c, int64_t n, int dim, int K, int R, KmWs& w) {
    const int64_t nr = n * R;
    const size_t cent = (size_t)R * K * dim;
    w.Y = c.take<double>((size_t)n * dim);
    w.Yt = c.take<double>((size_t)n * dim);
    w.dv = c.take<YDiv>((size_t)n);
    w.D2 = c.take<double>(nr);
    w.C = c.take<double>(cent);
    w.Cold = c.take<double>(cent);
    w.Ct = c.take<double>((size_t)R * assign_kpad(K) * dim);
    w.ub = c.take<float>(nr);
    w.lb = c.take<float>(nr);
    w.delta = c.take<double>((size_t)R * K);
    w.dinfo = c.take<double>(3 * (size_t)R);
    w.part = c.take<double>(ceil_div(n, TH * 16) + 1);
    w.inertia = c.take<double>(1);
    w.tsum = c.take<uint64_t>((size_t)R * ceil_div(n, SEED_TILE));
    w.lhist = c.take<uint64_t>((size_t)R * K * ceil_div(n, LS_TILE));
    w.lscan_tmp = c.take<uint64_t>(scan_u64_batched_tmp_elems(K * ceil_div(n, LS_TILE), R));
    w.vals = c.take<uint32_t>(nr);
    w.pts = c.take<uint32_t>(nr);
    w.fl = c.take<uint32_t>(nr);              // full-scan lists
    w.lab = c.take<int32_t>(nr);
    w.changed = c.take<int>(R);
    w.active = c.take<int>(R);
    w.cnt = c.take<int>(R);
    w.fcnt = c.take<int>(R);
    w.status = c.take<int>(1);
    w.dirty = c.take<int>((size_t)R * K);
    w.order = c.take<int>((size_t)R * K);
    w.seg = c.take<int64_t>(2 * (size_t)R * K);
    w.Rpad = seed_stride(R);
    w.ccur = c.take<double>((size_t)w.Rpad * dim);
    w.hsv = c.take<double>((size_t)R * K * K);
    w.secf = c.take<float>((size_t)nr);
    w.hsi = c.take<uint16_t>((size_t)R * K * K);
    w.m2 = c.take<unsigned long long>(1);
    w.q = c.take<unsigned long long>(R);
    return c.size();
}

sc_status km_validate(sc_ctx* ctx, int64_t n, int dim, const sc_kmeans_opts* o) {
    if (!o) return sc_fail(ctx, SC_E_INVAL, "kmeans: opts is NULL");
    if (n <= 0 || dim <= 0) return sc_fail(ctx, SC_E_INVAL, "kmeans: need n > 0 and dim > 0");
    if (o->n_clusters < 1 || o->n_clusters > n || o->n_clusters > 1024)
        return sc_fail(ctx, SC_E_INVAL, "kmeans: need 1 <= K <= min(n, 1024)");
    if (o->restarts < 1 || o->max_iter < 0)
        return sc_fail(ctx, SC_E_INVAL, "kmeans: need restarts >= 1 and max_iter >= 0");
    if (o->scan != SC_KM_SCAN_AUTO && o->scan != SC_KM_SCAN_PRUNED && o->scan != SC_KM_SCAN_FULL)
        return sc_fail(ctx, SC_E_INVAL, "kmeans: unknown scan mode %d", o->scan);
    if ((int64_t)o->restarts * n >= (int64_t(1) << 31))
        return sc_fail(ctx, SC_E_UNSUPPORTED, "kmeans: restarts * n >= 2^31");
    return SC_OK;
}

// full scans of the lists (list, lcnt); max_cnt bounds every restart's count
template <int JB>
void launch_assign(sc_ctx* ctx, int64_t n, int dim, int K, int R, const KmWs& w, int first,
                   const uint32_t* list, const int* lcnt, int64_t max_cnt) {
    dim3 grid((unsigned)ceil_div(max_cnt, 64), (unsigned)R);
    if (w.yt32)
        hipLaunchKernelGGL((k_assign_list<JB, float>), grid, dim3(TH), 0, ctx->stream, n, dim, K,
                           assign_kpad(K), static_cast<const float*>(w.Ysrc), w.ldy, w.dv, w.Ct,
                           list, lcnt, w.active, w.lab, w.ub, w.lb, w.changed, w.dirty, first);
    else
        hipLaunchKernelGGL((k_assign_list<JB, double>), grid, dim3(TH), 0, ctx->stream, n, dim, K,
                           assign_kpad(K), static_cast<const double*>(w.Ysrc), w.ldy, w.dv, w.Ct,
                           list, lcnt, w.active, w.lab, w.ub, w.lb, w.changed, w.dirty, first);
}

template <int WB>
void seed_d2_go(sc_ctx* ctx, int64_t n, int dim, int R, int Rpad, int j, const KmWs& w, int shift) {
    if (w.yt32)
        hipLaunchKernelGGL((k_seed_d2<WB, float>), dim3(ceil_div(n, TH)), dim3(TH), 0, ctx->stream, n,
                           dim, R, Rpad, j, static_cast<const float*>(w.Yt), w.dv, w.ccur, w.D2,
                           w.tsum, shift, w.lab, w.secf);
    else
        hipLaunchKernelGGL((k_seed_d2<WB, double>), dim3(ceil_div(n, TH)), dim3(TH), 0, ctx->stream,
                           n, dim, R, Rpad, j, static_cast<const double*>(w.Yt), w.dv, w.ccur, w.D2,
                           w.tsum, shift, w.lab, w.secf);
}

template <int WB>
void final_d2_go(sc_ctx* ctx, int64_t n, int dim, int K, int Kpad, int R, const KmWs& w) {
    if (w.yt32)
        hipLaunchKernelGGL((k_final_d2<WB, float>), dim3(ceil_div(n, TH)), dim3(TH), 0, ctx->stream,
                           n, dim, K, Kpad, R, static_cast<const float*>(w.Yt), w.dv, w.Ct, w.lab,
                           w.D2);
    else
        hipLaunchKernelGGL((k_final_d2<WB, double>), dim3(ceil_div(n, TH)), dim3(TH), 0, ctx->stream,
                           n, dim, K, Kpad, R, static_cast<const double*>(w.Yt), w.dv, w.Ct, w.lab,
                           w.D2);
}

void seed_d2(sc_ctx* ctx, int64_t n, int dim, int R, int Rpad, int j, const KmWs& w, int shift) {
    switch (seed_width(R)) {
    case 1: seed_d2_go<1>(ctx, n, dim, R, Rpad, j, w, shift); break;
    case 2: seed_d2_go<2>(ctx, n, dim, R, Rpad, j, w, shift); break;
    case 4: seed_d2_go<4>(ctx, n, dim, R, Rpad, j, w, shift); break;
    case 8: seed_d2_go<8>(ctx, n, dim, R, Rpad, j, w, shift); break;
    case 10: seed_d2_go<10>(ctx, n, dim, R, Rpad, j, w, shift); break;
    case 12: seed_d2_go<12>(ctx, n, dim, R, Rpad, j, w, shift); break;
    default: seed_d2_go<RB>(ctx, n, dim, R, Rpad, j, w, shift); break;
    }
}

template <int JB>
void launch_pruned(sc_ctx* ctx, int64_t n, int dim, int K, int R, const KmWs& w,
                   const uint32_t* list, int max_cnt) {
    dim3 grid((unsigned)ceil_div(max_cnt, TH), (unsigned)R);
    if (w.yt32)
        hipLaunchKernelGGL((k_assign_pruned<JB, float>), grid, dim3(TH), 0, ctx->stream, n, dim, K,
                           assign_kpad(K), static_cast<const float*>(w.Ysrc), w.ldy, w.dv, w.Ct,
                           w.C, w.hsv, w.hsi, list, w.cnt, w.active, w.lab, w.ub, w.lb, w.changed,
                           w.dirty, w.fl, w.fcnt);
    else
        hipLaunchKernelGGL((k_assign_pruned<JB, double>), grid, dim3(TH), 0, ctx->stream, n, dim, K,
                           assign_kpad(K), static_cast<const double*>(w.Ysrc), w.ldy, w.dv, w.Ct,
                           w.C, w.hsv, w.hsi, list, w.cnt, w.active, w.lab, w.ub, w.lb, w.changed,
                           w.dirty, w.fl, w.fcnt);
}

void assign(sc_ctx* ctx, int64_t n, int dim, int K, int R, const KmWs& w, int first,
            const uint32_t* list, const int* lcnt, int64_t max_cnt) {
    switch (assign_width(K)) {
        case 2: launch_assign<2>(ctx, n, dim, K, R, w, first, list, lcnt, max_cnt); break;
        case 8: launch_assign<8>(ctx, n, dim, K, R, w, first, list, lcnt, max_cnt); break;
        case 16: launch_assign<16>(ctx, n, dim, K, R, w, first, list, lcnt, max_cnt); break;
        case 24: launch_assign<24>(ctx, n, dim, K, R, w, first, list, lcnt, max_cnt); break;
        case 32: launch_assign<32>(ctx, n, dim, K, R, w, first, list, lcnt, max_cnt); break;
        case 40: launch_assign<40>(ctx, n, dim, K, R, w, first, list, lcnt, max_cnt); break;
        case 48: launch_assign<48>(ctx, n, dim, K, R, w, first, list, lcnt, max_cnt); break;
        case 56: launch_assign<56>(ctx, n, dim, K, R, w, first, list, lcnt, max_cnt); break;
        default: launch_assign<64>(ctx, n, dim, K, R, w, first, list, lcnt, max_cnt); break;
    }
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

// Fixed device scratch of the entry point for callers that cannot allocate:
// one copy per GPU, held until the process ends.  Host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
constexpr size_t KM_STATIC_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[KM_STATIC_BYTES];

namespace {

// Host arrays of one entry per restart: inline storage up to KM_HOST_INLINE
// restarts, heap beyond (only the entry point with a caller workspace admits
// more restarts).
constexpr int KM_HOST_INLINE = 64;
template <class T>
struct PerRestart {
    T inl[KM_HOST_INLINE];
    std::vector<T> heap;
    T* p;
    PerRestart(int R, T v) {
        if (R <= KM_HOST_INLINE) {
            p = inl;
        } else {
            heap.resize(R);
            p = heap.data();
        }
        for (int r = 0; r < R; ++r) p[r] = v;
    }
    T& operator[](int r) { return p[r]; }
    T* data() { return p; }
};

sc_status kmeans_run(sc_ctx* ctx, int64_t n, int dim, const void* X, int64_t ldx,
                     const sc_kmeans_opts* opts, const uint64_t* draws,
                     const double* init_centroids, int32_t* labels, double* centroids,
                     double* inertia, uint64_t* inertia_q, int* best_restart,
                     int* lloyd_iterations, void* ws, size_t ws_bytes, bool timed) {
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
    const dim3 gnr((unsigned)ceil_div(nr, TH));
    const size_t cent_bytes = (size_t)R * K * dim * sizeof(double);
    ProfScope ps(ctx, timed ? SC_KIND_KMEANS : -1);

    SC_CHECK_HIP(ctx, hipMemsetAsync(w.m2, 0, sizeof(unsigned long long), st));
    SC_CHECK_HIP(ctx, hipMemsetAsync(w.status, 0, sizeof(int), st));
    w.yt32 = opts->x_fp32 != 0;
    w.Ysrc = w.yt32 ? X : static_cast<const void*>(w.Y);
    w.ldy = w.yt32 ? ldx : dim;
    if (opts->x_fp32)
        hipLaunchKernelGGL((k_rownorm<float>), dim3(ceil_div(n, TH)), dim3(TH), 0, st, n, dim,
                           static_cast<const float*>(X), ldx, opts->normalize_rows, w.Y,
                           static_cast<float*>(w.Yt), w.dv, w.m2, w.status);
    else
        hipLaunchKernelGGL((k_rownorm<double>), dim3(ceil_div(n, TH)), dim3(TH), 0, st, n, dim,
                           static_cast<const double*>(X), ldx, opts->normalize_rows, w.Y,
                           static_cast<double*>(w.Yt), nullptr, w.m2, w.status);
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

    PerRestart<int> act_h(R, 1);
    SC_CHECK_HIP(ctx, hipMemcpyAsync(w.active, act_h.data(), R * sizeof(int), hipMemcpyHostToDevice, st));
    // seeding
    if (init_centroids) {
        SC_CHECK_HIP(ctx, hipMemcpyAsync(w.C, init_centroids, cent_bytes, hipMemcpyDeviceToDevice, st));
    } else {
        // this round's centres of restarts >= R stay 0.0
        hipLaunchKernelGGL(k_zero_i64, dim3(ceil_div((int64_t)w.Rpad * dim, TH)), dim3(TH), 0, st,
                           reinterpret_cast<int64_t*>(w.ccur), (int64_t)w.Rpad * dim);
        for (int j = 0; j < K; ++j) {
            if (w.yt32)
                hipLaunchKernelGGL(k_seed_pick<float>, dim3(R), dim3(PICK_NT), 0, st, n, dim, K, j,
                                   w.Rpad, static_cast<const float*>(w.Ysrc), w.ldy, w.dv,
                                   draws, w.tsum, w.D2, shift, w.C, w.ccur);
            else
                hipLaunchKernelGGL(k_seed_pick<double>, dim3(R), dim3(PICK_NT), 0, st, n, dim, K, j,
                                   w.Rpad, static_cast<const double*>(w.Ysrc), w.ldy, w.dv,
                                   draws, w.tsum, w.D2, shift, w.C, w.ccur);
            SC_CHECK_LAUNCH(ctx);
            // distances to centre j (also after the last one: they complete the
            // first assignment)
            seed_d2(ctx, n, dim, R, w.Rpad, j, w, shift);
            SC_CHECK_LAUNCH(ctx);
        }
    }
    const dim3 gcent((unsigned)ceil_div((int64_t)R * K * dim, TH));
    const int Kpad = assign_kpad(K);
    const dim3 gcentp((unsigned)ceil_div((int64_t)R * Kpad * dim, TH));
    // first assignment: every point of every restart (after a seeding, the
    // seeding rounds already hold the exact least and second least distances)
    hipLaunchKernelGGL(k_transpose_centroids, gcentp, dim3(TH), 0, st, R, K, Kpad, dim, w.C, w.Ct);
    if (init_centroids) {
        hipLaunchKernelGGL(k_fill_lists, gnr, dim3(TH), 0, st, n, R, w.pts, w.cnt);
        SC_CHECK_LAUNCH(ctx);
        assign(ctx, n, dim, K, R, w, 1, w.pts, w.cnt, n);
    } else {
        hipLaunchKernelGGL(k_first_bounds, gnr, dim3(TH), 0, st, nr, w.D2, w.ub, w.secf, w.lb);
    }
    hipLaunchKernelGGL(k_fill_i32, dim3(ceil_div((int64_t)R * K, TH)), dim3(TH), 0, st, w.dirty,
                       R * K, 1);
    SC_CHECK_LAUNCH(ctx);
    const int bits = ceil_log2_u64((uint64_t)K);
    int n_active = R;
    int iterations = 0;
    PerRestart<int> ch(R, 0), cnt_h(R, 0);
    for (int it = 1; it <= opts->max_iter && n_active > 0; ++it) {
        iterations = it;
        // centroid update from the stable member lists
        SC_CHECK_HIP(ctx, hipMemcpyAsync(w.Cold, w.C, cent_bytes, hipMemcpyDeviceToDevice, st));
        {
            // member lists sorted by label, and every label's segment
            const int lt = (int)ceil_div(n, LS_TILE);
            const dim3 glt((unsigned)lt, (unsigned)R);
            hipLaunchKernelGGL(k_lab_hist, glt, dim3(TH), 0, st, n, K, w.active, w.lab, nullptr, nullptr,
                               w.lhist, lt);
            SC_CHECK_LAUNCH(ctx);
            SC_TRY(scan_u64_batched_exclusive(ctx, w.lhist, w.lhist, (int64_t)K * lt, R, w.lscan_tmp));
            hipLaunchKernelGGL(k_lab_segments, dim3((unsigned)ceil_div((int64_t)R * K, TH)), dim3(TH), 0,
                               st, n, K, R, w.active, w.lhist, lt, w.seg);
            hipLaunchKernelGGL(k_lab_scatter, glt, dim3(TH), 0, st, n, K, bits, w.active, w.lab,
                               nullptr, nullptr, w.lhist, lt, w.vals);
            SC_CHECK_LAUNCH(ctx);
        }
        {
            // few clusters changed in the last assignment: the wide variant
            // (one workgroup per CU, more rows in flight per chain)
            const unsigned grid = (unsigned)((int64_t)R * K * ceil_div(dim, 64));
            int64_t moved = 0;
            for (int r = 0; r < R; ++r)
                if (act_h[r]) moved += ch[r];
            const bool wide = it > 1 && 2 * moved * ceil_div(dim, 64) <= ctx->num_cu;
            hipLaunchKernelGGL(k_centroid_order, dim3(1), dim3(CO_TH), 0, st, K, R * K, w.active,
                               w.dirty, w.seg, w.order);
            if (wide)
                hipLaunchKernelGGL(k_centroid_sum<7>, dim3(grid), dim3(CentroidShape<7>::NT), 0, st,
                                   dim, K, R, w.Y, w.vals, w.seg, w.active, w.dirty, w.order, w.C);
            else
                hipLaunchKernelGGL(k_centroid_sum<3>, dim3(grid), dim3(CentroidShape<3>::NT), 0, st,
                                   dim, K, R, w.Y, w.vals, w.seg, w.active, w.dirty, w.order, w.C);
        }
        SC_CHECK_LAUNCH(ctx);
        hipLaunchKernelGGL(k_delta, dim3((unsigned)ceil_div((int64_t)R * K, TH / 64)), dim3(TH), 0, st, K,
                           R, dim, w.C, w.Cold, w.active, w.dirty, w.delta);
        hipLaunchKernelGGL(k_delta_max, dim3(R), dim3(64), 0, st, K, w.active, w.delta, w.dinfo);
        hipLaunchKernelGGL(k_zero_i32, dim3(ceil_div((int64_t)R * K, TH)), dim3(TH), 0, st, w.dirty,
                           R * K);
        hipLaunchKernelGGL(k_transpose_centroids, gcentp, dim3(TH), 0, st, R, K, Kpad, dim, w.C,
                           w.Ct);
        SC_CHECK_LAUNCH(ctx);
        // points whose assignment may change, then their scans
        hipLaunchKernelGGL(k_zero_i32, dim3(ceil_div(R, TH)), dim3(TH), 0, st, w.cnt, R);
        hipLaunchKernelGGL(k_zero_i32, dim3(ceil_div(R, TH)), dim3(TH), 0, st, w.changed, R);
        hipLaunchKernelGGL(k_zero_i32, dim3(ceil_div(R, TH)), dim3(TH), 0, st, w.fcnt, R);
        hipLaunchKernelGGL(k_bounds, dim3((unsigned)ceil_div(n, TH * PPT), (unsigned)R), dim3(TH), 0,
                           st, n, K, w.lab, w.ub, w.lb, w.delta, w.dinfo, w.active, w.pts, w.cnt);
        SC_CHECK_LAUNCH(ctx);
        SC_CHECK_HIP(ctx, hipMemcpyAsync(cnt_h.data(), w.cnt, R * sizeof(int), hipMemcpyDeviceToHost, st));
        SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
        int max_cnt = 0;
        int64_t total = 0;
        for (int r = 0; r < R; ++r)
            if (act_h[r]) {
                max_cnt = std::max(max_cnt, cnt_h[r]);
                total += cnt_h[r];
            }
        const bool prune = opts->scan == SC_KM_SCAN_PRUNED ||
                           (opts->scan == SC_KM_SCAN_AUTO && total * K >= PR_WORK_MIN);
        if (prune) {
            hipLaunchKernelGGL(k_half_sep, dim3((unsigned)K, (unsigned)R), dim3(TH), 0, st, K, Kpad,
                               dim, w.Ct, w.active, w.hsv, w.hsi);
            // long lists: ordered by current label (stable: ascending point
            // within a label) into vals, pruned scans, then full scans of the
            // points those cannot settle
            {
                const int lt = (int)ceil_div(max_cnt, LS_TILE);
                const dim3 glt((unsigned)lt, (unsigned)R);
                hipLaunchKernelGGL(k_lab_hist, glt, dim3(TH), 0, st, n, K, w.active, w.lab, w.pts,
                                   w.cnt, w.lhist, lt);
                SC_CHECK_LAUNCH(ctx);
                SC_TRY(scan_u64_batched_exclusive(ctx, w.lhist, w.lhist, (int64_t)K * lt, R,
                                                  w.lscan_tmp));
                hipLaunchKernelGGL(k_lab_scatter, glt, dim3(TH), 0, st, n, K, bits, w.active, w.lab,
                                   w.pts, w.cnt, w.lhist, lt, w.vals);
                SC_CHECK_LAUNCH(ctx);
            }
            launch_pruned<8>(ctx, n, dim, K, R, w, w.vals, max_cnt);
            SC_CHECK_LAUNCH(ctx);
            assign(ctx, n, dim, K, R, w, 0, w.fl, w.fcnt, max_cnt);
            SC_CHECK_LAUNCH(ctx);
        } else if (max_cnt > 0) {
            // short lists: the fixed latency of the pruned path outweighs its saving
            assign(ctx, n, dim, K, R, w, 0, w.pts, w.cnt, max_cnt);
            SC_CHECK_LAUNCH(ctx);
        }
        SC_CHECK_HIP(ctx, hipMemcpyAsync(ch.data(), w.changed, R * sizeof(int), hipMemcpyDeviceToHost, st));
        SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
        bool any_stop = false;
        for (int r = 0; r < R; ++r)
            if (act_h[r] && ch[r] == 0) {
                act_h[r] = 0;
                --n_active;
                any_stop = true;
            }
        if (any_stop)
            SC_CHECK_HIP(ctx, hipMemcpyAsync(w.active, act_h.data(), R * sizeof(int),
                                             hipMemcpyHostToDevice, st));
    }
    // exact distances to the final centres, integer inertia, best restart
    if (R <= 4) final_d2_go<4>(ctx, n, dim, K, Kpad, R, w);
    else if (R <= 10) final_d2_go<10>(ctx, n, dim, K, Kpad, R, w);
    else final_d2_go<16>(ctx, n, dim, K, Kpad, R, w);
    SC_CHECK_HIP(ctx, hipMemsetAsync(w.q, 0, R * sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_inertia, dim3((unsigned)ceil_div(n, TH * INERTIA_PPT), (unsigned)R), dim3(TH), 0,
                       st, n,
                       w.D2, shift, w.q);
    SC_CHECK_LAUNCH(ctx);
    PerRestart<unsigned long long> qh(R, 0ull);
    SC_CHECK_HIP(ctx, hipMemcpyAsync(qh.data(), w.q, R * sizeof(unsigned long long),
                                     hipMemcpyDeviceToHost, st));
    SC_CHECK_HIP(ctx, hipStreamSynchronize(st));
    int best = 0;
    for (int r = 1; r < R; ++r)
        if (qh[r] < qh[best]) best = r;
    SC_CHECK_HIP(ctx, hipMemcpyAsync(labels, w.lab + (int64_t)best * n, n * sizeof(int32_t),
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
    if (lloyd_iterations) *lloyd_iterations = iterations;
    return SC_OK;
}

constexpr int KM_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[KM_MAX_DEVICES] = {};

// Address of this device's scratch (the device must be current), looked up
// once per device.
sc_status static_scratch(sc_ctx* ctx, void** out) {
    if (ctx->device < 0 || ctx->device >= KM_MAX_DEVICES)
        return sc_fail(ctx, SC_E_UNSUPPORTED, "kmeans_static: device %d", ctx->device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[ctx->device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return sc_fail(ctx, SC_E_HIP, "kmeans_static: hipGetSymbolAddress failed: %s",
                           hipGetErrorString(e));
        g_scratch_ptr[ctx->device] = p;
    }
    *out = g_scratch_ptr[ctx->device];
    return SC_OK;
}

}  // namespace

extern "C" sc_status sc_kmeans_assign(sc_ctx* ctx, int64_t n, int dim, const void* X,
                                      int64_t ldx, const sc_kmeans_opts* opts,
                                      const uint64_t* draws, const double* init_centroids,
                                      int32_t* labels, double* centroids, double* inertia,
                                      uint64_t* inertia_q, int* best_restart,
                                      int* lloyd_iterations, void* ws, size_t ws_bytes) {
    return kmeans_run(ctx, n, dim, X, ldx, opts, draws, init_centroids, labels, centroids,
                      inertia, inertia_q, best_restart, lloyd_iterations, ws, ws_bytes, true);
}

extern "C" sc_status sc_kmeans_assign_static(sc_ctx* ctx, int64_t n, int dim, const void* X,
                                             int64_t ldx, const sc_kmeans_opts* opts,
                                             const uint64_t* draws,
                                             const double* init_centroids, int32_t* labels,
                                             double* centroids, double* inertia,
                                             uint64_t* inertia_q, int* best_restart,
                                             int* lloyd_iterations) {
    if (!ctx) return SC_E_INVAL;
    SC_TRY(km_validate(ctx, n, dim, opts));
    if (opts->restarts > KM_HOST_INLINE)
        return sc_fail(ctx, SC_E_UNSUPPORTED, "kmeans_static: restarts %d > %d",
                       opts->restarts, KM_HOST_INLINE);
    Carver c(nullptr);
    KmWs w;
    const size_t need = carve_km(c, n, dim, opts->n_clusters, opts->restarts, w);
    if (need > KM_STATIC_BYTES)
        return sc_fail(ctx, SC_E_UNSUPPORTED,
                       "kmeans_static: needs %zu bytes of scratch, the fixed scratch holds %zu",
                       need, KM_STATIC_BYTES);
    SC_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    void* ws = nullptr;
    SC_TRY(static_scratch(ctx, &ws));
    return kmeans_run(ctx, n, dim, X, ldx, opts, draws, init_centroids, labels, centroids,
                      inertia, inertia_q, best_restart, lloyd_iterations, ws, KM_STATIC_BYTES,
                      false);
}
