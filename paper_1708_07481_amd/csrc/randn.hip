// Random start blocks X0 on the device (Section III: the iteration starts
// from Gaussian, or uniform on [-1, 1], random vectors when no previous
// eigenvectors exist).
//
// The 64-bit words come from the counter-based Philox4x64-10 generator of
// Salmon, Moraes, Dror and Shaw ("Parallel random numbers: as easy as 1, 2,
// 3", SC'11): a 256-bit counter and a 128-bit key pass through ten rounds of
// two 64 x 64 -> 128-bit multiplications and a key schedule with Weyl
// increments.  Word t of the stream keyed (seed, stream) is word t mod 4 of
// the generator applied to counter t / 4 + 1 (the counter is advanced before
// each block, so the stream is the same as a sequential generator started
// from counter 0).  One thread computes one block of four words, so the
// result does not depend on the launch shape.
//
// Element e = row * cols + col of the block takes:
//   raw      word e;
//   uniform  (word e >> 11) * 2^-52 - 1, an exact double in [-1, 1);
//   normal   Box-Muller on the word pair (2p, 2p + 1), p = e / 2:
//            u1 = ((w_2p >> 11) + 1) 2^-53 in (0, 1], u2 = (w_2p+1 >> 11) 2^-53,
//            r = sqrt(-2 ln u1), z = r cos(2 pi u2) (even e) or r sin(2 pi u2)
//            (odd e).
// FP32 output rounds the double to nearest.
#include "sc_internal.h"

namespace {

constexpr uint64_t PH_M0 = 0xD2E7470EE14C6C93ull;   // round multipliers
constexpr uint64_t PH_M1 = 0xCA5A826395121157ull;
constexpr uint64_t PH_W0 = 0x9E3779B97F4A7C15ull;   // key increments (golden ratio, sqrt(3) - 1)
constexpr uint64_t PH_W1 = 0xBB67AE8584CAA73Bull;
constexpr int RN_NT = 256;

struct Words4 {
    uint64_t v[4];
};

__device__ inline Words4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                       uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t hi0 = __umul64hi(PH_M0, c0), lo0 = PH_M0 * c0;
        const uint64_t hi1 = __umul64hi(PH_M1, c2), lo1 = PH_M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += PH_W0;
        k1 += PH_W1;
    }
    return Words4{{c0, c1, c2, c3}};
}

template <class T>
__device__ inline void put(T* out, int64_t ld, int cols, int64_t e, double v) {
    const int64_t r = e / cols;
    const int c = (int)(e - r * cols);
    out[r * ld + c] = (T)v;
}

// dist: 0 normal, 1 uniform on [-1, 1), 2 raw words (T = uint64_t)
template <class T, int DIST>
__global__ void __launch_bounds__(RN_NT)
k_randn(int64_t rows, int cols, int64_t ld, uint64_t k0, uint64_t k1, T* __restrict__ out) {
    const int64_t total = rows * (int64_t)cols;
    const int64_t b = (int64_t)blockIdx.x * RN_NT + threadIdx.x;     // block of four words
    const int64_t e0 = 4 * b;
    if (e0 >= total) return;
    // counter b + 1 as a 256-bit integer (b < 2^62: no carry into c1)
    const Words4 w = philox4x64_10((uint64_t)b + 1, 0, 0, 0, k0, k1);
    double v[4];
    if (DIST == 2) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (e0 + q < total) {
                const int64_t e = e0 + q;
                const int64_t r = e / cols;
                reinterpret_cast<uint64_t*>(out)[r * ld + (e - r * cols)] = w.v[q];
            }
        return;
    } else if (DIST == 1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (double)(w.v[q] >> 11) * 0x1p-52 - 1.0;
    } else {
        const double two_pi = 6.283185307179586;       // RN(2 pi)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double u1 = (double)((w.v[2 * h] >> 11) + 1) * 0x1p-53;
            const double u2 = (double)(w.v[2 * h + 1] >> 11) * 0x1p-53;
            const double r = sqrt(-2.0 * log(u1));
            const double a = two_pi * u2;
            v[2 * h] = r * cos(a);
            v[2 * h + 1] = r * sin(a);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (e0 + q < total) put(out, ld, cols, e0 + q, v[q]);
}

}  // namespace

extern "C" sc_status sc_randn(sc_ctx* ctx, int64_t rows, int cols, int64_t ld, uint64_t seed,
                              uint64_t stream, int dist, void* out, sc_precision prec) {
    if (!ctx) return SC_E_INVAL;
    if (rows < 0 || cols < 1 || ld < cols)
        return sc_fail(ctx, SC_E_INVAL, "randn: need rows >= 0, cols >= 1, ld >= cols");
    if (dist != SC_RAND_NORMAL && dist != SC_RAND_UNIFORM && dist != SC_RAND_RAW)
        return sc_fail(ctx, SC_E_INVAL, "randn: unknown distribution %d", dist);
    if (prec != SC_PREC_FP64 && prec != SC_PREC_FP32 && prec != SC_PREC_FP32_BF16GRAM)
        return sc_fail(ctx, SC_E_INVAL, "randn: unknown precision");
    if (rows * (int64_t)cols >= (int64_t(1) << 62))
        return sc_fail(ctx, SC_E_UNSUPPORTED, "randn: block too large");
    if (rows == 0) return SC_OK;
    if (!out) return sc_fail(ctx, SC_E_INVAL, "randn: out is NULL");
    SC_CHECK_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t blocks = ceil_div(rows * (int64_t)cols, 4);
    const dim3 grid((unsigned)ceil_div(blocks, RN_NT));
    hipStream_t st = ctx->stream;
    const bool f64 = prec == SC_PREC_FP64;
    if (dist == SC_RAND_RAW)
        hipLaunchKernelGGL((k_randn<uint64_t, 2>), grid, dim3(RN_NT), 0, st, rows, cols, ld, seed,
                           stream, static_cast<uint64_t*>(out));
    else if (dist == SC_RAND_UNIFORM && f64)
        hipLaunchKernelGGL((k_randn<double, 1>), grid, dim3(RN_NT), 0, st, rows, cols, ld, seed,
                           stream, static_cast<double*>(out));
    else if (dist == SC_RAND_UNIFORM)
        hipLaunchKernelGGL((k_randn<float, 1>), grid, dim3(RN_NT), 0, st, rows, cols, ld, seed,
                           stream, static_cast<float*>(out));
    else if (f64)
        hipLaunchKernelGGL((k_randn<double, 0>), grid, dim3(RN_NT), 0, st, rows, cols, ld, seed,
                           stream, static_cast<double*>(out));
    else
        hipLaunchKernelGGL((k_randn<float, 0>), grid, dim3(RN_NT), 0, st, rows, cols, ld, seed,
                           stream, static_cast<float*>(out));
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}
