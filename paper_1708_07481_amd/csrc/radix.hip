// Stable LSD radix sort of (uint64 key, uint32 value) pairs, 8-bit digits.
// Each pass: per-tile digit histograms, one device scan of the
// (digit-major, tile-minor) histogram, then every tile is sorted by the digit
// in LDS with four stable two-bit splits and scattered to its offsets.
#include "sc_internal.h"

namespace {

constexpr int TH = 256;
constexpr int ITEMS = 8;
constexpr int TILE = TH * ITEMS;
constexpr int NW = TH / 64;
constexpr int RADIX = 256;

// Exclusive scan over the workgroup of four 16-bit counters packed in a
// 64-bit word (a tile holds TILE < 2^15 keys, so no field overflows even with
// its digit base); *total = the block's sums.
static_assert(2 * TILE < 65536, "16-bit digit counters plus digit bases");
__device__ inline uint64_t block_excl_scan4(uint64_t v, uint64_t* total, uint64_t* wsum) {
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
        for (int w = 0; w < NW; ++w) {
            const uint64_t t = wsum[w];
            wsum[w] = acc;
            acc += t;
        }
        wsum[NW] = acc;
    }
    __syncthreads();
    const uint64_t r = x - v + wsum[wave];
    *total = wsum[NW];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(TH) k_digit_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                    int shift, uint64_t* __restrict__ hist,
                                                    int ntiles) {
    __shared__ uint32_t h[RADIX];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * TILE;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        int64_t idx = base + (int64_t)i * TH + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(TH) k_digit_scatter(const uint64_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ vals,
                                                       uint64_t* __restrict__ keys_out,
                                                       uint32_t* __restrict__ vals_out, int64_t n,
                                                       int shift,
                                                       const uint64_t* __restrict__ offsets,
                                                       int ntiles) {
    __shared__ uint64_t kbuf[2][TILE];
    __shared__ uint32_t vbuf[2][TILE];
    __shared__ uint64_t wsum4[NW + 1];
    __shared__ uint32_t lstart[RADIX];
    const int64_t base = (int64_t)blockIdx.x * TILE;
    const int cnt = (int)min<int64_t>(TILE, n - base);
    // load; padding keys carry digit 0xFF and sort after every real key of the tile
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        int p = i * TH + threadIdx.x;
        if (p < cnt) {
            kbuf[0][p] = keys[base + p];
            vbuf[0][p] = vals[base + p];
        } else {
            kbuf[0][p] = ~uint64_t(0);
            vbuf[0][p] = 0xFFFFFFFFu;
        }
    }
    __syncthreads();
    // stable split of the tile by the digit's bits, two per pass: a key goes
    // to its 2-bit value's base (the tile's keys with smaller values) plus the
    // keys with the same value before it (earlier threads, then earlier items)
    int cur = 0;
    for (int b = 0; b < 8; b += 2) {
        const int bit = shift + b;
        uint64_t k[ITEMS];
        uint32_t v[ITEMS];
        uint64_t cnt4 = 0;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            k[i] = kbuf[cur][threadIdx.x * ITEMS + i];
            v[i] = vbuf[cur][threadIdx.x * ITEMS + i];
            cnt4 += 1ull << (16 * (int)((k[i] >> bit) & 3));
        }
        uint64_t tot;
        uint64_t pos = block_excl_scan4(cnt4, &tot, wsum4);
        pos += (tot << 16) + (tot << 32) + (tot << 48);     // field d += totals below d
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int sh = 16 * (int)((k[i] >> bit) & 3);
            const uint32_t np = (uint32_t)((pos >> sh) & 0xFFFFu);
            pos += 1ull << sh;
            kbuf[cur ^ 1][np] = k[i];
            vbuf[cur ^ 1][np] = v[i];
        }
        cur ^= 1;
        __syncthreads();
    }
    // local start of every digit in the sorted tile
    if (threadIdx.x < RADIX) lstart[threadIdx.x] = TILE;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        int p = threadIdx.x * ITEMS + i;
        if (p < cnt) {
            uint32_t d = (kbuf[cur][p] >> shift) & 0xFF;
            uint32_t dprev = p > 0 ? (uint32_t)((kbuf[cur][p - 1] >> shift) & 0xFF) : 0x100u;
            if (d != dprev) lstart[d] = p;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        int p = i * TH + threadIdx.x;
        if (p < cnt) {
            uint64_t key = kbuf[cur][p];
            uint32_t d = (key >> shift) & 0xFF;
            int64_t dst = (int64_t)offsets[(int64_t)d * ntiles + blockIdx.x] + (p - (int)lstart[d]);
            keys_out[dst] = key;
            vals_out[dst] = vbuf[cur][p];
        }
    }
}

}  // namespace

size_t radix_tmp_elems(int64_t n) {
    const int64_t ntiles = std::max<int64_t>(1, ceil_div(n, TILE));
    return (size_t)(RADIX * ntiles) + scan_u64_tmp_elems(RADIX * ntiles);
}

sc_status radix_sort_pairs(sc_ctx* ctx, uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                           uint32_t* vals_alt, int64_t n, int bits, uint64_t* tmp) {
    if (n <= 1 || bits <= 0) return SC_OK;
    const int ntiles = (int)ceil_div(n, TILE);
    uint64_t* hist = tmp;
    uint64_t* scan_tmp = tmp + (size_t)RADIX * ntiles;
    uint64_t *kin = keys, *kout = keys_alt;
    uint32_t *vin = vals, *vout = vals_alt;
    const int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_digit_hist, dim3(ntiles), dim3(TH), 0, ctx->stream, kin, n, shift,
                           hist, ntiles);
        SC_CHECK_LAUNCH(ctx);
        SC_TRY(scan_u64(ctx, hist, hist, (int64_t)RADIX * ntiles, 0, scan_tmp));
        hipLaunchKernelGGL(k_digit_scatter, dim3(ntiles), dim3(TH), 0, ctx->stream, kin, vin,
                           kout, vout, n, shift, hist, ntiles);
        SC_CHECK_LAUNCH(ctx);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    if (kin != keys) {
        SC_CHECK_HIP(ctx, hipMemcpyAsync(keys, kin, n * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                                         ctx->stream));
        SC_CHECK_HIP(ctx, hipMemcpyAsync(vals, vin, n * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                                         ctx->stream));
    }
    return SC_OK;
}
