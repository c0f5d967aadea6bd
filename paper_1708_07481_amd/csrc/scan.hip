// Device-wide scans of uint64 values (exact, so the result does not depend on
// the reduction order): tile sums, a scan of the tile sums, then a scan of
// every tile with its offset.
#include "sc_internal.h"

namespace {

constexpr int TH = 256;
constexpr int ITEMS = 8;
constexpr int TILE = TH * ITEMS;
constexpr int NW = TH / 64;

__device__ inline uint64_t wave_incl_scan(uint64_t x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// exclusive block scan of one value per thread; returns the block total in *total
__device__ inline uint64_t block_excl_scan(uint64_t v, uint64_t* total) {
    __shared__ uint64_t wsum[NW + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t x = wave_incl_scan(v, lane);
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t acc = 0;
        for (int w = 0; w < NW; ++w) {
            uint64_t t = wsum[w];
            wsum[w] = acc;
            acc += t;
        }
        wsum[NW] = acc;
    }
    __syncthreads();
    uint64_t r = x - v + wsum[wave];
    *total = wsum[NW];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(TH) k_tile_sums(const uint64_t* __restrict__ in, int64_t n,
                                                   uint64_t* __restrict__ sums, int ntiles) {
    const int64_t row = blockIdx.y;
    const int64_t base = (int64_t)blockIdx.x * TILE;
    const uint64_t* x = in + row * n;
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        int64_t idx = base + (int64_t)i * TH + threadIdx.x;
        if (idx < n) s += x[idx];
    }
    uint64_t tot;
    (void)block_excl_scan(s, &tot);
    if (threadIdx.x == 0) sums[row * ntiles + blockIdx.x] = tot;
}

// exclusive scan of the tile sums of every row (one block per row)
__global__ void __launch_bounds__(TH) k_scan_tile_sums(uint64_t* sums, int ntiles) {
    uint64_t* s = sums + (int64_t)blockIdx.x * ntiles;
    uint64_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += TILE) {
        uint64_t v[ITEMS];
        uint64_t loc = 0;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            int64_t idx = base + (int64_t)threadIdx.x * ITEMS + i;
            v[i] = idx < ntiles ? s[idx] : 0;
            loc += v[i];
        }
        uint64_t tot;
        uint64_t ex = block_excl_scan(loc, &tot) + carry;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            int64_t idx = base + (int64_t)threadIdx.x * ITEMS + i;
            if (idx < ntiles) s[idx] = ex;
            ex += v[i];
        }
        carry += tot;
    }
}

__global__ void __launch_bounds__(TH) k_scan_apply(const uint64_t* __restrict__ in,
                                                    uint64_t* __restrict__ out, int64_t n,
                                                    const uint64_t* __restrict__ sums, int ntiles,
                                                    int inclusive) {
    __shared__ uint64_t buf[TILE];
    const int64_t row = blockIdx.y;
    const int64_t base = (int64_t)blockIdx.x * TILE;
    const uint64_t* x = in + row * n;
    uint64_t* y = out + row * n;
    // coalesced load into LDS, then each thread scans ITEMS consecutive values
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        int64_t idx = base + (int64_t)i * TH + threadIdx.x;
        buf[i * TH + threadIdx.x] = idx < n ? x[idx] : 0;
    }
    __syncthreads();
    uint64_t v[ITEMS], loc = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        v[i] = buf[threadIdx.x * ITEMS + i];
        loc += v[i];
    }
    uint64_t tot;
    uint64_t ex = block_excl_scan(loc, &tot) + sums[row * ntiles + blockIdx.x];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        uint64_t inc = ex + v[i];
        buf[threadIdx.x * ITEMS + i] = inclusive ? inc : ex;
        ex = inc;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        int64_t idx = base + (int64_t)i * TH + threadIdx.x;
        if (idx < n) y[idx] = buf[i * TH + threadIdx.x];
    }
}

}  // namespace

size_t scan_u64_batched_tmp_elems(int64_t n, int batch) {
    return (size_t)std::max<int64_t>(1, ceil_div(n, TILE)) * (size_t)batch;
}
size_t scan_u64_tmp_elems(int64_t n) { return scan_u64_batched_tmp_elems(n, 1); }

static sc_status scan_impl(sc_ctx* ctx, const uint64_t* in, uint64_t* out, int64_t n, int batch,
                           int inclusive, uint64_t* tmp) {
    if (n <= 0 || batch <= 0) return SC_OK;
    const int ntiles = (int)ceil_div(n, TILE);
    dim3 grid(ntiles, batch);
    hipLaunchKernelGGL(k_tile_sums, grid, dim3(TH), 0, ctx->stream, in, n, tmp, ntiles);
    SC_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(batch), dim3(TH), 0, ctx->stream, tmp, ntiles);
    SC_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(k_scan_apply, grid, dim3(TH), 0, ctx->stream, in, out, n, tmp, ntiles,
                       inclusive);
    SC_CHECK_LAUNCH(ctx);
    return SC_OK;
}

sc_status scan_u64(sc_ctx* ctx, const uint64_t* in, uint64_t* out, int64_t n, int inclusive,
                   uint64_t* tmp) {
    return scan_impl(ctx, in, out, n, 1, inclusive, tmp);
}

sc_status scan_u64_batched(sc_ctx* ctx, const uint64_t* in, uint64_t* out, int64_t n, int batch,
                           uint64_t* tmp) {
    return scan_impl(ctx, in, out, n, batch, 1, tmp);
}

sc_status scan_u64_batched_exclusive(sc_ctx* ctx, const uint64_t* in, uint64_t* out, int64_t n,
                                     int batch, uint64_t* tmp) {
    return scan_impl(ctx, in, out, n, batch, 0, tmp);
}
