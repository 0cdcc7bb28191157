// Sparse application of G and G^H: the O(S) term of Section 3.2's cost
// O(S + N^2 log N), S = stored taps.
//
// Degrid  y_k = sum_{j in row k} G_kj X[col_j].  One 64-lane wavefront per row:
//   lanes stream the row's (col, val) pairs with unit stride (coalesced HBM
//   reads), gather X (L2 / MALL resident when rows are uv-tile sorted), and
//   reduce the complex sum with cross-lane shuffles.  Blocks are renumbered so
//   each XCD walks a contiguous range of tile-sorted rows.
// Grid    X[col_j] += conj(G_kj) y_k.  One work item (a chunk of rows whose
//   visibilities fall in one uv tile) per block: taps accumulate with LDS float
//   atomics into a window covering the tile plus a halo; taps outside the
//   window go straight to global atomics; the window is then added to the grid
//   with one global atomic per non-zero cell, so global atomics happen only
//   where work items overlap (tile borders and halos).
#include "common.h"

namespace {

constexpr int SP_NTH = 256;
constexpr int WAVES = SP_NTH / 64;

template <bool BF16>
__device__ __forceinline__ float2 load_tap(const void *__restrict__ val, int64_t j) {
    if constexpr (BF16) return unpack_bf16x2(((const uint32_t *)val)[j]);
    else return ((const float2 *)val)[j];
}

template <bool BF16, int U>
__global__ __launch_bounds__(SP_NTH) void k_degrid(const int64_t *__restrict__ rowptr, const int *__restrict__ col,
                                                   const void *__restrict__ val, const float2 *__restrict__ grid,
                                                   const int *__restrict__ perm, float2 *__restrict__ y, int64_t M) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t r = blk * WAVES + wid;
    if (r >= M) return;
    const int64_t beg = rowptr[r], end = rowptr[r + 1];
    float ar = 0.f, ai = 0.f;
    for (int64_t j0 = beg + lane; j0 < end; j0 += 64 * U) {
        int c[U];
        float2 v[U];
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const int64_t j = j0 + 64 * t;
            if (j < end) {
                c[t] = col[j];
                v[t] = load_tap<BF16>(val, j);
            } else {
                c[t] = 0;
                v[t] = make_float2(0.f, 0.f);
            }
        }
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const float2 g = grid[c[t]];
            ar = fmaf(v[t].x, g.x, ar);
            ar = fmaf(-v[t].y, g.y, ar);
            ai = fmaf(v[t].x, g.y, ai);
            ai = fmaf(v[t].y, g.x, ai);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        ar += __shfl_xor(ar, o);
        ai += __shfl_xor(ai, o);
    }
    if (lane == 0) y[perm[r]] = make_float2(ar, ai);
}

template <bool BF16>
__global__ __launch_bounds__(SP_NTH) void k_scatter(const int *__restrict__ work, int64_t n_work,
                                                    const int64_t *__restrict__ rowptr, const int *__restrict__ col,
                                                    const void *__restrict__ val, const int *__restrict__ perm,
                                                    const float2 *__restrict__ y, float *__restrict__ grid, int logNg,
                                                    int tile, int halo) {
    extern __shared__ float win[];                  // [2][WS][WS]: real plane, imaginary plane
    const int Ng = 1 << logNg, mask = Ng - 1;
    const int WS = tile + 2 * halo;
    const int WS2 = WS * WS;
    const int64_t item = xcd_block(blockIdx.x, gridDim.x);
    const int tv = work[4 * item + 0], tu = work[4 * item + 1];
    const int rb = work[4 * item + 2], re = work[4 * item + 3];
    const int v0 = (tv * tile - halo) & mask, u0 = (tu * tile - halo) & mask;
    for (int e = threadIdx.x; e < 2 * WS2; e += SP_NTH) win[e] = 0.f;
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int r = rb + wid; r < re; r += WAVES) {
        const float2 yk = y[perm[r]];
        const int64_t end = rowptr[r + 1];
        for (int64_t j = rowptr[r] + lane; j < end; j += 64) {
            const int c = col[j];
            const float2 v = load_tap<BF16>(val, j);
            const float cr = v.x * yk.x + v.y * yk.y;      // conj(v) * y
            const float ci = v.x * yk.y - v.y * yk.x;
            const int dv = ((c >> logNg) - v0) & mask;
            const int du = ((c & mask) - u0) & mask;
            if (dv < WS && du < WS) {
                atomicAdd(&win[dv * WS + du], cr);
                atomicAdd(&win[WS2 + dv * WS + du], ci);
            } else {
                unsafeAtomicAdd(&grid[2 * (int64_t)c], cr);
                unsafeAtomicAdd(&grid[2 * (int64_t)c + 1], ci);
            }
        }
    }
    __syncthreads();
    const int WE = WS < Ng ? WS : Ng;
    for (int e = threadIdx.x; e < WE * WE; e += SP_NTH) {
        const int dv = e / WE, du = e % WE;
        const float a = win[dv * WS + du], b = win[WS2 + dv * WS + du];
        if (a != 0.f || b != 0.f) {
            const int64_t g = (int64_t)((v0 + dv) & mask) * Ng + ((u0 + du) & mask);
            unsafeAtomicAdd(&grid[2 * g], a);
            unsafeAtomicAdd(&grid[2 * g + 1], b);
        }
    }
}

__global__ void k_fill_zero(float4 *__restrict__ p, int64_t n4) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

}  // namespace

wp_status launch_fill_zero(float *buf, int64_t n, hipStream_t s) {
    // n floats, n % 4 == 0 and 16-byte aligned (the grid always is)
    const int64_t n4 = n / 4;
    int64_t nb = (n4 + 255) / 256;
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)nb), dim3(256), 0, s, (float4 *)buf, n4);
    return wp_check_launch("fill_zero");
}

wp_status launch_degrid(const wp_plan *p, const wp_G *G, const float2 *grid, float2 *y, hipStream_t s) {
    (void)p;
    if (G->M == 0) return WP_OK;
    const int64_t nb = (G->M + WAVES - 1) / WAVES;
    if (G->taps == WP_TAPS_BF16)
        hipLaunchKernelGGL((k_degrid<true, 4>), dim3((unsigned)nb), dim3(SP_NTH), 0, s, G->rowptr, G->col, G->val, grid,
                           G->perm, y, G->M);
    else
        hipLaunchKernelGGL((k_degrid<false, 4>), dim3((unsigned)nb), dim3(SP_NTH), 0, s, G->rowptr, G->col, G->val,
                           grid, G->perm, y, G->M);
    return wp_check_launch("degrid");
}

wp_status launch_scatter(const wp_plan *p, const wp_G *G, const float2 *y, float2 *grid, hipStream_t s) {
    wp_status st = launch_fill_zero((float *)grid, 2 * (int64_t)p->Ng * p->Ng, s);
    if (st != WP_OK || G->n_work == 0) return st;
    const int WS = p->tile + 2 * p->halo;
    const size_t lds = (size_t)2 * WS * WS * sizeof(float);
    if (G->taps == WP_TAPS_BF16)
        hipLaunchKernelGGL((k_scatter<true>), dim3((unsigned)G->n_work), dim3(SP_NTH), lds, s, G->work, G->n_work,
                           G->rowptr, G->col, G->val, G->perm, y, (float *)grid, p->logNg, p->tile, p->halo);
    else
        hipLaunchKernelGGL((k_scatter<false>), dim3((unsigned)G->n_work), dim3(SP_NTH), lds, s, G->work, G->n_work,
                           G->rowptr, G->col, G->val, G->perm, y, (float *)grid, p->logNg, p->tile, p->halo);
    return wp_check_launch("grid_scatter");
}
