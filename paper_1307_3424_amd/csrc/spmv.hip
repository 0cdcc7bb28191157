// Sparse application of G and G^H: the O(S) term of Section 3.2's cost
// O(S + N^2 log N), S = stored taps.
//
// Degrid  y_k = sum_{j in row k} G_kj X[col_j].  One 64-lane wavefront per row:
//   lanes stream the row's (col, val) pairs with unit stride (coalesced HBM
//   reads), gather X (L2 / MALL resident when rows are uv-tile sorted), and
//   reduce the complex sum with cross-lane shuffles.  Blocks are renumbered so
//   each XCD walks a contiguous range of tile-sorted rows.  From factor records
//   the taps are formed in registers as products of the row's two 1-D factors.
// Grid    X[col_j] += conj(G_kj) y_k.  One work item (a chunk of rows whose
//   visibilities fall in one uv tile) per block: taps accumulate with LDS float
//   atomics into a window covering the tile plus a halo; taps outside the
//   window go straight to global atomics; the window is then added to the grid
//   with one global atomic per non-zero cell, so global atomics happen only
//   where work items overlap (tile borders and halos).
// Gather  the same product from the transposed copy, every cell written once: one
//   wavefront per block of short cells (full-wave loads whatever the cell lengths),
//   or one lane group per cell when cells are long.
#include "gather_block.h"

namespace {

constexpr int SP_NTH = 256;
constexpr int WAVES = SP_NTH / 64;



// LPR lanes per row (64 / LPR rows per wave); each lane keeps U taps in flight.
template <int TK, int LPR, int U>
__global__ __launch_bounds__(SP_NTH) void k_degrid(const int64_t *__restrict__ rowptr, const int *__restrict__ col,
                                                   const void *__restrict__ val, const float *__restrict__ rscale,
                                                   const float2 *__restrict__ grid,
                                                   const int *__restrict__ perm, float2 *__restrict__ y, int64_t M) {
    // perm == nullptr: y in sorted row order
    const int sub = threadIdx.x & (LPR - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t r = (blk * SP_NTH + threadIdx.x) / LPR;
    float ar = 0.f, ai = 0.f;
    if (r < M) {
        const int64_t beg = rowptr[r], end = rowptr[r + 1];
        for (int64_t j0 = beg + sub; j0 < end; j0 += LPR * U) {
            int c[U];
            float2 v[U];
#pragma unroll
            for (int t = 0; t < U; ++t) {
                const int64_t j = j0 + LPR * t;
                if (j < end) {
                    c[t] = col[j];
                    v[t] = load_tap_raw<TK>(val, j);
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
    }
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) {
        ar += __shfl_xor(ar, o);
        ai += __shfl_xor(ai, o);
    }
    if (sub == 0 && r < M) {
        if constexpr (TK == WP_TAPS_I16) {
            const float sc = rscale[r];
            ar *= sc;
            ai *= sc;
        }
        y[perm ? perm[r] : r] = make_float2(ar, ai);
    }
}

// Degrid from factor records: R rows per wavefront, LPR = 64 / R lanes per row.  The lanes of a
// row copy its record into their LDS slice (coalesced) unless it is larger than the slice.  Lane
// l of a row takes u candidate i = l mod Pa (Pa a power of two >= nu, at most LPR) against v
// candidates b = l / Pa, l / Pa + LPR / Pa, ...; tap (b, i) is kept when i < nb[b].  nb does not
// increase along the v order, so a lane stops at the first b that drops its u candidate.  The
// tap gv[b] gu[i] is formed in registers: a row streams its two factor lists (about 10 bytes per
// candidate) instead of 12 bytes per tap, and the only other memory accesses are the grid reads.
constexpr int SEP_WAVE_LDS = 4096;        // bytes of LDS per wave, split between its R rows

template <int LPR, int UB>
__device__ __forceinline__ void sep_row(const unsigned char *rec, const float2 *__restrict__ grid, int logNg,
                                        int sl, float &ar, float &ai) {
    const uint32_t hdr = *(const uint32_t *)rec;
    const int nu = (int)(hdr & 0xffffu), nv = (int)(hdr >> 16);
    const uint16_t *ua = (const uint16_t *)rec + 2, *vb = ua + nu, *nbv = vb + nv;
    const float2 *gu = (const float2 *)(rec + ((4 + 2 * nu + 4 * nv + 7) & ~7)), *gv = gu + nu;
    int Pa = 1;
    while (Pa < nu && Pa < LPR) Pa <<= 1;
    const int Pb = LPR / Pa, g = sl / Pa;
    for (int i = sl & (Pa - 1); i < nu; i += Pa) {
        const int a = ua[i];
        const float2 fu = gu[i];
        for (int b0 = g; b0 < nv; b0 += Pb * UB) {
            int c[UB];
            float2 t[UB];
            bool keep = false;
#pragma unroll
            for (int q = 0; q < UB; ++q) {
                const int b = b0 + Pb * q;
                keep = b < nv && i < (int)nbv[b];
                c[q] = 0;
                t[q] = make_float2(0.f, 0.f);
                if (keep) {
                    const float2 f = gv[b];
                    c[q] = ((int)vb[b] << logNg) | a;
                    t[q] = make_float2(f.x * fu.x - f.y * fu.y, f.x * fu.y + f.y * fu.x);
                }
            }
            // a dropped tap reads cell 0 with a zero weight: cheaper than branching around the read
#pragma unroll
            for (int q = 0; q < UB; ++q) {
                const float2 x = grid[c[q]];
                ar = fmaf(t[q].x, x.x, ar);
                ar = fmaf(-t[q].y, x.y, ar);
                ai = fmaf(t[q].x, x.y, ai);
                ai = fmaf(t[q].y, x.x, ai);
            }
            if (!keep) break;             // the last b of the batch dropped i: so do all later ones
        }
    }
}

template <int R, int UB>
__global__ __launch_bounds__(SP_NTH) void k_degrid_sep(const int64_t *__restrict__ frec,
                                                       const unsigned char *__restrict__ fdat,
                                                       const float2 *__restrict__ grid, const int *__restrict__ perm,
                                                       float2 *__restrict__ y, int64_t M, int logNg) {
    constexpr int LPR = 64 / R, SLICE = SEP_WAVE_LDS / R;
    __shared__ uint2 s_rec[SP_NTH / 64][SEP_WAVE_LDS / 8];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, q = lane / LPR, sl = lane & (LPR - 1);
    const int64_t r = (xcd_block(blockIdx.x, gridDim.x) * (SP_NTH / 64) + wv) * R + q;
    uint2 *slice = s_rec[wv] + q * (SLICE / 8);
    int64_t o = 0;
    int bytes = 0;
    if (r < M) {
        o = frec[r];
        bytes = (int)(frec[r + 1] - o);
        if (bytes <= SLICE) {
            const uint2 *src = (const uint2 *)(fdat + o);
            for (int e = sl; e < bytes / 8; e += LPR) slice[e] = src[e];
        }
    }
    wave_sync();
    float ar = 0.f, ai = 0.f;
    if (r < M) {
        if (bytes <= SLICE) sep_row<LPR, UB>((const unsigned char *)slice, grid, logNg, sl, ar, ai);
        else sep_row<LPR, UB>(fdat + o, grid, logNg, sl, ar, ai);
    }
#pragma unroll
    for (int m = LPR / 2; m > 0; m >>= 1) {
        ar += __shfl_xor(ar, m);
        ai += __shfl_xor(ai, m);
    }
    if (sl == 0 && r < M) y[perm ? perm[r] : r] = make_float2(ar, ai);
}

template <int TK>
__global__ __launch_bounds__(SP_NTH) void k_scatter(const int *__restrict__ work, int64_t n_work,
                                                    const int64_t *__restrict__ rowptr, const int *__restrict__ col,
                                                    const void *__restrict__ val, const float *__restrict__ rscale,
                                                    const int *__restrict__ perm,
                                                    const float2 *__restrict__ y, float *__restrict__ grid, int logNg,
                                                    int tile, int halo, double tap_bound) {
    // The window accumulates in 64-bit fixed point: LDS integer atomics cost a few clocks per
    // wavefront instruction where LDS float atomics cost ~200 on this GPU, and integer sums do
    // not depend on the order of the adds.  Scale: every partial sum of a cell is at most
    // S = sum over the item's rows of |y_k| max |G_k.| (max |G| <= tap_bound; an int16 tap is at
    // most 46341 in modulus before its row scale), so q = 2^61 / S keeps it within int64 with a
    // quantum of S 2^-61, far below float rounding.
    extern __shared__ unsigned long long win[];     // [2][WS][WS]: real plane, imaginary plane
    __shared__ double s_red[WAVES];
    const int Ng = 1 << logNg, mask = Ng - 1;
    const int WS = tile + 2 * halo;
    const int WS2 = WS * WS;
    const int64_t item = blockIdx.x;      // round-robin over XCDs: work items near the uv centre are heavier
    const int tv = work[4 * item + 0], tu = work[4 * item + 1];
    const int rb = work[4 * item + 2], re = work[4 * item + 3];
    const int v0 = (tv * tile - halo) & mask, u0 = (tu * tile - halo) & mask;
    for (int e = threadIdx.x; e < 2 * WS2; e += SP_NTH) win[e] = 0ull;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double bsum = 0.0;
    for (int r = rb + threadIdx.x; r < re; r += SP_NTH) {
        const float2 yk = y[perm ? perm[r] : r];
        const double ay = sqrt((double)yk.x * yk.x + (double)yk.y * yk.y);
        bsum += TK == WP_TAPS_I16 ? 46341.0 * (double)rscale[r] * ay : tap_bound * ay;
    }
    for (int o = 32; o > 0; o >>= 1) bsum += __shfl_xor(bsum, o);
    if (lane == 0) s_red[wid] = bsum;
    __syncthreads();
    double S = 0.0;
    for (int i = 0; i < WAVES; ++i) S += s_red[i];
    const double q = S > 0.0 ? 2305843009213693952.0 / S : 1.0;     // 2^61 / S
    for (int r = rb + wid; r < re; r += WAVES) {
        float2 yk = y[perm ? perm[r] : r];
        if constexpr (TK == WP_TAPS_I16) {
            yk.x *= rscale[r];
            yk.y *= rscale[r];
        }
        const int64_t end = rowptr[r + 1];
        for (int64_t j = rowptr[r] + lane; j < end; j += 64) {
            const int c = col[j];
            const float2 v = load_tap_raw<TK>(val, j);
            const float cr = v.x * yk.x + v.y * yk.y;      // conj(v) * y
            const float ci = v.x * yk.y - v.y * yk.x;
            const int dv = ((c >> logNg) - v0) & mask;
            const int du = ((c & mask) - u0) & mask;
            if (dv < WS && du < WS) {
                atomicAdd(&win[dv * WS + du], (unsigned long long)__double2ll_rn((double)cr * q));
                atomicAdd(&win[WS2 + dv * WS + du], (unsigned long long)__double2ll_rn((double)ci * q));
            } else {
                unsafeAtomicAdd(&grid[2 * (int64_t)c], cr);
                unsafeAtomicAdd(&grid[2 * (int64_t)c + 1], ci);
            }
        }
    }
    __syncthreads();
    const double iq = 1.0 / q;
    const int WE = WS < Ng ? WS : Ng;
    for (int e = threadIdx.x; e < WE * WE; e += SP_NTH) {
        const int dv = e / WE, du = e % WE;
        const long long a = (long long)win[dv * WS + du], b = (long long)win[WS2 + dv * WS + du];
        if (a != 0 || b != 0) {
            const int64_t g = (int64_t)((v0 + dv) & mask) * Ng + ((u0 + du) & mask);
            unsafeAtomicAdd(&grid[2 * g], (float)((double)a * iq));
            unsafeAtomicAdd(&grid[2 * g + 1], (float)((double)b * iq));
        }
    }
}

// Scatter form of G^H from the factor records alone (no stored taps, no transposed copy): the work
// items and the fixed-point window of k_scatter; a wave takes one row at a time and its lanes walk
// the row's kept taps through the record's staircase as k_degrid_sep does (lane l: u candidate
// l mod Pa against v candidates l / Pa, l / Pa + 64 / Pa, ..., stopping at the first v candidate
// that drops it), forming each tap gv gu in registers.  The taps equal the degrid's, so the two
// products stay adjoint to FP32 rounding.
__global__ __launch_bounds__(SP_NTH) void k_scatter_sep(const int *__restrict__ work, int64_t n_work,
                                                        const int64_t *__restrict__ frec,
                                                        const unsigned char *__restrict__ fdat,
                                                        const int *__restrict__ perm, const float2 *__restrict__ y,
                                                        float *__restrict__ grid, int logNg, int tile, int halo,
                                                        double tap_bound) {
    extern __shared__ unsigned long long win[];     // [2][WS][WS]: real plane, imaginary plane
    __shared__ double s_red[WAVES];
    const int Ng = 1 << logNg, mask = Ng - 1;
    const int WS = tile + 2 * halo;
    const int WS2 = WS * WS;
    const int64_t item = blockIdx.x;
    const int tv = work[4 * item + 0], tu = work[4 * item + 1];
    const int rb = work[4 * item + 2], re = work[4 * item + 3];
    const int v0 = (tv * tile - halo) & mask, u0 = (tu * tile - halo) & mask;
    for (int e = threadIdx.x; e < 2 * WS2; e += SP_NTH) win[e] = 0ull;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double bsum = 0.0;
    for (int r = rb + threadIdx.x; r < re; r += SP_NTH) {
        const float2 yk = y[perm ? perm[r] : r];
        bsum += tap_bound * sqrt((double)yk.x * yk.x + (double)yk.y * yk.y);
    }
    for (int o = 32; o > 0; o >>= 1) bsum += __shfl_xor(bsum, o);
    if (lane == 0) s_red[wid] = bsum;
    __syncthreads();
    double S = 0.0;
    for (int i = 0; i < WAVES; ++i) S += s_red[i];
    const double q = S > 0.0 ? 2305843009213693952.0 / S : 1.0;     // 2^61 / S, as in k_scatter
    for (int r = rb + wid; r < re; r += WAVES) {
        const float2 yk = y[perm ? perm[r] : r];
        const unsigned char *rec = fdat + frec[r];
        const uint32_t hdr = *(const uint32_t *)rec;
        const int nu = (int)(hdr & 0xffffu), nv = (int)(hdr >> 16);
        const uint16_t *ua = (const uint16_t *)rec + 2, *vb = ua + nu, *nbv = vb + nv;
        const float2 *gu = (const float2 *)(rec + ((4 + 2 * nu + 4 * nv + 7) & ~7)), *gv = gu + nu;
        int Pa = 1;
        while (Pa < nu && Pa < 64) Pa <<= 1;
        const int Pb = 64 / Pa;
        for (int i = lane & (Pa - 1); i < nu; i += Pa) {
            const int a = ua[i];
            const float2 fu = gu[i];
            for (int b = lane / Pa; b < nv; b += Pb) {
                if (i >= (int)nbv[b]) break;          // nb falls along the v order: later b drop i too
                const float2 f = gv[b];
                const float tr = f.x * fu.x - f.y * fu.y, ti = f.x * fu.y + f.y * fu.x;
                const float cr = tr * yk.x + ti * yk.y;          // conj(t) * y
                const float ci = tr * yk.y - ti * yk.x;
                const int cv = vb[b];
                const int dv = (cv - v0) & mask;
                const int du = (a - u0) & mask;
                if (dv < WS && du < WS) {
                    atomicAdd(&win[dv * WS + du], (unsigned long long)__double2ll_rn((double)cr * q));
                    atomicAdd(&win[WS2 + dv * WS + du], (unsigned long long)__double2ll_rn((double)ci * q));
                } else {
                    const int64_t c = ((int64_t)cv << logNg) | a;
                    unsafeAtomicAdd(&grid[2 * c], cr);
                    unsafeAtomicAdd(&grid[2 * c + 1], ci);
                }
            }
        }
    }
    __syncthreads();
    const double iq = 1.0 / q;
    const int WE = WS < Ng ? WS : Ng;
    for (int e = threadIdx.x; e < WE * WE; e += SP_NTH) {
        const int dv = e / WE, du = e % WE;
        const long long a = (long long)win[dv * WS + du], b = (long long)win[WS2 + dv * WS + du];
        if (a != 0 || b != 0) {
            const int64_t g = (int64_t)((v0 + dv) & mask) * Ng + ((u0 + du) & mask);
            unsafeAtomicAdd(&grid[2 * g], (float)((double)a * iq));
            unsafeAtomicAdd(&grid[2 * g + 1], (float)((double)b * iq));
        }
    }
}

// Gather form of G^H: grid cell c sums conj(G_kc) y_k over its entries of the
// transposed copy.  LPR lanes per cell (64 / LPR cells per wave), U entries in
// flight per lane, cells in order, every cell written once (no atomics).
template <int TK, int LPR, int U>
__global__ __launch_bounds__(SP_NTH) void k_gather(const int64_t *__restrict__ tcolptr, const int *__restrict__ trow,
                                                   const void *__restrict__ tval, const float *__restrict__ rscale,
                                                   const float2 *__restrict__ y,
                                                   const int *__restrict__ perm, float2 *__restrict__ grid,
                                                   int64_t cells) {
    // perm == nullptr: y in sorted row order.  Blocks keep the hardware's round-robin XCD
    // order: cells near the uv centre hold several times the average number of entries, so
    // giving each XCD a contiguous range of cells would leave the edge XCDs idle.
    const int64_t blk = blockIdx.x;
    const int64_t c = (blk * SP_NTH + threadIdx.x) / LPR;
    const int sub = threadIdx.x & (LPR - 1);
    float ar = 0.f, ai = 0.f;
    if (c < cells) {
        const int64_t beg = tcolptr[c], end = tcolptr[c + 1];
        for (int64_t j0 = beg + sub; j0 < end; j0 += LPR * U) {
            int k[U];
            float2 v[U];
#pragma unroll
            for (int t = 0; t < U; ++t) {
                const int64_t j = j0 + LPR * t;
                if (j < end) {
                    const int r = trow[j];
                    k[t] = perm ? perm[r] : r;
                    v[t] = load_tap_raw<TK>(tval, j);
                    if constexpr (TK == WP_TAPS_I16) {
                        const float sc = rscale[r];
                        v[t].x *= sc;
                        v[t].y *= sc;
                    }
                } else {
                    k[t] = -1;
                    v[t] = make_float2(0.f, 0.f);
                }
            }
#pragma unroll
            for (int t = 0; t < U; ++t) {
                const float2 yk = k[t] >= 0 ? y[k[t]] : make_float2(0.f, 0.f);
                ar = fmaf(v[t].x, yk.x, ar);          // conj(v) * y
                ar = fmaf(v[t].y, yk.y, ar);
                ai = fmaf(v[t].x, yk.y, ai);
                ai = fmaf(-v[t].y, yk.x, ai);
            }
        }
    }
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) {
        ar += __shfl_xor(ar, o);
        ai += __shfl_xor(ai, o);
    }
    if (sub == 0 && c < cells) grid[c] = make_float2(ar, ai);
}

// Blocked gather form of G^H: one wavefront per block of the block table (at most GB_CELLS
// consecutive cells, entries starting within GB_ENT).  The wave streams the block's entries in
// chunks of GB_ENT with unit stride across its lanes, forms conj(G) y, and parks the products in
// its own LDS slice; then groups of L lanes (L = 64 / cells, rounded to a power of two) each sum
// one cell's stretch of the chunk.  Every load instruction carries a full wave of entries
// whatever the cell lengths; no workgroup barrier, no atomics, one fixed summation order.
constexpr int GW_WAVES = SP_NTH / 64;


template <int TK, int CH>
__global__ __launch_bounds__(SP_NTH) void k_gather_wave(const int64_t *__restrict__ tblk, int64_t nblk,
                                                        const int64_t *__restrict__ tcolptr,
                                                        const int *__restrict__ trow, const void *__restrict__ tval,
                                                        const float *__restrict__ rscale,
                                                        const float2 *__restrict__ y, const int *__restrict__ perm,
                                                        float2 *__restrict__ grid) {
    __shared__ float2 s_p[GW_WAVES][CH];
    const int64_t bi = (int64_t)blockIdx.x * GW_WAVES + (threadIdx.x >> 6);
    if (bi >= nblk) return;               // waves leave on their own: nothing in a block's sum syncs the workgroup
    gather_block<TK, CH>(tblk, bi, tcolptr, trow, tval, rscale, y, perm, grid, s_p[threadIdx.x >> 6],
                         threadIdx.x & 63);
}

__global__ void k_permute(const float2 *__restrict__ in, const int *__restrict__ perm, float2 *__restrict__ out,
                          int64_t M, bool to_sorted) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    if (to_sorted) out[r] = in[perm[r]];
    else out[perm[r]] = in[r];
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

// Lanes per row / cell: tune > 0 forces a value (plan tuning), else the power of
// two nearest mean / div in [4, 64] (measured on MI355X: rows of ~200 taps run best
// with a full wave and 4 loads in flight; grid cells of ~25 entries with 16 lanes
// and 8 loads).
int pick_lpr(double mean, double div, int tune) {
    if (tune > 0) return tune;
    int l = 4;
    while (l < 64 && (double)l * 1.5 < mean / div) l *= 2;
    return l;
}

#define WP_SPMV_DISPATCH(KERNEL, TK, LPR, U, GRID, ...)                                            \
    do {                                                                                             \
        switch ((LPR) * 100 + (U)) {                                                                 \
            case 404: hipLaunchKernelGGL((KERNEL<TK, 4, 4>), GRID, dim3(SP_NTH), 0, __VA_ARGS__); break;   \
            case 408: hipLaunchKernelGGL((KERNEL<TK, 4, 8>), GRID, dim3(SP_NTH), 0, __VA_ARGS__); break;   \
            case 804: hipLaunchKernelGGL((KERNEL<TK, 8, 4>), GRID, dim3(SP_NTH), 0, __VA_ARGS__); break;   \
            case 808: hipLaunchKernelGGL((KERNEL<TK, 8, 8>), GRID, dim3(SP_NTH), 0, __VA_ARGS__); break;   \
            case 1604: hipLaunchKernelGGL((KERNEL<TK, 16, 4>), GRID, dim3(SP_NTH), 0, __VA_ARGS__); break; \
            case 1608: hipLaunchKernelGGL((KERNEL<TK, 16, 8>), GRID, dim3(SP_NTH), 0, __VA_ARGS__); break; \
            case 1616: hipLaunchKernelGGL((KERNEL<TK, 16, 16>), GRID, dim3(SP_NTH), 0, __VA_ARGS__); break; \
            case 3204: hipLaunchKernelGGL((KERNEL<TK, 32, 4>), GRID, dim3(SP_NTH), 0, __VA_ARGS__); break; \
            case 3208: hipLaunchKernelGGL((KERNEL<TK, 32, 8>), GRID, dim3(SP_NTH), 0, __VA_ARGS__); break; \
            case 3216: hipLaunchKernelGGL((KERNEL<TK, 32, 16>), GRID, dim3(SP_NTH), 0, __VA_ARGS__); break; \
            case 6404: hipLaunchKernelGGL((KERNEL<TK, 64, 4>), GRID, dim3(SP_NTH), 0, __VA_ARGS__); break; \
            case 6408: hipLaunchKernelGGL((KERNEL<TK, 64, 8>), GRID, dim3(SP_NTH), 0, __VA_ARGS__); break; \
            default: hipLaunchKernelGGL((KERNEL<TK, 64, 16>), GRID, dim3(SP_NTH), 0, __VA_ARGS__); break; \
        }                                                                                            \
    } while (0)

// the permutation applied to visibility vectors (nullptr when they are in sorted order)
const int *yperm(const wp_G *G) { return G->order == WP_ORDER_SORTED ? nullptr : G->perm; }

bool valid_lpr_u(int lpr, int u) {
    switch (lpr * 100 + u) {
        case 404: case 408: case 804: case 808: case 1604: case 1608: case 1616: case 3204: case 3208: case 3216:
        case 6404: case 6408: case 6416: return true;
    }
    return false;
}

wp_status launch_degrid(const wp_plan *p, const wp_G *G, const float2 *grid, float2 *y, hipStream_t s) {
    if (G->M == 0) return WP_OK;
    if (G->frec && G->fdat) {
        // rows per wave: as many as keep about 16 taps per lane or more
        const double mean = (double)G->nnz / (double)G->M;
        int R = mean < 256 ? 4 : (mean < 512 ? 2 : 1);
        while (R > 1 && G->M / R < 16384) R >>= 1;     // small problems: keep the waves many
        if (p->tune_degrid_rows > 0) R = p->tune_degrid_rows;
        const int64_t waves = (G->M + R - 1) / R;
        const dim3 gr((unsigned)((waves + SP_NTH / 64 - 1) / (SP_NTH / 64)));
        const unsigned char *fd = (const unsigned char *)G->fdat;
        // measured on MI355X: four grid reads in flight per lane; rows of ~210 taps run best four
        // to a wave (2048 pixels: 7.47 ms against 9.64 from stored taps) but two at 32768 rows
        // (17.6 us), rows of ~900 one to a wave (1024 pixels: 5.47 against 8.46 ms)
        if (R == 4)
            hipLaunchKernelGGL((k_degrid_sep<4, 4>), gr, dim3(SP_NTH), 0, s, G->frec, fd, grid, yperm(G), y, G->M, p->logNg);
        else if (R == 2)
            hipLaunchKernelGGL((k_degrid_sep<2, 4>), gr, dim3(SP_NTH), 0, s, G->frec, fd, grid, yperm(G), y, G->M, p->logNg);
        else
            hipLaunchKernelGGL((k_degrid_sep<1, 4>), gr, dim3(SP_NTH), 0, s, G->frec, fd, grid, yperm(G), y, G->M, p->logNg);
        return wp_check_launch("degrid factor records");
    }
    const int U = p->tune_degrid_u > 0 ? p->tune_degrid_u : 4;
    const int lpr = pick_lpr((double)G->nnz / (double)G->M, 4.0, p->tune_degrid_lpr);
    if (!valid_lpr_u(lpr, U)) return wp_set_error(WP_EINVAL, "degrid: no kernel for lanes %d, unroll %d", lpr, U);
    const int64_t nb = (G->M * lpr + SP_NTH - 1) / SP_NTH;
    const dim3 g((unsigned)nb);
    if (G->taps == WP_TAPS_BF16)
        WP_SPMV_DISPATCH(k_degrid, WP_TAPS_BF16, lpr, U, g, s, G->rowptr, G->col, G->val, G->rscale, grid, yperm(G),
                         y, G->M);
    else if (G->taps == WP_TAPS_I16)
        WP_SPMV_DISPATCH(k_degrid, WP_TAPS_I16, lpr, U, g, s, G->rowptr, G->col, G->val, G->rscale, grid, yperm(G),
                         y, G->M);
    else
        WP_SPMV_DISPATCH(k_degrid, WP_TAPS_C64, lpr, U, g, s, G->rowptr, G->col, G->val, G->rscale, grid, yperm(G),
                         y, G->M);
    return wp_check_launch("degrid");
}

wp_status launch_gather(const wp_plan *p, const wp_G *G, const float2 *y, float2 *grid, hipStream_t s) {
    const int64_t cells = (int64_t)p->Ng * p->Ng;
    if (G->nnz == 0) return launch_fill_zero((float *)grid, 2 * cells, s);
    // measured on MI355X: blocks win while cells are short (26 entries: 20 vs 31 us; 210: 9.0 vs
    // 9.1 ms); with ~900 entries per cell the lane groups already run full and win (9.6 vs 10.2 ms)
    const double mean = (double)G->nnz / (double)cells;
    if (G->tblk && mean < 512.0) {
        const int64_t nblk = G->n_tblk;
        const dim3 gb((unsigned)((nblk + GW_WAVES - 1) / GW_WAVES));
        const int ch = p->tune_gather_chunk > 0 ? p->tune_gather_chunk : 512;
#define WP_GW(TKV, CHV) hipLaunchKernelGGL((k_gather_wave<TKV, CHV>), gb, dim3(SP_NTH), 0, s, G->tblk, nblk, \
                                           G->tcolptr, G->trow, G->tval, G->rscale, y, yperm(G), grid)
#define WP_GW_CH(TKV)                                    \
    do {                                                 \
        if (ch == 256) WP_GW(TKV, 256);                  \
        else if (ch == 768) WP_GW(TKV, 768);             \
        else if (ch == 1024) WP_GW(TKV, 1024);           \
        else WP_GW(TKV, 512);                            \
    } while (0)
        if (G->taps == WP_TAPS_BF16) WP_GW_CH(WP_TAPS_BF16);
        else if (G->taps == WP_TAPS_I16) WP_GW_CH(WP_TAPS_I16);
        else WP_GW_CH(WP_TAPS_C64);
#undef WP_GW_CH
#undef WP_GW
        return wp_check_launch("grid_gather blocks");
    }
    // measured on MI355X: 32 lanes per cell; 4 loads in flight for cells of ~25 entries,
    // 16 for cells of ~900
    const int U = p->tune_gather_u > 0 ? p->tune_gather_u : (mean < 128 ? 4 : (mean < 512 ? 8 : 16));
    const int lpr = p->tune_gather_lpr > 0 ? p->tune_gather_lpr : (mean < 12 ? 16 : 32);
    if (!valid_lpr_u(lpr, U)) return wp_set_error(WP_EINVAL, "gather: no kernel for lanes %d, unroll %d", lpr, U);
    const int64_t nb = (cells * lpr + SP_NTH - 1) / SP_NTH;
    const dim3 g((unsigned)nb);
    if (G->taps == WP_TAPS_BF16)
        WP_SPMV_DISPATCH(k_gather, WP_TAPS_BF16, lpr, U, g, s, G->tcolptr, G->trow, G->tval, G->rscale, y, yperm(G),
                         grid, cells);
    else if (G->taps == WP_TAPS_I16)
        WP_SPMV_DISPATCH(k_gather, WP_TAPS_I16, lpr, U, g, s, G->tcolptr, G->trow, G->tval, G->rscale, y, yperm(G),
                         grid, cells);
    else
        WP_SPMV_DISPATCH(k_gather, WP_TAPS_C64, lpr, U, g, s, G->tcolptr, G->trow, G->tval, G->rscale, y, yperm(G),
                         grid, cells);
    return wp_check_launch("grid_gather");
}

wp_status launch_scatter(const wp_plan *p, const wp_G *G, const float2 *y, float2 *grid, hipStream_t s) {
    wp_status st = launch_fill_zero((float *)grid, 2 * (int64_t)p->Ng * p->Ng, s);
    if (st != WP_OK || G->n_work == 0) return st;
    const int WS = p->tile + 2 * p->halo;
    const size_t lds = (size_t)2 * WS * WS * sizeof(unsigned long long);
    const dim3 gw((unsigned)G->n_work), bw(SP_NTH);
    if (!G->val) {                 // no stored taps: form them from the factor records
        hipLaunchKernelGGL(k_scatter_sep, gw, bw, lds, s, G->work, G->n_work, G->frec,
                           (const unsigned char *)G->fdat, yperm(G), y, (float *)grid, p->logNg, p->tile, p->halo,
                           p->tap_bound);
        return wp_check_launch("grid_scatter from factor records");
    }
    if (G->taps == WP_TAPS_BF16)
        hipLaunchKernelGGL((k_scatter<WP_TAPS_BF16>), gw, bw, lds, s, G->work, G->n_work, G->rowptr, G->col, G->val,
                           G->rscale, yperm(G), y, (float *)grid, p->logNg, p->tile, p->halo,
                           p->tap_bound);
    else if (G->taps == WP_TAPS_I16)
        hipLaunchKernelGGL((k_scatter<WP_TAPS_I16>), gw, bw, lds, s, G->work, G->n_work, G->rowptr, G->col, G->val,
                           G->rscale, yperm(G), y, (float *)grid, p->logNg, p->tile, p->halo,
                           p->tap_bound);
    else
        hipLaunchKernelGGL((k_scatter<WP_TAPS_C64>), gw, bw, lds, s, G->work, G->n_work, G->rowptr, G->col, G->val,
                           G->rscale, yperm(G), y, (float *)grid, p->logNg, p->tile, p->halo,
                           p->tap_bound);
    return wp_check_launch("grid_scatter");
}

wp_status launch_permute(const wp_G *G, const float2 *in, float2 *out, bool to_sorted, hipStream_t s) {
    if (G->M == 0) return WP_OK;
    hipLaunchKernelGGL(k_permute, dim3((unsigned)((G->M + 255) / 256)), dim3(256), 0, s, in, G->perm, out, G->M,
                       to_sorted);
    return wp_check_launch("permute");
}
