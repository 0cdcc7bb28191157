// Internal: one block of the blocked gather form of G^H, shared by the single-problem kernel
// (spmv.hip) and the persistent batch kernel (batch.hip).
//
// A block of the transposed copy's block table is a run of at most GB_CELLS consecutive grid
// cells (entries [ea, eb)).  One wavefront streams the entries in chunks of CH with unit stride
// across its lanes, forms conj(G) y and parks the products in its own LDS slice sp[CH]; then
// groups of L lanes (L = 64 / cells, rounded to a power of two) each sum one cell's stretch of the
// chunk.  Every load instruction carries a full wave of entries whatever the cell lengths; no
// workgroup barrier, no atomics, one fixed summation order.
#pragma once

#include "common.h"

// orders a wave's LDS stores before its later LDS loads by other lanes (no workgroup barrier)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int TK, int CH>
__device__ __forceinline__ void gather_block(const int64_t *__restrict__ tblk, int64_t bi,
                                             const int64_t *__restrict__ tcolptr, const int *__restrict__ trow,
                                             const void *__restrict__ tval, const float *__restrict__ rscale,
                                             const float2 *__restrict__ y, const int *__restrict__ perm,
                                             float2 *__restrict__ grid, float2 *sp, int lane) {
    const int64_t ca = tblk[2 * bi], ea = tblk[2 * bi + 1], cb = tblk[2 * bi + 2], eb = tblk[2 * bi + 3];
    const int nc = (int)(cb - ca);
    if (nc <= 0) return;                  // wave-uniform
    int L = 64;
    while (L > 1 && L * nc > 64) L >>= 1;
    const int q = lane / L, sub = lane & (L - 1);
    int64_t qb = 0, qe = 0;               // entries of this lane group's cell
    if (q < nc) {
        qb = tcolptr[ca + q];
        qe = tcolptr[ca + q + 1];
    }
    float ar = 0.f, ai = 0.f;
    for (int64_t c0 = ea; c0 < eb; c0 += CH) {
        const int n = (int)min((int64_t)CH, eb - c0);
        constexpr int PER = CH / 64;
        int k[PER];
        float2 v[PER];
        // Each phase issues all of a lane's loads before the next phase waits on them: entries, then
        // the permutation (one wave-uniform test, outside the loop), then y and the row scales.
        // Lanes past the chunk's end take row 0 (a valid row: there are entries) and store nothing.
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int e = t * 64 + lane;
            k[t] = 0;
            v[t] = make_float2(0.f, 0.f);
            if (e < n) {
                k[t] = trow[c0 + e];
                v[t] = load_tap_raw<TK>(tval, c0 + e);
            }
        }
        int yi[PER];
#pragma unroll
        for (int t = 0; t < PER; ++t) yi[t] = k[t];
        if (perm) {
#pragma unroll
            for (int t = 0; t < PER; ++t) yi[t] = perm[yi[t]];
        }
        float2 yk[PER];
        float sc[PER];
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            yk[t] = y[yi[t]];
            sc[t] = 1.f;
            if constexpr (TK == WP_TAPS_I16) sc[t] = rscale[k[t]];
        }
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int e = t * 64 + lane;
            if (e < n) {
                float2 g = v[t];
                if constexpr (TK == WP_TAPS_I16) {
                    g.x *= sc[t];
                    g.y *= sc[t];
                }
                sp[e] = make_float2(fmaf(g.x, yk[t].x, g.y * yk[t].y), fmaf(g.x, yk[t].y, -g.y * yk[t].x));   // conj(G) y
            }
        }
        wave_sync();
        if (q < nc) {
            const int lo = (int)(max(qb, c0) - c0), hi = (int)(min(qe, c0 + n) - c0);
            for (int e = lo + sub; e < hi; e += L) {
                const float2 p = sp[e];
                ar += p.x;
                ai += p.y;
            }
        }
        wave_sync();                      // the next chunk overwrites the slice
    }
    for (int o = L / 2; o > 0; o >>= 1) {
        ar += __shfl_xor(ar, o);
        ai += __shfl_xor(ai, o);
    }
    if (sub == 0 && q < nc) grid[ca + q] = make_float2(ar, ai);
}

