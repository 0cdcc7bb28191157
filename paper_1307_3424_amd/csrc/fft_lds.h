// Batched complex FFT in LDS: Stockham autosort with radix-8 stages and one
// final radix-4 or radix-2 stage when log2(n) is not a multiple of 3.  Used by
// the grid transforms (FP32) and by the kernel-row builder (FP64).
//
// Layout: batch member c, position j lives at
//     buf[j + c * LD]   (ROWS = true: members are contiguous rows)
//     buf[j * LD + c]   (ROWS = false: members are interleaved columns)
// tw[k] = exp(-2 pi i k / n), k in [0, n); inverse = true uses conj(tw)
// (unnormalised inverse).  Every stage stages its inputs in registers, then a
// barrier, then writes its outputs, which makes it safe in place.
//
// Stage with radix R and current sub-transform length Ns: butterfly j in
// [0, n/R) reads x[j + r n/R] (r < R), multiplies by tw[r k n/(R Ns)] with
// k = j mod Ns, takes an R-point DFT and writes it to positions
// (j - k) R + k + s Ns (s < R).
#pragma once

#include "common.h"

template <typename T2>
__device__ __forceinline__ void dft4(T2 *a, bool inverse) {
    T2 s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    T2 s13 = cadd(a[1], a[3]), d13 = csub(a[1], a[3]);
    T2 rot = inverse ? cmul_posi(d13) : cmul_negi(d13);
    a[0] = cadd(s02, s13);
    a[1] = cadd(d02, rot);
    a[2] = csub(s02, s13);
    a[3] = csub(d02, rot);
}

// 8-point DFT: even outputs are the 4-point DFT of a_r + a_(r+4), odd outputs the
// 4-point DFT of (a_r - a_(r+4)) w^r, w = exp(-+ 2 pi i / 8).
template <typename T2>
__device__ __forceinline__ void dft8(T2 *a, bool inverse) {
    using F = decltype(a[0].x);
    const F c = (F)0.70710678118654752440;
    T2 e[4], o[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        e[r] = cadd(a[r], a[r + 4]);
        o[r] = csub(a[r], a[r + 4]);
    }
    // o1 *= w, o2 *= w^2 (= -+i), o3 *= w^3
    T2 t;
    if (!inverse) {
        t = o[1]; o[1].x = c * (t.x + t.y); o[1].y = c * (t.y - t.x);
        o[2] = cmul_negi(o[2]);
        t = o[3]; o[3].x = c * (t.y - t.x); o[3].y = -c * (t.x + t.y);
    } else {
        t = o[1]; o[1].x = c * (t.x - t.y); o[1].y = c * (t.x + t.y);
        o[2] = cmul_posi(o[2]);
        t = o[3]; o[3].x = -c * (t.x + t.y); o[3].y = c * (t.x - t.y);
    }
    dft4(e, inverse);
    dft4(o, inverse);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        a[2 * p] = e[p];
        a[2 * p + 1] = o[p];
    }
}

template <typename T2, int R, int LOGN, int BATCH, int NTH, bool ROWS, int LD>
__device__ __forceinline__ void fft_stage(T2 *buf, const T2 *__restrict__ tw, bool inverse, int tid, int Ns) {
    constexpr int n = 1 << LOGN;
    constexpr int nq = n / R;
    constexpr int nb = BATCH * nq;
    constexpr int PER = (nb + NTH - 1) / NTH;
    const int step = n / (R * Ns);
    T2 reg[PER][R];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tid + i * NTH;
        if (nb % NTH == 0 || b < nb) {
            const int j = ROWS ? (b % nq) : (b / BATCH);
            const int c = ROWS ? (b / nq) : (b % BATCH);
#pragma unroll
            for (int r = 0; r < R; ++r)
                reg[i][r] = ROWS ? buf[(j + r * nq) + c * LD] : buf[(j + r * nq) * LD + c];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tid + i * NTH;
        if (nb % NTH == 0 || b < nb) {
            const int j = ROWS ? (b % nq) : (b / BATCH);
            const int c = ROWS ? (b / nq) : (b % BATCH);
            const int k = j & (Ns - 1);
            T2 *a = reg[i];
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    T2 t = tw[r * k * step];
                    if (inverse) t.y = -t.y;
                    a[r] = cmul(a[r], t);
                }
            }
            if constexpr (R == 8) {
                dft8(a, inverse);
            } else if constexpr (R == 4) {
                dft4(a, inverse);
            } else {
                const T2 a0 = a[0];
                a[0] = cadd(a0, a[1]);
                a[1] = csub(a0, a[1]);
            }
            const int base = (j - k) * R + k;
#pragma unroll
            for (int s = 0; s < R; ++s) {
                const int jj = base + s * Ns;
                if (ROWS) buf[jj + c * LD] = a[s];
                else buf[jj * LD + c] = a[s];
            }
        }
    }
    __syncthreads();
}

template <typename T2, int LOGN, int BATCH, int NTH, bool ROWS, int LD>
__device__ __forceinline__ void lds_fft(T2 *buf, const T2 *__restrict__ tw, bool inverse, int tid) {
    constexpr int N8 = LOGN / 3;
    constexpr int REM = LOGN % 3;
    int Ns = 1;
#pragma unroll
    for (int s = 0; s < N8; ++s) {
        fft_stage<T2, 8, LOGN, BATCH, NTH, ROWS, LD>(buf, tw, inverse, tid, Ns);
        Ns *= 8;
    }
    if constexpr (REM == 2) fft_stage<T2, 4, LOGN, BATCH, NTH, ROWS, LD>(buf, tw, inverse, tid, Ns);
    if constexpr (REM == 1) fft_stage<T2, 2, LOGN, BATCH, NTH, ROWS, LD>(buf, tw, inverse, tid, Ns);
}
