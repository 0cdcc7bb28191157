// Batched complex FFT in LDS: Stockham autosort, radix-4 stages with a final
// radix-2 stage when log2(n) is odd.  Used by the grid transforms (FP32) and
// by the kernel-row builder (FP64).
//
// Layout: batch member c, position j lives at
//     buf[j + c * LD]   (ROWS = true: members are contiguous rows)
//     buf[j * LD + c]   (ROWS = false: members are interleaved columns)
// tw[k] = exp(-2 pi i k / n), k in [0, n); inverse = true uses conj(tw)
// (unnormalised inverse).  Every stage stages its inputs in registers, then a
// barrier, then writes its outputs, which makes it safe in place.
#pragma once

#include "common.h"

template <typename T2, int R, int LOGN, int BATCH, int NTH, bool ROWS, int LD>
__device__ __forceinline__ void fft_stage(T2 *buf, const T2 *__restrict__ tw, bool inverse, int tid,
                                          int Ns) {
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
#pragma unroll
            for (int r = 1; r < R; ++r) {
                T2 t = tw[r * k * step];
                if (inverse) t.y = -t.y;
                a[r] = cmul(a[r], t);
            }
            const int base = (j - k) * R + k;
            T2 out[R];
            if constexpr (R == 4) {
                T2 s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
                T2 s13 = cadd(a[1], a[3]), d13 = csub(a[1], a[3]);
                T2 rot = inverse ? cmul_posi(d13) : cmul_negi(d13);
                out[0] = cadd(s02, s13);
                out[1] = cadd(d02, rot);
                out[2] = csub(s02, s13);
                out[3] = csub(d02, rot);
            } else {
                out[0] = cadd(a[0], a[1]);
                out[1] = csub(a[0], a[1]);
            }
#pragma unroll
            for (int s = 0; s < R; ++s) {
                const int jj = base + s * Ns;
                if (ROWS) buf[jj + c * LD] = out[s];
                else buf[jj * LD + c] = out[s];
            }
        }
    }
    __syncthreads();
}

template <typename T2, int LOGN, int BATCH, int NTH, bool ROWS, int LD>
__device__ __forceinline__ void lds_fft(T2 *buf, const T2 *__restrict__ tw, bool inverse, int tid) {
    constexpr int NR4 = LOGN / 2;
    int Ns = 1;
#pragma unroll
    for (int s = 0; s < NR4; ++s) {
        fft_stage<T2, 4, LOGN, BATCH, NTH, ROWS, LD>(buf, tw, inverse, tid, Ns);
        Ns *= 4;
    }
    if constexpr (LOGN & 1) fft_stage<T2, 2, LOGN, BATCH, NTH, ROWS, LD>(buf, tw, inverse, tid, Ns);
}
