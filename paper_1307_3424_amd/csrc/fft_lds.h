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

// pre (or null): this stage's twiddles, already conjugated for the inverse, pre[i][r - 1] for the
// thread's i-th butterfly
template <typename T2, int R, int LOGN, int BATCH, int NTH, bool ROWS, int LD>
__device__ __forceinline__ void fft_stage(T2 *buf, const T2 *__restrict__ tw, const T2 (*pre)[7], bool inverse,
                                          int tid, int Ns) {
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
                    T2 t;
                    if (pre) {
                        t = pre[i][r - 1];
                    } else {
                        t = tw[r * k * step];
                        if (inverse) t.y = -t.y;
                    }
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

// Stage s of an n-point transform: radix 8 for s < LOGN / 3, then radix 4 or 2; the sub-transform
// length before stage s is 8^s; per(s) is the number of butterflies per thread.
template <int LOGN>
struct FftStages {
    static constexpr int n = 1 << LOGN, N8 = LOGN / 3, REM = LOGN % 3, count = N8 + (REM ? 1 : 0);
    static constexpr int radix(int s) { return s < N8 ? 8 : (REM == 2 ? 4 : 2); }
    static constexpr int ns(int s) { return 1 << (3 * s); }
    static constexpr int per(int s, int batch, int nth) { return (batch * (n / radix(s)) + nth - 1) / nth; }
    static constexpr int per_max(int batch, int nth) {
        int m = 1;
        for (int s = 1; s < count; ++s) m = per(s, batch, nth) > m ? per(s, batch, nth) : m;
        return m;
    }
};

// The twiddles of every stage after the first, for all of a thread's butterflies.  Loaded before
// the caller stages its data, their latency overlaps those loads instead of stalling each stage.
// Only where they fit a modest register budget (enabled); otherwise the stages load their own.
template <typename T2, int LOGN, int BATCH, int NTH, bool ROWS>
struct FftTwiddles {
    using St = FftStages<LOGN>;
    static constexpr int NT = St::count > 1 ? St::count - 1 : 1, PM = St::per_max(BATCH, NTH);
    static constexpr bool enabled = St::count > 1 && NT * PM * 7 <= 14;
    T2 t[enabled ? NT : 1][enabled ? PM : 1][7];

    __device__ __forceinline__ void load(const T2 *__restrict__ tw, bool inverse, int tid) {
        if constexpr (enabled) load_stage<1>(tw, inverse, tid);
    }
    template <int S>
    __device__ __forceinline__ void load_stage(const T2 *__restrict__ tw, bool inverse, int tid) {
        if constexpr (S < St::count) {
            constexpr int R = St::radix(S), Ns = St::ns(S), nq = St::n / R, nb = BATCH * nq;
            constexpr int PER = St::per(S, BATCH, NTH), step = St::n / (R * Ns);
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int b = tid + i * NTH;
                const int j = ROWS ? (b % nq) : (b / BATCH);
                const int k = j & (Ns - 1);                     // k < Ns, so r k step < n
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    T2 v = tw[r * k * step];
                    if (inverse) v.y = -v.y;
                    t[S - 1][i][r - 1] = (nb % NTH == 0 || b < nb) ? v : T2{};
                }
            }
            load_stage<S + 1>(tw, inverse, tid);
        }
    }
};

// pre (or null): twiddles loaded by FftTwiddles::load with the same inverse flag
template <typename T2, int LOGN, int BATCH, int NTH, bool ROWS, int LD>
__device__ __forceinline__ void lds_fft(T2 *buf, const T2 *__restrict__ tw,
                                        const FftTwiddles<T2, LOGN, BATCH, NTH, ROWS> *pre, bool inverse, int tid) {
    using Pre = FftTwiddles<T2, LOGN, BATCH, NTH, ROWS>;
    constexpr int N8 = LOGN / 3;
    constexpr int REM = LOGN % 3;
    int Ns = 1;
#pragma unroll
    for (int s = 0; s < N8; ++s) {
        const T2(*ps)[7] = nullptr;
        if constexpr (Pre::enabled) ps = (pre && s > 0) ? pre->t[s - 1] : nullptr;
        fft_stage<T2, 8, LOGN, BATCH, NTH, ROWS, LD>(buf, tw, ps, inverse, tid, Ns);
        Ns *= 8;
    }
    const T2(*pl)[7] = nullptr;
    if constexpr (Pre::enabled && REM != 0) pl = pre ? pre->t[N8 - 1] : nullptr;
    if constexpr (REM == 2) fft_stage<T2, 4, LOGN, BATCH, NTH, ROWS, LD>(buf, tw, pl, inverse, tid, Ns);
    if constexpr (REM == 1) fft_stage<T2, 2, LOGN, BATCH, NTH, ROWS, LD>(buf, tw, pl, inverse, tid, Ns);
}

template <typename T2, int LOGN, int BATCH, int NTH, bool ROWS, int LD>
__device__ __forceinline__ void lds_fft(T2 *buf, const T2 *__restrict__ tw, bool inverse, int tid) {
    lds_fft<T2, LOGN, BATCH, NTH, ROWS, LD>(buf, tw, (const FftTwiddles<T2, LOGN, BATCH, NTH, ROWS> *)nullptr,
                                            inverse, tid);
}
