// Rows of G made whole in 2-D: the exact w-term (Eq. 4), which is not separable, and any chirp
// times a per-visibility direction-dependent effect (Sections 3.1 and 3.2).
//
// Row k, for a visibility at grid coordinates (u~, v~) with component w:
//   1. modulation c(l, m) on the padded grid, l = t_u delta, m = t_v delta, t in
//      [-Ng/2, Ng/2) stored at index t mod Ng: the exact chirp
//      exp(-2 pi i w (sqrt(1 - l^2 - m^2) - 1)), with sqrt(1 - r^2) - 1 evaluated as
//      -r^2 / (1 + sqrt(1 - r^2)) (no cancellation) and the phase 2 w r^2 / (1 + sqrt(1 - r^2))
//      given to sincospi in FP64, or the linear chirp exp(i pi w r^2); with a beam
//      (l0, m0, sigma) per visibility, times exp(-((l - l0)^2 + (m - m0)^2) / (2 sigma^2));
//   2. H(d) = Ng^-2 sum_t c(t) exp(-2 pi i t.d / Ng): a 2-D FFT in FP64, rows in one
//      kernel and columns in the next, both in LDS;
//   3. g(q) = sum_{a,b} KB(u~ - q'_a) KB(v~ - q'_b) H(q' - q) (indices mod Ng).  The
//      window is separable, so the correlation runs per axis inside the FFT kernels:
//      along u after the row transform, along v after the column transform (both
//      are linear and act on different axes, so the order is free);
//   4. tau = the largest value with K(tau) >= E T, K(tau) = sum of the energies
//      |g|^2 >= tau, T = K(0).  The search runs on the IEEE-754 bit patterns of the
//      non-negative doubles (monotone): each pass evaluates K at 15 points splitting
//      the bracket [lo, hi) into 16 (K(lo) >= E T > K(hi)), so 16 passes close a
//      64-bit bracket; once the bracket holds few entries, they alone are kept (in
//      LDS) and K(c) = K(hi) + their sum >= c.  It ends on an energy of the row, and the kept
//      set {|g|^2 >= tau} (ties kept) is the sort-defined set; E >= 1 keeps every
//      non-zero entry.
// Rows are made in chunks (the 2-D rows of a chunk live in the builder's workspace);
// the count pass stores each row's energies only, the fill pass its values, and the
// fill writes the kept entries in ascending flattened column q_v Ng + q_u.
#pragma once

#include <cfloat>

#include "builder_util.h"
#include "fft_lds.h"

namespace {

constexpr int EX_LINES = 4;                      // rows / columns per block of the FFT passes
constexpr int64_t EX_CHUNK_BYTES = 1ll << 30;    // 2-D rows in flight: at most this many bytes
constexpr int TNT = 1024;                        // threads of the threshold search (one workgroup per row)
constexpr int TAU_CAP = 8192;                    // entries of a narrowed bracket the search keeps in LDS

template <typename T>
__device__ inline T tau_block_sum(T v, T *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = 0;
    for (int i = 0; i < TNT / 64; ++i) s += red[i];
    return s;
}

// exclusive scan of one int per thread over the TNT threads; returns the total
__device__ inline int tau_block_excl_scan(int v, int *red, int &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) red[wid] = x;
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < TNT / 64; ++i) {
        if (i < wid) off += red[i];
        tot += red[i];
    }
    total = tot;
    return off + x - v;
}

__device__ inline double tau_block_max(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < TNT / 64; ++i) s = fmax(s, red[i]);
    return s;
}

// rows per chunk for a plan: as many Ng x Ng rows (complex FP64 values, then FP64 energies beside
// them) as EX_CHUNK_BYTES holds, at most 4096
constexpr int64_t EX_ROW_BYTES_PER_CELL = 24;
inline int64_t exact_chunk_rows(int Ng, int64_t M) {
    int64_t b = EX_CHUNK_BYTES / (EX_ROW_BYTES_PER_CELL * Ng * Ng);
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return b < M ? b : M;
}

__device__ inline bool exact_coords(const double *u, const double *v, const double *w, int64_t k, double cell,
                                    int Ng, double &ut, double &vt, double &wk) {
    ut = u[k] / cell;
    vt = v[k] / cell;
    wk = w[k];
    return isfinite(ut) && isfinite(vt) && isfinite(wk) && fabs(ut) < Ng / 2 && fabs(vt) < Ng / 2;
}

// a visibility's beam (l0, m0, sigma) is usable: finite, sigma > 0
__device__ inline bool beam_ok(const double *beam, int64_t k) {
    if (!beam) return true;
    const double l0 = beam[3 * k], m0 = beam[3 * k + 1], sg = beam[3 * k + 2];
    return isfinite(l0) && isfinite(m0) && isfinite(sg) && sg > 0.0;
}

// Pass 1 of a chunk: chirp rows t_v = line, FFT along u, correlation along u with the u window.
// Block (x, b) handles EX_LINES rows of chunk member b (visibility perm[base + b], or base + b
// when perm is null).  out[b][t_v][q_u] (double2).
template <int LOGNG>
__global__ __launch_bounds__(BNTH) void k_exact_rows(const double *__restrict__ u, const double *__restrict__ v,
                                                     const double *__restrict__ w, const double *__restrict__ beam,
                                                     int exact, const int *__restrict__ perm,
                                                     int64_t base, double cell, double delta, int W, double beta,
                                                     const double2 *__restrict__ tw64, double2 *__restrict__ out) {
    constexpr int Ng = 1 << LOGNG;
    __shared__ double2 buf[EX_LINES * Ng];
    __shared__ double s_wu[16];
    const int b = blockIdx.y;
    const int64_t k = perm ? (int64_t)perm[base + b] : base + b;
    double ut, vt, wk;
    const bool ok = exact_coords(u, v, w, k, cell, Ng, ut, vt, wk) && beam_ok(beam, k);
    double2 *dst = out + ((int64_t)b * Ng + (int64_t)blockIdx.x * EX_LINES) * Ng;
    if (!ok) {
        for (int e = threadIdx.x; e < EX_LINES * Ng; e += BNTH) dst[e] = make_double2(0.0, 0.0);
        return;
    }
    const Taps tu = kb_taps(ut, W, beta, Ng, s_wu);
    for (int e = threadIdx.x; e < EX_LINES * Ng; e += BNTH) {
        const int c = e / Ng, iu = e % Ng, iv = blockIdx.x * EX_LINES + c;
        const double l = (iu < Ng / 2 ? iu : iu - Ng) * delta, m = (iv < Ng / 2 ? iv : iv - Ng) * delta;
        const double r2 = l * l + m * m;
        double sn, cs;
        sincospi(exact ? 2.0 * wk * r2 / (1.0 + sqrt(1.0 - r2)) : wk * r2, &sn, &cs);
        if (beam) {
            const double dl = l - beam[3 * k], dm = m - beam[3 * k + 1], sg = beam[3 * k + 2];
            const double a = exp(-(dl * dl + dm * dm) / (2.0 * sg * sg));
            cs *= a;
            sn *= a;
        }
        buf[e] = make_double2(cs, sn);
    }
    __syncthreads();
    lds_fft<double2, LOGNG, EX_LINES, BNTH, true, Ng>(buf, tw64, false, threadIdx.x);
    for (int e = threadIdx.x; e < EX_LINES * Ng; e += BNTH) {
        const int c = e / Ng, q = e % Ng;
        double2 acc = make_double2(0.0, 0.0);
        for (int i = 0; i < W; ++i) {
            const double2 h = buf[c * Ng + ((tu.q0 + i - q) & (Ng - 1))];
            acc.x += tu.wt[i] * h.x;
            acc.y += tu.wt[i] * h.y;
        }
        dst[e] = acc;
    }
}

// Pass 2 of a chunk: FFT along v of EX_LINES columns, correlation along v with the v window,
// scale Ng^-2.  ENERGY: write |g|^2 to energy_out (double, [b][q_v][q_u], a region apart from
// rows: other blocks still read their columns of rows) instead of g (double2, in place).
template <int LOGNG, bool ENERGY>
__global__ __launch_bounds__(BNTH) void k_exact_cols(const double *__restrict__ u, const double *__restrict__ v,
                                                     const double *__restrict__ w, const double *__restrict__ beam,
                                                     const int *__restrict__ perm,
                                                     int64_t base, double cell, double beta, int W,
                                                     const double2 *__restrict__ tw64, double2 *__restrict__ rows,
                                                     double *__restrict__ energy_out) {
    constexpr int Ng = 1 << LOGNG;
    __shared__ double2 buf[Ng * EX_LINES];
    __shared__ double s_wv[16];
    const int b = blockIdx.y;
    const int64_t k = perm ? (int64_t)perm[base + b] : base + b;
    double ut, vt, wk;
    const bool ok = exact_coords(u, v, w, k, cell, Ng, ut, vt, wk) && beam_ok(beam, k);
    const int qu0 = blockIdx.x * EX_LINES;
    double2 *src = rows + (int64_t)b * Ng * Ng;
    const Taps tv = kb_taps(ok ? vt : 0.0, W, beta, Ng, s_wv);
    for (int e = threadIdx.x; e < Ng * EX_LINES; e += BNTH) {
        const int iv = e / EX_LINES, c = e % EX_LINES;
        buf[e] = src[(int64_t)iv * Ng + qu0 + c];
    }
    __syncthreads();
    lds_fft<double2, LOGNG, EX_LINES, BNTH, false, EX_LINES>(buf, tw64, false, threadIdx.x);
    const double scale = 1.0 / ((double)Ng * (double)Ng);
    for (int e = threadIdx.x; e < Ng * EX_LINES; e += BNTH) {
        const int q = e / EX_LINES, c = e % EX_LINES;
        double2 acc = make_double2(0.0, 0.0);
        for (int i = 0; i < W; ++i) {
            const double2 h = buf[((tv.q0 + i - q) & (Ng - 1)) * EX_LINES + c];
            acc.x += tv.wt[i] * h.x;
            acc.y += tv.wt[i] * h.y;
        }
        const double2 g = ok ? make_double2(acc.x * scale, acc.y * scale) : make_double2(0.0, 0.0);
        const int64_t at = (int64_t)q * Ng + qu0 + c;
        if (ENERGY) energy_out[(int64_t)b * Ng * Ng + at] = energy(g);
        else src[at] = g;
    }
}

// Count pass, per row: tau, kept count, sort key.  One workgroup of TNT threads per chunk member
// (visibility base + b): the 15 sums of a pass are a long dependent stream per lane, so many waves
// per row keep the CU busy.
template <int LOGNG>
__global__ __launch_bounds__(TNT) void k_exact_tau(const double *__restrict__ u, const double *__restrict__ v,
                                                    const double *__restrict__ w, const double *__restrict__ beam,
                                                    int64_t base, double cell, double E, const double *__restrict__ en,
                                                    double *__restrict__ tau_out, int *__restrict__ nnz_out,
                                                    int *__restrict__ key_out, int *__restrict__ fsz_out,
                                                    int *__restrict__ err) {
    constexpr int Ng = 1 << LOGNG;
    constexpr int64_t CELLS = (int64_t)Ng * Ng;
    constexpr int S = 16;                 // sub-brackets per pass
    __shared__ double redd[TNT / 64];
    __shared__ long long redl[TNT / 64];
    __shared__ int s_red_i[TNT / 64];
    __shared__ double s_acc[S];
    __shared__ double s_list[TAU_CAP];
    const int b = blockIdx.x;
    const int64_t k = base + b;
    double ut, vt, wk;
    if (!exact_coords(u, v, w, k, cell, Ng, ut, vt, wk) || !beam_ok(beam, k)) {
        if (threadIdx.x == 0) {
            atomicOr(err, 1);
            tau_out[k] = INFINITY;
            nnz_out[k] = 0;
            key_out[k] = 0;
            fsz_out[k] = 0;
        }
        return;
    }
    const double *m = en + (int64_t)b * CELLS;
    double tsum = 0.0, mmax = 0.0;
    for (int64_t i = threadIdx.x; i < CELLS; i += TNT) {
        tsum += m[i];
        mmax = fmax(mmax, m[i]);
    }
    const double T = tau_block_sum(tsum, redd);
    mmax = tau_block_max(mmax, redd);
    double tau;
    long long cnt;
    if (E >= 1.0) {
        tau = DBL_TRUE_MIN;                        // every non-zero entry
        long long c = 0;
        for (int64_t i = threadIdx.x; i < CELLS; i += TNT) c += m[i] >= tau;
        cnt = tau_block_sum(c, redl);
    } else {
        const double target = E * T;
        // bracket [lo, hi) with K(lo) >= target > K(hi), khi = K(hi)
        unsigned long long lo = 0ull, hi = (unsigned long long)__double_as_longlong(mmax) + 1ull;
        double khi = 0.0;
        // once the bracket holds at most TAU_CAP entries they are copied to LDS, and a pass reads
        // only them: K(c) = base + (sum of the copied entries >= c), base = K(hi) at the copy
        bool listed = false;
        int nlist = 0;
        double base = 0.0;
        long long base_n = 0;                      // #{m >= hi} at the copy
        while (hi - lo > 1ull) {
            const unsigned long long span = hi - lo;
            const int ns = span >= (unsigned long long)S ? S - 1 : (int)span - 1;   // interior points
            unsigned long long cand[S - 1];
#pragma unroll
            for (int s = 0; s < S - 1; ++s) {
                // lo + span (s + 1) / S without overflow, or lo + s + 1 for a short bracket
                cand[s] = span >= (unsigned long long)S
                              ? lo + (span / S) * (s + 1) + ((span % S) * (s + 1)) / S
                              : lo + (unsigned long long)(s + 1);
            }
            double acc[S - 1];
#pragma unroll
            for (int s = 0; s < S - 1; ++s) acc[s] = 0.0;
            // one loop for both sources (a generic pointer: LDS list or the row in global memory)
            const double *src = listed ? (const double *)s_list : m;
            const int64_t nsrc = listed ? (int64_t)nlist : CELLS;
            for (int64_t i = threadIdx.x; i < nsrc; i += TNT) {
                const double mi = src[i];
                const unsigned long long bits = (unsigned long long)__double_as_longlong(mi);
#pragma unroll
                for (int s = 0; s < S - 1; ++s) acc[s] += bits >= cand[s] ? mi : 0.0;
            }
            for (int s = 0; s < ns; ++s) {
                const double K = tau_block_sum(acc[s], redd);
                if (threadIdx.x == 0) s_acc[s] = base + K;
            }
            __syncthreads();
            // the largest candidate still holding the target, and the next one above it
            unsigned long long nlo = lo, nhi = hi;
            for (int s = 0; s < ns; ++s) {
                if (s_acc[s] >= target) {
                    nlo = cand[s];
                } else {
                    nhi = cand[s];
                    khi = s_acc[s];
                    break;
                }
            }
            __syncthreads();
            lo = nlo;
            hi = nhi;
            if (!listed && hi - lo > 1ull) {
                int in = 0, above = 0;
                for (int64_t i = threadIdx.x; i < CELLS; i += TNT) {
                    const unsigned long long bits = (unsigned long long)__double_as_longlong(m[i]);
                    in += bits >= lo && bits < hi;
                    above += bits >= hi;
                }
                int total;
                const int pos0 = tau_block_excl_scan(in, s_red_i, total);
                const long long n_above = tau_block_sum((long long)above, redl);
                if (total <= TAU_CAP) {
                    // ordered copy of the entries in [lo, hi) (the order fixes the sums' rounding)
                    int pos = pos0;
                    for (int64_t i = threadIdx.x; i < CELLS; i += TNT) {
                        const double mi = m[i];
                        const unsigned long long bits = (unsigned long long)__double_as_longlong(mi);
                        if (bits >= lo && bits < hi) s_list[pos++] = mi;
                    }
                    __syncthreads();
                    listed = true;
                    nlist = total;
                    base = khi;
                    base_n = n_above;
                }
            }
        }
        tau = __longlong_as_double((long long)lo);
        // #{m >= tau}
        long long c = 0;
        if (listed) {
            for (int i = threadIdx.x; i < nlist; i += TNT) c += s_list[i] >= tau;
        } else {
            for (int64_t i = threadIdx.x; i < CELLS; i += TNT) c += m[i] >= tau;
        }
        cnt = (listed ? base_n : 0) + tau_block_sum(c, redl);
    }
    if (threadIdx.x == 0) {
        tau_out[k] = tau;
        nnz_out[k] = (int)cnt;
        fsz_out[k] = 0;                            // no factor records: the rows are not separable
        const int cu = min(max((int)floor(ut + Ng / 2), 0), Ng - 1);
        const int cv = min(max((int)floor(vt + Ng / 2), 0), Ng - 1);
        key_out[k] = morton2(cv, cu);
    }
}

// Fill pass, per sorted row r = base + b: the kept entries in ascending flattened column.
template <int LOGNG, int TK>
__global__ __launch_bounds__(BNTH) void k_exact_fill(const double2 *__restrict__ rows, int64_t base,
                                                     const double *__restrict__ tau_in, const int *__restrict__ perm,
                                                     const int64_t *__restrict__ rowptr, int *__restrict__ col,
                                                     void *__restrict__ val, float *__restrict__ rscale,
                                                     int *__restrict__ err) {
    constexpr int Ng = 1 << LOGNG;
    constexpr int64_t CELLS = (int64_t)Ng * Ng;
    constexpr int PER = 4;                          // consecutive entries per thread per tile
    constexpr int TILE = BNTH * PER;
    __shared__ double redd[BNTH / 64];
    __shared__ int redi[BNTH / 64];
    const int b = blockIdx.x;
    const int64_t r = base + b;
    const int k = perm[r];
    const double tau = tau_in[k];
    const int64_t beg = rowptr[r], len = rowptr[r + 1] - beg;
    const double2 *g = rows + (int64_t)b * CELLS;
    double i16_scale = 1.0;
    if (TK == WP_TAPS_I16) {
        // int16 block floating point: every entry |g| <= sqrt(max |g|^2)
        double mmax = 0.0;
        for (int64_t i = threadIdx.x; i < CELLS; i += BNTH) mmax = fmax(mmax, energy(g[i]));
        mmax = block_max(mmax, redd);
        i16_scale = sqrt(mmax) / 32767.0;
        if (threadIdx.x == 0) rscale[r] = (float)i16_scale;
    }
    if (len == 0) return;
    int64_t pos = beg;
    for (int64_t t0 = 0; t0 < CELLS; t0 += TILE) {
        double2 gv[PER];
        int c = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int64_t q = t0 + threadIdx.x * PER + i;
            gv[i] = g[q];
            c += energy(gv[i]) >= tau;
        }
        int total;
        int64_t p = pos + block_excl_scan(c, redi, total);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int64_t q = t0 + threadIdx.x * PER + i;
            if (energy(gv[i]) >= tau) {
                if (p < beg + len) {
                    col[p] = (int)q;
                    if (TK == WP_TAPS_BF16) ((uint32_t *)val)[p] = pack_bf16x2((float)gv[i].x, (float)gv[i].y);
                    else if (TK == WP_TAPS_I16)
                        ((uint32_t *)val)[p] = pack_i16x2((float)(gv[i].x / i16_scale), (float)(gv[i].y / i16_scale));
                    else ((float2 *)val)[p] = make_float2((float)gv[i].x, (float)gv[i].y);
                }
                ++p;
            }
        }
        pos += total;
    }
    if (threadIdx.x == 0 && pos - beg != len) atomicOr(err, 2);
}

}  // namespace
