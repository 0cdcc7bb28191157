// Builder of the sparse w-projection matrix G (Sections 3.1 and 3.2).
//
// Row k of G, for a visibility at grid coordinates (u~, v~) with component w:
//   1. chirp exp(i pi w l^2) sampled on the padded grid, l = t delta,
//      t in [-Ng/2, Ng/2); phase argument w delta^2 t^2 in FP64 (sincospi);
//   2. its 1-D spectrum h(d) = Ng^-1 sum_t c(t) exp(-2 pi i t d / Ng) (FP64 FFT
//      in LDS).  The linear chirp and the KB window are both separable, so the
//      2-D row is g(q_v, q_u) = g_v(q_v) g_u(q_u) exactly, with
//   3. g_u(q) = sum_i KB(u~ - q'_i) h((q'_i - q) mod Ng) over the W window cells
//      q'_i (u~ - q'_i in [-W/2, W/2)), KB(t) = I0(beta sqrt(1 - (2t/W)^2));
//   4. energies A_a = |g_u(a)|^2, B_b = |g_v(b)|^2; a tap's energy is A_a B_b.
//      Threshold tau = the largest value with K(tau) >= E T, where K(tau) sums
//      the tap energies >= tau and T = K(0) (Section 3.2: keep a fraction E of
//      the row energy).  tau is found by bisection on the IEEE-754 bit pattern
//      of non-negative doubles (monotone), 64 steps at most; with B sorted
//      descending and its prefix sums, K(tau) = sum_a A_a PB[#{b: A_a B_b >= tau}]
//      costs O(Ng log Ng).  The bisection converges to a tap energy, so the kept
//      set {A_a B_b >= tau} (ties kept) is the sort-defined set.  E >= 1 keeps
//      every non-zero tap.
//   5. CSR: rows are sorted by the Z-order code of their centre cell (stable radix
//      sort made of 1-bit stable partitions; every aligned 32 x 32 tile of cells is
//      then a contiguous range of rows), row lengths are scanned into int64 offsets,
//      and the fill pass writes each row's taps in ascending flattened column
//      q_v Ng + q_u, values g_v g_u rounded to complex float32 (or bf16 pairs).
// Pass 1 (count) computes tau, row lengths, the tile sort, the offsets and the
// adjoint work list sizes; pass 2 (fill) recomputes the row factors and writes
// the taps.
#include <cfloat>
#include <climits>
#include <cstdio>

#include "builder_exact.h"
#include "builder_lowrank.h"
#include "builder_util.h"
#include "fft_lds.h"

namespace {

constexpr int ROWS_PER_ITEM = 32;
constexpr int64_t ROW_CHUNK = 1 << 22;     // rows per launch of the per-row kernels

// Row setup shared by both passes: chirp, FFT, window taps.  h must hold Ng double2.
template <int LOGNG>
__device__ inline void chirp_spectrum(double2 *h, double wk, double delta, const double2 *tw64) {
    constexpr int Ng = 1 << LOGNG;
    const double a = wk * delta * delta;
    for (int i = threadIdx.x; i < Ng; i += BNTH) {
        const double t = (double)(i < Ng / 2 ? i : i - Ng);
        double sn, cs;
        sincospi(a * t * t, &sn, &cs);       // exp(i pi w delta^2 t^2)
        h[i] = make_double2(cs, sn);
    }
    __syncthreads();
    lds_fft<double2, LOGNG, 1, BNTH, true, Ng>(h, tw64, false, threadIdx.x);
}

// K(tau): energy and count of taps with A_a B_b >= tau.  Bs sorted descending,
// PB[i] = sum of the first i entries of Bs.
template <int LOGNG>
__device__ inline void kept_energy(const double *A, const double *Bs, const double *PB, double tau,
                                   double &K, long long &cnt, double *redd, long long *redl) {
    constexpr int Ng = 1 << LOGNG;
    double k = 0.0;
    long long c = 0;
    for (int a = threadIdx.x; a < Ng; a += BNTH) {
        const double Aa = A[a];
        if (!(Aa * Bs[0] >= tau)) continue;
        int lo = 1, hi = Ng;                 // largest n with Aa * Bs[n-1] >= tau
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (Aa * Bs[mid - 1] >= tau) lo = mid; else hi = mid - 1;
        }
        k += Aa * PB[lo];
        c += lo;
    }
    K = block_sum(k, redd);
    cnt = block_sum(c, redl);
}

// ---------------------------------------------------------------------------- pass 1: threshold and count

template <int LOGNG>
__global__ __launch_bounds__(BNTH) void k_row_count(const double *__restrict__ u, const double *__restrict__ v,
                                                    const double *__restrict__ w, int64_t M, double E,
                                                    double cell, double delta, int W, double beta, int tile,
                                                    int ntile, const double2 *__restrict__ tw64,
                                                    double *__restrict__ tau_out, int *__restrict__ nnz_out,
                                                    int *__restrict__ key_out, int *__restrict__ fsz_out,
                                                    int *__restrict__ err, int64_t r0) {
    constexpr int Ng = 1 << LOGNG;
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *h = (double2 *)smem;                 // Ng double2, later PB (Ng+1 doubles)
    double *A = (double *)(smem + 16 * Ng);       // Ng
    double *B = A + Ng;                           // Ng (sorted descending in place)
    double *PB = (double *)smem;
    __shared__ double redd[BNTH / 64];
    __shared__ long long redl[BNTH / 64];
    __shared__ int redi[BNTH / 64];
    __shared__ double s_wu[16], s_wv[16];

    const int64_t k = r0 + blockIdx.x;
    const double ut = u[k] / cell, vt = v[k] / cell, wk = w[k];
    const bool ok = isfinite(ut) && isfinite(vt) && isfinite(wk) && fabs(ut) < Ng / 2 && fabs(vt) < Ng / 2;
    if (!ok) {
        if (threadIdx.x == 0) {
            atomicOr(err, 1);
            tau_out[k] = INFINITY;
            nnz_out[k] = 0;
            key_out[k] = 0;
            fsz_out[k] = factor_record_bytes(0, 0);
        }
        return;
    }
    const Taps tu = kb_taps(ut, W, beta, Ng, s_wu);
    const Taps tv = kb_taps(vt, W, beta, Ng, s_wv);
    chirp_spectrum<LOGNG>(h, wk, delta, tw64);        // ends with a barrier: the weights are visible
    for (int q = threadIdx.x; q < Ng; q += BNTH) {
        const double2 gu = row_factor(h, tu, W, q, Ng);
        const double2 gv = row_factor(h, tv, W, q, Ng);
        A[q] = energy(gu);
        B[q] = energy(gv);
    }
    __syncthreads();
    // bitonic sort of B, descending
    for (int kk = 2; kk <= Ng; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < Ng; i += BNTH) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const double x0 = B[i], x1 = B[ixj];
                    const bool desc = (i & kk) == 0;
                    if (desc ? (x0 < x1) : (x0 > x1)) { B[i] = x1; B[ixj] = x0; }
                }
            }
            __syncthreads();
        }
    }
    // prefix sums of the sorted B (sequential per wave chunk: Ng values, 256 threads)
    {
        constexpr int PER = (Ng + BNTH - 1) / BNTH;
        double loc[PER];
        double s = 0.0;
        const int b0 = threadIdx.x * PER;
        for (int i = 0; i < PER; ++i) {
            loc[i] = (b0 + i < Ng) ? B[b0 + i] : 0.0;
            s += loc[i];
        }
        // exclusive scan of s across the block (FP64)
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        double x = s;
        for (int o = 1; o < 64; o <<= 1) {
            double y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        __syncthreads();
        if (lane == 63) redd[wid] = x;
        __syncthreads();
        double off = 0.0;
        for (int i = 0; i < wid; ++i) off += redd[i];
        double run = off + x - s;
        __syncthreads();
        for (int i = 0; i < PER; ++i) {
            if (b0 + i < Ng) PB[b0 + i] = run;
            run += loc[i];
        }
        if (b0 + PER == Ng) PB[Ng] = run;
        __syncthreads();
    }
    double T;
    long long cnt;
    kept_energy<LOGNG>(A, B, PB, 0.0, T, cnt, redd, redl);
    double tau;
    if (E >= 1.0) {
        tau = DBL_TRUE_MIN;                        // every non-zero tap
    } else {
        double amax = 0.0;
        for (int a = threadIdx.x; a < Ng; a += BNTH) amax = fmax(amax, A[a]);
        amax = block_max(amax, redd);
        const double target = E * T;
        unsigned long long lo = 0ull;
        unsigned long long hi = (unsigned long long)__double_as_longlong(amax * B[0]) + 1ull;
        while (hi - lo > 1ull) {
            const unsigned long long mid = lo + ((hi - lo) >> 1);
            double Km;
            long long cm;
            kept_energy<LOGNG>(A, B, PB, __longlong_as_double((long long)mid), Km, cm, redd, redl);
            if (Km >= target) lo = mid; else hi = mid;
        }
        tau = __longlong_as_double((long long)lo);
    }
    double Kt;
    kept_energy<LOGNG>(A, B, PB, tau, Kt, cnt, redd, redl);
    // candidates of the factor record, with the fill pass's expressions: u cells with A_a bmax >= tau,
    // v cells with amax B_b >= tau (B is sorted: B[0] = bmax)
    double amax = 0.0;
    for (int a = threadIdx.x; a < Ng; a += BNTH) amax = fmax(amax, A[a]);
    amax = block_max(amax, redd);
    const double bmax = B[0];
    int na = 0, nb = 0;
    for (int q = threadIdx.x; q < Ng; q += BNTH) {
        na += (A[q] * bmax >= tau);
        nb += (amax * B[q] >= tau);
    }
    na = block_sum(na, redi);
    nb = block_sum(nb, redi);
    if (threadIdx.x == 0) {
        tau_out[k] = tau;
        nnz_out[k] = (int)cnt;
        fsz_out[k] = factor_record_bytes(na, nb);
        // rows are sorted by the Z-order code of their centre cell (tiles of the scatter are then
        // contiguous ranges, and rows close in the uv plane are close in memory)
        const int cu = min(max((int)floor(ut + Ng / 2), 0), Ng - 1);
        const int cv = min(max((int)floor(vt + Ng / 2), 0), Ng - 1);
        key_out[k] = morton2(cv, cu);
        (void)tile;
        (void)ntile;
        (void)redi;
    }
}

// ---------------------------------------------------------------------------- pass 2: fill

template <int LOGNG, int TK>
__global__ __launch_bounds__(BNTH) void k_row_fill(const double *__restrict__ u, const double *__restrict__ v,
                                                   const double *__restrict__ w, int64_t M,
                                                   double cell, double delta, int W, double beta,
                                                   const double2 *__restrict__ tw64, const double *__restrict__ tau_in,
                                                   const int *__restrict__ perm, const int64_t *__restrict__ rowptr,
                                                   int *__restrict__ col, void *__restrict__ val,
                                                   float *__restrict__ rscale, const int64_t *__restrict__ frec,
                                                   unsigned char *__restrict__ fdat, int *__restrict__ err, int64_t r0) {
    constexpr int Ng = 1 << LOGNG;
    constexpr int PER = (Ng + BNTH - 1) / BNTH;
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *h = (double2 *)smem;                 // Ng
    double *A = (double *)(smem + 16 * Ng);       // Ng energies along u (those along v are recomputed)
    int *off = (int *)(A + Ng);                   // Ng per-candidate-row output offsets
    uint16_t *ca = (uint16_t *)(off + Ng);        // Ng candidate columns (u)
    uint16_t *cb = ca + Ng;                       // Ng candidate rows (v)
    __shared__ double redd[BNTH / 64];
    __shared__ int redi[BNTH / 64];
    __shared__ int s_nca, s_ncb;
    __shared__ double s_wu[16], s_wv[16];

    const int64_t r = r0 + blockIdx.x;
    const int k = perm[r];
    const double tau = tau_in[k];
    const int64_t beg = rowptr[r], len = rowptr[r + 1] - beg;
    if (len == 0) {
        if (fdat && threadIdx.x == 0) *(uint2 *)(fdat + frec[r]) = make_uint2(0u, 0u);   // nu = nv = 0
        return;
    }
    const double ut = u[k] / cell, vt = v[k] / cell, wk = w[k];
    const Taps tu = kb_taps(ut, W, beta, Ng, s_wu);
    const Taps tv = kb_taps(vt, W, beta, Ng, s_wv);
    chirp_spectrum<LOGNG>(h, wk, delta, tw64);        // ends with a barrier: the weights are visible
    double amax = 0.0, bmax = 0.0;
    double bq[PER];                                    // energies along v of this thread's cells q0 + i
    const int q0 = threadIdx.x * PER;
    for (int q = threadIdx.x; q < Ng; q += BNTH) {
        const double Aq = energy(row_factor(h, tu, W, q, Ng));
        A[q] = Aq;
        amax = fmax(amax, Aq);
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int q = q0 + i;
        bq[i] = q < Ng ? energy(row_factor(h, tv, W, q, Ng)) : 0.0;
        bmax = fmax(bmax, bq[i]);
    }
    amax = block_max(amax, redd);                      // its barriers also publish A
    bmax = block_max(bmax, redd);
    // int16 block floating point: every tap |g| <= sqrt(amax bmax), so re / s and im / s fit in +-32767
    const double i16_scale = sqrt(amax * bmax) / 32767.0;
    if (TK == WP_TAPS_I16 && threadIdx.x == 0) rscale[r] = (float)i16_scale;
    // candidate compaction (ascending index); a kept tap needs A_a bmax >= tau and amax B_b >= tau
    {
        int na = 0, nb = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = q0 + i;
            if (q < Ng) {
                na += (A[q] * bmax >= tau);
                nb += (amax * bq[i] >= tau);
            }
        }
        int ta, tb;
        int oa = block_excl_scan(na, redi, ta);
        int ob = block_excl_scan(nb, redi, tb);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = q0 + i;
            if (q < Ng) {
                if (A[q] * bmax >= tau) ca[oa++] = (uint16_t)q;
                if (amax * bq[i] >= tau) cb[ob++] = (uint16_t)q;
            }
        }
        if (threadIdx.x == 0) { s_nca = ta; s_ncb = tb; }
        __syncthreads();
    }
    const int nca = s_nca, ncb = s_ncb;
    // kept taps per candidate row, then offsets
    {
        int cntl[PER];
        int tot = 0;
        for (int i = 0; i < PER; ++i) {
            const int ib = threadIdx.x * PER + i;
            int c = 0;
            if (ib < ncb) {
                const double Bb = energy(row_factor(h, tv, W, cb[ib], Ng));
                for (int ia = 0; ia < nca; ++ia) c += (A[ca[ia]] * Bb >= tau);
            }
            cntl[i] = c;
            tot += c;
        }
        int total;
        int o = block_excl_scan(tot, redi, total);
        for (int i = 0; i < PER; ++i) {
            const int ib = threadIdx.x * PER + i;
            if (ib < ncb) off[ib] = o;
            o += cntl[i];
        }
        if (threadIdx.x == 0 && total != len) atomicOr(err, 2);
        __syncthreads();
    }
    // factor record: candidates ranked by descending energy (ties by ascending cell); a v candidate's
    // kept u candidates are then the first nb of that order, nb = its tap count
    if (fdat) {
        unsigned char *rec = fdat + frec[r];
        const int nu = nca, nv = ncb;
        if ((int64_t)factor_record_bytes(nu, nv) != frec[r + 1] - frec[r]) {
            if (threadIdx.x == 0) atomicOr(err, 4);
        } else {
            uint16_t *ua = (uint16_t *)rec + 2, *vb = ua + nu, *nbv = vb + nv;
            const int vals = (4 + 2 * nu + 4 * nv + 7) & ~7;
            float2 *gu = (float2 *)(rec + vals), *gv = gu + nu;
            if (threadIdx.x == 0) {
                *(uint32_t *)rec = (uint32_t)nu | ((uint32_t)nv << 16);
                for (int z = 4 + 2 * nu + 4 * nv; z < vals; ++z) rec[z] = 0;
            }
            for (int ia = threadIdx.x; ia < nu; ia += BNTH) {
                const int a = ca[ia];
                const double Aa = A[a];
                int rank = 0;
                for (int j = 0; j < nu; ++j) {
                    const double Aj = A[ca[j]];
                    rank += (Aj > Aa) || (Aj == Aa && j < ia);
                }
                const double2 g = row_factor(h, tu, W, a, Ng);
                ua[rank] = (uint16_t)a;
                gu[rank] = make_float2((float)g.x, (float)g.y);
            }
            for (int ib = threadIdx.x; ib < nv; ib += BNTH) {
                const int b = cb[ib];
                const double2 g = row_factor(h, tv, W, b, Ng);
                const double Bb = energy(g);
                int rank = 0;
                for (int j = 0; j < nv; ++j) {
                    const double Bj = energy(row_factor(h, tv, W, cb[j], Ng));
                    rank += (Bj > Bb) || (Bj == Bb && j < ib);
                }
                vb[rank] = (uint16_t)b;
                nbv[rank] = (uint16_t)((ib + 1 < nv ? off[ib + 1] : (int)len) - off[ib]);
                gv[rank] = make_float2((float)g.x, (float)g.y);
            }
        }
    }
    if (!col) return;                                  // factor-record form: no stored taps
    // emit: one wave per candidate row, ballot-compacted, ascending a
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int ib = wid; ib < ncb; ib += BNTH / 64) {
        const int b = cb[ib];
        const double2 gv = row_factor(h, tv, W, b, Ng);
        const double Bb = energy(gv);
        int64_t pos = beg + off[ib];
        for (int ia0 = 0; ia0 < nca; ia0 += 64) {
            const int ia = ia0 + lane;
            int a = 0;
            bool keep = false;
            if (ia < nca) {
                a = ca[ia];
                keep = A[a] * Bb >= tau;
            }
            const unsigned long long m = __ballot(keep);
            if (keep) {
                const int rank = __popcll(m & ((1ull << lane) - 1ull));
                const double2 gu = row_factor(h, tu, W, a, Ng);
                const double2 g = cmul(gv, gu);
                const int64_t p = pos + rank;
                if (p < beg + len) {
                    col[p] = b * Ng + a;
                    if (TK == WP_TAPS_BF16) ((uint32_t *)val)[p] = pack_bf16x2((float)g.x, (float)g.y);
                    else if (TK == WP_TAPS_I16)
                        ((uint32_t *)val)[p] = pack_i16x2((float)(g.x / i16_scale), (float)(g.y / i16_scale));
                    else ((float2 *)val)[p] = make_float2((float)g.x, (float)g.y);
                }
            }
            pos += __popcll(m);
        }
    }
}

// ---------------------------------------------------------------------------- device-wide scan

constexpr int SCAN_NTH = 256, SCAN_IPT = 8, SCAN_TILE = SCAN_NTH * SCAN_IPT;

template <typename T>
__device__ inline T block_excl_scan_T(T v, T *red, T &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T x = v;
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) red[wid] = x;
    __syncthreads();
    T off = 0, tot = 0;
    for (int i = 0; i < SCAN_NTH / 64; ++i) {
        if (i < wid) off += red[i];
        tot += red[i];
    }
    total = tot;
    return off + x - v;
}

// out[i] = sum_{j<i} in[j] within each tile of SCAN_TILE; bsum[tile] = tile total
template <typename Tin, typename T>
__global__ __launch_bounds__(SCAN_NTH) void k_scan_tiles(const Tin *__restrict__ in, T *__restrict__ out, int64_t n,
                                                         T *__restrict__ bsum) {
    __shared__ T red[SCAN_NTH / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_IPT;
    T loc[SCAN_IPT];
    T s = 0;
    for (int i = 0; i < SCAN_IPT; ++i) {
        loc[i] = (base + i < n) ? (T)in[base + i] : (T)0;
        s += loc[i];
    }
    T total;
    T run = block_excl_scan_T(s, red, total);
    for (int i = 0; i < SCAN_IPT; ++i) {
        if (base + i < n) out[base + i] = run;
        run += loc[i];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(SCAN_NTH) void k_scan_add(T *__restrict__ out, int64_t n, const T *__restrict__ boff) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    const T o = boff[blockIdx.x];
    for (int i = threadIdx.x; i < SCAN_TILE; i += SCAN_NTH)
        if (base + i < n) out[base + i] += o;
}

template <typename T>
__global__ void k_put_total(T *__restrict__ out, int64_t n, const T *__restrict__ bsum_scanned, int64_t nb,
                            const T *__restrict__ bsum) {
    // out[n] = exclusive offset of the last tile + its total
    out[n] = bsum_scanned[nb - 1] + bsum[nb - 1];
}

int64_t scan_scratch_elems(int64_t n) {
    int64_t tot = 0;
    while (true) {
        int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
        tot += 2 * nb + 2;
        if (nb <= 1) break;
        n = nb;
    }
    return tot;
}

// Exclusive scan of n inputs into out[0..n], out[n] = total.  scratch holds scan_scratch_elems(n) T.
template <typename Tin, typename T>
void device_scan(const Tin *in, T *out, int64_t n, T *scratch, hipStream_t s) {
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    T *bsum = scratch, *boff = scratch + nb;
    hipLaunchKernelGGL((k_scan_tiles<Tin, T>), dim3(nb), dim3(SCAN_NTH), 0, s, in, out, n, bsum);
    if (nb > 1) {
        device_scan<T, T>(bsum, boff, nb, scratch + 2 * nb + 2, s);
        hipLaunchKernelGGL((k_scan_add<T>), dim3(nb), dim3(SCAN_NTH), 0, s, out, n, boff);
    } else {
        hipMemsetAsync(boff, 0, sizeof(T), s);
    }
    hipLaunchKernelGGL((k_put_total<T>), dim3(1), dim3(1), 0, s, out, n, boff, nb, bsum);
}

// ---------------------------------------------------------------------------- tile sort and layout kernels

__global__ void k_iota_keys(const int *__restrict__ key, int *__restrict__ k0, int *__restrict__ i0, int64_t M) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) { k0[i] = key[i]; i0[i] = (int)i; }
}

__global__ void k_bit_flags(const int *__restrict__ keys, int bit, int *__restrict__ flags, int64_t M) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) flags[i] = ((keys[i] >> bit) & 1) ? 0 : 1;
}

__global__ void k_split_scatter(const int *__restrict__ kin, const int *__restrict__ iin, const int *__restrict__ zpos,
                                int *__restrict__ kout, int *__restrict__ iout, int bit, int64_t M) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int Z = zpos[M];
    const int k = kin[i];
    const int d = ((k >> bit) & 1) ? (int)(Z + i - zpos[i]) : zpos[i];
    kout[d] = k;
    iout[d] = iin[i];
}

__global__ void k_gather_nnz(const int *__restrict__ perm, const int *__restrict__ nnz, int64_t *__restrict__ snnz,
                             int64_t M) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < M) snnz[r] = nnz[perm[r]];
}

// row range of every tile: the tile's Z-order code is the row key shifted by the tile's bits
__global__ void k_tile_bounds(const int *__restrict__ skey, int64_t M, int shift, int *__restrict__ tstart,
                              int *__restrict__ tend) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= M) return;
    const int k = skey[r] >> shift;
    if (r == 0 || (skey[r - 1] >> shift) != k) tstart[k] = (int)r;
    if (r == M - 1 || (skey[r + 1] >> shift) != k) tend[k] = (int)r + 1;
}

__global__ void k_tile_chunks(const int *__restrict__ tstart, const int *__restrict__ tend, int T,
                              int *__restrict__ nchunk) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < T) nchunk[t] = (tend[t] - tstart[t] + ROWS_PER_ITEM - 1) / ROWS_PER_ITEM;
}

__global__ void k_write_items(const int *__restrict__ tstart, const int *__restrict__ tend,
                              const int *__restrict__ choff, int T, int ntile, int *__restrict__ work) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const int s = tstart[t], e = tend[t];
    int it = choff[t];
    int tv, tu;
    demorton2(t, tv, tu);
    (void)ntile;
    for (int r = s; r < e; r += ROWS_PER_ITEM, ++it) {
        work[4 * it + 0] = tv;
        work[4 * it + 1] = tu;
        work[4 * it + 2] = r;
        work[4 * it + 3] = min(r + ROWS_PER_ITEM, e);
    }
}

// ---------------------------------------------------------------------------- transposed copy (gather form of G^H)

__global__ void k_t_count(const int *__restrict__ col, int64_t nnz, int *__restrict__ cnt) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nnz; j += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[col[j]], 1);
}

template <typename TapT>
__global__ void k_t_fill(const int64_t *__restrict__ rowptr, const int *__restrict__ col, const TapT *__restrict__ val,
                         const int *__restrict__ perm, int64_t M, const int64_t *__restrict__ tcolptr,
                         int *__restrict__ cur, int *__restrict__ trow, TapT *__restrict__ tval) {
    const int lane = threadIdx.x & 63;
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (r >= M) return;
    for (int64_t j = rowptr[r] + lane; j < rowptr[r + 1]; j += 64) {
        const int c = col[j];
        const int64_t pos = tcolptr[c] + atomicAdd(&cur[c], 1);
        trow[pos] = (int)r;
        tval[pos] = val[j];
    }
    (void)perm;
}

// order each cell's entries by sorted row index: a bitonic sort of (row, position) pairs in LDS, then
// the values moved with their rows (a row has at most one entry per cell, so the keys are distinct
// and the order is unique).  Cells of at most TS_CAP entries take one wavefront each, cells of up to
// TS_BIG one workgroup each, longer cells a thread each (shell sort in global memory).
constexpr int TS_CAP = 1024, TS_BIG = 4096;

// sort one cell's n entries (1 < n <= CAP) in LDS with the NT threads of a group; sync() orders the
// group's LDS accesses
template <typename TapT, int CAP, int NT, typename Sync>
__device__ inline void sort_cell(int64_t b, int n, int lt, int *key, unsigned short *pos, TapT *val,
                                 int *__restrict__ trow, TapT *__restrict__ tval, Sync sync) {
    int P = 2;
    while (P < n) P <<= 1;
    for (int i = lt; i < P; i += NT) {
        key[i] = i < n ? trow[b + i] : INT_MAX;  // padding sorts last
        pos[i] = (unsigned short)i;
        if (i < n) val[i] = tval[b + i];
    }
    sync();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lt; i < P; i += NT) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const int k0 = key[i], k1 = key[ixj];
                    if ((i & k) == 0 ? (k0 > k1) : (k0 < k1)) {
                        key[i] = k1;
                        key[ixj] = k0;
                        const unsigned short p0 = pos[i];
                        pos[i] = pos[ixj];
                        pos[ixj] = p0;
                    }
                }
            }
            sync();
        }
    }
    for (int i = lt; i < n; i += NT) {
        trow[b + i] = key[i];
        tval[b + i] = val[pos[i]];
    }
}

__global__ void k_zero_int(int *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// cells of at most TS_CAP entries: one wavefront each, four per workgroup; cells of TS_CAP + 1 ..
// TS_BIG entries are appended to big[] (count in *nbig) for k_t_sort_big
template <typename TapT>
__global__ __launch_bounds__(256) void k_t_sort_small(const int64_t *__restrict__ tcolptr, int64_t cells,
                                                      int *__restrict__ trow, TapT *__restrict__ tval,
                                                      int *__restrict__ big, int *__restrict__ nbig) {
    __shared__ int s_key[4][TS_CAP];
    __shared__ unsigned short s_pos[4][TS_CAP];
    __shared__ TapT s_val[4][TS_CAP];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + wv;
    if (c >= cells) return;                      // per wavefront: nothing below syncs the workgroup
    const int64_t b = tcolptr[c];
    const int n = (int)(tcolptr[c + 1] - b);
    if (n > TS_CAP) {
        if (n <= TS_BIG && lane == 0) big[atomicAdd(nbig, 1)] = (int)c;
        return;
    }
    if (n <= 1) return;
    sort_cell<TapT, TS_CAP, 64>(b, n, lane, s_key[wv], s_pos[wv], s_val[wv], trow, tval, [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    });
}

// the listed cells of TS_CAP + 1 .. TS_BIG entries: one workgroup per cell (workgroups loop over the list)
template <typename TapT>
__global__ __launch_bounds__(256) void k_t_sort_big(const int64_t *__restrict__ tcolptr, const int *__restrict__ big,
                                                    const int *__restrict__ nbig, int *__restrict__ trow,
                                                    TapT *__restrict__ tval) {
    __shared__ int s_key[TS_BIG];
    __shared__ unsigned short s_pos[TS_BIG];
    __shared__ TapT s_val[TS_BIG];
    const int nb = *nbig;
    for (int q = blockIdx.x; q < nb; q += gridDim.x) {
        const int64_t c = big[q];
        const int64_t b = tcolptr[c];
        const int n = (int)(tcolptr[c + 1] - b);
        sort_cell<TapT, TS_BIG, 256>(b, n, threadIdx.x, s_key, s_pos, s_val, trow, tval, [] { __syncthreads(); });
        __syncthreads();                         // the next cell reuses the arrays
    }
}

// the same order for the cells the LDS sorts leave (more than TS_BIG entries): shell sort, one
// thread per cell
template <typename TapT>
__global__ void k_t_sort(const int64_t *__restrict__ tcolptr, int64_t cells, int *__restrict__ trow,
                         TapT *__restrict__ tval) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const int64_t b = tcolptr[c];
    const int n = (int)(tcolptr[c + 1] - b);
    if (n <= TS_BIG) return;
    int *kr = trow + b;
    TapT *kv = tval + b;
    int gap = 1;
    while (gap < n / 3) gap = 3 * gap + 1;
    for (; gap > 0; gap /= 3) {
        for (int i = gap; i < n; ++i) {
            const int key = kr[i];
            const TapT vv = kv[i];
            int j = i;
            while (j >= gap && kr[j - gap] > key) {
                kr[j] = kr[j - gap];
                kv[j] = kv[j - gap];
                j -= gap;
            }
            kr[j] = key;
            kv[j] = vv;
        }
    }
}

// gather blocks: flag the cells that start a block ...
__global__ void k_gb_flags(const int64_t *__restrict__ tcolptr, int64_t cells, int ent, int *__restrict__ flag) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const int64_t slot = tcolptr[c] / ent + c / GB_CELLS;
    flag[c] = (c == 0 || slot != tcolptr[c - 1] / ent + (c - 1) / GB_CELLS) ? 1 : 0;
}

// ... and write (first cell, first entry) of block pos[c] for each of them; the pairs from the
// block count up to index n_tblk are (cells, nnz)
__global__ void k_gb_write(const int64_t *__restrict__ tcolptr, const int *__restrict__ flag,
                           const int *__restrict__ pos, int64_t cells, int64_t nnz, int64_t n_tblk,
                           int64_t *__restrict__ tblk) {
    const int64_t n = cells > n_tblk + 1 ? cells : n_tblk + 1;
    const int64_t total = pos[cells];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < cells && flag[i]) {
            const int64_t b = pos[i];
            tblk[2 * b] = i;
            tblk[2 * b + 1] = tcolptr[i];
        }
        if (i >= total && i <= n_tblk) {
            tblk[2 * i] = cells;
            tblk[2 * i + 1] = nnz;
        }
    }
}

inline int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }

struct WsLayout {
    int64_t tau, nnz, key, k0, k1, i0, i1, flags, zpos, snnz, rowptr, sc32, sc64, tstart, tend, nch, choff, err,
        tcnt, sc64t, gpos, fsz, frec, ex, total;
};

// rows2d: the rows are made whole in 2-D (the exact chirp, or a beam per visibility)
WsLayout ws_layout(const wp_plan *p, int64_t M, bool rows2d) {
    const int64_t T = (int64_t)p->ntile * p->ntile;
    WsLayout L;
    int64_t o = 0;
    auto take = [&](int64_t bytes) { int64_t r = o; o += align256(bytes); return r; };
    L.tau = take(8 * M);
    L.nnz = take(4 * M);
    L.key = take(4 * M);
    L.k0 = take(4 * M);
    L.k1 = take(4 * M);
    L.i0 = take(4 * M);
    L.i1 = take(4 * M);
    L.flags = take(4 * M);
    L.zpos = take(4 * (M + 1));
    L.snnz = take(8 * M);
    L.rowptr = take(8 * (M + 1));
    L.sc32 = take(4 * scan_scratch_elems(M > T ? M : T));
    L.sc64 = take(8 * scan_scratch_elems(M));
    L.tstart = take(4 * T);
    L.tend = take(4 * T);
    L.nch = take(4 * T);
    L.choff = take(4 * (T + 1));
    L.err = take(16);
    const int64_t cells = (int64_t)p->Ng * p->Ng;
    L.tcnt = take(4 * cells);
    L.sc64t = take(8 * scan_scratch_elems(cells));
    L.gpos = take(4 * (cells + 1));
    L.fsz = take(4 * M);
    L.frec = take(8 * (M + 1));
    // the exact chirp's 2-D rows of one chunk (values, or energies in the count pass)
    L.ex = take(rows2d && p->Ng <= EXACT_MAX_NG ? EX_ROW_BYTES_PER_CELL * exact_chunk_rows(p->Ng, M) * p->Ng * p->Ng
                                                : 0);
    L.total = o;
    return L;
}

// the exact chirp's rows come from the separable expansion above Ng = 512, or when the plan asks for it
// (no beam: a beam's rows stay whole in 2-D)
inline bool exact_lowrank(const wp_plan *p, const double *beam) {
    if (beam || p->chirp != WP_CHIRP_EXACT) return false;
    return p->exact_rows == 1 || (p->exact_rows == 0 && p->Ng > EXACT_MAX_NG);
}

template <int LOGNG>
size_t count_lds() { return (size_t)32 << LOGNG; }
template <int LOGNG>
size_t fill_lds() { return (size_t)32 << LOGNG; }

template <int LOGNG>
wp_status count_rows(const wp_plan *p, int64_t M, const double *u, const double *v, const double *w, double E,
                     unsigned char *ws, const WsLayout &L, hipStream_t s) {
    const size_t lds = count_lds<LOGNG>();
    if (lds > 160 * 1024) return wp_set_error(WP_EUNSUPPORTED, "build: Ng = %d exceeds the LDS budget", p->Ng);
    // one workgroup per row, in launches of at most ROW_CHUNK rows (a grid dimension holds
    // fewer than 2^32 work-items)
    for (int64_t r0 = 0; r0 < M; r0 += ROW_CHUNK) {
        const int64_t n = std::min<int64_t>(ROW_CHUNK, M - r0);
        hipLaunchKernelGGL((k_row_count<LOGNG>), dim3((unsigned)n), dim3(BNTH), lds, s, u, v, w, M, E, p->cell,
                           p->delta, p->W, p->beta, p->tile, p->ntile, p->tw64, (double *)(ws + L.tau),
                           (int *)(ws + L.nnz), (int *)(ws + L.key), (int *)(ws + L.fsz), (int *)(ws + L.err), r0);
    }
    return wp_check_launch("build_G_count rows");
}

template <int LOGNG>
wp_status fill_rows(const wp_plan *p, int64_t M, const double *u, const double *v, const double *w,
                    const unsigned char *ws, const WsLayout &L, wp_G *G, hipStream_t s) {
    const size_t lds = fill_lds<LOGNG>();
    if (lds > 160 * 1024) return wp_set_error(WP_EUNSUPPORTED, "build: Ng = %d exceeds the LDS budget", p->Ng);
    int *err = (int *)(ws + L.err);
    const bool rec = G->frec && G->fdat;
    const int64_t *frec = rec ? (const int64_t *)(ws + L.frec) : nullptr;
    unsigned char *fdat = rec ? (unsigned char *)G->fdat : nullptr;
    for (int64_t r0 = 0; r0 < M; r0 += ROW_CHUNK) {
        const dim3 g((unsigned)std::min<int64_t>(ROW_CHUNK, M - r0));
        if (G->taps == WP_TAPS_BF16)
            hipLaunchKernelGGL((k_row_fill<LOGNG, WP_TAPS_BF16>), g, dim3(BNTH), lds, s, u, v, w, M, p->cell,
                               p->delta, p->W, p->beta, p->tw64, (const double *)(ws + L.tau), G->perm, G->rowptr,
                               G->col, G->val, G->rscale, frec, fdat, err, r0);
        else if (G->taps == WP_TAPS_I16)
            hipLaunchKernelGGL((k_row_fill<LOGNG, WP_TAPS_I16>), g, dim3(BNTH), lds, s, u, v, w, M, p->cell,
                               p->delta, p->W, p->beta, p->tw64, (const double *)(ws + L.tau), G->perm, G->rowptr,
                               G->col, G->val, G->rscale, frec, fdat, err, r0);
        else
            hipLaunchKernelGGL((k_row_fill<LOGNG, WP_TAPS_C64>), g, dim3(BNTH), lds, s, u, v, w, M, p->cell,
                               p->delta, p->W, p->beta, p->tw64, (const double *)(ws + L.tau), G->perm, G->rowptr,
                               G->col, G->val, G->rscale, frec, fdat, err, r0);
    }
    return wp_check_launch("build_G_fill rows");
}

template <int LOGNG>
wp_status count_rows_exact(const wp_plan *p, int64_t M, const double *u, const double *v, const double *w,
                           const double *beam, double E, unsigned char *ws, const WsLayout &L, hipStream_t s) {
    const int exact = p->chirp == WP_CHIRP_EXACT;
    constexpr int Ng = 1 << LOGNG;
    const int64_t B = exact_chunk_rows(Ng, M);
    double2 *rows = (double2 *)(ws + L.ex);
    double *en = (double *)(rows + B * Ng * Ng);       // energies beside the values
    for (int64_t k0 = 0; k0 < M; k0 += B) {
        const unsigned nb = (unsigned)std::min<int64_t>(B, M - k0);
        hipLaunchKernelGGL((k_exact_rows<LOGNG>), dim3(Ng / EX_LINES, nb), dim3(BNTH), 0, s, u, v, w, beam, exact,
                           nullptr, k0, p->cell, p->delta, p->W, p->beta, p->tw64, rows);
        hipLaunchKernelGGL((k_exact_cols<LOGNG, true>), dim3(Ng / EX_LINES, nb), dim3(BNTH), 0, s, u, v, w, beam,
                           nullptr, k0, p->cell, p->beta, p->W, p->tw64, rows, en);
        hipLaunchKernelGGL((k_exact_tau<LOGNG>), dim3(nb), dim3(TNT), 0, s, u, v, w, beam, k0, p->cell, E,
                           (const double *)en, (double *)(ws + L.tau), (int *)(ws + L.nnz), (int *)(ws + L.key),
                           (int *)(ws + L.fsz), (int *)(ws + L.err));
    }
    return wp_check_launch("build_G_count exact rows");
}

// the exact chirp's rows from the separable expansion (builder_lowrank.h): one workgroup per row
template <int LOGNG>
wp_status lowrank_rows(const wp_plan *p, int64_t M, const double *u, const double *v, const double *w, double E,
                       unsigned char *ws, const WsLayout &L, const wp_G *G, hipStream_t s) {
    constexpr size_t lds = lowrank_lds<LOGNG>();
    static_assert(lds <= 160 * 1024, "LDS budget");
    const double L2 = p->L * p->L;
    for (int64_t r0 = 0; r0 < M; r0 += ROW_CHUNK) {
        const dim3 g((unsigned)std::min<int64_t>(ROW_CHUNK, M - r0));
        if (!G)
            hipLaunchKernelGGL((k_lowrank_rows<LOGNG, false, WP_TAPS_C64>), g, dim3(BNTH), lds, s, u, v, w, E, p->cell,
                               p->delta, p->W, p->beta, L2, p->tw64, r0, nullptr, (double *)(ws + L.tau),
                               (int *)(ws + L.nnz), (int *)(ws + L.key), (int *)(ws + L.fsz), nullptr, nullptr,
                               nullptr, nullptr, (int *)(ws + L.err));
        else if (G->taps == WP_TAPS_BF16)
            hipLaunchKernelGGL((k_lowrank_rows<LOGNG, true, WP_TAPS_BF16>), g, dim3(BNTH), lds, s, u, v, w, E, p->cell,
                               p->delta, p->W, p->beta, L2, p->tw64, r0, G->perm, (double *)(ws + L.tau), nullptr,
                               nullptr, nullptr, G->rowptr, G->col, G->val, G->rscale, (int *)(ws + L.err));
        else if (G->taps == WP_TAPS_I16)
            hipLaunchKernelGGL((k_lowrank_rows<LOGNG, true, WP_TAPS_I16>), g, dim3(BNTH), lds, s, u, v, w, E, p->cell,
                               p->delta, p->W, p->beta, L2, p->tw64, r0, G->perm, (double *)(ws + L.tau), nullptr,
                               nullptr, nullptr, G->rowptr, G->col, G->val, G->rscale, (int *)(ws + L.err));
        else
            hipLaunchKernelGGL((k_lowrank_rows<LOGNG, true, WP_TAPS_C64>), g, dim3(BNTH), lds, s, u, v, w, E, p->cell,
                               p->delta, p->W, p->beta, L2, p->tw64, r0, G->perm, (double *)(ws + L.tau), nullptr,
                               nullptr, nullptr, G->rowptr, G->col, G->val, G->rscale, (int *)(ws + L.err));
    }
    return wp_check_launch(G ? "build_G_fill exact rows (separable expansion)" : "build_G_count exact rows (separable expansion)");
}

template <int LOGNG>
wp_status fill_rows_exact(const wp_plan *p, int64_t M, const double *u, const double *v, const double *w,
                          const double *beam, const unsigned char *ws, const WsLayout &L, wp_G *G, hipStream_t s) {
    const int exact = p->chirp == WP_CHIRP_EXACT;
    constexpr int Ng = 1 << LOGNG;
    const int64_t B = exact_chunk_rows(Ng, M);
    double2 *rows = (double2 *)(const_cast<unsigned char *>(ws) + L.ex);    // scratch region of the workspace
    const double *tau = (const double *)(ws + L.tau);
    int *err = (int *)(const_cast<unsigned char *>(ws) + L.err);
    for (int64_t r0 = 0; r0 < M; r0 += B) {
        const unsigned nb = (unsigned)std::min<int64_t>(B, M - r0);
        hipLaunchKernelGGL((k_exact_rows<LOGNG>), dim3(Ng / EX_LINES, nb), dim3(BNTH), 0, s, u, v, w, beam, exact,
                           G->perm, r0, p->cell, p->delta, p->W, p->beta, p->tw64, rows);
        hipLaunchKernelGGL((k_exact_cols<LOGNG, false>), dim3(Ng / EX_LINES, nb), dim3(BNTH), 0, s, u, v, w, beam,
                           G->perm, r0, p->cell, p->beta, p->W, p->tw64, rows, nullptr);
        if (G->taps == WP_TAPS_BF16)
            hipLaunchKernelGGL((k_exact_fill<LOGNG, WP_TAPS_BF16>), dim3(nb), dim3(BNTH), 0, s, rows, r0, tau,
                               G->perm, G->rowptr, G->col, G->val, G->rscale, err);
        else if (G->taps == WP_TAPS_I16)
            hipLaunchKernelGGL((k_exact_fill<LOGNG, WP_TAPS_I16>), dim3(nb), dim3(BNTH), 0, s, rows, r0, tau,
                               G->perm, G->rowptr, G->col, G->val, G->rscale, err);
        else
            hipLaunchKernelGGL((k_exact_fill<LOGNG, WP_TAPS_C64>), dim3(nb), dim3(BNTH), 0, s, rows, r0, tau,
                               G->perm, G->rowptr, G->col, G->val, G->rscale, err);
    }
    return wp_check_launch("build_G_fill exact rows");
}

}  // namespace

static int64_t al256(int64_t b) { return (b + 255) & ~(int64_t)255; }

int64_t scan_workspace_bytes(int64_t n) { return al256(4 * scan_scratch_elems(n)); }

wp_status launch_scan_int(const int *in, int *out, int64_t n, void *ws, hipStream_t s) {
    if (n <= 0) return wp_set_error(WP_EINVAL, "scan of %lld elements", (long long)n);
    device_scan<int, int>(in, out, n, (int *)ws, s);
    return wp_check_launch("scan");
}

int64_t sort_workspace_bytes(int64_t n) {
    return 4 * al256(4 * (n + 1)) + scan_workspace_bytes(n);
}

wp_status launch_sort_pairs(const int *key, int64_t n, int bits, int *keys_out, int *idx_out, void *wsv,
                            hipStream_t s) {
    if (n <= 0) return wp_set_error(WP_EINVAL, "sort of %lld elements", (long long)n);
    if (bits < 1 || bits > 31) return wp_set_error(WP_EINVAL, "sort of %d key bits", bits);
    unsigned char *ws = (unsigned char *)wsv;
    const int64_t blk = al256(4 * (n + 1));
    int *k1 = (int *)ws, *i1 = (int *)(ws + blk), *flags = (int *)(ws + 2 * blk), *zpos = (int *)(ws + 3 * blk);
    int *scratch = (int *)(ws + 4 * blk);
    int *k0 = keys_out, *i0 = idx_out;
    const dim3 g((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_iota_keys, g, dim3(256), 0, s, key, k0, i0, n);
    const int passes = bits + (bits & 1);     // even: the result ends in keys_out / idx_out
    for (int b = 0; b < passes; ++b) {
        hipLaunchKernelGGL(k_bit_flags, g, dim3(256), 0, s, k0, b, flags, n);
        device_scan<int, int>(flags, zpos, n, scratch, s);
        hipLaunchKernelGGL(k_split_scatter, g, dim3(256), 0, s, k0, i0, zpos, k1, i1, b, n);
        int *t = k0; k0 = k1; k1 = t;
        t = i0; i0 = i1; i1 = t;
    }
    return wp_check_launch("sort");
}

// every field sits at the same offset whatever rows2d says: the 2-D rows' region is the last one
int64_t builder_workspace_bytes(const wp_plan *p, int64_t M, bool rows2d) { return ws_layout(p, M, rows2d).total; }

// offsets of the factor records in sorted row order (after the count pass) and their total
wp_status launch_build_factor_bytes(const wp_plan *p, int64_t M, void *wsv, int64_t *bytes, hipStream_t s) {
    unsigned char *ws = (unsigned char *)wsv;
    const WsLayout L = ws_layout(p, M, false);
    const int nthr = 256;
    const dim3 gM((unsigned)((M + nthr - 1) / nthr));
    hipLaunchKernelGGL(k_gather_nnz, gM, dim3(nthr), 0, s, (const int *)(ws + L.i0), (const int *)(ws + L.fsz),
                       (int64_t *)(ws + L.snnz), M);
    device_scan<int64_t, int64_t>((const int64_t *)(ws + L.snnz), (int64_t *)(ws + L.frec), M,
                                  (int64_t *)(ws + L.sc64), s);
    wp_status st = wp_check_launch("build factor offsets");
    if (st != WP_OK) return st;
    // the total also goes next to the error flags (the count pass clears them), where the fill pass
    // checks it against the caller's buffer
    WP_HIP(hipMemcpyAsync(ws + L.err + 8, ws + L.frec + 8 * M, 8, hipMemcpyDeviceToDevice, s));
    WP_HIP(hipMemcpyAsync(bytes, ws + L.frec + 8 * M, 8, hipMemcpyDeviceToHost, s));
    WP_HIP(hipStreamSynchronize(s));
    return WP_OK;
}

wp_status launch_build_count(const wp_plan *p, int64_t M, const double *u, const double *v, const double *w,
                             const double *beam, double E, void *wsv, int64_t *nnz_total, int64_t *nwork,
                             hipStream_t s) {
    unsigned char *ws = (unsigned char *)wsv;
    const bool rows2d = p->chirp == WP_CHIRP_EXACT || beam;
    const WsLayout L = ws_layout(p, M, rows2d);
    const int T = p->ntile * p->ntile;
    WP_HIP(hipMemsetAsync(ws + L.err, 0, 16, s));
    wp_status st;
    if (rows2d && exact_lowrank(p, beam)) {
        switch (p->logNg) {
            case 6: st = lowrank_rows<6>(p, M, u, v, w, E, ws, L, nullptr, s); break;
            case 7: st = lowrank_rows<7>(p, M, u, v, w, E, ws, L, nullptr, s); break;
            case 8: st = lowrank_rows<8>(p, M, u, v, w, E, ws, L, nullptr, s); break;
            case 9: st = lowrank_rows<9>(p, M, u, v, w, E, ws, L, nullptr, s); break;
            case 10: st = lowrank_rows<10>(p, M, u, v, w, E, ws, L, nullptr, s); break;
            case 11: st = lowrank_rows<11>(p, M, u, v, w, E, ws, L, nullptr, s); break;
            case 12: st = lowrank_rows<12>(p, M, u, v, w, E, ws, L, nullptr, s); break;
            default: return wp_set_error(WP_EUNSUPPORTED, "build: Ng = %d", p->Ng);
        }
    } else if (rows2d) {
        switch (p->logNg) {
            case 6: st = count_rows_exact<6>(p, M, u, v, w, beam, E, ws, L, s); break;
            case 7: st = count_rows_exact<7>(p, M, u, v, w, beam, E, ws, L, s); break;
            case 8: st = count_rows_exact<8>(p, M, u, v, w, beam, E, ws, L, s); break;
            case 9: st = count_rows_exact<9>(p, M, u, v, w, beam, E, ws, L, s); break;
            default: return wp_set_error(WP_EUNSUPPORTED, "build: 2-D rows need Ng <= %d (Ng = %d)",
                                         EXACT_MAX_NG, p->Ng);
        }
    } else switch (p->logNg) {
        case 6: st = count_rows<6>(p, M, u, v, w, E, ws, L, s); break;
        case 7: st = count_rows<7>(p, M, u, v, w, E, ws, L, s); break;
        case 8: st = count_rows<8>(p, M, u, v, w, E, ws, L, s); break;
        case 9: st = count_rows<9>(p, M, u, v, w, E, ws, L, s); break;
        case 10: st = count_rows<10>(p, M, u, v, w, E, ws, L, s); break;
        case 11: st = count_rows<11>(p, M, u, v, w, E, ws, L, s); break;
        case 12: st = count_rows<12>(p, M, u, v, w, E, ws, L, s); break;
        default: return wp_set_error(WP_EUNSUPPORTED, "build: Ng = %d", p->Ng);
    }
    if (st != WP_OK) return st;
    // stable sort of the rows by the Z-order code of their centre cell: one stable partition per key bit
    const int nthr = 256;
    const dim3 gM((unsigned)((M + nthr - 1) / nthr));
    int *k0 = (int *)(ws + L.k0), *k1 = (int *)(ws + L.k1), *i0 = (int *)(ws + L.i0), *i1 = (int *)(ws + L.i1);
    int *flags = (int *)(ws + L.flags), *zpos = (int *)(ws + L.zpos);
    hipLaunchKernelGGL(k_iota_keys, gM, dim3(nthr), 0, s, (const int *)(ws + L.key), k0, i0, M);
    const int bits = 2 * p->logNg;            // Z-order code of the centre cell
    for (int b = 0; b < bits; ++b) {
        hipLaunchKernelGGL(k_bit_flags, gM, dim3(nthr), 0, s, k0, b, flags, M);
        device_scan<int, int>(flags, zpos, M, (int *)(ws + L.sc32), s);
        hipLaunchKernelGGL(k_split_scatter, gM, dim3(nthr), 0, s, k0, i0, zpos, k1, i1, b, M);
        int *t = k0; k0 = k1; k1 = t;
        t = i0; i0 = i1; i1 = t;
    }
    // the sorted keys / permutation end in k0 / i0; keep them at the k0 / i0 slots
    if (bits & 1) {
        WP_HIP(hipMemcpyAsync(ws + L.k0, k0, 4 * M, hipMemcpyDeviceToDevice, s));
        WP_HIP(hipMemcpyAsync(ws + L.i0, i0, 4 * M, hipMemcpyDeviceToDevice, s));
    }
    const int *skey = (const int *)(ws + L.k0), *perm = (const int *)(ws + L.i0);
    hipLaunchKernelGGL(k_gather_nnz, gM, dim3(nthr), 0, s, perm, (const int *)(ws + L.nnz), (int64_t *)(ws + L.snnz), M);
    device_scan<int64_t, int64_t>((const int64_t *)(ws + L.snnz), (int64_t *)(ws + L.rowptr), M,
                                  (int64_t *)(ws + L.sc64), s);
    // adjoint work items: chunks of rows inside each tile
    WP_HIP(hipMemsetAsync(ws + L.tstart, 0, 4 * T, s));
    WP_HIP(hipMemsetAsync(ws + L.tend, 0, 4 * T, s));
    int tbits = 0;
    while ((1 << tbits) < p->tile) ++tbits;
    hipLaunchKernelGGL(k_tile_bounds, gM, dim3(nthr), 0, s, skey, M, 2 * tbits, (int *)(ws + L.tstart),
                       (int *)(ws + L.tend));
    const dim3 gT((unsigned)((T + nthr - 1) / nthr));
    hipLaunchKernelGGL(k_tile_chunks, gT, dim3(nthr), 0, s, (const int *)(ws + L.tstart), (const int *)(ws + L.tend),
                       T, (int *)(ws + L.nch));
    device_scan<int, int>((const int *)(ws + L.nch), (int *)(ws + L.choff), T, (int *)(ws + L.sc32), s);
    if ((st = wp_check_launch("build_G_count layout")) != WP_OK) return st;
    int64_t host_rowptr_end = 0;
    int host_items = 0, host_err = 0;
    WP_HIP(hipMemcpyAsync(&host_rowptr_end, ws + L.rowptr + 8 * M, 8, hipMemcpyDeviceToHost, s));
    WP_HIP(hipMemcpyAsync(&host_items, ws + L.choff + 4 * (int64_t)T, 4, hipMemcpyDeviceToHost, s));
    WP_HIP(hipMemcpyAsync(&host_err, ws + L.err, 4, hipMemcpyDeviceToHost, s));
    WP_HIP(hipStreamSynchronize(s));
    if (host_err & 1)
        return wp_set_error(WP_EINVAL, "build_G_count: a visibility has non-finite (u, v, w), lies outside the band "
                            "|u|,|v| < N/(2L)%s", beam ? " or has a beam that is not finite with sigma > 0" : "");
    if (host_err & 16)
        return wp_set_error(WP_EUNSUPPORTED, "build_G_count: an exact-chirp row spreads over more than %d cells "
                            "(the separable expansion's window); reduce w", LR_WMAX - 2 * LR_MARGIN);
    if (host_err & 8)
        return wp_set_error(WP_EHIP, "build_G_count: an exact-chirp row keeps entries outside its window");
    *nnz_total = host_rowptr_end;
    *nwork = host_items;
    return WP_OK;
}

wp_status launch_build_fill(const wp_plan *p, int64_t M, const double *u, const double *v, const double *w,
                            const double *beam, double E, const void *wsv, wp_G *G, hipStream_t s) {
    (void)E;
    unsigned char *ws = (unsigned char *)const_cast<void *>(wsv);
    const bool rows2d = p->chirp == WP_CHIRP_EXACT || beam;
    const WsLayout L = ws_layout(p, M, rows2d);
    const int T = p->ntile * p->ntile;
    WP_HIP(hipMemcpyAsync(G->rowptr, ws + L.rowptr, 8 * (M + 1), hipMemcpyDeviceToDevice, s));
    WP_HIP(hipMemcpyAsync(G->perm, ws + L.i0, 4 * M, hipMemcpyDeviceToDevice, s));
    if (G->frec && G->fdat) {
        int64_t total = 0;
        WP_HIP(hipMemcpyAsync(&total, ws + L.err + 8, 8, hipMemcpyDeviceToHost, s));
        WP_HIP(hipStreamSynchronize(s));
        if (total == 0 || total != G->fbytes)
            return wp_set_error(WP_EINVAL, "factor records: G->fbytes = %lld, the workspace holds %lld (call "
                                "wp_build_factor_bytes after wp_build_G_count)", (long long)G->fbytes, (long long)total);
        WP_HIP(hipMemcpyAsync(G->frec, ws + L.frec, 8 * (M + 1), hipMemcpyDeviceToDevice, s));
    }
    wp_status st;
    if (rows2d && exact_lowrank(p, beam)) {
        switch (p->logNg) {
            case 6: st = lowrank_rows<6>(p, M, u, v, w, E, ws, L, G, s); break;
            case 7: st = lowrank_rows<7>(p, M, u, v, w, E, ws, L, G, s); break;
            case 8: st = lowrank_rows<8>(p, M, u, v, w, E, ws, L, G, s); break;
            case 9: st = lowrank_rows<9>(p, M, u, v, w, E, ws, L, G, s); break;
            case 10: st = lowrank_rows<10>(p, M, u, v, w, E, ws, L, G, s); break;
            case 11: st = lowrank_rows<11>(p, M, u, v, w, E, ws, L, G, s); break;
            case 12: st = lowrank_rows<12>(p, M, u, v, w, E, ws, L, G, s); break;
            default: return wp_set_error(WP_EUNSUPPORTED, "build: Ng = %d", p->Ng);
        }
    } else if (rows2d) {
        switch (p->logNg) {
            case 6: st = fill_rows_exact<6>(p, M, u, v, w, beam, ws, L, G, s); break;
            case 7: st = fill_rows_exact<7>(p, M, u, v, w, beam, ws, L, G, s); break;
            case 8: st = fill_rows_exact<8>(p, M, u, v, w, beam, ws, L, G, s); break;
            case 9: st = fill_rows_exact<9>(p, M, u, v, w, beam, ws, L, G, s); break;
            default: return wp_set_error(WP_EUNSUPPORTED, "build: 2-D rows need Ng <= %d (Ng = %d)",
                                         EXACT_MAX_NG, p->Ng);
        }
    } else switch (p->logNg) {
        case 6: st = fill_rows<6>(p, M, u, v, w, ws, L, G, s); break;
        case 7: st = fill_rows<7>(p, M, u, v, w, ws, L, G, s); break;
        case 8: st = fill_rows<8>(p, M, u, v, w, ws, L, G, s); break;
        case 9: st = fill_rows<9>(p, M, u, v, w, ws, L, G, s); break;
        case 10: st = fill_rows<10>(p, M, u, v, w, ws, L, G, s); break;
        case 11: st = fill_rows<11>(p, M, u, v, w, ws, L, G, s); break;
        case 12: st = fill_rows<12>(p, M, u, v, w, ws, L, G, s); break;
        default: return wp_set_error(WP_EUNSUPPORTED, "build: Ng = %d", p->Ng);
    }
    if (st != WP_OK) return st;
    const int nthr = 256;
    const dim3 gT((unsigned)((T + nthr - 1) / nthr));
    hipLaunchKernelGGL(k_write_items, gT, dim3(nthr), 0, s, (const int *)(ws + L.tstart), (const int *)(ws + L.tend),
                       (const int *)(ws + L.choff), T, p->ntile, G->work);
    if ((st = wp_check_launch("build_G_fill layout")) != WP_OK) return st;
    if (G->tcolptr) {
        const int64_t cells = (int64_t)p->Ng * p->Ng;
        int *cnt = (int *)(ws + L.tcnt);          // the workspace is const to callers; this region is scratch
        WP_HIP(hipMemsetAsync(cnt, 0, 4 * cells, s));
        if (G->nnz > 0) {
            int64_t nb = (G->nnz + nthr - 1) / nthr;
            if (nb > 65536) nb = 65536;
            hipLaunchKernelGGL(k_t_count, dim3((unsigned)nb), dim3(nthr), 0, s, G->col, G->nnz, cnt);
        }
        device_scan<int, int64_t>(cnt, G->tcolptr, cells, (int64_t *)(ws + L.sc64t), s);
        WP_HIP(hipMemsetAsync(cnt, 0, 4 * cells, s));
        const dim3 gR((unsigned)((M * 64 + nthr - 1) / nthr));
        if (G->taps != WP_TAPS_C64)
            hipLaunchKernelGGL((k_t_fill<uint32_t>), gR, dim3(nthr), 0, s, G->rowptr, G->col,
                               (const uint32_t *)G->val, G->perm, M, G->tcolptr, cnt, G->trow, (uint32_t *)G->tval);
        else
            hipLaunchKernelGGL((k_t_fill<float2>), gR, dim3(nthr), 0, s, G->rowptr, G->col, (const float2 *)G->val,
                               G->perm, M, G->tcolptr, cnt, G->trow, (float2 *)G->tval);
        const dim3 gC((unsigned)((cells + nthr - 1) / nthr));
        // cnt (free again after the fill) lists the cells of TS_CAP + 1 .. TS_BIG entries, counted in gpos[0]
        int *nbig = (int *)(ws + L.gpos);
        hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, nbig, 1);
        const dim3 gS((unsigned)((cells + 3) / 4)), gB(1024);
        if (G->taps != WP_TAPS_C64) {
            hipLaunchKernelGGL((k_t_sort_small<uint32_t>), gS, dim3(256), 0, s, G->tcolptr, cells, G->trow,
                               (uint32_t *)G->tval, cnt, nbig);
            hipLaunchKernelGGL((k_t_sort_big<uint32_t>), gB, dim3(256), 0, s, G->tcolptr, cnt, nbig, G->trow,
                               (uint32_t *)G->tval);
            hipLaunchKernelGGL((k_t_sort<uint32_t>), gC, dim3(nthr), 0, s, G->tcolptr, cells, G->trow,
                               (uint32_t *)G->tval);
        } else {
            hipLaunchKernelGGL((k_t_sort_small<float2>), gS, dim3(256), 0, s, G->tcolptr, cells, G->trow,
                               (float2 *)G->tval, cnt, nbig);
            hipLaunchKernelGGL((k_t_sort_big<float2>), gB, dim3(256), 0, s, G->tcolptr, cnt, nbig, G->trow,
                               (float2 *)G->tval);
            hipLaunchKernelGGL((k_t_sort<float2>), gC, dim3(nthr), 0, s, G->tcolptr, cells, G->trow,
                               (float2 *)G->tval);
        }
        if ((st = wp_check_launch("build_G_fill transpose")) != WP_OK) return st;
        if (G->tblk) {
            // cnt (free again) holds the block-start flags; their scan gives each block's index
            hipLaunchKernelGGL(k_gb_flags, gC, dim3(nthr), 0, s, G->tcolptr, cells, p->gb_ent, cnt);
            int *gpos = (int *)(ws + L.gpos);
            device_scan<int, int>(cnt, gpos, cells, (int *)(ws + L.sc64t), s);
            const int64_t n = cells > G->n_tblk + 1 ? cells : G->n_tblk + 1;
            int64_t nb = (n + nthr - 1) / nthr;
            if (nb > 65536) nb = 65536;
            hipLaunchKernelGGL(k_gb_write, dim3((unsigned)nb), dim3(nthr), 0, s, G->tcolptr, cnt, gpos, cells,
                               G->nnz, G->n_tblk, G->tblk);
            if ((st = wp_check_launch("build_G_fill gather blocks")) != WP_OK) return st;
        }
    }
    // the fill pass recomputes every row: its kept counts must equal the count pass's
    int host_err = 0;
    WP_HIP(hipMemcpyAsync(&host_err, ws + L.err, 4, hipMemcpyDeviceToHost, s));
    WP_HIP(hipStreamSynchronize(s));
    if (host_err & 6)
        return wp_set_error(WP_EHIP, "build_G_fill: a row's kept entries or factor record differ from pass 1 (flags %d)",
                            host_err);
    return WP_OK;
}
