// Rows of the exact chirp (Eq. 4) on large padded grids, without a 2-D FFT per row.
//
// On the padded grid the exact chirp factors as
//     c(l, m) = exp(i pi w l^2) exp(i pi w m^2) q(l^2 + m^2),
//     q(s) = exp(-2 pi i w (sqrt(1 - s) - 1 + s / 2)) = exp(i pi w s^2 / (1 + sqrt(1 - s))^2),
// the linear chirp (Eq. 5) times the part of Eq. 4 beyond it.  Over the padded field (s <= 2 L^2)
// that part turns by a few hundredths of a radian at the workloads' largest w, so x -> q(x + y) is
// smooth on [0, L^2] and its interpolation at LR_R Chebyshev points x_i gives a separable expansion
//     q(l^2 + m^2) ~ sum_i ell_i(l^2) q(x_i + m^2)        (ell_i: Lagrange polynomials of the points),
// written, since the ell_i sum to 1, as q(x_0 + m^2) + sum_{i>=1} ell_i(l^2) (q(x_i + m^2) - q(x_0 + m^2)):
// a leading term that is a linear chirp in l, and corrections whose v factors are small (q varies by a
// few hundredths over the field) and vanish at w = 0.  A row of G (Section 3.1: the window correlated
// with the chirp's 2-D spectrum) is then a sum of LR_R outer products of 1-D rows,
//     g(q_v, q_u) = sum_i U_i(q_u) V_i(q_v),   U_i = KB_u (x) Ng^-1 F[p_i(l^2) exp(i pi w l^2)],
//     V_i = KB_v (x) Ng^-1 F[d_i(m^2) exp(i pi w m^2)],
// p_0 = 1, d_0(y) = q(x_0 + y); p_i = ell_i, d_i(y) = q(x_i + y) - q(x_0 + y) for i >= 1;
// 2 LR_R one-dimensional FP64 FFTs per row.  With LR_R = 8 the expansion's largest error over every pair
// of padded-grid samples stays below 1e-10 up to four times the 1024-pixel form's largest w (checked
// over all sample pairs on the CPU); |c| = 1, so by Parseval a row's relative error is at most W times
// that.
//
// The row is formed on a window of Wd x Wd cells around its nearest cell, Wd covering the chirp's spread
// 4 w L^2 / sqrt(1 - 2 L^2) cells plus the gridding window and LR_MARGIN cells per side.  The threshold
// (Section 3.2) is searched over the window's energies with the row's total energy in closed form,
// T = (sum KB_u^2)(sum KB_v^2) (shifted spectra of a unit-modulus chirp are orthonormal): bisection on
// the bit patterns of the non-negative FP64 energies, as in the other builders.  The window's kept set
// and threshold are the row's when every entry outside the window lies below tau.  By the triangle
// inequality over the expansion's terms, an entry outside the window is at most
// max(sum_i max_out|U_i| max|V_i|, sum_i max|U_i| max_out|V_i|)^2 (max_out: over the cells of the axis
// outside the window); a row where that bound is not below tau sets error bit 8, and a row whose
// spread needs a window wider than LR_WMAX sets bit 16 (the build then fails).  The small corrections
// keep the bound within a few per cent of the true largest outside entry, which at the workloads'
// largest w is about 2 % of tau.
#pragma once

#include <cfloat>

#include "builder_util.h"
#include "fft_lds.h"

namespace {

constexpr int LR_R = 8;          // Chebyshev points of the separable expansion
constexpr int LR_MARGIN = 8;     // cells of margin per side of the window
constexpr int LR_WMAX = 88;      // widest window (cells)

// LDS: one spectrum (16 Ng), the window factors, and the window's energies (in the spectrum's space
// when it is large enough, after the last transform)
template <int LOGNG>
constexpr bool lowrank_en_in_h() {
    return (size_t)16 * (1 << LOGNG) >= (size_t)LR_WMAX * LR_WMAX * 8;
}
template <int LOGNG>
constexpr size_t lowrank_lds() {
    return (size_t)16 * (1 << LOGNG) + (size_t)2 * LR_R * LR_WMAX * 16 +
           (lowrank_en_in_h<LOGNG>() ? 0 : (size_t)LR_WMAX * LR_WMAX * 8);
}

// Chebyshev point i of [0, x_max]
__device__ inline double lr_node(int i, double x_max) {
    return 0.5 * x_max * (1.0 - cospi((2.0 * i + 1.0) / (2.0 * LR_R)));
}

// One workgroup per row.  Count pass (FILL = false): row r is visibility r; writes tau, the kept count,
// the sort key.  Fill pass: row r is sorted row r (visibility perm[r]); recomputes the energies with the
// same code, keeps those >= tau (from the count pass) and writes them in ascending flattened column.
template <int LOGNG, bool FILL, int TK>
__global__ __launch_bounds__(BNTH) void k_lowrank_rows(const double *__restrict__ u, const double *__restrict__ v,
                                                       const double *__restrict__ w, double E, double cell,
                                                       double delta, int W, double beta, double L2,
                                                       const double2 *__restrict__ tw64, int64_t r0,
                                                       const int *__restrict__ perm, double *__restrict__ tau_io,
                                                       int *__restrict__ nnz_out, int *__restrict__ key_out,
                                                       int *__restrict__ fsz_out, const int64_t *__restrict__ rowptr,
                                                       int *__restrict__ col, void *__restrict__ val,
                                                       float *__restrict__ rscale, int *__restrict__ err) {
    constexpr int Ng = 1 << LOGNG;
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *h = (double2 *)smem;                              // Ng: one 1-D spectrum at a time
    double2 *Uf = (double2 *)(smem + 16 * Ng);                 // [LR_R][LR_WMAX]
    double2 *Vf = Uf + LR_R * LR_WMAX;                         // [LR_R][LR_WMAX]
    double *en = lowrank_en_in_h<LOGNG>() ? (double *)h        // [Wd][Wd] energies, row b = v, column a = u
                                          : (double *)(Vf + LR_R * LR_WMAX);
    __shared__ double redd[BNTH / 64];
    __shared__ long long redl[BNTH / 64];
    __shared__ int redi[BNTH / 64];
    __shared__ double s_wu[16], s_wv[16];
    __shared__ double s_node[LR_R];
    __shared__ double s_mx[4][LR_R];               // per term: max |U_i| outside, everywhere; same for V_i
    __shared__ int s_off[LR_WMAX + 1];

    const int64_t r = r0 + blockIdx.x;
    const int64_t k = FILL ? (int64_t)perm[r] : r;
    const double ut = u[k] / cell, vt = v[k] / cell, wk = w[k];
    const bool ok = isfinite(ut) && isfinite(vt) && isfinite(wk) && fabs(ut) < Ng / 2 && fabs(vt) < Ng / 2;
    if (!ok) {
        if (!FILL && threadIdx.x == 0) {
            atomicOr(err, 1);
            tau_io[k] = INFINITY;
            nnz_out[k] = 0;
            key_out[k] = 0;
            fsz_out[k] = 0;
        }
        return;
    }
    // window: half width from the chirp's spread, centred on the nearest cell
    const double spread = 4.0 * fabs(wk) * L2 / sqrt(1.0 - 2.0 * L2);
    const int hw = (int)ceil(0.5 * spread) + W / 2 + LR_MARGIN;
    const bool whole = 2 * hw + 1 >= Ng;                       // the window covers the whole axis
    const int Wd = whole ? Ng : 2 * hw + 1;
    if (Wd > LR_WMAX) {
        if (threadIdx.x == 0) {
            atomicOr(err, 16);
            if (!FILL) {
                tau_io[k] = INFINITY;
                nnz_out[k] = 0;
                key_out[k] = 0;
                fsz_out[k] = 0;
            }
        }
        return;
    }
    const int cu0 = whole ? 0 : (int)floor(ut + 0.5) + Ng / 2 - hw;       // first window cells
    const int cv0 = whole ? 0 : (int)floor(vt + 0.5) + Ng / 2 - hw;
    const Taps tu = kb_taps(ut, W, beta, Ng, s_wu);
    const Taps tv = kb_taps(vt, W, beta, Ng, s_wv);
    if (threadIdx.x < LR_R) s_node[threadIdx.x] = lr_node(threadIdx.x, L2);
    __syncthreads();
    const double a = wk * delta * delta;
    for (int i = 0; i < LR_R; ++i) {
        // u side: ell_i(l^2) exp(i pi w l^2)
        for (int t = threadIdx.x; t < Ng; t += BNTH) {
            const double tt = (double)(t < Ng / 2 ? t : t - Ng);
            const double x = tt * tt * delta * delta;
            double ell = 1.0;                                   // p_0 = 1, p_i = ell_i
            if (i > 0)
                for (int j = 0; j < LR_R; ++j)
                    if (j != i) ell *= (x - s_node[j]) / (s_node[i] - s_node[j]);
            double sn, cs;
            sincospi(a * tt * tt, &sn, &cs);
            h[t] = make_double2(ell * cs, ell * sn);
        }
        __syncthreads();
        lds_fft<double2, LOGNG, 1, BNTH, true, Ng>(h, tw64, false, threadIdx.x);
        __syncthreads();
        double mo = 0.0, ma = 0.0;
        for (int q = threadIdx.x; q < Ng; q += BNTH) {
            const double2 f = row_factor(h, tu, W, q, Ng);
            const double e2 = energy(f);
            ma = fmax(ma, e2);
            const int j = (q - cu0) & (Ng - 1);
            if (j < Wd) Uf[i * LR_WMAX + j] = f;
            else mo = fmax(mo, e2);
        }
        mo = block_max(mo, redd);
        ma = block_max(ma, redd);
        if (threadIdx.x == 0) {
            s_mx[0][i] = sqrt(mo);
            s_mx[1][i] = sqrt(ma);
        }
        __syncthreads();
        // v side: d_i(m^2) exp(i pi w m^2), d_0(y) = q(x_0 + y), d_i(y) = q(x_i + y) - q(x_0 + y)
        for (int t = threadIdx.x; t < Ng; t += BNTH) {
            const double tt = (double)(t < Ng / 2 ? t : t - Ng);
            const double y = tt * tt * delta * delta;
            const double s = s_node[i] + y, s0 = s_node[0] + y;
            const double d = 1.0 + sqrt(1.0 - s), d0 = 1.0 + sqrt(1.0 - s0);
            double sn, cs;
            sincospi(a * tt * tt + wk * s * s / (d * d), &sn, &cs);
            if (i > 0) {
                double sn0, cs0;
                sincospi(a * tt * tt + wk * s0 * s0 / (d0 * d0), &sn0, &cs0);
                cs -= cs0;
                sn -= sn0;
            }
            h[t] = make_double2(cs, sn);
        }
        __syncthreads();
        lds_fft<double2, LOGNG, 1, BNTH, true, Ng>(h, tw64, false, threadIdx.x);
        __syncthreads();
        mo = 0.0;
        ma = 0.0;
        for (int q = threadIdx.x; q < Ng; q += BNTH) {
            const double2 f = row_factor(h, tv, W, q, Ng);
            const double e2 = energy(f);
            ma = fmax(ma, e2);
            const int j = (q - cv0) & (Ng - 1);
            if (j < Wd) Vf[i * LR_WMAX + j] = f;
            else mo = fmax(mo, e2);
        }
        mo = block_max(mo, redd);
        ma = block_max(ma, redd);
        if (threadIdx.x == 0) {
            s_mx[2][i] = sqrt(mo);
            s_mx[3][i] = sqrt(ma);
        }
        __syncthreads();
    }
    // the window's values and energies
    const int n = Wd * Wd;
    double emax = 0.0, etot = 0.0;
    for (int e = threadIdx.x; e < n; e += BNTH) {
        const int b = e / Wd, c = e % Wd;
        double gx = 0.0, gy = 0.0;
        for (int i = 0; i < LR_R; ++i) {
            const double2 x = Uf[i * LR_WMAX + c], y = Vf[i * LR_WMAX + b];
            gx = fma(x.x, y.x, fma(-x.y, y.y, gx));
            gy = fma(x.x, y.y, fma(x.y, y.x, gy));
        }
        const double m = energy(make_double2(gx, gy));
        en[e] = m;
        emax = fmax(emax, m);
        etot += m;
    }
    emax = block_max(emax, redd);                   // its barriers also publish en
    etot = block_sum(etot, redd);
    double tau;
    if (FILL) {
        tau = tau_io[k];
    } else {
        double T0u = 0.0, T0v = 0.0;
        for (int i = 0; i < W; ++i) {
            T0u += s_wu[i] * s_wu[i];
            T0v += s_wv[i] * s_wv[i];
        }
        const double T = T0u * T0v;
        const double target = E * T;
        unsigned long long lo = 0ull, hi = (unsigned long long)__double_as_longlong(emax) + 1ull;
        while (hi - lo > 1ull) {
            const unsigned long long mid = lo + ((hi - lo) >> 1);
            const double tm = __longlong_as_double((long long)mid);
            double Km = 0.0;
            for (int e = threadIdx.x; e < n; e += BNTH) Km += en[e] >= tm ? en[e] : 0.0;
            Km = block_sum(Km, redd);
            if (Km >= target) lo = mid; else hi = mid;
        }
        tau = __longlong_as_double((long long)lo);
        long long c = 0;
        for (int e = threadIdx.x; e < n; e += BNTH) c += en[e] >= tau;
        c = block_sum(c, redl);
        if (threadIdx.x == 0) {
            // bound on the entries outside the window (triangle inequality over the expansion's terms)
            double bu = 0.0, bv = 0.0;
            for (int i = 0; i < LR_R; ++i) {
                bu += s_mx[0][i] * s_mx[3][i];
                bv += s_mx[1][i] * s_mx[2][i];
            }
            const double bound = fmax(bu, bv) * fmax(bu, bv);
            if (!(bound < tau) || !(etot >= target)) atomicOr(err, 8);
            tau_io[k] = tau;
            nnz_out[k] = (int)c;
            fsz_out[k] = 0;                        // no factor records: the rows are not separable
            const int cu = min(max((int)floor(ut + Ng / 2), 0), Ng - 1);
            const int cv = min(max((int)floor(vt + Ng / 2), 0), Ng - 1);
            key_out[k] = morton2(cv, cu);
        }
        return;
    }
    // fill: window rows and columns in ascending grid index (the window may wrap around the grid)
    const int b0 = (cv0 & (Ng - 1)) + Wd > Ng ? Ng - (cv0 & (Ng - 1)) : 0;     // first window row in grid order
    const int a0 = (cu0 & (Ng - 1)) + Wd > Ng ? Ng - (cu0 & (Ng - 1)) : 0;
    const int64_t beg = rowptr[r], len = rowptr[r + 1] - beg;
    const double i16_scale = sqrt(emax) / 32767.0;
    if (TK == WP_TAPS_I16 && threadIdx.x == 0) rscale[r] = (float)i16_scale;
    {
        // kept entries per window row (grid order), then offsets
        int cnt = 0;
        if ((int)threadIdx.x < Wd) {
            const int b = (b0 + threadIdx.x) % Wd;
            for (int c = 0; c < Wd; ++c) cnt += en[b * Wd + c] >= tau;
        }
        int total;
        const int o = block_excl_scan(cnt, redi, total);
        if ((int)threadIdx.x < Wd) s_off[threadIdx.x] = o;
        if (threadIdx.x == 0 && total != len) atomicOr(err, 2);
        __syncthreads();
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int jb = wid; jb < Wd; jb += BNTH / 64) {
        const int b = (b0 + jb) % Wd;
        const int qv = (cv0 + b) & (Ng - 1);
        int64_t pos = beg + s_off[jb];
        for (int c0 = 0; c0 < Wd; c0 += 64) {
            const int jc = c0 + lane;
            const int c = (a0 + jc) % Wd;
            const bool keep = jc < Wd && en[b * Wd + c] >= tau;
            const unsigned long long msk = __ballot(keep);
            if (keep) {
                double gx = 0.0, gy = 0.0;
                for (int i = 0; i < LR_R; ++i) {
                    const double2 x = Uf[i * LR_WMAX + c], y = Vf[i * LR_WMAX + b];
                    gx = fma(x.x, y.x, fma(-x.y, y.y, gx));
                    gy = fma(x.x, y.y, fma(x.y, y.x, gy));
                }
                const int64_t p = pos + __popcll(msk & ((1ull << lane) - 1ull));
                if (p < beg + len) {
                    col[p] = qv * Ng + ((cu0 + c) & (Ng - 1));
                    if (TK == WP_TAPS_BF16) ((uint32_t *)val)[p] = pack_bf16x2((float)gx, (float)gy);
                    else if (TK == WP_TAPS_I16)
                        ((uint32_t *)val)[p] = pack_i16x2((float)(gx / i16_scale), (float)(gy / i16_scale));
                    else ((float2 *)val)[p] = make_float2((float)gx, (float)gy);
                }
            }
            pos += __popcll(msk);
        }
    }
}

}  // namespace
