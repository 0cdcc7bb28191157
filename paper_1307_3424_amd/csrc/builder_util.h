// Device helpers shared by the builders of G (separable rows in builder.hip, the exact
// chirp's 2-D rows in builder_exact.hip): the Kaiser-Bessel window, tap energies and
// block-wide reductions over BNTH threads.
#pragma once

#include "common.h"

namespace {

constexpr int BNTH = 256;      // builder block size

__device__ inline double bessel_i0(double x) {
    // power series sum_k ((x/2)^2)^k / (k!)^2
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 200; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

__device__ inline double kb_weight(double t, int W, double beta) {
    const double r = 1.0 - (2.0 * t / W) * (2.0 * t / W);
    return r >= 0.0 ? bessel_i0(beta * sqrt(r)) : 0.0;
}

struct Taps {
    int q0;              // grid index (may be < 0 or >= Ng: taken mod Ng) of the first window cell
    const double *wt;    // W window weights (LDS)
};

// Window cells and weights of one axis; the weights go to LDS (wt_lds[W]), written by the first W threads.
__device__ inline Taps kb_taps(double gt, int W, double beta, int Ng, double *wt_lds) {
    const int base = (int)floor(gt) - W / 2 + 1;     // centred index of the first cell
    if ((int)threadIdx.x < W) wt_lds[threadIdx.x] = kb_weight(gt - (double)(base + (int)threadIdx.x), W, beta);
    Taps t;
    t.q0 = base + Ng / 2;
    t.wt = wt_lds;
    return t;
}

// g(q) = Ng^-1 sum_i wt_i h((q0 + i - q) mod Ng)
__device__ inline double2 row_factor(const double2 *h, const Taps &t, int W, int q, int Ng) {
    double2 g = make_double2(0.0, 0.0);
    for (int i = 0; i < W; ++i) {
        const double2 hv = h[(t.q0 + i - q) & (Ng - 1)];
        g.x += t.wt[i] * hv.x;
        g.y += t.wt[i] * hv.y;
    }
    const double s = 1.0 / Ng;
    return make_double2(g.x * s, g.y * s);
}

// |g|^2 with one explicit fused multiply-add, so that every kernel that evaluates it
// (both passes of the builder) gets the same bits
__device__ inline double energy(double2 g) { return fma(g.x, g.x, g.y * g.y); }

template <typename T>
__device__ inline T block_sum(T v, T *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    T s = 0;
    for (int i = 0; i < BNTH / 64; ++i) s += red[i];
    return s;
}

__device__ inline double block_max(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < BNTH / 64; ++i) s = fmax(s, red[i]);
    return s;
}

// exclusive scan of one int per thread over the block; returns the total
__device__ inline int block_excl_scan(int v, int *red, int &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) red[wid] = x;
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < BNTH / 64; ++i) {
        if (i < wid) off += red[i];
        tot += red[i];
    }
    total = tot;
    return off + x - v;
}

}  // namespace
