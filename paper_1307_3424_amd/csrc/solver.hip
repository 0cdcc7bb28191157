// Constrained l1 reconstruction (Eq. 7 in its analysis form) on the GPU.
//
//   min_x ||Psi^T x||_1  s.t.  ||y - Phi x||_2 <= eps,  x >= 0 (real)
//
// Psi: Daubechies wavelets with p = 8 vanishing moments (16 taps), periodic,
// multi-level, rows then columns per level (Section 4.2 uses Daubechies 8), or
// with zero levels the Dirac basis Psi = I (Section 4.2's other dictionary).
// Splitting: primal-dual with one dual variable per term (Condat 2013 / Vu 2013):
//   x+  = max(0, x - tau (Psi v1 + Re Phi^H v2)) ;  xb = 2 x+ - x ;  x = x+
//   v1  = clip(v1 + s1 Psi^T xb, -1, 1)
//   u   = v2 + s2 Phi xb ;  v2 = u - s2 P(u / s2),  P(z) = y + (z - y) min(1, eps / ||z - y||)
// with tau = 0.49, s1 = 1, s2 = 1 / ||Phi||^2 and ||Phi||^2 from power iteration.
// Every step runs in the kernels below or in the operator's kernels; the host
// loop only enqueues them (no synchronisation inside an iteration).  The
// residual norm is reduced in FP64 on the device.
#include <cmath>
#include <complex>
#include <vector>

#include "common.h"

namespace {

constexpr int NT = 256;

// ---------------------------------------------------------------------------- Daubechies filter (host, FP64)
// |m0(xi)|^2 = cos^(2p)(xi/2) Q(sin^2(xi/2)), Q(y) = sum_{k<p} C(p-1+k, k) y^k.  Each root y_i of
// Q gives z + 1/z = 2 (1 - 2 y_i); the minimum-phase factor keeps the z with |z| < 1.  The filter is
// the polynomial with p zeros at -1 and those z, highest power first, scaled to sum sqrt(2).
bool daubechies(int p, double *h) {
    using cd = std::complex<double>;
    std::vector<double> q(p);
    for (int k = 0; k < p; ++k) {
        double c = 1.0;
        for (int i = 1; i <= k; ++i) c = c * (p - 1 + i) / i;   // C(p-1+k, k)
        q[k] = c;
    }
    const int deg = p - 1;
    std::vector<cd> roots(deg);
    // Durand-Kerner on the monic polynomial Q / q[deg]
    for (int i = 0; i < deg; ++i) roots[i] = std::pow(cd(0.4, 0.9), i);
    auto Qm = [&](cd yv) {
        cd acc = 0.0;
        for (int k = deg; k >= 0; --k) acc = acc * yv + q[k] / q[deg];
        return acc;
    };
    for (int it = 0; it < 2000; ++it) {
        double delta = 0.0;
        for (int i = 0; i < deg; ++i) {
            cd den = 1.0;
            for (int j = 0; j < deg; ++j)
                if (j != i) den *= roots[i] - roots[j];
            const cd step = Qm(roots[i]) / den;
            roots[i] -= step;
            delta = std::max(delta, std::abs(step));
        }
        if (delta < 1e-15) break;
    }
    std::vector<cd> z;
    for (int k = 0; k < p; ++k) z.push_back(-1.0);
    for (int i = 0; i < deg; ++i) {
        const cd b = 1.0 - 2.0 * roots[i];
        const cd d = std::sqrt(b * b - 1.0);
        const cd z1 = b + d, z2 = b - d;
        z.push_back(std::abs(z1) < 1.0 ? z1 : z2);
    }
    // expand prod (x - z_i), coefficients highest power first
    std::vector<cd> c(1, 1.0);
    for (const cd &r : z) {
        std::vector<cd> n(c.size() + 1, 0.0);
        for (size_t i = 0; i < c.size(); ++i) {
            n[i] += c[i];
            n[i + 1] -= c[i] * r;
        }
        c.swap(n);
    }
    double sum = 0.0;
    for (int i = 0; i < 2 * p; ++i) sum += c[i].real();
    if (!(std::fabs(sum) > 0)) return false;
    for (int i = 0; i < 2 * p; ++i) h[i] = c[i].real() * std::sqrt(2.0) / sum;
    return true;
}

struct Filt {
    float h[16], g[16];
};

// Filters of several bases (a batch of transforms takes basis blockIdx.y): Daubechies with p + 1
// vanishing moments at f[p] for the SARA dictionary, or Daubechies 8 alone at f[0]
struct FiltSet {
    Filt f[8];
};

// ---------------------------------------------------------------------------- DWT kernels (FP32)
// One level along a line of length L (a power of two), H = L / 2.  Analysis:
// a_k = sum_n h_n x_(2k+n mod L), d_k = sum_n g_n x_(2k+n mod L), stored [a | d].  Synthesis (the
// transpose): x_m = sum over n of m's parity of h_n a_((m-n)/2 mod H) + g_n d_((m-n)/2 mod H);
// m - n is even there, so (m - n) >> 1 is exact and & (H - 1) reduces it.  at(j) reads the line.
template <typename At>
__device__ __forceinline__ float dwt_tap_sum(At at, int m, int L, const Filt &f, bool synth) {
    const int H = L >> 1;
    float acc = 0.f;
    if (!synth) {
        const bool lo = m < H;
        const int k = lo ? m : m - H;
#pragma unroll
        for (int n = 0; n < 16; ++n) acc = fmaf(lo ? f.h[n] : f.g[n], at((2 * k + n) & (L - 1)), acc);
    } else {
        const int odd = m & 1;
#pragma unroll
        for (int n = 0; n < 16; n += 2) {
            const int nn = n + odd;
            const int k = ((m - nn) >> 1) & (H - 1);
            acc = fmaf(odd ? f.h[n + 1] : f.h[n], at(k), acc);
            acc = fmaf(odd ? f.g[n + 1] : f.g[n], at(H + k), acc);
        }
    }
    return acc;
}

// One pass of one level over `lines` lines of an image of row stride N: line i, element e at
// [i * ls + e * es].  Element (i, e) is read from `in` when i < q and e < q, else from `in2`:
// the synthesis reads the coarser levels' result (in) in the top-left quadrant and the original
// coefficients (in2) elsewhere, which spares a copy of the coefficients; q = 0 reads in2 only.
__global__ void k_dwt_lines(const float *__restrict__ in, const float *__restrict__ in2, int q,
                            float *__restrict__ out, int L, int lines, int ls, int es, Filt f, bool synth) {
    extern __shared__ float line[];
    for (int i = blockIdx.x; i < lines; i += gridDim.x) {
        for (int e = threadIdx.x; e < L; e += blockDim.x) {
            const int64_t at = (int64_t)i * ls + (int64_t)e * es;
            line[e] = (i < q && e < q) ? in[at] : in2[at];
        }
        __syncthreads();
        for (int m = threadIdx.x; m < L; m += blockDim.x)
            out[(int64_t)i * ls + (int64_t)m * es] = dwt_tap_sum([&](int j) { return line[j]; }, m, L, f, synth);
        __syncthreads();
    }
}

// Optional store epilogues of the tiled level kernels, used by the primal-dual loop to fold its
// elementwise steps into the transforms (null pointers: plain stores).
// Dual: in place of storing coefficient c_i, v1_i = clip(v1_i + s1 c_i, -1, 1) (the l1 dual step).
struct DualEpi {
    float *v1;
    float s1;
};
// Primal: in place of storing the synthesis x_i = (Psi v1)_i, the primal step with it:
// x+ = max(0, x - tau (Psi v1 + Re(Phi^H v2))); xb = 2 x+ - x; x = x+; xbc = complex(xb).
struct PrimalEpi {
    float *x;
    const float2 *phit;
    float *xb;
    float2 *xbc;
    float tau;
    double *acc_zero;                     // set to zero (the next ball norm's accumulator)
};

// One whole level (both axes) per kernel, tiled.  A coefficient (r, c) of a level depends on a
// 16 x 16 window of its input, so a workgroup makes a tile of t x t positions of all four
// subbands (t = min(DT, H)) from a (2t + 14)^2 window staged in LDS: first the row filters of every
// window row, then the column filters, in the same order of operations as one pass per axis.
constexpr int DT = 8;
constexpr int DWIN = 2 * DT + 14;
constexpr int DNT = 256;

// Analysis of the top-left L x L block of `in` (row stride N; periodic in L).  The three detail
// subbands go to det, the approximation (top-left H x H) to ll; both have row stride N.  Basis
// b = blockIdx.y reads in + b in_zs and writes det + b N^2, ll + b N^2.
__global__ __launch_bounds__(DNT) void k_dwt2_fwd(const float *__restrict__ in, int64_t in_zs, float *__restrict__ det,
                                                  float *__restrict__ ll, int N, int L, const FiltSet fs,
                                                  DualEpi de = {nullptr, 0.f}, int ll_final = 0) {
    __shared__ float win[DWIN * DWIN];
    const Filt f = fs.f[blockIdx.y];                              // taps in registers, read once
    in += blockIdx.y * in_zs;
    det += (int64_t)blockIdx.y * N * N;
    ll += (int64_t)blockIdx.y * N * N;
    __shared__ float R[DWIN * 2 * DT];
    const int H = L >> 1, t = H < DT ? H : DT, tiles = H / t, w = 2 * t + 14;
    const int kr0 = (blockIdx.x / tiles) * t, kc0 = (blockIdx.x % tiles) * t;
    // stage the window: all of a thread's loads in flight before the first LDS write (positions
    // past the window load a clamped in-window address and are not stored)
    constexpr int PW = (DWIN * DWIN + DNT - 1) / DNT;
    float v[PW];
#pragma unroll
    for (int k = 0; k < PW; ++k) {
        const int e = min((int)threadIdx.x + k * DNT, w * w - 1), i = e / w, j = e % w;
        v[k] = in[(int64_t)((2 * kr0 + i) & (L - 1)) * N + ((2 * kc0 + j) & (L - 1))];
    }
#pragma unroll
    for (int k = 0; k < PW; ++k) {
        const int e = threadIdx.x + k * DNT;
        if (e < w * w) win[(e / w) * DWIN + e % w] = v[k];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < w * 2 * t; e += DNT) {          // rows: R[i][band * t + kc]
        const int i = e / (2 * t), q = e % (2 * t), band = q / t, kc = q % t;
        float acc = 0.f;
#pragma unroll
        for (int n = 0; n < 16; ++n) acc = fmaf(band ? f.g[n] : f.h[n], win[i * DWIN + 2 * kc + n], acc);
        R[i * (2 * DT) + q] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 4 * t * t; e += DNT) {          // columns
        const int q = e % (2 * t), rr = e / (2 * t), band1 = rr / t, kr = rr % t;
        float acc = 0.f;
#pragma unroll
        for (int n = 0; n < 16; ++n) acc = fmaf(band1 ? f.g[n] : f.h[n], R[(2 * kr + n) * (2 * DT) + q], acc);
        const int band2 = q / t, kc = q % t;
        const int r = band1 * H + kr0 + kr, c = band2 * H + kc0 + kc;
        const bool is_ll = band1 == 0 && band2 == 0;
        if (de.v1 && (!is_ll || ll_final)) {        // a final coefficient: the dual step instead
            float *v = de.v1 + (int64_t)r * N + c;
            *v = fminf(1.f, fmaxf(-1.f, *v + de.s1 * acc));
        } else if (is_ll) {
            ll[(int64_t)r * N + c] = acc;
        } else {
            det[(int64_t)r * N + c] = acc;
        }
    }
}

// Synthesis of one level: the L x L result (row stride N) from coefficients whose top-left H x H
// quadrant (the coarser levels' result) is read from llin and the three detail quadrants from
// coef.  A tile of 2t x 2t outputs reads t + 8 positions of each band per axis.  Basis
// b = blockIdx.y offsets all three images by b N^2.
__global__ __launch_bounds__(DNT) void k_dwt2_inv(const float *__restrict__ coef, const float *__restrict__ llin,
                                                  float *__restrict__ out, int N, int L, const FiltSet fs,
                                                  PrimalEpi pe = {nullptr, nullptr, nullptr, nullptr, 0.f, nullptr}) {
    constexpr int CW = 2 * (DT + 8);
    // taps in registers, read once, split by parity: an output at parity o uses h_(n+o), g_(n+o)
    float he[8], ho[8], ge[8], go[8];
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        he[n] = fs.f[blockIdx.y].h[2 * n];
        ho[n] = fs.f[blockIdx.y].h[2 * n + 1];
        ge[n] = fs.f[blockIdx.y].g[2 * n];
        go[n] = fs.f[blockIdx.y].g[2 * n + 1];
    }
    coef += (int64_t)blockIdx.y * N * N;
    llin += (int64_t)blockIdx.y * N * N;
    out += (int64_t)blockIdx.y * N * N;
    __shared__ float C[CW * CW];
    __shared__ float Y[2 * DT * CW];
    const int H = L >> 1, t = H < DT ? H : DT, tiles = H / t, w = t + 8;
    const int mr0 = (blockIdx.x / tiles) * 2 * t, mc0 = (blockIdx.x % tiles) * 2 * t;
    const int kr0 = (mr0 >> 1) - 8, kc0 = (mc0 >> 1) - 8;        // first coefficient of each window
    // stage the four band windows, every load in flight before the first LDS write; the source
    // (coarser result or detail coefficients) is a pointer select, not a branch
    constexpr int PC = (CW * CW + DNT - 1) / DNT;
    float v[PC];
#pragma unroll
    for (int k = 0; k < PC; ++k) {
        const int e = min((int)threadIdx.x + k * DNT, 4 * w * w - 1), i = e / (2 * w), j = e % (2 * w);
        const int r = (i / w) * H + ((kr0 + i % w) & (H - 1)), c = (j / w) * H + ((kc0 + j % w) & (H - 1));
        const float *src = (r < H && c < H) ? llin : coef;
        v[k] = src[(int64_t)r * N + c];
    }
#pragma unroll
    for (int k = 0; k < PC; ++k) {
        const int e = threadIdx.x + k * DNT;
        if (e < 4 * w * w) C[(e / (2 * w)) * CW + e % (2 * w)] = v[k];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * t * 2 * w; e += DNT) {      // columns: Y[mr][j]
        const int mr = e / (2 * w), j = e % (2 * w);
        const int m = mr0 + mr, odd = m & 1;
        float acc = 0.f;
#pragma unroll
        for (int n = 0; n < 16; n += 2) {
            const int nn = n + odd, i = ((m - nn) >> 1) - kr0;
            acc = fmaf(odd ? ho[n / 2] : he[n / 2], C[i * CW + j], acc);
            acc = fmaf(odd ? go[n / 2] : ge[n / 2], C[(w + i) * CW + j], acc);
        }
        Y[mr * CW + j] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 4 * t * t; e += DNT) {          // rows
        const int mr = e / (2 * t), mc = e % (2 * t);
        const int m = mc0 + mc, odd = m & 1;
        float acc = 0.f;
#pragma unroll
        for (int n = 0; n < 16; n += 2) {
            const int nn = n + odd, j = ((m - nn) >> 1) - kc0;
            acc = fmaf(odd ? ho[n / 2] : he[n / 2], Y[mr * CW + j], acc);
            acc = fmaf(odd ? go[n / 2] : ge[n / 2], Y[mr * CW + w + j], acc);
        }
        const int64_t i = (int64_t)(mr0 + mr) * N + mc0 + mc;
        if (pe.x) {                               // the primal step with (Psi v1)_i = acc
            const float xo = pe.x[i];
            const float xn = fmaxf(0.f, xo - pe.tau * (acc + pe.phit[i].x));
            const float b = 2.f * xn - xo;
            pe.x[i] = xn;
            pe.xb[i] = b;
            pe.xbc[i] = make_float2(b, 0.f);
        } else {
            out[i] = acc;
        }
    }
    if (pe.x && blockIdx.x == 0 && threadIdx.x == 0) *pe.acc_zero = 0.0;
}

// ---------------------------------------------------------------------------- iteration kernels

// Dirac basis (Psi = I), pixel by pixel: the primal step x+ = max(0, x - tau (v1 + Re(phit_v2))),
// xb = 2 x+ - x, x = x+, xbc = complex(xb); then the l1 dual step v1 = clip(v1 + s1 xb, -1, 1)
// (v1 is read for the primal step before its update)
__global__ void k_primal_dual1_dirac(float *__restrict__ x, float *__restrict__ v1, const float2 *__restrict__ phit_v2,
                                     float *__restrict__ xb, float2 *__restrict__ xbc, int64_t n, float tau, float s1,
                                     double *__restrict__ acc_zero) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *acc_zero = 0.0;
    if (i >= n) return;
    const float xo = x[i], vo = v1[i];
    const float xn = fmaxf(0.f, xo - tau * (vo + phit_v2[i].x));
    const float b = 2.f * xn - xo;
    x[i] = xn;
    xb[i] = b;
    xbc[i] = make_float2(b, 0.f);
    v1[i] = fminf(1.f, fmaxf(-1.f, vo + s1 * b));
}

// SARA analysis, last step: c_0 = x / 3 (Dirac), c_b = W_b x / 3 (the transforms are in c_1..c_8)
__global__ void k_sara_scale(const float *__restrict__ x, float *__restrict__ c, int64_t n2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n2) return;
    constexpr float third = 1.0f / 3.0f;
    c[i] = x[i] * third;
#pragma unroll
    for (int b = 1; b < 9; ++b) c[b * n2 + i] *= third;
}

// SARA synthesis, last step: x = (c_0 + sum_b W_b^T c_b) / 3 (the eight syntheses are in r_0..r_7)
__global__ void k_sara_sum(const float *__restrict__ c0, const float *__restrict__ r, float *__restrict__ x,
                           int64_t n2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n2) return;
    float acc = c0[i];
#pragma unroll
    for (int b = 0; b < 8; ++b) acc += r[b * n2 + i];
    x[i] = acc * (1.0f / 3.0f);
}

// SARA loop: k_sara_scale, then the dual step of the weighted norm ||W Psi^T x||_1,
// v1 = clip(v1 + s1 c, -w, w), over the nine bases, per pixel, in one pass (c is not stored)
__global__ void k_sara_scale_dual(const float *__restrict__ x, const float *__restrict__ c, float *__restrict__ v1,
                                  const float *__restrict__ w, int64_t n2, float s1) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n2) return;
    constexpr float third = 1.0f / 3.0f;
#pragma unroll
    for (int b = 0; b < 9; ++b) {
        const int64_t j = b * n2 + i;
        const float cb = b == 0 ? x[i] * third : c[j] * third;
        v1[j] = fminf(w[j], fmaxf(-w[j], v1[j] + s1 * cb));
    }
}

// SARA loop: k_sara_sum, then the primal step (as in k_primal_dual1_dirac) with Psi v1 = that sum
__global__ void k_sara_sum_primal(const float *__restrict__ c0, const float *__restrict__ r, float *__restrict__ x,
                                  const float2 *__restrict__ phit_v2, float *__restrict__ xb,
                                  float2 *__restrict__ xbc, int64_t n2, float tau, double *__restrict__ acc_zero) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *acc_zero = 0.0;
    if (i >= n2) return;
    float acc = c0[i];
#pragma unroll
    for (int b = 0; b < 8; ++b) acc += r[b * n2 + i];
    const float psi = acc * (1.0f / 3.0f);
    const float xo = x[i];
    const float xn = fmaxf(0.f, xo - tau * (psi + phit_v2[i].x));
    const float b2 = 2.f * xn - xo;
    x[i] = xn;
    xb[i] = b2;
    xbc[i] = make_float2(b2, 0.f);
}

// weights delta / (delta + |alpha|)
__global__ void k_sara_weights(const float *__restrict__ alpha, float *__restrict__ w, int64_t n, double d) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    w[i] = (float)(d / (d + fabs((double)alpha[i])));
}

__global__ void k_fill_f32(float *__restrict__ a, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// first pass (second = 0): acc[0] += sum a; second pass: acc[1] += sum (a - mean)^2, mean = acc[0] / n (FP64)
__global__ void k_sum_dev(const float *__restrict__ a, int64_t n, double *__restrict__ acc, int second) {
    __shared__ double red[NT / 64];
    const double mean = second ? acc[0] / (double)n : 0.0;
    double sum = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = (double)a[i] - mean;
        sum += second ? v * v : (double)a[i];
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < NT / 64; ++w) t += red[w];
        atomicAdd(acc + second, t);
    }
}

// Douglas-Rachford elementwise steps
// x = z - Re t (and xc = complex(x) when given)
__global__ void k_dr_sub(const float *__restrict__ z, const float2 *__restrict__ t, float *__restrict__ x,
                         float2 *__restrict__ xc, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = z[i] - t[i].x;
    x[i] = v;
    if (xc) xc[i] = make_float2(v, 0.f);
}

// r = 2 x - z
__global__ void k_dr_reflect(const float *__restrict__ x, const float *__restrict__ z, float *__restrict__ r,
                             int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) r[i] = 2.f * x[i] - z[i];
}

// a = sign(a) max(|a| - g, 0)
__global__ void k_soft(float *__restrict__ a, int64_t n, float g) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float m = fabsf(a[i]) - g;
    a[i] = m > 0.f ? copysignf(m, a[i]) : 0.f;
}

// z = z + q - x
__global__ void k_dr_update(float *__restrict__ z, const float *__restrict__ q, const float *__restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = z[i] + q[i] - x[i];
}

// acc += sum |u / s2 - y|^2, u = v2 + s2 p  (FP64)
__global__ void k_ball_norm(const float2 *__restrict__ v2, const float2 *__restrict__ p, const float2 *__restrict__ y,
                            int64_t n, float s2, double *__restrict__ acc) {
    __shared__ double red[NT / 64];
    double sum = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double zr = ((double)v2[i].x + (double)s2 * p[i].x) / s2 - y[i].x;
        const double zi = ((double)v2[i].y + (double)s2 * p[i].y) / s2 - y[i].y;
        sum += zr * zr + zi * zi;
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < NT / 64; ++w) t += red[w];
        atomicAdd(acc, t);
    }
}

// v2 = u - s2 (y + (u/s2 - y) min(1, eps / ||u/s2 - y||)), u = v2 + s2 p
__global__ void k_dual2(float2 *__restrict__ v2, const float2 *__restrict__ p, const float2 *__restrict__ y,
                        int64_t n, float s2, double eps, const double *__restrict__ acc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double nrm = sqrt(*acc);
    const double sc = nrm > eps ? eps / nrm : 1.0;
    const double ur = (double)v2[i].x + (double)s2 * p[i].x, ui = (double)v2[i].y + (double)s2 * p[i].y;
    const double zr = ur / s2, zi = ui / s2;
    const double pr = y[i].x + (zr - y[i].x) * sc, pi = y[i].y + (zi - y[i].y) * sc;
    v2[i] = make_float2((float)(ur - s2 * pr), (float)(ui - s2 * pi));
}

// power iteration helpers: acc = sum x^2 (FP64); x = Re(z) / sqrt(acc_prev) etc.
__global__ void k_sumsq_real(const float2 *__restrict__ z, int64_t n, double *__restrict__ acc) {
    __shared__ double red[NT / 64];
    double sum = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        sum += (double)z[i].x * z[i].x;
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < NT / 64; ++w) t += red[w];
        atomicAdd(acc, t);
    }
}

__global__ void k_normalise_real(const float2 *__restrict__ z, float2 *__restrict__ xc, int64_t n,
                                 const double *__restrict__ acc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = 1.0 / sqrt(*acc);
    xc[i] = make_float2((float)(z[i].x * s), 0.f);
}

__global__ void k_copy_f32(const float *__restrict__ x, float *__restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

__global__ void k_real_to_c64(const float *__restrict__ x, float2 *__restrict__ xc, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) xc[i] = make_float2(x[i], 0.f);
}

__global__ void k_zero_f64(double *a, int n) {
    if ((int)threadIdx.x < n) a[threadIdx.x] = 0.0;
}

inline dim3 blocks_for(int64_t n) { return dim3((unsigned)((n + NT - 1) / NT)); }
inline dim3 blocks_reduce(int64_t n) {
    int64_t b = (n + NT - 1) / NT;
    return dim3((unsigned)(b > 1024 ? 1024 : (b < 1 ? 1 : b)));
}

// Daubechies with p vanishing moments: 2p taps, high-pass g_n = (-1)^n h_(2p-1-n), zero-padded to 16
Filt build_filter(int p, bool &ok) {
    double h[16] = {0.0};
    Filt f{};
    ok = daubechies(p, h);
    for (int n = 0; n < 2 * p; ++n) {
        f.h[n] = (float)h[n];
        f.g[n] = (float)(((n & 1) ? -1.0 : 1.0) * h[2 * p - 1 - n]);
    }
    return f;
}

FiltSet build_set(bool sara, bool &ok) {
    FiltSet fs{};
    ok = true;
    for (int b = 0; b < (sara ? 8 : 1); ++b) {
        bool okb;
        fs.f[b] = build_filter(sara ? b + 1 : 8, okb);
        ok = ok && okb;
    }
    return fs;
}

}  // namespace

// ---------------------------------------------------------------------------- host side

int64_t solver_workspace_bytes(const wp_plan *p, int64_t M) {
    const int64_t N2 = (int64_t)p->N * p->N, G2 = (int64_t)p->Ng * p->Ng;
    auto al = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    return al(8 * G2) + 4 * al(4 * N2) + 2 * al(8 * N2) + 2 * al(8 * M) + al(64);
}

// 0 (Dirac basis) or 1 .. while the coarsest level still has at least 8 samples per line
static wp_status check_levels(const wp_plan *p, int levels) {
    if (levels < 0 || levels > 30 || (levels > 0 && (p->N >> (levels - 1)) < 8))
        return wp_set_error(WP_EINVAL, "levels = %d: need 0 (Dirac) or 1 .. with N >> (levels-1) >= 8, N = %d",
                            levels, p->N);
    return WP_OK;
}

// the taps are computed once per process (thread-safe static initialisation)
static const FiltSet *filter_set(bool sara) {
    static bool ok8 = false, oks = false;
    static const FiltSet db8 = build_set(false, ok8);
    static const FiltSet all = build_set(true, oks);
    return sara ? (oks ? &all : nullptr) : (ok8 ? &db8 : nullptr);
}

// de (analysis) / pe (synthesis), when given, replace the stores of the final coefficients / of the
// final synthesis (the tiled path only: c != x and levels > 0)
static wp_status launch_dwt2_epi(const wp_plan *p, int levels, const float *x, float *c, float *tmp, bool synth,
                                 hipStream_t s, const DualEpi *de, const PrimalEpi *pe) {
    if (wp_status st = check_levels(p, levels)) return st;
    const FiltSet *fsp = filter_set(false);
    if (!fsp) return wp_set_error(WP_EHIP, "Daubechies filter construction failed");
    const FiltSet &fs = *fsp;
    const Filt &f = fs.f[0];
    const int N = p->N;
    if ((de || pe) && (levels == 0 || c == x))
        return wp_set_error(WP_EINVAL, "dwt2: store epilogues need the tiled path (levels > 0, c != x)");
    if (levels == 0) {                            // Dirac basis: a copy
        if (c != x) hipLaunchKernelGGL(k_copy_f32, blocks_for((int64_t)N * N), dim3(NT), 0, s, x, c, (int64_t)N * N);
        return wp_check_launch(synth ? "idwt2" : "dwt2");
    }
    if (c == x) {
        // in place: one pass per axis and level, through tmp
        for (int lv = 0; lv < levels; ++lv) {
            const int L = synth ? (N >> (levels - 1 - lv)) : (N >> lv);
            const size_t lds = sizeof(float) * L;
            const int th = L < NT ? L : NT;
            const int ls1 = synth ? 1 : N, es1 = synth ? N : 1;     // first pass: rows (analysis), columns
            hipLaunchKernelGGL(k_dwt_lines, dim3(L), dim3(th), lds, s, nullptr, c, 0, tmp, L, L, ls1, es1, f, synth);
            hipLaunchKernelGGL(k_dwt_lines, dim3(L), dim3(th), lds, s, nullptr, tmp, 0, c, L, L, es1, ls1, f, synth);
        }
        return wp_check_launch(synth ? "idwt2" : "dwt2");
    }
    // one tiled kernel per level.  The approximation passed between levels lives in tmp at
    // disjoint column ranges, so a level never reads the region it writes.
    auto tiles = [](int L) { const int H = L / 2, t = H < DT ? H : DT; return dim3((unsigned)((H / t) * (H / t))); };
    if (!synth) {
        const float *src = x;
        for (int lv = 0; lv < levels; ++lv) {
            const int L = N >> lv;
            float *ll = lv == levels - 1 ? c : tmp + (lv == 0 ? 0 : N - (N >> lv));
            hipLaunchKernelGGL(k_dwt2_fwd, tiles(L), dim3(DNT), 0, s, src, (int64_t)0, c, ll, N, L, fs,
                               de ? *de : DualEpi{nullptr, 0.f}, (int)(lv == levels - 1));
            src = ll;
        }
    } else {
        const float *llin = x;                    // the coarsest approximation is in the coefficients
        for (int st = 0; st < levels; ++st) {
            const int L = N >> (levels - 1 - st);
            float *out = st == levels - 1 ? c : tmp + ((levels - 2 - st) % 2 == 0 ? 0 : N / 2);
            const PrimalEpi none{nullptr, nullptr, nullptr, nullptr, 0.f, nullptr};
            hipLaunchKernelGGL(k_dwt2_inv, tiles(L), dim3(DNT), 0, s, x, llin, out, N, L, fs,
                               pe && st == levels - 1 ? *pe : none);
            llin = out;
        }
    }
    return wp_check_launch(synth ? "idwt2" : "dwt2");
}

// synthesis levels [st_begin, st_end) of the tiled path (as launch_dwt2_epi with synth, c != x): the
// primal epilogue, when given, applies at the last level; a range that starts past level 0 reads the
// previous level's output where launch_dwt2_epi leaves it in tmp
static wp_status launch_idwt2_range(const wp_plan *p, int levels, const float *x, float *c, float *tmp, int st_begin,
                                    int st_end, const PrimalEpi *pe, hipStream_t s) {
    const FiltSet *fsp = filter_set(false);
    if (!fsp) return wp_set_error(WP_EHIP, "Daubechies filter construction failed");
    const int N = p->N;
    auto tiles = [](int L) { const int H = L / 2, t = H < DT ? H : DT; return dim3((unsigned)((H / t) * (H / t))); };
    auto out_of = [&](int st) -> float * { return st == levels - 1 ? c : tmp + ((levels - 2 - st) % 2 == 0 ? 0 : N / 2); };
    const float *llin = st_begin == 0 ? x : out_of(st_begin - 1);
    for (int st = st_begin; st < st_end; ++st) {
        const int L = N >> (levels - 1 - st);
        float *out = out_of(st);
        const PrimalEpi none{nullptr, nullptr, nullptr, nullptr, 0.f, nullptr};
        hipLaunchKernelGGL(k_dwt2_inv, tiles(L), dim3(DNT), 0, s, x, llin, out, N, L, *fsp,
                           pe && st == levels - 1 ? *pe : none);
        llin = out;
    }
    return wp_check_launch("idwt2");
}

wp_status launch_dwt2(const wp_plan *p, int levels, const float *x, float *c, float *tmp, bool synth, hipStream_t s) {
    return launch_dwt2_epi(p, levels, x, c, tmp, synth, s, nullptr, nullptr);
}

wp_status op_phi(const wp_plan *p, const wp_operator &op, const float2 *x, float2 *y, float2 *grid, hipStream_t s) {
    return op.S ? wp_surrogate_apply_Phi(p, op.S, op.G, x, y, grid, s) : wp_apply_Phi(p, op.G, x, y, grid, s);
}

wp_status op_phiT(const wp_plan *p, const wp_operator &op, const float2 *y, float2 *x, float2 *grid, hipStream_t s) {
    return op.S ? wp_surrogate_apply_PhiT(p, op.S, op.G, y, x, grid, s) : wp_apply_PhiT(p, op.G, y, x, grid, s);
}

wp_status launch_power_norm2(const wp_plan *p, const wp_operator &op, const float *x0, int iters, double *nu,
                             unsigned char *ws, hipStream_t s) {
    const int64_t N2 = (int64_t)p->N * p->N, G2 = (int64_t)p->Ng * p->Ng;
    auto al = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    float2 *grid = (float2 *)ws;
    float2 *xc = (float2 *)(ws + al(8 * G2));
    float2 *z = (float2 *)(ws + al(8 * G2) + al(8 * N2));
    float2 *yv = (float2 *)(ws + al(8 * G2) + 2 * al(8 * N2));
    double *acc = (double *)(ws + al(8 * G2) + 2 * al(8 * N2) + al(8 * op.M));
    hipLaunchKernelGGL(k_real_to_c64, blocks_for(N2), dim3(NT), 0, s, x0, xc, N2);
    // normalise the start vector
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, acc, 2);
    hipLaunchKernelGGL(k_sumsq_real, blocks_reduce(N2), dim3(NT), 0, s, xc, N2, acc);
    hipLaunchKernelGGL(k_normalise_real, blocks_for(N2), dim3(NT), 0, s, xc, xc, N2, acc);
    for (int it = 0; it < iters; ++it) {
        if (wp_status st = op_phi(p, op, xc, yv, grid, s)) return st;
        if (wp_status st = op_phiT(p, op, yv, z, grid, s)) return st;
        hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, acc, 1);
        hipLaunchKernelGGL(k_sumsq_real, blocks_reduce(N2), dim3(NT), 0, s, z, N2, acc);
        hipLaunchKernelGGL(k_normalise_real, blocks_for(N2), dim3(NT), 0, s, z, xc, N2, acc);
    }
    double host = 0.0;
    WP_HIP(hipMemcpyAsync(&host, acc, sizeof(double), hipMemcpyDeviceToHost, s));
    WP_HIP(hipStreamSynchronize(s));
    *nu = std::sqrt(host);
    return wp_check_launch("power_norm2");
}

// Iterations per captured graph of the solver loop.
constexpr int GRAPH_ITERS = 10;

// A captured and instantiated HIP graph of solver iterations; releases everything it made.
struct SolveGraph {
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    template <typename F>
    wp_status capture(F &&iterate) {
        WP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        WP_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        const wp_status st = iterate(GRAPH_ITERS, cs);
        const hipError_t e = hipStreamEndCapture(cs, &graph);     // always end the capture
        if (st != WP_OK) return st;
        if (e != hipSuccess) return wp_set_error(WP_EHIP, "solve: graph capture: %s", hipGetErrorString(e));
        WP_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        return WP_OK;
    }
    ~SolveGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) (void)hipStreamDestroy(cs);
    }
};

wp_status launch_solve(const wp_plan *p, const wp_operator &op, const float2 *y, double eps, double nu, int iters,
                       int levels, float *x, unsigned char *ws, hipStream_t s) {
    const int64_t N2 = (int64_t)p->N * p->N, G2 = (int64_t)p->Ng * p->Ng, M = op.M;
    auto al = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    int64_t o = 0;
    auto take = [&](int64_t b) { unsigned char *r = ws + o; o += al(b); return r; };
    float2 *grid = (float2 *)take(8 * G2);
    float *v1 = (float *)take(4 * N2);
    float *t1 = (float *)take(4 * N2);
    float *xb = (float *)take(4 * N2);
    float *tmp = (float *)take(4 * N2);
    float2 *t2 = (float2 *)take(8 * N2);
    float2 *xbc = (float2 *)take(8 * N2);
    float2 *v2 = (float2 *)take(8 * M);
    float2 *pv = (float2 *)take(8 * M);
    double *acc = (double *)take(64);
    if (wp_status st = check_levels(p, levels)) return st;
    // Dirac basis (levels 0, Psi = I): the primal and dual steps in one elementwise pass
    const bool dirac = levels == 0;
    const float tau = 0.49f, s1 = 1.0f, s2 = (float)(1.0 / nu);
    WP_HIP(hipMemsetAsync(v1, 0, 4 * N2, s));
    WP_HIP(hipMemsetAsync(v2, 0, 8 * M, s));
    // With wavelets, the primal step is the last synthesis level's store epilogue and the l1 dual
    // step the analysis's (the same arithmetic as the elementwise kernels, two launches fewer).
    const PrimalEpi pe{x, t2, xb, xbc, tau, acc};
    const DualEpi de{v1, s1};
    auto iterate = [&](int n, hipStream_t st_) -> wp_status {
        for (int it = 0; it < n; ++it) {
            if (wp_status st = op_phiT(p, op, v2, t2, grid, st_)) return st;                        // Phi^H v2
            if (!dirac) {
                if (wp_status st = launch_dwt2_epi(p, levels, v1, t1, tmp, true, st_, nullptr, &pe))  // Psi v1, primal
                    return st;
                if (wp_status st = launch_dwt2_epi(p, levels, xb, t1, tmp, false, st_, &de, nullptr)) // Psi^T xb, dual
                    return st;
            } else {
                hipLaunchKernelGGL(k_primal_dual1_dirac, blocks_for(N2), dim3(NT), 0, st_, x, v1, t2, xb, xbc, N2, tau,
                                   s1, acc);
            }
            if (wp_status st = op_phi(p, op, xbc, pv, grid, st_)) return st;                        // Phi xb
            hipLaunchKernelGGL(k_ball_norm, blocks_reduce(M), dim3(NT), 0, st_, v2, pv, y, M, s2, acc);
            hipLaunchKernelGGL(k_dual2, blocks_for(M), dim3(NT), 0, st_, v2, pv, y, M, s2, eps, acc);
        }
        return wp_check_launch("solve");
    };
    // On request (plan tuning "solve_streams" = 2), with wavelets, on two streams: the analysis of xb
    // (and its l1 dual step) and the synthesis of the next v1 up to its last level depend only on xb,
    // so they run on a second stream while the caller's stream applies Phi xb, the ball step and the
    // next Phi^H v2; the last synthesis level (the primal step, which needs Phi^H v2) waits for them.
    // Events order the two streams each iteration; the loop ends with the caller's stream waiting for
    // the second one.  Measured on MI355X at the 256-pixel form: 48.2 ms per 500 iterations against
    // 44.9 ms on one stream (the cross-stream waits cost more than the overlap gains), so one stream
    // stays the default.
    if (!dirac && p->solve_graph != 1 && p->solve_streams == 2 && iters > 0) {
        wp_plan *pm = const_cast<wp_plan *>(p);      // the plan owns the stream and events (made once)
        if (!pm->aux_stream) {
            WP_HIP(hipStreamCreateWithFlags(&pm->aux_stream, hipStreamNonBlocking));
            for (hipEvent_t &e : pm->aux_ev) WP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        }
        hipStream_t sb = pm->aux_stream;
        hipEvent_t e_start = pm->aux_ev[0], e_xb = pm->aux_ev[1], e_v1 = pm->aux_ev[2];
        WP_HIP(hipEventRecord(e_start, s));         // the second stream starts after the caller's earlier work
        WP_HIP(hipStreamWaitEvent(sb, e_start, 0));
        if (wp_status st = launch_idwt2_range(p, levels, v1, t1, tmp, 0, levels - 1, nullptr, sb)) return st;
        WP_HIP(hipEventRecord(e_v1, sb));
        for (int it = 0; it < iters; ++it) {
            if (wp_status st = op_phiT(p, op, v2, t2, grid, s)) return st;                          // Phi^H v2
            WP_HIP(hipStreamWaitEvent(s, e_v1, 0));
            if (wp_status st = launch_idwt2_range(p, levels, v1, t1, tmp, levels - 1, levels, &pe, s))  // primal
                return st;
            WP_HIP(hipEventRecord(e_xb, s));
            if (wp_status st = op_phi(p, op, xbc, pv, grid, s)) return st;                          // Phi xb
            hipLaunchKernelGGL(k_ball_norm, blocks_reduce(M), dim3(NT), 0, s, v2, pv, y, M, s2, acc);
            hipLaunchKernelGGL(k_dual2, blocks_for(M), dim3(NT), 0, s, v2, pv, y, M, s2, eps, acc);
            WP_HIP(hipStreamWaitEvent(sb, e_xb, 0));
            if (wp_status st = launch_dwt2_epi(p, levels, xb, t1, tmp, false, sb, &de, nullptr))    // Psi^T xb, dual
                return st;
            if (it + 1 < iters)
                if (wp_status st = launch_idwt2_range(p, levels, v1, t1, tmp, 0, levels - 1, nullptr, sb)) return st;
            WP_HIP(hipEventRecord(e_v1, sb));
        }
        WP_HIP(hipStreamWaitEvent(s, e_v1, 0));
        return wp_check_launch("solve");
    }
    if (p->solve_graph != 1 || iters < 2 * GRAPH_ITERS) return iterate(iters, s);
    // On request (plan tuning "solve_graph" = 1): a chunk of GRAPH_ITERS iterations (16 dependent
    // launches each) captured once into a HIP graph on a private stream and replayed on the caller's.
    // The loop holds no memset and no host synchronisation, so every replay repeats the same work on
    // the same buffers.  Measured on MI355X at the 256-pixel form, the replays ran slower than the
    // direct launches (49.2 against 44.6 ms per 500 iterations), so direct launches stay the default.
    SolveGraph g;
    if (wp_status st = g.capture(iterate)) return st;
    wp_status st = WP_OK;
    for (int i = 0; i < iters / GRAPH_ITERS && st == WP_OK; ++i) {
        const hipError_t e = hipGraphLaunch(g.exec, s);
        if (e != hipSuccess) st = wp_set_error(WP_EHIP, "solve: graph launch: %s", hipGetErrorString(e));
    }
    if (st == WP_OK) st = iterate(iters % GRAPH_ITERS, s);
    const hipError_t e = hipStreamSynchronize(s);     // the replays must end before the graph is released
    if (st == WP_OK && e != hipSuccess) st = wp_set_error(WP_EHIP, "solve: %s", hipGetErrorString(e));
    return st;
}

// ---------------------------------------------------------------------------- SARA (Section 4.2)
// Psi = [I, W_1, ..., W_8] / 3 with W_p the Daubechies wavelets of p vanishing moments (`levels`
// levels, periodic): a tight frame with Psi Psi^T = I.  Coefficients are [9][N][N] (Dirac first);
// the eight wavelet transforms of a level run in one launch (basis = blockIdx.y).

static wp_status check_sara_levels(const wp_plan *p, int levels) {
    if (levels < 1 || levels > 30 || (p->N >> (levels - 1)) < 8)
        return wp_set_error(WP_EINVAL, "levels = %d: SARA needs 1 .. with N >> (levels-1) >= 8, N = %d", levels,
                            p->N);
    return WP_OK;
}

static dim3 sara_tiles(int L) {
    const int H = L / 2, t = H < DT ? H : DT;
    return dim3((unsigned)((H / t) * (H / t)), 8);
}

// the eight wavelet analyses of x into c_1 .. c_8 (unscaled); tmp holds 8 N^2 floats
static wp_status sara_analysis_levels(const wp_plan *p, int levels, const float *x, float *c, float *tmp,
                                      hipStream_t s) {
    if (wp_status st = check_sara_levels(p, levels)) return st;
    const FiltSet *fs = filter_set(true);
    if (!fs) return wp_set_error(WP_EHIP, "Daubechies filter construction failed");
    const int N = p->N;
    const int64_t N2 = (int64_t)N * N;
    const float *src = x;
    int64_t in_zs = 0;                            // every basis reads x at the first level
    for (int lv = 0; lv < levels; ++lv) {
        const int L = N >> lv;
        float *ll = lv == levels - 1 ? c + N2 : tmp + (lv == 0 ? 0 : N - (N >> lv));
        hipLaunchKernelGGL(k_dwt2_fwd, sara_tiles(L), dim3(DNT), 0, s, src, in_zs, c + N2, ll, N, L, *fs);
        src = ll;
        in_zs = N2;
    }
    return WP_OK;
}

// c = Psi^T x; tmp holds 8 N^2 floats (the approximations between levels, one image per basis)
wp_status launch_sara_analysis(const wp_plan *p, int levels, const float *x, float *c, float *tmp, hipStream_t s) {
    if (wp_status st = sara_analysis_levels(p, levels, x, c, tmp, s)) return st;
    const int64_t N2 = (int64_t)p->N * p->N;
    hipLaunchKernelGGL(k_sara_scale, blocks_for(N2), dim3(NT), 0, s, x, c, N2);
    return wp_check_launch("sara_analysis");
}

// the eight wavelet syntheses of c_1 .. c_8 into tmp + 8 N^2 (one image per basis); tmp holds 16 N^2
// floats (per basis: the coarser levels' results, then its synthesis)
static wp_status sara_synthesis_levels(const wp_plan *p, int levels, const float *c, float *tmp, hipStream_t s) {
    if (wp_status st = check_sara_levels(p, levels)) return st;
    const FiltSet *fs = filter_set(true);
    if (!fs) return wp_set_error(WP_EHIP, "Daubechies filter construction failed");
    const int N = p->N;
    const int64_t N2 = (int64_t)N * N;
    const float *coef = c + N2, *llin = c + N2;
    for (int st = 0; st < levels; ++st) {
        const int L = N >> (levels - 1 - st);
        float *out = st == levels - 1 ? tmp + 8 * N2 : tmp + ((levels - 2 - st) % 2 == 0 ? 0 : N / 2);
        hipLaunchKernelGGL(k_dwt2_inv, sara_tiles(L), dim3(DNT), 0, s, coef, llin, out, N, L, *fs);
        llin = out;
    }
    return WP_OK;
}

// x = Psi c; tmp holds 16 N^2 floats
wp_status launch_sara_synthesis(const wp_plan *p, int levels, const float *c, float *x, float *tmp, hipStream_t s) {
    if (wp_status st = sara_synthesis_levels(p, levels, c, tmp, s)) return st;
    const int64_t N2 = (int64_t)p->N * p->N;
    hipLaunchKernelGGL(k_sara_sum, blocks_for(N2), dim3(NT), 0, s, c, tmp + 8 * N2, x, N2);
    return wp_check_launch("sara_synthesis");
}

int64_t sara_workspace_bytes(const wp_plan *p, int64_t M) {
    const int64_t N2 = (int64_t)p->N * p->N, G2 = (int64_t)p->Ng * p->Ng;
    auto al = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    return al(8 * G2) + 3 * al(4 * 9 * N2) + al(4 * N2) + al(4 * 16 * N2) + 2 * al(8 * N2) + 2 * al(8 * M) + al(64);
}

// Reweighted analysis over the SARA dictionary: `rounds` primal-dual solves of `iters` iterations
// with the weighted norm ||W Psi^T x||_1, x carried over, duals restarted at zero; round 0 has
// unit weights, round r >= 1 w = delta_r / (delta_r + |Psi^T x|), delta_1 = the standard
// deviation of Psi^T x, delta_(r+1) = delta_r / 10.
wp_status launch_sara_solve(const wp_plan *p, const wp_operator &op, const float2 *y, double eps, double nu, int iters,
                            int rounds, int levels, float *x, unsigned char *ws, hipStream_t s) {
    if (wp_status st = check_sara_levels(p, levels)) return st;
    const int64_t N2 = (int64_t)p->N * p->N, G2 = (int64_t)p->Ng * p->Ng, M = op.M, NC = 9 * N2;
    auto al = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    int64_t o = 0;
    auto take = [&](int64_t b) { unsigned char *r = ws + o; o += al(b); return r; };
    float2 *grid = (float2 *)take(8 * G2);
    float *v1 = (float *)take(4 * NC);
    float *tc = (float *)take(4 * NC);
    float *w = (float *)take(4 * NC);
    float *xb = (float *)take(4 * N2);
    float *tmp = (float *)take(4 * 16 * N2);
    float2 *t2 = (float2 *)take(8 * N2);
    float2 *xbc = (float2 *)take(8 * N2);
    float2 *v2 = (float2 *)take(8 * M);
    float2 *pv = (float2 *)take(8 * M);
    double *acc = (double *)take(64);
    const float tau = 0.49f, s1 = 1.0f, s2 = (float)(1.0 / nu);
    double delta = 0.0;
    for (int r = 0; r < rounds; ++r) {
        if (r == 0) {
            hipLaunchKernelGGL(k_fill_f32, blocks_for(NC), dim3(NT), 0, s, w, NC, 1.0f);
        } else {
            if (wp_status st = launch_sara_analysis(p, levels, x, tc, tmp, s)) return st;       // alpha
            if (r == 1) {
                double h[2] = {0.0, 0.0};
                hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, acc, 2);
                hipLaunchKernelGGL(k_sum_dev, blocks_reduce(NC), dim3(NT), 0, s, tc, NC, acc, 0);
                hipLaunchKernelGGL(k_sum_dev, blocks_reduce(NC), dim3(NT), 0, s, tc, NC, acc, 1);
                WP_HIP(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
                WP_HIP(hipStreamSynchronize(s));
                delta = std::sqrt(h[1] / (double)NC);
            } else {
                delta /= 10.0;
            }
            hipLaunchKernelGGL(k_sara_weights, blocks_for(NC), dim3(NT), 0, s, tc, w, NC, delta);
        }
        WP_HIP(hipMemsetAsync(v1, 0, 4 * NC, s));
        WP_HIP(hipMemsetAsync(v2, 0, 8 * M, s));
        // the primal step joins the synthesis's final sum and the dual step the analysis's final
        // scaling (the same arithmetic as the separate kernels); Phi^H v2 goes first (independent)
        for (int it = 0; it < iters; ++it) {
            if (wp_status st = op_phiT(p, op, v2, t2, grid, s)) return st;                      // Phi^H v2
            if (wp_status st = sara_synthesis_levels(p, levels, v1, tmp, s)) return st;         // Psi v1
            hipLaunchKernelGGL(k_sara_sum_primal, blocks_for(N2), dim3(NT), 0, s, v1, tmp + 8 * N2, x, t2, xb, xbc,
                               N2, tau, acc);
            if (wp_status st = sara_analysis_levels(p, levels, xb, tc, tmp, s)) return st;      // Psi^T xb
            hipLaunchKernelGGL(k_sara_scale_dual, blocks_for(N2), dim3(NT), 0, s, xb, tc, v1, w, N2, s1);
            if (wp_status st = op_phi(p, op, xbc, pv, grid, s)) return st;                      // Phi xb
            hipLaunchKernelGGL(k_ball_norm, blocks_reduce(M), dim3(NT), 0, s, v2, pv, y, M, s2, acc);
            hipLaunchKernelGGL(k_dual2, blocks_for(M), dim3(NT), 0, s, v2, pv, y, M, s2, eps, acc);
        }
    }
    return wp_check_launch("sara_solve");
}

// ---------------------------------------------------------------------------- Douglas-Rachford
// Eq. 7 as printed (no positivity), the splitting Section 2.3 names:
//   x = P_C(z);  z = z + Psi soft_gamma(Psi^T (2 x - z)) - x,   z_0 = 0,
// C = {x : ||y - Phi x|| <= eps}.  P_C by forward-backward on its dual u (carried over between
// outer iterations, zero at the start): `inner` times p = Phi (z - Re Phi^H u), then the ball step
// of the primal-dual solver's second dual variable with sigma = 1 / ||Phi||^2; P_C(z) = z - Re Phi^H u.

int64_t dr_workspace_bytes(const wp_plan *p, int64_t M) {
    const int64_t N2 = (int64_t)p->N * p->N, G2 = (int64_t)p->Ng * p->Ng;
    auto al = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    return al(8 * G2) + 5 * al(4 * N2) + 2 * al(8 * N2) + 2 * al(8 * M) + al(64);
}

wp_status launch_dr_solve(const wp_plan *p, const wp_operator &op, const float2 *y, double eps, double nu, int iters,
                          int inner, double gamma, int levels, float *x, unsigned char *ws, hipStream_t s) {
    if (wp_status st = check_levels(p, levels)) return st;
    const int64_t N2 = (int64_t)p->N * p->N, G2 = (int64_t)p->Ng * p->Ng, M = op.M;
    auto al = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    int64_t o = 0;
    auto take = [&](int64_t b) { unsigned char *r = ws + o; o += al(b); return r; };
    float2 *grid = (float2 *)take(8 * G2);
    float *z = (float *)take(4 * N2);
    float *xi = (float *)take(4 * N2);
    float *r = (float *)take(4 * N2);
    float *c = (float *)take(4 * N2);
    float *tmp = (float *)take(4 * N2);
    float2 *t2 = (float2 *)take(8 * N2);
    float2 *xc = (float2 *)take(8 * N2);
    float2 *u = (float2 *)take(8 * M);
    float2 *pv = (float2 *)take(8 * M);
    double *acc = (double *)take(64);
    const float mu = (float)(1.0 / nu), g = (float)gamma;
    WP_HIP(hipMemsetAsync(z, 0, 4 * N2, s));
    WP_HIP(hipMemsetAsync(u, 0, 8 * M, s));
    for (int it = 0; it < iters; ++it) {
        for (int i = 0; i < inner; ++i) {
            if (wp_status st = op_phiT(p, op, u, t2, grid, s)) return st;                 // Phi^H u
            hipLaunchKernelGGL(k_dr_sub, blocks_for(N2), dim3(NT), 0, s, z, t2, xi, xc, N2);
            if (wp_status st = op_phi(p, op, xc, pv, grid, s)) return st;                 // Phi (z - Re Phi^H u)
            hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, acc, 1);
            hipLaunchKernelGGL(k_ball_norm, blocks_reduce(M), dim3(NT), 0, s, u, pv, y, M, mu, acc);
            hipLaunchKernelGGL(k_dual2, blocks_for(M), dim3(NT), 0, s, u, pv, y, M, mu, eps, acc);
        }
        if (wp_status st = op_phiT(p, op, u, t2, grid, s)) return st;
        hipLaunchKernelGGL(k_dr_sub, blocks_for(N2), dim3(NT), 0, s, z, t2, x, nullptr, N2);   // x = P_C(z)
        hipLaunchKernelGGL(k_dr_reflect, blocks_for(N2), dim3(NT), 0, s, x, z, r, N2);
        if (levels == 0) {
            hipLaunchKernelGGL(k_soft, blocks_for(N2), dim3(NT), 0, s, r, N2, g);                // Dirac basis
            hipLaunchKernelGGL(k_dr_update, blocks_for(N2), dim3(NT), 0, s, z, r, x, N2);
        } else {
            if (wp_status st = launch_dwt2(p, levels, r, c, tmp, false, s)) return st;
            hipLaunchKernelGGL(k_soft, blocks_for(N2), dim3(NT), 0, s, c, N2, g);
            if (wp_status st = launch_dwt2(p, levels, c, r, tmp, true, s)) return st;
            hipLaunchKernelGGL(k_dr_update, blocks_for(N2), dim3(NT), 0, s, z, r, x, N2);
        }
    }
    return wp_check_launch("dr_solve");
}

wp_status filter_db8(double *h) { return daubechies(8, h) ? WP_OK : wp_set_error(WP_EHIP, "filter"); }
