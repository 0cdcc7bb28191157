// Learned surrogate of the sparsified rows: the network's forward and backward
// passes, Adam, the training loop, the exact training targets taken from rows the
// builder made, and the per-row energy error of the surrogate against exact rows.
//
// The surrogate maps (w, du, dv) -- w and the offset of (u~, v~) from its nearest
// grid cell c = floor(u~ + 1/2) -- to the taps of the row (Section 3.1 kernel,
// Section 3.2 energy rule) on the 32 x 32 cells (c_v - 16 .. c_v + 15) x
// (c_u - 16 .. c_u + 15), modulo Ng.  Output 2 p (+1) is the real (imaginary) part
// of box cell p = 32 oy + ox, times the output scale s_out.
//
// Mixed precision: products W_l a_{l-1} (l = 2..4) and the backward products take
// bfloat16 operands with FP32 accumulation; the first layer (3 inputs), biases,
// GELU, the loss, bias and W1 gradients and Adam run in FP32.
#include <cmath>
#include <cstring>

#include "mlp_core.h"

using namespace mlpc;

namespace {

constexpr int NTH = 256;

// ---------------------------------------------------------------------------- products

template <int BM, int BN, int LA, int LB, class Epi>
__global__ __launch_bounds__(NTH) void k_gemm(const uint16_t *__restrict__ A, int64_t lda,
                                              const uint16_t *__restrict__ B, int64_t ldb, int M, int N,
                                              int64_t kper, Epi epi) {
    constexpr int FM = BM / 64, FN = BN / 64;
    __shared__ __align__(16) uint16_t As[BM * LDK];
    __shared__ __align__(16) uint16_t Bs[BN * LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int64_t kbeg = (int64_t)blockIdx.z * kper, kend = kbeg + kper;
    f32x16 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
        stage_tile<BM, LA, NTH>(As, A, lda, M, m0, k0, tid);
        stage_tile<BN, LB, NTH>(Bs, B, ldb, N, n0, k0, tid);
        __syncthreads();
        mma_bk<FM, FN>(acc, As, Bs, wm * (BM / 2), wn * (BN / 2), lane);
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = m0 + wm * (BM / 2) + 32 * a + acc_row(r, lane);
                const int j = n0 + wn * (BN / 2) + 32 * b + acc_col(lane);
                if (i < M && j < N) epi(i, j, acc[a][b][r]);
            }
}

// z = acc + b; a = gelu(z)
struct EpiHidden {
    const float *bias;
    float *z;
    uint16_t *a;
    int ld;
    __device__ void operator()(int i, int j, float v) const {
        const float zz = v + bias[j];
        z[(int64_t)i * ld + j] = zz;
        a[(int64_t)i * ld + j] = to_bf16(gelu(zz));
    }
};
// o = acc + b
struct EpiOut {
    const float *bias;
    float *o;
    int ld;
    __device__ void operator()(int i, int j, float v) const { o[(int64_t)i * ld + j] = v + bias[j]; }
};
// dz = acc * gelu'(z)
struct EpiDGelu {
    const float *z;
    float *dz;
    uint16_t *dzb;
    int ld;
    __device__ void operator()(int i, int j, float v) const {
        const int64_t e = (int64_t)i * ld + j;
        const float d = v * gelu_grad(z[e]);
        dz[e] = d;
        dzb[e] = to_bf16(d);
    }
};
// C += acc (split-K partial products)
struct EpiAtomic {
    float *C;
    int ld;
    __device__ void operator()(int i, int j, float v) const { atomicAdd(C + (int64_t)i * ld + j, v); }
};

template <int BM, int BN, int LA, int LB, class Epi>
wp_status gemm(const uint16_t *A, int64_t lda, const uint16_t *B, int64_t ldb, int M, int N, int64_t K, int ksplit,
               Epi epi, hipStream_t s) {
    if (K % ((int64_t)BK * ksplit)) return wp_set_error(WP_EINVAL, "product depth %lld not a multiple of %d",
                                                        (long long)K, BK * ksplit);
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, ksplit);
    k_gemm<BM, BN, LA, LB, Epi><<<grid, NTH, 0, s>>>(A, lda, B, ldb, M, N, K / ksplit, epi);
    return wp_check_launch("k_gemm");
}

// ---------------------------------------------------------------------------- elementwise kernels

__global__ void k_layer1(const float *__restrict__ X, int n, const float *__restrict__ W1,
                         const float *__restrict__ b1, float *__restrict__ z1, uint16_t *__restrict__ a1) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * H) return;
    const int64_t i = e / H;
    const int j = (int)(e % H);
    const float z = X[3 * i] * W1[3 * j] + X[3 * i + 1] * W1[3 * j + 1] + X[3 * i + 2] * W1[3 * j + 2] + b1[j];
    z1[e] = z;
    a1[e] = to_bf16(gelu(z));
}

// dO = (o - t) * scale (scale = 2 / (n NOUT)); loss += sum (o - t)^2
__global__ void k_loss(const float *__restrict__ o, const float *__restrict__ t, int64_t total, float scale,
                       float *__restrict__ dO, uint16_t *__restrict__ dOb, double *__restrict__ loss) {
    __shared__ double red[NTH / 64];
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * NTH + threadIdx.x; e < total; e += (int64_t)gridDim.x * NTH) {
        const float d = o[e] - t[e];
        acc += (double)d * d;
        const float g = d * scale;
        dO[e] = g;
        dOb[e] = to_bf16(g);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < NTH / 64; ++w) s += red[w];
        atomicAdd(loss, s);
    }
}

// out[j] += sum over rows i of d[i ld + j]; 64 columns per block, rows split over gridDim.y
__global__ void k_colsum(const float *__restrict__ d, int n, int ld, float *__restrict__ out) {
    __shared__ float red[NTH];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    float acc = 0.0f;
    for (int i = blockIdx.y * 4 + g; i < n; i += gridDim.y * 4) acc += d[(int64_t)i * ld + j];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (g == 0) atomicAdd(out + j, red[c] + red[c + 64] + red[c + 128] + red[c + 192]);
}

// first-layer gradients: dW1[j][c] += sum_i dz1[i][j] X[i][c], db1[j] += sum_i dz1[i][j]
__global__ void k_grad_layer1(const float *__restrict__ dz1, const float *__restrict__ X, int n,
                              float *__restrict__ dW1, float *__restrict__ db1) {
    __shared__ float red[4][NTH];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, sb = 0.f;
    for (int i = blockIdx.y * 4 + g; i < n; i += gridDim.y * 4) {
        const float d = dz1[(int64_t)i * H + j];
        s0 += d * X[3 * (int64_t)i];
        s1 += d * X[3 * (int64_t)i + 1];
        s2 += d * X[3 * (int64_t)i + 2];
        sb += d;
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    red[3][threadIdx.x] = sb;
    __syncthreads();
    if (g == 0) {
        float r[4];
        for (int q = 0; q < 4; ++q) r[q] = red[q][c] + red[q][c + 64] + red[q][c + 128] + red[q][c + 192];
        atomicAdd(dW1 + 3 * j, r[0]);
        atomicAdd(dW1 + 3 * j + 1, r[1]);
        atomicAdd(dW1 + 3 * j + 2, r[2]);
        atomicAdd(db1 + j, r[3]);
    }
}

__global__ void k_adam(float *__restrict__ p, float *__restrict__ m1, float *__restrict__ m2,
                       const float *__restrict__ g, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    for (int64_t e = (int64_t)blockIdx.x * NTH + threadIdx.x; e < n; e += (int64_t)gridDim.x * NTH) {
        const float ge = g[e];
        const float a = b1 * m1[e] + (1.0f - b1) * ge;
        const float b = b2 * m2[e] + (1.0f - b2) * ge * ge;
        m1[e] = a;
        m2[e] = b;
        p[e] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
    }
}

__global__ void k_to_bf16(const float *__restrict__ src, uint16_t *__restrict__ dst, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * NTH + threadIdx.x; e < n; e += (int64_t)gridDim.x * NTH)
        dst[e] = to_bf16(src[e]);
}

// minibatch b: sample (a i + c) mod n for i < nb
__global__ void k_gather_batch(const float *__restrict__ feat, const float *__restrict__ targ, int64_t n,
                               int64_t a, int64_t c, int nb, float *__restrict__ xb, float *__restrict__ tb) {
    const int i = blockIdx.x;
    const int64_t src = (a * i + c) % n;
    if (threadIdx.x < 3) xb[3 * i + threadIdx.x] = feat[3 * src + threadIdx.x];
    const float4 *ts = (const float4 *)(targ + src * NOUT);
    float4 *td = (float4 *)(tb + (int64_t)i * NOUT);
    for (int e = threadIdx.x; e < NOUT / 4; e += NTH) td[e] = ts[e];
    (void)nb;
}

// features (2 w / w_top - 1, 2 du, 2 dv) with du = u~ - floor(u~ + 1/2)
__global__ void k_features(const double *__restrict__ u, const double *__restrict__ v, const double *__restrict__ w,
                           int64_t n, double cell, double half, double w_top, float *__restrict__ feat,
                           int *__restrict__ err) {
    const int64_t k = (int64_t)blockIdx.x * NTH + threadIdx.x;
    if (k >= n) return;
    const double ut = u[k] / cell, vt = v[k] / cell, wk = w[k];
    if (!(isfinite(ut) && isfinite(vt) && isfinite(wk) && fabs(ut) < half && fabs(vt) < half)) atomicOr(err, 1);
    const double du = ut - floor(ut + 0.5), dv = vt - floor(vt + 0.5);
    feat[3 * k] = (float)(2.0 * wk / w_top - 1.0);
    feat[3 * k + 1] = (float)(2.0 * du);
    feat[3 * k + 2] = (float)(2.0 * dv);
}

__device__ inline int box_cell(double gt, int Ng) {
    const long long c = (long long)floor(gt + 0.5) + Ng / 2;
    return (int)(((c % Ng) + Ng) % Ng);
}

__device__ inline double wave_sum(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off);
    return __shfl(x, 0);
}

// exact training targets: row of visibility k (sorted row r, k = perm[r]) scattered
// into its box, divided by s_out; lost[k] = row energy outside the box / row energy
__global__ void k_box_targets(const int64_t *__restrict__ rowptr, const int *__restrict__ col,
                              const float2 *__restrict__ val, const int *__restrict__ perm, int64_t M,
                              const double *__restrict__ u, const double *__restrict__ v, double cell, int logNg,
                              float inv_s, float *__restrict__ target, float *__restrict__ lost) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (NTH / 64) + (threadIdx.x >> 6);
    if (r >= M) return;
    const int Ng = 1 << logNg;
    const int k = perm[r];
    const int cu = box_cell(u[k] / cell, Ng), cv = box_cell(v[k] / cell, Ng);
    double tot = 0.0, out = 0.0;
    for (int64_t e = rowptr[r] + lane; e < rowptr[r + 1]; e += 64) {
        const int c = col[e];
        const int oy = ((c >> logNg) - cv + BOX / 2) & (Ng - 1);
        const int ox = ((c & (Ng - 1)) - cu + BOX / 2) & (Ng - 1);
        const float2 g = val[e];
        const double e2 = (double)g.x * g.x + (double)g.y * g.y;
        tot += e2;
        if (oy < BOX && ox < BOX) {
            float *t = target + (int64_t)k * NOUT + 2 * (oy * BOX + ox);
            t[0] = g.x * inv_s;
            t[1] = g.y * inv_s;
        } else {
            out += e2;
        }
    }
    tot = wave_sum(tot);
    out = wave_sum(out);
    if (lane == 0) lost[k] = tot > 0.0 ? (float)(out / tot) : 0.0f;
}

// features of sorted rows r0 .. r0 + n - 1
__global__ void k_gather_feat(const float *__restrict__ feat, const int *__restrict__ perm, int64_t r0, int n,
                              float *__restrict__ out) {
    const int i = blockIdx.x * NTH + threadIdx.x;
    if (i >= 3 * n) return;
    out[i] = feat[3 * (int64_t)perm[r0 + i / 3] + i % 3];
}

// eps[k] = ||t - g||^2 / ||g||^2 for sorted rows r0 .. r0 + n - 1 (network outputs o in that order)
__global__ __launch_bounds__(NTH) void k_row_errors(const float *__restrict__ o, int64_t r0, int n,
                                                    const int64_t *__restrict__ rowptr, const int *__restrict__ col,
                                                    const float2 *__restrict__ val, const int *__restrict__ perm,
                                                    const double *__restrict__ u, const double *__restrict__ v,
                                                    double cell, int logNg, float s_out, float *__restrict__ eps,
                                                    float *__restrict__ energy) {
    __shared__ float2 box[NTH / 64][BOX * BOX];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * (NTH / 64) + wv;
    const bool live = i < n;
    const int Ng = 1 << logNg;
    const int64_t r = r0 + (live ? i : 0);
    const int k = perm[r];
    float2 *bx = box[wv];
    for (int p = lane; p < BOX * BOX; p += 64) {
        const float2 t = live ? ((const float2 *)(o + (int64_t)i * NOUT))[p] : make_float2(0.f, 0.f);
        bx[p] = make_float2(t.x * s_out, t.y * s_out);
    }
    __syncthreads();
    double tot = 0.0, out = 0.0;
    if (live) {
        const int cu = box_cell(u[k] / cell, Ng), cv = box_cell(v[k] / cell, Ng);
        for (int64_t e = rowptr[r] + lane; e < rowptr[r + 1]; e += 64) {
            const int c = col[e];
            const int oy = ((c >> logNg) - cv + BOX / 2) & (Ng - 1);
            const int ox = ((c & (Ng - 1)) - cu + BOX / 2) & (Ng - 1);
            const float2 g = val[e];
            tot += (double)g.x * g.x + (double)g.y * g.y;
            if (oy < BOX && ox < BOX) {
                float2 &b = bx[oy * BOX + ox];
                b.x -= g.x;
                b.y -= g.y;
            } else {
                out += (double)g.x * g.x + (double)g.y * g.y;
            }
        }
    }
    __syncthreads();
    double d = 0.0;
    for (int p = lane; p < BOX * BOX; p += 64) d += (double)bx[p].x * bx[p].x + (double)bx[p].y * bx[p].y;
    d = wave_sum(d);
    tot = wave_sum(tot);
    out = wave_sum(out);
    if (live && lane == 0) {
        eps[k] = tot > 0.0 ? (float)((d + out) / tot) : 0.0f;
        if (energy) energy[k] = (float)tot;
    }
}

// Check lattice: node i = (iw nd + iv) nd + iu at w = w_top iw / (nw - 1) and offsets du = -1/2 + iu / (nd - 1)
// (dv likewise) from the centre cell; the last offset node sits just below +1/2, so that it keeps the
// centre cell (at +1/2 the nearest cell would change).
__global__ void k_lattice_coords(int nw, int nd, double w_top, double cell, double *__restrict__ u,
                                 double *__restrict__ v, double *__restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * NTH + threadIdx.x;
    const int64_t n = (int64_t)nw * nd * nd;
    if (i >= n) return;
    const int iu = (int)(i % nd), iv = (int)((i / nd) % nd), iw = (int)(i / ((int64_t)nd * nd));
    auto off = [nd](int j) { return j == nd - 1 ? 0.5 - 0x1p-20 : -0.5 + (double)j / (double)(nd - 1); };
    u[i] = off(iu) * cell;
    v[i] = off(iv) * cell;
    w[i] = w_top * (double)iw / (double)(nw - 1);
}

// Run-time per-row check of network rows k0 .. k0 + n - 1 (caller order; outputs o of those rows), from
// the check lattice alone (no exact row):
//   est = max( largest node error of the lattice cell holding (w, du, dv),
//              (| ||t|| - sqrt(K) | / sqrt(K))^2 )
// with K the kept energy interpolated trilinearly between the cell's nodes.  The second term is a lower
// bound of the row's error ||t - g||^2 / ||g||^2 by the reverse triangle inequality when K = ||g||^2.
// A row outside the lattice (w beyond the trained range) or with a non-finite value gets +infinity.
__global__ __launch_bounds__(NTH) void k_row_check(const float *__restrict__ o, int64_t k0, int n,
                                                   const float *__restrict__ feat, const float *__restrict__ table,
                                                   int nw, int nd, float s_out, float *__restrict__ est) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (NTH / 64) + (threadIdx.x >> 6);
    if (i >= n) return;
    const float *oi = o + (int64_t)i * NOUT;
    double e = 0.0;
    for (int p = lane; p < NOUT; p += 64) e += (double)oi[p] * oi[p];
    e = wave_sum(e);
    if (lane != 0) return;
    const int64_t k = k0 + i;
    const float *f = feat + 3 * k;
    const double wf = (0.5 * ((double)f[0] + 1.0)) * (nw - 1);
    const double uf = (0.5 * (double)f[1] + 0.5) * (nd - 1), vf = (0.5 * (double)f[2] + 0.5) * (nd - 1);
    float r = INFINITY;
    if (wf >= 0.0 && wf <= (double)(nw - 1) && uf >= 0.0 && uf <= (double)(nd - 1) && vf >= 0.0 &&
        vf <= (double)(nd - 1) && isfinite(e)) {
        const int iw = min((int)wf, nw - 2), iu = min((int)uf, nd - 2), iv = min((int)vf, nd - 2);
        const double tw = wf - iw, tu = uf - iu, tv = vf - iv;
        const int64_t nodes = (int64_t)nw * nd * nd;
        float emax = 0.0f;
        double K = 0.0;
        for (int c = 0; c < 8; ++c) {
            const int a = c & 1, b = (c >> 1) & 1, d = c >> 2;
            const int64_t node = ((int64_t)(iw + d) * nd + (iv + b)) * nd + (iu + a);
            const float en = table[node];
            emax = (en > emax || en != en) ? en : emax;            // a NaN node error propagates
            K += (a ? tu : 1.0 - tu) * (b ? tv : 1.0 - tv) * (d ? tw : 1.0 - tw) * (double)table[nodes + node];
        }
        const double tn = (double)s_out * sqrt(e);
        const double lb = K > 0.0 ? (tn - sqrt(K)) * (tn - sqrt(K)) / K : INFINITY;
        r = fmaxf(emax, (float)lb);
        if (emax != emax) r = emax;
    }
    est[k] = r;
}

int blocks_for(int64_t n, int per = NTH) { return (int)std::min<int64_t>((n + per - 1) / per, 65536); }

wp_status refresh_bf16(wp_mlp *m, hipStream_t s) {
    k_to_bf16<<<blocks_for((int64_t)H * H), NTH, 0, s>>>(m->params + OW2, m->W2b, (int64_t)H * H);
    k_to_bf16<<<blocks_for((int64_t)H * H), NTH, 0, s>>>(m->params + OW3, m->W3b, (int64_t)H * H);
    k_to_bf16<<<blocks_for((int64_t)NOUT * H), NTH, 0, s>>>(m->params + OW4, m->W4b, (int64_t)NOUT * H);
    return wp_check_launch("k_to_bf16");
}

wp_status check_mlp(const wp_mlp *m) {
    if (!m) return wp_set_error(WP_EINVAL, "mlp is NULL");
    return WP_OK;
}

// forward and backward of n rows; gradients into m->grad (zeroed first), loss sum into m->loss (added)
wp_status mlp_backward(wp_mlp *m, int n, const float *X, const float *T, hipStream_t s) {
    wp_status st = mlp_forward(m, n, X, m->o, s);
    if (st != WP_OK) return st;
    if ((st = launch_fill_zero(m->grad, NPARAM, s)) != WP_OK) return st;
    const int64_t tot = (int64_t)n * NOUT;
    k_loss<<<blocks_for(tot, NTH * 8), NTH, 0, s>>>(m->o, T, tot, 2.0f / (float)tot, m->dO, m->dOb, m->loss);
    if ((st = wp_check_launch("k_loss")) != WP_OK) return st;
    int ks = 1;                                     // split-K over the batch for the weight gradients
    while (2 * ks <= n / 512 && n % (BK * 2 * ks) == 0) ks *= 2;
    const int rows_split = std::max(1, std::min(64, n / 64));
    // layer 4
    if ((st = gemm<128, 128, RC, RC>(m->dOb, NOUT, m->a3, H, NOUT, H, n, ks, EpiAtomic{m->grad + OW4, H}, s)) != WP_OK)
        return st;
    k_colsum<<<dim3(NOUT / 64, rows_split), NTH, 0, s>>>(m->dO, n, NOUT, m->grad + OB4);
    if ((st = gemm<64, 64, KC, RC>(m->dOb, NOUT, m->W4b, H, n, H, NOUT, 1, EpiDGelu{m->z3, m->dzA, m->dzAb, H}, s)) !=
        WP_OK)
        return st;
    // layer 3
    if ((st = gemm<64, 64, RC, RC>(m->dzAb, H, m->a2, H, H, H, n, ks, EpiAtomic{m->grad + OW3, H}, s)) != WP_OK)
        return st;
    k_colsum<<<dim3(H / 64, rows_split), NTH, 0, s>>>(m->dzA, n, H, m->grad + OB3);
    if ((st = gemm<64, 64, KC, RC>(m->dzAb, H, m->W3b, H, n, H, H, 1, EpiDGelu{m->z2, m->dzB, m->dzBb, H}, s)) != WP_OK)
        return st;
    // layer 2
    if ((st = gemm<64, 64, RC, RC>(m->dzBb, H, m->a1, H, H, H, n, ks, EpiAtomic{m->grad + OW2, H}, s)) != WP_OK)
        return st;
    k_colsum<<<dim3(H / 64, rows_split), NTH, 0, s>>>(m->dzB, n, H, m->grad + OB2);
    if ((st = gemm<64, 64, KC, RC>(m->dzBb, H, m->W2b, H, n, H, H, 1, EpiDGelu{m->z1, m->dzA, m->dzAb, H}, s)) != WP_OK)
        return st;
    // layer 1
    k_grad_layer1<<<dim3(H / 64, rows_split), NTH, 0, s>>>(m->dzA, X, n, m->grad + OW1, m->grad + OB1);
    return wp_check_launch("mlp backward");
}

wp_status mlp_adam(wp_mlp *m, float lr, float b1, float b2, float eps, hipStream_t s) {
    m->step += 1;
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)m->step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)m->step));
    k_adam<<<blocks_for(NPARAM, NTH * 4), NTH, 0, s>>>(m->params, m->m1, m->m2, m->grad, NPARAM, lr, b1, b2, eps, c1,
                                                       c2);
    wp_status st = wp_check_launch("k_adam");
    return st != WP_OK ? st : refresh_bf16(m, s);
}

int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

}  // namespace

wp_status mlp_forward(wp_mlp *m, int n, const float *X, float *out, hipStream_t s) {
    if (n <= 0) return WP_OK;
    k_layer1<<<blocks_for((int64_t)n * H), NTH, 0, s>>>(X, n, m->params + OW1, m->params + OB1, m->z1, m->a1);
    wp_status st = wp_check_launch("k_layer1");
    if (st != WP_OK) return st;
    if ((st = gemm<64, 64, KC, KC>(m->a1, H, m->W2b, H, n, H, H, 1, EpiHidden{m->params + OB2, m->z2, m->a2, H}, s)) !=
        WP_OK)
        return st;
    if ((st = gemm<64, 64, KC, KC>(m->a2, H, m->W3b, H, n, H, H, 1, EpiHidden{m->params + OB3, m->z3, m->a3, H}, s)) !=
        WP_OK)
        return st;
    if (!out) return WP_OK;
    return gemm<128, 128, KC, KC>(m->a3, H, m->W4b, H, n, NOUT, H, 1, EpiOut{m->params + OB4, out, NOUT}, s);
}

// ---------------------------------------------------------------------------- C ABI

extern "C" {

int64_t wp_mlp_param_count(void) { return NPARAM; }

wp_status wp_mlp_create(wp_mlp **out, int max_batch) {
    if (!out) return wp_set_error(WP_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_batch < 64 || max_batch > (1 << 20) || max_batch % 64)
        return wp_set_error(WP_EINVAL, "max_batch = %d: need a multiple of 64 in [64, 2^20]", max_batch);
    wp_mlp *m = (wp_mlp *)calloc(1, sizeof(wp_mlp));
    if (!m) return wp_set_error(WP_ENOMEM, "mlp allocation");
    m->max_batch = max_batch;
    m->w_top = 1.0;
    m->s_out = 1.0;
    if (hipGetDevice(&m->device) != hipSuccess) {
        free(m);
        return wp_set_error(WP_EHIP, "hipGetDevice failed");
    }
    const int64_t B = max_batch;
    struct { void **p; int64_t bytes; } a[] = {
        {(void **)&m->params, NPARAM * 4}, {(void **)&m->m1, NPARAM * 4}, {(void **)&m->m2, NPARAM * 4},
        {(void **)&m->grad, NPARAM * 4},   {(void **)&m->W2b, (int64_t)H * H * 2}, {(void **)&m->W3b, (int64_t)H * H * 2},
        {(void **)&m->W4b, (int64_t)NOUT * H * 2},
        {(void **)&m->z1, B * H * 4}, {(void **)&m->z2, B * H * 4}, {(void **)&m->z3, B * H * 4},
        {(void **)&m->a1, B * H * 2}, {(void **)&m->a2, B * H * 2}, {(void **)&m->a3, B * H * 2},
        {(void **)&m->o, B * NOUT * 4}, {(void **)&m->dO, B * NOUT * 4}, {(void **)&m->dOb, B * NOUT * 2},
        {(void **)&m->dzA, B * H * 4}, {(void **)&m->dzB, B * H * 4}, {(void **)&m->dzAb, B * H * 2},
        {(void **)&m->dzBb, B * H * 2}, {(void **)&m->xb, B * 3 * 4}, {(void **)&m->tb, B * NOUT * 4},
        {(void **)&m->loss, 8},
    };
    for (auto &e : a) {
        if (hipMalloc(e.p, e.bytes) != hipSuccess) {
            wp_mlp_destroy(m);
            return wp_set_error(WP_ENOMEM, "mlp buffers (%lld bytes)", (long long)e.bytes);
        }
    }
    WP_HIP(hipMemset(m->params, 0, NPARAM * 4));
    WP_HIP(hipMemset(m->m1, 0, NPARAM * 4));
    WP_HIP(hipMemset(m->m2, 0, NPARAM * 4));
    *out = m;
    return WP_OK;
}

wp_status wp_mlp_destroy(wp_mlp *m) {
    if (!m) return WP_OK;
    void *bufs[] = {m->params, m->m1, m->m2, m->grad, m->W2b, m->W3b, m->W4b, m->z1, m->z2, m->z3, m->a1, m->a2,
                    m->a3, m->o, m->dO, m->dOb, m->dzA, m->dzB, m->dzAb, m->dzBb, m->xb, m->tb, m->loss};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    free(m);
    return WP_OK;
}

wp_status wp_mlp_set_params(wp_mlp *m, const float *params, double w_top, double s_out) {
    wp_status st = check_mlp(m);
    if (st != WP_OK) return st;
    if (!params) return wp_set_error(WP_EINVAL, "params is NULL");
    if (!(w_top > 0.0) || !std::isfinite(w_top)) return wp_set_error(WP_EINVAL, "w_top = %g: need > 0", w_top);
    if (!(s_out > 0.0) || !std::isfinite(s_out)) return wp_set_error(WP_EINVAL, "s_out = %g: need > 0", s_out);
    for (int64_t i = 0; i < NPARAM; ++i)
        if (!std::isfinite(params[i])) return wp_set_error(WP_EINVAL, "params[%lld] is not finite", (long long)i);
    WP_HIP(hipMemcpy(m->params, params, NPARAM * 4, hipMemcpyHostToDevice));
    WP_HIP(hipMemset(m->m1, 0, NPARAM * 4));
    WP_HIP(hipMemset(m->m2, 0, NPARAM * 4));
    m->step = 0;
    m->w_top = w_top;
    m->s_out = s_out;
    if ((st = refresh_bf16(m, 0)) != WP_OK) return st;
    WP_HIP(hipDeviceSynchronize());
    return WP_OK;
}

wp_status wp_mlp_get_params(const wp_mlp *m, float *params, double *w_top, double *s_out) {
    wp_status st = check_mlp(m);
    if (st != WP_OK) return st;
    if (!params) return wp_set_error(WP_EINVAL, "params is NULL");
    WP_HIP(hipDeviceSynchronize());
    WP_HIP(hipMemcpy(params, m->params, NPARAM * 4, hipMemcpyDeviceToHost));
    if (w_top) *w_top = m->w_top;
    if (s_out) *s_out = m->s_out;
    return WP_OK;
}

wp_status wp_mlp_features(const wp_plan *p, const wp_mlp *m, int64_t n, const double *u, const double *v,
                          const double *w, float *feat, int *err, void *stream) {
    if (!p) return wp_set_error(WP_EINVAL, "plan is NULL");
    wp_status st = check_mlp(m);
    if (st != WP_OK) return st;
    if (n < 0) return wp_set_error(WP_EINVAL, "n < 0");
    if (n == 0) return WP_OK;
    if (!u || !v || !w || !feat || !err) return wp_set_error(WP_EINVAL, "NULL array");
    k_features<<<blocks_for(n), NTH, 0, (hipStream_t)stream>>>(u, v, w, n, p->cell, p->Ng / 2.0, m->w_top, feat, err);
    return wp_check_launch("k_features");
}

wp_status wp_mlp_forward(wp_mlp *m, int n, const float *feat, float *out, void *stream) {
    wp_status st = check_mlp(m);
    if (st != WP_OK) return st;
    if (n < 0 || n > m->max_batch) return wp_set_error(WP_EINVAL, "n = %d: need 0 <= n <= max_batch = %d", n, m->max_batch);
    if (n > 0 && (!feat || !out)) return wp_set_error(WP_EINVAL, "NULL array");
    return mlp_forward(m, n, feat, out, (hipStream_t)stream);
}

wp_status wp_mlp_gradients(wp_mlp *m, int n, const float *feat, const float *target, float *grads, double *loss,
                           void *stream) {
    wp_status st = check_mlp(m);
    if (st != WP_OK) return st;
    if (n < 64 || n > m->max_batch || n % 64)
        return wp_set_error(WP_EINVAL, "n = %d: need a multiple of 64 in [64, max_batch = %d]", n, m->max_batch);
    if (!feat || !target) return wp_set_error(WP_EINVAL, "NULL array");
    hipStream_t s = (hipStream_t)stream;
    WP_HIP(hipMemsetAsync(m->loss, 0, 8, s));
    if ((st = mlp_backward(m, n, feat, target, s)) != WP_OK) return st;
    if (grads) WP_HIP(hipMemcpyAsync(grads, m->grad, NPARAM * 4, hipMemcpyDeviceToDevice, s));
    if (loss) {
        double acc = 0.0;
        WP_HIP(hipMemcpyAsync(&acc, m->loss, 8, hipMemcpyDeviceToHost, s));
        WP_HIP(hipStreamSynchronize(s));
        *loss = acc / ((double)n * NOUT);
    }
    return WP_OK;
}

wp_status wp_mlp_adam_step(wp_mlp *m, float lr, float beta1, float beta2, float eps, void *stream) {
    wp_status st = check_mlp(m);
    if (st != WP_OK) return st;
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f))
        return wp_set_error(WP_EINVAL, "Adam hyper-parameters out of range");
    return mlp_adam(m, lr, beta1, beta2, eps, (hipStream_t)stream);
}

wp_status wp_mlp_train(wp_mlp *m, int64_t n, const float *feat, const float *target, int batch, int epochs,
                       float lr_max, double *loss_hist, void *stream) {
    wp_status st = check_mlp(m);
    if (st != WP_OK) return st;
    if (batch < 64 || batch > m->max_batch || batch % 64)
        return wp_set_error(WP_EINVAL, "batch = %d: need a multiple of 64 in [64, max_batch = %d]", batch, m->max_batch);
    if (n < batch) return wp_set_error(WP_EINVAL, "n = %lld < batch", (long long)n);
    if (epochs < 1) return wp_set_error(WP_EINVAL, "epochs < 1");
    if (!feat || !target) return wp_set_error(WP_EINVAL, "NULL array");
    if (!(lr_max > 0.0f)) return wp_set_error(WP_EINVAL, "lr_max must be > 0");
    hipStream_t s = (hipStream_t)stream;
    const int64_t nb = n / batch;
    const int64_t T = nb * epochs, warm = std::max<int64_t>(1, T / 32);
    int64_t t = 0;
    for (int e = 0; e < epochs; ++e) {
        // per-epoch order: sample (a i + c) mod n, a coprime to n
        int64_t a = (int64_t)((0x9E3779B97F4A7C15ull * (uint64_t)(e + 1)) % (uint64_t)n) | 1;
        while (gcd64(a, n) != 1) a += 2;
        const int64_t c = (int64_t)((0xD1B54A32D192ED03ull * (uint64_t)(e + 7)) % (uint64_t)n);
        WP_HIP(hipMemsetAsync(m->loss, 0, 8, s));
        for (int64_t b = 0; b < nb; ++b, ++t) {
            k_gather_batch<<<batch, NTH, 0, s>>>(feat, target, n, a, (c + a * b * batch) % n, batch, m->xb, m->tb);
            if ((st = wp_check_launch("k_gather_batch")) != WP_OK) return st;
            if ((st = mlp_backward(m, batch, m->xb, m->tb, s)) != WP_OK) return st;
            const double ramp = std::min(1.0, (double)(t + 1) / (double)warm);
            const float lr = (float)(lr_max * ramp * 0.5 * (1.0 + std::cos(M_PI * (double)t / (double)T)));
            if ((st = mlp_adam(m, lr, 0.9f, 0.999f, 1e-8f, s)) != WP_OK) return st;
        }
        if (loss_hist) {
            double acc = 0.0;
            WP_HIP(hipMemcpyAsync(&acc, m->loss, 8, hipMemcpyDeviceToHost, s));
            WP_HIP(hipStreamSynchronize(s));
            loss_hist[e] = acc / ((double)nb * batch * NOUT);
        }
    }
    return WP_OK;
}

wp_status wp_mlp_output_scale(const wp_plan *p, double *s_out) {
    if (!p) return wp_set_error(WP_EINVAL, "plan is NULL");
    if (!s_out) return wp_set_error(WP_EINVAL, "s_out is NULL");
    // A row's energy is (sum over the u window of KB^2) (sum over the v window of KB^2): shifts of
    // the chirp spectrum are orthonormal because the chirp has unit modulus on the padded grid.
    // T0: that energy for a visibility on a cell centre; s_out = sqrt(T0 / BOX^2).
    double e = 0.0;
    const int base = -p->W / 2 + 1;
    for (int i = 0; i < p->W; ++i) {
        const double t = -(double)(base + i);
        const double r = 1.0 - (2.0 * t / p->W) * (2.0 * t / p->W);
        if (r < 0.0) continue;
        const double x = p->beta * std::sqrt(r);
        double term = 1.0, sum = 1.0;          // I0(x) = sum (x/2)^2k / (k!)^2
        for (int k = 1; k < 200 && term > 1e-17 * sum; ++k) {
            term *= (x * x / 4.0) / ((double)k * (double)k);
            sum += term;
        }
        e += sum * sum;
    }
    *s_out = std::sqrt(e * e / (double)(BOX * BOX));
    return WP_OK;
}

wp_status wp_mlp_box_targets(const wp_plan *p, const wp_G *G, const double *u, const double *v, double s_out,
                             float *target, float *lost, void *stream) {
    if (!p) return wp_set_error(WP_EINVAL, "plan is NULL");
    if (!G) return wp_set_error(WP_EINVAL, "G is NULL");
    if (G->taps != WP_TAPS_C64 || (G->nnz > 0 && (!G->col || !G->val)))
        return wp_set_error(WP_EINVAL, "box targets need stored complex64 taps");
    if (!(s_out > 0.0)) return wp_set_error(WP_EINVAL, "s_out must be > 0");
    if (p->Ng < 2 * BOX) return wp_set_error(WP_EINVAL, "Ng = %d < %d", p->Ng, 2 * BOX);
    if (G->M == 0) return WP_OK;
    if (!u || !v || !target || !lost || !G->rowptr || !G->perm) return wp_set_error(WP_EINVAL, "NULL array");
    hipStream_t s = (hipStream_t)stream;
    wp_status st = launch_fill_zero(target, G->M * NOUT, s);
    if (st != WP_OK) return st;
    k_box_targets<<<(int)((G->M + 3) / 4), NTH, 0, s>>>(G->rowptr, G->col, (const float2 *)G->val, G->perm, G->M, u, v,
                                                        p->cell, p->logNg, (float)(1.0 / s_out), target, lost);
    return wp_check_launch("k_box_targets");
}

}  // extern "C"

namespace {
wp_status row_errors(const wp_plan *p, wp_mlp *m, const wp_G *G, const double *u, const double *v, const float *feat,
                     float *eps, float *energy, void *stream) {
    if (!p) return wp_set_error(WP_EINVAL, "plan is NULL");
    wp_status st = check_mlp(m);
    if (st != WP_OK) return st;
    if (!G) return wp_set_error(WP_EINVAL, "G is NULL");
    if (G->taps != WP_TAPS_C64 || (G->nnz > 0 && (!G->col || !G->val)))
        return wp_set_error(WP_EINVAL, "the energy check needs stored complex64 taps");
    if (p->Ng < 2 * BOX) return wp_set_error(WP_EINVAL, "Ng = %d < %d", p->Ng, 2 * BOX);
    if (G->M == 0) return WP_OK;
    if (!u || !v || !feat || !eps || !G->rowptr || !G->perm) return wp_set_error(WP_EINVAL, "NULL array");
    hipStream_t s = (hipStream_t)stream;
    const int chunk = m->max_batch;
    for (int64_t r0 = 0; r0 < G->M; r0 += chunk) {
        const int nr = (int)std::min<int64_t>(chunk, G->M - r0);
        k_gather_feat<<<(3 * nr + NTH - 1) / NTH, NTH, 0, s>>>(feat, G->perm, r0, nr, m->xb);
        if ((st = wp_check_launch("k_gather_feat")) != WP_OK) return st;
        if ((st = mlp_forward(m, nr, m->xb, m->o, s)) != WP_OK) return st;
        k_row_errors<<<(nr + 3) / 4, NTH, 0, s>>>(m->o, r0, nr, G->rowptr, G->col, (const float2 *)G->val, G->perm, u,
                                                  v, p->cell, p->logNg, (float)m->s_out, eps, energy);
        if ((st = wp_check_launch("k_row_errors")) != WP_OK) return st;
    }
    return WP_OK;
}

}  // namespace

extern "C" {

wp_status wp_mlp_row_errors(const wp_plan *p, wp_mlp *m, const wp_G *G, const double *u, const double *v,
                            const float *feat, float *eps, void *stream) {
    return row_errors(p, m, G, u, v, feat, eps, nullptr, stream);
}

wp_status wp_mlp_lattice_coords(const wp_plan *p, const wp_mlp *m, int nw, int nd, double *u, double *v, double *w,
                                void *stream) {
    if (!p) return wp_set_error(WP_EINVAL, "plan is NULL");
    wp_status st = check_mlp(m);
    if (st != WP_OK) return st;
    if (nw < 2 || nd < 2 || (int64_t)nw * nd * nd > (1 << 26))
        return wp_set_error(WP_EINVAL, "lattice %d x %d x %d: need nw, nd >= 2 and at most 2^26 nodes", nw, nd, nd);
    if (!u || !v || !w) return wp_set_error(WP_EINVAL, "NULL array");
    if (!(m->w_top > 0.0)) return wp_set_error(WP_EINVAL, "the network's w_top is not set");
    const int64_t n = (int64_t)nw * nd * nd;
    k_lattice_coords<<<(int)((n + NTH - 1) / NTH), NTH, 0, (hipStream_t)stream>>>(nw, nd, m->w_top, p->cell, u, v, w);
    return wp_check_launch("k_lattice_coords");
}

wp_status wp_mlp_check_table(const wp_plan *p, wp_mlp *m, const wp_G *G, int nw, int nd, const double *u,
                             const double *v, const float *feat, float *table, void *stream) {
    if (!G) return wp_set_error(WP_EINVAL, "G is NULL");
    if (nw < 2 || nd < 2 || G->M != (int64_t)nw * nd * nd)
        return wp_set_error(WP_EINVAL, "G->M = %lld is not the lattice's %d x %d x %d nodes", (long long)G->M, nw, nd,
                            nd);
    if (!table) return wp_set_error(WP_EINVAL, "table is NULL");
    return row_errors(p, m, G, u, v, feat, table, table + G->M, stream);
}

wp_status wp_mlp_row_check(const wp_plan *p, wp_mlp *m, int nw, int nd, const float *table, int64_t n,
                           const float *feat, float *est, void *stream) {
    if (!p) return wp_set_error(WP_EINVAL, "plan is NULL");
    wp_status st = check_mlp(m);
    if (st != WP_OK) return st;
    if (nw < 2 || nd < 2 || (int64_t)nw * nd * nd > (1 << 26))
        return wp_set_error(WP_EINVAL, "lattice %d x %d x %d: need nw, nd >= 2 and at most 2^26 nodes", nw, nd, nd);
    if (n < 0) return wp_set_error(WP_EINVAL, "n = %lld", (long long)n);
    if (n == 0) return WP_OK;
    if (!table || !feat || !est) return wp_set_error(WP_EINVAL, "NULL array");
    hipStream_t s = (hipStream_t)stream;
    for (int64_t k0 = 0; k0 < n; k0 += m->max_batch) {
        const int nr = (int)std::min<int64_t>(m->max_batch, n - k0);
        if ((st = mlp_forward(m, nr, feat + 3 * k0, m->o, s)) != WP_OK) return st;
        k_row_check<<<(nr + 3) / 4, NTH, 0, s>>>(m->o, k0, nr, feat, table, nw, nd, (float)m->s_out, est);
        if ((st = wp_check_launch("k_row_check")) != WP_OK) return st;
    }
    return WP_OK;
}

}  // extern "C"
