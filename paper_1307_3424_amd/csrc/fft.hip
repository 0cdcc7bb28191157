// A, Z, F and their adjoint: apodise + zero-pad + centred 2-D FFT of the image,
// and the unnormalised inverse + crop + apodise back (Sections 2.2 and 3.1; the
// upsampling U of Eq. 6 is done here in the image domain as zero-padding).
//
// Centring.  With c = Ng/2, the centred DFT
//     X[q] = sum_j z_j exp(-2 pi i (j - c).(q - c) / Ng)
// equals (-1)^(q_u+q_v) FFT((-1)^(j_u+j_v) z)[q] (Ng even), so the signs are
// folded into the first and last pass.  Pruning: the padded image is non-zero
// only in its central N rows and columns, so the forward row pass runs on N
// rows only and the column pass reads N rows; the adjoint column pass writes
// only those N rows and the row pass keeps the central N outputs.
#include "fft_lds.h"

namespace {

// Launch shape per grid size: rows per block / threads of the row passes, columns per
// block / threads of the column passes.  Small grids favour many small blocks (the
// transform is latency-bound there); large ones favour wider column strips (coalescing).
// At Ng = 512, timed inside Phi + Phi^H: these shapes beat rows of (2, 128), (1, 128), (2, 64) and
// columns of (1, 64), (4, 256) by 0.5-2 us per step.
template <int LOGNG> struct Shape;
template <> struct Shape<6> { static constexpr int CR = 4, TR = 64, CC = 4, TC = 64; };
template <> struct Shape<7> { static constexpr int CR = 2, TR = 64, CC = 4, TC = 64; };
template <> struct Shape<8> { static constexpr int CR = 1, TR = 64, CC = 2, TC = 64; };
template <> struct Shape<9> { static constexpr int CR = 1, TR = 64, CC = 2, TC = 128; };
template <> struct Shape<10> { static constexpr int CR = 1, TR = 128, CC = 4, TC = 256; };
template <> struct Shape<11> { static constexpr int CR = 1, TR = 256, CC = 4, TC = 512; };
template <> struct Shape<12> { static constexpr int CR = 1, TR = 512, CC = 2, TC = 512; };

// INVN: the physical apodisation carries the 1/n(l, m) factor.  A template parameter rather than
// a runtime test, so that a kernel's loads are not split by a branch.
template <bool INVN>
__device__ inline float apod_at(const float *__restrict__ apod, int N, float delta, int im, int iu) {
    float a = apod[im] * apod[iu];
    if constexpr (INVN) {
        const float l = (iu - N / 2) * delta, m = (im - N / 2) * delta;
        a *= rsqrtf(1.0f - l * l - m * m);
    }
    return a;
}

__device__ inline float sgn(int k) { return (k & 1) ? -1.0f : 1.0f; }

// Every kernel loads all of a thread's elements (and the apodisation factors) into registers
// before it writes any of them to LDS, so the loads are in flight together instead of one
// round trip per element.

// Forward, pass 1: rows.  Block handles C image rows (padded rows jv = im + N/2).
template <int LOGNG, int C, int NTH, bool INVN>
__global__ __launch_bounds__(NTH) void k_fwd_rows(const float2 *__restrict__ x, float2 *__restrict__ grid,
                                                      const float *__restrict__ apod, const float2 *__restrict__ tw,
                                                      float delta) {
    constexpr int Ng = 1 << LOGNG, N = Ng / 2, PE = C * Ng / NTH, PZ = C * N / NTH;
    static_assert(C * N % NTH == 0, "shape");
    __shared__ float2 buf[C * Ng];
    const int tid = threadIdx.x;
    const int im0 = blockIdx.x * C;
    x += (int64_t)blockIdx.y * N * N;
    grid += (int64_t)blockIdx.y * Ng * Ng;
    FftTwiddles<float2, LOGNG, C, NTH, true> twp;
    twp.load(tw, false, tid);
    // the padded row is non-zero only at j in [N/2, 3N/2): load those, write zeros elsewhere
    float2 v[PZ];
    float a[PZ];
#pragma unroll
    for (int i = 0; i < PZ; ++i) {
        const int e = tid + i * NTH, c = e / N, iu = e % N, im = im0 + c;
        v[i] = x[(int64_t)im * N + iu];
        a[i] = apod_at<INVN>(apod, N, delta, im, iu) * sgn(iu + N / 2 + im + N / 2);
    }
#pragma unroll
    for (int i = 0; i < PZ; ++i) {
        const int e = tid + i * NTH, c = e / N, iu = e % N;
        buf[c * Ng + iu + N / 2] = make_float2(v[i].x * a[i], v[i].y * a[i]);
        buf[c * Ng + (iu < N / 2 ? iu : iu + N)] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    lds_fft<float2, LOGNG, C, NTH, true, Ng>(buf, tw, &twp, false, tid);
#pragma unroll
    for (int i = 0; i < PE; ++i) {
        const int e = tid + i * NTH, c = e / Ng, q = e % Ng, jv = im0 + c + N / 2;
        grid[(int64_t)jv * Ng + q] = buf[e];
    }
}

// Forward, pass 2: columns (block handles C adjacent columns), in place.
template <int LOGNG, int C, int NTH>
__global__ __launch_bounds__(NTH) void k_fwd_cols(float2 *__restrict__ grid, const float2 *__restrict__ tw) {
    constexpr int Ng = 1 << LOGNG, N = Ng / 2, PE = Ng * C / NTH, PZ = N * C / NTH;
    static_assert(N * C % NTH == 0, "shape");
    __shared__ float2 buf[Ng * C];
    const int tid = threadIdx.x;
    const int qu0 = xcd_block(blockIdx.x, gridDim.x) * C;
    grid += (int64_t)blockIdx.y * Ng * Ng;
    FftTwiddles<float2, LOGNG, C, NTH, false> twp;
    twp.load(tw, false, tid);
    // only rows jv in [N/2, 3N/2) are non-zero: load those, write zeros elsewhere
    float2 v[PZ];
#pragma unroll
    for (int i = 0; i < PZ; ++i) {
        const int e = tid + i * NTH, jv = N / 2 + e / C, c = e % C;
        v[i] = grid[(int64_t)jv * Ng + qu0 + c];
    }
#pragma unroll
    for (int i = 0; i < PZ; ++i) {
        const int e = tid + i * NTH, r = e / C, c = e % C;
        buf[(N / 2 + r) * C + c] = v[i];
        buf[(r < N / 2 ? r : r + N) * C + c] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    lds_fft<float2, LOGNG, C, NTH, false, C>(buf, tw, &twp, false, tid);
#pragma unroll
    for (int i = 0; i < PE; ++i) {
        const int e = tid + i * NTH, qv = e / C, c = e % C;
        const float2 w = buf[e];
        const float s = sgn(qv + qu0 + c);
        grid[(int64_t)qv * Ng + qu0 + c] = make_float2(w.x * s, w.y * s);
    }
}

// Adjoint, pass 1: columns, inverse, keep the central N rows, in place.
template <int LOGNG, int C, int NTH>
__global__ __launch_bounds__(NTH) void k_adj_cols(float2 *__restrict__ grid, const float2 *__restrict__ tw) {
    constexpr int Ng = 1 << LOGNG, N = Ng / 2, PE = Ng * C / NTH, PO = N * C / NTH;
    static_assert(Ng * C % NTH == 0 && N * C % NTH == 0, "shape");
    __shared__ float2 buf[Ng * C];
    const int tid = threadIdx.x;
    const int qu0 = xcd_block(blockIdx.x, gridDim.x) * C;
    grid += (int64_t)blockIdx.y * Ng * Ng;
    FftTwiddles<float2, LOGNG, C, NTH, false> twp;
    twp.load(tw, true, tid);
    float2 v[PE];
#pragma unroll
    for (int i = 0; i < PE; ++i) {
        const int e = tid + i * NTH, qv = e / C, c = e % C;
        v[i] = grid[(int64_t)qv * Ng + qu0 + c];
    }
#pragma unroll
    for (int i = 0; i < PE; ++i) {
        const int e = tid + i * NTH, qv = e / C, c = e % C;
        const float s = sgn(qv + qu0 + c);
        buf[e] = make_float2(v[i].x * s, v[i].y * s);          // e = qv C + c
    }
    __syncthreads();
    lds_fft<float2, LOGNG, C, NTH, false, C>(buf, tw, &twp, true, tid);
#pragma unroll
    for (int i = 0; i < PO; ++i) {
        const int e = tid + i * NTH, jv = N / 2 + e / C, c = e % C;
        grid[(int64_t)jv * Ng + qu0 + c] = buf[jv * C + c];
    }
}

// Adjoint, pass 2: rows, inverse, crop the central N, apodise, write the image.
template <int LOGNG, int C, int NTH, bool INVN>
__global__ __launch_bounds__(NTH) void k_adj_rows(const float2 *__restrict__ grid, float2 *__restrict__ x,
                                                      const float *__restrict__ apod, const float2 *__restrict__ tw,
                                                      float delta) {
    constexpr int Ng = 1 << LOGNG, N = Ng / 2, PE = C * Ng / NTH, PO = C * N / NTH;
    static_assert(C * Ng % NTH == 0 && C * N % NTH == 0, "shape");
    __shared__ float2 buf[C * Ng];
    const int tid = threadIdx.x;
    const int im0 = blockIdx.x * C;
    grid += (int64_t)blockIdx.y * Ng * Ng;
    x += (int64_t)blockIdx.y * N * N;
    FftTwiddles<float2, LOGNG, C, NTH, true> twp;
    twp.load(tw, true, tid);
    float a[PO];                                                // output factors, needed after the transform
#pragma unroll
    for (int i = 0; i < PO; ++i) {
        const int e = tid + i * NTH, c = e / N, iu = e % N, im = im0 + c;
        a[i] = apod_at<INVN>(apod, N, delta, im, iu) * sgn(iu + N / 2 + im + N / 2);
    }
    float2 v[PE];
#pragma unroll
    for (int i = 0; i < PE; ++i) {
        const int e = tid + i * NTH, c = e / Ng, q = e % Ng, jv = im0 + c + N / 2;
        v[i] = grid[(int64_t)jv * Ng + q];
    }
#pragma unroll
    for (int i = 0; i < PE; ++i) buf[tid + i * NTH] = v[i];   // e = c Ng + q
    __syncthreads();
    lds_fft<float2, LOGNG, C, NTH, true, Ng>(buf, tw, &twp, true, tid);
#pragma unroll
    for (int i = 0; i < PO; ++i) {
        const int e = tid + i * NTH, c = e / N, iu = e % N, im = im0 + c;
        const float2 w = buf[c * Ng + iu + N / 2];
        x[(int64_t)im * N + iu] = make_float2(w.x * a[i], w.y * a[i]);
    }
}

template <int LOGNG>
wp_status fwd(const wp_plan *p, const float2 *x, float2 *grid, int batch, hipStream_t s) {
    constexpr int Ng = 1 << LOGNG, N = Ng / 2;
    using S = Shape<LOGNG>;
    static_assert(N % S::CR == 0 && Ng % S::CC == 0, "shape");
    if (p->aphys == WP_APHYS_INV_N)
        hipLaunchKernelGGL((k_fwd_rows<LOGNG, S::CR, S::TR, true>), dim3(N / S::CR, batch), dim3(S::TR), 0, s, x,
                           grid, p->apod, p->tw32, (float)p->delta);
    else
        hipLaunchKernelGGL((k_fwd_rows<LOGNG, S::CR, S::TR, false>), dim3(N / S::CR, batch), dim3(S::TR), 0, s, x,
                           grid, p->apod, p->tw32, (float)p->delta);
    hipLaunchKernelGGL((k_fwd_cols<LOGNG, S::CC, S::TC>), dim3(Ng / S::CC, batch), dim3(S::TC), 0, s, grid, p->tw32);
    return wp_check_launch("grid_forward");
}

template <int LOGNG>
wp_status adj(const wp_plan *p, float2 *grid, float2 *x, int batch, hipStream_t s) {
    constexpr int Ng = 1 << LOGNG, N = Ng / 2;
    using S = Shape<LOGNG>;
    hipLaunchKernelGGL((k_adj_cols<LOGNG, S::CC, S::TC>), dim3(Ng / S::CC, batch), dim3(S::TC), 0, s, grid, p->tw32);
    if (p->aphys == WP_APHYS_INV_N)
        hipLaunchKernelGGL((k_adj_rows<LOGNG, S::CR, S::TR, true>), dim3(N / S::CR, batch), dim3(S::TR), 0, s, grid,
                           x, p->apod, p->tw32, (float)p->delta);
    else
        hipLaunchKernelGGL((k_adj_rows<LOGNG, S::CR, S::TR, false>), dim3(N / S::CR, batch), dim3(S::TR), 0, s, grid,
                           x, p->apod, p->tw32, (float)p->delta);
    return wp_check_launch("grid_adjoint");
}

}  // namespace

wp_status launch_grid_forward(const wp_plan *p, const float2 *x, float2 *grid, hipStream_t s, int batch) {
    switch (p->logNg) {
        case 6: return fwd<6>(p, x, grid, batch, s);
        case 7: return fwd<7>(p, x, grid, batch, s);
        case 8: return fwd<8>(p, x, grid, batch, s);
        case 9: return fwd<9>(p, x, grid, batch, s);
        case 10: return fwd<10>(p, x, grid, batch, s);
        case 11: return fwd<11>(p, x, grid, batch, s);
        case 12: return fwd<12>(p, x, grid, batch, s);
    }
    return wp_set_error(WP_EUNSUPPORTED, "grid_forward: Ng = %d", p->Ng);
}

wp_status launch_grid_adjoint(const wp_plan *p, float2 *grid, float2 *x, hipStream_t s, int batch) {
    switch (p->logNg) {
        case 6: return adj<6>(p, grid, x, batch, s);
        case 7: return adj<7>(p, grid, x, batch, s);
        case 8: return adj<8>(p, grid, x, batch, s);
        case 9: return adj<9>(p, grid, x, batch, s);
        case 10: return adj<10>(p, grid, x, batch, s);
        case 11: return adj<11>(p, grid, x, batch, s);
        case 12: return adj<12>(p, grid, x, batch, s);
    }
    return wp_set_error(WP_EUNSUPPORTED, "grid_adjoint: Ng = %d", p->Ng);
}
