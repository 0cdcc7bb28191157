// Internal: sizes of the surrogate network and the bfloat16 MFMA tile machinery
// shared by its training kernels (mlp.hip) and the surrogate operator (surrogate.hip).
//
// Network: 3 -> H -> H -> H -> NOUT with GELU after the hidden layers; NOUT =
// 2 BOX^2 outputs are the real and imaginary parts of the taps of a BOX x BOX
// box of grid cells.  Parameters are packed in FP32 in the order
// W1 [H,3], b1 [H], W2 [H,H], b2, W3 [H,H], b3, W4 [NOUT,H], b4 [NOUT]
// (row-major, W_l maps layer l-1 to layer l).
//
// Matrix products: C[M,N] = A[M,K] B[N,K]^T with bfloat16 operands and FP32
// accumulation on v_mfma_f32_32x32x16_bf16.  An operand is either
// K-contiguous (KC: element (r, k) at p[r ld + k]) or row-contiguous
// (RC: element (r, k) at p[k ld + r]); both are staged in LDS K-contiguous,
// BK = 32 deep, rows padded to LDK elements.
#pragma once

#include "common.h"

namespace mlpc {

constexpr int H = 256;
constexpr int BOX = 32;
constexpr int NOUT = 2 * BOX * BOX;
constexpr int64_t OW1 = 0;
constexpr int64_t OB1 = OW1 + (int64_t)H * 3;
constexpr int64_t OW2 = OB1 + H;
constexpr int64_t OB2 = OW2 + (int64_t)H * H;
constexpr int64_t OW3 = OB2 + H;
constexpr int64_t OB3 = OW3 + (int64_t)H * H;
constexpr int64_t OW4 = OB3 + H;
constexpr int64_t OB4 = OW4 + (int64_t)NOUT * H;
constexpr int64_t NPARAM = OB4 + NOUT;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int BK = 32;
constexpr int LDK = BK + 8;   // 80-byte LDS rows: consecutive rows start 20 banks apart
enum { KC = 0, RC = 1 };

__device__ inline uint16_t to_bf16(float f) { return (uint16_t)bf16_bits_rne(f); }
__device__ inline float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// gelu(x) = x Phi(x) (error-function form) and its derivative Phi(x) + x phi(x)
__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// Stage the ROWS x BK tile (rows r0.., depth k0..) of an operand into LDS s[ROWS][LDK];
// rows at or beyond nrows read as zero.  KC needs ld % 8 == 0; RC needs ld % 8 == 0 and
// nrows % 8 == 0.  Both need a 16-byte aligned base.
template <int ROWS, int LAYOUT, int NTH>
__device__ __forceinline__ void stage_tile(uint16_t *s, const uint16_t *__restrict__ p, int64_t ld, int nrows,
                                           int r0, int64_t k0, int tid) {
    constexpr int CH = ROWS * BK / 8;
    if constexpr (LAYOUT == KC) {
#pragma unroll
        for (int c = tid; c < CH; c += NTH) {
            const int r = c / (BK / 8), kc = (c % (BK / 8)) * 8;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (r0 + r < nrows) v = *(const u32x4 *)(p + (int64_t)(r0 + r) * ld + k0 + kc);
            *(u32x4 *)(s + r * LDK + kc) = v;
        }
    } else {
#pragma unroll
        for (int c = tid; c < CH; c += NTH) {
            const int k = c / (ROWS / 8), rc = (c % (ROWS / 8)) * 8;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (r0 + rc < nrows) v = *(const u32x4 *)(p + (k0 + k) * ld + r0 + rc);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                s[(rc + 2 * e) * LDK + k] = (uint16_t)(v[e] & 0xffffu);
                s[(rc + 2 * e + 1) * LDK + k] = (uint16_t)(v[e] >> 16);
            }
        }
    }
}

// acc[fm][fn] += A rows [arow0 + 32 fm, +32) times B rows [brow0 + 32 fn, +32), one BK-deep step;
// LDS row strides SA and SB (elements).  Lane l feeds A[row l % 32][k 8 (l / 32) .. +7] and
// B[row l % 32][same k].
template <int FM, int FN, int SA = LDK, int SB = LDK>
__device__ __forceinline__ void mma_bk(f32x16 (&acc)[FM][FN], const uint16_t *As, const uint16_t *Bs, int arow0,
                                       int brow0, int lane) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
        bf16x8 a[FM], b[FN];
        const int ko = kk + 8 * (lane >> 5), ro = lane & 31;
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
            a[fm] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(As + (arow0 + 32 * fm + ro) * SA + ko));
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
            b[fn] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(Bs + (brow0 + 32 * fn + ro) * SB + ko));
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn)
                acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[fm], b[fn], acc[fm][fn], 0, 0, 0);
    }
}

// position of accumulator register r of lane l inside its 32 x 32 block
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
__device__ __forceinline__ int acc_col(int lane) { return lane & 31; }

}  // namespace mlpc

// surrogate network object (mlp.hip)
struct wp_mlp {
    int device;
    int max_batch;
    double w_top, s_out;
    int64_t step;                          // Adam steps taken
    float *params, *m1, *m2, *grad;        // [NPARAM] FP32: parameters, Adam moments, gradients
    uint16_t *W2b, *W3b, *W4b;             // bfloat16 copies of W2, W3, W4
    float *z1, *z2, *z3;                   // [max_batch H] pre-activations
    uint16_t *a1, *a2, *a3;                // [max_batch H] activations (bfloat16)
    float *o;                              // [max_batch NOUT] outputs
    float *dO;                             // [max_batch NOUT] dL/do
    uint16_t *dOb;
    float *dzA, *dzB;                      // [max_batch H]
    uint16_t *dzAb, *dzBb;
    float *xb, *tb;                        // [max_batch 3], [max_batch NOUT] minibatch copies
    double *loss;                          // [1] running sum of squared errors
};

// forward pass of n <= max_batch feature rows: hidden layers into m->a3 (and z1..z3);
// with `out`, the outputs too
wp_status mlp_forward(wp_mlp *m, int n, const float *feat, float *out, hipStream_t s);
