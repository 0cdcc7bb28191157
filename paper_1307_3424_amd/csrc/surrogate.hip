// Surrogate measurement operator: Phi and Phi^H where the rows of the visibilities
// that pass the per-row energy check come from the surrogate network, and the other
// rows from an exact G built for them (the fallback).
//
// The network's taps are linear in its last hidden layer h_k (256 values per
// visibility) -- t_k(p) = s_out (sum_j (W4[2p][j] + i W4[2p+1][j]) h_kj + b4[2p] + i b4[2p+1])
// for box cell p -- so the output layer (4/5 of the network's arithmetic) can be moved
// from the visibilities to the occupied grid cells.  For the visibilities in nearest
// cell c:
//   degrid  y_k = s_out (sum_j h_kj r_c[j] + beta_c),
//           r_c[j] = sum_p (W4[2p][j] + i W4[2p+1][j]) X(c + p),  beta_c = sum_p b4_p X(c + p);
//   grid    sum_{k in c} conj(t_k(p)) y_k = s_out (sum_j (W4[2p][j] - i W4[2p+1][j]) s_c[j] + conj(b4_p) Y_c),
//           s_c[j] = sum_{k in c} h_kj y_k,  Y_c = sum_{k in c} y_k.
// r is one dense product per group of up to 128 cells, [cells x 2048 box values] x [2048 x 512]
// (as two workgroups of 256 outputs), and the box contributions one per group and slice of 256
// outputs, [cells x 512] x [512 x 256] (the default forms; the register-staged gridding takes groups
// of up to 32 cells and all 2048 outputs), both on bfloat16 MFMA with FP32 accumulation.  The
// hidden layers run once, at set-up.  The taps are never stored.
//
// Visibility order ("slots"): slots [0, Ms) hold the surrogate rows sorted by the Z-order
// code of their nearest cell; slots [Ms, M) the fallback rows in the caller's order, which
// is the order of the coordinates wp_surrogate_fallback_coords returns (build the fallback
// G from those, in caller order, or keep its sorted order consistently).
#include <climits>
#include <cmath>
#include <type_traits>
#include <vector>

#include "mlp_core.h"

using namespace mlpc;

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// loads of data read once per product (hidden layers, visibilities): non-temporal, so that they do
// not evict the output-layer weights that every workgroup reads
__device__ __forceinline__ uint2 nt_load_u2(const uint16_t *p) {
    const u32x2 v = __builtin_nontemporal_load((const u32x2 *)p);
    return make_uint2(v.x, v.y);
}
__device__ __forceinline__ u32x4 nt_load_u4(const uint16_t *p) {
    return __builtin_nontemporal_load((const u32x4 *)p);
}
// sum over each row of 16 lanes, left in every lane of the row (quad swaps, then half-row and row mirrors)
__device__ __forceinline__ float dpp_sum16(float x) {
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));   // quad [1,0,3,2]
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));   // quad [2,3,0,1]
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xF, 0xF, false));  // half-row mirror
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xF, 0xF, false));  // row mirror
    return x;
}
__device__ __forceinline__ float2 nt_load_f2(const float2 *p) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const f32x2 v = __builtin_nontemporal_load((const f32x2 *)p);
    return make_float2(v.x, v.y);
}

struct wp_surrogate {
    int device;
    int logNg;
    int64_t M, Ms, Mf, ncell;
    int ngrp_d, ngrp_a;
    float s_out;
    int *slot_vis;      // [M] caller index of each slot
    int *cell_key;      // [ncell] Z-order code of each occupied cell (v, u grid indices)
    int *cell_start;    // [ncell + 1] first slot of each cell
    int *grp_d;         // [ngrp_d + 1] first cell of each degridding group
    int *grp_a;         // [ngrp_a + 1] first cell of each gridding group
    int2 *grp_org;      // [ngrp_a] grid (v, u) of each gridding group's LDS window origin
    uint16_t *h3;       // [Ms H] last hidden layer, bfloat16, slot order
    uint16_t *Bdeg;     // [2H][NOUT] bfloat16: r = Bdeg x box
    uint16_t *Bgrd;     // [NOUT][2H] bfloat16: box contributions = Bgrd x s
    float *b4;          // [NOUT] output bias
    float *wmax;        // [2] largest output weight norm and |b4| (bounds of the gridding's fixed-point window)
    double *fb;         // [3 Mf] fallback u, v, w (slot order)
    uint32_t *gbf;      // [Ng][Ng + 2 PADC] the degridding's grid in bfloat16 pairs, columns wrapped by PADC
    // the gridding through the LDS ring
    uint16_t *Bgrd2;    // [NSL][ND / 32][256][32] weights of each slice of 256 outputs, step-major
    uint16_t *Sg;       // [ncell + 1][ND] s of each cell in bfloat16, rewritten by every gridding; the last row
                        // stays zero (the A rows past a group of the ring gridding)
    float4 *cY;         // [ncell] (sum of y re, sum of y im, bound on the cell's outputs / s_out, 0)
    int *grp_g;         // [ngrp_g + 1] first cell of each ring-gridding group
    int4 *grp_gorg;     // [ngrp_g] smallest (v, u) of each ring-gridding group's cells, and its (v, u) spans
    int ngrp_g;
};

namespace {

constexpr int DG = 128;             // cells per degridding group
constexpr int DNT = 512;            // threads of a degridding workgroup (8 waves)
constexpr int ND = 2 * H;           // 512 outputs per cell (r re, r im) / depth of the gridding product
constexpr int DBN = H;              // outputs per degridding workgroup: r re (part 0) or r im (part 1)
constexpr int KDEP = NOUT;          // degridding depth: 1024 box cells x (re, im)
constexpr size_t DEG_LDS = (size_t)(2 * DG + 2 * DBN) * LDK * 2;
constexpr int RPASS = 32;           // cells per epilogue pass of the degridding
constexpr int RLD = DBN + 4;        // FP32 row stride of r in LDS
static_assert((size_t)RPASS * RLD * 4 <= DEG_LDS, "epilogue rows must fit the staging buffers");

constexpr int AG = 32;              // cells per gridding group
constexpr int ANT = 256;            // threads of a gridding workgroup (4 waves)
constexpr int WV = 64, WU = 64;     // LDS window (cells); a group's cells span at most WV - BOX + 1 rows
constexpr int SLD = ND + 8;         // row stride of the staged A operand (s, 512 values)
constexpr size_t GRD_LDS = (size_t)AG * SLD * 2 + (size_t)WV * WU * 8;
constexpr int NSL = NOUT / 256;      // slices of 256 outputs (4 box rows) of the ring gridding
constexpr int GSPAN = 64;            // a ring-gridding group's cells span at most GSPAN rows and GSPAN columns
constexpr int GWR = GSPAN + 4, GWC = GSPAN + BOX;   // its LDS window per slice (cells)

__device__ inline int cell_index(double gt, int Ng) {
    const long long c = (long long)floor(gt + 0.5) + Ng / 2;
    return (int)(((c % Ng) + Ng) % Ng);
}

// key: Z-order code of the nearest cell, or `fallback_key` (larger than every code) for a
// row whose energy error exceeds tol (or is not a number)
__global__ void k_slot_keys(const double *__restrict__ u, const double *__restrict__ v, int64_t M, double cell,
                            int logNg, const float *__restrict__ eps, float tol, int fallback_key,
                            int *__restrict__ key, int *__restrict__ isfb) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= M) return;
    const int Ng = 1 << logNg;
    const bool fb = eps && !(eps[k] <= tol);
    key[k] = fb ? fallback_key : morton2(cell_index(v[k] / cell, Ng), cell_index(u[k] / cell, Ng));
    isfb[k] = fb ? 1 : 0;
}

// new-cell flags over the sorted surrogate slots
__global__ void k_cell_flags(const int *__restrict__ skey, int64_t Ms, int *__restrict__ flag) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < Ms) flag[j] = (j == 0 || skey[j] != skey[j - 1]) ? 1 : 0;
}

__global__ void k_cell_table(const int *__restrict__ skey, const int *__restrict__ flag, const int *__restrict__ cid,
                             int64_t Ms, int *__restrict__ cell_key, int *__restrict__ cell_start) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= Ms) return;
    if (flag[j]) {
        cell_key[cid[j]] = skey[j];
        cell_start[cid[j]] = (int)j;
    }
    if (j == Ms - 1) cell_start[cid[Ms]] = (int)Ms;
}

__global__ void k_feat_slots(const float *__restrict__ feat, const int *__restrict__ slot_vis, int64_t j0, int n,
                             float *__restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < 3 * n) out[i] = feat[3 * (int64_t)slot_vis[j0 + i / 3] + i % 3];
}

__global__ void k_fallback_coords(const double *__restrict__ u, const double *__restrict__ v,
                                  const double *__restrict__ w, const int *__restrict__ slot_vis, int64_t Ms,
                                  int64_t Mf, double *__restrict__ fb) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= Mf) return;
    const int k = slot_vis[Ms + i];
    fb[i] = u[k];
    fb[Mf + i] = v[k];
    fb[2 * Mf + i] = w[k];
}

// The two output-layer matrices, rounded to bfloat16, stored in the order the products read them:
//   Bdeg[n][kk] (n < 256: r re of hidden n, n >= 256: r im of hidden n - 256; kk = 2p + c) as
//     [part = n / 256][step t = kk / 32][n % 256][kk % 32]: one degridding stage is contiguous;
//   Bgrd[o][k] (o = 2p + c; k < 256: s re, k >= 256: s im) as
//     [block o / 32][step k / 16][lane = o % 32 + 32 ((k % 16) / 8)][k % 8]: one MFMA fragment of
//     a wave is 1 KB contiguous.
__device__ inline int64_t deg_index(int n, int kk) {
    return ((int64_t)((n / H) * (KDEP / 32) + kk / 32) * H + (n % H)) * 32 + (kk % 32);
}
__device__ inline int64_t grd_index(int o, int k) {
    return ((int64_t)((o / 32) * (ND / 16) + k / 16) * 64 + (o % 32) + 32 * ((k % 16) / 8)) * 8 + (k % 8);
}
//   Bgrd2[o][k], the same weights for the ring gridding: [slice o / 256][step k / 32][o % 256][k % 32]
__device__ inline int64_t grd2_index(int o, int k) {
    return ((int64_t)((o / 256) * (ND / 32) + k / 32) * 256 + (o % 256)) * 32 + (k % 32);
}

// largest Euclidean norm of an output's bfloat16 weights in the gridding product (over its 512
// inputs) and largest |b4| (non-negative floats order like their bit patterns, so an integer
// maximum serves); one thread per output
__global__ void k_weight_max(const uint16_t *__restrict__ Bgrd, const float *__restrict__ b4, float *__restrict__ wmax) {
    const int o = blockIdx.x * 256 + threadIdx.x;
    if (o >= NOUT) return;
    float ss = 0.f;
    for (int k = 0; k < ND; ++k) {
        const float b = from_bf16(Bgrd[grd_index(o, k)]);
        ss = fmaf(b, b, ss);
    }
    atomicMax((int *)&wmax[0], __float_as_int(sqrtf(ss) * 1.0001f));
    atomicMax((int *)&wmax[1], __float_as_int(fabsf(b4[o])));
}

__global__ void k_make_B(const float *__restrict__ W4, uint16_t *__restrict__ Bdeg, uint16_t *__restrict__ Bgrd,
                         uint16_t *__restrict__ Bgrd2) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)NOUT * H) return;
    const int p = (int)(e / H), j = (int)(e % H);      // box cell p, hidden j
    if (p >= BOX * BOX) return;
    const float wr = W4[(int64_t)(2 * p) * H + j], wi = W4[(int64_t)(2 * p + 1) * H + j];
    const uint16_t br = to_bf16(wr), bi = to_bf16(wi), nbi = to_bf16(-wi);
    Bdeg[deg_index(j, 2 * p)] = br;
    Bdeg[deg_index(j, 2 * p + 1)] = nbi;
    Bdeg[deg_index(H + j, 2 * p)] = bi;
    Bdeg[deg_index(H + j, 2 * p + 1)] = br;
    Bgrd[grd_index(2 * p, j)] = br;
    Bgrd[grd_index(2 * p, H + j)] = bi;
    Bgrd[grd_index(2 * p + 1, j)] = nbi;
    Bgrd[grd_index(2 * p + 1, H + j)] = br;
    Bgrd2[grd2_index(2 * p, j)] = br;
    Bgrd2[grd2_index(2 * p, H + j)] = bi;
    Bgrd2[grd2_index(2 * p + 1, j)] = nbi;
    Bgrd2[grd2_index(2 * p + 1, H + j)] = br;
}

// ---------------------------------------------------------------------------- degridding

// Two workgroups per group of <= DG occupied cells (consecutive in Z-order): part 0 forms
// r re = A Bdeg[0:256]^T and writes Re y, part 1 forms r im and writes Im y, A[i][2p + c] = the box
// of cell i in bfloat16.  Waves: 2 along cells (64 each) x 4 along outputs (64 each);
// double-buffered LDS stages with the next stage's loads in flight during the MFMAs.  Epilogue:
// 32 cells of r at a time in LDS (FP32), then one visibility per wave: a coalesced load of its
// hidden layer, a dot product and a wave reduction.
__global__ __launch_bounds__(DNT, 4) void k_sur_degrid(const float2 *__restrict__ grid, int logNg,
                                                       const int *__restrict__ grp, int ngrp,
                                                       const int *__restrict__ cell_key,
                                                       const int *__restrict__ cell_start,
                                                       const uint16_t *__restrict__ h3,
                                                       const uint16_t *__restrict__ Bdeg,
                                                       const float *__restrict__ b4, float s_out,
                                                       float2 *__restrict__ y) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *As = (uint16_t *)smem;                 // [2][DG][LDK]
    uint16_t *Bs = As + 2 * DG * LDK;                // [2][DBN][LDK]
    float *Rl = (float *)smem;                       // after the product: [RPASS][RLD]
    __shared__ int s_cv[DG], s_cu[DG], s_cs[DG + 1];
    __shared__ float s_beta[DG];
    __shared__ float2 s_b4[BOX * BOX];               // output bias (no global loads inside the loop)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 2, wn = wave & 3;
    const int part = blockIdx.y;
    for (int i = tid; i < BOX * BOX; i += DNT) s_b4[i] = ((const float2 *)b4)[i];
    const int g = (int)xcd_block(blockIdx.x, ngrp);
    const int c0 = grp[g], nc = grp[g + 1] - c0;
    const int Ng = 1 << logNg;
    for (int i = tid; i < DG; i += DNT) {
        int cv = 0, cu = 0;
        if (i < nc) demorton2(cell_key[c0 + i], cv, cu);
        s_cv[i] = cv;
        s_cu[i] = cu;
    }
    for (int i = tid; i <= nc; i += DNT) s_cs[i] = cell_start[c0 + i];
    __syncthreads();

    // staging of A: thread -> cell si, 4 consecutive box cells of the step's 16
    const int si = tid >> 2, sq = tid & 3;
    const bool slive = si < nc;
    const int scv = s_cv[si], scu = s_cu[si];
    const uint16_t *Bpart = Bdeg + (int64_t)part * DBN * KDEP;   // [step][256][32]
    float2 areg[4];
    u32x4 breg[2];
    float bacc = 0.0f;
    auto load = [&](int t) {
        const int oy = t >> 1, ox0 = 16 * (t & 1) + 4 * sq;
        const int64_t row = (int64_t)((scv + oy - BOX / 2) & (Ng - 1)) * Ng;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int gx = (scu + ox0 + e - BOX / 2) & (Ng - 1);
            areg[e] = slive ? grid[row + gx] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + DNT * q, n = c >> 2, kc = (c & 3) * 8;
            breg[q] = *(const u32x4 *)(Bpart + ((int64_t)t * DBN + n) * 32 + kc);
        }
    };
    auto store = [&](int t, int buf) {
        const int oy = t >> 1, ox0 = 16 * (t & 1) + 4 * sq;
        u32x4 a;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            a[e] = (uint32_t)to_bf16(areg[e].x) | ((uint32_t)to_bf16(areg[e].y) << 16);
            const float2 bb = s_b4[oy * BOX + ox0 + e];
            bacc += part == 0 ? bb.x * areg[e].x - bb.y * areg[e].y : bb.x * areg[e].y + bb.y * areg[e].x;
        }
        *(u32x4 *)(As + buf * DG * LDK + si * LDK + 8 * sq) = a;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + DNT * q, n = c >> 2, kc = (c & 3) * 8;
            *(u32x4 *)(Bs + buf * DBN * LDK + n * LDK + kc) = breg[q];
        }
    };

    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    constexpr int NSTEP = KDEP / BK;
    load(0);
    store(0, 0);
    __syncthreads();
    for (int t = 0; t < NSTEP; ++t) {
        const int cur = t & 1;
        if (t + 1 < NSTEP) load(t + 1);
        mma_bk<2, 2>(acc, As + cur * DG * LDK, Bs + cur * DBN * LDK, 64 * wm, 64 * wn, lane);
        if (t + 1 < NSTEP) store(t + 1, cur ^ 1);
        __syncthreads();
    }
    // bias term of each cell: the 4 staging threads of a cell are consecutive lanes
    bacc += __shfl_xor(bacc, 1);
    bacc += __shfl_xor(bacc, 2);
    if (sq == 0) s_beta[si] = bacc;
    for (int pass = 0; pass < DG / RPASS; ++pass) {
        const int c_lo = RPASS * pass;
        if (c_lo >= nc) break;                       // uniform over the workgroup
        const int c_hi = min(c_lo + RPASS, nc);
        if (wm == (pass >> 1)) {
            const int fm = pass & 1;
#pragma unroll
            for (int fn = 0; fn < 2; ++fn)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    Rl[acc_row(r, lane) * RLD + 64 * wn + 32 * fn + (lane & 31)] = acc[fm][fn][r];
        }
        __syncthreads();
        const int vb = s_cs[c_lo], ve = s_cs[c_hi];
        for (int v0 = vb + wave; v0 < ve; v0 += 4 * (DNT / 64)) {
            uint2 hv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int v = v0 + q * (DNT / 64);
                hv[q] = v < ve ? nt_load_u2(h3 + (int64_t)v * H + 4 * lane) : make_uint2(0u, 0u);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int v = v0 + q * (DNT / 64);
                if (v >= ve) break;                  // uniform over the wave
                int lo = c_lo, hi = c_hi - 1;        // cell of visibility v
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_cs[mid] <= v) lo = mid; else hi = mid - 1;
                }
                const float4 rr = *(const float4 *)(Rl + (lo - c_lo) * RLD + 4 * lane);
                float sum = __uint_as_float(hv[q].x << 16) * rr.x + __uint_as_float(hv[q].x & 0xffff0000u) * rr.y +
                            __uint_as_float(hv[q].y << 16) * rr.z + __uint_as_float(hv[q].y & 0xffff0000u) * rr.w;
                for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
                if (lane == 0) ((float *)&y[v])[part] = s_out * (sum + s_beta[lo]);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------- degridding, LDS ring

// The degridding's A operand (each cell's 32 x 32 box) read straight into LDS: the grid is first
// rounded to bfloat16 (re, im) pairs, 4 bytes per cell, with PADC wrapped columns on each side, so a
// box row's 32 cells are one contiguous run whatever the cell (the box never wraps along u), and each
// product step's 16 cells are 64 bytes.  Workgroups stream both operands with direct global-to-LDS
// loads (16 bytes per lane, no registers) through a ring of three stages, each issued two steps before
// its product; the step loop is unrolled by three, so every LDS access names its stage at compile time.
// LDS rows are 64 bytes with their four 16-byte chunks permuted (chunk c of row r at slot
// c ^ ((r >> 2) & 3)): a fragment read takes one chunk of 32 consecutive rows, and any 16 consecutive
// rows then cover 256 distinct bytes of banks (measured: 3.5 % faster than permuting by r >> 1).
constexpr int PADC = 16;
constexpr int RA = DG * 64, RB = DBN * 64;              // bytes of a stage: A rows, B rows
constexpr int STG = RA + RB;
constexpr int RPASS2 = 64;                              // cells per epilogue pass
static_assert((size_t)RPASS2 * RLD * 4 + (6 * DG + 1) * 4 <= 3 * (size_t)STG, "epilogue must fit the ring");
static_assert((KDEP / BK) % 3 == 1, "the step loop runs in threes plus one");

typedef __attribute__((address_space(3))) void lds_void_t;

__device__ __forceinline__ int swz(int r, int c) { return c ^ ((r >> 2) & 3); }

// acc[fm][fn] += A rows [arow0 + 32 fm, +32) times B rows [brow0 + 32 fn, +32), one 32-deep step, from
// a stage's permuted 64-byte rows
template <int FM, int FN>
__device__ __forceinline__ void mma_ring(f32x16 (&acc)[FM][FN], const unsigned char *As, const unsigned char *Bs,
                                         int arow0, int brow0, int lane) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
        const int c = kk / 8 + (lane >> 5), ro = lane & 31;
        bf16x8 a[FM], b[FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm) {
            const int r = arow0 + 32 * fm + ro;
            a[fm] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(As + r * 64 + swz(r, c) * 16));
        }
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
            const int r = brow0 + 32 * fn + ro;
            b[fn] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(Bs + r * 64 + swz(r, c) * 16));
        }
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn)
                acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[fm], b[fn], acc[fm][fn], 0, 0, 0);
    }
}

// gbf[gy][pc] = the cell (gy, (pc - PADC) mod Ng) of the grid as a bfloat16 pair (re low, im high)
__global__ void k_grid_bf16_pad(const float2 *__restrict__ grid, int logNg, uint32_t *__restrict__ gbf) {
    const int Ng = 1 << logNg, RS = Ng + 2 * PADC;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)Ng * RS) return;
    const int gy = (int)(e / RS), pc = (int)(e % RS);
    const float2 g = grid[(int64_t)gy * Ng + ((pc - PADC) & (Ng - 1))];
    gbf[e] = (uint32_t)to_bf16(g.x) | ((uint32_t)to_bf16(g.y) << 16);
}

// s_waitcnt: vector memory count <= N (N < 16), LDS count 0, export count unconstrained
template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
    static_assert(N >= 0 && N < 16, "vmcnt");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | (0x7 << 4));
}

template <int V>
using ic = std::integral_constant<int, V>;

// Same work and outputs as k_sur_degrid (two workgroups per group of <= DG cells, part 0 / 1 form
// r re / r im), operands through the LDS ring.  Per step each wave loads one 16-row piece of A (1 KB)
// and two of B: three loads, the only vector memory operations of the loop, so "this wave's stage t
// has landed" is "at most the three loads of stage t + 1 are outstanding".  Epilogue: r of 64 cells at
// a time in the ring (FP32), then one visibility per 16 lanes, two per group of lanes in flight: the
// hidden layer read in two 16-byte pieces per lane, the dot product summed across the row of lanes.
__global__ __launch_bounds__(DNT, 4) void k_sur_degrid_ring(const uint32_t *__restrict__ gbf, int logNg,
                                                            const int *__restrict__ grp, int ngrp,
                                                            const int *__restrict__ cell_key,
                                                            const int *__restrict__ cell_start,
                                                            const uint16_t *__restrict__ h3,
                                                            const uint16_t *__restrict__ Bdeg,
                                                            const float *__restrict__ b4, float s_out,
                                                            float2 *__restrict__ y) {
    __shared__ __align__(16) unsigned char ring[3 * STG];
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 2, wn = wave & 3;
    const int part = blockIdx.y;
    const int g = (int)xcd_block(blockIdx.x, ngrp);
    const int c0 = grp[g], nc = grp[g + 1] - c0;
    const int Ng = 1 << logNg, RS = Ng + 2 * PADC;
    // this lane's pieces: A row ra (its grid cell), B rows rb0, rb1; the permuted chunk it carries
    const int ra = 16 * wave + (lane >> 2), rb0 = 32 * wave + (lane >> 2), rb1 = rb0 + 16;
    const int ca = swz(ra, lane & 3), cb0 = swz(rb0, lane & 3), cb1 = swz(rb1, lane & 3);
    int acv = 0, acu = 0;                            // rows past the group read cell (0, 0): in bounds, unused
    if (ra < nc) demorton2(cell_key[c0 + ra], acv, acu);
    // byte offsets: a uniform base plus a 32-bit per-lane part (the padded grid is < 4 GiB)
    const char *gA = (const char *)gbf;
    const char *gB = (const char *)(Bdeg + (int64_t)part * DBN * KDEP);   // [step][256][32]
    const uint32_t a_col = 4u * (uint32_t)(acu + 4 * ca), a_row = 4u * (uint32_t)RS;
    const uint32_t b_off0 = 2u * (uint32_t)(rb0 * 32 + 8 * cb0), b_off1 = 2u * (uint32_t)(rb1 * 32 + 8 * cb1);
    auto stage = [&](auto sc) -> unsigned char * {
        constexpr int S = decltype(sc)::value;
        return ring + S * STG;
    };
    // the loads' LDS destinations as wave-uniform 32-bit addresses: the ring's waits are the explicit ones
    // of each step, not ones derived from the destinations
    auto lds_dst = [&](const unsigned char *p) {
        const uint32_t a = (uint32_t)(uintptr_t)(const lds_void_t *)p;
        return (lds_void_t *)(uintptr_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)a);
    };
    auto issue = [&](int t, auto sc) {
        unsigned char *st = stage(sc);
        const uint32_t gy = (uint32_t)((acv + (t >> 1) - BOX / 2) & (Ng - 1));
        __builtin_amdgcn_global_load_lds((const void *)(gA + (gy * a_row + a_col + 64u * (t & 1))),
                                         lds_dst(st + 16 * wave * 64), 16, 0, 0);
        const char *gBt = gB + (size_t)t * DBN * 64;
        __builtin_amdgcn_global_load_lds((const void *)(gBt + b_off0), lds_dst(st + RA + 32 * wave * 64), 16, 0, 0);
        __builtin_amdgcn_global_load_lds((const void *)(gBt + b_off1), lds_dst(st + RA + (32 * wave + 16) * 64), 16,
                                         0, 0);
    };
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    // bias term of each cell: thread -> cell si, one 16-byte chunk sq (4 box cells) of the step's 16; the
    // chunk is the same over a wave, so its four output biases are scalar loads
    const int si = tid & (DG - 1), sq = wave >> 1;
    static_assert(DNT == 4 * DG, "four chunks per cell");
    float bacc = 0.0f;
    constexpr int NSTEP = KDEP / BK;
    auto step = [&](int t, auto sc) {
        constexpr int S = decltype(sc)::value;
        if (t + 1 < NSTEP) wait_vm_lgkm0<3>(); else wait_vm_lgkm0<0>();
        __builtin_amdgcn_s_barrier();                // every wave's stage t is in; every wave is past step t - 1
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (t + 2 < NSTEP) issue(t + 2, ic<(S + 2) % 3>{});
        const unsigned char *st = stage(sc);
        {
            const u32x4 a = *(const u32x4 *)(st + si * 64 + swz(si, sq) * 16);
            const float *bq = b4 + 2 * (16 * t + 4 * sq);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float xr = __uint_as_float(a[e] << 16), xi = __uint_as_float(a[e] & 0xffff0000u);
                const float br = bq[2 * e], bim = bq[2 * e + 1];
                bacc += part == 0 ? br * xr - bim * xi : br * xi + bim * xr;
            }
        }
        mma_ring<2, 2>(acc, st, st + RA, 64 * wm, 64 * wn, lane);
    };
    issue(0, ic<0>{});
    issue(1, ic<1>{});
    for (int t = 0; t < NSTEP - 1; t += 3) {
        step(t, ic<0>{});
        step(t + 1, ic<1>{});
        step(t + 2, ic<2>{});
    }
    step(NSTEP - 1, ic<0>{});
    __syncthreads();                                 // the ring becomes the epilogue's r, starts and biases
    float *Rl = (float *)ring;                       // [RPASS2][RLD] FP32
    int *s_cs = (int *)(ring + RPASS2 * RLD * 4);
    float *s_beta = (float *)(s_cs + DG + 1);
    float *s_bp = s_beta + DG;                       // [4][DG] the chunks' partial sums
    for (int i = tid; i <= nc; i += DNT) s_cs[i] = cell_start[c0 + i];
    s_bp[sq * DG + si] = bacc;
    __syncthreads();
    if (tid < DG) s_beta[tid] = (s_bp[tid] + s_bp[DG + tid]) + (s_bp[2 * DG + tid] + s_bp[3 * DG + tid]);
    const int lg = wave * 4 + (lane >> 4), lj = lane & 15;   // 32 groups of 16 lanes; lane lj of its group
    for (int pass = 0; pass < DG / RPASS2; ++pass) {
        const int c_lo = RPASS2 * pass;
        if (c_lo >= nc) break;                       // uniform over the workgroup
        const int c_hi = min(c_lo + RPASS2, nc);
        if (wm == pass) {                            // cells [64 pass, +64): the accumulators of the waves of row pass
#pragma unroll
            for (int fm = 0; fm < 2; ++fm)
#pragma unroll
                for (int fn = 0; fn < 2; ++fn)
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        Rl[(32 * fm + acc_row(r, lane)) * RLD + 64 * wn + 32 * fn + (lane & 31)] = acc[fm][fn][r];
        }
        __syncthreads();
        const int vb = s_cs[c_lo], ve = s_cs[c_hi];
        // the cell of visibility v is c_lo plus the number of the pass's later cells starting at or before
        // v: lane lj holds the starts of cells c_lo + 1 + 4 lj .. + 3 (past the pass: never at or before v)
        int cs4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = c_lo + 1 + 4 * lj + k;
            cs4[k] = c < c_hi ? s_cs[c] : INT_MAX;
        }
        // visibilities v0 = vb + lg + 64 i and v0 + 32: hidden units 8 lj .. 8 lj + 7 and 128 + 8 lj .. + 7
        for (int v0 = vb + lg; v0 < ve; v0 += 64) {
            const int v1 = v0 + 32;
            const bool ok1 = v1 < ve;
            const uint16_t *h0 = h3 + (int64_t)v0 * H + 8 * lj, *h1 = h3 + (int64_t)(ok1 ? v1 : v0) * H + 8 * lj;
            const u32x4 a0 = nt_load_u4(h0), b0 = nt_load_u4(h0 + H / 2);
            const u32x4 a1 = nt_load_u4(h1), b1 = nt_load_u4(h1 + H / 2);
            int cl[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int v = q == 0 ? v0 : (ok1 ? v1 : v0);
                const int n = (cs4[0] <= v) + (cs4[1] <= v) + (cs4[2] <= v) + (cs4[3] <= v);
                cl[q] = c_lo + (int)dpp_sum16((float)n);   // at most 64: exact in FP32
            }
            float sum[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const u32x4 ha = q == 0 ? a0 : a1, hb = q == 0 ? b0 : b1;
                const float *rr = Rl + (cl[q] - c_lo) * RLD + 8 * lj;
                const float4 r0 = *(const float4 *)rr, r1 = *(const float4 *)(rr + 4);
                const float4 r2 = *(const float4 *)(rr + H / 2), r3 = *(const float4 *)(rr + H / 2 + 4);
                float acc_s = __uint_as_float(ha[0] << 16) * r0.x + __uint_as_float(ha[0] & 0xffff0000u) * r0.y;
                acc_s += __uint_as_float(ha[1] << 16) * r0.z + __uint_as_float(ha[1] & 0xffff0000u) * r0.w;
                acc_s += __uint_as_float(ha[2] << 16) * r1.x + __uint_as_float(ha[2] & 0xffff0000u) * r1.y;
                acc_s += __uint_as_float(ha[3] << 16) * r1.z + __uint_as_float(ha[3] & 0xffff0000u) * r1.w;
                acc_s += __uint_as_float(hb[0] << 16) * r2.x + __uint_as_float(hb[0] & 0xffff0000u) * r2.y;
                acc_s += __uint_as_float(hb[1] << 16) * r2.z + __uint_as_float(hb[1] & 0xffff0000u) * r2.w;
                acc_s += __uint_as_float(hb[2] << 16) * r3.x + __uint_as_float(hb[2] & 0xffff0000u) * r3.y;
                acc_s += __uint_as_float(hb[3] << 16) * r3.z + __uint_as_float(hb[3] & 0xffff0000u) * r3.w;
                sum[q] = dpp_sum16(acc_s);
            }
            if (lj == 0) {
                ((float *)&y[v0])[part] = s_out * (sum[0] + s_beta[cl[0]]);
                if (ok1) ((float *)&y[v1])[part] = s_out * (sum[1] + s_beta[cl[1]]);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------- gridding

// One workgroup per group of <= AG consecutive occupied cells whose boxes fit the LDS window:
// A[i] = s of cell i (bfloat16, staged in LDS, then held in registers by every wave), box
// contributions = A Bgrd^T in blocks of 32 outputs (wave w takes blocks w, w + 4, ...; the weight
// fragments come from L2 straight into registers), accumulated in the window and added to the
// grid with atomics.
__global__ __launch_bounds__(ANT, 2) void k_sur_grid(const float2 *__restrict__ y, int logNg,
                                                     const int *__restrict__ grp, const int2 *__restrict__ org,
                                                     int ngrp, const int *__restrict__ cell_key,
                                                     const int *__restrict__ cell_start,
                                                     const uint16_t *__restrict__ h3,
                                                     const uint16_t *__restrict__ Bgrd, const float *__restrict__ b4,
                                                     const float *__restrict__ wmax, float s_out,
                                                     float2 *__restrict__ grid) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *Sa = (uint16_t *)smem;                               // [AG][SLD]
    int2 *win = (int2 *)(smem + (size_t)AG * SLD * 2);             // [WV][WU] fixed point (re, im)
    __shared__ int s_wv[AG], s_wu[AG];
    __shared__ float2 s_Y[AG];
    __shared__ float s_bnd[AG];                     // bound on |output| / s_out of each cell
    __shared__ float2 s_b4[BOX * BOX];               // output bias (no global loads inside the loop)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < BOX * BOX; i += ANT) s_b4[i] = ((const float2 *)b4)[i];
    const int g = blockIdx.x;
    const int c0 = grp[g], nc = grp[g + 1] - c0;
    const int2 o = org[g];                          // window origin: (min v - 16, min u - 16) of the group's cells
    const int Ng = 1 << logNg;
    for (int i = tid; i < AG; i += ANT) {
        int cv = 0, cu = 0;
        if (i < nc) demorton2(cell_key[c0 + i], cv, cu);
        s_wv[i] = i < nc ? cv - (o.x + BOX / 2) : 0;
        s_wu[i] = i < nc ? cu - (o.y + BOX / 2) : 0;
    }
    for (int e = tid; e < WV * WU; e += ANT) win[e] = make_int2(0, 0);
    // s of each cell: wave w takes the cells w + 4h (h < CP = 8: all eight of its cells) together; lane l hidden units
    // 4l .. 4l + 3.  The CP cells' loads are issued together (cells hold few visibilities).
    constexpr int NW = ANT / 64, CP = 8;
    for (int i0 = wave; i0 < AG; i0 += CP * NW) {
        float sr[CP][4] = {}, sm[CP][4] = {};
        float2 Y[CP] = {};
        int jb[CP], je[CP];
#pragma unroll
        for (int h = 0; h < CP; ++h) {
            const int i = i0 + h * NW;
            jb[h] = i < nc ? cell_start[c0 + i] : 0;
            je[h] = i < nc ? cell_start[c0 + i + 1] : 0;
        }
        int kmax = 0;
#pragma unroll
        for (int h = 0; h < CP; ++h) kmax = max(kmax, je[h] - jb[h]);
        for (int k0 = 0; k0 < kmax; k0 += 4) {
            uint2 hv[CP][4];
            float2 yk[CP][4];
#pragma unroll
            for (int h = 0; h < CP; ++h)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int k = jb[h] + k0 + q;
                    const bool ok = k < je[h];
                    hv[h][q] = ok ? nt_load_u2(h3 + (int64_t)k * H + 4 * lane) : make_uint2(0u, 0u);
                    yk[h][q] = ok ? nt_load_f2(y + k) : make_float2(0.f, 0.f);
                }
#pragma unroll
            for (int h = 0; h < CP; ++h)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float h0 = __uint_as_float(hv[h][q].x << 16), h1 = __uint_as_float(hv[h][q].x & 0xffff0000u);
                    const float h2 = __uint_as_float(hv[h][q].y << 16), h3v = __uint_as_float(hv[h][q].y & 0xffff0000u);
                    sr[h][0] += h0 * yk[h][q].x; sm[h][0] += h0 * yk[h][q].y;
                    sr[h][1] += h1 * yk[h][q].x; sm[h][1] += h1 * yk[h][q].y;
                    sr[h][2] += h2 * yk[h][q].x; sm[h][2] += h2 * yk[h][q].y;
                    sr[h][3] += h3v * yk[h][q].x; sm[h][3] += h3v * yk[h][q].y;
                    Y[h].x += yk[h][q].x;
                    Y[h].y += yk[h][q].y;
                }
        }
#pragma unroll
        for (int h = 0; h < CP; ++h) {
            const int i = i0 + h * NW;
            if (i >= AG) continue;                 // wave-uniform
            uint2 pr, pm;
            pr.x = (uint32_t)to_bf16(sr[h][0]) | ((uint32_t)to_bf16(sr[h][1]) << 16);
            pr.y = (uint32_t)to_bf16(sr[h][2]) | ((uint32_t)to_bf16(sr[h][3]) << 16);
            pm.x = (uint32_t)to_bf16(sm[h][0]) | ((uint32_t)to_bf16(sm[h][1]) << 16);
            pm.y = (uint32_t)to_bf16(sm[h][2]) | ((uint32_t)to_bf16(sm[h][3]) << 16);
            *(uint2 *)(Sa + i * SLD + 4 * lane) = pr;
            *(uint2 *)(Sa + i * SLD + H + 4 * lane) = pm;
            // |A_i . B_o| <= ||A_i||_2 ||B_o||_2 (Cauchy-Schwarz) and |bias| <= max|b4| (|Y re| + |Y im|):
            // a bound on every output of the cell (A_i: the bfloat16 values just stored)
            float l2 = 0.f;
            for (int e2 = 0; e2 < 4; ++e2) {
                const uint32_t wr = e2 < 2 ? (e2 == 0 ? pr.x : pr.y) : (e2 == 2 ? pm.x : pm.y);
                const float lo = from_bf16(wr & 0xffffu), hi = from_bf16(wr >> 16);
                l2 = fmaf(lo, lo, fmaf(hi, hi, l2));
            }
            for (int o2 = 32; o2 > 0; o2 >>= 1) l2 += __shfl_xor(l2, o2);
            if (lane == 0) {
                s_Y[i] = Y[h];
                s_bnd[i] = sqrtf(l2) * 1.0001f * wmax[0] + wmax[1] * (fabsf(Y[h].x) + fabsf(Y[h].y));
            }
        }
    }
    __syncthreads();
    // LDS float atomics are slow on this GPU, integer ones fast: the window accumulates in 32-bit
    // fixed point with a scale from the group's bound (at most AG cells reach one window cell, so
    // |sum| <= 2^29 < 2^31), and the flush converts back
    float gmax = 0.f;
    for (int i = 0; i < nc; ++i) gmax = fmaxf(gmax, s_bnd[i]);
    const float q = gmax > 0.f ? 536870912.0f / (gmax * s_out * (float)AG) : 1.0f;   // 2^29 / (AG max bound)
    const float qs = q * s_out;
    // the whole A operand of the group in registers: 32 steps of 16
    constexpr int KS = ND / 16;
    bf16x8 a[KS];
    const int ro = lane & 31, ko = 8 * (lane >> 5);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a[ks] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(Sa + ro * SLD + 16 * ks + ko));
    // per accumulator register r, this lane's cell i = acc_row(r, lane) is the same for every block:
    // its window offset and sum of y, in registers (-1: no cell)
    int wb[16];
    float2 Yr[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = acc_row(r, lane);
        wb[r] = i < nc ? s_wv[i] * WU + s_wu[i] : -1;
        Yr[r] = s_Y[i];
    }
    // two blocks of 32 outputs per pass (two independent accumulation chains, twice the loads in flight)
    for (int blk0 = 2 * wave; blk0 < NOUT / 32; blk0 += 2 * (ANT / 64)) {
        f32x16 acc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[h][r] = 0.0f;
        const uint16_t *brow0 = Bgrd + ((int64_t)blk0 * KS * 64 + lane) * 8;      // fragment-major
        const uint16_t *brow1 = brow0 + (int64_t)KS * 64 * 8;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const bf16x8 b0 = __builtin_bit_cast(bf16x8, *(const u32x4 *)(brow0 + 512 * ks));
            const bf16x8 b1 = __builtin_bit_cast(bf16x8, *(const u32x4 *)(brow1 + 512 * ks));
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ks], b0, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ks], b1, acc[1], 0, 0, 0);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // output o = 32 blk + lane % 32 of cell i: box cell p = o / 2, component o % 2
            const int oo = 32 * (blk0 + h) + ro;
            const int p = oo >> 1, comp = oo & 1;
            const int oy = p >> 5, ox = p & (BOX - 1);
            const float br = s_b4[p].x, bi = s_b4[p].y;
            const int woff = oy * WU + ox;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                if (wb[r] >= 0) {
                    const float2 Y = Yr[r];
                    const float bias = comp == 0 ? br * Y.x + bi * Y.y : br * Y.y - bi * Y.x;
                    int *dst = (int *)&win[wb[r] + woff] + comp;
                    atomicAdd(dst, __float2int_rn(qs * (acc[h][r] + bias)));
                }
            }
        }
    }
    __syncthreads();
    const float iq = 1.0f / q;
    for (int e = tid; e < WV * WU; e += ANT) {
        const int2 wi = win[e];
        const float2 val = make_float2((float)wi.x * iq, (float)wi.y * iq);
        if (wi.x != 0 || wi.y != 0) {
            const int gy = (o.x + e / WU) & (Ng - 1), gx = (o.y + e % WU) & (Ng - 1);
            float *dst = (float *)&grid[(int64_t)gy * Ng + gx];
            atomicAdd(dst, val.x);
            atomicAdd(dst + 1, val.y);
        }
    }
}

// ---------------------------------------------------------------------------- gridding, LDS ring

// s of every cell, the A operand of the ring gridding: s_c = sum over the cell's visibilities of
// h_k y_k (k < 256: with Re y, k >= 256: with Im y) in bfloat16, with the cell's sum of y and a bound
// on its outputs / s_out (as the register-staged gridding bounds them).  One cell per 16 lanes: lane j
// holds hidden units 8 j .. 8 j + 7 and 128 + 8 j .. + 7; two visibilities' loads in flight.
__global__ __launch_bounds__(256) void k_sur_cell_s(const float2 *__restrict__ y, const int *__restrict__ cell_start,
                                                    int ncell, const uint16_t *__restrict__ h3,
                                                    const float *__restrict__ wmax, uint16_t *__restrict__ Sg,
                                                    float4 *__restrict__ cY) {
    const int c = blockIdx.x * 16 + (threadIdx.x >> 4), j = threadIdx.x & 15;
    if (c >= ncell) return;                          // whole rows of 16 lanes
    const int vb = cell_start[c], ve = cell_start[c + 1];
    float sr[16], si[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) sr[e] = si[e] = 0.0f;
    float2 Y = make_float2(0.f, 0.f);
    for (int v = vb; v < ve; v += 2) {
        const bool two = v + 1 < ve;
        const uint16_t *h0 = h3 + (int64_t)v * H + 8 * j, *h1 = h3 + (int64_t)(two ? v + 1 : v) * H + 8 * j;
        const u32x4 a0 = nt_load_u4(h0), b0 = nt_load_u4(h0 + H / 2);
        const u32x4 a1 = nt_load_u4(h1), b1 = nt_load_u4(h1 + H / 2);
        const float2 y0 = y[v], y1 = two ? y[v + 1] : make_float2(0.f, 0.f);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const u32x4 ha = q == 0 ? a0 : a1, hb = q == 0 ? b0 : b1;
            const float2 yk = q == 0 ? y0 : y1;      // zero for the absent second visibility
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float l0 = __uint_as_float(ha[e] << 16), l1 = __uint_as_float(ha[e] & 0xffff0000u);
                const float m0 = __uint_as_float(hb[e] << 16), m1 = __uint_as_float(hb[e] & 0xffff0000u);
                sr[2 * e] += l0 * yk.x; si[2 * e] += l0 * yk.y;
                sr[2 * e + 1] += l1 * yk.x; si[2 * e + 1] += l1 * yk.y;
                sr[8 + 2 * e] += m0 * yk.x; si[8 + 2 * e] += m0 * yk.y;
                sr[8 + 2 * e + 1] += m1 * yk.x; si[8 + 2 * e + 1] += m1 * yk.y;
            }
            Y.x += yk.x;
            Y.y += yk.y;
        }
    }
    u32x4 o[4];                                      // re lo, re hi, im lo, im hi pieces
    float l2 = 0.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const uint16_t r0 = to_bf16(sr[2 * e]), r1 = to_bf16(sr[2 * e + 1]);
        const uint16_t r2 = to_bf16(sr[8 + 2 * e]), r3 = to_bf16(sr[8 + 2 * e + 1]);
        const uint16_t i0 = to_bf16(si[2 * e]), i1 = to_bf16(si[2 * e + 1]);
        const uint16_t i2 = to_bf16(si[8 + 2 * e]), i3 = to_bf16(si[8 + 2 * e + 1]);
        o[0][e] = (uint32_t)r0 | ((uint32_t)r1 << 16);
        o[1][e] = (uint32_t)r2 | ((uint32_t)r3 << 16);
        o[2][e] = (uint32_t)i0 | ((uint32_t)i1 << 16);
        o[3][e] = (uint32_t)i2 | ((uint32_t)i3 << 16);
        const uint16_t vals[8] = {r0, r1, r2, r3, i0, i1, i2, i3};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float f = from_bf16(vals[q]);
            l2 = fmaf(f, f, l2);
        }
    }
    uint16_t *row = Sg + (int64_t)c * ND + 8 * j;
    *(u32x4 *)row = o[0];
    *(u32x4 *)(row + H / 2) = o[1];
    *(u32x4 *)(row + H) = o[2];
    *(u32x4 *)(row + H + H / 2) = o[3];
    l2 = dpp_sum16(l2);
    // |A_c . B_o| <= ||A_c||_2 ||B_o||_2 (Cauchy-Schwarz) and |bias| <= max|b4| (|Y re| + |Y im|)
    if (j == 0) cY[c] = make_float4(Y.x, Y.y, sqrtf(l2) * 1.0001f * wmax[0] + wmax[1] * (fabsf(Y.x) + fabsf(Y.y)), 0.f);
}

// The box contributions s_out (W4 s_c + conj(b4) Y_c) of a group of <= DG cells spanning at most GSPAN
// rows and columns, for one slice of 256 outputs (box rows 4 sl .. 4 sl + 3): the product of the cells'
// s [DG x 512] and the slice's weights [256 x 512] through the same three-stage ring of direct loads as
// the degridding (16 steps of 32), then added in 32-bit fixed point into an LDS window over the ring
// (the slice's box rows of every cell: (span + 4) x (span + 32) cells) and flushed to the grid with
// atomics.  The eight slices of a group are consecutive blocks on one XCD, so they share its s in L2.
__global__ __launch_bounds__(DNT, 4) void k_sur_grid_ring(const uint16_t *__restrict__ Sg, int zrow,
                                                          const float4 *__restrict__ cY, int logNg,
                                                          const int *__restrict__ grp, const int4 *__restrict__ org,
                                                          int ngrp, const int *__restrict__ cell_key,
                                                          const uint16_t *__restrict__ Bgrd2,
                                                          const float *__restrict__ b4, float s_out,
                                                          float2 *__restrict__ grid) {
    __shared__ __align__(16) unsigned char ring[3 * STG];
    __shared__ __align__(16) int s_woff[DG];
    __shared__ __align__(16) float2 s_Y[DG];
    __shared__ float s_gm[DG / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 2, wn = wave & 3;
    const int lb = (int)xcd_block(blockIdx.x, (int64_t)ngrp * NSL);
    const int g = lb / NSL, sl = lb % NSL;
    const int c0 = grp[g], nc = grp[g + 1] - c0;
    const int Ng = 1 << logNg;
    // this lane's pieces: A row ra (a cell of the group; rows past it read the zero row zrow), B rows rb0, rb1
    const int ra = 16 * wave + (lane >> 2), rb0 = 32 * wave + (lane >> 2), rb1 = rb0 + 16;
    const int ca = swz(ra, lane & 3), cb0 = swz(rb0, lane & 3), cb1 = swz(rb1, lane & 3);
    const char *arow = (const char *)(Sg + (int64_t)(ra < nc ? c0 + ra : zrow) * ND) + 16 * ca;
    const char *gB = (const char *)(Bgrd2 + (int64_t)sl * 256 * ND);     // [step][256][32]
    const uint32_t b_off0 = 2u * (uint32_t)(rb0 * 32 + 8 * cb0), b_off1 = 2u * (uint32_t)(rb1 * 32 + 8 * cb1);
    auto stage = [&](auto sc) -> unsigned char * {
        constexpr int S = decltype(sc)::value;
        return ring + S * STG;
    };
    auto lds_dst = [&](const unsigned char *p) {
        const uint32_t a = (uint32_t)(uintptr_t)(const lds_void_t *)p;
        return (lds_void_t *)(uintptr_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)a);
    };
    auto issue = [&](int t, auto sc) {
        unsigned char *st = stage(sc);
        __builtin_amdgcn_global_load_lds((const void *)(arow + 64 * t), lds_dst(st + 16 * wave * 64), 16, 0, 0);
        const char *gBt = gB + (size_t)t * 256 * 64;
        __builtin_amdgcn_global_load_lds((const void *)(gBt + b_off0), lds_dst(st + RA + 32 * wave * 64), 16, 0, 0);
        __builtin_amdgcn_global_load_lds((const void *)(gBt + b_off1), lds_dst(st + RA + (32 * wave + 16) * 64), 16,
                                         0, 0);
    };
    // the first two stages go out first; the group's cells, needed only after the products, load into
    // registers while they land (no barrier before the loop)
    issue(0, ic<0>{});
    issue(1, ic<1>{});
    int ckey = 0;
    float4 cy = make_float4(0.f, 0.f, 0.f, 0.f);
    if (tid < nc && tid < DG) {
        ckey = cell_key[c0 + tid];
        cy = cY[c0 + tid];
    }
    const int4 o0 = org[g];                          // smallest (v, u) of the group's cells, their spans
    // this lane's two outputs (one per fn): window offset within a cell's box rows, component, bias weights
    int wo[2], comp[2];
    float br[2], bi[2];
#pragma unroll
    for (int fn = 0; fn < 2; ++fn) {
        const int oo = 256 * sl + 64 * wn + 32 * fn + (lane & 31);
        const int p = oo >> 1;
        comp[fn] = oo & 1;
        wo[fn] = ((p >> 5) - 4 * sl) * GWC + (p & (BOX - 1));
        br[fn] = b4[2 * p];
        bi[fn] = b4[2 * p + 1];
    }
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    constexpr int NSTEP = ND / BK;
    static_assert(NSTEP % 3 == 1, "the step loop runs in threes plus one");
    // a group cut short by its span has fewer than DG cells; the rows past it read the zero row, and a
    // wave none of whose rows holds a cell of the group skips the products
    const bool busy = 64 * wm < nc;
    auto step = [&](int t, auto sc) {
        constexpr int S = decltype(sc)::value;
        if (t + 1 < NSTEP) wait_vm_lgkm0<3>(); else wait_vm_lgkm0<0>();
        __builtin_amdgcn_s_barrier();                // every wave's stage t is in; every wave is past step t - 1
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (t + 2 < NSTEP) issue(t + 2, ic<(S + 2) % 3>{});
        const unsigned char *st = stage(sc);
        if (busy) mma_ring<2, 2>(acc, st, st + RA, 64 * wm, 64 * wn, lane);
    };
    for (int t = 0; t < NSTEP - 1; t += 3) {
        step(t, ic<0>{});
        step(t + 1, ic<1>{});
        step(t + 2, ic<2>{});
    }
    step(NSTEP - 1, ic<0>{});
    __syncthreads();                                 // the ring becomes the window
    static_assert(DG <= DNT && DG % 64 == 0, "one thread per cell of the group");
    if (tid < DG) {
        int woff = 0;
        if (tid < nc) {
            int cv, cu;
            demorton2(ckey, cv, cu);
            woff = (cv - o0.x) * GWC + (cu - o0.y);
        }
        s_woff[tid] = 8 * woff;                      // bytes
        s_Y[tid] = make_float2(cy.x, cy.y);
        float m = cy.z;                              // the cells' largest bound (zero past the group)
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        if (lane == 0) s_gm[tid >> 6] = m;
    }
    int2 *win = (int2 *)ring;                        // [GWR][GWC] fixed point (re, im)
    static_assert((size_t)GWR * GWC * 8 <= 3 * (size_t)STG, "window must fit the ring");
    // only the rows and columns the group's boxes reach: (span_v + 4) x (span_u + 32)
    // a wave per window row, a lane per column
    const int wr = o0.z + 4, wc = o0.w + BOX;
    for (int ry = wave; ry < wr; ry += DNT / 64)
        for (int rx = lane; rx < wc; rx += 64) win[ry * GWC + rx] = make_int2(0, 0);
    __syncthreads();
    // the scale: at most DG cells reach one window cell, each by at most the group's largest bound, so
    // every sum stays within 2^29 < 2^31
    float gmax = s_gm[0];
#pragma unroll
    for (int w2 = 1; w2 < DG / 64; ++w2) gmax = fmaxf(gmax, s_gm[w2]);
    const float q = gmax > 0.f ? 536870912.0f / (gmax * s_out * (float)DG) : 1.0f;
    const float qs = q * s_out;
    // this lane's output of a cell adds the bias ca Re Y + cb Im Y (the real or the imaginary part of
    // conj(b4) Y, by the lane's component); the coefficients carry the fixed-point scale.  Its byte
    // offset within a cell's place in the window: wob.
    float caq[2], cbq[2];
    int wob[2];
#pragma unroll
    for (int fn = 0; fn < 2; ++fn) {
        caq[fn] = (comp[fn] == 0 ? br[fn] : -bi[fn]) * qs;
        cbq[fn] = (comp[fn] == 0 ? bi[fn] : br[fn]) * qs;
        wob[fn] = 8 * wo[fn] + 4 * comp[fn];
    }
    // a lane's rows come in fours (registers 4 r4 .. 4 r4 + 3 hold rows i0 .. i0 + 3): one 16-byte read of
    // their window offsets and two of their sums of y.  Rows past the group (products of the zero row,
    // Y zero) add zero at offset 0.
    char *winb = (char *)win;
#pragma unroll
    for (int fm = 0; fm < 2; ++fm)
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
            if (64 * wm + 32 * fm + 8 * r4 >= nc) continue;   // no cell of the group in these rows
            const int i0 = 64 * wm + 32 * fm + acc_row(4 * r4, lane);
            const int4 wf = *(const int4 *)&s_woff[i0];
            const float4 ya = *(const float4 *)&s_Y[i0], yb = *(const float4 *)&s_Y[i0 + 2];
            const int wv[4] = {wf.x, wf.y, wf.z, wf.w};
            const float yr[4] = {ya.x, ya.z, yb.x, yb.z}, yi[4] = {ya.y, ya.w, yb.y, yb.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int fn = 0; fn < 2; ++fn) {
                    const float bq = fmaf(caq[fn], yr[e], cbq[fn] * yi[e]);
                    atomicAdd((int *)(winb + wv[e] + wob[fn]), __float2int_rn(fmaf(acc[fm][fn][4 * r4 + e], qs, bq)));
                }
        }
    __syncthreads();
    const float iq = 1.0f / q;
    const int gv0 = o0.x - BOX / 2 + 4 * sl, gu0 = o0.y - BOX / 2;
    for (int ry = wave; ry < wr; ry += DNT / 64)
        for (int rx = lane; rx < wc; rx += 64) {
            const int2 wi = win[ry * GWC + rx];
            if (wi.x != 0 || wi.y != 0) {
                const int gy = (gv0 + ry) & (Ng - 1), gx = (gu0 + rx) & (Ng - 1);
                float *dst = (float *)&grid[(int64_t)gy * Ng + gx];
                atomicAdd(dst, (float)wi.x * iq);
                atomicAdd(dst + 1, (float)wi.y * iq);
            }
        }
}

wp_status check_sur(const wp_plan *p, const wp_surrogate *s) {
    if (!p) return wp_set_error(WP_EINVAL, "plan is NULL");
    if (!s) return wp_set_error(WP_EINVAL, "surrogate is NULL");
    if (s->logNg != p->logNg) return wp_set_error(WP_EINVAL, "surrogate built for another grid size");
    return WP_OK;
}

wp_status sur_degrid(const wp_plan *p, const wp_surrogate *S, const float2 *grid, float2 *y, hipStream_t s) {
    if (S->Ms == 0) return WP_OK;
    const int form = p->sur_degrid > 0 ? p->sur_degrid : 2;
    if (form == 2) {
        const int64_t n = (int64_t)p->Ng * (p->Ng + 2 * PADC);
        hipLaunchKernelGGL(k_grid_bf16_pad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, grid, p->logNg, S->gbf);
        hipLaunchKernelGGL(k_sur_degrid_ring, dim3(S->ngrp_d, 2), dim3(DNT), 0, s, S->gbf, p->logNg, S->grp_d,
                           S->ngrp_d, S->cell_key, S->cell_start, S->h3, S->Bdeg, S->b4, S->s_out, y);
        return wp_check_launch("k_sur_degrid_ring");
    }
    hipLaunchKernelGGL(k_sur_degrid, dim3(S->ngrp_d, 2), dim3(DNT), DEG_LDS, s, grid, p->logNg, S->grp_d, S->ngrp_d,
                       S->cell_key, S->cell_start, S->h3, S->Bdeg, S->b4, S->s_out, y);
    return wp_check_launch("k_sur_degrid");
}

wp_status sur_grid_add(const wp_plan *p, const wp_surrogate *S, const float2 *y, float2 *grid, hipStream_t s) {
    if (S->Ms == 0) return WP_OK;
    const int form = p->sur_grid > 0 ? p->sur_grid : 2;
    if (form == 2) {
        hipLaunchKernelGGL(k_sur_cell_s, dim3((unsigned)((S->ncell + 15) / 16)), dim3(256), 0, s, y, S->cell_start,
                           (int)S->ncell, S->h3, S->wmax, S->Sg, S->cY);
        wp_status st = wp_check_launch("k_sur_cell_s");
        if (st != WP_OK) return st;
        hipLaunchKernelGGL(k_sur_grid_ring, dim3((unsigned)((int64_t)S->ngrp_g * NSL)), dim3(DNT), 0, s, S->Sg,
                           (int)S->ncell, S->cY,
                           p->logNg, S->grp_g, S->grp_gorg, S->ngrp_g, S->cell_key, S->Bgrd2, S->b4, S->s_out, grid);
        return wp_check_launch("k_sur_grid_ring");
    }
    hipLaunchKernelGGL(k_sur_grid, dim3(S->ngrp_a), dim3(ANT), GRD_LDS, s, y, p->logNg, S->grp_a, S->grp_org,
                       S->ngrp_a, S->cell_key, S->cell_start, S->h3, S->Bgrd, S->b4, S->wmax, S->s_out, grid);
    return wp_check_launch("k_sur_grid");
}

wp_status check_fallback(const wp_plan *p, const wp_surrogate *S, const wp_G *Gf) {
    if (S->Mf == 0) return WP_OK;
    if (!Gf) return wp_set_error(WP_EINVAL, "%lld fallback rows need their exact G", (long long)S->Mf);
    if (Gf->M != S->Mf) return wp_set_error(WP_EINVAL, "fallback G has %lld rows, expected %lld", (long long)Gf->M,
                                            (long long)S->Mf);
    if (p && Gf->tblk && (!Gf->tcolptr || Gf->n_tblk != gather_table_slots(Gf->nnz, (int64_t)p->Ng * p->Ng, p->gb_ent)))
        return wp_set_error(WP_EINVAL, "fallback G: block table without the transposed copy or of the wrong size");
    return WP_OK;
}

// out[r] = in[caller index of slot r]; fallback slots follow the fallback G's order
__global__ void k_to_slots(const float2 *__restrict__ in, const int *__restrict__ slot_vis, int64_t Ms, int64_t M,
                           const int *__restrict__ fperm, float2 *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= M) return;
    const int64_t s = r < Ms ? r : Ms + (fperm ? fperm[r - Ms] : r - Ms);
    out[r] = in[slot_vis[s]];
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

extern "C" {

wp_status wp_surrogate_create(wp_surrogate **out, const wp_plan *p, wp_mlp *m, int64_t M, const double *u,
                              const double *v, const double *w, const float *eps, double tol, int64_t *Mf_out,
                              void *stream) {
    if (!out) return wp_set_error(WP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return wp_set_error(WP_EINVAL, "plan is NULL");
    if (!m) return wp_set_error(WP_EINVAL, "mlp is NULL");
    if (M < 1 || M > 0x7ffffffe) return wp_set_error(WP_EINVAL, "M = %lld out of range", (long long)M);
    if (!u || !v || !w) return wp_set_error(WP_EINVAL, "NULL coordinates");
    if (p->Ng < 2 * BOX) return wp_set_error(WP_EINVAL, "Ng = %d < %d", p->Ng, 2 * BOX);
    if (!(tol >= 0.0)) return wp_set_error(WP_EINVAL, "tol must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    const int bits = 2 * p->logNg;
    DevBuf feat, key, isfb, skey, sidx, sws, flag, cid, err;
    WP_HIP(hipMalloc(&feat.p, 12 * M));
    WP_HIP(hipMalloc(&key.p, 4 * M));
    WP_HIP(hipMalloc(&isfb.p, 4 * (M + 1)));
    WP_HIP(hipMalloc(&skey.p, 4 * M));
    WP_HIP(hipMalloc(&sidx.p, 4 * M));
    WP_HIP(hipMalloc(&sws.p, std::max(sort_workspace_bytes(M), scan_workspace_bytes(M + 1))));
    WP_HIP(hipMalloc(&flag.p, 4 * (M + 1)));
    WP_HIP(hipMalloc(&cid.p, 4 * (M + 1)));
    WP_HIP(hipMalloc(&err.p, 4));
    WP_HIP(hipMemsetAsync(err.p, 0, 4, s));
    wp_status st = wp_mlp_features(p, m, M, u, v, w, (float *)feat.p, (int *)err.p, s);
    if (st != WP_OK) return st;
    const int gM = (int)((M + 255) / 256);
    hipLaunchKernelGGL(k_slot_keys, dim3(gM), dim3(256), 0, s, u, v, M, p->cell, p->logNg, eps, (float)tol, 1 << bits,
                       (int *)key.p, (int *)isfb.p);
    if ((st = wp_check_launch("k_slot_keys")) != WP_OK) return st;
    if ((st = launch_sort_pairs((const int *)key.p, M, bits + 1, (int *)skey.p, (int *)sidx.p, sws.p, s)) != WP_OK)
        return st;
    if ((st = launch_scan_int((const int *)isfb.p, (int *)flag.p, M, sws.p, s)) != WP_OK) return st;
    int h_err = 0, h_mf = 0;
    WP_HIP(hipMemcpyAsync(&h_err, err.p, 4, hipMemcpyDeviceToHost, s));
    WP_HIP(hipMemcpyAsync(&h_mf, (int *)flag.p + M, 4, hipMemcpyDeviceToHost, s));
    WP_HIP(hipStreamSynchronize(s));
    if (h_err) return wp_set_error(WP_EINVAL, "a coordinate is not finite or lies outside the grid");

    wp_surrogate *S = (wp_surrogate *)calloc(1, sizeof(wp_surrogate));
    if (!S) return wp_set_error(WP_ENOMEM, "surrogate allocation");
    auto fail = [&](wp_status code, const char *what) {
        wp_surrogate_destroy(S);
        return wp_set_error(code, "surrogate create: %s", what);
    };
    (void)hipGetDevice(&S->device);
    S->logNg = p->logNg;
    S->M = M;
    S->Mf = h_mf;
    S->Ms = M - h_mf;
    S->s_out = (float)m->s_out;
    if (hipMalloc((void **)&S->slot_vis, 4 * M) != hipSuccess) return fail(WP_ENOMEM, "slots");
    WP_HIP(hipMemcpyAsync(S->slot_vis, sidx.p, 4 * M, hipMemcpyDeviceToDevice, s));
    if (S->Mf > 0) {
        if (hipMalloc((void **)&S->fb, 24 * S->Mf) != hipSuccess) return fail(WP_ENOMEM, "fallback coordinates");
        hipLaunchKernelGGL(k_fallback_coords, dim3((unsigned)((S->Mf + 255) / 256)), dim3(256), 0, s, u, v, w,
                           S->slot_vis, S->Ms, S->Mf, S->fb);
    }
    if (hipMalloc((void **)&S->Bdeg, (size_t)ND * KDEP * 2) != hipSuccess ||
        hipMalloc((void **)&S->Bgrd, (size_t)NOUT * ND * 2) != hipSuccess ||
        hipMalloc((void **)&S->Bgrd2, (size_t)NOUT * ND * 2) != hipSuccess ||
        hipMalloc((void **)&S->b4, (size_t)NOUT * 4) != hipSuccess)
        return fail(WP_ENOMEM, "weights");
    hipLaunchKernelGGL(k_make_B, dim3((unsigned)((NOUT * H + 255) / 256)), dim3(256), 0, s, m->params + OW4, S->Bdeg,
                       S->Bgrd, S->Bgrd2);
    WP_HIP(hipMemcpyAsync(S->b4, m->params + OB4, NOUT * 4, hipMemcpyDeviceToDevice, s));
    if (hipMalloc((void **)&S->wmax, 8) != hipSuccess) return fail(WP_ENOMEM, "weight bounds");
    WP_HIP(hipMemsetAsync(S->wmax, 0, 8, s));
    hipLaunchKernelGGL(k_weight_max, dim3((unsigned)((NOUT + 255) / 256)), dim3(256), 0, s, S->Bgrd, S->b4, S->wmax);
    if (S->Ms > 0) {
        const int64_t Ms = S->Ms;
        const int gS = (int)((Ms + 255) / 256);
        hipLaunchKernelGGL(k_cell_flags, dim3(gS), dim3(256), 0, s, (const int *)skey.p, Ms, (int *)flag.p);
        if ((st = launch_scan_int((const int *)flag.p, (int *)cid.p, Ms, sws.p, s)) != WP_OK) {
            wp_surrogate_destroy(S);
            return st;
        }
        int h_nc = 0;
        WP_HIP(hipMemcpyAsync(&h_nc, (int *)cid.p + Ms, 4, hipMemcpyDeviceToHost, s));
        WP_HIP(hipStreamSynchronize(s));
        S->ncell = h_nc;
        if (hipMalloc((void **)&S->cell_key, 4 * (size_t)h_nc) != hipSuccess ||
            hipMalloc((void **)&S->cell_start, 4 * (size_t)(h_nc + 1)) != hipSuccess)
            return fail(WP_ENOMEM, "cell table");
        hipLaunchKernelGGL(k_cell_table, dim3(gS), dim3(256), 0, s, (const int *)skey.p, (const int *)flag.p,
                           (const int *)cid.p, Ms, S->cell_key, S->cell_start);
        // groups, on the host: degridding groups of <= DG consecutive cells; gridding groups of
        // <= AG consecutive cells whose rows and columns each span at most WV - BOX (WU - BOX) + 1
        std::vector<int> ckey(h_nc), cstart(h_nc + 1);
        WP_HIP(hipMemcpyAsync(ckey.data(), S->cell_key, 4 * (size_t)h_nc, hipMemcpyDeviceToHost, s));
        WP_HIP(hipMemcpyAsync(cstart.data(), S->cell_start, 4 * (size_t)(h_nc + 1), hipMemcpyDeviceToHost, s));
        WP_HIP(hipStreamSynchronize(s));
        std::vector<int> gd, ga, gg;
        std::vector<int2> go;
        std::vector<int4> ggo;
        int vmin = 0, vmax = 0, umin = 0, umax = 0;
        int gvmin = 0, gvmax = 0, gumin = 0, gumax = 0;
        for (int c = 0; c < h_nc; ++c) {
            if (c % DG == 0) gd.push_back(c);
            int cv, cu;
            demorton2(ckey[c], cv, cu);
            // ring gridding: <= DG consecutive cells spanning at most GSPAN rows and GSPAN columns
            const bool gfits = !gg.empty() && c - gg.back() < DG &&
                               std::max(gvmax, cv) - std::min(gvmin, cv) < GSPAN &&
                               std::max(gumax, cu) - std::min(gumin, cu) < GSPAN;
            if (gfits) {
                gvmin = std::min(gvmin, cv); gvmax = std::max(gvmax, cv);
                gumin = std::min(gumin, cu); gumax = std::max(gumax, cu);
            } else {
                if (!gg.empty()) ggo.push_back(make_int4(gvmin, gumin, gvmax - gvmin, gumax - gumin));
                gg.push_back(c);
                gvmin = gvmax = cv;
                gumin = gumax = cu;
            }
            const bool fits = !ga.empty() && c - ga.back() < AG && std::max(vmax, cv) - std::min(vmin, cv) <= WV - BOX &&
                              std::max(umax, cu) - std::min(umin, cu) <= WU - BOX;
            if (fits) {
                vmin = std::min(vmin, cv); vmax = std::max(vmax, cv);
                umin = std::min(umin, cu); umax = std::max(umax, cu);
            } else {
                if (!ga.empty()) go.push_back(make_int2(vmin - BOX / 2, umin - BOX / 2));
                ga.push_back(c);
                vmin = vmax = cv;
                umin = umax = cu;
            }
        }
        go.push_back(make_int2(vmin - BOX / 2, umin - BOX / 2));
        ggo.push_back(make_int4(gvmin, gumin, gvmax - gvmin, gumax - gumin));
        gd.push_back(h_nc);
        ga.push_back(h_nc);
        gg.push_back(h_nc);
        S->ngrp_d = (int)gd.size() - 1;
        S->ngrp_a = (int)ga.size() - 1;
        S->ngrp_g = (int)gg.size() - 1;
        if (hipMalloc((void **)&S->grp_d, 4 * gd.size()) != hipSuccess ||
            hipMalloc((void **)&S->grp_a, 4 * ga.size()) != hipSuccess ||
            hipMalloc((void **)&S->grp_org, sizeof(int2) * go.size()) != hipSuccess ||
            hipMalloc((void **)&S->grp_g, 4 * gg.size()) != hipSuccess ||
            hipMalloc((void **)&S->grp_gorg, sizeof(int4) * ggo.size()) != hipSuccess)
            return fail(WP_ENOMEM, "groups");
        WP_HIP(hipMemcpyAsync(S->grp_d, gd.data(), 4 * gd.size(), hipMemcpyHostToDevice, s));
        WP_HIP(hipMemcpyAsync(S->grp_a, ga.data(), 4 * ga.size(), hipMemcpyHostToDevice, s));
        WP_HIP(hipMemcpyAsync(S->grp_org, go.data(), sizeof(int2) * go.size(), hipMemcpyHostToDevice, s));
        WP_HIP(hipMemcpyAsync(S->grp_g, gg.data(), 4 * gg.size(), hipMemcpyHostToDevice, s));
        WP_HIP(hipMemcpyAsync(S->grp_gorg, ggo.data(), sizeof(int4) * ggo.size(), hipMemcpyHostToDevice, s));
        WP_HIP(hipStreamSynchronize(s));
        // last hidden layer of every surrogate row, in slot order
        if (hipMalloc((void **)&S->h3, (size_t)Ms * H * 2) != hipSuccess) return fail(WP_ENOMEM, "hidden features");
        // the degridding's bfloat16 copy of the grid, with wrapped columns; the ring gridding's per-cell s
        if (hipMalloc((void **)&S->gbf, (size_t)p->Ng * (p->Ng + 2 * PADC) * 4) != hipSuccess)
            return fail(WP_ENOMEM, "bfloat16 grid");
        if (hipMalloc((void **)&S->Sg, (size_t)(h_nc + 1) * ND * 2) != hipSuccess ||
            hipMalloc((void **)&S->cY, (size_t)h_nc * sizeof(float4)) != hipSuccess)
            return fail(WP_ENOMEM, "per-cell s");
        WP_HIP(hipMemsetAsync(S->Sg + (size_t)h_nc * ND, 0, ND * 2, s));
        for (int64_t j0 = 0; j0 < Ms; j0 += m->max_batch) {
            const int n = (int)std::min<int64_t>(m->max_batch, Ms - j0);
            hipLaunchKernelGGL(k_feat_slots, dim3((3 * n + 255) / 256), dim3(256), 0, s, (const float *)feat.p,
                               S->slot_vis, j0, n, m->xb);
            if ((st = mlp_forward(m, n, m->xb, nullptr, s)) != WP_OK) {
                wp_surrogate_destroy(S);
                return st;
            }
            WP_HIP(hipMemcpyAsync(S->h3 + j0 * H, m->a3, (size_t)n * H * 2, hipMemcpyDeviceToDevice, s));
        }
    }
    if ((st = wp_check_launch("surrogate create")) != WP_OK) {
        wp_surrogate_destroy(S);
        return st;
    }
    WP_HIP(hipStreamSynchronize(s));
    if (Mf_out) *Mf_out = S->Mf;
    *out = S;
    return WP_OK;
}

wp_status wp_surrogate_destroy(wp_surrogate *S) {
    if (!S) return WP_OK;
    void *bufs[] = {S->slot_vis, S->cell_key, S->cell_start, S->grp_d, S->grp_a, S->grp_org, S->h3, S->Bdeg,
                    S->Bgrd, S->b4, S->wmax, S->fb, S->gbf, S->Bgrd2, S->Sg, S->cY, S->grp_g, S->grp_gorg};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    free(S);
    return WP_OK;
}

wp_status wp_surrogate_info(const wp_surrogate *S, int64_t *info5) {
    if (!S || !info5) return wp_set_error(WP_EINVAL, "NULL argument");
    info5[0] = S->M;
    info5[1] = S->Ms;
    info5[2] = S->Mf;
    info5[3] = S->ncell;
    info5[4] = (int64_t)S->ngrp_d << 32 | (int64_t)S->ngrp_a;
    return WP_OK;
}

wp_status wp_surrogate_slots(const wp_surrogate *S, int *slot_vis, void *stream) {
    if (!S || !slot_vis) return wp_set_error(WP_EINVAL, "NULL argument");
    WP_HIP(hipMemcpyAsync(slot_vis, S->slot_vis, 4 * S->M, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return WP_OK;
}

wp_status wp_surrogate_fallback_coords(const wp_surrogate *S, double *u, double *v, double *w, void *stream) {
    if (!S) return wp_set_error(WP_EINVAL, "surrogate is NULL");
    if (S->Mf == 0) return WP_OK;
    if (!u || !v || !w) return wp_set_error(WP_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    WP_HIP(hipMemcpyAsync(u, S->fb, 8 * S->Mf, hipMemcpyDeviceToDevice, s));
    WP_HIP(hipMemcpyAsync(v, S->fb + S->Mf, 8 * S->Mf, hipMemcpyDeviceToDevice, s));
    WP_HIP(hipMemcpyAsync(w, S->fb + 2 * S->Mf, 8 * S->Mf, hipMemcpyDeviceToDevice, s));
    return WP_OK;
}

wp_status wp_surrogate_degrid(const wp_plan *p, const wp_surrogate *S, const void *grid, void *y, void *stream) {
    if (wp_status st = check_sur(p, S)) return st;
    if (!grid || (S->Ms > 0 && !y)) return wp_set_error(WP_EINVAL, "NULL argument");
    return sur_degrid(p, S, (const float2 *)grid, (float2 *)y, (hipStream_t)stream);
}

wp_status wp_surrogate_grid_add(const wp_plan *p, const wp_surrogate *S, const void *y, void *grid, void *stream) {
    if (wp_status st = check_sur(p, S)) return st;
    if (!grid || (S->Ms > 0 && !y)) return wp_set_error(WP_EINVAL, "NULL argument");
    return sur_grid_add(p, S, (const float2 *)y, (float2 *)grid, (hipStream_t)stream);
}

wp_status wp_surrogate_apply_Phi(const wp_plan *p, const wp_surrogate *S, const wp_G *Gf, const void *x, void *y,
                                 void *grid, void *stream) {
    if (wp_status st = check_sur(p, S)) return st;
    if (wp_status st = check_fallback(p, S, Gf)) return st;
    if (!x || !y || !grid) return wp_set_error(WP_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    wp_status st = launch_grid_forward(p, (const float2 *)x, (float2 *)grid, s);
    if (st != WP_OK) return st;
    if ((st = sur_degrid(p, S, (const float2 *)grid, (float2 *)y, s)) != WP_OK) return st;
    if (S->Mf > 0) return launch_degrid(p, Gf, (const float2 *)grid, (float2 *)y + S->Ms, s);
    return WP_OK;
}

wp_status wp_surrogate_apply_PhiT(const wp_plan *p, const wp_surrogate *S, const wp_G *Gf, const void *y, void *x,
                                  void *grid, void *stream) {
    if (wp_status st = check_sur(p, S)) return st;
    if (wp_status st = check_fallback(p, S, Gf)) return st;
    if (!x || !y || !grid) return wp_set_error(WP_EINVAL, "NULL argument");
    if (S->Mf > 0 && !Gf->tcolptr && (Gf->n_work > 0 && !Gf->work))
        return wp_set_error(WP_EINVAL, "fallback G needs its transposed copy or work items");
    hipStream_t s = (hipStream_t)stream;
    wp_status st;
    if (S->Mf > 0)
        st = Gf->tcolptr ? launch_gather(p, Gf, (const float2 *)y + S->Ms, (float2 *)grid, s)
                         : launch_scatter(p, Gf, (const float2 *)y + S->Ms, (float2 *)grid, s);
    else
        st = launch_fill_zero((float *)grid, 2 * (int64_t)p->Ng * p->Ng, s);
    if (st != WP_OK) return st;
    if ((st = sur_grid_add(p, S, (const float2 *)y, (float2 *)grid, s)) != WP_OK) return st;
    return launch_grid_adjoint(p, (float2 *)grid, (float2 *)x, s);
}

wp_status wp_surrogate_to_slots(const wp_surrogate *S, const wp_G *Gf, const void *in, void *out, void *stream) {
    if (!S) return wp_set_error(WP_EINVAL, "surrogate is NULL");
    if (wp_status st = check_fallback(nullptr, S, Gf)) return st;
    if (!in || !out || in == out) return wp_set_error(WP_EINVAL, "need distinct input and output vectors");
    const int *fperm = (S->Mf > 0 && Gf->order == WP_ORDER_SORTED) ? Gf->perm : nullptr;
    hipLaunchKernelGGL(k_to_slots, dim3((unsigned)((S->M + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       (const float2 *)in, S->slot_vis, S->Ms, S->M, fperm, (float2 *)out);
    return wp_check_launch("k_to_slots");
}

wp_status wp_surrogate_solver_workspace_bytes(const wp_plan *p, const wp_surrogate *S, int64_t *bytes) {
    if (wp_status st = check_sur(p, S)) return st;
    if (!bytes) return wp_set_error(WP_EINVAL, "bytes is NULL");
    *bytes = solver_workspace_bytes(p, S->M);
    return WP_OK;
}

wp_status wp_surrogate_power_norm2(const wp_plan *p, const wp_surrogate *S, const wp_G *Gf, const float *x0,
                                   int iters, void *workspace, double *nu_out, void *stream) {
    if (wp_status st = check_sur(p, S)) return st;
    if (wp_status st = check_fallback(p, S, Gf)) return st;
    if (!x0 || !workspace || !nu_out || iters < 1) return wp_set_error(WP_EINVAL, "bad argument");
    return launch_power_norm2(p, wp_operator{Gf, S, S->M}, x0, iters, nu_out, (unsigned char *)workspace,
                              (hipStream_t)stream);
}

wp_status wp_surrogate_solve(const wp_plan *p, const wp_surrogate *S, const wp_G *Gf, const void *y, double eps,
                             double nu, int iters, int levels, float *x, void *workspace, void *stream) {
    if (wp_status st = check_sur(p, S)) return st;
    if (wp_status st = check_fallback(p, S, Gf)) return st;
    if (!y || !x || !workspace || iters < 0 || !(nu > 0.0) || !(eps >= 0.0))
        return wp_set_error(WP_EINVAL, "bad argument");
    return launch_solve(p, wp_operator{Gf, S, S->M}, (const float2 *)y, eps, nu, iters, levels, x,
                        (unsigned char *)workspace, (hipStream_t)stream);
}

}  // extern "C"
