// Internal definitions shared by the HIP translation units of libwproj.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wproj.h"

// ---------------------------------------------------------------------------- plan

// largest padded grid the exact chirp's builder takes (its 2-D rows are made whole)
constexpr int EXACT_MAX_NG = 512;

struct wp_plan {
    int N;          // image side
    int Ng;         // padded grid side (2N)
    int logNg;
    int W;          // KB support (cells)
    int chirp;      // WP_CHIRP_*
    int aphys;      // WP_APHYS_*
    double L;       // planar field of view
    double beta;    // KB shape
    double delta;   // pixel size L / N
    double cell;    // uv cell 1 / (Ng delta) = 1 / (2L)
    double tap_bound;   // an upper bound on |G_kc| for every row the builder makes
    int tile;       // adjoint scatter: tile side in cells
    int halo;       // adjoint scatter: LDS window margin per side
    int ntile;      // tiles per axis
    int device;
    int tune_degrid_lpr, tune_degrid_u;   // 0: automatic (see spmv.hip)
    int tune_degrid_rows;                 // rows per wave of the degrid from factor records (0: automatic)
    int tune_gather_lpr, tune_gather_u;
    int tune_gather_chunk;                // entries per chunk of the blocked gather (256, 512, 1024)
    int gb_ent;                           // entries stretch of a gather block (see gather_table_slots)
    int solve_graph;                      // solver loop: 0 automatic (direct launches), 1 HIP graph, 2 direct
    int exact_rows;                       // exact chirp rows: 0 automatic, 1 separable expansion, 2 whole 2-D
    int sur_degrid;                       // surrogate degridding: 0 automatic (2), 1 register-staged, 2 LDS ring
    int sur_grid;                         // surrogate gridding: 0 automatic (2), 1 register-staged, 2 LDS ring
    int solve_streams;                    // solver loop with wavelets: 0 automatic (1), 1 one stream, 2 two streams
    hipStream_t aux_stream;               // the solver's second stream (made on first use, default priority)
    hipEvent_t aux_ev[3];                 // its events
    float *apod;    // [N]  1 / g(xi), xi = (p - N/2) / Ng       (device)
    float2 *tw32;   // [Ng] exp(-2 pi i k / Ng), FP32             (device)
    double2 *tw64;  // [Ng] exp(-2 pi i k / Ng), FP64             (device)
};

// ---------------------------------------------------------------------------- errors

wp_status wp_set_error(wp_status s, const char *fmt, ...);
wp_status wp_check_launch(const char *what);

#define WP_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return wp_set_error(WP_EHIP, "%s: %s", #call, hipGetErrorString(e_));      \
    } while (0)

// ---------------------------------------------------------------------------- complex helpers

__host__ __device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cmulc(float2 a, float2 b) {  // conj(a) * b
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
template <typename T2> __device__ inline T2 cconj(T2 a) { a.y = -a.y; return a; }
// multiply by -i (forward) or +i (inverse)
template <typename T2> __device__ inline T2 cmul_negi(T2 a) { T2 r; r.x = a.y; r.y = -a.x; return r; }
template <typename T2> __device__ inline T2 cmul_posi(T2 a) { T2 r; r.x = -a.y; r.y = a.x; return r; }

// bfloat16 pair (re in the low half) <-> float2
__host__ __device__ inline uint32_t bf16_bits_rne(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);  // inf / nan
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return u >> 16;
}
__host__ __device__ inline uint32_t pack_bf16x2(float re, float im) {
    return bf16_bits_rne(re) | (bf16_bits_rne(im) << 16);
}
__device__ inline float2 unpack_bf16x2(uint32_t p) {
    return make_float2(__uint_as_float(p << 16), __uint_as_float(p & 0xffff0000u));
}
// int16 pair (re in the low half), unscaled
__host__ __device__ inline uint32_t pack_i16x2(float re, float im) {
    const int a = (int)fminf(32767.f, fmaxf(-32767.f, rintf(re)));
    const int b = (int)fminf(32767.f, fmaxf(-32767.f, rintf(im)));
    return ((uint32_t)(uint16_t)(int16_t)a) | ((uint32_t)(uint16_t)(int16_t)b << 16);
}
__device__ inline float2 unpack_i16x2(uint32_t p) {
    return make_float2((float)(int16_t)(p & 0xffffu), (float)(int16_t)(p >> 16));
}
// raw tap value of kind TK (WP_TAPS_*); int16 taps come back unscaled
template <int TK>
__device__ __forceinline__ float2 load_tap_raw(const void *__restrict__ val, int64_t j) {
    if constexpr (TK == WP_TAPS_C64) return ((const float2 *)val)[j];
    else if constexpr (TK == WP_TAPS_BF16) return unpack_bf16x2(((const uint32_t *)val)[j]);
    else return unpack_i16x2(((const uint32_t *)val)[j]);
}

// ---------------------------------------------------------------------------- XCD-aware block order
// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8).
// This bijection gives each XCD a contiguous range of logical blocks, so the rows
// (sorted by uv tile) that share grid cells also share an L2.
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
    const int64_t X = 8;
    int64_t x = b % X, i = b / X, q = nb / X, r = nb % X;
    return x * q + (x < r ? x : r) + i;
}

// ---------------------------------------------------------------------------- Z-order

// Z-order (Morton) code of a cell: bits of u in the even positions, bits of v in the odd ones.
// Every aligned power-of-two block of cells is one contiguous range of codes.
__host__ __device__ inline int morton2(int v, int u) {
    int code = 0;
    for (int b = 0; b < 12; ++b) code |= (((u >> b) & 1) << (2 * b)) | (((v >> b) & 1) << (2 * b + 1));
    return code;
}
__host__ __device__ inline void demorton2(int code, int &v, int &u) {
    u = v = 0;
    for (int b = 0; b < 12; ++b) {
        u |= ((code >> (2 * b)) & 1) << b;
        v |= ((code >> (2 * b + 1)) & 1) << b;
    }
}

// ---------------------------------------------------------------------------- gather blocks
// The blocked gather walks the transposed copy in runs of consecutive grid cells: cell c starts
// a block when slot(c) = floor(tcolptr[c] / ent) + floor(c / GB_CELLS) differs from slot(c - 1)
// (ent: the plan's gb_ent, GB_ENT unless tuned).  Both terms are non-decreasing in c, so a block
// holds at most GB_CELLS cells whose entries start within one stretch of ent entries (its last
// cell may run past it), and there are at most gather_table_slots blocks.
constexpr int GB_ENT = 512;
constexpr int GB_CELLS = 64;
inline int64_t gather_table_slots(int64_t nnz, int64_t cells, int ent) { return nnz / ent + (cells - 1) / GB_CELLS + 1; }

// ---------------------------------------------------------------------------- factor records
// Separable form of a kept row: with the u candidates sorted by descending |g_u|^2 and the v
// candidates by descending |g_v|^2, candidate v cell i keeps the first nb[i] u candidates.
// Record: uint16 nu, nv; uint16 ua[nu], vb[nv], nb[nv]; zero padding to 8 bytes; complex
// float gu[nu], gv[nv].  Records start at multiples of 8 bytes.
__host__ __device__ inline int factor_record_bytes(int nu, int nv) {
    return ((4 + 2 * nu + 4 * nv + 7) & ~7) + 8 * (nu + nv);
}

// ---------------------------------------------------------------------------- launchers (host)

// FFT stages of A, Z, F and their adjoint (fft.hip)
// batch > 1: `batch` images / grids stored contiguously (N*N and Ng*Ng apart)
wp_status launch_grid_forward(const wp_plan *p, const float2 *x, float2 *grid, hipStream_t s, int batch = 1);
wp_status launch_grid_adjoint(const wp_plan *p, float2 *grid, float2 *x, hipStream_t s, int batch = 1);

// sparse products (spmv.hip)
wp_status launch_degrid(const wp_plan *p, const wp_G *G, const float2 *grid, float2 *y, hipStream_t s);
wp_status launch_scatter(const wp_plan *p, const wp_G *G, const float2 *y, float2 *grid, hipStream_t s);
wp_status launch_gather(const wp_plan *p, const wp_G *G, const float2 *y, float2 *grid, hipStream_t s);
wp_status launch_fill_zero(float *buf, int64_t n, hipStream_t s);
wp_status launch_permute(const wp_G *G, const float2 *in, float2 *out, bool to_sorted, hipStream_t s);

// builder (builder.hip)
// stable sort of n (key, index) pairs by the low `bits` bits of key: on return keys_out[i] is the
// i-th smallest key and idx_out[i] the input position it came from; ws: sort_workspace_bytes(n)
int64_t sort_workspace_bytes(int64_t n);
wp_status launch_sort_pairs(const int *key, int64_t n, int bits, int *keys_out, int *idx_out, void *ws,
                            hipStream_t s);
// exclusive scan of n ints into out[0..n] (out[n] = total); ws: scan_workspace_bytes(n)
int64_t scan_workspace_bytes(int64_t n);
wp_status launch_scan_int(const int *in, int *out, int64_t n, void *ws, hipStream_t s);
int64_t builder_workspace_bytes(const wp_plan *p, int64_t M, bool rows2d);
wp_status launch_build_factor_bytes(const wp_plan *p, int64_t M, void *ws, int64_t *bytes, hipStream_t s);
// beam: [M][3] (l0, m0, sigma) per visibility, or NULL; with a beam (or the exact chirp) rows are made in 2-D
wp_status launch_build_count(const wp_plan *p, int64_t M, const double *u, const double *v, const double *w,
                             const double *beam, double E, void *ws, int64_t *nnz_total, int64_t *nwork,
                             hipStream_t s);
wp_status launch_build_fill(const wp_plan *p, int64_t M, const double *u, const double *v, const double *w,
                            const double *beam, double E, const void *ws, wp_G *G, hipStream_t s);


// solver (solver.hip)
// The measurement operator the solver iterates with: the exact form (G) or the surrogate form
// (S, with G the exact rows of its fallback visibilities, NULL when there are none).
struct wp_operator {
    const wp_G *G;
    const wp_surrogate *S;
    int64_t M;
};
wp_status op_phi(const wp_plan *p, const wp_operator &op, const float2 *x, float2 *y, float2 *grid, hipStream_t s);
wp_status op_phiT(const wp_plan *p, const wp_operator &op, const float2 *y, float2 *x, float2 *grid, hipStream_t s);
int64_t solver_workspace_bytes(const wp_plan *p, int64_t M);
int64_t sara_workspace_bytes(const wp_plan *p, int64_t M);
int64_t dr_workspace_bytes(const wp_plan *p, int64_t M);
wp_status launch_dr_solve(const wp_plan *p, const wp_operator &op, const float2 *y, double eps, double nu, int iters,
                          int inner, double gamma, int levels, float *x, unsigned char *ws, hipStream_t s);
wp_status launch_sara_analysis(const wp_plan *p, int levels, const float *x, float *c, float *tmp, hipStream_t s);
wp_status launch_sara_synthesis(const wp_plan *p, int levels, const float *c, float *x, float *tmp, hipStream_t s);
wp_status launch_sara_solve(const wp_plan *p, const wp_operator &op, const float2 *y, double eps, double nu, int iters,
                            int rounds, int levels, float *x, unsigned char *ws, hipStream_t s);
wp_status launch_dwt2(const wp_plan *p, int levels, const float *x, float *c, float *tmp, bool synth, hipStream_t s);
wp_status launch_power_norm2(const wp_plan *p, const wp_operator &op, const float *x0, int iters, double *nu,
                             unsigned char *ws, hipStream_t s);
wp_status launch_solve(const wp_plan *p, const wp_operator &op, const float2 *y, double eps, double nu, int iters,
                       int levels, float *x, unsigned char *ws, hipStream_t s);
wp_status filter_db8(double *h);

// batch of problems (batch.hip)
wp_status batch_create(wp_batch **out, const wp_plan *p, int P, const wp_G *G);
void batch_destroy(wp_batch *b);
int64_t batch_total_vis(const wp_batch *b);
wp_status batch_phi(wp_batch *b, const float2 *x, float2 *y, float2 *grids, hipStream_t s);
wp_status batch_phiT(wp_batch *b, const float2 *y, float2 *x, float2 *grids, hipStream_t s);
wp_status batch_autotune(wp_batch *b, const float2 *x, float2 *y, float2 *grids, hipStream_t s, float *best_us);
void batch_set_mode(wp_batch *b, int deg, int gat, int *deg_out, int *gat_out);
void batch_shapes(const wp_batch *b, int *out6);
