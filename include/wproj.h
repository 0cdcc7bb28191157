/*
 * wproj.h -- C ABI of the sparse w-projection measurement operator for
 * AMD Instinct MI355X (gfx950).
 *
 * Operator (Wolz et al. 2013, Section 3, Eq. 8, generalised to continuous
 * (u, v) with a Kaiser-Bessel gridding window):
 *
 *     Phi   = G F Z A          y = Phi x          (visibilities from an image)
 *     Phi^H = A Z^H F^H G^H    x = Phi^H y        (adjoint, Section 3.1: solvers
 *                                                  need only Phi and its adjoint)
 *
 *   A    apodisation: a_phys(l, m) / (g(xi_l) g(xi_m)), g = FT of the KB window
 *   Z    zero-padding of the N x N image to the Ng x Ng grid, Ng = 2N (the
 *        upsampling U of Eq. 6, done in the image domain)
 *   F    centred, unnormalised 2-D DFT; F^H is the unnormalised inverse
 *   G    sparse matrix, one row per visibility (the mask M folded into the
 *        rows, Eq. 8): the visibility's KB taps convolved with the Fourier
 *        transform of its own w-chirp (Section 3.1), thresholded per row to
 *        keep a fraction E of the row energy (Section 3.2).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  - Pointers named "device" are HIP device memory owned by the caller; the
 *    library never frees them.  Host pointers are named so.
 *  - Complex values are interleaved float pairs (re, im) ("c64").
 *  - Images are N x N, row-major, indexed [m][l] (row along v / m, column
 *    along u / l); pixel p sits at (p - N/2) * L / N.
 *  - The uv grid is Ng x Ng row-major, flattened index q_v * Ng + q_u; cell q
 *    is at u = (q - Ng/2) / (2L) wavelengths.
 *  - Visibility coordinates u, v, w are float64, in wavelengths, in the
 *    caller's order.  Internally G's rows are sorted by uv tile; G.perm maps
 *    sorted row r to caller index perm[r].  Visibility vectors y are in the
 *    caller's order, or in the sorted row order when G.order is
 *    WP_ORDER_SORTED (an iterative solver keeps its vectors in that order:
 *    the sparse products then read and write y contiguously).
 *  - Every call is enqueued on the given HIP stream (NULL = default stream)
 *    and is asynchronous unless its comment says it synchronises.
 *  - No call throws or aborts.  Arguments are validated before any launch;
 *    on failure nothing is launched, a status < 0 is returned and
 *    wp_last_error() gives a message (thread-local).
 *  - N must be a power of two, 32 <= N <= 2048 (Ng <= 4096).
 */
#ifndef WPROJ_H
#define WPROJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum wp_status {
    WP_OK = 0,
    WP_EINVAL = -1,        /* bad argument (shape, range, NaN, null pointer)      */
    WP_ENOMEM = -2,        /* a library-owned table could not be allocated         */
    WP_EHIP = -3,          /* a HIP runtime call or kernel launch failed           */
    WP_ECAPACITY = -4,     /* a caller buffer or a count exceeds what is supported */
    WP_EUNSUPPORTED = -5   /* valid request this build does not implement          */
} wp_status;

enum { WP_CHIRP_LINEAR = 0,   /* exp(+i pi w (l^2+m^2)): first order of Eq. 4 (the paper's Eq. 5) */
       WP_CHIRP_EXACT = 1 };  /* exp(-2 pi i w (sqrt(1-l^2-m^2) - 1)) (Eq. 4)                    */
enum { WP_TAPS_C64 = 0,       /* G values as complex float32 (8 bytes)                          */
       WP_TAPS_BF16 = 1,      /* G values as a (re, im) pair of bfloat16 (4 bytes), FP32 accumulate */
       WP_TAPS_I16 = 2 };     /* G values as a (re, im) pair of int16 times the row's scale
                                 rscale[r] (block floating point: 4 bytes per tap + 4 per row)   */
enum { WP_APHYS_ONE = 0,      /* primary beam absorbed into the sky (Section 2.1)               */
       WP_APHYS_INV_N = 1 };  /* the 1/n(l, m) factor of Eq. 1                                 */
enum { WP_ORDER_CALLER = 0,   /* visibility vectors in the caller's order (default)             */
       WP_ORDER_SORTED = 1 }; /* visibility vectors in G's tile-sorted row order: entry r is
                                 visibility perm[r] (use wp_to_sorted / wp_to_caller once)     */

typedef struct wp_plan wp_plan;   /* opaque: geometry plus small device tables */

/* Sparse G in CSR form.  All arrays are caller-owned device memory. */
typedef struct wp_G {
    int64_t  M;        /* rows = visibilities                                        */
    int64_t  nnz;      /* stored taps                                                */
    int32_t  taps;     /* WP_TAPS_C64 or WP_TAPS_BF16                                */
    int32_t  order;    /* WP_ORDER_CALLER: y in caller order; WP_ORDER_SORTED: y[r] is row r */
    int64_t *rowptr;   /* [M+1] device, sorted-row order, rowptr[0] = 0              */
    int32_t *col;      /* [nnz] device, flattened grid index, ascending in a row    */
    void    *val;      /* [nnz] device, c64 or bf16 pairs.  col and val may both be NULL when the
                          factor records below are set (the factor-record form: no stored taps and
                          no transposed copy; Phi forms its taps from the records, the scatter
                          form of G^H too, and wp_build_G_fill then writes only the records) */
    int32_t *perm;     /* [M]   device, sorted row r is visibility perm[r]           */
    int32_t *work;     /* [4*n_work] device, adjoint work items (tile_v, tile_u, row_begin, row_end) */
    int64_t  n_work;
    float   *rscale;   /* [M] device, per sorted row scale of WP_TAPS_I16 values (else may be NULL):
                          tap = rscale[r] * (re, im), |re|, |im| <= 32767                      */
    /* Optional transposed copy for the gather form of G^H (tcolptr == NULL: not built).
     * Entries of grid cell c are [tcolptr[c], tcolptr[c+1]), ordered by sorted row index. */
    int64_t *tcolptr;  /* [Ng*Ng+1] device                                           */
    int32_t *trow;     /* [nnz] device, sorted row index r of the entry               */
    void    *tval;     /* [nnz] device, the entry's G value (not conjugated), same tap type */
    /* Optional block table of the transposed copy (tblk == NULL: the gather runs one lane
     * group per cell).  Blocks are runs of at most 64 consecutive cells whose entries start
     * within one stretch of 512 entries (the plan's gather_block_entries); block i is
     * (first cell, first entry) at
     * tblk[2i], tblk[2i+1], and the pair after the last block, and every later one up to
     * index n_tblk, is (Ng*Ng, nnz).  One wavefront sums one block.  n_tblk comes from
     * wp_gather_table_size; wp_build_G_fill writes the table with the transposed copy. */
    int64_t *tblk;     /* [2*(n_tblk+1)] device                                      */
    int64_t  n_tblk;
    /* Optional factor records (frec == NULL: the degrid reads the stored taps).  The linear
     * chirp and the KB window are separable, so row r is g_v(b) g_u(a) on the kept set
     * {|g_v(b)|^2 |g_u(a)|^2 >= tau_r} (Sections 3.1 and 3.2); with the u candidates ordered by
     * descending |g_u|^2 and the v candidates by descending |g_v|^2, v candidate i keeps the
     * first nb[i] u candidates.  Record of sorted row r at fdat + frec[r] (multiple of 8):
     * uint16 nu, nv; uint16 ua[nu] (u cells), vb[nv] (v cells), nb[nv]; zero padding to 8
     * bytes; complex float gu[nu], gv[nv].  The kept cells are exactly those of the stored
     * row; a tap is gv gu rounded to complex float before the product.  fbytes: size of
     * fdat from wp_build_factor_bytes.  Written by wp_build_G_fill. */
    int64_t *frec;     /* [M+1] device, byte offsets                                 */
    void    *fdat;     /* [fbytes] device                                            */
    int64_t  fbytes;
} wp_G;

/* Last error message of this thread ("" if none). */
const char *wp_last_error(void);

/* Library version string. */
const char *wp_version(void);

/*
 * Plan: geometry and small device tables (apodisation factors, FFT twiddles).
 *   N        image side (power of two, 32..2048); Ng = 2N
 *   fov_L    planar field of view L = 2 sin(theta/2) (Section 4.1), 0 < L < 1
 *   kb_W     KB support in grid cells, even, 2..16
 *   kb_beta  KB shape; <= 0 selects beta = pi sqrt((W/2)^2 (3/2)^2 - 0.8)
 *   chirp    WP_CHIRP_LINEAR or WP_CHIRP_EXACT
 *   aphys    WP_APHYS_ONE or WP_APHYS_INV_N
 * Allocates the tables on the current device; synchronises.
 */
wp_status wp_plan_create(wp_plan **out, int N, double fov_L, int kb_W, double kb_beta,
                         int chirp, int aphys);
wp_status wp_plan_destroy(wp_plan *plan);

/*
 * Launch-shape knobs of the sparse products, for the autotuner.  key is one of
 * "degrid_lanes", "degrid_unroll", "gather_lanes", "gather_unroll"; value 0
 * restores the automatic choice.  Lanes per row / cell: 4, 8, 16, 32 or 64;
 * loads in flight per lane: 4, 8 or 16 (not every pair exists: an apply with
 * an unavailable pair returns WP_EINVAL); the gather knobs apply to the form
 * without a block table.  "solve_graph": 1 replays the primal-dual loop of wp_solve from a captured
 * HIP graph, 0 (automatic) or 2 launches its kernels one by one.  "solve_streams": 2 runs the
 * wavelet analysis and most of the synthesis of each iteration on a second stream of the plan,
 * ordered by events, 0 (automatic) or 1 keeps one stream.  "exact_rows": how the exact chirp's
 * rows are made: 1 from the separable expansion at any Ng, 2 whole in 2-D (Ng <= 512), 0 automatic
 * (whole up to Ng = 512, the expansion above).  "gather_chunk": entries a wavefront of the blocked
 * gather stages at a time (256, 512, 768 or 1024); "gather_block_entries": the entry
 * stretch of a gather block (256, 384, 512 or 1024; it sets the block table that
 * wp_gather_table_size sizes and wp_build_G_fill writes, so change it only before
 * building G); "degrid_rows": rows per wavefront of
 * the degrid from factor records (1, 2 or 4).  "sur_degrid": the surrogate's
 * degridding (wp_surrogate_degrid and the apply calls): 1 stages each cell's box
 * through registers from the FP32 grid, 2 (the automatic choice) streams a
 * bfloat16 copy of the grid and the weights straight into a three-stage LDS
 * ring.  "sur_grid": the surrogate's gridding (wp_surrogate_grid_add and the
 * adjoint apply): 1 streams the weights from L2 into registers for groups of
 * <= 32 cells, 2 (the automatic choice) forms each cell's s once, then runs
 * groups of <= 128 cells in slices of 256 outputs through the LDS ring.  Not
 * thread-safe with concurrent applies on the same plan.
 */
wp_status wp_plan_set_tuning(wp_plan *plan, const char *key, int value);

/* Ng and the bytes of the Ng x Ng c64 grid workspace every apply needs. */
wp_status wp_plan_info(const wp_plan *plan, int64_t *Ng_out, int64_t *grid_bytes_out);

/* Bytes of the factor records of the visibilities counted by the last wp_build_G_count on
 * this workspace (same plan and M); also lays out the records' offsets in the workspace.
 * Call between wp_build_G_count and wp_build_G_fill when G->frec / G->fdat are wanted.
 * Synchronises the stream. */
wp_status wp_build_factor_bytes(const wp_plan *plan, int64_t M, void *workspace, int64_t *bytes_out,
                                void *stream);

/* n_tblk of a G with nnz taps: an upper bound on its number of gather blocks (the table
 * has 2*(n_tblk+1) int64 entries). */
wp_status wp_gather_table_size(const wp_plan *plan, int64_t nnz, int64_t *n_tblk_out);

/* Bytes of device workspace wp_build_G_count / wp_build_G_fill need for M visibilities. */
wp_status wp_build_workspace_bytes(const wp_plan *plan, int64_t M, int64_t *bytes_out);

/*
 * Build G, pass 1 of 2 (Section 3.1 kernel rows, Section 3.2 energy
 * threshold).  For each visibility: chirp of its w on the padded grid (FP64
 * phase), 1-D chirp spectrum, KB convolution, per-row threshold tau found by
 * bisection on the bit pattern of the row energies so that the kept entries
 * hold a fraction E of the row energy (ties kept; E >= 1 keeps every
 * non-zero entry); rows are then sorted by uv tile and their offsets
 * scanned.
 *   u, v, w    [M] device float64 in wavelengths; |u|, |v| < B = N/(2L), w finite
 *   E          preserved energy fraction, 0 < E <= 1
 *   workspace  device, wp_build_workspace_bytes(M) bytes, kept until pass 2
 *   nnz_out    host: total taps; n_work_out host: adjoint work items
 * Synchronises the stream (reads back two counts).
 * WP_CHIRP_EXACT (Eq. 4, not separable) needs 2 L^2 < 1 (the square root stays real over the
 * padded grid; else WP_EINVAL).  Up to Ng = 512 each row is made whole, a 2-D FP64 FFT of the
 * chirp on the Ng x Ng padded grid with the window's correlation per axis, in chunks of rows
 * held in the workspace (its tau search splits the bracket in 16 per pass over the row).  Above
 * Ng = 512 the chirp is the linear chirp times exp(i pi w s^2 / (1 + sqrt(1 - s))^2),
 * s = l^2 + m^2, whose interpolation at 8 Chebyshev points of l^2 makes each row a sum of 8 outer
 * products of 1-D rows (16 one-dimensional FP64 FFTs; expansion error below 1e-10 over the padded
 * grid); the row is formed on a window of at most 88 x 88 cells around its cell and thresholded
 * there, after checking that a bound on every entry outside the window lies below tau.  That form
 * needs E < 1 and rows spreading over at most 67 cells, 4 w L^2 / sqrt(1 - 2 L^2) <= 67 (else
 * WP_EUNSUPPORTED); a row whose outside bound reaches tau fails with WP_EHIP.
 */
wp_status wp_build_G_count(const wp_plan *plan, int64_t M, const double *u, const double *v,
                           const double *w, double E, void *workspace,
                           int64_t *nnz_out, int64_t *n_work_out, void *stream);

/*
 * Build G, pass 2 of 2: writes G->rowptr, G->perm, G->col, G->val, G->work,
 * and, when G->tcolptr is not NULL, the transposed copy (tcolptr, trow, tval) and,
 * when G->tblk is not NULL too, its block table (G->n_tblk must then equal
 * wp_gather_table_size's value, else WP_EINVAL); when G->frec and G->fdat are set, the
 * factor records (G->fbytes must equal wp_build_factor_bytes's value, else WP_EINVAL).
 * The caller sets G->M = M, G->nnz and G->n_work from pass 1, G->taps, and
 * points the arrays at buffers of the sizes listed in wp_G.  Same u, v, w, E
 * and workspace as pass 1 (pass 2 also uses part of it as scratch).  Synchronises the
 * stream at the end: pass 2 recomputes every row, and a row whose kept count (or factor
 * record) differs from pass 1's returns WP_EHIP.  Factor records are not made for the
 * exact chirp (WP_EUNSUPPORTED, also from wp_build_factor_bytes).
 */
wp_status wp_build_G_fill(const wp_plan *plan, int64_t M, const double *u, const double *v,
                          const double *w, double E, void *workspace, wp_G *G,
                          void *stream);

/*
 * Both build passes for a batch of P problems (the batched form's channels), problem p with its
 * own plan[p], M[p], u[p], v[p], w[p] (device float64), E[p] and workspace[p]
 * (wp_build_workspace_bytes(plan[p], M[p]) bytes).  Pass 1 writes nnz_out[p] and n_work_out[p]
 * (host arrays of P); pass 2 fills G[p] set up from them as for wp_build_G_fill.  The problems
 * are built one after another on `stream` (each pass-1 call synchronises it once); the first
 * failing problem stops the batch and its status is returned.
 */
wp_status wp_build_G_count_batch(int P, const wp_plan *const *plan, const int64_t *M,
                                 const double *const *u, const double *const *v,
                                 const double *const *w, const double *E, void *const *workspace,
                                 int64_t *nnz_out, int64_t *n_work_out, void *stream);
wp_status wp_build_G_fill_batch(int P, const wp_plan *const *plan, const int64_t *M,
                                const double *const *u, const double *const *v,
                                const double *const *w, const double *E, void *const *workspace,
                                wp_G *const *G, void *stream);

/*
 * y = Phi x  (Eq. 8 with the gridding window).
 *   x     [N*N] c64 device          y [M] c64 device (caller order)
 *   grid  device workspace of wp_plan_info's grid_bytes (contents overwritten)
 */
wp_status wp_apply_Phi(const wp_plan *plan, const wp_G *G, const void *x, void *y, void *grid,
                       void *stream);

/* y = Phi x like wp_apply_Phi, for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): no grid argument, and the call allocates
 * nothing.  Its grid workspace is a static device array of the library, one per GPU, of 2048 x 2048
 * complex floats (32 MiB, held until the process ends); plans with Ng > 2048 return WP_ECAPACITY.
 * The device of `stream` must be current.  Every call on a GPU uses that GPU's one array, so calls
 * that overlap on a GPU (other streams, other threads) race; serialise them.  Nothing carries over
 * between calls: the forward transform overwrites every cell the degrid reads. */
wp_status wp_apply_Phi_noalloc(const wp_plan *plan, const wp_G *G, const void *x, void *y, void *stream);

/* x = Phi^H y  (the adjoint; x is overwritten).  G^H y is the transposed-copy gather
 * when G->tcolptr is set, else the tiled scatter. */
wp_status wp_apply_PhiT(const wp_plan *plan, const wp_G *G, const void *y, void *x, void *grid,
                        void *stream);

/* Sub-steps of the two applies, exposed for testing and composition. */
/*
 * A direction-dependent effect through the same sparsifier (Section 3.2: the per-row energy
 * threshold assumes nothing about a row, so it applies to every direction-dependent effect, not
 * only to w).  Each visibility carries a Gaussian antenna power pattern with a pointing offset,
 * A_k(l, m) = exp(-((l - l0_k)^2 + (m - m0_k)^2) / (2 sigma_k^2)), multiplied into its
 * w-modulation (the plan's chirp) before the row's Fourier transform; rows are then made whole
 * in 2-D as for the exact chirp (Ng <= 512, else WP_EUNSUPPORTED).
 *   beam   [M][3] device float64 (l0, m0, sigma) in direction cosines; finite, sigma > 0
 * The other arguments, the two passes and their synchronisation are those of wp_build_G_count /
 * wp_build_G_fill; the workspace is wp_build_dde_workspace_bytes(M) bytes.  Factor records are
 * not made (WP_EUNSUPPORTED).  A visibility with an unusable beam fails pass 1 with WP_EINVAL.
 */
wp_status wp_build_dde_workspace_bytes(const wp_plan *plan, int64_t M, int64_t *bytes_out);
wp_status wp_build_G_dde_count(const wp_plan *plan, int64_t M, const double *u, const double *v,
                               const double *w, const double *beam, double E, void *workspace,
                               int64_t *nnz_out, int64_t *n_work_out, void *stream);
wp_status wp_build_G_dde_fill(const wp_plan *plan, int64_t M, const double *u, const double *v,
                              const double *w, const double *beam, double E, void *workspace,
                              wp_G *G, void *stream);

/* grid = F Z A x */
wp_status wp_grid_forward(const wp_plan *plan, const void *x, void *grid, void *stream);
/* x = A Z^H F^H grid  (grid is used as scratch and overwritten) */
wp_status wp_grid_adjoint(const wp_plan *plan, void *grid, void *x, void *stream);
/* y = G grid (degridding sparse matrix-vector product; from the factor records when
 * G->frec is set, taps formed in registers) */
wp_status wp_degrid(const wp_plan *plan, const wp_G *G, const void *grid, void *y, void *stream);
/* grid = G^H y (gridding: tile-binned scatter; each tile's window accumulates in LDS in 64-bit
 * fixed point scaled by a bound on its partial sums, then float atomics flush it and take the
 * entries beyond the window).  Without stored taps (G->val NULL) the taps come from the factor
 * records, each formed as the complex float product gv gu that the degrid forms (Section 3.1: the
 * separable kernel of the linear chirp, regenerated in registers).  The bound assumes taps the builder made: |G_kc| <= (W I0(beta))^2
 * (int16 taps: 46341 times the row scale); larger taps in a hand-made G can overflow the window. */
wp_status wp_grid_scatter(const wp_plan *plan, const wp_G *G, const void *y, void *grid,
                          void *stream);
/* grid = G^H y from the transposed copy (no atomics, deterministic); needs G->tcolptr.
 * With G->tblk and fewer than 512 entries per cell on average, one wavefront per block
 * of cells; else one lane group per cell. */
wp_status wp_grid_gather(const wp_plan *plan, const wp_G *G, const void *y, void *grid,
                         void *stream);

/* Reorder a c64 visibility vector between the caller's order and G's sorted row
 * order: sorted[r] = caller[perm[r]] (wp_to_sorted) and its inverse (wp_to_caller).
 * Out-of-place; [M] device each. */
wp_status wp_to_sorted(const wp_G *G, const void *caller, void *sorted, void *stream);
wp_status wp_to_caller(const wp_G *G, const void *sorted, void *caller, void *stream);

/* ----------------------------------------------------------------------------------------
 * Batches of independent problems sharing one plan (e.g. frequency channels, each with its
 * own visibilities and G).  Images are stored contiguously (problem p at x + p*N*N), grids
 * likewise (p*Ng*Ng), visibilities concatenated in problem order (problem p starts at the sum
 * of the earlier M).  Each sparse product is ONE persistent launch whose workgroups take
 * (problem, chunk) work items from a device queue; the FFTs are one launch pair for all.
 * ------------------------------------------------------------------------------------- */
typedef struct wp_batch wp_batch;

/* Bind P >= 1 problems (array of P wp_G; same tap type; the arrays stay caller-owned and must
 * outlive the batch).  The adjoint needs every G's transposed copy.  Allocates small device
 * tables (descriptors, work lists, one counter); synchronises. */
wp_status wp_batch_create(wp_batch **out, const wp_plan *plan, int P, const wp_G *G);
wp_status wp_batch_destroy(wp_batch *batch);
/* Total visibilities and the current launch shapes: [degrid lanes, unroll, rows per item,
 * gather lanes, unroll, cells per item]. */
wp_status wp_batch_info(const wp_batch *batch, int64_t *M_total, int *shapes6);
/* y = Phi_p x_p for every problem; x: P*N*N c64, y: M_total c64, grids: P*Ng*Ng c64 workspace.
 * Launches on one batch object must not run concurrently (they share the work counter). */
wp_status wp_apply_Phi_batch(wp_batch *batch, const void *x, void *y, void *grids, void *stream);
wp_status wp_apply_PhiT_batch(wp_batch *batch, const void *y, void *x, void *grids, void *stream);
/* Autotuner: times the candidate launch shapes of both persistent products on these buffers
 * (HIP events, 5 timed launches each) and keeps the fastest, then times the kept shape launched
 * flat (one workgroup per item, no work counter) and keeps that if faster; best_us2[0..1]
 * receive the kept times (host).  Synchronises; overwrites y and grids. */
wp_status wp_batch_autotune(wp_batch *batch, const void *x, void *y, void *grids, void *stream,
                            float *best_us2);
/* Launch mode of the two products: 0 = persistent (the ticket queue; the default), 1 = flat (one
 * workgroup per item).  *_out (host, may be NULL) receive the modes in force; a value < 0 keeps the
 * current mode. */
wp_status wp_batch_mode(wp_batch *batch, int degrid, int gather, int *degrid_out, int *gather_out);

/* ----------------------------------------------------------------------------------------
 * Learned surrogate of the rows of G.  A row (Section 3.1 kernel, Section 3.2 energy rule)
 * depends on the visibility only through w and the offset (du, dv) = (u~, v~) - c of its grid
 * coordinate from the nearest cell c = floor(u~ + 1/2): the row of u~ = c + du is the row of
 * du shifted by c.  The surrogate network maps the features
 *     f = (2 w / w_top - 1, 2 du, 2 dv)
 * through an MLP 3 -> 256 -> 256 -> 256 -> 2048 with GELU (x Phi(x), error-function form)
 * after the hidden layers, to the taps of the 32 x 32 box of cells (c_v - 16 .. c_v + 15) x
 * (c_u - 16 .. c_u + 15) (mod Ng): output 2p (2p + 1) is s_out times the real (imaginary)
 * part of box cell p = 32 oy + ox.  Parameters are packed in FP32 (wp_mlp_param_count()
 * floats) in the order W1 [256][3], b1 [256], W2 [256][256], b2, W3 [256][256], b3,
 * W4 [2048][256], b4 [2048], row-major, W_l mapping layer l-1 to layer l.
 * Products W_l a_{l-1} (l = 2..4) and the backward products take bfloat16 operands with FP32
 * accumulation on MFMA; the first layer, biases, GELU, loss, bias / W1 gradients and Adam are
 * FP32.  Training loss: mean over the 2048 outputs of (o - t)^2, t = exact taps / s_out.
 * The object owns its parameters, Adam moments and activation buffers for up to max_batch
 * rows; calls on one object must not overlap.
 * ------------------------------------------------------------------------------------- */
typedef struct wp_mlp wp_mlp;

/* Number of FP32 parameters (658944). */
int64_t wp_mlp_param_count(void);
/* Allocate a network with activation buffers for max_batch rows (multiple of 64, <= 2^20);
 * parameters start at zero.  Synchronous. */
wp_status wp_mlp_create(wp_mlp **out, int max_batch);
wp_status wp_mlp_destroy(wp_mlp *mlp);
/* Copy the packed parameters from HOST memory, set the feature scale w_top (> 0) and the
 * output scale s_out (> 0), and reset Adam (step 0, zero moments).  Synchronous. */
wp_status wp_mlp_set_params(wp_mlp *mlp, const float *params_host, double w_top, double s_out);
/* Copy the packed parameters to HOST memory; w_top / s_out may be NULL.  Synchronous. */
wp_status wp_mlp_get_params(const wp_mlp *mlp, float *params_host, double *w_top, double *s_out);
/* feat[3k..3k+2] = f of visibility k (device float32 [3n]) from u, v, w (device float64 [n]);
 * a non-finite coordinate or |u~|, |v~| >= Ng/2 sets bit 0 of *err (device int, caller
 * zeroes it). */
wp_status wp_mlp_features(const wp_plan *plan, const wp_mlp *mlp, int64_t n, const double *u,
                          const double *v, const double *w, float *feat, int *err, void *stream);
/* out[n][2048] = network outputs (device float32) of feat[n][3]; 0 <= n <= max_batch. */
wp_status wp_mlp_forward(wp_mlp *mlp, int n, const float *feat, float *out, void *stream);
/* Gradients of the loss for targets target[n][2048] (device float32, exact taps / s_out):
 * copied to grads (device float32 [param_count], may be NULL); *loss (host, may be NULL)
 * receives the loss, which synchronises the stream.  n: multiple of 64 in [64, max_batch]. */
wp_status wp_mlp_gradients(wp_mlp *mlp, int n, const float *feat, const float *target,
                           float *grads, double *loss, void *stream);
/* One Adam step (Kingma & Ba 2015, bias-corrected) with the gradients of the last
 * wp_mlp_gradients or training step. */
wp_status wp_mlp_adam_step(wp_mlp *mlp, float lr, float beta1, float beta2, float eps,
                           void *stream);
/* Train on n samples (feat [n][3], target [n][2048], device) for `epochs` passes of
 * floor(n / batch) minibatches; each pass visits the samples in the order (a i + c) mod n
 * with a coprime to n, changing per pass.  Adam (0.9, 0.999, 1e-8); learning rate
 * lr_max * min(1, t / warm) * (1 + cos(pi t / T)) / 2 over T steps, warm = T / 32.
 * loss_hist (HOST, may be NULL) receives each pass's mean loss, which synchronises once per
 * pass. */
wp_status wp_mlp_train(wp_mlp *mlp, int64_t n, const float *feat, const float *target, int batch,
                       int epochs, float lr_max, double *loss_hist, void *stream);
/* Output scale for training: s_out = sqrt(T0 / 1024), T0 the energy of the row of a visibility
 * on a cell centre, (sum over its KB window cells of KB^2)^2 (shifted chirp spectra are
 * orthonormal, so a row's energy depends only on its window weights).  Host result. */
wp_status wp_mlp_output_scale(const wp_plan *plan, double *s_out);
/* Training targets from exact rows: G (complex64 taps, built by wp_build_G_* from u, v of the
 * samples) scattered into each visibility's box and divided by s_out: target[k][2048]
 * (device float32, caller order k; cells of the box outside the row are 0), lost[k] = row
 * energy outside the box / row energy (device float32). */
wp_status wp_mlp_box_targets(const wp_plan *plan, const wp_G *G, const double *u, const double *v,
                             double s_out, float *target, float *lost, void *stream);
/* Per-row energy error of the surrogate against exact rows G (complex64 taps):
 * eps[k] = ||t_k - g_k||^2 / ||g_k||^2 (device float32 [G->M], caller order), t_k the network's
 * box taps for feat[k] (device float32 [3 G->M]), row entries outside the box counting in full.
 * Runs the network in chunks of max_batch rows (overwrites its activation buffers). */
wp_status wp_mlp_row_errors(const wp_plan *plan, wp_mlp *mlp, const wp_G *G, const double *u,
                            const double *v, const float *feat, float *eps, void *stream);

/* Run-time per-row check without exact rows (the energy rule of Section 3.2 applied to the
 * network's rows).  The check lattice holds nodes over (w, du, dv): node i = (iw nd + iv) nd + iu at
 * w = w_top iw / (nw - 1) (w_top: the network's feature scale) and du = -1/2 + iu / (nd - 1) cells
 * from the grid's centre cell (dv likewise; the last offset node sits 2^-20 cells below +1/2, so it
 * keeps the centre cell).  nw, nd >= 2, at most 2^26 nodes.
 * wp_mlp_lattice_coords writes the nodes' u, v, w (device float64 [nw nd nd] each, wavelengths).
 * wp_mlp_check_table takes G, the exact complex64 rows of those nodes (built from those
 * coordinates, caller order = node order), and the nodes' features, and writes table (device
 * float32 [2 nw nd nd]): table[i] = the network's row error ||t_i - g_i||^2 / ||g_i||^2 at node i
 * (as wp_mlp_row_errors) and table[nw nd nd + i] = the node's kept energy ||g_i||^2.
 * wp_mlp_row_check estimates the error of n network rows from the table alone, with no exact row:
 * est[k] = max(the largest node error of the lattice cell holding row k's (w, du, dv),
 * (| ||t_k|| - sqrt(K_k) | / sqrt(K_k))^2) with K_k the kept energy interpolated trilinearly
 * between the cell's nodes (the second term bounds the error from below when K_k is the row's
 * kept energy, by the reverse triangle inequality); +infinity outside the lattice (w beyond the
 * trained range), not a number if a node error is.  feat: device float32 [3n] (wp_mlp_features),
 * est: device float32 [n], both in the caller's order.  Runs the network in chunks of max_batch rows
 * (overwrites its activation buffers).  Rows with est > tol then fall back (wp_surrogate_create). */
wp_status wp_mlp_lattice_coords(const wp_plan *plan, const wp_mlp *mlp, int nw, int nd, double *u, double *v,
                                double *w, void *stream);
wp_status wp_mlp_check_table(const wp_plan *plan, wp_mlp *mlp, const wp_G *G, int nw, int nd, const double *u,
                             const double *v, const float *feat, float *table, void *stream);
wp_status wp_mlp_row_check(const wp_plan *plan, wp_mlp *mlp, int nw, int nd, const float *table, int64_t n,
                           const float *feat, float *est, void *stream);

/* ----------------------------------------------------------------------------------------
 * Surrogate operator.  Rows of visibilities whose per-row energy error (wp_mlp_row_errors)
 * is at most tol come from the surrogate network; the others ("fallback") from an exact G
 * the caller builds for them.  The network's taps are linear in its last hidden layer, so
 * the output layer is applied per occupied grid cell instead of per visibility: degridding
 * computes r_c = (W4 box of X) for every occupied nearest cell c and y_k = s_out (h_k . r_c
 * + b4 . box), gridding computes s_c = sum over the cell's visibilities of h_k y_k and adds
 * s_out (W4^H s_c + conj(b4) sum y_k) onto the cell's box; both are bfloat16 MFMA products
 * with FP32 accumulation.  The hidden layers h_k run once, in wp_surrogate_create; the taps
 * are never stored.
 * Visibility order ("slots"): slots [0, Ms) are the surrogate rows sorted by the Z-order code
 * of their nearest cell; slots [Ms, M) the fallback rows, in the order of the coordinates
 * that wp_surrogate_fallback_coords returns.  The fallback G must be built from exactly those
 * coordinates; its own G.order then decides the order within [Ms, M).
 * The object holds the products' workspaces (the degridding's bfloat16 grid copy, the
 * gridding's per-cell sums): its applies on different streams that overlap in time race on
 * them, so use one object per stream (calls in order on one stream are safe).
 * ------------------------------------------------------------------------------------- */
typedef struct wp_surrogate wp_surrogate;

/* Set up the surrogate operator for M visibilities (u, v, w: device float64, caller order):
 * features, the network's hidden layers (in chunks of mlp's max_batch, overwriting its
 * activation buffers), the cell tables and the output-layer matrices (a snapshot of the
 * network's current parameters).  eps (device float32 [M], caller order, may be NULL: no
 * fallback) are the per-row energy errors; rows with eps > tol or eps not a number fall back.
 * *Mf_out (host, may be NULL) receives the number of fallback rows.  Allocates device
 * memory owned by the object (512 B per surrogate row for its hidden layer, 1040 B per
 * occupied cell for the gridding's per-cell sums and 1 KB more, Ng (Ng + 32) 4 B for the
 * degridding's bfloat16 grid copy, 6 MB of weights); synchronises. */
wp_status wp_surrogate_create(wp_surrogate **out, const wp_plan *plan, wp_mlp *mlp, int64_t M,
                              const double *u, const double *v, const double *w, const float *eps,
                              double tol, int64_t *Mf_out, void *stream);
wp_status wp_surrogate_destroy(wp_surrogate *sur);
/* info5 (host): M, Ms (surrogate rows), Mf (fallback rows), occupied cells,
 * (degridding groups << 32) | groups of the register-staged gridding. */
wp_status wp_surrogate_info(const wp_surrogate *sur, int64_t *info5);
/* slot_vis[r] = caller index of slot r (device int32 [M]). */
wp_status wp_surrogate_slots(const wp_surrogate *sur, int *slot_vis, void *stream);
/* Coordinates of the fallback rows in slot order (device float64 [Mf] each). */
wp_status wp_surrogate_fallback_coords(const wp_surrogate *sur, double *u, double *v, double *w,
                                       void *stream);
/* y[0, Ms) = surrogate rows times the grid (device c64 Ng*Ng); y[Ms, M) untouched. */
wp_status wp_surrogate_degrid(const wp_plan *plan, const wp_surrogate *sur, const void *grid,
                              void *y, void *stream);
/* grid += surrogate rows^H y[0, Ms) (atomic adds; the grid must hold its other terms first). */
wp_status wp_surrogate_grid_add(const wp_plan *plan, const wp_surrogate *sur, const void *y,
                                void *grid, void *stream);
/* y = Phi_s x (slot order) and x = Phi_s^H y, with Gf the exact G of the Mf fallback rows (NULL
 * if Mf = 0; its adjoint needs the transposed copy or the work items).  x: N*N c64, y: M c64,
 * grid: Ng*Ng c64 workspace (all device). */
wp_status wp_surrogate_apply_Phi(const wp_plan *plan, const wp_surrogate *sur, const wp_G *Gf,
                                 const void *x, void *y, void *grid, void *stream);
wp_status wp_surrogate_apply_PhiT(const wp_plan *plan, const wp_surrogate *sur, const wp_G *Gf,
                                  const void *y, void *x, void *grid, void *stream);

/* out[r] = in[caller index of slot r] (device c64 [M], distinct buffers): a caller-order
 * visibility vector in slot order; slots [Ms, M) follow Gf's order (Gf->perm when
 * Gf->order is WP_ORDER_SORTED). */
wp_status wp_surrogate_to_slots(const wp_surrogate *sur, const wp_G *Gf, const void *in, void *out,
                                void *stream);
/* The solver entry points below with the surrogate operator (y in slot order). */
wp_status wp_surrogate_solver_workspace_bytes(const wp_plan *plan, const wp_surrogate *sur,
                                              int64_t *bytes_out);
wp_status wp_surrogate_power_norm2(const wp_plan *plan, const wp_surrogate *sur, const wp_G *Gf,
                                   const float *x0, int iters, void *workspace, double *nu_out,
                                   void *stream);
wp_status wp_surrogate_solve(const wp_plan *plan, const wp_surrogate *sur, const wp_G *Gf,
                             const void *y, double eps, double nu, int iters, int levels, float *x,
                             void *workspace, void *stream);

/* ----------------------------------------------------------------------------------------
 * Reconstruction (Eq. 7): min ||Psi^T x||_1 s.t. ||y - Phi x||_2 <= eps, x >= 0, with Psi the
 * Daubechies wavelets of 8 vanishing moments (Section 4.2), periodic, `levels` levels, or with
 * levels = 0 the Dirac (pixel) basis Psi = I, Section 4.2's other dictionary (Section 2.3: maximally
 * incoherent with the Fourier basis).
 * ------------------------------------------------------------------------------------- */

/* The 16 low-pass taps of Daubechies-8 (spectral factorisation, minimum phase, sum sqrt 2); host. */
wp_status wp_db8_filter(double *h16);

/* c = Psi^T x (analysis) and x = Psi c (synthesis) of a real N x N float image; x and c may
 * alias; scratch is N*N floats of device memory.  levels = 0 (Dirac basis: a copy) or levels >= 1
 * with N >> (levels-1) >= 8; other values return WP_EINVAL. */
wp_status wp_dwt2(const wp_plan *plan, int levels, const float *x, float *c, float *scratch,
                  void *stream);
wp_status wp_idwt2(const wp_plan *plan, int levels, const float *c, float *x, float *scratch,
                   void *stream);

/* Device workspace of wp_power_norm2 and wp_solve for this plan and G. */
wp_status wp_solver_workspace_bytes(const wp_plan *plan, const wp_G *G, int64_t *bytes_out);

/* ||Phi||^2 by power iteration on Re Phi^H Phi from the real image x0 (device, N*N floats):
 * iters steps; the result is written to *nu_out (host).  Synchronises the stream. */
wp_status wp_power_norm2(const wp_plan *plan, const wp_G *G, const float *x0, int iters,
                         void *workspace, double *nu_out, void *stream);

/* Primal-dual solve (Condat / Vu splitting with dual variables for the l1 term and the
 * l2 ball): tau = 0.49, sigma_1 = 1, sigma_2 = 1 / nu.  x (device, real N*N floats) holds
 * the start on entry and the estimate on exit; y is c64 [M] in G's visibility order
 * (G->order); eps is the ball radius, nu = ||Phi||^2.  Dual variables start at zero.
 * Asynchronous: the iterations' kernels are enqueued one by one.  With the plan's tuning key
 * "solve_graph" = 1 and 20 iterations or more, chunks of 10 iterations are instead captured once into
 * a HIP graph (on a private stream) and replayed on `stream`, and the call then synchronises the
 * stream before it returns (the graph is released). */
wp_status wp_solve(const wp_plan *plan, const wp_G *G, const void *y, double eps, double nu,
                   int iters, int levels, float *x, void *workspace, void *stream);

/* Douglas-Rachford splitting (Section 2.3) for Eq. 7 as printed: min ||Psi^T x||_1 subject to
 * ||y - Phi x||_2 <= eps, x real, without the positivity wp_solve adds; Psi is Daubechies 8 with
 * `levels` levels, or the Dirac basis for levels = 0.  From z = 0, each of `iters` iterations sets
 * x = P_C(z), the projection onto the constraint, then z = z + Psi soft_gamma(Psi^T (2x - z)) - x
 * (soft threshold gamma >= 0).  Phi is not a tight frame, so P_C runs `inner` (>= 1) steps of
 * forward-backward on its dual, warm-started from the previous iteration's dual, each one Phi
 * and one Phi^H with step 1 / nu (nu = ||Phi||^2).  x (device, real N*N floats) receives the last
 * projection.  Asynchronous. */
wp_status wp_dr_workspace_bytes(const wp_plan *plan, const wp_G *G, int64_t *bytes_out);
wp_status wp_dr_solve(const wp_plan *plan, const wp_G *G, const void *y, double eps, double nu,
                      int iters, int inner, double gamma, int levels, float *x, void *workspace,
                      void *stream);

/* ----------------------------------------------------------------------------------------
 * SARA (Section 4.2's third dictionary; the paper cites Carrillo, McEwen & Wiaux 2012 for it):
 * Psi = [I, W_1, ..., W_8] / 3, W_p the periodic Daubechies wavelets with p vanishing moments
 * (`levels` levels, 1 <= levels, N >> (levels-1) >= 8), a tight frame (Psi Psi^T = I), and
 * reweighted l1 analysis.
 * ------------------------------------------------------------------------------------- */

/* c = Psi^T x: x is a real N x N float image, c is [9][N][N] floats (Dirac part first); scratch is
 * 16 N^2 floats of device memory.  x and c must not overlap. */
wp_status wp_sara_analysis(const wp_plan *plan, int levels, const float *x, float *c, float *scratch,
                           void *stream);
/* x = Psi c, same layouts and scratch; c and x must not overlap. */
wp_status wp_sara_synthesis(const wp_plan *plan, int levels, const float *c, float *x, float *scratch,
                            void *stream);

/* Device workspace of wp_sara_solve for this plan and G. */
wp_status wp_sara_workspace_bytes(const wp_plan *plan, const wp_G *G, int64_t *bytes_out);

/* Reweighted analysis solve: `rounds` (>= 1) runs of the wp_solve iteration (same splitting and
 * step sizes, ||Psi|| = 1) with the weighted norm ||W Psi^T x||_1, the dual step clipping
 * coefficient i to [-w_i, w_i].  Round 0 has unit weights; before round r >= 1 the weights are
 * w_i = delta / (delta + |(Psi^T x)_i|) with x the current estimate, delta = the standard
 * deviation of Psi^T x before round 1 and a tenth of the previous delta afterwards.  x (device,
 * real N*N floats) holds the start on entry and the estimate on exit and carries over between
 * rounds; the dual variables restart at zero each round.  Synchronises the stream once per
 * round from round 1 on (it reads back the coefficients' spread). */
wp_status wp_sara_solve(const wp_plan *plan, const wp_G *G, const void *y, double eps, double nu,
                        int iters, int rounds, int levels, float *x, void *workspace, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* WPROJ_H */
