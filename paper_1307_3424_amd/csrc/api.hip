// C ABI entry points: validation, plan tables, dispatch to the kernels.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "common.h"

namespace {
thread_local char g_err[512] = "";

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2(int x) {
    int r = 0;
    while ((1 << r) < x) ++r;
    return r;
}

// KB window Fourier transform, W sinh(sqrt(beta^2 - (pi W xi)^2)) / sqrt(...)
double kb_transform(double xi, int W, double beta) {
    const double z = beta * beta - (M_PI * W * xi) * (M_PI * W * xi);
    if (z > 0) {
        const double s = std::sqrt(z);
        return W * std::sinh(s) / s;
    }
    if (z < 0) {
        const double s = std::sqrt(-z);
        return W * std::sin(s) / s;
    }
    return W;
}

// I0 by its power series sum_k ((x/2)^2)^k / (k!)^2
static double bessel_i0_host(double x) {
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 500 && term > 1e-17 * sum; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
    }
    return sum;
}

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

wp_status check_plan(const wp_plan *p) {
    if (!p) return wp_set_error(WP_EINVAL, "plan is NULL");
    return WP_OK;
}

wp_status check_G(const wp_plan *p, const wp_G *G, bool need_work) {
    if (!G) return wp_set_error(WP_EINVAL, "G is NULL");
    if (G->M < 0 || G->M > 0x7fffffff) return wp_set_error(WP_EINVAL, "G->M = %lld out of range", (long long)G->M);
    if (G->nnz < 0) return wp_set_error(WP_EINVAL, "G->nnz < 0");
    if (G->taps != WP_TAPS_C64 && G->taps != WP_TAPS_BF16 && G->taps != WP_TAPS_I16)
        return wp_set_error(WP_EINVAL, "G->taps = %d", G->taps);
    if (G->taps == WP_TAPS_I16 && G->M > 0 && !G->rscale) return wp_set_error(WP_EINVAL, "WP_TAPS_I16 needs G->rscale");
    if (G->order != WP_ORDER_CALLER && G->order != WP_ORDER_SORTED) return wp_set_error(WP_EINVAL, "G->order = %d", G->order);
    if (G->M > 0 && (!G->rowptr || !G->perm)) return wp_set_error(WP_EINVAL, "G has a NULL array");
    // no stored taps (col and val both NULL) is the factor-record form: it needs the records
    if (G->nnz > 0 && (!G->col || !G->val) && !(!G->col && !G->val && G->frec && G->fdat))
        return wp_set_error(WP_EINVAL, "G has a NULL array (col / val may be NULL together only with factor records)");
    if (!G->val && G->tcolptr) return wp_set_error(WP_EINVAL, "the transposed copy needs the stored taps");
    if (need_work && G->n_work > 0 && !G->work) return wp_set_error(WP_EINVAL, "G->work is NULL");
    if (need_work && G->n_work > 0x7fffffff) return wp_set_error(WP_ECAPACITY, "G->n_work too large");
    if (G->tcolptr && G->nnz > 0 && (!G->trow || !G->tval))
        return wp_set_error(WP_EINVAL, "G->tcolptr set without trow / tval");
    if (G->tblk && !G->tcolptr) return wp_set_error(WP_EINVAL, "G->tblk set without the transposed copy");
    if ((G->frec == nullptr) != (G->fdat == nullptr)) return wp_set_error(WP_EINVAL, "G->frec and G->fdat go together");
    if (G->tblk && p) {
        const int64_t want = gather_table_slots(G->nnz, (int64_t)p->Ng * p->Ng, p->gb_ent);
        if (G->n_tblk != want)
            return wp_set_error(WP_EINVAL, "G->n_tblk = %lld, expected %lld", (long long)G->n_tblk, (long long)want);
    }
    return WP_OK;
}
}  // namespace

wp_status wp_set_error(wp_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

wp_status wp_check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wp_set_error(WP_EHIP, "%s: %s", what, hipGetErrorString(e));
    return WP_OK;
}

extern "C" {

const char *wp_last_error(void) { return g_err; }

const char *wp_version(void) { return "wproj 0.1 gfx950"; }

wp_status wp_plan_create(wp_plan **out, int N, double fov_L, int kb_W, double kb_beta, int chirp, int aphys) {
    if (!out) return wp_set_error(WP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!is_pow2(N) || N < 32 || N > 2048) return wp_set_error(WP_EINVAL, "N = %d: need a power of two in [32, 2048]", N);
    if (!(fov_L > 0.0 && fov_L < 1.0)) return wp_set_error(WP_EINVAL, "fov_L = %g: need 0 < L < 1", fov_L);
    if (kb_W < 2 || kb_W > 16 || (kb_W & 1)) return wp_set_error(WP_EINVAL, "kb_W = %d: need an even value in [2, 16]", kb_W);
    if (chirp != WP_CHIRP_LINEAR && chirp != WP_CHIRP_EXACT) return wp_set_error(WP_EINVAL, "chirp = %d", chirp);
    if (aphys != WP_APHYS_ONE && aphys != WP_APHYS_INV_N) return wp_set_error(WP_EINVAL, "aphys = %d", aphys);
    if (!std::isfinite(kb_beta)) return wp_set_error(WP_EINVAL, "kb_beta is not finite");
    wp_plan *p = new (std::nothrow) wp_plan();
    if (!p) return wp_set_error(WP_ENOMEM, "plan allocation");
    p->N = N;
    p->Ng = 2 * N;
    p->gb_ent = GB_ENT;
    p->logNg = ilog2(p->Ng);
    p->W = kb_W;
    p->chirp = chirp;
    p->aphys = aphys;
    p->L = fov_L;
    p->beta = kb_beta > 0 ? kb_beta : M_PI * std::sqrt((kb_W / 2.0) * (kb_W / 2.0) * 1.5 * 1.5 - 0.8);
    p->delta = fov_L / N;
    p->cell = 1.0 / (p->Ng * p->delta);
    // |tap| <= (sum of one axis' W window weights)^2 <= (W I0(beta))^2: each 1-D chirp spectrum value
    // has modulus at most 1 (and a beam at most 1), the window weights peak at I0(beta)
    p->tap_bound = (kb_W * bessel_i0_host(p->beta)) * (kb_W * bessel_i0_host(p->beta));
    p->tile = 32;
    p->halo = 16;
    p->ntile = p->Ng / p->tile;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return wp_set_error(WP_EHIP, "hipGetDevice failed");
    }
    // tables, computed in FP64 on the host
    const int Ng = p->Ng;
    float *apod = (float *)std::malloc(sizeof(float) * N);
    float2 *tw32 = (float2 *)std::malloc(sizeof(float2) * Ng);
    double2 *tw64 = (double2 *)std::malloc(sizeof(double2) * Ng);
    if (!apod || !tw32 || !tw64) {
        std::free(apod); std::free(tw32); std::free(tw64);
        delete p;
        return wp_set_error(WP_ENOMEM, "plan tables");
    }
    for (int i = 0; i < N; ++i) apod[i] = (float)(1.0 / kb_transform((i - N / 2) / (double)Ng, kb_W, p->beta));
    for (int k = 0; k < Ng; ++k) {
        // exp(-2 pi i k / Ng), argument reduced through the exact ratio k / Ng
        const double a = 2.0 * M_PI * (double)k / (double)Ng;
        tw64[k] = make_double2(std::cos(a), -std::sin(a));
        tw32[k] = make_float2((float)tw64[k].x, (float)tw64[k].y);
    }
    hipError_t e = hipMalloc(&p->apod, sizeof(float) * N);
    if (e == hipSuccess) e = hipMalloc(&p->tw32, sizeof(float2) * Ng);
    if (e == hipSuccess) e = hipMalloc(&p->tw64, sizeof(double2) * Ng);
    if (e == hipSuccess) e = hipMemcpy(p->apod, apod, sizeof(float) * N, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->tw32, tw32, sizeof(float2) * Ng, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->tw64, tw64, sizeof(double2) * Ng, hipMemcpyHostToDevice);
    std::free(apod); std::free(tw32); std::free(tw64);
    if (e != hipSuccess) {
        wp_plan_destroy(p);
        return wp_set_error(e == hipErrorOutOfMemory ? WP_ENOMEM : WP_EHIP, "plan tables: %s", hipGetErrorString(e));
    }
    *out = p;
    return WP_OK;
}

wp_status wp_plan_destroy(wp_plan *p) {
    if (!p) return WP_OK;
    if (p->aux_stream) {
        (void)hipStreamSynchronize(p->aux_stream);
        (void)hipStreamDestroy(p->aux_stream);
        for (hipEvent_t e : p->aux_ev)
            if (e) (void)hipEventDestroy(e);
    }
    if (p->apod) (void)hipFree(p->apod);
    if (p->tw32) (void)hipFree(p->tw32);
    if (p->tw64) (void)hipFree(p->tw64);
    delete p;
    return WP_OK;
}

wp_status wp_plan_set_tuning(wp_plan *p, const char *key, int value) {
    if (wp_status s = check_plan(p)) return s;
    if (!key) return wp_set_error(WP_EINVAL, "key is NULL");
    if (!std::strcmp(key, "gather_block_entries")) {
        if (value != 0 && value != 256 && value != 384 && value != 512 && value != 1024)
            return wp_set_error(WP_EINVAL, "gather_block_entries %d: 0, 256, 384, 512 or 1024", value);
        p->gb_ent = value > 0 ? value : GB_ENT;
        return WP_OK;
    }
    if (!std::strcmp(key, "gather_chunk")) {
        if (value != 0 && value != 256 && value != 512 && value != 768 && value != 1024)
            return wp_set_error(WP_EINVAL, "gather_chunk %d: 0, 256, 512, 768 or 1024", value);
        p->tune_gather_chunk = value;
        return WP_OK;
    }
    if (!std::strcmp(key, "sur_grid")) {
        if (value < 0 || value > 2) return wp_set_error(WP_EINVAL, "sur_grid %d: 0, 1 or 2", value);
        p->sur_grid = value;
        return WP_OK;
    }
    if (!std::strcmp(key, "sur_degrid")) {
        if (value < 0 || value > 2) return wp_set_error(WP_EINVAL, "sur_degrid %d: 0, 1 or 2", value);
        p->sur_degrid = value;
        return WP_OK;
    }
    if (!std::strcmp(key, "exact_rows")) {
        if (value < 0 || value > 2) return wp_set_error(WP_EINVAL, "exact_rows %d: 0, 1 or 2", value);
        p->exact_rows = value;
        return WP_OK;
    }
    if (!std::strcmp(key, "solve_streams")) {
        if (value < 0 || value > 2) return wp_set_error(WP_EINVAL, "solve_streams %d: 0, 1 or 2", value);
        p->solve_streams = value;
        return WP_OK;
    }
    if (!std::strcmp(key, "solve_graph")) {
        if (value < 0 || value > 2) return wp_set_error(WP_EINVAL, "solve_graph %d: 0, 1 or 2", value);
        p->solve_graph = value;
        return WP_OK;
    }
    if (!std::strcmp(key, "degrid_rows")) {
        if (value != 0 && value != 1 && value != 2 && value != 4)
            return wp_set_error(WP_EINVAL, "degrid_rows %d: 0, 1, 2 or 4", value);
        p->tune_degrid_rows = value;
        return WP_OK;
    }
    if (value < 0 || value > 64) return wp_set_error(WP_EINVAL, "tuning value %d out of range", value);
    if (!std::strcmp(key, "degrid_lanes")) p->tune_degrid_lpr = value;
    else if (!std::strcmp(key, "degrid_unroll")) p->tune_degrid_u = value;
    else if (!std::strcmp(key, "gather_lanes")) p->tune_gather_lpr = value;
    else if (!std::strcmp(key, "gather_unroll")) p->tune_gather_u = value;
    else return wp_set_error(WP_EINVAL, "unknown tuning key '%s'", key);
    return WP_OK;
}

wp_status wp_plan_info(const wp_plan *p, int64_t *Ng_out, int64_t *grid_bytes_out) {
    if (wp_status s = check_plan(p)) return s;
    if (Ng_out) *Ng_out = p->Ng;
    if (grid_bytes_out) *grid_bytes_out = (int64_t)p->Ng * p->Ng * 8;
    return WP_OK;
}

wp_status wp_build_factor_bytes(const wp_plan *p, int64_t M, void *workspace, int64_t *bytes, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (p->chirp == WP_CHIRP_EXACT)
        return wp_set_error(WP_EUNSUPPORTED, "build: the exact chirp's rows are not separable (no factor records)");
    if (!workspace || !bytes) return wp_set_error(WP_EINVAL, "workspace or bytes_out is NULL");
    if (M < 1 || M > 0x7fffffff) return wp_set_error(WP_EINVAL, "M = %lld out of range", (long long)M);
    return launch_build_factor_bytes(p, M, workspace, bytes, as_stream(stream));
}

wp_status wp_gather_table_size(const wp_plan *p, int64_t nnz, int64_t *n) {
    if (wp_status s = check_plan(p)) return s;
    if (!n) return wp_set_error(WP_EINVAL, "n_tblk_out is NULL");
    if (nnz < 0) return wp_set_error(WP_EINVAL, "nnz < 0");
    *n = gather_table_slots(nnz, (int64_t)p->Ng * p->Ng, p->gb_ent);
    return WP_OK;
}

// the exact chirp: whole 2-D rows up to Ng = EXACT_MAX_NG, the separable expansion above (or when the
// plan asks for it; never with a beam), which keeps a window of the row and so needs E < 1; and
// sqrt(1 - l^2 - m^2) real over the padded grid (its corner sits at l = m = -L)
static wp_status check_exact(const wp_plan *p, double E, bool beam = false) {
    if (p->chirp != WP_CHIRP_EXACT) return WP_OK;
    const bool lowrank = !beam && (p->exact_rows == 1 || (p->exact_rows == 0 && p->Ng > EXACT_MAX_NG));
    if (!lowrank && p->Ng > EXACT_MAX_NG)
        return wp_set_error(WP_EUNSUPPORTED, "build: whole 2-D rows of the exact chirp need Ng <= %d (Ng = %d)",
                            EXACT_MAX_NG, p->Ng);
    if (lowrank && !(E < 1.0))
        return wp_set_error(WP_EUNSUPPORTED, "build: the exact chirp's separable expansion keeps a window of each "
                            "row and needs E < 1 (E = %g)", E);
    if (!(2.0 * p->L * p->L < 1.0))
        return wp_set_error(WP_EINVAL, "build: the exact chirp needs 2 L^2 < 1 (L = %g)", p->L);
    return WP_OK;
}

wp_status wp_build_workspace_bytes(const wp_plan *p, int64_t M, int64_t *bytes) {
    if (wp_status s = check_plan(p)) return s;
    if (!bytes) return wp_set_error(WP_EINVAL, "bytes_out is NULL");
    if (M < 1 || M > 0x7fffffff) return wp_set_error(WP_EINVAL, "M = %lld out of range", (long long)M);
    *bytes = builder_workspace_bytes(p, M, p->chirp == WP_CHIRP_EXACT);
    return WP_OK;
}

wp_status wp_build_G_count(const wp_plan *p, int64_t M, const double *u, const double *v, const double *w, double E,
                           void *ws, int64_t *nnz_out, int64_t *n_work_out, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (M < 1 || M > 0x7fffffff) return wp_set_error(WP_EINVAL, "M = %lld out of range", (long long)M);
    if (!u || !v || !w || !ws || !nnz_out || !n_work_out) return wp_set_error(WP_EINVAL, "NULL argument");
    if (!(E > 0.0 && E <= 1.0)) return wp_set_error(WP_EINVAL, "E = %g: need 0 < E <= 1", E);
    if (wp_status s = check_exact(p, E)) return s;
    return launch_build_count(p, M, u, v, w, nullptr, E, ws, nnz_out, n_work_out, as_stream(stream));
}

wp_status wp_build_G_fill(const wp_plan *p, int64_t M, const double *u, const double *v, const double *w, double E,
                          void *ws, wp_G *G, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (M < 1 || M > 0x7fffffff) return wp_set_error(WP_EINVAL, "M = %lld out of range", (long long)M);
    if (!u || !v || !w || !ws) return wp_set_error(WP_EINVAL, "NULL argument");
    if (!(E > 0.0 && E <= 1.0)) return wp_set_error(WP_EINVAL, "E = %g: need 0 < E <= 1", E);
    if (wp_status s = check_exact(p, E)) return s;
    if (wp_status s = check_G(p, G, true)) return s;
    if (p->chirp == WP_CHIRP_EXACT && (G->frec || G->fdat))
        return wp_set_error(WP_EUNSUPPORTED, "build: the exact chirp's rows are not separable (no factor records)");
    if (G->M != M) return wp_set_error(WP_EINVAL, "G->M = %lld differs from M = %lld", (long long)G->M, (long long)M);
    return launch_build_fill(p, M, u, v, w, nullptr, E, ws, G, as_stream(stream));
}

wp_status wp_build_G_count_batch(int P, const wp_plan *const *plan, const int64_t *M, const double *const *u,
                                 const double *const *v, const double *const *w, const double *E,
                                 void *const *workspace, int64_t *nnz_out, int64_t *n_work_out, void *stream) {
    if (P < 1) return wp_set_error(WP_EINVAL, "P = %d", P);
    if (!plan || !M || !u || !v || !w || !E || !workspace || !nnz_out || !n_work_out)
        return wp_set_error(WP_EINVAL, "NULL argument");
    for (int p = 0; p < P; ++p)
        if (wp_status st = wp_build_G_count(plan[p], M[p], u[p], v[p], w[p], E[p], workspace[p], nnz_out + p,
                                            n_work_out + p, stream))
            return st;
    return WP_OK;
}

wp_status wp_build_G_fill_batch(int P, const wp_plan *const *plan, const int64_t *M, const double *const *u,
                                const double *const *v, const double *const *w, const double *E,
                                void *const *workspace, wp_G *const *G, void *stream) {
    if (P < 1) return wp_set_error(WP_EINVAL, "P = %d", P);
    if (!plan || !M || !u || !v || !w || !E || !workspace || !G) return wp_set_error(WP_EINVAL, "NULL argument");
    for (int p = 0; p < P; ++p)
        if (wp_status st = wp_build_G_fill(plan[p], M[p], u[p], v[p], w[p], E[p], workspace[p], G[p], stream))
            return st;
    return WP_OK;
}

wp_status wp_build_dde_workspace_bytes(const wp_plan *p, int64_t M, int64_t *bytes) {
    if (wp_status s = check_plan(p)) return s;
    if (!bytes) return wp_set_error(WP_EINVAL, "bytes_out is NULL");
    if (M < 1 || M > 0x7fffffff) return wp_set_error(WP_EINVAL, "M = %lld out of range", (long long)M);
    *bytes = builder_workspace_bytes(p, M, true);
    return WP_OK;
}

wp_status wp_build_G_dde_count(const wp_plan *p, int64_t M, const double *u, const double *v, const double *w,
                               const double *beam, double E, void *ws, int64_t *nnz_out, int64_t *n_work_out,
                               void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (M < 1 || M > 0x7fffffff) return wp_set_error(WP_EINVAL, "M = %lld out of range", (long long)M);
    if (!u || !v || !w || !beam || !ws || !nnz_out || !n_work_out) return wp_set_error(WP_EINVAL, "NULL argument");
    if (!(E > 0.0 && E <= 1.0)) return wp_set_error(WP_EINVAL, "E = %g: need 0 < E <= 1", E);
    if (wp_status s = check_exact(p, E, true)) return s;
    if (p->Ng > EXACT_MAX_NG)
        return wp_set_error(WP_EUNSUPPORTED, "build: 2-D rows need Ng <= %d (Ng = %d)", EXACT_MAX_NG, p->Ng);
    return launch_build_count(p, M, u, v, w, beam, E, ws, nnz_out, n_work_out, as_stream(stream));
}

wp_status wp_build_G_dde_fill(const wp_plan *p, int64_t M, const double *u, const double *v, const double *w,
                              const double *beam, double E, void *ws, wp_G *G, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (M < 1 || M > 0x7fffffff) return wp_set_error(WP_EINVAL, "M = %lld out of range", (long long)M);
    if (!u || !v || !w || !beam || !ws) return wp_set_error(WP_EINVAL, "NULL argument");
    if (!(E > 0.0 && E <= 1.0)) return wp_set_error(WP_EINVAL, "E = %g: need 0 < E <= 1", E);
    if (wp_status s = check_exact(p, E, true)) return s;
    if (p->Ng > EXACT_MAX_NG)
        return wp_set_error(WP_EUNSUPPORTED, "build: 2-D rows need Ng <= %d (Ng = %d)", EXACT_MAX_NG, p->Ng);
    if (wp_status s = check_G(p, G, true)) return s;
    if (G->M != M) return wp_set_error(WP_EINVAL, "G->M = %lld differs from M = %lld", (long long)G->M, (long long)M);
    if (G->frec || G->fdat)
        return wp_set_error(WP_EUNSUPPORTED, "build: rows with a beam are made in 2-D (no factor records)");
    return launch_build_fill(p, M, u, v, w, beam, E, ws, G, as_stream(stream));
}

wp_status wp_grid_forward(const wp_plan *p, const void *x, void *grid, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (!x || !grid) return wp_set_error(WP_EINVAL, "NULL argument");
    return launch_grid_forward(p, (const float2 *)x, (float2 *)grid, as_stream(stream));
}

wp_status wp_grid_adjoint(const wp_plan *p, void *grid, void *x, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (!x || !grid) return wp_set_error(WP_EINVAL, "NULL argument");
    return launch_grid_adjoint(p, (float2 *)grid, (float2 *)x, as_stream(stream));
}

wp_status wp_degrid(const wp_plan *p, const wp_G *G, const void *grid, void *y, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (wp_status s = check_G(p, G, false)) return s;
    if (!grid || (G->M > 0 && !y)) return wp_set_error(WP_EINVAL, "NULL argument");
    return launch_degrid(p, G, (const float2 *)grid, (float2 *)y, as_stream(stream));
}

wp_status wp_grid_scatter(const wp_plan *p, const wp_G *G, const void *y, void *grid, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (wp_status s = check_G(p, G, true)) return s;
    if (!grid || (G->M > 0 && !y)) return wp_set_error(WP_EINVAL, "NULL argument");
    return launch_scatter(p, G, (const float2 *)y, (float2 *)grid, as_stream(stream));
}

wp_status wp_apply_Phi(const wp_plan *p, const wp_G *G, const void *x, void *y, void *grid, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (wp_status s = check_G(p, G, false)) return s;
    if (!x || !grid || (G->M > 0 && !y)) return wp_set_error(WP_EINVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    if (wp_status st = launch_grid_forward(p, (const float2 *)x, (float2 *)grid, s)) return st;
    return launch_degrid(p, G, (const float2 *)grid, (float2 *)y, s);
}

}  // extern "C"

// Grid workspace of wp_apply_Phi_noalloc: a file-scope device array, one copy per GPU, held until the
// process ends.  Host code never passes `scratch` itself (in host code the name is only a stand-in
// for the symbol); it looks up each device's address once, with that device current, and passes that.
namespace {
constexpr int64_t NOALLOC_MAX_CELLS = (int64_t)2048 * 2048;     // Ng <= 2048: 32 MiB of complex float
constexpr int NOALLOC_MAX_DEVICES = 64;
__device__ __align__(256) float2 scratch[NOALLOC_MAX_CELLS];
std::mutex g_scratch_mu;
float2 *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

wp_status scratch_grid(float2 **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return wp_set_error(WP_EHIP, "wp_apply_Phi_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return wp_set_error(WP_EUNSUPPORTED, "wp_apply_Phi_noalloc: device %d beyond the %d supported", dev,
                            NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return wp_set_error(WP_EHIP, "wp_apply_Phi_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (float2 *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return WP_OK;
}
}  // namespace

extern "C" {

wp_status wp_apply_Phi_noalloc(const wp_plan *p, const wp_G *G, const void *x, void *y, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (wp_status s = check_G(p, G, false)) return s;
    if (!x || (G->M > 0 && !y)) return wp_set_error(WP_EINVAL, "NULL argument");
    if ((int64_t)p->Ng * p->Ng > NOALLOC_MAX_CELLS)
        return wp_set_error(WP_ECAPACITY, "wp_apply_Phi_noalloc: Ng = %d exceeds the static grid of %lld cells "
                            "(Ng <= 2048); use wp_apply_Phi with a caller grid", p->Ng, (long long)NOALLOC_MAX_CELLS);
    float2 *grid = nullptr;
    if (wp_status st = scratch_grid(&grid)) return st;
    hipStream_t s = as_stream(stream);
    // the forward transform writes every cell of the grid: nothing left by an earlier call is read
    if (wp_status st = launch_grid_forward(p, (const float2 *)x, grid, s)) return st;
    return launch_degrid(p, G, grid, (float2 *)y, s);
}

wp_status wp_grid_gather(const wp_plan *p, const wp_G *G, const void *y, void *grid, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (wp_status s = check_G(p, G, false)) return s;
    if (!G->tcolptr) return wp_set_error(WP_EINVAL, "wp_grid_gather: G has no transposed copy");
    if (!grid || (G->M > 0 && !y)) return wp_set_error(WP_EINVAL, "NULL argument");
    return launch_gather(p, G, (const float2 *)y, (float2 *)grid, as_stream(stream));
}

wp_status wp_to_sorted(const wp_G *G, const void *caller, void *sorted, void *stream) {
    if (wp_status s = check_G(nullptr, G, false)) return s;
    if (G->M > 0 && (!caller || !sorted)) return wp_set_error(WP_EINVAL, "NULL argument");
    if (caller == sorted && G->M > 0) return wp_set_error(WP_EINVAL, "wp_to_sorted is out-of-place");
    return launch_permute(G, (const float2 *)caller, (float2 *)sorted, true, as_stream(stream));
}

wp_status wp_to_caller(const wp_G *G, const void *sorted, void *caller, void *stream) {
    if (wp_status s = check_G(nullptr, G, false)) return s;
    if (G->M > 0 && (!caller || !sorted)) return wp_set_error(WP_EINVAL, "NULL argument");
    if (caller == sorted && G->M > 0) return wp_set_error(WP_EINVAL, "wp_to_caller is out-of-place");
    return launch_permute(G, (const float2 *)sorted, (float2 *)caller, false, as_stream(stream));
}

wp_status wp_apply_PhiT(const wp_plan *p, const wp_G *G, const void *y, void *x, void *grid, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (wp_status s = check_G(p, G, !G || !G->tcolptr)) return s;
    if (!x || !grid || (G->M > 0 && !y)) return wp_set_error(WP_EINVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    wp_status st = G->tcolptr ? launch_gather(p, G, (const float2 *)y, (float2 *)grid, s)
                              : launch_scatter(p, G, (const float2 *)y, (float2 *)grid, s);
    if (st != WP_OK) return st;
    return launch_grid_adjoint(p, (float2 *)grid, (float2 *)x, s);
}

wp_status wp_batch_create(wp_batch **out, const wp_plan *p, int P, const wp_G *G) {
    if (!out) return wp_set_error(WP_EINVAL, "out is NULL");
    *out = nullptr;
    if (wp_status s = check_plan(p)) return s;
    if (P < 1 || !G) return wp_set_error(WP_EINVAL, "batch: P = %d, G = %p", P, (const void *)G);
    for (int i = 0; i < P; ++i)
        if (wp_status s = check_G(p, &G[i], false)) return s;
    return batch_create(out, p, P, G);
}

wp_status wp_batch_destroy(wp_batch *b) {
    batch_destroy(b);
    return WP_OK;
}

wp_status wp_batch_info(const wp_batch *b, int64_t *M_total, int *shapes6) {
    if (!b) return wp_set_error(WP_EINVAL, "batch is NULL");
    if (M_total) *M_total = batch_total_vis(b);
    if (shapes6) batch_shapes(b, shapes6);
    return WP_OK;
}

wp_status wp_apply_Phi_batch(wp_batch *b, const void *x, void *y, void *grids, void *stream) {
    if (!b) return wp_set_error(WP_EINVAL, "batch is NULL");
    if (!x || !y || !grids) return wp_set_error(WP_EINVAL, "NULL argument");
    return batch_phi(b, (const float2 *)x, (float2 *)y, (float2 *)grids, as_stream(stream));
}

wp_status wp_apply_PhiT_batch(wp_batch *b, const void *y, void *x, void *grids, void *stream) {
    if (!b) return wp_set_error(WP_EINVAL, "batch is NULL");
    if (!x || !y || !grids) return wp_set_error(WP_EINVAL, "NULL argument");
    return batch_phiT(b, (const float2 *)y, (float2 *)x, (float2 *)grids, as_stream(stream));
}

wp_status wp_batch_autotune(wp_batch *b, const void *x, void *y, void *grids, void *stream, float *best_us2) {
    if (!b) return wp_set_error(WP_EINVAL, "batch is NULL");
    if (!x || !y || !grids || !best_us2) return wp_set_error(WP_EINVAL, "NULL argument");
    return batch_autotune(b, (const float2 *)x, (float2 *)y, (float2 *)grids, as_stream(stream), best_us2);
}

wp_status wp_batch_mode(wp_batch *b, int degrid, int gather, int *degrid_out, int *gather_out) {
    if (!b) return wp_set_error(WP_EINVAL, "batch is NULL");
    if (degrid > 1 || gather > 1) return wp_set_error(WP_EINVAL, "mode %d / %d: 0, 1 or < 0", degrid, gather);
    batch_set_mode(b, degrid, gather, degrid_out, gather_out);
    return WP_OK;
}

wp_status wp_db8_filter(double *h16) {
    if (!h16) return wp_set_error(WP_EINVAL, "NULL argument");
    return filter_db8(h16);
}

wp_status wp_dwt2(const wp_plan *p, int levels, const float *x, float *c, float *scratch, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (!x || !c || !scratch) return wp_set_error(WP_EINVAL, "NULL argument");
    return launch_dwt2(p, levels, x, c, scratch, false, as_stream(stream));
}

wp_status wp_idwt2(const wp_plan *p, int levels, const float *c, float *x, float *scratch, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (!x || !c || !scratch) return wp_set_error(WP_EINVAL, "NULL argument");
    return launch_dwt2(p, levels, c, x, scratch, true, as_stream(stream));
}

wp_status wp_solver_workspace_bytes(const wp_plan *p, const wp_G *G, int64_t *bytes) {
    if (wp_status s = check_plan(p)) return s;
    if (wp_status s = check_G(p, G, !G || !G->tcolptr)) return s;
    if (!bytes) return wp_set_error(WP_EINVAL, "NULL argument");
    *bytes = solver_workspace_bytes(p, G->M);
    return WP_OK;
}

wp_status wp_power_norm2(const wp_plan *p, const wp_G *G, const float *x0, int iters, void *workspace,
                         double *nu_out, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (wp_status s = check_G(p, G, !G || !G->tcolptr)) return s;
    if (!x0 || !workspace || !nu_out) return wp_set_error(WP_EINVAL, "NULL argument");
    if (iters < 1) return wp_set_error(WP_EINVAL, "iters = %d", iters);
    return launch_power_norm2(p, wp_operator{G, nullptr, G->M}, x0, iters, nu_out, (unsigned char *)workspace,
                              as_stream(stream));
}

wp_status wp_solve(const wp_plan *p, const wp_G *G, const void *y, double eps, double nu, int iters, int levels,
                   float *x, void *workspace, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (wp_status s = check_G(p, G, !G || !G->tcolptr)) return s;
    if (!y || !x || !workspace) return wp_set_error(WP_EINVAL, "NULL argument");
    if (!(eps >= 0.0) || !(nu > 0.0) || !std::isfinite(eps) || !std::isfinite(nu))
        return wp_set_error(WP_EINVAL, "eps = %g, nu = %g: need eps >= 0 and nu > 0, finite", eps, nu);
    if (iters < 0) return wp_set_error(WP_EINVAL, "iters = %d", iters);
    return launch_solve(p, wp_operator{G, nullptr, G->M}, (const float2 *)y, eps, nu, iters, levels, x,
                        (unsigned char *)workspace,
                        as_stream(stream));
}

wp_status wp_sara_analysis(const wp_plan *p, int levels, const float *x, float *c, float *scratch, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (!x || !c || !scratch) return wp_set_error(WP_EINVAL, "NULL argument");
    return launch_sara_analysis(p, levels, x, c, scratch, as_stream(stream));
}

wp_status wp_sara_synthesis(const wp_plan *p, int levels, const float *c, float *x, float *scratch, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (!x || !c || !scratch) return wp_set_error(WP_EINVAL, "NULL argument");
    return launch_sara_synthesis(p, levels, c, x, scratch, as_stream(stream));
}

wp_status wp_sara_workspace_bytes(const wp_plan *p, const wp_G *G, int64_t *bytes) {
    if (wp_status s = check_plan(p)) return s;
    if (wp_status s = check_G(p, G, !G || !G->tcolptr)) return s;
    if (!bytes) return wp_set_error(WP_EINVAL, "NULL argument");
    *bytes = sara_workspace_bytes(p, G->M);
    return WP_OK;
}

wp_status wp_sara_solve(const wp_plan *p, const wp_G *G, const void *y, double eps, double nu, int iters, int rounds,
                        int levels, float *x, void *workspace, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (wp_status s = check_G(p, G, !G || !G->tcolptr)) return s;
    if (!y || !x || !workspace) return wp_set_error(WP_EINVAL, "NULL argument");
    if (!(eps >= 0.0) || !(nu > 0.0) || !std::isfinite(eps) || !std::isfinite(nu))
        return wp_set_error(WP_EINVAL, "eps = %g, nu = %g: need eps >= 0 and nu > 0, finite", eps, nu);
    if (iters < 0 || rounds < 1) return wp_set_error(WP_EINVAL, "iters = %d, rounds = %d", iters, rounds);
    return launch_sara_solve(p, wp_operator{G, nullptr, G->M}, (const float2 *)y, eps, nu, iters, rounds, levels, x,
                             (unsigned char *)workspace, as_stream(stream));
}

wp_status wp_dr_workspace_bytes(const wp_plan *p, const wp_G *G, int64_t *bytes) {
    if (wp_status s = check_plan(p)) return s;
    if (wp_status s = check_G(p, G, !G || !G->tcolptr)) return s;
    if (!bytes) return wp_set_error(WP_EINVAL, "NULL argument");
    *bytes = dr_workspace_bytes(p, G->M);
    return WP_OK;
}

wp_status wp_dr_solve(const wp_plan *p, const wp_G *G, const void *y, double eps, double nu, int iters, int inner,
                      double gamma, int levels, float *x, void *workspace, void *stream) {
    if (wp_status s = check_plan(p)) return s;
    if (wp_status s = check_G(p, G, !G || !G->tcolptr)) return s;
    if (!y || !x || !workspace) return wp_set_error(WP_EINVAL, "NULL argument");
    if (!(eps >= 0.0) || !(nu > 0.0) || !std::isfinite(eps) || !std::isfinite(nu))
        return wp_set_error(WP_EINVAL, "eps = %g, nu = %g: need eps >= 0 and nu > 0, finite", eps, nu);
    if (!(gamma >= 0.0) || !std::isfinite(gamma)) return wp_set_error(WP_EINVAL, "gamma = %g", gamma);
    if (iters < 0 || inner < 1) return wp_set_error(WP_EINVAL, "iters = %d, inner = %d", iters, inner);
    return launch_dr_solve(p, wp_operator{G, nullptr, G->M}, (const float2 *)y, eps, nu, iters, inner, gamma, levels,
                           x, (unsigned char *)workspace, as_stream(stream));
}

}  // extern "C"
