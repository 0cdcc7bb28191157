// Batch of independent problems sharing one plan (e.g. frequency channels): the
// forward / inverse FFTs run as one launch pair over all images, and each sparse
// product runs as ONE persistent launch whose workgroups pull work items
// (problem, chunk of rows) or (problem, chunk of grid cells) from a device work
// counter until the queue is empty, which balances problems of very uneven size.
//
// The work counter is never reset: it only grows, and each launch receives the
// counter value it starts from (`base`).  A workgroup asks for its next ticket as soon
// as it has read the current one (the atomic's latency overlaps the item's work), so
// it takes two tickets more than it has items and a launch takes exactly
// n_items + 2 nblocks tickets: the host knows the next base without reading the
// counter back and needs no reset launch.
//
// The same kernels also run "flat": one workgroup per item (blockIdx.x), the hardware
// dispatcher balancing the items, no counter.  wp_batch_autotune times both and keeps the
// faster per product, with the launch shapes (rows or cells per item, lanes per row or cell,
// loads in flight), every candidate timed with HIP events.
#include <algorithm>
#include <new>
#include <vector>

#include "gather_block.h"

namespace {

constexpr int BT = 256;

struct ProbDesc {
    const int64_t *rowptr;
    const int *col;
    const void *val;
    const int *perm;       // nullptr: visibilities in sorted row order
    const int64_t *tcolptr;
    const int *trow;
    const void *tval;
    const float *rscale;
    const int64_t *tblk;   // block table of the transposed copy (nullptr: none)
    int64_t n_tblk;
    int64_t M;
    int64_t y_off;
};

// The workgroup's current item; thread 0 keeps the ticket of the following one in `ahead` (asked for
// here, used on the next call).  Start with ahead = first_ticket(...).
__device__ __forceinline__ long long first_ticket(unsigned long long *counter, unsigned long long base) {
    return threadIdx.x == 0 ? (long long)(atomicAdd(counter, 1ull) - base) : 0;
}
__device__ __forceinline__ int next_item(unsigned long long *counter, unsigned long long base, int *slot,
                                         long long &ahead) {
    if (threadIdx.x == 0) {
        const long long t = ahead;
        *slot = (t < 0 || t > 0x7fffffffLL) ? 0x7fffffff : (int)t;     // out of range: stop
        ahead = (long long)(atomicAdd(counter, 1ull) - base);
    }
    __syncthreads();
    const int it = *slot;
    __syncthreads();
    return it;
}

// FLAT: the workgroup's one item is blockIdx.x (pass 0), then it stops; else the ticket queue
template <bool FLAT>
__device__ __forceinline__ int take_item(unsigned long long *counter, unsigned long long base, int *slot,
                                         long long &ahead, int pass) {
    if (FLAT) return pass == 0 ? (int)blockIdx.x : 0x7fffffff;
    return next_item(counter, base, slot, ahead);
}

template <int TK, int LPR, int U, bool FLAT>
__global__ __launch_bounds__(BT) void k_degrid_persist(const ProbDesc *__restrict__ pd, const int2 *__restrict__ items,
                                                       int n_items, int R, unsigned long long *counter,
                                                       unsigned long long base, const float2 *__restrict__ grids,
                                                       int64_t grid_stride, float2 *__restrict__ y) {
    __shared__ int slot;
    const int grp = threadIdx.x / LPR, sub = threadIdx.x & (LPR - 1);
    constexpr int NGRP = BT / LPR;
    long long ahead = FLAT ? 0 : first_ticket(counter, base);
    for (int pass = 0;; ++pass) {
        const int it = take_item<FLAT>(counter, base, &slot, ahead, pass);
        if (it >= n_items) break;
        const int2 w = items[it];
        const ProbDesc d = pd[w.x];
        const float2 *__restrict__ grid = grids + (int64_t)w.x * grid_stride;
        const int64_t rend = min((int64_t)w.y + R, d.M);
        for (int64_t r = w.y + grp; r < rend; r += NGRP) {
            const int64_t beg = d.rowptr[r], end = d.rowptr[r + 1];
            float ar = 0.f, ai = 0.f;
            for (int64_t j0 = beg + sub; j0 < end; j0 += LPR * U) {
                int c[U];
                float2 v[U];
#pragma unroll
                for (int t = 0; t < U; ++t) {
                    const int64_t j = j0 + LPR * t;
                    if (j < end) {
                        c[t] = d.col[j];
                        v[t] = load_tap_raw<TK>(d.val, j);
                    } else {
                        c[t] = 0;
                        v[t] = make_float2(0.f, 0.f);
                    }
                }
#pragma unroll
                for (int t = 0; t < U; ++t) {
                    const float2 g = grid[c[t]];
                    ar = fmaf(v[t].x, g.x, ar);
                    ar = fmaf(-v[t].y, g.y, ar);
                    ai = fmaf(v[t].x, g.y, ai);
                    ai = fmaf(v[t].y, g.x, ai);
                }
            }
#pragma unroll
            for (int o = LPR / 2; o > 0; o >>= 1) {
                ar += __shfl_xor(ar, o);
                ai += __shfl_xor(ai, o);
            }
            if (sub == 0) {
                if constexpr (TK == WP_TAPS_I16) {
                    ar *= d.rscale[r];
                    ai *= d.rscale[r];
                }
                y[d.y_off + (d.perm ? d.perm[r] : r)] = make_float2(ar, ai);
            }
        }
    }
}

template <int TK, int LPR, int U, bool FLAT>
__global__ __launch_bounds__(BT) void k_gather_persist(const ProbDesc *__restrict__ pd, const int2 *__restrict__ items,
                                                       int n_items, int C, int64_t cells, unsigned long long *counter,
                                                       unsigned long long base, const float2 *__restrict__ y,
                                                       float2 *__restrict__ grids, int64_t grid_stride) {
    __shared__ int slot;
    const int grp = threadIdx.x / LPR, sub = threadIdx.x & (LPR - 1);
    constexpr int NGRP = BT / LPR;
    long long ahead = FLAT ? 0 : first_ticket(counter, base);
    for (int pass = 0;; ++pass) {
        const int it = take_item<FLAT>(counter, base, &slot, ahead, pass);
        if (it >= n_items) break;
        const int2 w = items[it];
        const ProbDesc d = pd[w.x];
        float2 *__restrict__ grid = grids + (int64_t)w.x * grid_stride;
        const float2 *__restrict__ yp = y + d.y_off;
        const int64_t cend = min((int64_t)w.y + C, cells);
        // groups sweep the item's cells together: every lane of the block runs the same trip count
        for (int64_t c0 = w.y; c0 < cend; c0 += NGRP) {
            const int64_t c = c0 + grp;
            float ar = 0.f, ai = 0.f;
            if (c < cend) {
                const int64_t beg = d.tcolptr[c], end = d.tcolptr[c + 1];
                for (int64_t j0 = beg + sub; j0 < end; j0 += LPR * U) {
                    int k[U];
                    float2 v[U];
#pragma unroll
                    for (int t = 0; t < U; ++t) {
                        const int64_t j = j0 + LPR * t;
                        if (j < end) {
                            const int rr = d.trow[j];
                            k[t] = d.perm ? d.perm[rr] : rr;
                            v[t] = load_tap_raw<TK>(d.tval, j);
                            if constexpr (TK == WP_TAPS_I16) {
                                v[t].x *= d.rscale[rr];
                                v[t].y *= d.rscale[rr];
                            }
                        } else {
                            k[t] = -1;
                            v[t] = make_float2(0.f, 0.f);
                        }
                    }
#pragma unroll
                    for (int t = 0; t < U; ++t) {
                        const float2 yk = k[t] >= 0 ? yp[k[t]] : make_float2(0.f, 0.f);
                        ar = fmaf(v[t].x, yk.x, ar);
                        ar = fmaf(v[t].y, yk.y, ar);
                        ai = fmaf(v[t].x, yk.y, ai);
                        ai = fmaf(-v[t].y, yk.x, ai);
                    }
                }
            }
#pragma unroll
            for (int o = LPR / 2; o > 0; o >>= 1) {
                ar += __shfl_xor(ar, o);
                ai += __shfl_xor(ai, o);
            }
            if (sub == 0 && c < cend) grid[c] = make_float2(ar, ai);
        }
    }
}

// Blocked gather over the problems' block tables: an item is (problem, first block) and covers
// GB_ITEM blocks; each wavefront of the workgroup sums every fourth of them (gather_block).
constexpr int GB_ITEM = 32;

template <int TK, bool FLAT>
__global__ __launch_bounds__(BT) void k_gather_persist_blk(const ProbDesc *__restrict__ pd,
                                                           const int2 *__restrict__ items, int n_items,
                                                           unsigned long long *counter, unsigned long long base,
                                                           const float2 *__restrict__ y, float2 *__restrict__ grids,
                                                           int64_t grid_stride) {
    __shared__ int slot;
    __shared__ float2 s_p[BT / 64][GB_ENT];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    long long ahead = FLAT ? 0 : first_ticket(counter, base);
    for (int pass = 0;; ++pass) {
        const int it = take_item<FLAT>(counter, base, &slot, ahead, pass);
        if (it >= n_items) break;
        const int2 w = items[it];
        const ProbDesc d = pd[w.x];
        const int64_t bend = min((int64_t)w.y + GB_ITEM, d.n_tblk);
        for (int64_t bi = w.y + wv; bi < bend; bi += BT / 64)
            gather_block<TK, GB_ENT>(d.tblk, bi, d.tcolptr, d.trow, d.tval, d.rscale, y + d.y_off, d.perm,
                                     grids + (int64_t)w.x * grid_stride, s_p[wv], lane);
    }
}

struct Shape {
    int lpr, u, chunk;
};

}  // namespace

struct wp_batch {
    const wp_plan *plan;
    int P;
    int taps;
    bool transpose;
    int64_t M_total;
    std::vector<int64_t> M, y_off;
    ProbDesc *d_desc = nullptr;
    int2 *d_items_deg = nullptr, *d_items_gat = nullptr, *d_items_blk = nullptr;
    int n_items_deg = 0, n_items_gat = 0, n_items_blk = 0;
    bool blocks = false;           // every problem has a block table: the gather runs over blocks
    unsigned long long *d_counter = nullptr;
    unsigned long long base = 0;   // next launch's first ticket
    Shape deg{64, 4, 64}, gat{16, 8, 256};
    bool flat_deg = false, flat_gat = false;   // one workgroup per item instead of the ticket queue
    int nblocks;                   // persistent grid size
};

namespace {

template <int TK>
wp_status launch_deg(wp_batch *b, const float2 *grids, float2 *y, hipStream_t s) {
    const int64_t G2 = (int64_t)b->plan->Ng * b->plan->Ng;
    const bool flat = b->flat_deg;
    if (flat && b->n_items_deg == 0) return WP_OK;
    const dim3 g(flat ? b->n_items_deg : b->nblocks), t(BT);
#define DEG(L, U)                                                                                                   \
    do {                                                                                                            \
        if (flat)                                                                                                   \
            hipLaunchKernelGGL((k_degrid_persist<TK, L, U, true>), g, t, 0, s, b->d_desc, b->d_items_deg,         \
                               b->n_items_deg, b->deg.chunk, b->d_counter, b->base, grids, G2, y);                 \
        else                                                                                                        \
            hipLaunchKernelGGL((k_degrid_persist<TK, L, U, false>), g, t, 0, s, b->d_desc, b->d_items_deg,        \
                               b->n_items_deg, b->deg.chunk, b->d_counter, b->base, grids, G2, y);                 \
    } while (0)
    switch (b->deg.lpr * 100 + b->deg.u) {
        case 1604: DEG(16, 4); break;
        case 1608: DEG(16, 8); break;
        case 3204: DEG(32, 4); break;
        case 3208: DEG(32, 8); break;
        case 6404: DEG(64, 4); break;
        case 6408: DEG(64, 8); break;
        default: return wp_set_error(WP_EINVAL, "batch degrid shape %d x %d", b->deg.lpr, b->deg.u);
    }
#undef DEG
    if (wp_status st = wp_check_launch("batch degrid")) return st;
    if (!flat) b->base += (unsigned long long)b->n_items_deg + 2ull * (unsigned long long)b->nblocks;
    return WP_OK;
}

template <int TK>
wp_status launch_gat(wp_batch *b, const float2 *y, float2 *grids, hipStream_t s) {
    const int64_t G2 = (int64_t)b->plan->Ng * b->plan->Ng;
    const bool flat = b->flat_gat;
    if (flat && b->n_items_gat == 0) return WP_OK;
    const dim3 g(flat ? b->n_items_gat : b->nblocks), t(BT);
#define GAT(L, U)                                                                                                   \
    do {                                                                                                            \
        if (flat)                                                                                                   \
            hipLaunchKernelGGL((k_gather_persist<TK, L, U, true>), g, t, 0, s, b->d_desc, b->d_items_gat,         \
                               b->n_items_gat, b->gat.chunk, G2, b->d_counter, b->base, y, grids, G2);             \
        else                                                                                                        \
            hipLaunchKernelGGL((k_gather_persist<TK, L, U, false>), g, t, 0, s, b->d_desc, b->d_items_gat,        \
                               b->n_items_gat, b->gat.chunk, G2, b->d_counter, b->base, y, grids, G2);             \
    } while (0)
    switch (b->gat.lpr * 100 + b->gat.u) {
        case 804: GAT(8, 4); break;
        case 808: GAT(8, 8); break;
        case 1604: GAT(16, 4); break;
        case 1608: GAT(16, 8); break;
        case 3204: GAT(32, 4); break;
        case 3208: GAT(32, 8); break;
        default: return wp_set_error(WP_EINVAL, "batch gather shape %d x %d", b->gat.lpr, b->gat.u);
    }
#undef GAT
    if (wp_status st = wp_check_launch("batch gather")) return st;
    if (!flat) b->base += (unsigned long long)b->n_items_gat + 2ull * (unsigned long long)b->nblocks;
    return WP_OK;
}

wp_status run_deg(wp_batch *b, const float2 *grids, float2 *y, hipStream_t s) {
    if (b->taps == WP_TAPS_BF16) return launch_deg<WP_TAPS_BF16>(b, grids, y, s);
    if (b->taps == WP_TAPS_I16) return launch_deg<WP_TAPS_I16>(b, grids, y, s);
    return launch_deg<WP_TAPS_C64>(b, grids, y, s);
}

template <int TK>
wp_status launch_gat_blk(wp_batch *b, const float2 *y, float2 *grids, hipStream_t s) {
    const int64_t G2 = (int64_t)b->plan->Ng * b->plan->Ng;
    if (b->flat_gat && b->n_items_blk == 0) return WP_OK;
    if (b->flat_gat)
        hipLaunchKernelGGL((k_gather_persist_blk<TK, true>), dim3(b->n_items_blk), dim3(BT), 0, s, b->d_desc,
                           b->d_items_blk, b->n_items_blk, b->d_counter, b->base, y, grids, G2);
    else
        hipLaunchKernelGGL((k_gather_persist_blk<TK, false>), dim3(b->nblocks), dim3(BT), 0, s, b->d_desc,
                           b->d_items_blk, b->n_items_blk, b->d_counter, b->base, y, grids, G2);
    if (wp_status st = wp_check_launch("batch gather blocks")) return st;
    if (!b->flat_gat) b->base += (unsigned long long)b->n_items_blk + 2ull * (unsigned long long)b->nblocks;
    return WP_OK;
}

wp_status run_gat(wp_batch *b, const float2 *y, float2 *grids, hipStream_t s) {
    if (b->blocks) {
        if (b->taps == WP_TAPS_BF16) return launch_gat_blk<WP_TAPS_BF16>(b, y, grids, s);
        if (b->taps == WP_TAPS_I16) return launch_gat_blk<WP_TAPS_I16>(b, y, grids, s);
        return launch_gat_blk<WP_TAPS_C64>(b, y, grids, s);
    }
    if (b->taps == WP_TAPS_BF16) return launch_gat<WP_TAPS_BF16>(b, y, grids, s);
    if (b->taps == WP_TAPS_I16) return launch_gat<WP_TAPS_I16>(b, y, grids, s);
    return launch_gat<WP_TAPS_C64>(b, y, grids, s);
}

wp_status make_items(wp_batch *b, bool deg) {
    std::vector<int2> items;
    const int64_t cells = (int64_t)b->plan->Ng * b->plan->Ng;
    const int chunk = deg ? b->deg.chunk : b->gat.chunk;
    for (int p = 0; p < b->P; ++p) {
        const int64_t n = deg ? b->M[p] : cells;
        for (int64_t r = 0; r < n; r += chunk) items.push_back(make_int2(p, (int)r));
    }
    if (items.size() > 0x7fffffff) return wp_set_error(WP_ECAPACITY, "too many batch work items");
    int2 *&dst = deg ? b->d_items_deg : b->d_items_gat;
    if (dst) (void)hipFree(dst);
    dst = nullptr;
    WP_HIP(hipMalloc(&dst, sizeof(int2) * std::max<size_t>(items.size(), 1)));
    WP_HIP(hipMemcpy(dst, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice));
    (deg ? b->n_items_deg : b->n_items_gat) = (int)items.size();
    return WP_OK;
}

}  // namespace

wp_status batch_create(wp_batch **out, const wp_plan *p, int P, const wp_G *G) {
    wp_batch *b = new (std::nothrow) wp_batch();
    if (!b) return wp_set_error(WP_ENOMEM, "batch allocation");
    b->plan = p;
    b->P = P;
    b->taps = G[0].taps;
    b->transpose = true;
    b->M.resize(P);
    b->y_off.resize(P);
    std::vector<ProbDesc> desc(P);
    int64_t off = 0;
    for (int i = 0; i < P; ++i) {
        if (G[i].taps != b->taps) {
            delete b;
            return wp_set_error(WP_EINVAL, "batch: problem %d has a different tap type", i);
        }
        if (G[i].nnz > 0 && (!G[i].col || !G[i].val)) {
            delete b;
            return wp_set_error(WP_EINVAL, "batch: problem %d has no stored taps (factor-record form)", i);
        }
        if (!G[i].tcolptr) b->transpose = false;
        b->M[i] = G[i].M;
        b->y_off[i] = off;
        desc[i] = ProbDesc{G[i].rowptr, G[i].col, G[i].val, G[i].order == WP_ORDER_SORTED ? nullptr : G[i].perm,
                           G[i].tcolptr, G[i].trow, G[i].tval, G[i].rscale, G[i].tblk, G[i].n_tblk, G[i].M, off};
        off += G[i].M;
    }
    b->M_total = off;
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    b->nblocks = ncu * 8;
    hipError_t e = hipMalloc(&b->d_desc, sizeof(ProbDesc) * P);
    if (e == hipSuccess) e = hipMemcpy(b->d_desc, desc.data(), sizeof(ProbDesc) * P, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&b->d_counter, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(b->d_counter, 0, sizeof(unsigned long long));
    if (e != hipSuccess) {
        batch_destroy(b);
        return wp_set_error(WP_EHIP, "batch tables: %s", hipGetErrorString(e));
    }
    wp_status st = make_items(b, true);
    if (st == WP_OK && b->transpose) st = make_items(b, false);
    // blocks when every problem has a block table and cells are short on average (as for one problem)
    bool tables = b->transpose;
    int64_t nnz = 0;
    for (int i = 0; i < P; ++i) {
        tables = tables && G[i].tblk;
        nnz += G[i].nnz;
    }
    const double mean = (double)nnz / ((double)P * (double)p->Ng * (double)p->Ng);
    if (st == WP_OK && tables && mean < 512.0) {
        std::vector<int2> items;
        int64_t maxn = 0;
        for (int i = 0; i < P; ++i) {
            maxn = std::max(maxn, G[i].n_tblk);
            for (int64_t bi = 0; bi < G[i].n_tblk; bi += GB_ITEM) items.push_back(make_int2(i, (int)bi));
        }
        if (items.size() > 0x7fffffff || maxn > 0x7fffffff) {
            st = wp_set_error(WP_ECAPACITY, "too many batch gather blocks");
        } else if (!items.empty()) {
            hipError_t e2 = hipMalloc(&b->d_items_blk, sizeof(int2) * items.size());
            if (e2 == hipSuccess)
                e2 = hipMemcpy(b->d_items_blk, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice);
            if (e2 != hipSuccess) st = wp_set_error(WP_EHIP, "batch block items: %s", hipGetErrorString(e2));
            b->n_items_blk = (int)items.size();
            b->blocks = st == WP_OK;
        }
    }
    if (st != WP_OK) {
        batch_destroy(b);
        return st;
    }
    *out = b;
    return WP_OK;
}

void batch_destroy(wp_batch *b) {
    if (!b) return;
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_items_deg) (void)hipFree(b->d_items_deg);
    if (b->d_items_gat) (void)hipFree(b->d_items_gat);
    if (b->d_items_blk) (void)hipFree(b->d_items_blk);
    if (b->d_counter) (void)hipFree(b->d_counter);
    delete b;
}

int64_t batch_total_vis(const wp_batch *b) { return b->M_total; }

wp_status batch_phi(wp_batch *b, const float2 *x, float2 *y, float2 *grids, hipStream_t s) {
    if (wp_status st = launch_grid_forward(b->plan, x, grids, s, b->P)) return st;
    return run_deg(b, grids, y, s);
}

wp_status batch_phiT(wp_batch *b, const float2 *y, float2 *x, float2 *grids, hipStream_t s) {
    if (!b->transpose) return wp_set_error(WP_EUNSUPPORTED, "batch adjoint needs the transposed copy of every G");
    wp_status st = run_gat(b, y, grids, s);
    if (st != WP_OK) return st;
    return launch_grid_adjoint(b->plan, grids, x, s, b->P);
}

// Times every candidate shape (2 warm-up + 5 timed launches each) and keeps the fastest.
wp_status batch_autotune(wp_batch *b, const float2 *x, float2 *y, float2 *grids, hipStream_t s, float *best_us) {
    hipEvent_t e0, e1;
    WP_HIP(hipEventCreate(&e0));
    WP_HIP(hipEventCreate(&e1));
    if (wp_status st = launch_grid_forward(b->plan, x, grids, s, b->P)) return st;
    auto time_it = [&](bool deg, float &us) -> wp_status {
        for (int i = 0; i < 7; ++i) {
            if (i == 2) WP_HIP(hipEventRecord(e0, s));
            wp_status st;
            if (deg) st = run_deg(b, grids, y, s);
            else st = run_gat(b, y, grids, s);
            if (st != WP_OK) return st;
        }
        WP_HIP(hipEventRecord(e1, s));
        WP_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        WP_HIP(hipEventElapsedTime(&ms, e0, e1));
        us = ms * 1e3f / 5.f;
        return WP_OK;
    };
    const Shape deg_c[] = {{64, 4, 16}, {64, 4, 64}, {64, 4, 256}, {64, 8, 64}, {32, 4, 64}, {32, 8, 64}, {16, 8, 64}};
    const Shape gat_c[] = {{16, 8, 128}, {16, 8, 512}, {16, 8, 2048}, {16, 4, 512}, {8, 8, 512}, {32, 4, 512},
                           {32, 8, 512}};
    float best = 1e30f;
    Shape keep = b->deg;
    for (const Shape &c : deg_c) {
        b->deg = c;
        if (wp_status st = make_items(b, true)) return st;
        float us;
        if (wp_status st = time_it(true, us)) return st;
        if (us < best) { best = us; keep = c; }
    }
    b->deg = keep;
    if (wp_status st = make_items(b, true)) return st;
    {   // one workgroup per item against the ticket queue, for the kept shape
        b->flat_deg = true;
        float us;
        if (wp_status st = time_it(true, us)) return st;
        if (us < best) best = us;
        else b->flat_deg = false;
    }
    best_us[0] = best;
    if (b->transpose) {
        best = 1e30f;
        keep = b->gat;
        for (const Shape &c : gat_c) {
            b->gat = c;
            if (wp_status st = make_items(b, false)) return st;
            float us;
            if (wp_status st = time_it(false, us)) return st;
            if (us < best) { best = us; keep = c; }
        }
        b->gat = keep;
        if (wp_status st = make_items(b, false)) return st;
        b->flat_gat = true;
        float us;
        if (wp_status st = time_it(false, us)) return st;
        if (us < best) best = us;
        else b->flat_gat = false;
        best_us[1] = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return WP_OK;
}

void batch_set_mode(wp_batch *b, int deg, int gat, int *deg_out, int *gat_out) {
    if (deg >= 0) b->flat_deg = deg == 1;
    if (gat >= 0) b->flat_gat = gat == 1;
    if (deg_out) *deg_out = b->flat_deg ? 1 : 0;
    if (gat_out) *gat_out = b->flat_gat ? 1 : 0;
}

void batch_shapes(const wp_batch *b, int *out6) {
    out6[0] = b->deg.lpr; out6[1] = b->deg.u; out6[2] = b->deg.chunk;
    out6[3] = b->gat.lpr; out6[4] = b->gat.u; out6[5] = b->gat.chunk;
}
