// C ABI of the core-elements ALS library: argument checks, workspace carving,
// setup (validation, CSC, schedules) and the half-sweep / selection /
// objective entry points declared in include/coreals.h.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "internal.hpp"

using namespace coreals;

namespace {

thread_local std::string g_init_error;

inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct Carve {
    char *base;
    size_t off = 0;
    size_t cap;
    template <typename T>
    T *take(size_t count) {
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += a256(sizeof(T) * (count ? count : 1));
        return p;
    }
};

// The fixed layout of the workspace; with base == nullptr it only measures.
struct Layout {
    int64_t *col_ptr;
    int32_t *row_idx;
    float *val_t;
    int32_t *perm_u;
    int32_t *perm_m;
    unsigned long long *stats;
    unsigned int *queues;  // [2 * 16]
    int64_t *class_count;  // [2 * NCLASS]
    int64_t *max_deg;      // [2]
    int *err_flags;
    double *obj_partials;
    double *obj_out;
    float *partials;
    double *resid;
    uint16_t *key16;
    int32_t *fb_rows;      // rows the Woodbury classes leave to the n_f x n_f solve
    double *gram_part;     // implicit: per-block partial Grams
    float *G;              // implicit: the Gram of the other factor matrix
    void *gsel;            // fast variant: radix-select state
    int32_t *gT, *gK;      // fast variant: the global cut [64]
    struct SideArrays {
        uint32_t *uT;      // UNIF: per-row cut of the draw
        int32_t *uK;
        int32_t *pair_slot, *pair_chunk, *cutT, *cutK, *flag;
        int64_t *pair_off;
    } side[2];
    void *temp;
    size_t temp_bytes;
    size_t total;
};

// Ranks above 64 take the wide-rank kernels for every non-empty row.
bool wide_of(const als_problem &p) { return p.n_f > NF; }

// Light-row degree limit; 0 at wide ranks (every non-empty row is heavy).
int32_t heavy_n_of(const als_problem &p) {
    if (wide_of(p)) return 0;
    int32_t h = p.heavy_min_degree > 0 ? p.heavy_min_degree : DEFAULT_HEAVY_N;
    return h < 64 ? 64 : h;
}

int64_t pair_cap_of(const als_problem &p) {
    const int64_t cap = wide_of(p) ? PAIR_CAP_WIDE : PAIR_CAP;
    return p.heavy_pair_cap > 0 ? std::min<int64_t>(p.heavy_pair_cap, cap) : cap;
}

// Floats of one partial system (n x n plus the right-hand side), and cut
// entries per heavy row.
int64_t slot_floats(const als_problem &p) { return wide_of(p) ? (int64_t)(NFW + 1) * NFW : (int64_t)(NF + 1) * 64; }
int64_t cut_stride(const als_problem &p) { return wide_of(p) ? NFW : 64; }

int32_t chunk_of(const als_problem &p) {
    int32_t c = p.heavy_chunk > 0 ? p.heavy_chunk : DEFAULT_CHUNK;
    return c < CK ? CK : c;
}

// Heavy rows have s > 32 or degree > heavy_n >= 64, so there are at most
// nnz / 33 of them (at wide ranks every non-empty row); their chunk pairs
// number at most nnz / chunk + n_heavy.
int64_t heavy_bound(const als_problem &p, int64_t n_rows) {
    return std::min<int64_t>(n_rows, wide_of(p) ? p.nnz : p.nnz / 33 + 1);
}

int64_t pair_bound(const als_problem &p, int64_t n_rows) {
    return p.nnz / chunk_of(p) + heavy_bound(p, n_rows) + 1;
}

Layout carve(const als_problem &p, void *base) {
    Carve c{reinterpret_cast<char *>(base), 0, 0};
    Layout L;
    // ALS_USERS_ONLY: no column view and no items-side schedule; a column
    // view given by the caller is not built either
    const bool uo = (p.flags & ALS_USERS_ONLY) != 0;
    const bool own_csc = !uo && !p.col_ptr;
    L.col_ptr = c.take<int64_t>(own_csc ? (size_t)p.n_m + 1 : 1);
    L.row_idx = c.take<int32_t>(own_csc ? (size_t)p.nnz : 0);
    L.val_t = c.take<float>(own_csc ? (size_t)p.nnz : 0);
    L.perm_u = c.take<int32_t>((size_t)p.n_u);
    L.perm_m = c.take<int32_t>(uo ? 0 : (size_t)p.n_m);
    L.stats = c.take<unsigned long long>(NSTATS);
    L.queues = c.take<unsigned int>(2 * 16);
    L.class_count = c.take<int64_t>(2 * NCLASS);
    L.max_deg = c.take<int64_t>(2);
    L.err_flags = c.take<int>(4);
    L.obj_partials = c.take<double>((size_t)5 * objective_blocks());
    L.obj_out = c.take<double>(4);
    L.partials = c.take<float>((size_t)pair_cap_of(p) * slot_floats(p));
    L.resid = c.take<double>((size_t)pair_cap_of(p) * 2 * cut_stride(p));
    // core-elements runs: top 16 bits of each |x| of the fixed factor
    // matrix, read by the first two selection passes
    const int64_t other_max = uo ? p.n_m : std::max(p.n_u, p.n_m);
    const bool fast = (p.flags & ALS_FAST_VARIANT) != 0;
    L.key16 = c.take<uint16_t>(p.budget_num < p.budget_den && !fast ? (size_t)other_max * p.n_f : 0);
    L.gsel = c.take<char>(fast ? global_select_state_bytes() : 0);
    const bool impl = (p.flags & ALS_IMPLICIT) != 0;
    L.gram_part = c.take<double>(impl ? (size_t)implicit_gram_blocks() * NF * NF : 0);
    L.G = c.take<float>(impl ? (size_t)NF * NF : 0);
    L.fb_rows = c.take<int32_t>((size_t)std::max(p.n_u, uo ? (int64_t)0 : p.n_m));
    L.gT = c.take<int32_t>(64);
    L.gK = c.take<int32_t>(64);
    for (int sd = 0; sd < 2; ++sd) {
        const int64_t nr = sd == 0 ? p.n_u : (uo ? 0 : p.n_m);
        const int64_t hb = heavy_bound(p, nr), pb = nr ? pair_bound(p, nr) : 0;
        L.side[sd].pair_slot = c.take<int32_t>((size_t)pb);
        L.side[sd].pair_chunk = c.take<int32_t>((size_t)pb);
        L.side[sd].pair_off = c.take<int64_t>((size_t)hb + 1);
        L.side[sd].cutT = c.take<int32_t>((size_t)hb * cut_stride(p));
        L.side[sd].cutK = c.take<int32_t>((size_t)hb * cut_stride(p));
        L.side[sd].flag = c.take<int32_t>((size_t)hb);
        const bool unif = (p.flags & ALS_UNIF) != 0;
        L.side[sd].uT = c.take<uint32_t>(unif ? (size_t)nr : 0);
        L.side[sd].uK = c.take<int32_t>(unif ? (size_t)nr : 0);
    }
    size_t tb = own_csc ? csc_temp_bytes(p.nnz, p.n_m) : 0;
    size_t tp = perm_temp_bytes(uo ? p.n_u : std::max(p.n_u, p.n_m));
    L.temp_bytes = tb > tp ? tb : tp;
    L.temp = c.take<char>(L.temp_bytes);
    L.total = c.off;
    return L;
}

bool sizes_ok(const als_problem *p) {
    if (!p) return false;
    if (p->n_u < 0 || p->n_m < 0 || p->nnz < 0) return false;
    if (p->n_u > INT32_MAX || p->n_m > INT32_MAX || p->nnz > INT32_MAX) return false;
    if (p->n_f < 1 || p->n_f > NFW) return false;
    return true;
}

als_status fail(als_ctx *c, als_status st, const char *fmt, const char *detail = "") {
    char buf[512];
    std::snprintf(buf, sizeof(buf), fmt, detail);
    if (c) c->err = buf;
    else g_init_error = buf;
    return st;
}

#define HIP_CHECK(ctx, expr)                                                              \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail((ctx), ALS_E_DEVICE, "HIP error: %s", hipGetErrorString(e_)); \
    } while (0)

SweepScratch workspace_scratch(const als_ctx *c) { return SweepScratch{c->stats, c->queues, c->partials, c->resid}; }

// All launches of one half-sweep, in stream order (also what a graph captures).
// chk (fold-in answers, users side): keep each row's candidate when its
// relative residual passes, solve the others exactly.
// sc: where the call's counters, row queues, partial systems and residuals
// live (the context's workspace, or the allocation-free entry point's array);
// marks: record the profiling events when profiling is on.
als_status enqueue_half_sweep(als_ctx *c, int side, const float *other, float *out, const CheckArgs *chk,
                              const SweepScratch &sc, bool marks = true) {
    const Side &S = c->side[side];
    unsigned int *queues = sc.queues + side * 16;
    const bool prof = marks && c->profiling;
    // counters are cleared by a kernel, not a memset node, so that replays of a
    // captured graph start from zero every time
    HIP_CHECK(c, launch_zero_u64(sc.stats, NSTATS, c->stream));
    HIP_CHECK(c, launch_zero_u64(reinterpret_cast<unsigned long long *>(queues), 8, c->stream));
    auto mark_begin = [&](int cls, als_ctx::Mark &mk) -> hipError_t {
        if (!prof) return hipSuccess;
        hipError_t e = hipEventCreate(&mk.start);
        if (e == hipSuccess) e = hipEventCreate(&mk.stop);
        mk.side = side;
        mk.cls = cls;
        if (e == hipSuccess) e = hipEventRecord(mk.start, c->stream);
        return e;
    };
    auto mark_end = [&](als_ctx::Mark &mk) -> hipError_t {
        if (!prof) return hipSuccess;
        hipError_t e = hipEventRecord(mk.stop, c->stream);
        c->marks.push_back(mk);
        return e;
    };
    if (c->fast) {
        if (chk) return fail(c, ALS_E_STATE, "fold-in answers need the per-row method%s");
        // the global sketch of `other`, then every light row in one launch
        als_ctx::Mark mg{}, ml{};
        HIP_CHECK(c, mark_begin(PROF_HSELECT, mg));
        HIP_CHECK(c, launch_global_select(other, S.n_other, c->p.n_f, c->p.budget_num, c->p.budget_den,
                                          c->p.min_keep, c->gsel, c->gT, c->gK, c->stream));
        HIP_CHECK(c, mark_end(mg));
        SweepArgs a{};
        a.ptr = S.ptr;
        a.idx = S.idx;
        a.val = S.val;
        a.other = other;
        a.out = out;
        a.perm = S.perm;
        a.count = S.class_off[CLS_HEAVY];
        a.nf = c->p.n_f;
        a.lam = (float)c->p.lambda;
        a.num = c->p.budget_num;
        a.den = c->p.budget_den;
        a.min_keep = c->p.min_keep;
        a.stats = sc.stats;
        a.queue = queues;
        a.gT = c->gT;
        a.gK = c->gK;
        HIP_CHECK(c, mark_begin(CLS_FULL, ml));
        HIP_CHECK(c, launch_sweep_fast(a, c->light_blocks, c->stream));
        HIP_CHECK(c, mark_end(ml));
    }
    if (c->unif) {
        if (chk) return fail(c, ALS_E_STATE, "fold-in answers need the per-row method%s");
        // every row's uniform draw, then every light row in one launch
        als_ctx::Mark mg{}, ml{};
        HIP_CHECK(c, mark_begin(PROF_HSELECT, mg));
        HIP_CHECK(c, launch_unif_select(S.ptr, S.idx, S.n_rows, S.n_other, c->p.budget_num, c->p.budget_den,
                                        c->p.min_keep, c->seed, c->uT[side], c->uK[side], c->stream));
        HIP_CHECK(c, mark_end(mg));
        SweepArgs a{};
        a.ptr = S.ptr;
        a.idx = S.idx;
        a.val = S.val;
        a.other = other;
        a.out = out;
        a.perm = S.perm;
        a.count = S.class_off[CLS_HEAVY];
        a.nf = c->p.n_f;
        a.lam = (float)c->p.lambda;
        a.num = c->p.budget_num;
        a.den = c->p.budget_den;
        a.min_keep = c->p.min_keep;
        a.stats = sc.stats;
        a.queue = queues;
        HIP_CHECK(c, mark_begin(CLS_FULL, ml));
        HIP_CHECK(c, launch_sweep_unif(a, c->seed, S.n_other, c->uT[side], c->uK[side], c->light_blocks, c->stream));
        HIP_CHECK(c, mark_end(ml));
    }
    if (c->implicit) {
        if (chk) return fail(c, ALS_E_STATE, "fold-in answers need explicit feedback%s");
        // G = Y^T Y of the whole other factor matrix, shared by every row
        HIP_CHECK(c, launch_global_gram(other, S.n_other, c->p.n_f, c->gram_part, c->G, c->stream));
    }
    for (int cls = 0; cls < CLS_HEAVY && !c->fast && !c->unif; ++cls) {
        SweepArgs a{};
        a.ptr = S.ptr;
        a.idx = S.idx;
        a.val = S.val;
        a.other = other;
        a.out = out;
        a.perm = S.perm + S.class_off[cls];
        a.count = S.class_off[cls + 1] - S.class_off[cls];
        a.nf = c->p.n_f;
        a.lam = (float)c->p.lambda;
        a.num = c->p.budget_num;
        a.den = c->p.budget_den;
        a.min_keep = c->p.min_keep;
        a.stats = sc.stats;
        a.queue = queues + cls;
        // queue slots 9 .. 12: the Woodbury classes' fallback counts and queues
        a.fb_rows = c->fb_rows;
        a.fb_count = queues + 9 + (cls == CLS_NET2 ? 1 : 0);
        a.fb_queue = queues + 11 + (cls == CLS_NET2 ? 1 : 0);
        a.guess = chk ? chk->guess : nullptr;
        a.tol = chk ? chk->tol : 0.f;
        a.path = chk ? chk->path : nullptr;
        a.rho = chk ? chk->rho : nullptr;
        if (a.count <= 0) continue;
        als_ctx::Mark mk{};
        HIP_CHECK(c, mark_begin(cls, mk));
        a.alpha = (float)c->p.alpha;
        a.G = c->G;
        if (c->wide) HIP_CHECK(c, launch_wide_empty(a, c->stream));  // the only light rows: no entries
        else if (c->implicit) HIP_CHECK(c, launch_sweep_implicit(cls, a, c->light_blocks, c->stream));
        else if (chk) HIP_CHECK(c, launch_check_class(cls, a, c->light_blocks, c->stream));
        else HIP_CHECK(c, launch_sweep_class(cls, a, c->light_blocks, c->stream));
        HIP_CHECK(c, mark_end(mk));
    }
    const HeavyPlan &H = S.heavy;
    if (H.n_heavy > 0) {
        HeavyArgs h{};
        h.ptr = S.ptr;
        h.idx = S.idx;
        h.val = S.val;
        h.other = other;
        // 0: unknown size, which makes the heavy-row kernels use 64-bit gathers
        h.other_rows = (c->p.flags & ALS_GENERIC_GATHERS) ? 0 : (side == 0 ? c->p.n_m : c->p.n_u);
        h.out = out;
        h.rows = S.perm + S.class_off[CLS_HEAVY];
        h.count = H.n_heavy;
        h.nf = c->p.n_f;
        h.lam = (float)c->p.lambda;
        h.num = c->p.budget_num;
        h.den = c->p.budget_den;
        h.min_keep = c->p.min_keep;
        h.heavy_n = c->heavy_n;
        h.chunk = c->chunk;
        h.pair_slot = H.pair_slot;
        h.pair_chunk = H.pair_chunk;
        h.pair_off = H.pair_off;
        h.cutT = H.cutT;
        h.cutK = H.cutK;
        h.cstride = c->wide ? NFW : 64;
        // cutT still holds this side's cuts of its previous half-sweep
        h.hint = c->wide ? 0 : 1;
        h.col_base = 0;
        h.flag = c->flag[side];
        h.pass = 0;
        h.gpos = 0;
        h.implicit = c->implicit ? 1 : 0;
        h.alpha = (float)c->p.alpha;
        h.G = c->G;
        h.unif = c->unif ? 1 : 0;
        h.seed = c->seed;
        h.n_cols = S.n_other;
        h.uT = c->uT[side];
        h.uK = c->uK[side];
        if (c->fast) {
            // one cut per column for every heavy row, ties by row index
            h.gpos = 1;
            h.cstride = 0;
            h.cutT = c->gT;
            h.cutK = c->gK;
        }
        h.partials = sc.partials;
        h.resid = sc.resid;
        h.refine = 0;
        h.keep = c->bf16 ? 1 : 0;
        h.fp64res = c->fp64res;
        h.stats = sc.stats;
        h.queue = queues + CLS_HEAVY;
        h.guess = nullptr;
        h.tol = 0.f;
        h.path = nullptr;
        h.rho = nullptr;
        if (c->p.budget_num < c->p.budget_den && !c->fast && !c->unif) {
            if (c->key16 && h.other_rows > 0 && h.other_rows * h.nf * 4 <= (int64_t)0x7FFFFFFF) {
                // (the selection reads the copy only where it gathers by buffer loads)
                HIP_CHECK(c, launch_key16(other, h.other_rows * h.nf, c->key16, c->stream));
                h.key16 = c->key16;
            }
            als_ctx::Mark mk{};
            HIP_CHECK(c, mark_begin(PROF_HSELECT, mk));
            HIP_CHECK(c, launch_heavy_select(h, 0, c->stream));
            if (c->wide) {
                // columns 64 .. n_f - 1: a second launch with its own row counter
                h.col_base = 64;
                h.queue = queues + 8;
                HIP_CHECK(c, launch_heavy_select(h, 0, c->stream));
                h.col_base = 0;
                h.queue = queues + CLS_HEAVY;
            }
            h.key16 = nullptr;
            HIP_CHECK(c, mark_end(mk));
        }
        for (const auto &b : H.batches) {
            if (c->wide) {
                if (chk) return fail(c, ALS_E_STATE, "fold-in answers need n_f <= 64%s");
                als_ctx::Mark mg{}, ms{};
                HIP_CHECK(c, mark_begin(PROF_HGRAM, mg));
                HIP_CHECK(c, launch_wide_gram(h, b.pair_begin, b.pair_end, !c->bf16, c->stream));
                HIP_CHECK(c, mark_end(mg));
                HIP_CHECK(c, mark_begin(PROF_HSOLVE, ms));
                h.refine = 0;
                HIP_CHECK(c, launch_wide_solve(h, b.slot_begin, b.slot_end, b.pair_begin, c->stream));
                // pass 1, rows whose core system was singular: full-data Gram
                // (FP32 products) and solve, eq. (U); pass 2 (ALS_PREC_AUTO),
                // rows too ill-conditioned for one refinement step from a bf16
                // Gram: the Gram again with FP32 products
                for (int pass = 1; pass <= (c->fp64res == RES_PER_ROW ? 2 : 1); ++pass) {
                    h.pass = pass;
                    HIP_CHECK(c, launch_wide_gram(h, b.pair_begin, b.pair_end, true, c->stream));
                    HIP_CHECK(c, launch_wide_solve(h, b.slot_begin, b.slot_end, b.pair_begin, c->stream));
                }
                h.pass = 0;
                HIP_CHECK(c, mark_end(ms));
                if (c->bf16) {
                    als_ctx::Mark mr{}, m2{};
                    HIP_CHECK(c, mark_begin(PROF_HRESID, mr));
                    HIP_CHECK(c, launch_wide_resid(h, b.pair_begin, b.pair_end, c->stream));
                    HIP_CHECK(c, mark_end(mr));
                    HIP_CHECK(c, mark_begin(PROF_HREFINE, m2));
                    h.refine = 1;
                    HIP_CHECK(c, launch_wide_solve(h, b.slot_begin, b.slot_end, b.pair_begin, c->stream));
                    h.refine = 0;
                    HIP_CHECK(c, mark_end(m2));
                }
                continue;
            }
            if (chk) {
                // candidate residuals of the batch's rows; accepted rows are then
                // skipped by every kernel below (path 0)
                h.guess = chk->guess;
                h.tol = chk->tol;
                h.path = nullptr;
                h.rho = chk->rho;
                HIP_CHECK(c, launch_heavy_check(h, b.pair_begin, b.pair_end, c->stream));
                h.path = chk->path;
                HIP_CHECK(c, launch_heavy_check_reduce(h, b.slot_begin, b.slot_end, b.pair_begin, c->stream));
            }
            als_ctx::Mark mg{}, ms{};
            HIP_CHECK(c, mark_begin(PROF_HGRAM, mg));
            if (c->bf16) HIP_CHECK(c, launch_heavy_gram_bf16(h, b.pair_begin, b.pair_end, c->stream));
            else HIP_CHECK(c, launch_heavy_gram(h, b.pair_begin, b.pair_end, c->stream));
            HIP_CHECK(c, mark_end(mg));
            HIP_CHECK(c, mark_begin(PROF_HSOLVE, ms));
            h.refine = 0;
            HIP_CHECK(c, launch_heavy_solve(h, b.slot_begin, b.slot_end, b.pair_begin, c->stream));
            if (c->fp64res == RES_PER_ROW) {
                // rows too ill-conditioned for one refinement step from a bf16
                // Gram: the Gram again with FP32 products, and a new solve
                h.pass = 2;
                HIP_CHECK(c, launch_heavy_gram(h, b.pair_begin, b.pair_end, c->stream));
                HIP_CHECK(c, launch_heavy_solve(h, b.slot_begin, b.slot_end, b.pair_begin, c->stream));
                h.pass = 0;
            }
            HIP_CHECK(c, mark_end(ms));
            if (c->bf16) {
                // one refinement step: chunk residuals, then the correction solve
                als_ctx::Mark mr{}, m2{};
                HIP_CHECK(c, mark_begin(PROF_HRESID, mr));
                HIP_CHECK(c, launch_heavy_resid(h, b.pair_begin, b.pair_end, c->stream));
                HIP_CHECK(c, mark_end(mr));
                HIP_CHECK(c, mark_begin(PROF_HREFINE, m2));
                h.refine = 1;
                HIP_CHECK(c, launch_heavy_solve(h, b.slot_begin, b.slot_end, b.pair_begin, c->stream));
                HIP_CHECK(c, mark_end(m2));
            }
        }
    }
    return ALS_OK;
}

als_status run_half_sweep(als_ctx *c, int side, const float *other, float *out, als_sweep_stats *st) {
    if (!c) return ALS_E_STATE;
    if (side == 1 && c->users_only) return fail(c, ALS_E_STATE, "context was created with ALS_USERS_ONLY%s");
    if (!other || !out) return fail(c, ALS_E_ARG, "NULL factor pointer%s");
    if (other == out) return fail(c, ALS_E_ARG, "input and output factor matrices alias%s");
    if (c->use_graphs && !c->profiling) {
        als_ctx::Graph &G = c->graph[side];
        if (!G.exec || G.other != other || G.out != out || G.seed != c->seed) {
            if (G.exec) {
                (void)hipGraphExecDestroy(G.exec);
                G.exec = nullptr;
            }
            hipGraph_t g = nullptr;
            HIP_CHECK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            als_status rs = enqueue_half_sweep(c, side, other, out, nullptr, workspace_scratch(c));
            hipError_t ec = hipStreamEndCapture(c->stream, &g);
            if (rs != ALS_OK) {
                if (g) (void)hipGraphDestroy(g);
                return rs;
            }
            HIP_CHECK(c, ec);
            hipError_t ei = hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIP_CHECK(c, ei);
            G.other = other;
            G.out = out;
            G.seed = c->seed;
        }
        HIP_CHECK(c, hipGraphLaunch(G.exec, c->stream));
    } else {
        als_status rs = enqueue_half_sweep(c, side, other, out, nullptr, workspace_scratch(c));
        if (rs != ALS_OK) return rs;
    }
    if (st) return fill_stats(c, side, c->stats, st);
    return ALS_OK;
}

}  // namespace

namespace coreals {

als_status enqueue_checked_users(als_ctx *c, const float *M, float *out, const CheckArgs &chk) {
    if (!c) return ALS_E_STATE;
    HIP_CHECK(c, launch_zero_u64(c->stats, NSTATS, c->stream));
    return enqueue_half_sweep(c, 0, M, out, &chk, workspace_scratch(c));
}

als_status read_stats(als_ctx *c, unsigned long long *h) {
    HIP_CHECK(c, hipMemcpyAsync(h, c->stats, sizeof(unsigned long long) * NSTATS, hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(c, hipStreamSynchronize(c->stream));
    return ALS_OK;
}

als_status set_error(als_ctx *c, als_status st, const char *msg) { return fail(c, st, "%s", msg); }

als_status fill_stats(als_ctx *c, int side, const unsigned long long *stats, als_sweep_stats *st) {
    unsigned long long h[NSTATS];
    HIP_CHECK(c, hipMemcpyAsync(h, stats, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(c, hipStreamSynchronize(c->stream));
    st->n_empty = (int64_t)h[ST_EMPTY];
    st->n_singular_fallback = (int64_t)h[ST_FALLBACK];
    st->n_fp64_residual = (int64_t)h[ST_FP64RES];
    st->n_rows = c->side[side].n_rows;
    st->n_fp32_gram = (int64_t)h[ST_FP32GRAM];
    double mr;
    std::memcpy(&mr, &h[ST_MAXRES], sizeof(mr));
    st->max_rel_residual = mr;
    st->n_select_hinted = (int64_t)h[ST_HINTED];
    st->n_pivoted = (int64_t)h[ST_PIVOTED];
    return ALS_OK;
}

als_status enqueue_half_sweep_scratch(als_ctx *c, int side, const float *other, float *out, const SweepScratch &sc) {
    if (!c) return ALS_E_STATE;
    if (side == 1 && c->users_only) return fail(c, ALS_E_STATE, "context was created with ALS_USERS_ONLY%s");
    if (!other || !out) return fail(c, ALS_E_ARG, "NULL factor pointer%s");
    if (other == out) return fail(c, ALS_E_ARG, "input and output factor matrices alias%s");
    return enqueue_half_sweep(c, side, other, out, nullptr, sc, false);
}

}  // namespace coreals

extern "C" {

size_t als_workspace_size(const als_problem *p) {
    if (!sizes_ok(p)) return 0;
    return carve(*p, nullptr).total;
}

als_status als_init(const als_problem *p, als_ctx **out) {
    if (!out) return fail(nullptr, ALS_E_ARG, "out is NULL%s");
    *out = nullptr;
    if (!sizes_ok(p)) return fail(nullptr, ALS_E_ARG, "invalid sizes (need 1 <= n_f <= 128, sizes < 2^31)%s");
    if (!(p->lambda >= 0.0)) return fail(nullptr, ALS_E_ARG, "lambda must be >= 0%s");
    if (p->budget_den == 0 || p->budget_num == 0 || p->budget_num > p->budget_den)
        return fail(nullptr, ALS_E_ARG, "budget rate must satisfy 0 < num <= den%s");
    if (p->min_keep < 0) return fail(nullptr, ALS_E_ARG, "min_keep must be >= 0%s");
    if ((p->flags & ALS_IMPLICIT) &&
        (p->n_f > NF || p->precision != ALS_PREC_FP32 || (p->flags & (ALS_FAST_VARIANT | ALS_UNIF))))
        return fail(nullptr, ALS_E_ARG, "implicit feedback needs n_f <= 64, FP32 and the per-row method%s");
    if ((p->flags & ALS_IMPLICIT) && !(p->alpha >= 0.0))
        return fail(nullptr, ALS_E_ARG, "alpha must be >= 0%s");
    if ((p->flags & ALS_UNIF) &&
        (p->n_f > NF || p->precision != ALS_PREC_FP32 || (p->flags & ALS_FAST_VARIANT)))
        return fail(nullptr, ALS_E_ARG, "UNIF needs n_f <= 64, FP32 and not the fast variant%s");
    if ((p->flags & ALS_FAST_VARIANT) &&
        (p->n_f > NF || p->precision != ALS_PREC_FP32 || (p->flags & ALS_USERS_ONLY)))
        return fail(nullptr, ALS_E_ARG, "the fast variant needs n_f <= 64, FP32 and both sides%s");
    if (p->precision < ALS_PREC_FP32 || p->precision > ALS_PREC_AUTO)
        return fail(nullptr, ALS_E_ARG, "unknown precision mode%s");
    if (!p->row_ptr || (p->nnz > 0 && (!p->col_idx || !p->val)))
        return fail(nullptr, ALS_E_ARG, "NULL CSR pointer%s");
    if (p->col_ptr && (p->nnz > 0 && (!p->row_idx || !p->val_t)))
        return fail(nullptr, ALS_E_ARG, "col_ptr given without row_idx and val_t%s");
    Layout probe = carve(*p, nullptr);
    if (!p->workspace || p->workspace_bytes < probe.total)
        return fail(nullptr, ALS_E_NOMEM, "workspace too small (see als_workspace_size)%s");

    als_ctx *c = new (std::nothrow) als_ctx();
    if (!c) return fail(nullptr, ALS_E_NOMEM, "host allocation failed%s");
    c->p = *p;
    c->stream = reinterpret_cast<hipStream_t>(p->stream);
    Layout L = carve(*p, p->workspace);
    const bool given_csc = p->col_ptr && !(p->flags & ALS_USERS_ONLY);
    c->col_ptr = given_csc ? const_cast<int64_t *>(p->col_ptr) : L.col_ptr;
    c->row_idx = given_csc ? const_cast<int32_t *>(p->row_idx) : L.row_idx;
    c->val_t = given_csc ? const_cast<float *>(p->val_t) : L.val_t;
    c->stats = L.stats;
    c->queues = L.queues;
    c->light_blocks = p->light_blocks;
    c->obj_partials = L.obj_partials;
    c->obj_out = L.obj_out;
    c->partials = L.partials;
    c->resid = L.resid;
    c->fast = (p->flags & ALS_FAST_VARIANT) != 0;
    c->unif = (p->flags & ALS_UNIF) != 0;
    c->implicit = (p->flags & ALS_IMPLICIT) != 0;
    c->fb_rows = L.fb_rows;
    c->gram_part = L.gram_part;
    c->G = L.G;
    c->key16 = p->budget_num < p->budget_den && !c->fast && !c->unif ? L.key16 : nullptr;
    c->gsel = L.gsel;
    c->gT = L.gT;
    c->gK = L.gK;
    c->bf16 = p->precision != ALS_PREC_FP32;
    // FP64 residual: always (FP64RES), per row (AUTO: lambda < 1e-3 and a
    // large pivot ratio), or never
    c->fp64res = p->precision == ALS_PREC_BF16_IR_FP64RES ? RES_FP64
                 : p->precision == ALS_PREC_AUTO          ? RES_PER_ROW
                                                          : RES_FP32;
    c->wide = wide_of(*p);
    c->heavy_n = heavy_n_of(*p);
    c->chunk = chunk_of(*p);
    c->pair_cap = pair_cap_of(*p);
    c->temp = L.temp;
    c->temp_bytes = L.temp_bytes;
    c->users_only = (p->flags & ALS_USERS_ONLY) != 0;
    const int n_sides = c->users_only ? 1 : 2;

    auto bail = [&](als_status st, const std::string &msg) {
        g_init_error = msg;
        delete c;
        return st;
    };
    hipStream_t s = c->stream;
    hipError_t e;
#define INIT_HIP(expr)                                                                  \
    do {                                                                                \
        e = (expr);                                                                     \
        if (e != hipSuccess) return bail(ALS_E_DEVICE, std::string("HIP error: ") + hipGetErrorString(e)); \
    } while (0)

    // 1. validate R
    INIT_HIP(hipMemsetAsync(L.err_flags, 0, sizeof(int) * 4, s));
    INIT_HIP(launch_validate(p->n_u, p->n_m, p->nnz, p->row_ptr, p->col_idx, p->val,
                             (p->flags & ALS_VALIDATE) ? 1 : 0, L.err_flags, s));
    int flags = 0;
    INIT_HIP(hipMemcpyAsync(&flags, L.err_flags, sizeof(int), hipMemcpyDeviceToHost, s));
    INIT_HIP(hipStreamSynchronize(s));
    if (flags & 3) return bail(ALS_E_INDEX, "row_ptr or col_idx invalid (range, order or repeats)");
    if (flags & 4) return bail(ALS_E_VALUE, "NaN or Inf among the ratings");

    // 2. column view: built, or the caller's (checked as the CSR is: pointers
    // monotone from 0 to nnz, row indices in range and strictly increasing)
    if (given_csc) {
        INIT_HIP(hipMemsetAsync(L.err_flags, 0, sizeof(int) * 4, s));
        INIT_HIP(launch_validate(p->n_m, p->n_u, p->nnz, p->col_ptr, p->row_idx, p->val_t,
                                 (p->flags & ALS_VALIDATE) ? 1 : 0, L.err_flags, s));
        INIT_HIP(hipMemcpyAsync(&flags, L.err_flags, sizeof(int), hipMemcpyDeviceToHost, s));
        INIT_HIP(hipStreamSynchronize(s));
        if (flags & 3) return bail(ALS_E_INDEX, "col_ptr or row_idx invalid (range, order or repeats)");
        if (flags & 4) return bail(ALS_E_VALUE, "NaN or Inf among the column view's ratings");
    } else if (!c->users_only) {
        INIT_HIP(build_csc(p->n_u, p->n_m, p->nnz, p->row_ptr, p->col_idx, p->val, L.col_ptr, L.row_idx, L.val_t,
                           L.temp, s));
    }

    // 3. schedules
    Side &U = c->side[0];
    U.n_rows = p->n_u;
    U.n_other = p->n_m;
    U.ptr = p->row_ptr;
    U.idx = p->col_idx;
    U.val = p->val;
    U.perm = L.perm_u;
    Side &M = c->side[1];
    M.n_rows = c->users_only ? 0 : p->n_m;
    M.n_other = p->n_u;
    M.ptr = c->col_ptr;
    M.idx = c->row_idx;
    M.val = c->val_t;
    M.perm = L.perm_m;
    int64_t host_counts[2 * NCLASS] = {};
    int64_t host_max[2] = {};
    INIT_HIP(hipMemsetAsync(L.class_count, 0, sizeof(int64_t) * 2 * NCLASS, s));
    INIT_HIP(hipMemsetAsync(L.max_deg, 0, sizeof(int64_t) * 2, s));
    for (int sd = 0; sd < n_sides; ++sd) {
        Side &S = c->side[sd];
        INIT_HIP(build_schedule(S.n_rows, S.ptr, p->budget_num, p->budget_den, p->min_keep, c->heavy_n, S.perm,
                                L.class_count + sd * NCLASS, L.max_deg + sd, L.temp, s));
    }
    INIT_HIP(hipMemcpyAsync(host_counts, L.class_count, sizeof(host_counts), hipMemcpyDeviceToHost, s));
    INIT_HIP(hipMemcpyAsync(host_max, L.max_deg, sizeof(host_max), hipMemcpyDeviceToHost, s));
    INIT_HIP(hipStreamSynchronize(s));
    for (int sd = 0; sd < 2; ++sd) {
        Side &S = c->side[sd];
        S.class_off[0] = 0;
        for (int k = 0; k < NCLASS; ++k) S.class_off[k + 1] = S.class_off[k] + host_counts[sd * NCLASS + k];
        S.max_deg = host_max[sd];
    }
    // heavy-row plan: chunk pairs and batches that fit the partial scratch
    for (int sd = 0; sd < n_sides; ++sd) {
        Side &S = c->side[sd];
        HeavyPlan &H = S.heavy;
        H.n_heavy = S.class_off[CLS_HEAVY + 1] - S.class_off[CLS_HEAVY];
        H.pair_slot = L.side[sd].pair_slot;
        H.pair_chunk = L.side[sd].pair_chunk;
        H.pair_off = L.side[sd].pair_off;
        H.cutT = L.side[sd].cutT;
        H.cutK = L.side[sd].cutK;
        c->flag[sd] = L.side[sd].flag;
        c->uT[sd] = L.side[sd].uT;
        c->uK[sd] = L.side[sd].uK;
        if (H.n_heavy == 0) continue;
        if (H.n_heavy > heavy_bound(*p, S.n_rows)) return bail(ALS_E_STATE, "heavy-row bound violated");
        // no previous cuts yet: the selection's first half-sweep takes no hint
        INIT_HIP(hipMemsetAsync(H.cutT, 0xFF, sizeof(int32_t) * (size_t)H.n_heavy * cut_stride(*p), s));
        std::vector<int32_t> rows((size_t)H.n_heavy);
        std::vector<int64_t> ptr((size_t)S.n_rows + 1);
        INIT_HIP(hipMemcpyAsync(rows.data(), S.perm + S.class_off[CLS_HEAVY], sizeof(int32_t) * rows.size(),
                                hipMemcpyDeviceToHost, s));
        INIT_HIP(hipMemcpyAsync(ptr.data(), S.ptr, sizeof(int64_t) * ptr.size(), hipMemcpyDeviceToHost, s));
        INIT_HIP(hipStreamSynchronize(s));
        std::vector<int64_t> off((size_t)H.n_heavy + 1, 0);
        for (int64_t t = 0; t < H.n_heavy; ++t) {
            const int64_t n = ptr[rows[t] + 1] - ptr[rows[t]];
            const int64_t chunks = std::max<int64_t>(1, (n + c->chunk - 1) / c->chunk);
            off[t + 1] = off[t] + chunks;
        }
        H.n_pairs = off[H.n_heavy];
        if (H.n_pairs > pair_bound(*p, S.n_rows)) return bail(ALS_E_STATE, "pair bound violated");
        std::vector<int32_t> pslot((size_t)H.n_pairs), pchunk((size_t)H.n_pairs);
        for (int64_t t = 0; t < H.n_heavy; ++t)
            for (int64_t q = off[t]; q < off[t + 1]; ++q) {
                pslot[q] = (int32_t)t;
                pchunk[q] = (int32_t)(q - off[t]);
            }
        H.batches.clear();
        int64_t t0 = 0;
        while (t0 < H.n_heavy) {
            int64_t t1 = t0 + 1;
            while (t1 < H.n_heavy && off[t1 + 1] - off[t0] <= c->pair_cap) ++t1;
            if (off[t1] - off[t0] > c->pair_cap)
                return bail(ALS_E_NOMEM, "a heavy row needs more partial systems than heavy_pair_cap");
            H.batches.push_back({t0, t1, off[t0], off[t1]});
            t0 = t1;
        }
        INIT_HIP(hipMemcpyAsync(H.pair_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice, s));
        INIT_HIP(hipMemcpyAsync(H.pair_slot, pslot.data(), sizeof(int32_t) * pslot.size(), hipMemcpyHostToDevice, s));
        INIT_HIP(hipMemcpyAsync(H.pair_chunk, pchunk.data(), sizeof(int32_t) * pchunk.size(), hipMemcpyHostToDevice,
                                s));
        INIT_HIP(hipStreamSynchronize(s));
    }
#undef INIT_HIP
    *out = c;
    return ALS_OK;
}

als_status half_sweep_users(als_ctx *c, const float *M, float *U, als_sweep_stats *st) {
    return run_half_sweep(c, 0, M, U, st);
}

als_status half_sweep_items(als_ctx *c, const float *U, float *M, als_sweep_stats *st) {
    return run_half_sweep(c, 1, U, M, st);
}

als_status core_select_count(als_ctx *c, int side, int64_t row_begin, int64_t row_end, int64_t *count) {
    if (!c) return ALS_E_STATE;
    if (side != 0 && side != 1) return fail(c, ALS_E_ARG, "side must be 0 or 1%s");
    if (side == 1 && c->users_only) return fail(c, ALS_E_STATE, "context was created with ALS_USERS_ONLY%s");
    if (!count) return fail(c, ALS_E_ARG, "count is NULL%s");
    const Side &S = c->side[side];
    if (row_begin < 0 || row_end < row_begin || row_end > S.n_rows) return fail(c, ALS_E_ARG, "bad row range%s");
    int64_t cnt = row_end - row_begin;
    int64_t *tmp_ptr = reinterpret_cast<int64_t *>(c->temp);
    void *tmp_rest = reinterpret_cast<char *>(c->temp) + a256(sizeof(int64_t) * (size_t)(cnt + 1));
    HIP_CHECK(c, launch_select_sizes(S.ptr, row_begin, row_end, c->p.n_f, c->p.budget_num, c->p.budget_den,
                                     c->p.min_keep, tmp_ptr, tmp_rest, c->stream));
    HIP_CHECK(c, hipMemcpyAsync(count, tmp_ptr + cnt, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(c, hipStreamSynchronize(c->stream));
    return ALS_OK;
}

als_status core_select(als_ctx *c, int side, const float *other, int64_t row_begin, int64_t row_end,
                       int64_t *sel_ptr, int32_t *sel_pos, int64_t sel_cap) {
    if (!c) return ALS_E_STATE;
    if (side != 0 && side != 1) return fail(c, ALS_E_ARG, "side must be 0 or 1%s");
    if (side == 1 && c->users_only) return fail(c, ALS_E_STATE, "context was created with ALS_USERS_ONLY%s");
    if (!other || !sel_ptr || (!sel_pos && sel_cap > 0)) return fail(c, ALS_E_ARG, "NULL pointer%s");
    const Side &S = c->side[side];
    if (row_begin < 0 || row_end < row_begin || row_end > S.n_rows) return fail(c, ALS_E_ARG, "bad row range%s");
    HIP_CHECK(c, launch_select_sizes(S.ptr, row_begin, row_end, c->p.n_f, c->p.budget_num, c->p.budget_den,
                                     c->p.min_keep, sel_ptr, c->temp, c->stream));
    int64_t total = 0;
    HIP_CHECK(c, hipMemcpyAsync(&total, sel_ptr + (row_end - row_begin), sizeof(int64_t), hipMemcpyDeviceToHost,
                                c->stream));
    HIP_CHECK(c, hipStreamSynchronize(c->stream));
    if (total > sel_cap) return fail(c, ALS_E_NOMEM, "sel_pos capacity below core_select_count%s");
    // heavy rows of the range: cuts by the sweep's own heavy-row selection,
    // stored in the partial scratch, processed in sub-ranges that fit it
    const int64_t cs = cut_stride(c->p);
    const int64_t sub = c->pair_cap * slot_floats(c->p) / (2 * cs);
    for (int64_t r0 = row_begin; r0 < row_end; r0 += sub) {
        const int64_t r1 = std::min(row_end, r0 + sub);
        int32_t *cutT = reinterpret_cast<int32_t *>(c->partials);
        int32_t *cutK = cutT + (r1 - r0) * cs;
        HeavyArgs h{};
        h.ptr = S.ptr;
        h.idx = S.idx;
        h.other = other;
        h.other_rows = (c->p.flags & ALS_GENERIC_GATHERS) ? 0 : (side == 0 ? c->p.n_m : c->p.n_u);
        h.rows = nullptr;
        h.count = r1 - r0;
        h.nf = c->p.n_f;
        h.num = c->p.budget_num;
        h.den = c->p.budget_den;
        h.min_keep = c->p.min_keep;
        h.heavy_n = c->heavy_n;
        h.cutT = cutT;
        h.cutK = cutK;
        h.cstride = (int32_t)cs;
        h.col_base = 0;
        HIP_CHECK(c, launch_heavy_select(h, r0, c->stream));
        if (c->wide) {
            h.col_base = 64;
            HIP_CHECK(c, launch_heavy_select(h, r0, c->stream));
        }
        SelectArgs a;
        a.ptr = S.ptr;
        a.idx = S.idx;
        a.other = other;
        a.row_begin = r0;
        a.row_end = r1;
        a.nf = c->p.n_f;
        a.num = c->p.budget_num;
        a.den = c->p.budget_den;
        a.min_keep = c->p.min_keep;
        a.heavy_n = c->heavy_n;
        a.sel_ptr = sel_ptr + (r0 - row_begin);
        a.sel_pos = sel_pos;
        a.cutT = cutT;
        a.cutK = cutK;
        if (c->wide) HIP_CHECK(c, launch_select_wide(a, c->stream));
        else HIP_CHECK(c, launch_select(a, c->stream));
    }
    return ALS_OK;
}

als_status core_select_global(als_ctx *c, int side, const float *other, int32_t *T, int32_t *K) {
    if (!c) return ALS_E_STATE;
    if (side != 0 && side != 1) return fail(c, ALS_E_ARG, "side must be 0 or 1%s");
    if (side == 1 && c->users_only) return fail(c, ALS_E_STATE, "context was created with ALS_USERS_ONLY%s");
    if (!c->fast) return fail(c, ALS_E_STATE, "context was created without ALS_FAST_VARIANT%s");
    if (!other || !T || !K) return fail(c, ALS_E_ARG, "NULL pointer%s");
    HIP_CHECK(c, launch_global_select(other, c->side[side].n_other, c->p.n_f, c->p.budget_num, c->p.budget_den,
                                      c->p.min_keep, c->gsel, c->gT, c->gK, c->stream));
    HIP_CHECK(c, hipMemcpyAsync(T, c->gT, sizeof(int32_t) * c->p.n_f, hipMemcpyDeviceToDevice, c->stream));
    HIP_CHECK(c, hipMemcpyAsync(K, c->gK, sizeof(int32_t) * c->p.n_f, hipMemcpyDeviceToDevice, c->stream));
    return ALS_OK;
}

als_status objective(als_ctx *c, const float *U, const float *M, als_objective *out) {
    if (!c) return ALS_E_STATE;
    if (c->users_only) return fail(c, ALS_E_STATE, "context was created with ALS_USERS_ONLY%s");
    if (c->implicit) return fail(c, ALS_E_STATE, "objective computes the explicit loss; context is ALS_IMPLICIT%s");
    if (!U || !M || !out) return fail(c, ALS_E_ARG, "NULL pointer%s");
    HIP_CHECK(c, launch_objective(c->p.n_u, c->p.n_m, c->p.n_f, c->p.row_ptr, c->p.col_idx, c->p.val, c->col_ptr, U,
                                  M, c->p.lambda, c->obj_partials, c->obj_out, c->stream));
    double h[4];
    HIP_CHECK(c, hipMemcpyAsync(h, c->obj_out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(c, hipStreamSynchronize(c->stream));
    out->f = h[0];
    out->sse = h[1];
    out->rmse = h[2];
    out->remse = h[3];
    return ALS_OK;
}

als_status als_profile_begin(als_ctx *c) {
    if (!c) return ALS_E_STATE;
    for (auto &m : c->marks) {
        (void)hipEventDestroy(m.start);
        (void)hipEventDestroy(m.stop);
    }
    c->marks.clear();
    c->profiling = true;
    return ALS_OK;
}

als_status als_profile_end(als_ctx *c, double *ms, int64_t *launches) {
    if (!c) return ALS_E_STATE;
    if (ms)
        for (int k = 0; k < 2 * NPROF; ++k) ms[k] = 0.0;
    if (launches)
        for (int k = 0; k < 2 * NPROF; ++k) launches[k] = 0;
    HIP_CHECK(c, hipStreamSynchronize(c->stream));
    for (auto &m : c->marks) {
        float t = 0.f;
        HIP_CHECK(c, hipEventElapsedTime(&t, m.start, m.stop));
        if (ms) ms[m.side * NPROF + m.cls] += t;
        if (launches) launches[m.side * NPROF + m.cls] += 1;
        (void)hipEventDestroy(m.start);
        (void)hipEventDestroy(m.stop);
    }
    c->marks.clear();
    c->profiling = false;
    return ALS_OK;
}

als_status als_class_counts(const als_ctx *c, int64_t *out) {
    if (!c || !out) return ALS_E_STATE;
    for (int sd = 0; sd < 2; ++sd)
        for (int k = 0; k < NCLASS; ++k) out[sd * NCLASS + k] = c->side[sd].class_off[k + 1] - c->side[sd].class_off[k];
    return ALS_OK;
}

als_status als_set_sample_seed(als_ctx *c, uint64_t seed) {
    if (!c) return ALS_E_STATE;
    c->seed = seed;
    return ALS_OK;
}

als_status als_use_graphs(als_ctx *c, int enable) {
    if (!c) return ALS_E_STATE;
    if (enable && c->stream == nullptr)
        return fail(c, ALS_E_STATE, "graph capture needs a non-default stream%s");
    c->use_graphs = enable != 0;
    return ALS_OK;
}

void als_destroy(als_ctx *c) {
    if (!c) return;
    for (auto &g : c->graph)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    for (auto &m : c->marks) {
        (void)hipEventDestroy(m.start);
        (void)hipEventDestroy(m.stop);
    }
    delete c;
}

const char *als_last_error(const als_ctx *c) { return c ? c->err.c_str() : g_init_error.c_str(); }

}  // extern "C"
