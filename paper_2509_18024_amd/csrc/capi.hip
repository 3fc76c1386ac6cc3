// C ABI of the core-elements ALS library: argument checks, workspace carving,
// setup (validation, CSC, schedules) and the half-sweep / selection /
// objective entry points declared in include/coreals.h.
#include <cstdio>
#include <cstring>
#include <new>

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
    int64_t *class_count;  // [2 * NCLASS]
    int64_t *max_deg;      // [2]
    int *err_flags;
    double *obj_partials;
    double *obj_out;
    void *temp;
    size_t temp_bytes;
    size_t total;
};

Layout carve(const als_problem &p, void *base) {
    Carve c{reinterpret_cast<char *>(base), 0, 0};
    Layout L;
    L.col_ptr = c.take<int64_t>((size_t)p.n_m + 1);
    L.row_idx = c.take<int32_t>((size_t)p.nnz);
    L.val_t = c.take<float>((size_t)p.nnz);
    L.perm_u = c.take<int32_t>((size_t)p.n_u);
    L.perm_m = c.take<int32_t>((size_t)p.n_m);
    L.stats = c.take<unsigned long long>(NSTATS);
    L.class_count = c.take<int64_t>(2 * NCLASS);
    L.max_deg = c.take<int64_t>(2);
    L.err_flags = c.take<int>(4);
    L.obj_partials = c.take<double>((size_t)5 * objective_blocks());
    L.obj_out = c.take<double>(4);
    size_t tb = csc_temp_bytes(p.nnz, p.n_m);
    size_t tp = perm_temp_bytes(p.n_u > p.n_m ? p.n_u : p.n_m);
    L.temp_bytes = tb > tp ? tb : tp;
    L.temp = c.take<char>(L.temp_bytes);
    L.total = c.off;
    return L;
}

bool sizes_ok(const als_problem *p) {
    if (!p) return false;
    if (p->n_u < 0 || p->n_m < 0 || p->nnz < 0) return false;
    if (p->n_u > INT32_MAX || p->n_m > INT32_MAX || p->nnz > INT32_MAX) return false;
    if (p->n_f < 1 || p->n_f > NF) return false;
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

als_status run_half_sweep(als_ctx *c, int side, const float *other, float *out, als_sweep_stats *st) {
    if (!c) return ALS_E_STATE;
    if (!other || !out) return fail(c, ALS_E_ARG, "NULL factor pointer%s");
    if (other == out) return fail(c, ALS_E_ARG, "input and output factor matrices alias%s");
    const Side &S = c->side[side];
    HIP_CHECK(c, hipMemsetAsync(c->stats, 0, sizeof(unsigned long long) * NSTATS, c->stream));
    for (int cls = 0; cls < NCLASS; ++cls) {
        SweepArgs a;
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
        a.stats = c->stats;
        HIP_CHECK(c, launch_sweep_class(cls, a, c->stream));
    }
    if (st) {
        unsigned long long h[NSTATS];
        HIP_CHECK(c, hipMemcpyAsync(h, c->stats, sizeof(h), hipMemcpyDeviceToHost, c->stream));
        HIP_CHECK(c, hipStreamSynchronize(c->stream));
        st->n_empty = (int64_t)h[ST_EMPTY];
        st->n_singular_fallback = (int64_t)h[ST_FALLBACK];
        st->n_fp64_residual = (int64_t)h[ST_FP64RES];
        st->n_rows = S.n_rows;
    }
    return ALS_OK;
}

}  // namespace

extern "C" {

size_t als_workspace_size(const als_problem *p) {
    if (!sizes_ok(p)) return 0;
    return carve(*p, nullptr).total;
}

als_status als_init(const als_problem *p, als_ctx **out) {
    if (!out) return fail(nullptr, ALS_E_ARG, "out is NULL%s");
    *out = nullptr;
    if (!sizes_ok(p)) return fail(nullptr, ALS_E_ARG, "invalid sizes (need 1 <= n_f <= 64, sizes < 2^31)%s");
    if (!(p->lambda >= 0.0)) return fail(nullptr, ALS_E_ARG, "lambda must be >= 0%s");
    if (p->budget_den == 0 || p->budget_num == 0 || p->budget_num > p->budget_den)
        return fail(nullptr, ALS_E_ARG, "budget rate must satisfy 0 < num <= den%s");
    if (p->min_keep < 0) return fail(nullptr, ALS_E_ARG, "min_keep must be >= 0%s");
    if (p->precision != ALS_PREC_FP32)
        return fail(nullptr, ALS_E_ARG, "precision not supported by this build%s");
    if (!p->row_ptr || (p->nnz > 0 && (!p->col_idx || !p->val)))
        return fail(nullptr, ALS_E_ARG, "NULL CSR pointer%s");
    Layout probe = carve(*p, nullptr);
    if (!p->workspace || p->workspace_bytes < probe.total)
        return fail(nullptr, ALS_E_NOMEM, "workspace too small (see als_workspace_size)%s");

    als_ctx *c = new (std::nothrow) als_ctx();
    if (!c) return fail(nullptr, ALS_E_NOMEM, "host allocation failed%s");
    c->p = *p;
    c->stream = reinterpret_cast<hipStream_t>(p->stream);
    Layout L = carve(*p, p->workspace);
    c->col_ptr = L.col_ptr;
    c->row_idx = L.row_idx;
    c->val_t = L.val_t;
    c->stats = L.stats;
    c->obj_partials = L.obj_partials;
    c->obj_out = L.obj_out;
    c->temp = L.temp;
    c->temp_bytes = L.temp_bytes;

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

    // 2. column view
    INIT_HIP(build_csc(p->n_u, p->n_m, p->nnz, p->row_ptr, p->col_idx, p->val, L.col_ptr, L.row_idx, L.val_t,
                       L.temp, s));

    // 3. schedules
    Side &U = c->side[0];
    U.n_rows = p->n_u;
    U.n_other = p->n_m;
    U.ptr = p->row_ptr;
    U.idx = p->col_idx;
    U.val = p->val;
    U.perm = L.perm_u;
    Side &M = c->side[1];
    M.n_rows = p->n_m;
    M.n_other = p->n_u;
    M.ptr = L.col_ptr;
    M.idx = L.row_idx;
    M.val = L.val_t;
    M.perm = L.perm_m;
    int64_t host_counts[2 * NCLASS];
    int64_t host_max[2];
    for (int sd = 0; sd < 2; ++sd) {
        Side &S = c->side[sd];
        INIT_HIP(build_schedule(S.n_rows, S.ptr, p->budget_num, p->budget_den, p->min_keep, S.perm,
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
    SelectArgs a;
    a.ptr = S.ptr;
    a.idx = S.idx;
    a.other = other;
    a.row_begin = row_begin;
    a.row_end = row_end;
    a.nf = c->p.n_f;
    a.num = c->p.budget_num;
    a.den = c->p.budget_den;
    a.min_keep = c->p.min_keep;
    a.sel_ptr = sel_ptr;
    a.sel_pos = sel_pos;
    HIP_CHECK(c, launch_select(a, c->stream));
    return ALS_OK;
}

als_status objective(als_ctx *c, const float *U, const float *M, als_objective *out) {
    if (!c) return ALS_E_STATE;
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

void als_destroy(als_ctx *c) { delete c; }

const char *als_last_error(const als_ctx *c) { return c ? c->err.c_str() : g_init_error.c_str(); }

}  // extern "C"
