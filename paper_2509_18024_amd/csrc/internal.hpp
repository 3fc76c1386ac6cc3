// Internal declarations of the core-elements ALS library (gfx950).
// Not part of the public ABI; see include/coreals.h for that.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/coreals.h"

namespace coreals {

// Compile-time rank of the register-resident regression (lane a owns row a of
// the n_f x n_f system).  Problems with n_f < 64 are padded with identity rows.
constexpr int NF = 64;
// Widest rank: ranks 64 < n_f <= NFW take the wide-rank kernels (wide.hip),
// one workgroup per row with the n_f x n_f system spread over its threads.
constexpr int NFW = 128;
// Waves per workgroup of the row kernels; each wave solves its own rows.
constexpr int WPB = 4;
// Rows of the design matrix staged in LDS per chunk.
constexpr int CK = 64;
// Keys per column the heavy-row selection ranks directly in LDS (the lists
// share LDS with the radix histogram).
constexpr int HEAVY_CAP = 62;
// Defaults of the schedule (als_problem fields set to 0 select them).
constexpr int DEFAULT_HEAVY_N = 1024;    // light rows have degree <= this
constexpr int DEFAULT_CHUNK = 1024;      // entries per partial Gram of a heavy row
constexpr int64_t PAIR_CAP = 65536;      // partial systems held in scratch at once
constexpr int64_t PAIR_CAP_WIDE = 8192;  // the same at ranks above 64 (66 KB per system)
// Per-row precision of the BF16 + refinement mode ALS_PREC_AUTO, from the
// condition estimate kappa = |A|_inf |A^-1 e|_inf / |e|_inf of the row's system
// (one extra solve with the kept LU factors, e = kappa_probe):
//  - kappa > KAPPA_BF16 = 2^8: one refinement step from bf16-rounded products
//    (unit roundoff 2^-8) is not expected to contract, so the row's Gram is
//    built again with FP32 products (exact three-way split) and refactored;
//  - lambda < FP64_LAMBDA and kappa > KAPPA_FP64 = 2^10: an FP32 residual
//    would limit the refined row to about kappa 2^-24, above 6e-5, so its
//    refinement residual is accumulated in FP64.
constexpr float KAPPA_BF16 = 256.f;
constexpr double FP64_LAMBDA = 1e-3;
constexpr float KAPPA_FP64 = 1024.f;
// fp64res modes of HeavyArgs
enum Fp64Mode : int { RES_FP32 = 0, RES_FP64 = 1, RES_PER_ROW = 2 };

// Degree classes that schedule a half-sweep.  Light rows (degree <= heavy_n
// and budget s <= 32) are solved by one wavefront each: FULL when s == n
// (r = 1, or tiny rows), otherwise the smallest insertion-network class whose
// capacity holds s.  Every other row is HEAVY (radix selection by a workgroup,
// Gram split into chunks, separate solve).
enum RowClass : int {
    CLS_FULL = 0,
    CLS_NET1 = 1,
    CLS_NET2 = 2,
    CLS_NET4 = 3,
    CLS_NET8 = 4,
    CLS_NET16 = 5,
    CLS_NET32 = 6,
    CLS_HEAVY = 7,
    NCLASS = 8
};

// Index of the calling wavefront in its workgroup, as a wave-uniform value
// (threadIdx.x alone is taken as divergent, which would put every row index
// derived from it, and the loops it bounds, in vector registers).
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

__host__ __device__ inline int64_t budget_of(int64_t n, uint32_t num, uint32_t den, int32_t min_keep) {
    int64_t s = (n * (int64_t)num) / (int64_t)den;
    if (s < min_keep) s = min_keep;
    if (s > n) s = n;
    if (s < 0) s = 0;
    return s;
}

__host__ __device__ inline int class_of(int64_t n, int64_t s, int64_t heavy_n) {
    if (n > heavy_n) return CLS_HEAVY;
    if (s == n) return CLS_FULL;
    if (s <= 1) return CLS_NET1;
    if (s <= 2) return CLS_NET2;
    if (s <= 4) return CLS_NET4;
    if (s <= 8) return CLS_NET8;
    if (s <= 16) return CLS_NET16;
    if (s <= 32) return CLS_NET32;
    return CLS_HEAVY;
}

// Work plan of the heavy rows of one side: the rows are perm[heavy_begin ..
// heavy_begin + n_heavy); heavy slot t is the t-th of them.  Each row is cut
// into ceil(n / chunk) pairs (slot, chunk); pairs are processed in batches
// that fit the partial-system scratch.
struct HeavyPlan {
    int64_t n_heavy = 0;
    int64_t n_pairs = 0;
    int32_t *pair_slot = nullptr;   // [n_pairs]
    int32_t *pair_chunk = nullptr;  // [n_pairs]
    int64_t *pair_off = nullptr;    // [n_heavy + 1]
    int32_t *cutT = nullptr;        // [n_heavy * 64]
    int32_t *cutK = nullptr;
    struct Batch {
        int64_t slot_begin, slot_end, pair_begin, pair_end;
    };
    std::vector<Batch> batches;
};

// One side of the problem (users: CSR of R; items: CSC of R).
struct Side {
    int64_t n_rows = 0;
    int64_t n_other = 0;
    const int64_t *ptr = nullptr;
    const int32_t *idx = nullptr;
    const float *val = nullptr;
    int32_t *perm = nullptr;           // rows ordered by (class, degree descending)
    int64_t class_off[NCLASS + 1] = {};  // host copy of class boundaries in perm
    int64_t max_deg = 0;
    HeavyPlan heavy;
};

// Device-side counters of per-row events (cleared before each half-sweep).
// Kernel groups timed by als_profile_begin / als_profile_end, per side.
constexpr int NPROF = 12;
enum ProfSlot : int { PROF_HSELECT = 7, PROF_HGRAM = 8, PROF_HSOLVE = 9, PROF_HRESID = 10, PROF_HREFINE = 11 };

enum StatSlot : int {
    ST_EMPTY = 0,
    ST_FALLBACK = 1,
    ST_FP64RES = 2,
    ST_ROWS = 3,
    ST_FOLDIN_EXACT = 4,
    ST_FP32GRAM = 5,
    ST_MAXRES = 6,  // bits of the largest relative refinement residual (non-negative double)
    ST_HINTED = 7,  // heavy rows whose selection started from the previous cuts
    ST_PIVOTED = 8, // light core and heavy rows whose unpivoted elimination was rejected
    NSTATS = 10
};

struct SweepArgs {
    const int64_t *ptr;
    const int32_t *idx;
    const float *val;
    const float *other;      // [n_other * nf]
    float *out;              // [n_rows * nf]
    const int32_t *perm;     // row list
    int64_t count;           // rows in the list
    int32_t nf;
    float lam;
    uint32_t num, den;
    int32_t min_keep;
    unsigned long long *stats;
    unsigned int *queue;     // row counter of this class (persistent launch)
    // fold-in check mode: candidate answers, acceptance threshold on the
    // relative residual, per-row outcome (0 candidate kept, 1 solved) and residual
    const float *guess;
    float tol;
    int32_t *path;
    float *rho;
    // fast variant: the global cut of `other` (column a keeps key > gT[a], or
    // key == gT[a] and row index <= gK[a]) replaces each row's selection
    const int32_t *gT;
    const int32_t *gK;
    // implicit feedback: confidence weight and the Gram of `other` (NF x NF)
    float alpha;
    const float *G;
    // Woodbury classes: rows the n x n form does not solve are listed here
    // (fb_rows[0 .. *fb_count)) and solved by a second launch, whose row
    // count is *count_dev (nullptr: count)
    int32_t *fb_rows;
    unsigned int *fb_count;
    unsigned int *fb_queue;
    const unsigned int *count_dev;
};

struct HeavyArgs {
    const int64_t *ptr;
    const int32_t *idx;
    const float *val;
    const float *other;
    int64_t other_rows;       // rows of `other` (0: unknown)
    const uint16_t *key16;    // bits 30..15 of `other`'s entries, or nullptr (selection)
    float *out;
    const int32_t *rows;      // heavy slot -> row (nullptr: row_begin + slot)
    int64_t count;            // heavy rows
    int32_t nf;
    float lam;
    uint32_t num, den;
    int32_t min_keep;
    int32_t heavy_n;
    int32_t chunk;
    const int32_t *pair_slot;
    const int32_t *pair_chunk;
    const int64_t *pair_off;
    int32_t *cutT;            // [heavy slot * cstride + column]
    int32_t hint;             // selection: cutT holds this side's previous cuts (-1 where none)
    int32_t *cutK;
    int32_t cstride;          // cut entries per row: 64, or NFW at ranks above 64
    int32_t col_base;         // selection: the launch ranks columns col_base .. + 63
    float *partials;
    double *resid;            // [pair_cap * 2 * cut stride]: per pair, residual and
                              // right-hand side shares (refinement, fold-in check)
    int32_t refine;           // solve: 0 first solve, 1 apply the refinement step
    int32_t keep;             // first solve keeps its LU factors for the refinement step
    int32_t fp64res;          // Fp64Mode of the refinement residual
    int32_t *flag;            // per heavy slot: 0, or the pass that redoes the row
    int32_t implicit;         // implicit feedback: X*^T W X + G + lambda E, W = alpha y
    float alpha;
    const float *G;           //   the Gram of `other`, NF x NF
    int32_t unif;             // UNIF: entries outside the row's uniform draw are zeroed
    uint64_t seed;            //   (key = unif_key(seed, row, n_cols, col) against the
    int64_t n_cols;           //   row's cut uT / uK), lambda s on the diagonal
    const uint32_t *uT;
    const int32_t *uK;
    int32_t gpos;             // fast variant: one cut per column (cstride 0), ties
                              // decided by the row index of `other`, not the position
    int32_t pass;             // 0: all rows; 1 (wide ranks): rows with a singular core
                              // system, from the full data; 2 (ALS_PREC_AUTO): rows
                              // whose Gram is built again with FP32 products
    unsigned long long *stats;
    unsigned int *queue;      // heavy-row selection counter (nullptr: grid-stride)
    // fold-in check mode (see SweepArgs); with path set, the Gram, solve and
    // refinement kernels skip rows whose candidate was accepted (path 0)
    const float *guess;
    float tol;
    int32_t *path;
    float *rho;
};

struct SelectArgs {
    const int64_t *ptr;
    const int32_t *idx;
    const float *other;
    int64_t row_begin, row_end;
    int32_t nf;
    uint32_t num, den;
    int32_t min_keep;
    int32_t heavy_n;
    const int64_t *sel_ptr;
    int32_t *sel_pos;
    const int32_t *cutT;      // cuts of heavy rows, indexed by row - row_begin
    const int32_t *cutK;
};

// Fold-in check mode of a users half-sweep (see SweepArgs).
struct CheckArgs {
    const float *guess;
    float tol;
    int32_t *path;
    float *rho;
};

// launchers (sweep.hip)
hipError_t launch_sweep_class(int cls, const SweepArgs &a, int max_blocks, hipStream_t s);
hipError_t launch_select(const SelectArgs &a, hipStream_t s);
hipError_t launch_check_class(int cls, const SweepArgs &a, int max_blocks, hipStream_t s);

// launchers (heavy.hip)
hipError_t launch_heavy_select(const HeavyArgs &a, int64_t row_begin, hipStream_t s);
hipError_t launch_key16(const float *other, int64_t count, uint16_t *key16, hipStream_t s);
hipError_t launch_heavy_gram(const HeavyArgs &a, int64_t pair_begin, int64_t pair_end, hipStream_t s);
hipError_t launch_heavy_solve(const HeavyArgs &a, int64_t slot_begin, int64_t slot_end, int64_t pair_base,
                              hipStream_t s);
hipError_t launch_heavy_gram_bf16(const HeavyArgs &a, int64_t pair_begin, int64_t pair_end, hipStream_t s);
hipError_t launch_heavy_resid(const HeavyArgs &a, int64_t pair_begin, int64_t pair_end, hipStream_t s);
hipError_t launch_heavy_check(const HeavyArgs &a, int64_t pair_begin, int64_t pair_end, hipStream_t s);
hipError_t launch_heavy_check_reduce(const HeavyArgs &a, int64_t slot_begin, int64_t slot_end, int64_t pair_base,
                                     hipStream_t s);

// launchers (wide.hip): ranks 64 < n_f <= NFW.  Every non-empty row is a
// heavy row (cuts from launch_heavy_select, one launch per 64 columns).
hipError_t launch_wide_empty(const SweepArgs &a, hipStream_t s);
hipError_t launch_wide_gram(const HeavyArgs &a, int64_t pair_begin, int64_t pair_end, bool x6, hipStream_t s);
hipError_t launch_wide_solve(const HeavyArgs &a, int64_t slot_begin, int64_t slot_end, int64_t pair_base,
                             hipStream_t s);
hipError_t launch_wide_resid(const HeavyArgs &a, int64_t pair_begin, int64_t pair_end, hipStream_t s);
hipError_t launch_select_wide(const SelectArgs &a, hipStream_t s);

// launchers (fast.hip): the global cut of the fast variant, T / K device [64]
size_t global_select_state_bytes();
hipError_t launch_global_select(const float *other, int64_t n_other, int nf, uint32_t num, uint32_t den,
                                int32_t min_keep, void *state, int32_t *T, int32_t *K, hipStream_t s);
// light rows of the fast variant (sweep.hip): every class, one kernel
hipError_t launch_sweep_fast(const SweepArgs &a, int max_blocks, hipStream_t s);

// implicit feedback (implicit.hip): the Gram of `other` (float NF x NF, from
// FP64 sums; partials: blocks x NF x NF doubles) and the light rows
int implicit_gram_blocks();
hipError_t launch_global_gram(const float *other, int64_t n_other, int nf, double *partials, float *G,
                              hipStream_t s);
hipError_t launch_sweep_implicit(int cls, const SweepArgs &a, int max_blocks, hipStream_t s);

// UNIF (unif.hip): each row's cut of the uniform draw, the light rows
hipError_t launch_unif_select(const int64_t *ptr, const int32_t *idx, int64_t n_rows, int64_t n_cols, uint32_t num,
                              uint32_t den, int32_t min_keep, uint64_t seed, uint32_t *T, int32_t *K,
                              hipStream_t s);
hipError_t launch_sweep_unif(const SweepArgs &a, uint64_t seed, int64_t n_cols, const uint32_t *T, const int32_t *K,
                             int max_blocks, hipStream_t s);

// launchers (setup.hip)
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s);
size_t csc_temp_bytes(int64_t nnz, int64_t n_rows);
size_t perm_temp_bytes(int64_t n_rows);
hipError_t launch_validate(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *ptr,
                           const int32_t *idx, const float *val, int check_values,
                           int *err_flags, hipStream_t s);
hipError_t build_csc(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                     const int32_t *col_idx, const float *val, int64_t *col_ptr,
                     int32_t *row_idx, float *val_t, void *temp, hipStream_t s);
hipError_t build_schedule(int64_t n_rows, const int64_t *ptr, uint32_t num, uint32_t den,
                          int32_t min_keep, int32_t heavy_n, int32_t *perm, int64_t *class_count_dev,
                          int64_t *max_deg_dev, void *temp, hipStream_t s);
hipError_t launch_select_sizes(const int64_t *ptr, int64_t row_begin, int64_t row_end, int32_t nf,
                               uint32_t num, uint32_t den, int32_t min_keep, int64_t *sel_ptr,
                               void *temp, hipStream_t s);

// launchers (objective.hip)
int objective_blocks();
hipError_t launch_objective(int64_t n_u, int64_t n_m, int32_t nf, const int64_t *row_ptr,
                            const int32_t *col_idx, const float *val, const int64_t *col_ptr,
                            const float *U, const float *M, double lam, double *partials,
                            double *out4, hipStream_t s);

}  // namespace coreals

struct als_ctx {
    als_problem p{};
    hipStream_t stream = nullptr;
    coreals::Side side[2];
    int64_t *col_ptr = nullptr;
    int32_t *row_idx = nullptr;
    float *val_t = nullptr;
    unsigned long long *stats = nullptr;  // [NSTATS]
    double *obj_partials = nullptr;
    double *obj_out = nullptr;            // [4]
    float *partials = nullptr;            // [pair_cap * (NF + 1) * 64]
    double *resid = nullptr;              // [pair_cap * 128]
    uint16_t *key16 = nullptr;            // [max(n_u, n_m) * n_f] when budget < 1
    int32_t heavy_n = coreals::DEFAULT_HEAVY_N;
    int32_t chunk = coreals::DEFAULT_CHUNK;
    int64_t pair_cap = coreals::PAIR_CAP;
    int32_t light_blocks = 0;  // grid of the persistent light-row kernels (0: one row per wave)
    bool bf16 = false;     // heavy-row Gram on bf16 MFMA + one refinement step
    int fp64res = 0;       // Fp64Mode of the refinement residual
    bool wide = false;     // 64 < n_f <= NFW: wide-rank kernels for every row
    bool fast = false;     // ALS_FAST_VARIANT: one global sketch per half-sweep
    bool unif = false;     // ALS_UNIF: uniform subsampling (the comparator)
    bool implicit = false; // ALS_IMPLICIT: implicit-feedback Core-ALS
    int32_t *fb_rows = nullptr;   // rows the Woodbury classes leave to the n_f x n_f solve
    double *gram_part = nullptr;  // implicit: per-block partial Grams
    float *G = nullptr;           // implicit: the Gram of the other factor matrix
    uint64_t seed = 0;     // UNIF draws (als_set_sample_seed)
    uint32_t *uT[2] = {nullptr, nullptr};  // UNIF: per-row cut of each side
    int32_t *uK[2] = {nullptr, nullptr};
    void *gsel = nullptr;  // fast variant: radix-select state and the cut
    int32_t *gT = nullptr, *gK = nullptr;
    int32_t *flag[2] = {nullptr, nullptr};  // per heavy slot: the pass that redoes the row
    void *temp = nullptr;
    size_t temp_bytes = 0;
    std::string err;
    // kernel timing (als_profile_begin / als_profile_end)
    struct Mark {
        hipEvent_t start, stop;
        int side, cls;
    };
    bool profiling = false;
    std::vector<Mark> marks;
    // HIP graphs of the two half-sweeps, keyed by the factor pointers
    struct Graph {
        hipGraphExec_t exec = nullptr;
        const float *other = nullptr;
        float *out = nullptr;
        uint64_t seed = 0;  // UNIF draws are part of the captured launches
    };
    bool use_graphs = false;
    Graph graph[2];
    unsigned int *queues = nullptr;  // [2 * 16] row counters
    bool users_only = false;         // ALS_USERS_ONLY: no column view, users side only
};

namespace coreals {

// Per-call scratch of a half-sweep: event counters, row-queue counters,
// heavy-row partial systems and residuals.  Batches of the heavy-row plan
// hold at most the context's pair_cap pairs, which the partial and residual
// arrays must fit.
struct SweepScratch {
    unsigned long long *stats;  // [NSTATS]
    unsigned int *queues;       // [2 * 16]
    float *partials;            // [pair_cap * (NF + 1) * 64]
    double *resid;              // [pair_cap * 128]
};

// Enqueue one half-sweep of c with the given scratch (no graph, no profiling
// marks); argument errors as for half_sweep_users / half_sweep_items.
als_status enqueue_half_sweep_scratch(als_ctx *c, int side, const float *other, float *out, const SweepScratch &sc);
// Copy per-row event counters to st (syncs the context's stream).
als_status fill_stats(als_ctx *c, int side, const unsigned long long *stats, als_sweep_stats *st);

// Users half-sweep of c in fold-in check mode (stats cleared first); used by
// the fold-in entry points.
als_status enqueue_checked_users(als_ctx *c, const float *M, float *out, const CheckArgs &chk);
// Copy the per-row event counters to the host (syncs the context's stream).
als_status read_stats(als_ctx *c, unsigned long long *h);
// Record an error message on c and return st.
als_status set_error(als_ctx *c, als_status st, const char *msg);

}  // namespace coreals
