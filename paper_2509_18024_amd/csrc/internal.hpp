// Internal declarations of the core-elements ALS library (gfx950).
// Not part of the public ABI; see include/coreals.h for that.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/coreals.h"

namespace coreals {

// Compile-time rank of the register-resident regression (lane a owns row a of
// the n_f x n_f system).  Problems with n_f < 64 are padded with identity rows.
constexpr int NF = 64;
// Waves per workgroup of the row kernels; each wave solves its own rows.
constexpr int WPB = 4;
// Rows of the design matrix staged in LDS per chunk (one per lane).
constexpr int CK = 64;

// Degree classes that schedule a half-sweep.  A row with budget s and degree n
// goes to FULL when s == n (r = 1, or tiny rows), otherwise to the smallest
// insertion-network class whose capacity holds s, otherwise to RADIX.
enum RowClass : int {
    CLS_FULL = 0,
    CLS_NET1 = 1,
    CLS_NET2 = 2,
    CLS_NET4 = 3,
    CLS_NET8 = 4,
    CLS_NET16 = 5,
    CLS_NET32 = 6,
    CLS_RADIX = 7,
    NCLASS = 8
};

__host__ __device__ inline int64_t budget_of(int64_t n, uint32_t num, uint32_t den, int32_t min_keep) {
    int64_t s = (n * (int64_t)num) / (int64_t)den;
    if (s < min_keep) s = min_keep;
    if (s > n) s = n;
    if (s < 0) s = 0;
    return s;
}

__host__ __device__ inline int class_of(int64_t n, int64_t s) {
    if (s == n) return CLS_FULL;
    if (s <= 1) return CLS_NET1;
    if (s <= 2) return CLS_NET2;
    if (s <= 4) return CLS_NET4;
    if (s <= 8) return CLS_NET8;
    if (s <= 16) return CLS_NET16;
    if (s <= 32) return CLS_NET32;
    return CLS_RADIX;
}

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
};

// Device-side counters of per-row events (cleared before each half-sweep).
enum StatSlot : int { ST_EMPTY = 0, ST_FALLBACK = 1, ST_FP64RES = 2, ST_ROWS = 3, NSTATS = 8 };

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
};

struct SelectArgs {
    const int64_t *ptr;
    const int32_t *idx;
    const float *other;
    int64_t row_begin, row_end;
    int32_t nf;
    uint32_t num, den;
    int32_t min_keep;
    const int64_t *sel_ptr;
    int32_t *sel_pos;
};

// launchers (sweep.hip)
hipError_t launch_sweep_class(int cls, const SweepArgs &a, hipStream_t s);
hipError_t launch_select(const SelectArgs &a, hipStream_t s);

// launchers (setup.hip)
size_t csc_temp_bytes(int64_t nnz, int64_t n_rows);
size_t perm_temp_bytes(int64_t n_rows);
hipError_t launch_validate(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *ptr,
                           const int32_t *idx, const float *val, int check_values,
                           int *err_flags, hipStream_t s);
hipError_t build_csc(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                     const int32_t *col_idx, const float *val, int64_t *col_ptr,
                     int32_t *row_idx, float *val_t, void *temp, hipStream_t s);
hipError_t build_schedule(int64_t n_rows, const int64_t *ptr, uint32_t num, uint32_t den,
                          int32_t min_keep, int32_t *perm, int64_t *class_count_dev,
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
    void *temp = nullptr;
    size_t temp_bytes = 0;
    std::string err;
};
