// Per-wavefront building blocks of one row regression (gfx950), shared by the
// light-row kernels (one wavefront per row) and the heavy-row kernels.
//
// Lane a owns column a of the design matrix X (for CES) and row a of the
// n_f x n_f system (for the solve).  Design rows X[k] = other[idx[k]] are
// staged in LDS in chunks of CK; keys are the bit patterns of |x| compared as
// integers, so the selection is exact.
#pragma once

#include <utility>

#include "internal.hpp"

namespace coreals {

constexpr int KEYMASK = 0x7FFFFFFF;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float readlane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int key_of(float x) { return __float_as_int(x) & KEYMASK; }

// Key of entry (row, col) in the UNIF draw of a seed: the upper 32 bits of
// splitmix64 (Steele, Lea and Flood, 2014) at seed * 0x9E3779B97F4A7C15 +
// row * n_cols + col.  A row's draw keeps its budget of smallest keys.
__device__ __forceinline__ uint32_t unif_key(uint64_t seed, int64_t row, int64_t n_cols, int32_t col) {
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + (uint64_t)(row * n_cols + (int64_t)col) + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return (uint32_t)((z ^ (z >> 31)) >> 32);
}

// The lane index as a value the compiler cannot hoist out of a row loop.
// Without it, the 64 per-step lane comparisons of the solve are precomputed
// once per kernel as scalar masks and spilled.
__device__ __forceinline__ int opaque_lane(int lane) {
    asm volatile("" : "+v"(lane));
    return lane;
}

// One wavefront's LDS: ROWS staged design rows (a chunk), their ratings and
// the solve's scratch.  The classes of short rows stage 32-row chunks, which
// halves the LDS per wavefront.
// COLS (fast variant): the staged rows' indices into `other` are kept too,
// and ties of the cut are decided by them instead of the positions.
// Columns per panel of the blocked elimination.
constexpr int LU_BLK = 4;

template <int ROWS, bool COLS = false>
struct alignas(16) WaveLdsT {
    static constexpr int rows = ROWS;
    static constexpr bool has_cols = COLS;
    float X[ROWS][NF + 4];    // staged design rows (select, Gram)
    float y[ROWS];
    float urhs[2 * NF];       // solve: solution components parked by the back substitution
    double rres[ROWS];        // refinement: residuals y_k - x_k . u of the staged rows
    float pbuf[LU_BLK][NF];   // blocked elimination: the panel's pivot rows
    int col[COLS ? ROWS : 1]; // indices of the staged rows into `other`
};
using WaveLds = WaveLdsT<CK>;

// The value a cut's tie rule compares for staged row k of the chunk at k0:
// its position in the row, or (fast variant) its row index in `other`.
template <class LDS>
__device__ __forceinline__ int tie_pos(const LDS &L, int k0, int k) {
    if constexpr (LDS::has_cols) return L.col[k];
    else return k0 + k;
}

// Largest value over the wave of a non-negative-or-(-1) integer key: DPP
// within each row of 16 lanes (xor 1, xor 2, half-row and row mirrors), then
// the four row results through scalar registers.
__device__ __forceinline__ int wave_max_key(int v) {
    // every lane has a source lane in these patterns; with bound_ctrl set the
    // moves fold into the max instructions as DPP operands
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true));   // quad_perm [1,0,3,2]
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true));   // quad_perm [2,3,0,1]
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true));  // row_half_mirror
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true));  // row_mirror
    // across rows: lane 15 into row 1 and lane 47 into row 3, then lane 31
    // into rows 2 and 3; lane 63 ends with the wave's maximum
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// Per-row view used by the device helpers.
struct RowCtx {
    const int32_t *idx;
    const float *val;
    const float *other;
    int64_t beg;
    int n;
    int nf;
    bool vec4;
    int staged;  // chunk start currently in LDS, -1 if none
};

// Gather chunk [k0, k0 + cnt) of the design matrix into LDS, cnt = min(rows,
// n - k0), from its column indices and ratings already loaded: lane j < cnt
// holds those of position k0 + j (col = 0 and yv = 0 elsewhere).
template <class LDS>
__device__ __forceinline__ void stage_loaded(LDS &L, RowCtx &r, int k0, int col, float yv, int lane) {
    wave_sync();
    const int cnt = min(LDS::rows, r.n - k0);
    if (lane < LDS::rows) L.y[lane] = yv;
    if constexpr (LDS::has_cols)
        if (lane < LDS::rows) L.col[lane] = col;
    // Gathers are unconditional (positions past cnt read factor row 0, which
    // exists) so the whole chunk's loads are in flight together; the padding
    // is zeroed afterwards.
    if (r.vec4) {
        float4 v[LDS::rows / 4];
#pragma unroll
        for (int t = 0; t < LDS::rows / 4; ++t) {
            const int kk = t * 4 + (lane >> 4);
            const int c = __shfl(col, kk);
            v[t] = *reinterpret_cast<const float4 *>(r.other + (size_t)c * NF + (lane & 15) * 4);
        }
#pragma unroll
        for (int t = 0; t < LDS::rows / 4; ++t) {
            const int kk = t * 4 + (lane >> 4);
            if (kk >= cnt) v[t] = make_float4(0.f, 0.f, 0.f, 0.f);
            *reinterpret_cast<float4 *>(&L.X[kk][(lane & 15) * 4]) = v[t];
        }
    } else {
        const int lc = min(lane, r.nf - 1);
        for (int kk = 0; kk < LDS::rows; ++kk) {
            const int c = __shfl(col, kk);
            const float v = r.other[(size_t)c * r.nf + lc];
            L.X[kk][lane] = (kk < cnt && lane < r.nf) ? v : 0.f;
        }
    }
    r.staged = k0;
    wave_sync();
}

// Gather chunk [k0, k0 + min(rows, n - k0)) of the design matrix into LDS.
template <class LDS>
__device__ __forceinline__ void stage(LDS &L, RowCtx &r, int k0, int lane) {
    if (r.staged == k0) return;
    const int cnt = min(LDS::rows, r.n - k0);
    int col = 0;
    float yv = 0.f;
    if (lane < cnt) {
        col = r.idx[r.beg + k0 + lane];
        if (r.val) yv = r.val[r.beg + k0 + lane];
    }
    stage_loaded(L, r, k0, col, yv, lane);
}

// Selection result for the lane's column: k is kept iff
// key > T, or key == T and position <= K.  none: nothing kept (s == 0).
struct Cut {
    int T;
    int K;
    bool none;
    bool all;
};

__device__ __forceinline__ bool kept(const Cut &c, int key, int pos) {
    return c.all || (!c.none && (key > c.T || (key == c.T && pos <= c.K)));
}

// Position of the need-th key equal to T in ascending order (lanes with tie).
template <class LDS>
__device__ __forceinline__ void tie_pass(LDS &L, RowCtx &r, int lane, bool tie, int T, int need, int &K) {
    if (__ballot(tie) == 0ull) return;
    int cnt = 0;
    for (int k0 = 0; k0 < r.n; k0 += LDS::rows) {
        stage(L, r, k0, lane);
        const int m = min(LDS::rows, r.n - k0);
        for (int k = 0; k < m; ++k) {
            const int key = key_of(L.X[k][lane]);
            if (tie && key == T) {
                ++cnt;
                if (cnt == need) K = k0 + k;
            }
        }
    }
}

// Compare-exchange leaving the larger key in a.
__device__ __forceinline__ void cex_desc(int &a, int &b) {
    const int hi = max(a, b);
    b = min(a, b);
    a = hi;
}

// Bitonic sort of N keys (N a power of two) into descending order.
template <int N>
__device__ __forceinline__ void bitonic_sort_desc(int (&v)[N]) {
#pragma unroll
    for (int k = 2; k <= N; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    if ((i & k) == 0) cex_desc(v[i], v[l]);
                    else cex_desc(v[l], v[i]);
                }
            }
}

// Top-s of the lane's column for the larger classes, by blocks of SMAX keys:
// each block is sorted, merged with the kept keys (both descending) by one
// bitonic split, which leaves the SMAX largest of the two as a bitonic
// sequence, and that is sorted again.  The same kept multiset, threshold and
// largest dropped key as select_net, in about a third of the instructions.
template <int SMAX, class LDS>
__device__ __forceinline__ Cut select_merge(LDS &L, RowCtx &r, int s, int lane) {
    int kept_[SMAX];
#pragma unroll
    for (int j = 0; j < SMAX; ++j) kept_[j] = (j < SMAX - s) ? 0x7FFFFFFF : -1;
    int D = -1;  // largest key that fell out
    for (int k0 = 0; k0 < r.n; k0 += LDS::rows) {
        stage(L, r, k0, lane);
        const int m = min(LDS::rows, r.n - k0);
        for (int b0 = 0; b0 < m; b0 += SMAX) {
            int blk[SMAX];
#pragma unroll
            for (int j = 0; j < SMAX; ++j) blk[j] = b0 + j < m ? key_of(L.X[b0 + j][lane]) : -1;
            bitonic_sort_desc<SMAX>(blk);
#pragma unroll
            for (int j = 0; j < SMAX; ++j) {
                const int a = kept_[j], b = blk[SMAX - 1 - j];
                kept_[j] = max(a, b);
                D = max(D, min(a, b));
            }
            // kept_ is bitonic: merge it into descending order
#pragma unroll
            for (int j = SMAX >> 1; j > 0; j >>= 1)
#pragma unroll
                for (int i = 0; i < SMAX; ++i) {
                    const int l = i ^ j;
                    if (l > i) cex_desc(kept_[i], kept_[l]);
                }
        }
    }
    Cut c;
    c.T = kept_[SMAX - 1];
    c.none = false;
    c.all = false;
    int gt = 0;
#pragma unroll
    for (int j = 0; j < SMAX; ++j) gt += kept_[j] > c.T;
    gt -= SMAX - s;
    const int need = s - gt;
    const bool tie = (D == c.T);
    c.K = 0x7FFFFFFF;
    tie_pass(L, r, lane, tie, c.T, need, c.K);
    return c;
}

// Top-s by an insertion network of SMAX registers kept in descending order.
// Unused slots (SMAX - s of them) hold INT_MAX and pass every key through.
template <int SMAX, class LDS>
__device__ __forceinline__ Cut select_net(LDS &L, RowCtx &r, int s, int lane) {
    int kept_[SMAX];
#pragma unroll
    for (int j = 0; j < SMAX; ++j) kept_[j] = (j < SMAX - s) ? 0x7FFFFFFF : -1;
    int D = -1;  // largest key that fell out of the network
    for (int k0 = 0; k0 < r.n; k0 += LDS::rows) {
        stage(L, r, k0, lane);
        const int m = min(LDS::rows, r.n - k0);
        for (int k = 0; k < m; ++k) {
            int v = key_of(L.X[k][lane]);
#pragma unroll
            for (int j = 0; j < SMAX; ++j) {
                const int hi = max(kept_[j], v);
                v = min(kept_[j], v);
                kept_[j] = hi;
            }
            D = max(D, v);
        }
    }
    Cut c;
    c.T = kept_[SMAX - 1];
    c.none = false;
    c.all = false;
    int gt = 0;
#pragma unroll
    for (int j = 0; j < SMAX; ++j) gt += kept_[j] > c.T;
    gt -= SMAX - s;
    const int need = s - gt;
    const bool tie = (D == c.T);
    c.K = 0x7FFFFFFF;
    tie_pass(L, r, lane, tie, c.T, need, c.K);
    return c;
}

// Row a of X*^T X and entry a of X*^T y for the lane's column, summed over
// positions [kb, ke) of the row (chunks of CK staged in LDS; ascending k).
template <class LDS>
__device__ __forceinline__ void gram_range(LDS &L, RowCtx &r, const Cut &c, int kb, int ke, int lane,
                                           float (&A)[NF], float &rhs) {
#pragma unroll
    for (int b = 0; b < NF; ++b) A[b] = 0.f;
    rhs = 0.f;
    if (c.none) return;
    for (int k0 = kb; k0 < ke; k0 += LDS::rows) {
        stage(L, r, k0, lane);
        const int m = min(LDS::rows, ke - k0);
        for (int k = 0; k < m; ++k) {
            const float xa = L.X[k][lane];
            const float w = kept(c, key_of(xa), k0 + k) ? xa : 0.f;
#pragma unroll
            for (int b4 = 0; b4 < NF / 4; ++b4) {
                const float4 xr = *reinterpret_cast<const float4 *>(&L.X[k][b4 * 4]);
                A[4 * b4 + 0] = fmaf(w, xr.x, A[4 * b4 + 0]);
                A[4 * b4 + 1] = fmaf(w, xr.y, A[4 * b4 + 1]);
                A[4 * b4 + 2] = fmaf(w, xr.z, A[4 * b4 + 2]);
                A[4 * b4 + 3] = fmaf(w, xr.w, A[4 * b4 + 3]);
            }
            rhs = fmaf(w, L.y[k], rhs);
        }
    }
}

// The same row of X*^T X and entry of X*^T y, visiting only the lane's kept
// positions: per staged chunk each lane marks its kept positions in a 64-bit
// mask, then walks them in ascending order (the wave iterates as often as its
// busiest lane).  Only the zero products of the unkept positions are skipped,
// so the sums equal gram_range's.
// WEIGHTED (implicit feedback): row a of X*^T W X with W = diag(alpha y_k),
// and b_a = sum over kept k of x_ka (1 + alpha y_k).
template <class LDS, bool WEIGHTED = false>
__device__ __forceinline__ void gram_range_sparse(LDS &L, RowCtx &r, const Cut &c, int kb, int ke, int lane,
                                                  float (&A)[NF], float &rhs, float alpha = 0.f) {
#pragma unroll
    for (int b = 0; b < NF; ++b) A[b] = 0.f;
    rhs = 0.f;
    if (c.none) return;
    // chunks from the last one down: the selection leaves the last chunk of
    // the row staged, so one gather of the row is saved
    const int klast = kb + ((ke - kb - 1) / LDS::rows) * LDS::rows;
    for (int k0 = klast; k0 >= kb; k0 -= LDS::rows) {
        stage(L, r, k0, lane);
        const int m = min(LDS::rows, ke - k0);
        uint64_t bits = 0;
        for (int k = 0; k < m; ++k)
            if (kept(c, key_of(L.X[k][lane]), tie_pos(L, k0, k))) bits |= 1ull << k;
        // uniform loop, one kept entry per lane per trip: lanes with none
        // left add zero times staged row 0 (a branch here would make the
        // compiler copy all 64 accumulators at every trip)
        for (;;) {
            const bool has = bits != 0ull;
            if (__ballot(has) == 0ull) break;
            const int k = has ? __ffsll((unsigned long long)bits) - 1 : 0;
            bits &= bits - 1;
            const float xk = has ? L.X[k][lane] : 0.f;
            const float w = WEIGHTED ? xk * (alpha * L.y[k]) : xk;
#pragma unroll
            for (int b4 = 0; b4 < NF / 4; ++b4) {
                const float4 xr = *reinterpret_cast<const float4 *>(&L.X[k][b4 * 4]);
                A[4 * b4 + 0] = fmaf(w, xr.x, A[4 * b4 + 0]);
                A[4 * b4 + 1] = fmaf(w, xr.y, A[4 * b4 + 1]);
                A[4 * b4 + 2] = fmaf(w, xr.z, A[4 * b4 + 2]);
                A[4 * b4 + 3] = fmaf(w, xr.w, A[4 * b4 + 3]);
            }
            rhs = WEIGHTED ? fmaf(xk, fmaf(alpha, L.y[k], 1.f), rhs) : fmaf(w, L.y[k], rhs);
        }
    }
}

// Matrix-free residual of a candidate solution g of the row's system, with
// g_a parked in L.urhs[a]: over positions [kb, ke), lane a accumulates
// rho_a = sum over kept k of x_ka (y_k - x_k . g) and b_a = sum over kept k of
// x_ka y_k (the right-hand side of eq. core_ui).  Products in FP32, sums in FP64.
template <class LDS>
__device__ __forceinline__ void resid_range(LDS &L, RowCtx &r, const Cut &c, int kb, int ke, int lane,
                                            double &rho, double &bsum) {
    rho = 0.0;
    bsum = 0.0;
    if (c.none) return;
    for (int k0 = kb; k0 < ke; k0 += LDS::rows) {
        stage(L, r, k0, lane);
        const int m = min(LDS::rows, ke - k0);
        float rk = 0.f;
        if (lane < m) {
            float dot = 0.f;
#pragma unroll
            for (int b4 = 0; b4 < NF / 4; ++b4) {
                const float4 xr = *reinterpret_cast<const float4 *>(&L.X[lane][4 * b4]);
                dot = fmaf(xr.x, L.urhs[4 * b4 + 0], dot);
                dot = fmaf(xr.y, L.urhs[4 * b4 + 1], dot);
                dot = fmaf(xr.z, L.urhs[4 * b4 + 2], dot);
                dot = fmaf(xr.w, L.urhs[4 * b4 + 3], dot);
            }
            rk = L.y[lane] - dot;
        }
        if (lane < LDS::rows) L.rres[lane] = (double)rk;
        wave_sync();
        // every staged row, unrolled and without branches (unkept and
        // past-the-end rows add zero): the LDS reads of a batch overlap
#pragma unroll 16
        for (int k = 0; k < LDS::rows; ++k) {
            const float x = L.X[k][lane];
            const float xm = (k < m && kept(c, key_of(x), tie_pos(L, k0, k))) ? x : 0.f;
            rho += (double)xm * L.rres[k];
            bsum += (double)xm * (double)L.y[k];
        }
        wave_sync();
    }
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Relative residual |b - A g| / |b| from the lanes' rho_a (already minus
// lambda n g_a) and b_a; +inf when b = 0 (no answer is accepted then).
__device__ __forceinline__ double rel_residual(double rho, double bsum, int lane, int nf) {
    if (lane >= nf) rho = bsum = 0.0;
    const double rr = wave_sum_d(rho * rho);
    const double bb = wave_sum_d(bsum * bsum);
    return bb > 0.0 ? sqrt(rr / bb) : __builtin_inf();
}

template <class LDS>
__device__ __forceinline__ void gram(LDS &L, RowCtx &r, const Cut &c, int lane, float (&A)[NF], float &rhs) {
    gram_range(L, r, c, 0, r.n, lane, A, rhs);
}

// Diagonal penalty lambda n_i and identity padding for lanes >= nf.
__device__ __forceinline__ void finish_system(float (&A)[NF], float &rhs, float lamn, int lane, int nf) {
    // the lane through opaque_lane: else the 64 comparisons are hoisted out of
    // the row loop and their results spilled
    const int ol = opaque_lane(lane);
    const bool pad = ol >= nf;
#pragma unroll
    for (int b = 0; b < NF; ++b) {
        float v = A[b] + ((b == ol) ? lamn : 0.f);
        A[b] = pad ? ((b == ol) ? 1.f : 0.f) : v;
    }
    if (pad) rhs = 0.f;
}

// Elimination step J of the register-resident solve.  Every step has its own
// code (the steps are expanded at compile time), so every index into A is a
// constant and A stays in VGPRs; rows stay in place (A[c] is column c) and
// each pivot row stays in its lane.  PIVOT: partial pivoting (first lane of
// largest |entry| among rows not yet used, found by a DPP max); otherwise
// row J is the pivot (symmetric positive definite systems).  The pivot row
// reaches the other lanes through scalar broadcasts (v_readlane).
// KEEP: the multiplier of each eliminated row is stored in its column J (no
// longer needed there), so that the factors can solve later right-hand sides.
// The pivot candidate of column J for the lane's row: its magnitude with the
// low 6 bits replaced by 63 - lane, so that one maximum gives the pivot lane
// (the first of equal candidates; magnitudes within 2^-17 of each other count
// as equal); -1 for rows already used as pivots.
template <int J>
__device__ __forceinline__ int pivot_key(const float (&A)[NF], int lane, int my_step) {
    const int cand = my_step == NF ? ((__float_as_int(fabsf(A[J])) & ~63) | (63 - lane)) : -1;
    return wave_max_key(cand);
}

// pk: with PIVOT, the wave's maximum pivot key of column J, computed by the
// previous step as soon as column J was final (lookahead: the reduction runs
// beside the rest of that step's update); on return, the key of column J + 1.
// Bounds under which an elimination without row exchanges is kept: entries of
// the eliminated matrix within UNPIV_GROWTH max|A|, multipliers within
// UNPIV_MULT in magnitude.
constexpr float UNPIV_GROWTH = 4.f;
constexpr float UNPIV_MULT = 4.f;

// MCHK (without pivoting only): a multiplier above UNPIV_MULT in magnitude
// clears the lane's ok, which is then no longer uniform over the wave.
template <bool PIVOT, int NR, int J, bool KEEP, bool MCHK = false>
__device__ __forceinline__ void elim_step_u(float (&A)[NF], float (&rhs)[NR], int lane, int nf, float tol,
                                            int &my_step, bool &ok, int &pk) {
    int p;
    bool active;
    if constexpr (PIVOT) {
        active = my_step == NF;
        p = 63 - (pk & 63);
    } else {
        active = lane >= J;
        p = J;
    }
    const float piv = readlane_f(A[J], p);
    ok = ok && (J >= nf || fabsf(piv) > tol);
    if constexpr (MCHK) ok = ok && !(lane > J && fabsf(A[J]) > UNPIV_MULT * fabsf(piv));
    const bool elim = active && lane != p;
    // multipliers by the hardware reciprocal (1 ulp) instead of an IEEE
    // division sequence: one uniform reciprocal per step
    const float l = elim ? A[J] * __builtin_amdgcn_rcpf(piv) : 0.f;
    if constexpr (KEEP) A[J] = elim ? l : A[J];
    if (lane == p) my_step = J;
    // the pivot row in batches of 8: all readlanes of a batch first, into
    // distinct scalars, then its updates, so that no update waits on the
    // readlane just before it
#pragma unroll
    for (int c0 = J + 1; c0 < NF; c0 += 8) {
        float pr[8];
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (c0 + t < NF) pr[t] = readlane_f(A[c0 + t], p);
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (c0 + t < NF) A[c0 + t] = fmaf(-l, pr[t], A[c0 + t]);
        if constexpr (PIVOT && J + 1 < NF)
            if (c0 == J + 1) pk = pivot_key<J + 1>(A, lane, my_step);  // column J + 1 is final
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) rhs[q] = fmaf(-l, readlane_f(rhs[q], p), rhs[q]);
}

// Blocked elimination (panels of LU_BLK columns).  Step J eliminates column J
// exactly as elim_step_u, but updates only the panel's later columns at once;
// the columns after the panel wait for the panel's end, where every row
// subtracts one combination of the panel's pivot rows (their values at the
// panel's start, broadcast through LDS instead of one v_readlane per entry).
// With l_j the row's multiplier at panel step j and p_j that step's pivot row,
// the row's total update of a later column c is
//     sum_j l_j U_j[c],  U_j = A_{p_j} - sum_{i<j} l_i(p_j) U_i,
// = sum_j l'_j A_{p_j}[c] with l' solving the unit upper triangular system
// l'_i = l_i - sum_{j>i} l_i(p_j) l'_j (the panel's own multipliers).
template <bool PIVOT, int NR, int J, bool KEEP>
__device__ __forceinline__ void blk_step(float (&A)[NF], float (&rhs)[NR], int lane, int nf, float tol,
                                         int &my_step, bool &ok, int &pk, float (&lp)[LU_BLK], int (&pv)[LU_BLK],
                                         float (*pb)[NF]) {
    constexpr int JJ = J % LU_BLK;
    constexpr int P0 = J - JJ;
    constexpr int PE = P0 + LU_BLK;  // first column after the panel
    int p;
    bool active;
    if constexpr (PIVOT) {
        active = my_step == NF;
        p = 63 - (pk & 63);
    } else {
        active = lane >= J;
        p = J;
    }
    const float piv = readlane_f(A[J], p);
    ok = ok && (J >= nf || fabsf(piv) > tol);
    const bool elim = active && lane != p;
    const float l = elim ? A[J] * __builtin_amdgcn_rcpf(piv) : 0.f;
    if constexpr (KEEP) A[J] = elim ? l : A[J];
    if (lane == p) my_step = J;
    lp[JJ] = l;
    pv[JJ] = p;
    // the panel's later columns now
#pragma unroll
    for (int c = J + 1; c < PE; ++c) {
        A[c] = fmaf(-l, readlane_f(A[c], p), A[c]);
        if constexpr (PIVOT)
            if (c == J + 1) pk = pivot_key<J + 1>(A, lane, my_step);  // column J + 1 is final
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) rhs[q] = fmaf(-l, readlane_f(rhs[q], p), rhs[q]);
    if constexpr (JJ == LU_BLK - 1 && PE < NF) {
        // panel end: the rows' combined update of columns PE .. NF - 1
        float lt[LU_BLK];
#pragma unroll
        for (int i = LU_BLK - 1; i >= 0; --i) {
            lt[i] = lp[i];
#pragma unroll
            for (int j = i + 1; j < LU_BLK; ++j) lt[i] = fmaf(-readlane_f(lp[i], pv[j]), lt[j], lt[i]);
        }
        int slot = -1;
#pragma unroll
        for (int j = 0; j < LU_BLK; ++j)
            if (lane == pv[j]) slot = j;
        wave_sync();
        if (slot >= 0) {
#pragma unroll
            for (int c = PE; c < NF; c += 4)
                *reinterpret_cast<float4 *>(&pb[slot][c]) = make_float4(A[c], A[c + 1], A[c + 2], A[c + 3]);
        }
        wave_sync();
#pragma unroll
        for (int c = PE; c < NF; c += 4) {
#pragma unroll
            for (int j = 0; j < LU_BLK; ++j) {
                const float4 v = *reinterpret_cast<const float4 *>(&pb[j][c]);
                A[c + 0] = fmaf(-lt[j], v.x, A[c + 0]);
                A[c + 1] = fmaf(-lt[j], v.y, A[c + 1]);
                A[c + 2] = fmaf(-lt[j], v.z, A[c + 2]);
                A[c + 3] = fmaf(-lt[j], v.w, A[c + 3]);
            }
            if constexpr (PIVOT)
                if (c == PE) pk = pivot_key<PE>(A, lane, my_step);  // column PE is final
        }
    }
}

template <bool PIVOT, int NR, bool KEEP, int... J>
__device__ __forceinline__ void blk_all(std::integer_sequence<int, J...>, float (&A)[NF], float (&rhs)[NR], int lane,
                                        int nf, float tol, int &my_step, bool &ok, float (*pb)[NF]) {
    int pk = PIVOT ? pivot_key<0>(A, lane, my_step) : 0;
    float lp[LU_BLK];
    int pv[LU_BLK];
    (blk_step<PIVOT, NR, J, KEEP>(A, rhs, lane, nf, tol, my_step, ok, pk, lp, pv, pb), ...);
}

template <bool PIVOT, int NR, int J>
__device__ __forceinline__ void back_step_u(const float (&A)[NF], float (&rhs)[NR], int lane, int my_step,
                                            float *xs) {
    int p;
    if constexpr (PIVOT) {
        asm volatile("" : "+v"(my_step));  // see fwd_step_u
        const uint64_t bal = __ballot(my_step == J);
        p = bal ? (__ffsll((unsigned long long)bal) - 1) : 0;
        p = __builtin_amdgcn_readfirstlane(p);
    } else {
        p = J;
    }
    const float dinv = __builtin_amdgcn_rcpf(readlane_f(A[J], p));
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const float x = readlane_f(rhs[q], p) * dinv;
        if (lane == p) xs[q * NF + J] = x;
        if (my_step < J) rhs[q] = fmaf(-A[J], x, rhs[q]);
    }
}

template <bool PIVOT, int NR, bool KEEP, bool MCHK = false, int... J>
__device__ __forceinline__ void elim_all_u(std::integer_sequence<int, J...>, float (&A)[NF], float (&rhs)[NR],
                                           int lane, int nf, float tol, int &my_step, bool &ok) {
    int pk = PIVOT ? pivot_key<0>(A, lane, my_step) : 0;
    (elim_step_u<PIVOT, NR, J, KEEP, MCHK>(A, rhs, lane, nf, tol, my_step, ok, pk), ...);
}

// Forward elimination of a new right-hand side with kept factors: at step J
// the rows pivoted later (my_step > J) subtract their multiplier times the
// pivot row's entry, exactly as during the factorisation.
template <int NR, int J>
__device__ __forceinline__ void fwd_step_u(const float (&A)[NF], float (&rhs)[NR], int my_step) {
    // opaque per step: otherwise the 64 step masks of a loaded my_step are
    // all computed up front and spilled
    asm volatile("" : "+v"(my_step));
    const uint64_t bal = __ballot(my_step == J);
    int p = bal ? (__ffsll((unsigned long long)bal) - 1) : 0;
    p = __builtin_amdgcn_readfirstlane(p);
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const float rp = readlane_f(rhs[q], p);
        if (my_step > J) rhs[q] = fmaf(-A[J], rp, rhs[q]);
    }
}

template <int NR, int... J>
__device__ __forceinline__ void fwd_all_u(std::integer_sequence<int, J...>, const float (&A)[NF], float (&rhs)[NR],
                                          int my_step) {
    (fwd_step_u<NR, J>(A, rhs, my_step), ...);
}

template <bool PIVOT, int NR, int... J>
__device__ __forceinline__ void back_all_u(std::integer_sequence<int, J...>, const float (&A)[NF],
                                           float (&rhs)[NR], int lane, int my_step, float *xs) {
    (back_step_u<PIVOT, NR, NF - 1 - J>(A, rhs, lane, my_step, xs), ...);
}

// Solve the register-resident system for NR right-hand sides at once; returns
// false when a pivot of the first nf steps is <= tol.  On success x[q] holds
// component `lane` of the solution for right-hand side q.
// BLOCKED: panels with LDS-broadcast updates (measured faster in the heavy-row
// solve, which has the LDS to itself; the light-row kernels, whose Gram is
// bound by LDS reads, keep the per-step broadcasts).
template <bool PIVOT, int NR, class LDS, bool BLOCKED = false>
__device__ __forceinline__ bool solve_n(float (&A)[NF], float (&rhs)[NR], int lane, int nf, float tol,
                                        float (&x)[NR], LDS &L) {
    int my_step = NF;  // elimination step at which this lane's row was the pivot
    bool ok = true;
    if constexpr (BLOCKED)
        blk_all<PIVOT, NR, false>(std::make_integer_sequence<int, NF>{}, A, rhs, lane, nf, tol, my_step, ok, L.pbuf);
    else
        elim_all_u<PIVOT, NR, false>(std::make_integer_sequence<int, NF>{}, A, rhs, lane, nf, tol, my_step, ok);
    if (!PIVOT) my_step = lane;
    if (!ok) return false;
    wave_sync();
    back_all_u<PIVOT, NR>(std::make_integer_sequence<int, NF>{}, A, rhs, lane, my_step, L.urhs);
    wave_sync();
#pragma unroll
    for (int q = 0; q < NR; ++q) x[q] = L.urhs[q * NF + lane];
    wave_sync();
    return true;
}

template <bool PIVOT, class LDS, bool BLOCKED = false>
__device__ __forceinline__ bool solve(float (&A)[NF], float rhs, int lane, int nf, float tol, float &u,
                                      LDS &L) {
    float r[1] = {rhs};
    float x[1];
    const bool ok = solve_n<PIVOT, 1, LDS, BLOCKED>(A, r, lane, nf, tol, x, L);
    if (ok) u = x[0];
    return ok;
}

// Gaussian elimination without row exchanges (row J is the pivot of step J),
// accepted only when no pivot is small, no entry of the eliminated matrix
// exceeds UNPIV_GROWTH times the largest entry of A and no multiplier
// exceeds UNPIV_MULT in magnitude: with |L| and |U| so bounded, the computed
// factors have the backward error bound of the pivoted LU up to those
// factors.  Returns false otherwise; A is then spent and the caller builds
// the system again for the pivoted LU.
// BLOCKED: panels as in solve_n (the heavy-row solve).
template <class LDS, bool BLOCKED = false>
__device__ __forceinline__ bool solve_unpivoted(float (&A)[NF], float rhs, int lane, int nf, float tol, float &u,
                                                LDS &L) {
    float amax = 0.f;
#pragma unroll
    for (int b = 0; b < NF; ++b) amax = fmaxf(amax, fabsf(A[b]));
    amax = __int_as_float(wave_max_key(__float_as_int(amax)));
    int my_step = NF;
    bool ok = true;
    float r[1] = {rhs};
    if constexpr (BLOCKED)
        blk_all<false, 1, false>(std::make_integer_sequence<int, NF>{}, A, r, lane, nf, tol, my_step, ok, L.pbuf);
    else
        elim_all_u<false, 1, false, true>(std::make_integer_sequence<int, NF>{}, A, r, lane, nf, tol, my_step, ok);
    float g = 0.f;
#pragma unroll
    for (int b = 0; b < NF; ++b) g = fmaxf(g, fabsf(A[b]));
    g = __int_as_float(wave_max_key(__float_as_int(g)));
    if (__ballot(!ok) != 0 || !(g <= UNPIV_GROWTH * amax)) return false;
    if constexpr (BLOCKED) {
        // the multipliers, from what the elimination left: column J of a row
        // below J still holds that row's entry when it was eliminated, l u_JJ,
        // and row J holds u_JJ
        uint64_t big = 0;
#pragma unroll
        for (int j0 = 0; j0 < NF; j0 += 8) {
            float ud[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) ud[t] = readlane_f(A[j0 + t], j0 + t);
#pragma unroll
            for (int t = 0; t < 8; ++t)
                big |= __ballot(lane > j0 + t && fabsf(A[j0 + t]) > UNPIV_MULT * fabsf(ud[t]));
        }
        if (big) return false;
    }
    my_step = lane;
    wave_sync();
    back_all_u<false, 1>(std::make_integer_sequence<int, NF>{}, A, r, lane, my_step, L.urhs);
    wave_sync();
    u = L.urhs[lane];
    wave_sync();
    return true;
}

// Pivoted LU that keeps its factors in A (multipliers below, U above the
// pivots) and the lane's pivot step in my_step; returns false on a pivot of
// the first nf steps <= tol.
// Blocked (heavy-row solve).
template <class LDS>
__device__ __forceinline__ bool lu_keep(float (&A)[NF], float (&rhs)[1], int lane, int nf, float tol, int &my_step,
                                        LDS &L) {
    my_step = NF;
    bool ok = true;
    blk_all<true, 1, true>(std::make_integer_sequence<int, NF>{}, A, rhs, lane, nf, tol, my_step, ok, L.pbuf);
    return ok;
}

// Entry a of the fixed right-hand side whose solution estimates |A^-1|: signs
// alternate, magnitudes 1, 2, 3 in turn (|e|_inf = 3).
__device__ __forceinline__ float kappa_probe(int a) { return (a & 1 ? -1.f : 1.f) * (float)(1 + a % 3); }

// Back substitution of an eliminated right-hand side; x = component `lane`.
template <class LDS>
__device__ __forceinline__ float lu_back(const float (&A)[NF], float (&rhs)[1], int lane, int my_step, LDS &L) {
    wave_sync();
    back_all_u<true, 1>(std::make_integer_sequence<int, NF>{}, A, rhs, lane, my_step, L.urhs);
    wave_sync();
    const float x = L.urhs[lane];
    wave_sync();
    return x;
}

// ---------------------------------------------------------------------------
// Light core rows with few entries (n <= WB_D): by the Woodbury identity the
// solution of (lambda n E + W^T X) u = W^T y, with W the kept entries of X
// (n x n_f), is u = (b - W^T z) / (lambda n), b = W^T y, where z solves the
// n x n system G z = X b, G = lambda n E + X W^T.  The pivoted LU then has n
// steps instead of n_f.  Used only while max_k |x_k|^2 <= WB_AMP lambda, which
// bounds the cancellation in b - W^T z (error growth below WB_AMP).
constexpr int WB_D = 32;
constexpr float WB_AMP = 256.f;

template <int J>
__device__ __forceinline__ int wb_pivot_key(const float (&G)[WB_D], int lane, int my_step) {
    // as pivot_key
    const int cand = my_step == WB_D + 1 ? ((__float_as_int(fabsf(G[J])) & ~63) | (63 - lane)) : -1;
    return wave_max_key(cand);
}

// PIV: pivoted; pk is the pivot key of column J, computed by the previous
// step (lookahead as in elim_step_u), and on return that of column J + 1.
// Otherwise row J is the pivot of step J.
template <int J, bool PIV>
__device__ __forceinline__ void wb_elim_step(float (&G)[WB_D], float &t, int lane, int n, float tol, int &my_step,
                                             bool &ok, int &pk) {
    if (J >= n) return;  // uniform: the system has n rows
    bool active;
    int p;
    if constexpr (PIV) {
        active = my_step == WB_D + 1;
        p = 63 - (pk & 63);
    } else {
        active = lane > J;
        p = J;
    }
    const float piv = readlane_f(G[J], p);
    ok = ok && fabsf(piv) > tol;
    const bool elim = active && lane != p;
    const float l = elim ? G[J] * __builtin_amdgcn_rcpf(piv) : 0.f;
    if constexpr (PIV)
        if (lane == p) my_step = J;
    // columns n.. of every row stay as they are: the pivot row is zero there
#pragma unroll
    for (int c0 = J + 1; c0 < WB_D; c0 += 8) {  // batched as in elim_step_u
        if (c0 >= n) break;
        float pr[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (c0 + k < WB_D) pr[k] = readlane_f(G[c0 + k], p);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (c0 + k < WB_D) G[c0 + k] = fmaf(-l, pr[k], G[c0 + k]);
        if constexpr (PIV && J + 1 < WB_D)
            if (c0 == J + 1) pk = wb_pivot_key<J + 1>(G, lane, my_step);  // column J + 1 is final (J + 1 < n)
    }
    t = fmaf(-l, readlane_f(t, p), t);
}

template <int J, bool PIV>
__device__ __forceinline__ void wb_back_step(const float (&G)[WB_D], float &t, int lane, int n, int my_step,
                                             float *zs) {
    if (J >= n) return;
    int p;
    if constexpr (PIV) {
        asm volatile("" : "+v"(my_step));
        const uint64_t bal = __ballot(my_step == J);
        p = bal ? (__ffsll((unsigned long long)bal) - 1) : 0;
        p = __builtin_amdgcn_readfirstlane(p);
    } else {
        p = J;
    }
    const float x = readlane_f(t, p) * __builtin_amdgcn_rcpf(readlane_f(G[J], p));
    if (lane == 0) zs[J] = x;
    if (my_step < J) t = fmaf(-G[J], x, t);
}

// PIV false: elimination without row exchanges, kept only under the bounds of
// solve_unpivoted (no small pivot, entries of the eliminated rows within
// UNPIV_GROWTH gm, multipliers within UNPIV_MULT); gm = max |G| before.
// Returns false on a rejection or a small pivot; G and t are then spent.
template <bool PIV, int... J>
__device__ __forceinline__ bool wb_lu(std::integer_sequence<int, J...>, float (&G)[WB_D], float &t, int lane, int n,
                                      float tol, float gm, float *zs) {
    int my_step = WB_D + 1;
    bool ok = true;
    int pk = PIV ? wb_pivot_key<0>(G, lane, my_step) : 0;
    (wb_elim_step<J, PIV>(G, t, lane, n, tol, my_step, ok, pk), ...);
    if (!ok) return false;
    if constexpr (!PIV) {
        float g = 0.f;
#pragma unroll
        for (int l = 0; l < WB_D; ++l) g = fmaxf(g, fabsf(G[l]));
        g = __int_as_float(wave_max_key(__float_as_int(lane < n ? g : 0.f)));
        if (!(g <= UNPIV_GROWTH * gm)) return false;
        // multipliers: column J of a row below J holds l u_JJ, row J holds u_JJ
        uint64_t big = 0;
#pragma unroll
        for (int j0 = 0; j0 < WB_D; j0 += 8) {
            float ud[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) ud[q] = readlane_f(G[j0 + q], j0 + q);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                big |= __ballot(j0 + q < n && lane > j0 + q && fabsf(G[j0 + q]) > UNPIV_MULT * fabsf(ud[q]));
        }
        if (big) return false;
        my_step = lane;
    }
    (wb_back_step<WB_D - 1 - J, PIV>(G, t, lane, n, my_step, zs), ...);
    return true;
}

// Woodbury solve of a staged light row (n <= WB_D rows of X in L.X, cut c of
// the lane's column).  Returns false when the guard fails or G is singular
// (L.X is never modified: the caller's staged chunk stays valid).  On success
// u is component `lane` of the solution.
// W has s_i nonzeros per column, so G = lambda n E + X W^T is formed from the
// kept (row, column) pairs only: G[k][l] sums x_ka x_la over the columns a
// that keep row l, found from one ballot of the columns' kept masks per row.
template <class LDS>
__device__ __forceinline__ bool woodbury_solve(LDS &L, const Cut &c, int lane, int n, int nf, float lam,
                                               float lamn, bool &masked, float &u) {
    masked = false;
    static_assert(LDS::rows >= WB_D, "the Woodbury form stages the whole row");
    static_assert(WB_D <= 32, "kept masks are 32-bit");
    // lane k < rows: design row k (rows n.. are the staged zero padding);
    // lanes past the staged rows see zeros
    const int kr = min(lane, LDS::rows - 1);
    const bool lrow = lane < LDS::rows;
    float nrm = 0.f;
#pragma unroll
    for (int b4 = 0; b4 < NF / 4; ++b4) {
        float4 v = *reinterpret_cast<const float4 *>(&L.X[kr][4 * b4]);
        if (!lrow) v = make_float4(0.f, 0.f, 0.f, 0.f);
        nrm = fmaf(v.x, v.x, fmaf(v.y, v.y, fmaf(v.z, v.z, fmaf(v.w, v.w, nrm))));
    }
    const float mx = __int_as_float(wave_max_key(__float_as_int(nrm)));  // nrm >= 0
    if (!(mx <= WB_AMP * lam)) return false;
    // the lane's column: kept rows (bit k) and b_a = sum over kept k of x_ka y_k
    uint32_t km = 0u;
    float b = 0.f;
#pragma unroll
    for (int k = 0; k < WB_D; ++k) {
        const float x = L.X[k][lane];
        const bool kp = k < n && kept(c, key_of(x), tie_pos(L, 0, k));
        km |= kp ? (1u << k) : 0u;
        b = fmaf(kp ? x : 0.f, L.y[k], b);
    }
    if (lane >= nf) {
        b = 0.f;
        km = 0u;
    }
    wave_sync();
    L.urhs[lane] = b;
    wave_sync();
    // t_k = x_k . b
    float t = 0.f;
#pragma unroll
    for (int b4 = 0; b4 < NF / 4; ++b4) {
        float4 v = *reinterpret_cast<const float4 *>(&L.X[kr][4 * b4]);
        if (!lrow) v = make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 bv = *reinterpret_cast<const float4 *>(&L.urhs[4 * b4]);
        t = fmaf(v.x, bv.x, t);
        t = fmaf(v.y, bv.y, t);
        t = fmaf(v.z, bv.z, t);
        t = fmaf(v.w, bv.w, t);
    }
    // G row `lane` (rows n.. of the padded system are identity rows)
    float G[WB_D];
    auto build_g = [&]() {
#pragma unroll
        for (int l = 0; l < WB_D; ++l) {
            float g = 0.f;
            if (l < n) {
                uint64_t cols = __ballot((km >> l) & 1u);  // the columns keeping row l
                while (cols) {
                    const int a = __ffsll((unsigned long long)cols) - 1;
                    cols &= cols - 1;
                    g = fmaf(lrow ? L.X[kr][a] : 0.f, L.X[l][a], g);
                }
            }
            G[l] = g + (l == lane ? lamn : 0.f);
        }
        if (lane >= n) {
#pragma unroll
            for (int l = 0; l < WB_D; ++l) G[l] = (l == lane) ? 1.f : 0.f;
        }
    };
    build_g();
    if (lane >= n) t = 0.f;
    float gm = 0.f;
#pragma unroll
    for (int l = 0; l < WB_D; ++l) gm = fmaxf(gm, fabsf(G[l]));
    gm = __int_as_float(wave_max_key(__float_as_int(gm)));
    const float tol = (float)n * 1.1920928955078125e-7f * gm;
    float *zs = &L.urhs[NF];  // z_k, written by lane 0 of the back substitution
    const float t0 = t;
    if (!wb_lu<false>(std::make_integer_sequence<int, WB_D>{}, G, t, lane, n, tol, gm, zs)) {
        build_g();  // the elimination without row exchanges was rejected: pivoted LU
        t = t0;
        if (!wb_lu<true>(std::make_integer_sequence<int, WB_D>{}, G, t, lane, n, tol, gm, zs)) return false;
    }
    wave_sync();
    // u_a = (b_a - sum over kept k of x_ka z_k) / (lambda n)
    float sacc = b;
#pragma unroll
    for (int k = 0; k < WB_D; ++k)
        if (k < n) sacc = fmaf(-(((km >> k) & 1u) ? L.X[k][lane] : 0.f), zs[k], sacc);
    u = lane < nf ? sacc / lamn : 0.f;
    wave_sync();
    return true;
}

// Implicit feedback: the global Gram G = Y^T Y (row-major, stride NF, zero
// outside n_f) and lambda on the diagonal; identity rows for lanes >= nf.
__device__ __forceinline__ void finish_system_implicit(float (&A)[NF], float &rhs, const float *G, float lam,
                                                       int lane, int nf) {
    const int ol = opaque_lane(lane);
    const bool pad = ol >= nf;
    const float *g = G + (pad ? 0 : ol) * NF;
#pragma unroll
    for (int b4 = 0; b4 < NF / 4; ++b4) {
        const float4 gv = *reinterpret_cast<const float4 *>(g + 4 * b4);
        const float gg[4] = {gv.x, gv.y, gv.z, gv.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = 4 * b4 + q;
            const float v = A[b] + gg[q] + ((b == ol) ? lam : 0.f);
            A[b] = pad ? ((b == ol) ? 1.f : 0.f) : v;
        }
    }
    if (pad) rhs = 0.f;
}

__device__ __forceinline__ float system_tol(const float (&A)[NF], int nf) {
    float m = 0.f;
#pragma unroll
    for (int b = 0; b < NF; ++b) m = fmaxf(m, fabsf(A[b]));
    m = __int_as_float(wave_max_key(__float_as_int(m)));  // m >= 0: integer order = value order
    return (float)nf * 1.1920928955078125e-7f * m;
}


}  // namespace coreals
