// Rows of a half-sweep at ranks 64 < n_f <= 128 (gfx950).
//
// An n_f x n_f system of rank above 64 does not fit the one-row-per-lane
// layout of the rank-64 kernels, so at these ranks every non-empty row takes
// a workgroup path (the selection is launch_heavy_select, run once per half of
// the columns, cuts at stride NFW):
//
//   k_wide_gram   one workgroup of four wavefronts per (row, chunk) pair.
//                 Wavefront w builds rows 32w .. 32w + 31 of the chunk's part
//                 of X*^T X (against all 128 columns) and of X*^T y
//                 (eq. core_ui) on 32x32x16 bf16 MFMA tiles: FP32 products
//                 from the exact three-way bf16 split of each operand, or
//                 plain bf16 operands in the BF16 precision modes.
//   k_wide_solve  one workgroup per row sums the row's partial systems in
//                 chunk order, adds lambda n_i, and solves by LU with partial
//                 pivoting.  The system is spread over the 256 threads in
//                 8 x 8 blocks (thread 16 bj + bi owns rows 8 bi .. 8 bi + 7
//                 and columns 8 bj .. 8 bj + 7, so the 16 owners of a column
//                 block are one 16-lane DPP row of one wavefront); each
//                 elimination step broadcasts its multipliers and pivot row
//                 through LDS and updates every block with 64 FMAs.  Rows stay
//                 in place; each row remembers the step it was pivot of.  A
//                 singular core system flags the row: a second Gram and solve
//                 pass over the flagged rows uses the full data (eq. (U)).
//   k_wide_resid, k_wide_refine
//                 the refinement step of the BF16 modes: residual
//                 X*^T (y - X u) per chunk (FP32, or FP64 per row), then a
//                 correction solve with the LU factors the first solve kept.
//   k_wide_empty  rows without entries: u = 0.
//   k_select_wide positions of the kept entries for the core_select entry point.
#include "rowops.hpp"

namespace coreals {

namespace {

constexpr int WT = 256;                         // threads of the row workgroups
constexpr int64_t WSLOT = (int64_t)(NFW + 1) * NFW;  // floats of one partial system
constexpr uint32_t WF_NONE = 0x80000000u;       // buffer offset past any factor matrix

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

__device__ __forceinline__ uint32_t pack_bf16_2(float lo, float hi) {
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

unsigned grid_of(int64_t items, int64_t cap) {
    int64_t b = items < 1 ? 1 : items;
    return (unsigned)(b > cap ? cap : b);
}

// ---------------------------------------------------------------------------
// Partial system of one (row, chunk) pair.  A = X*^T (kept entries of the
// row's columns 32w + m), B = X (all columns 32 tb + m, tb = 0..3); lane
// (m, h) holds entries 8h .. 8h + 7 of a 16-entry step.  The tile layout and
// the split are those of the rank-64 heavy-row Gram: x = hi + mid + lo in
// bf16 (round to nearest, exact remainders), six products per tile give the
// FP32 product within 2^-23 |x x'|.  Output: element (a, b) at b * NFW + a,
// right-hand side at NFW * NFW + a.  Entries past the chunk and padded columns
// read zeros (buffer offsets past the matrix, or explicit zeros without BUF).
template <bool BUF, bool X6>
__global__ __launch_bounds__(WT) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_wide_gram(
    HeavyArgs a, int64_t pair_begin, int64_t pair_end) {
    __shared__ int s_col[64];
    __shared__ float s_y[64];
    const int tid = threadIdx.x;
    const int w = wave_index();
    const int lane = tid & 63;
    const int m = lane & 31, h = lane >> 5;
    const int nf = a.nf;
    const int stride = 4 * nf;
    const int ca = 32 * w + m;  // column of the lane's A operand
    uint32_t offb[4];
#pragma unroll
    for (int tb = 0; tb < 4; ++tb) offb[tb] = 32 * tb + m < nf ? 4u * (32 * tb + m) : WF_NONE;
    const uint32_t offa = ca < nf ? 4u * ca : WF_NONE;
    const int rows = BUF ? (int)a.other_rows : -1;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float *>(a.other), (short)0, BUF ? (int)(a.other_rows * nf * 4) : 0, 0x00020000);
    for (int64_t p = pair_begin + blockIdx.x; p < pair_end; p += gridDim.x) {
        const int64_t slot = a.pair_slot[p];
        if (a.pass && a.flag[slot] != a.pass) continue;  // uniform over the workgroup
        const int chunk = a.pair_chunk[p];
        const int64_t i = a.rows[slot];
        const int64_t beg = a.ptr[i];
        const int n = (int)(a.ptr[i + 1] - beg);
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        // kept(k) <=> (key, ~k) >= (T, ~K) as unsigned 64-bit pairs
        int T = 0, K = 0x7FFFFFFF;  // every entry kept (full data)
        if (a.pass != 1 && s < n) {
            if (s == 0) {
                T = 0x7FFFFFFF;
                K = -1;
            } else {
                T = a.cutT[slot * NFW + ca];
                K = a.cutK[slot * NFW + ca];
            }
        }
        const uint64_t bt = ((uint64_t)(uint32_t)T << 32) | (uint32_t)~K;
        f32x16 acc[4];
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[tb][q] = 0.f;
        float racc = 0.f;
        const int kb = chunk * a.chunk;
        const int ke = min(n, kb + a.chunk);
        for (int k0 = kb; k0 < ke; k0 += 64) {
            __syncthreads();  // the previous block's LDS reads are done
            if (tid < 64) {
                s_col[tid] = k0 + tid < ke ? a.idx[beg + k0 + tid] : rows;
                s_y[tid] = k0 + tid < ke ? a.val[beg + k0 + tid] : 0.f;
            }
            __syncthreads();
#pragma unroll 1
            for (int e0 = k0; e0 < min(ke, k0 + 64); e0 += 16) {
                const int j0 = e0 - k0;
                float xb[4][8], xa[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int col = s_col[j0 + 8 * h + e];
                    if constexpr (BUF) {
                        const uint32_t off = __umul24((unsigned)col, (unsigned)stride);
#pragma unroll
                        for (int tb = 0; tb < 4; ++tb)
                            xb[tb][e] = __int_as_float(
                                __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(off + offb[tb]), 0, 0));
                        xa[e] = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)(off + offa), 0, 0));
                    } else {
                        const size_t ro = (size_t)max(col, 0) * nf;
#pragma unroll
                        for (int tb = 0; tb < 4; ++tb) {
                            const int cb = 32 * tb + m;
                            const float v = a.other[ro + min(cb, nf - 1)];
                            xb[tb][e] = (col >= 0 && cb < nf) ? v : 0.f;
                        }
                        const float v = a.other[ro + min(ca, nf - 1)];
                        xa[e] = (col >= 0 && ca < nf) ? v : 0.f;
                    }
                }
                // every gather of the step is issued before the first use
                __builtin_amdgcn_sched_barrier(0);
                const uint32_t nkb = ~(uint32_t)(e0 + 8 * h);  // ~k of the lane's first entry
                uint32_t ah[4], am[4], al[4];
#pragma unroll
                for (int e2 = 0; e2 < 4; ++e2) {
                    uint32_t km[2];
#pragma unroll
                    for (int o = 0; o < 2; ++o) {
                        const int e = 2 * e2 + o;
                        const float x = xa[e];
                        const uint64_t key =
                            ((uint64_t)(__float_as_uint(x) & 0x7FFFFFFFu) << 32) | (nkb - (uint32_t)e);
                        const bool kp = key >= bt;
                        km[o] = kp ? 0xFFFFu : 0u;
                        racc = fmaf(kp ? x : 0.f, s_y[j0 + 8 * h + e], racc);
                    }
                    const uint32_t mk = km[0] | (km[1] << 16);
                    const uint32_t qh = pack_bf16_2(xa[2 * e2], xa[2 * e2 + 1]);
                    ah[e2] = qh & mk;
                    if constexpr (X6) {
                        const float r0 = xa[2 * e2] - __uint_as_float(qh << 16);
                        const float r1 = xa[2 * e2 + 1] - __uint_as_float(qh & 0xFFFF0000u);
                        const uint32_t qm = pack_bf16_2(r0, r1);
                        const float s0 = r0 - __uint_as_float(qm << 16);
                        const float s1 = r1 - __uint_as_float(qm & 0xFFFF0000u);
                        am[e2] = qm & mk;
                        al[e2] = pack_bf16_2(s0, s1) & mk;
                    }
                }
                bf16x8 Ah = __builtin_bit_cast(bf16x8, ah), Am, Al;
                if constexpr (X6) {
                    Am = __builtin_bit_cast(bf16x8, am);
                    Al = __builtin_bit_cast(bf16x8, al);
                }
                bf16x8 Bh[4], Bm[4], Bl[4];
#pragma unroll
                for (int tb = 0; tb < 4; ++tb) {
                    uint32_t ph[4], pm[4], pl[4];
#pragma unroll
                    for (int e2 = 0; e2 < 4; ++e2) {
                        const float x0 = xb[tb][2 * e2], x1 = xb[tb][2 * e2 + 1];
                        const uint32_t qh = pack_bf16_2(x0, x1);
                        ph[e2] = qh;
                        if constexpr (X6) {
                            const float r0 = x0 - __uint_as_float(qh << 16);
                            const float r1 = x1 - __uint_as_float(qh & 0xFFFF0000u);
                            const uint32_t qm = pack_bf16_2(r0, r1);
                            pm[e2] = qm;
                            pl[e2] = pack_bf16_2(r0 - __uint_as_float(qm << 16), r1 - __uint_as_float(qm & 0xFFFF0000u));
                        }
                    }
                    Bh[tb] = __builtin_bit_cast(bf16x8, ph);
                    if constexpr (X6) {
                        Bm[tb] = __builtin_bit_cast(bf16x8, pm);
                        Bl[tb] = __builtin_bit_cast(bf16x8, pl);
                    }
                }
                // the four tiles interleaved so that consecutive MFMAs are independent
#define WG_MFMA(A, B) \
    _Pragma("unroll") for (int tb = 0; tb < 4; ++tb) acc[tb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B[tb], acc[tb], 0, 0, 0);
                if constexpr (X6) {
                    WG_MFMA(Al, Bh)
                    WG_MFMA(Ah, Bl)
                    WG_MFMA(Am, Bm)
                    WG_MFMA(Am, Bh)
                    WG_MFMA(Ah, Bm)
                }
                WG_MFMA(Ah, Bh)
#undef WG_MFMA
            }
        }
        racc += __shfl_xor(racc, 32);
        float *dst = a.partials + (p - pair_begin) * WSLOT;
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int row = 8 * (q >> 2) + 4 * h + (q & 3);
                dst[(32 * tb + m) * NFW + 32 * w + row] = acc[tb][q];
            }
        if (h == 0) dst[NFW * NFW + ca] = racc;
    }
}

// ---------------------------------------------------------------------------
// The distributed LU.

struct WideLds {
    float l[2][NFW];  // multipliers of the step (double-buffered)
    float u[2][NFW];  // pivot row of the step, zero at columns <= the step
    float rhs[NFW];
    float x[NFW];
    int row_of_step[NFW];
    int piv[2];
    float pval[2];
    float rsum[NFW];  // row sums of |A|
    double rr[NFW];   // refinement: squares of the residual and right-hand side
    double bb[NFW];
    int amax;         // bits of max |A| (non-negative floats order as integers)
    int anorm;        // bits of |A|_inf
    int zmax;         // bits of |A^-1 e|_inf
    int ok;
};

// Largest key over each 16-lane DPP row; every lane of the row ends with it.
__device__ __forceinline__ int row16_max_key(int v) {
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true));   // quad_perm [1,0,3,2]
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true));   // quad_perm [2,3,0,1]
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true));  // row_half_mirror
    v = max(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true));  // row_mirror
    return v;
}

// Entry (q, C) of the thread's block for a workgroup-uniform q: a scalar
// branch per row instead of an indexed register access.
template <int C>
__device__ __forceinline__ float block_at(const float (&A)[8][8], int q) {
    switch (q) {
        case 0: return A[0][C];
        case 1: return A[1][C];
        case 2: return A[2][C];
        case 3: return A[3][C];
        case 4: return A[4][C];
        case 5: return A[5][C];
        case 6: return A[6][C];
        default: return A[7][C];
    }
}

__device__ __forceinline__ void block_row(const float (&A)[8][8], int q, float (&v)[8]) {
    switch (q) {
#define WB_ROW(Q) \
    case Q:       \
        _Pragma("unroll") for (int c = 0; c < 8; ++c) v[c] = A[Q][c]; break;
        WB_ROW(0)
        WB_ROW(1)
        WB_ROW(2)
        WB_ROW(3)
        WB_ROW(4)
        WB_ROW(5)
        WB_ROW(6)
        default:
#pragma unroll
            for (int c = 0; c < 8; ++c) v[c] = A[7][c];
            break;
#undef WB_ROW
    }
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Factor the system in place (multipliers stored below the pivots, in the
// eliminated rows' columns) and eliminate S.rhs with it.  step[q]: the step
// at which row 8 bi + q was the pivot.  Returns false (uniformly) when a pivot
// of the first nf steps is at most tol.
__device__ __forceinline__ bool wide_lu(float (&A)[8][8], int (&step)[8], WideLds &S, int nf, float tol) {
    const int tid = threadIdx.x;
    const int bi = tid & 15, bj = tid >> 4;
    const int w = wave_index();
    const int lane = tid & 63;
#pragma unroll
    for (int q = 0; q < 8; ++q) step[q] = NFW;
#pragma unroll 1
    for (int jb = 0; jb < NFW / 8; ++jb) {
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const int J = 8 * jb + jj;
            const int buf = jj & 1;
            if (w == (jb >> 2)) {
                // pivot search over column J by its 16 owners: |value| with the
                // low 7 bits replaced by 127 - row (first row among equals)
                const bool mine = bj == jb;
                int key = -1;
                float cv = 0.f;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int k = (__float_as_int(fabsf(A[q][jj])) & ~127) | (127 - (8 * bi + q));
                    if (mine && step[q] == NFW && k > key) {
                        key = k;
                        cv = A[q][jj];
                    }
                }
                // the owners' DPP row holds the maximum; other rows hold -1
                const int kmax = __builtin_amdgcn_readlane(row16_max_key(key), 16 * (jb & 3));
                const int p = 127 - (kmax & 127);
                const float piv = readlane_f(cv, 16 * (jb & 3) + (p >> 3));
                const float rp = __builtin_amdgcn_rcpf(piv);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int r = 8 * bi + q;
                    float l = 0.f;
                    if (mine && step[q] == NFW && r != p) {
                        l = A[q][jj] * rp;
                        A[q][jj] = l;
                    }
                    if (mine) S.l[buf][r] = l;
                }
                if (lane == 16 * (jb & 3)) {
                    S.piv[buf] = p;
                    S.pval[buf] = piv;
                    if (J < nf && !(fabsf(piv) > tol)) S.ok = 0;
                }
            }
            __syncthreads();
            const int p = uniform(S.piv[buf]);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (8 * bi + q == p) step[q] = J;
            if (tid == 0) S.row_of_step[J] = p;
            if (bi == (p >> 3)) {
                float v[8];
                block_row(A, p & 7, v);
#pragma unroll
                for (int c = 0; c < 8; ++c) S.u[buf][8 * bj + c] = (8 * bj + c > J) ? v[c] : 0.f;
            }
            __syncthreads();
            if (32 * w + 31 > J) {  // waves whose columns are all <= J have nothing left
                float lv[8], uv[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) lv[q] = S.l[buf][8 * bi + q];
#pragma unroll
                for (int c = 0; c < 8; ++c) uv[c] = S.u[buf][8 * bj + c];
#pragma unroll
                for (int q = 0; q < 8; ++q)
#pragma unroll
                    for (int c = 0; c < 8; ++c) A[q][c] = fmaf(-lv[q], uv[c], A[q][c]);
            }
            if (tid < 16) {  // right-hand side rows 8 tid .. 8 tid + 7
                const float rp_ = S.rhs[p];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float l = S.l[buf][8 * tid + q];
                    if (l != 0.f) S.rhs[8 * tid + q] = fmaf(-l, rp_, S.rhs[8 * tid + q]);
                }
            }
        }
    }
    __syncthreads();
    return S.ok != 0;
}

// Forward elimination of S.rhs with the kept multipliers (a new right-hand
// side for factors from wide_lu): at step J the rows pivoted later subtract
// their multiplier times the pivot row's entry.  S.row_of_step must be set.
__device__ __forceinline__ void wide_forward(const float (&A)[8][8], const int (&step)[8], WideLds &S) {
    const int tid = threadIdx.x;
    const int bi = tid & 15, bj = tid >> 4;
    const int w = wave_index();
#pragma unroll 1
    for (int jb = 0; jb < NFW / 8; ++jb) {
        __syncthreads();
        if (w == (jb >> 2)) {
            const bool mine = bj == jb;
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) {
                const int J = 8 * jb + jj;
                const int p = uniform(S.row_of_step[J]);
                const float rp = S.rhs[p];
                if (mine) {
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (step[q] > J) S.rhs[8 * bi + q] = fmaf(-A[q][jj], rp, S.rhs[8 * bi + q]);
                }
                wave_sync();
            }
        }
    }
    __syncthreads();
}

// Back substitution of an eliminated S.rhs: S.x[J] = component J.
__device__ __forceinline__ void wide_back(const float (&A)[8][8], const int (&step)[8], WideLds &S) {
    const int tid = threadIdx.x;
    const int bi = tid & 15, bj = tid >> 4;
    const int w = wave_index();
    const int lane = tid & 63;
#pragma unroll 1
    for (int jb = NFW / 8 - 1; jb >= 0; --jb) {
        __syncthreads();
        if (w == (jb >> 2)) {
            const bool mine = bj == jb;
#pragma unroll
            for (int jj = 7; jj >= 0; --jj) {
                const int J = 8 * jb + jj;
                const int p = uniform(S.row_of_step[J]);
                float d = 0.f;
                switch (jj) {  // jj is a constant of the unrolled loop
                    case 0: d = block_at<0>(A, p & 7); break;
                    case 1: d = block_at<1>(A, p & 7); break;
                    case 2: d = block_at<2>(A, p & 7); break;
                    case 3: d = block_at<3>(A, p & 7); break;
                    case 4: d = block_at<4>(A, p & 7); break;
                    case 5: d = block_at<5>(A, p & 7); break;
                    case 6: d = block_at<6>(A, p & 7); break;
                    default: d = block_at<7>(A, p & 7); break;
                }
                const float diag = readlane_f(d, 16 * (jb & 3) + (p >> 3));
                const float xj = S.rhs[p] * __builtin_amdgcn_rcpf(diag);
                if (lane == 16 * (jb & 3)) S.x[J] = xj;
                if (mine) {
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (step[q] < J) S.rhs[8 * bi + q] = fmaf(-A[q][jj], xj, S.rhs[8 * bi + q]);
                }
                wave_sync();
            }
        }
    }
    __syncthreads();
}

// One workgroup per heavy slot: the row's system from its partial systems,
// solved (pass 0), or the rows flagged for pass 1 (singular core system,
// full-data partials) or pass 2 (ALS_PREC_AUTO: partials with FP32 products).
// With keep, the LU factors and each row's pivot step (bit 16: refine this row
// with an FP64 residual) go to the row's first partial slot for the
// refinement step; -1 there means no refinement.
__global__ __launch_bounds__(WT) void k_wide_solve(HeavyArgs a, int64_t slot_begin, int64_t slot_end,
                                                   int64_t pair_base) {
    __shared__ WideLds S;
    const int tid = threadIdx.x;
    const int bi = tid & 15, bj = tid >> 4;
    const int nf = a.nf;
    for (int64_t slot = slot_begin + blockIdx.x; slot < slot_end; slot += gridDim.x) {
        if (a.pass && a.flag[slot] != a.pass) continue;  // uniform
        const int64_t i = a.rows[slot];
        const int n = (int)(a.ptr[i + 1] - a.ptr[i]);
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        const float lamn = (float)((double)a.lam * (double)n);
        float *fac = a.partials + (a.pair_off[slot] - pair_base) * WSLOT;
        float A[8][8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int c = 0; c < 8; ++c) A[q][c] = 0.f;
        float rhs[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int64_t pp = a.pair_off[slot]; pp < a.pair_off[slot + 1]; ++pp) {
            const float *src = a.partials + (pp - pair_base) * WSLOT;
#pragma unroll
            for (int c = 0; c < 8; ++c)
#pragma unroll
                for (int q = 0; q < 8; ++q) A[q][c] += src[(8 * bj + c) * NFW + 8 * bi + q];
            if (tid < 16)
#pragma unroll
                for (int q = 0; q < 8; ++q) rhs[q] += src[NFW * NFW + 8 * tid + q];
        }
        float amax = 0.f, rs[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            rs[q] = 0.f;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int r = 8 * bi + q, col = 8 * bj + c;
                float v = A[q][c] + (r == col ? lamn : 0.f);
                if (r >= nf) v = (r == col) ? 1.f : 0.f;  // padding: identity rows
                A[q][c] = v;
                amax = fmaxf(amax, fabsf(v));
                rs[q] += fabsf(v);
            }
        }
        if (tid == 0) {
            S.amax = 0;
            S.anorm = 0;
            S.zmax = 0;
            S.ok = 1;
        }
        if (tid < NFW) S.rsum[tid] = 0.f;
        __syncthreads();
        if (tid < 16)
#pragma unroll
            for (int q = 0; q < 8; ++q) S.rhs[8 * tid + q] = 8 * tid + q < nf ? rhs[q] : 0.f;
        atomicMax(&S.amax, __float_as_int(amax));
#pragma unroll
        for (int q = 0; q < 8; ++q) atomicAdd(&S.rsum[8 * bi + q], rs[q]);
        __syncthreads();
        if (tid < NFW) atomicMax(&S.anorm, __float_as_int(S.rsum[tid]));
        const float tol = (float)nf * 1.1920928955078125e-7f * __int_as_float(S.amax);
        int step[8];
        const bool ok = wide_lu(A, step, S, nf, tol);  // (its barriers publish S.anorm)
        bool keep_fac = false, regram = false;
        int need64 = 0;
        if (ok) {
            wide_back(A, step, S);
            if (tid < nf) a.out[i * nf + tid] = S.x[tid];
            keep_fac = a.keep && a.pass != 1;
            if (keep_fac && a.fp64res == RES_PER_ROW) {
                // condition estimate |A|_inf |A^-1 e|_inf / |e|_inf
                __syncthreads();
                if (tid < NFW) S.rhs[tid] = tid < nf ? kappa_probe(tid) : 0.f;
                wide_forward(A, step, S);
                wide_back(A, step, S);
                if (tid < nf) atomicMax(&S.zmax, __float_as_int(fabsf(S.x[tid])));
                __syncthreads();
                const float kest = __int_as_float(S.anorm) * __int_as_float(S.zmax) * (1.f / 3.f);
                need64 = ((double)a.lam < FP64_LAMBDA && kest > KAPPA_FP64) ? 1 : 0;
                regram = a.pass == 0 && kest > KAPPA_BF16;
                keep_fac = !regram;
            } else if (a.fp64res == RES_FP64) {
                need64 = 1;
            }
        } else if (tid < nf) {
            a.out[i * nf + tid] = 0.f;
        }
        if (a.pass == 0 && tid == 0) {
            // pass 1: singular core system, solved again from the full data;
            // pass 2: Gram again with FP32 products
            const bool singular = !ok && s < n;
            a.flag[slot] = singular ? 1 : regram ? 2 : 0;
            if (singular) atomicAdd(&a.stats[ST_FALLBACK], 1ull);
            if (regram) atomicAdd(&a.stats[ST_FP32GRAM], 1ull);
        }
        if (a.keep) {
            if (keep_fac) {
#pragma unroll
                for (int c = 0; c < 8; ++c)
#pragma unroll
                    for (int q = 0; q < 8; ++q) fac[(8 * bj + c) * NFW + 8 * bi + q] = A[q][c];
            }
            if (tid < 16)
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    fac[NFW * NFW + 8 * tid + q] = __int_as_float(keep_fac ? (step[q] | (need64 << 16)) : -1);
        }
        __syncthreads();  // S is reused by the next row
    }
}

// Refinement step: u + A^-1 (rho - lambda n u), rho = sum of the chunk
// residuals, with the factors the first solve kept.
__global__ __launch_bounds__(WT) void k_wide_refine(HeavyArgs a, int64_t slot_begin, int64_t slot_end,
                                                    int64_t pair_base) {
    __shared__ WideLds S;
    const int tid = threadIdx.x;
    const int bi = tid & 15, bj = tid >> 4;
    const int nf = a.nf;
    for (int64_t slot = slot_begin + blockIdx.x; slot < slot_end; slot += gridDim.x) {
        const int64_t i = a.rows[slot];
        const int n = (int)(a.ptr[i + 1] - a.ptr[i]);
        const float *fac = a.partials + (a.pair_off[slot] - pair_base) * WSLOT;
        const int st0 = uniform(__float_as_int(fac[NFW * NFW]));
        if (st0 < 0) continue;  // no factors kept (singular system, or the full-data pass)
        const bool need64 = (st0 >> 16) & 1;
        float A[8][8];
#pragma unroll
        for (int c = 0; c < 8; ++c)
#pragma unroll
            for (int q = 0; q < 8; ++q) A[q][c] = fac[(8 * bj + c) * NFW + 8 * bi + q];
        int step[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) step[q] = __float_as_int(fac[NFW * NFW + 8 * bi + q]) & 0xFFFF;
        float u0 = 0.f;
        if (tid < NFW) {
            const int r = tid;
            S.row_of_step[__float_as_int(fac[NFW * NFW + r]) & 0xFFFF] = r;
            u0 = r < nf ? a.out[i * nf + r] : 0.f;
            double rho = 0.0, bsum = 0.0;
            for (int64_t pp = a.pair_off[slot]; pp < a.pair_off[slot + 1]; ++pp) {
                rho += a.resid[(pp - pair_base) * 2 * NFW + r];
                bsum += a.resid[(pp - pair_base) * 2 * NFW + NFW + r];
            }
            rho -= (double)a.lam * (double)n * (double)u0;
            if (r >= nf) rho = bsum = 0.0;
            S.rhs[r] = (float)rho;
            S.rr[r] = rho * rho;
            S.bb[r] = bsum * bsum;
        }
        __syncthreads();
        if (tid == 0) {
            // relative residual |b - A u0| / |b| of the first solution
            double rr = 0.0, bb = 0.0;
            for (int r = 0; r < NFW; ++r) {
                rr += S.rr[r];
                bb += S.bb[r];
            }
            if (bb > 0.0)
                atomicMax(&a.stats[ST_MAXRES], (unsigned long long)__double_as_longlong(sqrt(rr / bb)));
        }
        wide_forward(A, step, S);
        wide_back(A, step, S);
        if (tid < nf) a.out[i * nf + tid] = u0 + S.x[tid];
        if (need64 && tid == 0) atomicAdd(&a.stats[ST_FP64RES], 1ull);
        __syncthreads();
    }
}

// Chunk residual of a (row, chunk) pair: rho_a = sum over kept k of
// x_ka (y_k - x_k . u), u the row's first solution (in out).  The row's
// design rows are staged in LDS 64 at a time; FP64 products and sums when the
// first solve asked for them.
struct WideResLds {
    float X[64][NFW + 1];
    float y[64];
    float u[NFW];
    double r[64];
    double half[NFW];
    double bhalf[NFW];
};

template <typename acc_t>
__device__ __forceinline__ void wide_resid_row(const HeavyArgs &a, WideResLds &L, int64_t p, int64_t pair_begin,
                                               int64_t slot, int64_t beg, int n, int s) {
    const int tid = threadIdx.x;
    const int nf = a.nf;
    const int col = tid & (NFW - 1), half = tid >> 7;
    Cut c{0, 0, false, true};
    if (s < n) {
        if (s == 0) c = Cut{0, 0, true, false};
        else c = Cut{a.cutT[slot * NFW + col], a.cutK[slot * NFW + col], false, false};
    }
    const int kb = a.pair_chunk[p] * a.chunk;
    const int ke = min(n, kb + a.chunk);
    acc_t acc = 0;
    double bs = 0.0;  // the chunk's share of b = X*^T y
    for (int k0 = kb; k0 < ke; k0 += 64) {
        const int m = min(64, ke - k0);
        __syncthreads();
        // stage: thread (col, half) loads column col of rows half, half + 2, ...
        for (int k = half; k < 64; k += 2) {
            float v = 0.f;
            if (k < m && col < nf) v = a.other[(size_t)a.idx[beg + k0 + k] * nf + col];
            L.X[k][col] = v;
        }
        if (tid < 64) L.y[tid] = tid < m ? a.val[beg + k0 + tid] : 0.f;
        __syncthreads();
        if (tid < 64) {
            acc_t dot = 0;
            for (int b = 0; b < nf; ++b) dot += (acc_t)L.X[tid][b] * (acc_t)L.u[b];
            L.r[tid] = (double)((acc_t)L.y[tid] - dot);
        }
        __syncthreads();
        for (int k = half * 32; k < half * 32 + 32 && k < m; ++k) {
            const float x = L.X[k][col];
            if (kept(c, key_of(x), k0 + k)) {
                acc += (acc_t)x * (acc_t)L.r[k];
                bs += (double)x * (double)L.y[k];
            }
        }
    }
    __syncthreads();
    if (half == 1) {
        L.half[col] = (double)acc;
        L.bhalf[col] = bs;
    }
    __syncthreads();
    if (half == 0) {
        double *dst = a.resid + (p - pair_begin) * 2 * NFW;
        dst[col] = col < nf ? (double)acc + L.half[col] : 0.0;
        dst[NFW + col] = col < nf ? bs + L.bhalf[col] : 0.0;
    }
}

__global__ __launch_bounds__(WT) void k_wide_resid(HeavyArgs a, int64_t pair_begin, int64_t pair_end) {
    __shared__ WideResLds L;
    const int tid = threadIdx.x;
    for (int64_t p = pair_begin + blockIdx.x; p < pair_end; p += gridDim.x) {
        const int64_t slot = a.pair_slot[p];
        const float *fac = a.partials + (a.pair_off[slot] - pair_begin) * WSLOT;
        const int st0 = uniform(__float_as_int(fac[NFW * NFW]));
        if (st0 < 0) continue;  // no refinement for this row
        const int64_t i = a.rows[slot];
        const int64_t beg = a.ptr[i];
        const int n = (int)(a.ptr[i + 1] - beg);
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        __syncthreads();
        if (tid < NFW) L.u[tid] = tid < a.nf ? a.out[i * a.nf + tid] : 0.f;
        if ((st0 >> 16) & 1) wide_resid_row<double>(a, L, p, pair_begin, slot, beg, n, s);
        else wide_resid_row<float>(a, L, p, pair_begin, slot, beg, n, s);
    }
}

// Rows without entries (the only full-data light rows at these ranks).
__global__ __launch_bounds__(WT) void k_wide_empty(SweepArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * WT + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * WT) >> 6;
    for (int64_t t = wave; t < a.count; t += nw) {
        const int64_t i = a.perm[t];
        for (int c = lane; c < a.nf; c += 64) a.out[i * a.nf + c] = 0.f;
        if (lane == 0) atomicAdd(&a.stats[ST_EMPTY], 1ull);
    }
}

// Kept positions of rows [row_begin, row_end) (core_select): one wavefront per
// row, lane a walks the row for columns a and 64 + a.
__global__ __launch_bounds__(WT) void k_select_wide(SelectArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * WT + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * WT) >> 6;
    const int64_t cnt = a.row_end - a.row_begin;
    for (int64_t t = wave; t < cnt; t += nw) {
        const int64_t i = a.row_begin + t;
        const int64_t beg = a.ptr[i];
        const int n = (int)(a.ptr[i + 1] - beg);
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        if (s == 0) continue;
        for (int hc = 0; hc < 2; ++hc) {
            const int col = 64 * hc + lane;
            const bool live = col < a.nf;
            Cut c{0, 0, false, true};
            if (s < n && live) c = Cut{a.cutT[t * NFW + col], a.cutK[t * NFW + col], false, false};
            int32_t *dst = a.sel_pos + a.sel_ptr[t] + (int64_t)min(col, a.nf - 1) * s;
            int q = 0;
            for (int k0 = 0; k0 < n; k0 += 64) {
                const int m = min(64, n - k0);
                const int colv = lane < m ? a.idx[beg + k0 + lane] : 0;
                for (int j = 0; j < m; ++j) {
                    const int r = __builtin_amdgcn_readlane(colv, j);
                    const float x = live ? a.other[(size_t)r * a.nf + col] : 0.f;
                    if (live && kept(c, key_of(x), k0 + j)) {
                        if (q < s) dst[q] = k0 + j;
                        ++q;
                    }
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_wide_empty(const SweepArgs &a, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wide_empty, dim3(grid_of((a.count + 3) / 4, 65536)), dim3(WT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_wide_gram(const HeavyArgs &a, int64_t pair_begin, int64_t pair_end, bool x6, hipStream_t s) {
    if (pair_end <= pair_begin) return hipSuccess;
    if (a.nf <= NF || a.nf > NFW) return hipErrorInvalidValue;
    // buffer offsets are 24-bit products row * 4 n_f plus 32-bit sums
    const bool buf = a.other_rows > 0 && a.other_rows < (1 << 24) &&
                     a.other_rows * (int64_t)a.nf * 4 <= (int64_t)0x7FFFFFFF;
    const dim3 grid(grid_of(pair_end - pair_begin, 65536));
    if (buf && x6) hipLaunchKernelGGL((k_wide_gram<true, true>), grid, dim3(WT), 0, s, a, pair_begin, pair_end);
    else if (buf) hipLaunchKernelGGL((k_wide_gram<true, false>), grid, dim3(WT), 0, s, a, pair_begin, pair_end);
    else if (x6) hipLaunchKernelGGL((k_wide_gram<false, true>), grid, dim3(WT), 0, s, a, pair_begin, pair_end);
    else hipLaunchKernelGGL((k_wide_gram<false, false>), grid, dim3(WT), 0, s, a, pair_begin, pair_end);
    return hipGetLastError();
}

hipError_t launch_wide_solve(const HeavyArgs &a, int64_t slot_begin, int64_t slot_end, int64_t pair_base,
                             hipStream_t s) {
    if (slot_end <= slot_begin) return hipSuccess;
    if (a.nf <= NF || a.nf > NFW) return hipErrorInvalidValue;
    const dim3 grid(grid_of(slot_end - slot_begin, 65536));
    if (a.refine) hipLaunchKernelGGL(k_wide_refine, grid, dim3(WT), 0, s, a, slot_begin, slot_end, pair_base);
    else hipLaunchKernelGGL(k_wide_solve, grid, dim3(WT), 0, s, a, slot_begin, slot_end, pair_base);
    return hipGetLastError();
}

hipError_t launch_wide_resid(const HeavyArgs &a, int64_t pair_begin, int64_t pair_end, hipStream_t s) {
    if (pair_end <= pair_begin) return hipSuccess;
    if (a.nf <= NF || a.nf > NFW) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_wide_resid, dim3(grid_of(pair_end - pair_begin, 65536)), dim3(WT), 0, s, a, pair_begin,
                       pair_end);
    return hipGetLastError();
}

hipError_t launch_select_wide(const SelectArgs &a, hipStream_t s) {
    const int64_t cnt = a.row_end - a.row_begin;
    if (cnt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select_wide, dim3(grid_of((cnt + 3) / 4, 65536)), dim3(WT), 0, s, a);
    return hipGetLastError();
}

}  // namespace coreals
