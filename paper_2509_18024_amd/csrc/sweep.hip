// Light rows of an ALS half-sweep (gfx950): one wavefront solves one row
// regression at a time; a workgroup holds WPB independent wavefronts.
//
//   1. stage:  design rows X[k] = other[idx[k]] gathered into LDS in chunks of
//              CK (16 lanes per 256-byte factor row, float4 loads).
//   2. select: CES (Algorithm 1) by an insertion network of SMAX registers per
//              lane (lane a keeps the s largest keys of column a), the tie cut
//              fixed by a position pass when the threshold key repeats.
//   3. Gram:   row a of X*^T X and entry a of X*^T y (eq. core_ui), lambda n_i
//              on the diagonal; core rows visit only each column's kept rows.
//   4. solve:  pivoted LU in registers, or LDL^T when s == n (eq. (U)).  A
//              pivot below n_f 2^-23 max|A| sends a core row to the full-data
//              update.
//
// Rows of the two smallest network classes with at most 32 entries solve the
// same system in its n x n Woodbury form (woodbury_solve), when the data
// bound the cancellation that form incurs.
//
// The check variant (fold-in answers) inserts between 2 and 3 the relative
// residual |b - A g| / |b| of a candidate g, formed matrix-free from the
// staged rows (b - A g = X*^T (y - X g) - lambda n_i g), and skips 3 and 4
// when it is within the tolerance.
#include "rowops.hpp"

namespace coreals {

namespace {

constexpr int WB_WAVES = 3;  // waves per SIMD of the Woodbury-class kernels

template <int SEL, class LDS>
__device__ __forceinline__ Cut select_for_class(LDS &L, RowCtx &r, int s, int lane) {
    if constexpr (SEL == CLS_NET1) return select_net<1>(L, r, s, lane);
    else if constexpr (SEL == CLS_NET2) return select_net<2>(L, r, s, lane);
    else if constexpr (SEL == CLS_NET4) return select_net<4>(L, r, s, lane);
    else if constexpr (SEL == CLS_NET8) return select_merge<8>(L, r, s, lane);
    else if constexpr (SEL == CLS_NET16) return select_merge<16>(L, r, s, lane);
    else return select_merge<32>(L, r, s, lane);
}

// CHECK (fold-in answers): the row's candidate solution a.guess[i] is kept when
// the relative residual of the row's system (the one the sweep would solve)
// is at most a.tol; otherwise the row is solved exactly as in the sweep.
template <int CLS, bool CHECK>
__device__ __forceinline__ void sweep_rows(const SweepArgs &a) {
    // the two smallest classes solve in Woodbury form from one chunk of at
    // most WB_D rows: 32-row chunks, half the LDS per wavefront
    using LDS = WaveLdsT<(!CHECK && (CLS == CLS_NET1 || CLS == CLS_NET2)) ? WB_D : CK>;
    __shared__ LDS lds[WPB];
    const int w = wave_index();
    const int lane0 = threadIdx.x & 63;
    LDS &L = lds[w];
    const bool vec4 = (a.nf == NF) && ((reinterpret_cast<uintptr_t>(a.other) & 15) == 0);

    // persistent launch: each wavefront takes the next row of the class from
    // an atomic counter (rows are ordered by decreasing degree)
    for (;;) {
        unsigned int got = 0;
        if (lane0 == 0) got = atomicAdd(a.queue, 1u);
        const int64_t slot = (int64_t)(unsigned int)__builtin_amdgcn_readfirstlane((int)got);
        if (slot >= a.count) break;
        const int lane = opaque_lane(lane0);
        const int64_t i = a.perm[slot];
        const int64_t beg = a.ptr[i];
        const int n = (int)(a.ptr[i + 1] - beg);
        RowCtx r{a.idx, a.val, a.other, beg, n, a.nf, vec4, -1};
        if (n == 0) {
            if (lane < a.nf) a.out[i * a.nf + lane] = 0.f;
            if (lane == 0) {
                atomicAdd(&a.stats[ST_EMPTY], 1ull);
                if constexpr (CHECK) {
                    a.path[i] = 1;
                    a.rho[i] = __builtin_inff();
                }
            }
            continue;
        }
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        const float lamn = (float)((double)a.lam * (double)n);
        constexpr bool kCore = CLS != CLS_FULL;
        float g = 0.f;
        if constexpr (CHECK) {
            g = lane < a.nf ? a.guess[i * a.nf + lane] : 0.f;
            wave_sync();
            L.urhs[lane] = g;
            wave_sync();
        }
        Cut c{0, 0, false, true};
        if constexpr (kCore) {
            if (s == 0) c = Cut{0, 0, true, false};
            else c = select_for_class<CLS>(L, r, s, lane);
        }
        if constexpr (CHECK) {
            double rho, bsum;
            resid_range(L, r, c, 0, n, lane, rho, bsum);
            rho -= (double)a.lam * (double)n * (double)g;
            const double rel = rel_residual(rho, bsum, lane, a.nf);
            const bool accept = rel <= (double)a.tol;  // false for NaN
            if (lane == 0) {
                a.rho[i] = (float)rel;
                a.path[i] = accept ? 0 : 1;
                if (!accept) atomicAdd(&a.stats[ST_FOLDIN_EXACT], 1ull);
            }
            if (accept) {
                if (lane < a.nf) a.out[i * a.nf + lane] = g;
                continue;
            }
        }
        if constexpr (!CHECK && (CLS == CLS_NET1 || CLS == CLS_NET2)) {
            // few entries: the n x n Woodbury form of the same system
            if (n <= WB_D && s > 0 && a.lam > 0.f) {
                stage(L, r, 0, lane);  // the whole row is chunk 0
                bool masked;
                float uw;
                if (woodbury_solve(L, c, lane, n, a.nf, a.lam, lamn, masked, uw)) {
                    if (lane < a.nf) a.out[i * a.nf + lane] = uw;
                    continue;
                }
                if (masked) r.staged = -1;  // L.X holds the masked rows: re-stage
            }
        }
        float A[NF];
        float rhs;
        float u = 0.f;
        // attempt 0: the core system; attempt 1 (core rows whose system is
        // singular): the full-data update of eq. (U)
#pragma unroll 1
        for (int attempt = 0; attempt < 2; ++attempt) {
            if constexpr (kCore) gram_range_sparse(L, r, c, 0, n, lane, A, rhs);
            else gram(L, r, c, lane, A, rhs);
            finish_system(A, rhs, lamn, lane, a.nf);
            const bool ok = solve<kCore>(A, rhs, lane, a.nf, system_tol(A, a.nf), u, L);
            if (ok) break;
            u = 0.f;
            if (!kCore || attempt == 1) break;
            if (lane == 0) atomicAdd(&a.stats[ST_FALLBACK], 1ull);
            c = Cut{0, 0, false, true};
        }
        if (lane < a.nf) a.out[i * a.nf + lane] = u;
    }
}

// Full-data light rows (LDL^T, no pivot search): fits two waves per SIMD as is.
__global__ __launch_bounds__(WPB * 64) void k_sweep_full(SweepArgs a) { sweep_rows<CLS_FULL, false>(a); }

// Core light rows: the pivot search raises register demand; capping the
// kernel at two waves per SIMD beats one wave per SIMD.
template <int CLS>
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_sweep_core(SweepArgs a) {
    sweep_rows<CLS, false>(a);
}

// The two smallest classes (Woodbury form, 32-row LDS chunks): latency bound,
// so more waves per SIMD; the registers of the rarely taken 64 x 64 fallback
// spill instead.
template <int CLS>
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(WB_WAVES, WB_WAVES))) void k_sweep_wb(
    SweepArgs a) {
    sweep_rows<CLS, false>(a);
}

// Fold-in answers: residual check of the candidates, exact solve of the rest.
__global__ __launch_bounds__(WPB * 64) void k_check_full(SweepArgs a) { sweep_rows<CLS_FULL, true>(a); }

template <int CLS>
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_check_core(SweepArgs a) {
    sweep_rows<CLS, true>(a);
}

// CES positions for a contiguous row range (the core_select entry point).
// Light rows select here with the same insertion networks as the sweep;
// heavy rows take the cut computed beforehand by the heavy-row selection.
__global__ __launch_bounds__(WPB * 64) void k_select(SelectArgs a) {
    __shared__ WaveLds lds[WPB];
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    WaveLds &L = lds[w];
    const bool vec4 = (a.nf == NF) && ((reinterpret_cast<uintptr_t>(a.other) & 15) == 0);
    const int64_t cnt = a.row_end - a.row_begin;
    for (int64_t t = (int64_t)blockIdx.x * WPB + w; t < cnt; t += (int64_t)gridDim.x * WPB) {
        const int64_t i = a.row_begin + t;
        const int64_t beg = a.ptr[i];
        const int n = (int)(a.ptr[i + 1] - beg);
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        if (s == 0) continue;
        int32_t *dst = a.sel_pos + a.sel_ptr[t] + (int64_t)lane * s;
        RowCtx r{a.idx, nullptr, a.other, beg, n, a.nf, vec4, -1};
        Cut c;
        const int cls = class_of(n, s, a.heavy_n);
        if (s == n) {
            c = Cut{0, 0, false, true};
        } else {
            switch (cls) {
                case CLS_NET1: c = select_net<1>(L, r, s, lane); break;
                case CLS_NET2: c = select_net<2>(L, r, s, lane); break;
                case CLS_NET4: c = select_net<4>(L, r, s, lane); break;
                case CLS_NET8: c = select_merge<8>(L, r, s, lane); break;
                case CLS_NET16: c = select_merge<16>(L, r, s, lane); break;
                case CLS_NET32: c = select_merge<32>(L, r, s, lane); break;
                default: c = Cut{a.cutT[t * 64 + lane], a.cutK[t * 64 + lane], false, false}; break;
            }
        }
        int q = 0;
        for (int k0 = 0; k0 < n; k0 += CK) {
            stage(L, r, k0, lane);
            const int m = min(CK, n - k0);
            for (int k = 0; k < m; ++k) {
                if (kept(c, key_of(L.X[k][lane]), k0 + k)) {
                    if (lane < a.nf && q < s) dst[q] = k0 + k;
                    ++q;
                }
            }
        }
    }
}

template <int CLS, bool CHECK>
hipError_t launch_one(const SweepArgs &a, int max_blocks, hipStream_t s) {
    int64_t blocks = (a.count + WPB - 1) / WPB;
    if (max_blocks > 0 && blocks > max_blocks) blocks = max_blocks;
    if (blocks > 256 * 64) blocks = 256 * 64;
    if constexpr (CHECK) {
        if constexpr (CLS == CLS_FULL)
            hipLaunchKernelGGL(k_check_full, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, a);
        else
            hipLaunchKernelGGL(k_check_core<CLS>, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, a);
    } else {
        if constexpr (CLS == CLS_FULL)
            hipLaunchKernelGGL(k_sweep_full, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, a);
        else if constexpr (CLS == CLS_NET1 || CLS == CLS_NET2)
            hipLaunchKernelGGL(k_sweep_wb<CLS>, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, a);
        else
            hipLaunchKernelGGL(k_sweep_core<CLS>, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, a);
    }
    return hipGetLastError();
}

template <bool CHECK>
hipError_t launch_class(int cls, const SweepArgs &a, int max_blocks, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    switch (cls) {
        case CLS_FULL: return launch_one<CLS_FULL, CHECK>(a, max_blocks, s);
        case CLS_NET1: return launch_one<CLS_NET1, CHECK>(a, max_blocks, s);
        case CLS_NET2: return launch_one<CLS_NET2, CHECK>(a, max_blocks, s);
        case CLS_NET4: return launch_one<CLS_NET4, CHECK>(a, max_blocks, s);
        case CLS_NET8: return launch_one<CLS_NET8, CHECK>(a, max_blocks, s);
        case CLS_NET16: return launch_one<CLS_NET16, CHECK>(a, max_blocks, s);
        case CLS_NET32: return launch_one<CLS_NET32, CHECK>(a, max_blocks, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_sweep_class(int cls, const SweepArgs &a, int max_blocks, hipStream_t s) {
    return launch_class<false>(cls, a, max_blocks, s);
}

hipError_t launch_check_class(int cls, const SweepArgs &a, int max_blocks, hipStream_t s) {
    if (!a.guess || !a.path || !a.rho) return hipErrorInvalidValue;
    return launch_class<true>(cls, a, max_blocks, s);
}

hipError_t launch_select(const SelectArgs &a, hipStream_t s) {
    int64_t cnt = a.row_end - a.row_begin;
    if (cnt <= 0) return hipSuccess;
    int64_t blocks = (cnt + WPB - 1) / WPB;
    if (blocks > 256 * 64) blocks = 256 * 64;
    hipLaunchKernelGGL(k_select, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, a);
    return hipGetLastError();
}

}  // namespace coreals
