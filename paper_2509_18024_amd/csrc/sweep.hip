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
// STRIDED: rows dealt out by wave index with the next rows' indices
// prefetched (the grid must be resident at once); else an atomic row queue.
// FAST (fast variant): no per-row selection; every row, of any class, keeps
// the entries its column's global cut (a.gT, a.gK) keeps, ties decided by
// the row index in `other`.
// IMPL (implicit feedback): the system G + X*^T W X + lambda E with W =
// diag(alpha y), right-hand side X*^T (1 + alpha y), G = a.G.
// WB: 1 (default) the two smallest classes try the Woodbury form first and
// fall back to the n_f x n_f system in the same kernel; 2 Woodbury only,
// rows it does not solve are listed for a second launch (which frees the
// registers of the n_f x n_f solve); 0 never.
template <int CLS, bool CHECK, bool STRIDED, bool FAST = false, bool IMPL = false, int WB = 1>
__device__ __forceinline__ void sweep_rows(const SweepArgs &a) {
    constexpr bool kWb = WB > 0 && !CHECK && !IMPL && (FAST || CLS == CLS_NET1 || CLS == CLS_NET2);
    // the two smallest classes solve in Woodbury form from one chunk of at
    // most WB_D rows: 32-row chunks, half the LDS per wavefront
    using LDS = WaveLdsT<(kWb && !FAST) ? WB_D : CK, FAST>;
    __shared__ LDS lds[WPB];
    const int w = wave_index();
    const int lane0 = threadIdx.x & 63;
    LDS &L = lds[w];
    const bool vec4 = (a.nf == NF) && ((reinterpret_cast<uintptr_t>(a.other) & 15) == 0);
    const int gT = FAST ? a.gT[lane0] : 0, gK = FAST ? a.gK[lane0] : 0;

    // One row: i its index, [beg, beg + n) its entries; if STRIDED, col0 / y0
    // hold the column indices and ratings of its first LDS chunk (lane j:
    // entry j).
    auto row = [&](int64_t i, int64_t beg, int n, int lane, int col0, float y0) {
        RowCtx r{a.idx, a.val, a.other, beg, n, a.nf, vec4, -1};
        if constexpr (STRIDED)
            if (n > 0) stage_loaded(L, r, 0, col0, y0, lane);  // indices prefetched
        if (n == 0) {
            if (lane < a.nf) a.out[i * a.nf + lane] = 0.f;
            if (lane == 0) {
                atomicAdd(&a.stats[ST_EMPTY], 1ull);
                if constexpr (CHECK) {
                    a.path[i] = 1;
                    a.rho[i] = __builtin_inff();
                }
            }
            return;
        }
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        const float lamn = (float)((double)a.lam * (double)n);
        constexpr bool kCore = FAST || CLS != CLS_FULL;
        float g = 0.f;
        if constexpr (CHECK) {
            g = lane < a.nf ? a.guess[i * a.nf + lane] : 0.f;
            wave_sync();
            L.urhs[lane] = g;
            wave_sync();
        }
        Cut c{0, 0, false, true};
        if constexpr (FAST) {
            c = Cut{gT, gK, false, false};
        } else if constexpr (kCore) {
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
                return;
            }
        }
        if constexpr (kWb) {
            // few entries: the n x n Woodbury form of the same system
            if (n <= WB_D && (FAST || s > 0) && a.lam > 0.f) {
                stage(L, r, 0, lane);  // the whole row is chunk 0 (staged above)
                bool masked;
                float uw;
                if (woodbury_solve(L, c, lane, n, a.nf, a.lam, lamn, masked, uw)) {
                    if (lane < a.nf) a.out[i * a.nf + lane] = uw;
                    return;
                }
                if (masked) r.staged = -1;  // L.X holds the masked rows: re-stage
            }
            if constexpr (WB == 2) {
                if (lane == 0) a.fb_rows[atomicAdd(a.fb_count, 1u)] = (int32_t)i;
                return;
            }
        }
        float A[NF];
        float rhs;
        float u = 0.f;
        // attempt 0: the core system by elimination without row exchanges;
        // attempt 1 (growth or a small pivot): the same system, pivoted LU;
        // attempt 2 (core rows whose system is singular): the full-data
        // update of eq. (U)
#pragma unroll 1
        for (int attempt = 0; attempt < 3; ++attempt) {
            if constexpr (IMPL) {
                gram_range_sparse<LDS, true>(L, r, c, 0, n, lane, A, rhs, a.alpha);
                finish_system_implicit(A, rhs, a.G, a.lam, lane, a.nf);
            } else {
                if constexpr (kCore) gram_range_sparse(L, r, c, 0, n, lane, A, rhs);
                else gram(L, r, c, lane, A, rhs);
                finish_system(A, rhs, lamn, lane, a.nf);
            }
            bool ok;
            if constexpr (kCore) {
                if (attempt == 0) ok = solve_unpivoted(A, rhs, lane, a.nf, system_tol(A, a.nf), u, L);
                else ok = solve<true>(A, rhs, lane, a.nf, system_tol(A, a.nf), u, L);
            } else {
                ok = solve<false>(A, rhs, lane, a.nf, system_tol(A, a.nf), u, L);
            }
            if (ok) break;
            u = 0.f;
            if (!kCore || attempt == 2) break;
            if (attempt == 0 && lane == 0) atomicAdd(&a.stats[ST_PIVOTED], 1ull);
            if (attempt == 1) {
                if (lane == 0) atomicAdd(&a.stats[ST_FALLBACK], 1ull);
                c = Cut{0, 0, false, true};
            }
        }
        if (lane < a.nf) a.out[i * a.nf + lane] = u;
    };

    if constexpr (STRIDED) {
        // Wave g takes rows g, g + G, g + 2G, ... of the class (G waves in the
        // grid, all resident; rows of similar degree, so the shares balance).
        // No row counter: for rows this small a single atomic counter limits
        // the class by its throughput.  And the next rows are known, so their
        // bounds and indices load while this one is solved.  Pipeline: indices
        // of row t + 1, bounds of row t + 2 and the row number of row t + 3 are
        // fetched during row t.
        const int64_t G = (int64_t)gridDim.x * WPB;
        const int64_t cnt = a.count;
        const int lane = opaque_lane(lane0);
        // z = 0, opaque to the compiler: the prefetched values stay in vector
        // registers (per-lane loads) and become scalars only when their row
        // starts, so no wait for them is placed right after their loads
        const int z = lane >> 6;
        auto uni = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
        auto uni64 = [](int64_t v) {
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
            return (int64_t)(((uint64_t)hi << 32) | lo);
        };
        // row number of slot t (row 0, which exists, past the class: never solved)
        auto row_of = [&](int64_t t) -> int { return t < cnt ? a.perm[t + z] : 0; };
        int64_t slot = (int64_t)blockIdx.x * WPB + w;
        int i0 = row_of(slot), i1 = row_of(slot + G), i2 = row_of(slot + 2 * G);
        int64_t beg0 = a.ptr[i0 + z], end0 = a.ptr[i0 + 1 + z];
        int64_t beg1 = a.ptr[i1 + z], end1 = a.ptr[i1 + 1 + z];
        int col0 = 0;
        float y0 = 0.f;
        if (lane < min((int64_t)LDS::rows, end0 - beg0)) {
            col0 = a.idx[beg0 + lane];
            y0 = a.val ? a.val[beg0 + lane] : 0.f;
        }
        for (; slot < cnt; slot += G) {
            const int64_t i = uni(i0), beg = uni64(beg0);
            const int n = uni((int)(end0 - beg0));
            const int colc = col0;
            const float yc = y0;
            // prefetch (each load depends only on values of the previous row)
            col0 = 0;
            y0 = 0.f;
            if (lane < min((int64_t)LDS::rows, end1 - beg1)) {
                col0 = a.idx[beg1 + lane];
                y0 = a.val ? a.val[beg1 + lane] : 0.f;
            }
            beg0 = beg1;
            end0 = end1;
            beg1 = a.ptr[i2 + z];
            end1 = a.ptr[i2 + 1 + z];
            i0 = i1;
            i1 = i2;
            i2 = row_of(slot + 3 * G);
            row(i, beg, n, lane, colc, yc);
        }
    } else {
        // persistent launch: each wavefront takes the next row of the class from
        // an atomic counter (rows are ordered by decreasing degree)
        const int64_t cnt = a.count_dev ? (int64_t)*a.count_dev : a.count;
        for (;;) {
            unsigned int got = 0;
            if (lane0 == 0) got = atomicAdd(a.queue, 1u);
            const int64_t slot = (int64_t)(unsigned int)__builtin_amdgcn_readfirstlane((int)got);
            if (slot >= cnt) break;
            const int lane = opaque_lane(lane0);
            const int64_t i = a.perm[slot];
            const int64_t beg = a.ptr[i];
            row(i, beg, (int)(a.ptr[i + 1] - beg), lane, 0, 0.f);
        }
    }
}

// Full-data light rows (LDL^T, no pivot search): fits two waves per SIMD as is.
__global__ __launch_bounds__(WPB * 64) void k_sweep_full(SweepArgs a) { sweep_rows<CLS_FULL, false, false>(a); }

// Core light rows: the pivot search raises register demand; capping the
// kernel at two waves per SIMD beats one wave per SIMD.  The smallest class
// (rows of at most 19 entries at r = 1/10, solved in Woodbury form from one
// 32-row chunk) claims rows faster than one atomic counter serves them: its
// rows are dealt out by wave index, with the next rows' indices prefetched.
// The larger classes keep the atomic queue, whose dynamic balance measured
// faster for them.
template <int CLS>
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_sweep_core(SweepArgs a) {
    sweep_rows<CLS, false, false>(a);
}

// The smallest class in Woodbury form only (rows it leaves go to k_sweep_rest).
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(WB_WAVES, WB_WAVES))) void k_sweep_net1(
    SweepArgs a) {
    sweep_rows<CLS_NET1, false, true, false, false, 2>(a);
}

// Rows of a Woodbury class that the n x n form left (listed by the class's
// launch): the n_f x n_f system, atomic queue over the list.
template <int CLS>
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_sweep_rest(SweepArgs a) {
    sweep_rows<CLS, false, false, false, false, 0>(a);
}

// The second Woodbury class (rows of 20 to 29 entries at r = 1/10): more
// compute per row, so three waves per SIMD and the atomic row queue (the
// prefetch state does not fit three waves without spilling the Woodbury
// solve); the registers of the rarely taken 64 x 64 fallback spill instead.
template <int CLS>
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(WB_WAVES, WB_WAVES))) void k_sweep_wb(
    SweepArgs a) {
    sweep_rows<CLS, false, false, false, false, 2>(a);
}

// Light rows of the fast variant, every class in one launch (the schedule's
// light rows are contiguous in the row order).
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_sweep_fast(SweepArgs a) {
    sweep_rows<CLS_NET1, false, false, true>(a);
}

// Implicit-feedback Core-ALS, one kernel per degree class.
template <int CLS>
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_sweep_implicit(
    SweepArgs a) {
    sweep_rows<CLS, false, false, false, true>(a);
}

// Fold-in answers: residual check of the candidates, exact solve of the rest.
__global__ __launch_bounds__(WPB * 64) void k_check_full(SweepArgs a) { sweep_rows<CLS_FULL, true, false>(a); }

template <int CLS>
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_check_core(SweepArgs a) {
    sweep_rows<CLS, true, false>(a);
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

// Workgroups of WPB waves of `kernel` that the device holds at once.
int64_t resident_blocks(const void *kernel) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, WPB * 64, 0) != hipSuccess) return 0;
    return (int64_t)cus * per_cu;
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
        else if constexpr (CLS == CLS_NET2)
            hipLaunchKernelGGL(k_sweep_wb<CLS>, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, a);
        else {
            if constexpr (CLS == CLS_NET1) {
                // rows are dealt out by wave index: the grid must be resident at once
                const int64_t fit = resident_blocks(reinterpret_cast<const void *>(&k_sweep_net1));
                if (fit <= 0) return hipErrorLaunchFailure;
                if (blocks > fit) blocks = fit;
                hipLaunchKernelGGL(k_sweep_net1, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, a);
            } else {
                hipLaunchKernelGGL(k_sweep_core<CLS>, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, a);
            }
        }
        if constexpr (CLS == CLS_NET1 || CLS == CLS_NET2) {
            // the rows the Woodbury form left, in a second persistent launch
            // (grid for the worst case; each wave stops at the listed count)
            if (!a.fb_rows || !a.fb_count || !a.fb_queue) return hipErrorInvalidValue;
            SweepArgs b = a;
            b.perm = a.fb_rows;
            b.count_dev = a.fb_count;
            b.queue = a.fb_queue;
            int64_t fb = (a.count + WPB - 1) / WPB;
            if (fb > 1024) fb = 1024;
            hipLaunchKernelGGL(k_sweep_rest<CLS>, dim3((unsigned)fb), dim3(WPB * 64), 0, s, b);
        }
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

hipError_t launch_sweep_implicit(int cls, const SweepArgs &a, int max_blocks, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    if (!a.G) return hipErrorInvalidValue;
    int64_t blocks = (a.count + WPB - 1) / WPB;
    if (max_blocks > 0 && blocks > max_blocks) blocks = max_blocks;
    if (blocks > 256 * 64) blocks = 256 * 64;
    const dim3 g((unsigned)blocks), b(WPB * 64);
    switch (cls) {
        case CLS_FULL: hipLaunchKernelGGL(k_sweep_implicit<CLS_FULL>, g, b, 0, s, a); break;
        case CLS_NET1: hipLaunchKernelGGL(k_sweep_implicit<CLS_NET1>, g, b, 0, s, a); break;
        case CLS_NET2: hipLaunchKernelGGL(k_sweep_implicit<CLS_NET2>, g, b, 0, s, a); break;
        case CLS_NET4: hipLaunchKernelGGL(k_sweep_implicit<CLS_NET4>, g, b, 0, s, a); break;
        case CLS_NET8: hipLaunchKernelGGL(k_sweep_implicit<CLS_NET8>, g, b, 0, s, a); break;
        case CLS_NET16: hipLaunchKernelGGL(k_sweep_implicit<CLS_NET16>, g, b, 0, s, a); break;
        case CLS_NET32: hipLaunchKernelGGL(k_sweep_implicit<CLS_NET32>, g, b, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sweep_fast(const SweepArgs &a, int max_blocks, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    if (!a.gT || !a.gK) return hipErrorInvalidValue;
    int64_t blocks = (a.count + WPB - 1) / WPB;
    if (max_blocks > 0 && blocks > max_blocks) blocks = max_blocks;
    if (blocks > 256 * 64) blocks = 256 * 64;
    hipLaunchKernelGGL(k_sweep_fast, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, a);
    return hipGetLastError();
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
