// Fused core-elements regressions of one ALS half-sweep (gfx950).
//
// One wavefront (64 lanes) solves one row regression at a time; a workgroup
// holds WPB independent wavefronts.  Lane a owns column a of the design
// matrix X (for CES) and row a of the n_f x n_f system (for the solve):
//
//   1. stage:  the row's observed entries are read in chunks of CK; the other
//              side's factor rows X[k] = other[idx[k]] are gathered into LDS
//              (16 lanes per 256-byte factor row, float4 loads).
//   2. select: CES (Algorithm 1).  Lane a finds the s-th largest key of its
//              column, key = bit pattern of |x| (integer compare, so the
//              result is exact and identical to any correct ordering of the
//              fp32 magnitudes), and the tie cut: ties at the threshold are
//              kept at the smallest positions.  Small budgets use an
//              insertion network of SMAX registers; large budgets use a
//              4-bit MSD radix select with per-lane LDS histograms.
//   3. Gram:   row a of X*^T X and entry a of X*^T y (eq. core_ui):
//              A[a][:] += w_a X[k][:],  w_a = x_ka if k is kept in column a.
//              X[k][:] is broadcast from LDS.  lambda n_i goes on the diagonal.
//   4. solve:  Gaussian elimination with partial pivoting in registers (pivot
//              search = wave max + first lane), or symmetric elimination
//              without pivoting (LDL^T) when s == n (full-data rows, eq. (U)).
//              A pivot below n_f 2^-23 max|A| sends the row to the full-data
//              update (LDL^T of X^T X + lambda n E).
#include <utility>

#include "internal.hpp"

namespace coreals {

namespace {

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

struct alignas(16) WaveLds {
    float X[CK][NF + 4];
    float y[CK];
};

struct RadixLds {
    int hist[16][64];
};

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

// Gather chunk [k0, k0 + min(CK, n - k0)) of the design matrix into LDS.
__device__ __forceinline__ void stage(WaveLds &L, RowCtx &r, int k0, int lane) {
    if (r.staged == k0) return;
    wave_sync();
    const int cnt = min(CK, r.n - k0);
    int col = 0;
    float yv = 0.f;
    if (lane < cnt) {
        col = r.idx[r.beg + k0 + lane];
        if (r.val) yv = r.val[r.beg + k0 + lane];
    }
    if (lane < CK) L.y[lane] = yv;
    if (r.vec4) {
#pragma unroll
        for (int t = 0; t < CK / 4; ++t) {
            const int kk = t * 4 + (lane >> 4);
            const int c = __shfl(col, kk);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (kk < cnt) v = *reinterpret_cast<const float4 *>(r.other + (size_t)c * NF + (lane & 15) * 4);
            *reinterpret_cast<float4 *>(&L.X[kk][(lane & 15) * 4]) = v;
        }
    } else {
        for (int kk = 0; kk < CK; ++kk) {
            const int c = __shfl(col, kk);
            float v = 0.f;
            if (kk < cnt && lane < r.nf) v = r.other[(size_t)c * r.nf + lane];
            L.X[kk][lane] = v;
        }
    }
    r.staged = k0;
    wave_sync();
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
__device__ __forceinline__ void tie_pass(WaveLds &L, RowCtx &r, int lane, bool tie, int T, int need, int &K) {
    if (__ballot(tie) == 0ull) return;
    int cnt = 0;
    for (int k0 = 0; k0 < r.n; k0 += CK) {
        stage(L, r, k0, lane);
        const int m = min(CK, r.n - k0);
        for (int k = 0; k < m; ++k) {
            const int key = key_of(L.X[k][lane]);
            if (tie && key == T) {
                ++cnt;
                if (cnt == need) K = k0 + k;
            }
        }
    }
}

// Top-s by an insertion network of SMAX registers kept in descending order.
// Unused slots (SMAX - s of them) hold INT_MAX and pass every key through.
template <int SMAX>
__device__ __forceinline__ Cut select_net(WaveLds &L, RowCtx &r, int s, int lane) {
    int kept_[SMAX];
#pragma unroll
    for (int j = 0; j < SMAX; ++j) kept_[j] = (j < SMAX - s) ? 0x7FFFFFFF : -1;
    int D = -1;  // largest key that fell out of the network
    for (int k0 = 0; k0 < r.n; k0 += CK) {
        stage(L, r, k0, lane);
        const int m = min(CK, r.n - k0);
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

// Exact s-th largest key by a most-significant-digit radix select over 31 key
// bits (7 digits of 4 bits, one of 3), with per-lane histograms in LDS.
__device__ __forceinline__ Cut select_radix(WaveLds &L, RadixLds &H, RowCtx &r, int s, int lane) {
    int prefix = 0, hmask = 0, rem = s, ceq = 0;
    bool done = false;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = pass < 7 ? 27 - 4 * pass : 0;
        const int dmask = pass < 7 ? 15 : 7;
#pragma unroll
        for (int d = 0; d < 16; ++d) H.hist[d][lane] = 0;
        wave_sync();
        for (int k0 = 0; k0 < r.n; k0 += CK) {
            stage(L, r, k0, lane);
            const int m = min(CK, r.n - k0);
            for (int k = 0; k < m; ++k) {
                const int key = key_of(L.X[k][lane]);
                if (!done && (key & hmask) == prefix) atomicAdd(&H.hist[(key >> shift) & dmask][lane], 1);
            }
        }
        wave_sync();
        if (!done) {
            int cum = 0, dsel = 0, below = 0, hsel = 0;
            for (int d = dmask; d >= 0; --d) {
                const int h = H.hist[d][lane];
                if (cum < rem && cum + h >= rem) {
                    dsel = d;
                    below = cum;
                    hsel = h;
                }
                cum += h;
            }
            rem -= below;
            prefix |= dsel << shift;
            hmask |= dmask << shift;
            ceq = hsel;
            // every key carrying this prefix is kept: the cut is the prefix itself
            if (hsel == rem) done = true;
        }
        if (__ballot(!done) == 0ull) break;
    }
    Cut c;
    c.T = prefix;
    c.none = false;
    c.all = false;
    c.K = 0x7FFFFFFF;
    const bool tie = !done && ceq > rem;
    tie_pass(L, r, lane, tie, c.T, rem, c.K);
    return c;
}

// Row a of X*^T X and entry a of X*^T y for the lane's column.
__device__ __forceinline__ void gram(WaveLds &L, RowCtx &r, const Cut &c, int lane, float (&A)[NF], float &rhs) {
#pragma unroll
    for (int b = 0; b < NF; ++b) A[b] = 0.f;
    rhs = 0.f;
    if (c.none) return;
    for (int k0 = 0; k0 < r.n; k0 += CK) {
        stage(L, r, k0, lane);
        const int m = min(CK, r.n - k0);
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

// Diagonal penalty lambda n_i and identity padding for lanes >= nf.
__device__ __forceinline__ void finish_system(float (&A)[NF], float &rhs, float lamn, int lane, int nf) {
    const bool pad = lane >= nf;
#pragma unroll
    for (int b = 0; b < NF; ++b) {
        float v = A[b] + ((b == lane) ? lamn : 0.f);
        A[b] = pad ? ((b == lane) ? 1.f : 0.f) : v;
    }
    if (pad) rhs = 0.f;
}

// Elimination step J of the register-resident solve.  PIVOT: partial pivoting
// (first lane of largest |entry| among rows not yet used); otherwise the pivot
// of step J is row J (symmetric positive definite systems).  The steps are
// expanded at compile time so that every index into A is a constant and A
// stays in VGPRs.
template <bool PIVOT, int J>
__device__ __forceinline__ void elim_step(float (&A)[NF], float &rhs, int lane, int nf, float tol, int &my_step,
                                          bool &ok) {
    int p;
    if constexpr (PIVOT) {
        const bool active = my_step == NF;
        const float cand = active ? fabsf(A[J]) : -1.f;
        const float mx = wave_max(cand);
        const uint64_t bal = __ballot(active && cand == mx);
        p = bal ? (__ffsll((unsigned long long)bal) - 1) : 0;
        p = __builtin_amdgcn_readfirstlane(p);
    } else {
        p = J;
    }
    const float piv = readlane_f(A[J], p);
    ok = ok && (J >= nf || fabsf(piv) > tol);
    const float inv = 1.f / piv;
    const bool elim = PIVOT ? (my_step == NF && lane != p) : (lane > J);
    const float l = elim ? A[J] * inv : 0.f;
    if (lane == p) my_step = J;
#pragma unroll
    for (int c = J + 1; c < NF; ++c) A[c] = fmaf(-l, readlane_f(A[c], p), A[c]);
    rhs = fmaf(-l, readlane_f(rhs, p), rhs);
    if (elim) A[J] = l;
}

// Back substitution step J (pivot rows are found by the step they were used at).
template <bool PIVOT, int J>
__device__ __forceinline__ void back_step(const float (&A)[NF], float &rhs, int lane, int my_step, float &u) {
    int p;
    if constexpr (PIVOT) {
        const uint64_t bal = __ballot(my_step == J);
        p = bal ? (__ffsll((unsigned long long)bal) - 1) : 0;
        p = __builtin_amdgcn_readfirstlane(p);
    } else {
        p = J;
    }
    const float x = readlane_f(rhs, p) / readlane_f(A[J], p);
    if (lane == J) u = x;
    if (my_step < J) rhs = fmaf(-A[J], x, rhs);
}

template <bool PIVOT, int... J>
__device__ __forceinline__ void elim_all(std::integer_sequence<int, J...>, float (&A)[NF], float &rhs, int lane,
                                         int nf, float tol, int &my_step, bool &ok) {
    (elim_step<PIVOT, J>(A, rhs, lane, nf, tol, my_step, ok), ...);
}

template <bool PIVOT, int... J>
__device__ __forceinline__ void back_all(std::integer_sequence<int, J...>, const float (&A)[NF], float &rhs,
                                         int lane, int my_step, float &u) {
    (back_step<PIVOT, NF - 1 - J>(A, rhs, lane, my_step, u), ...);
}

// Solve the register-resident system; returns false when a pivot of the first
// nf steps is <= tol.  On success u holds solution component `lane`.
template <bool PIVOT>
__device__ __forceinline__ bool solve(float (&A)[NF], float rhs, int lane, int nf, float tol, float &u) {
    int my_step = NF;  // elimination step at which this lane's row was the pivot
    bool ok = true;
    elim_all<PIVOT>(std::make_integer_sequence<int, NF>{}, A, rhs, lane, nf, tol, my_step, ok);
    if (!PIVOT) my_step = lane;
    if (!ok) return false;
    u = 0.f;
    back_all<PIVOT>(std::make_integer_sequence<int, NF>{}, A, rhs, lane, my_step, u);
    return true;
}

__device__ __forceinline__ float system_tol(const float (&A)[NF], int nf) {
    float m = 0.f;
#pragma unroll
    for (int b = 0; b < NF; ++b) m = fmaxf(m, fabsf(A[b]));
    m = wave_max(m);
    return (float)nf * 1.1920928955078125e-7f * m;
}

template <int SEL>
__device__ __forceinline__ Cut select_for_class(WaveLds &L, RadixLds *H, RowCtx &r, int s, int lane) {
    if constexpr (SEL == CLS_NET1) return select_net<1>(L, r, s, lane);
    else if constexpr (SEL == CLS_NET2) return select_net<2>(L, r, s, lane);
    else if constexpr (SEL == CLS_NET4) return select_net<4>(L, r, s, lane);
    else if constexpr (SEL == CLS_NET8) return select_net<8>(L, r, s, lane);
    else if constexpr (SEL == CLS_NET16) return select_net<16>(L, r, s, lane);
    else if constexpr (SEL == CLS_NET32) return select_net<32>(L, r, s, lane);
    else return select_radix(L, *H, r, s, lane);
}

template <int CLS>
__global__ __launch_bounds__(WPB * 64) void k_sweep(SweepArgs a) {
    __shared__ WaveLds lds[WPB];
    __shared__ RadixLds rlds[CLS == CLS_RADIX ? WPB : 1];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    WaveLds &L = lds[w];
    RadixLds *H = &rlds[CLS == CLS_RADIX ? w : 0];
    const bool vec4 = (a.nf == NF) && ((reinterpret_cast<uintptr_t>(a.other) & 15) == 0);

    for (int64_t slot = (int64_t)blockIdx.x * WPB + w; slot < a.count; slot += (int64_t)gridDim.x * WPB) {
        const int64_t i = a.perm[slot];
        const int64_t beg = a.ptr[i];
        const int n = (int)(a.ptr[i + 1] - beg);
        RowCtx r{a.idx, a.val, a.other, beg, n, a.nf, vec4, -1};
        if (n == 0) {
            if (lane < a.nf) a.out[i * a.nf + lane] = 0.f;
            if (lane == 0) atomicAdd(&a.stats[ST_EMPTY], 1ull);
            continue;
        }
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        const float lamn = (float)((double)a.lam * (double)n);
        float A[NF];
        float rhs;
        float u = 0.f;
        bool ok;
        if constexpr (CLS == CLS_FULL) {
            Cut c{0, 0, false, true};
            gram(L, r, c, lane, A, rhs);
            finish_system(A, rhs, lamn, lane, a.nf);
            ok = solve<false>(A, rhs, lane, a.nf, system_tol(A, a.nf), u);
            if (!ok) u = 0.f;
        } else {
            Cut c;
            if (s == 0) {
                c = Cut{0, 0, true, false};
            } else {
                c = select_for_class<CLS>(L, H, r, s, lane);
            }
            gram(L, r, c, lane, A, rhs);
            finish_system(A, rhs, lamn, lane, a.nf);
            ok = solve<true>(A, rhs, lane, a.nf, system_tol(A, a.nf), u);
            if (!ok) {
                // singular core system: full-data update of eq. (U)
                if (lane == 0) atomicAdd(&a.stats[ST_FALLBACK], 1ull);
                Cut full{0, 0, false, true};
                gram(L, r, full, lane, A, rhs);
                finish_system(A, rhs, lamn, lane, a.nf);
                ok = solve<false>(A, rhs, lane, a.nf, system_tol(A, a.nf), u);
                if (!ok) u = 0.f;
            }
        }
        if (lane < a.nf) a.out[i * a.nf + lane] = u;
    }
}

// CES positions for a contiguous row range (the core_select entry point).
__global__ __launch_bounds__(WPB * 64) void k_select(SelectArgs a) {
    __shared__ WaveLds lds[WPB];
    __shared__ RadixLds rlds[WPB];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    WaveLds &L = lds[w];
    RadixLds &H = rlds[w];
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
        const int cls = class_of(n, s);
        switch (cls) {
            case CLS_FULL: c = Cut{0, 0, false, true}; break;
            case CLS_NET1: c = select_net<1>(L, r, s, lane); break;
            case CLS_NET2: c = select_net<2>(L, r, s, lane); break;
            case CLS_NET4: c = select_net<4>(L, r, s, lane); break;
            case CLS_NET8: c = select_net<8>(L, r, s, lane); break;
            case CLS_NET16: c = select_net<16>(L, r, s, lane); break;
            case CLS_NET32: c = select_net<32>(L, r, s, lane); break;
            default: c = select_radix(L, H, r, s, lane); break;
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

template <int CLS>
hipError_t launch_one(const SweepArgs &a, hipStream_t s) {
    int64_t blocks = (a.count + WPB - 1) / WPB;
    if (blocks > 256 * 64) blocks = 256 * 64;
    hipLaunchKernelGGL(k_sweep<CLS>, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep_class(int cls, const SweepArgs &a, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    switch (cls) {
        case CLS_FULL: return launch_one<CLS_FULL>(a, s);
        case CLS_NET1: return launch_one<CLS_NET1>(a, s);
        case CLS_NET2: return launch_one<CLS_NET2>(a, s);
        case CLS_NET4: return launch_one<CLS_NET4>(a, s);
        case CLS_NET8: return launch_one<CLS_NET8>(a, s);
        case CLS_NET16: return launch_one<CLS_NET16>(a, s);
        case CLS_NET32: return launch_one<CLS_NET32>(a, s);
        case CLS_RADIX: return launch_one<CLS_RADIX>(a, s);
        default: return hipErrorInvalidValue;
    }
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
