// UNIF, the uniform-subsampling comparator of Section 5 (gfx950).
//
// Each regression draws s = budget(n) of its n entries uniformly without
// replacement and solves that sample's ridge system
//     (X_S^T X_S + lambda s E) u = X_S^T y_S.
// The draw keeps the s entries with the smallest key h(seed, row, col), the
// upper 32 bits of splitmix64 (Steele, Lea and Flood, 2014) at
// seed * 0x9E3779B97F4A7C15 + row * n_cols + col; ties keep the smaller
// position.  Keys are computed where they are needed, never stored.
//
//   k_unif_select  one wavefront per row finds the row's cut (T, K): kept iff
//                  key < T, or key == T and position <= K.  Four radix passes
//                  over 8-bit digits of the key (smallest first, a per-wave
//                  LDS histogram and a wave prefix sum), then one position
//                  pass when keys tie at T.
//   k_sweep_unif   light rows: one wavefront per row stages the row, walks
//                  the kept entries (a row mask, the same for every column)
//                  and accumulates X_S^T X_S and X_S^T y_S in registers, then
//                  the register LDL^T solve (the system is symmetric positive
//                  definite for lambda s > 0).
// Heavy rows use the heavy-row Gram with the unkept entries zeroed and the
// heavy-row solve with lambda s on the diagonal.
#include "rowops.hpp"

namespace coreals {

namespace {

struct UnifSelLds {
    uint32_t hist[256];
};

// Cut of every row in [0, n_rows): T[i] (key threshold) and K[i] (position
// bound among keys equal to T).  s >= n keeps everything (T = 2^32 - 1, K =
// INT_MAX), s = 0 nothing (T = 0, K = -1).
__global__ __launch_bounds__(WPB * 64) void k_unif_select(const int64_t *ptr, const int32_t *idx, int64_t n_rows,
                                                          int64_t n_cols, uint32_t num, uint32_t den,
                                                          int32_t min_keep, uint64_t seed, uint32_t *T,
                                                          int32_t *K) {
    __shared__ UnifSelLds lds[WPB];
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    UnifSelLds &L = lds[w];
    for (int64_t i = (int64_t)blockIdx.x * WPB + w; i < n_rows; i += (int64_t)gridDim.x * WPB) {
        const int64_t beg = ptr[i];
        const int n = (int)(ptr[i + 1] - beg);
        const int s = (int)budget_of(n, num, den, min_keep);
        if (s >= n || s == 0) {
            if (lane == 0) {
                T[i] = s == 0 ? 0u : 0xFFFFFFFFu;
                K[i] = s == 0 ? -1 : 0x7FFFFFFF;
            }
            continue;
        }
        uint32_t prefix = 0;
        int rem = s;  // entries still to keep among those on the prefix
        bool done = false;
        uint32_t tT = 0;
        int tK = 0x7FFFFFFF;
        for (int pass = 0; pass < 4 && !done; ++pass) {
            const int shift = 24 - 8 * pass;
            const uint32_t hmask = pass == 0 ? 0u : ~((1u << (shift + 8)) - 1u);
            for (int d = lane; d < 256; d += 64) L.hist[d] = 0u;
            wave_sync();
            for (int k = lane; k < n; k += 64) {
                const uint32_t key = unif_key(seed, i, n_cols, idx[beg + k]);
                if ((key & hmask) == prefix) atomicAdd(&L.hist[(key >> shift) & 255u], 1u);
            }
            wave_sync();
            // lane l owns digits 4l .. 4l + 3; exclusive prefix over lanes
            uint32_t h[4];
            uint32_t tot = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                h[q] = L.hist[4 * lane + q];
                tot += h[q];
            }
            uint32_t incl = tot;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t v = __shfl_up(incl, o);
                if (lane >= o) incl += v;
            }
            uint32_t cum = incl - tot;
            int dsel = -1;
            uint32_t below = 0, hsel = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (dsel < 0 && cum + h[q] >= (uint32_t)rem) {
                    dsel = 4 * lane + q;
                    below = cum;
                    hsel = h[q];
                }
                cum += h[q];
            }
            // the first lane (smallest digits) whose range reaches rem
            const uint64_t hit = __ballot(dsel >= 0);
            const int src = __ffsll((unsigned long long)hit) - 1;
            const int d = __shfl(dsel, src);
            const uint32_t bl = __shfl(below, src), hs = __shfl(hsel, src);
            prefix |= (uint32_t)d << shift;
            rem -= (int)bl;
            if ((int)hs == rem) {  // every key on this prefix is kept
                done = true;
                tT = prefix | ((1u << shift) - 1u);
                tK = 0x7FFFFFFF;
            }
            wave_sync();
        }
        if (!done) {
            // keys equal to T = prefix: keep the first rem of them by position
            tT = prefix;
            int cnt = 0;
            for (int k0 = 0; k0 < n && tK == 0x7FFFFFFF; k0 += 64) {
                const int k = k0 + lane;
                const bool eq = k < n && unif_key(seed, i, n_cols, idx[beg + min(k, n - 1)]) == tT;
                const uint64_t b = __ballot(eq);
                const int c = __popcll(b);
                if (cnt + c >= rem) {
                    // the (rem - cnt)-th set bit of b
                    uint64_t bb = b;
                    for (int t = 1; t < rem - cnt; ++t) bb &= bb - 1;
                    tK = k0 + __ffsll((unsigned long long)bb) - 1;
                }
                cnt += c;
            }
        }
        if (lane == 0) {
            T[i] = tT;
            K[i] = tK;
        }
    }
}

// Light rows: every class of the schedule in one persistent launch.
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_sweep_unif(
    SweepArgs a, uint64_t seed, int64_t n_cols, const uint32_t *uT, const int32_t *uK) {
    using LDS = WaveLdsT<CK, true>;
    __shared__ LDS lds[WPB];
    const int w = wave_index();
    const int lane0 = threadIdx.x & 63;
    LDS &L = lds[w];
    const bool vec4 = (a.nf == NF) && ((reinterpret_cast<uintptr_t>(a.other) & 15) == 0);
    for (;;) {
        unsigned int got = 0;
        if (lane0 == 0) got = atomicAdd(a.queue, 1u);
        const int64_t slot = (int64_t)(unsigned int)__builtin_amdgcn_readfirstlane((int)got);
        if (slot >= a.count) break;
        const int lane = opaque_lane(lane0);
        const int64_t i = a.perm[slot];
        const int64_t beg = a.ptr[i];
        const int n = (int)(a.ptr[i + 1] - beg);
        if (n == 0) {
            if (lane < a.nf) a.out[i * a.nf + lane] = 0.f;
            if (lane == 0) atomicAdd(&a.stats[ST_EMPTY], 1ull);
            continue;
        }
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        const uint32_t T = uT[i];
        const int K = uK[i];
        RowCtx r{a.idx, a.val, a.other, beg, n, a.nf, vec4, -1};
        float A[NF];
#pragma unroll
        for (int b = 0; b < NF; ++b) A[b] = 0.f;
        float rhs = 0.f;
        for (int k0 = 0; k0 < n; k0 += CK) {
            stage(L, r, k0, lane);
            const int m = min(CK, n - k0);
            bool kp = false;
            if (lane < m) {
                const uint32_t key = unif_key(seed, i, n_cols, L.col[lane]);
                kp = key < T || (key == T && k0 + lane <= K);
            }
            uint64_t km = __ballot(kp);  // the same kept rows for every column
            while (km) {
                const int k = __ffsll((unsigned long long)km) - 1;
                km &= km - 1;
                const float xa = L.X[k][lane];
#pragma unroll
                for (int b4 = 0; b4 < NF / 4; ++b4) {
                    const float4 xr = *reinterpret_cast<const float4 *>(&L.X[k][b4 * 4]);
                    A[4 * b4 + 0] = fmaf(xa, xr.x, A[4 * b4 + 0]);
                    A[4 * b4 + 1] = fmaf(xa, xr.y, A[4 * b4 + 1]);
                    A[4 * b4 + 2] = fmaf(xa, xr.z, A[4 * b4 + 2]);
                    A[4 * b4 + 3] = fmaf(xa, xr.w, A[4 * b4 + 3]);
                }
                rhs = fmaf(xa, L.y[k], rhs);
            }
        }
        finish_system(A, rhs, (float)((double)a.lam * (double)s), lane, a.nf);
        float u = 0.f;
        if (!solve<false>(A, rhs, lane, a.nf, system_tol(A, a.nf), u, L)) {
            u = 0.f;  // singular sample system (s = 0 rows never reach here)
            if (lane == 0) atomicAdd(&a.stats[ST_FALLBACK], 1ull);
        }
        if (lane < a.nf) a.out[i * a.nf + lane] = u;
    }
}

}  // namespace

hipError_t launch_unif_select(const int64_t *ptr, const int32_t *idx, int64_t n_rows, int64_t n_cols, uint32_t num,
                              uint32_t den, int32_t min_keep, uint64_t seed, uint32_t *T, int32_t *K,
                              hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    int64_t blocks = (n_rows + WPB - 1) / WPB;
    if (blocks > 256 * 64) blocks = 256 * 64;
    hipLaunchKernelGGL(k_unif_select, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, ptr, idx, n_rows, n_cols, num,
                       den, min_keep, seed, T, K);
    return hipGetLastError();
}

hipError_t launch_sweep_unif(const SweepArgs &a, uint64_t seed, int64_t n_cols, const uint32_t *T, const int32_t *K,
                             int max_blocks, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    int64_t blocks = (a.count + WPB - 1) / WPB;
    if (max_blocks > 0 && blocks > max_blocks) blocks = max_blocks;
    if (blocks > 256 * 64) blocks = 256 * 64;
    hipLaunchKernelGGL(k_sweep_unif, dim3((unsigned)blocks), dim3(WPB * 64), 0, s, a, seed, n_cols, T, K);
    return hipGetLastError();
}

}  // namespace coreals
