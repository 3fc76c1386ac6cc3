// Heavy rows of a half-sweep (gfx950): rows whose budget exceeds the register
// insertion networks (s > 32) or whose degree exceeds the light-row limit.
//
//   k_key16          the top 16 bits of every |x| of the fixed factor matrix
//                    (exponent and first mantissa byte), half the bytes of a
//                    factor row, for the selection's first two passes.
//   k_heavy_select   one 512-thread workgroup per row computes the CES cut of
//                    all 64 columns (Algorithm 1): an MSD radix select on the
//                    31-bit key |x|, 8 bits per pass, with per-column counters
//                    packed two per 32-bit LDS word (degrees < 65536).  After
//                    two passes (exponent byte, top mantissa byte) the few keys
//                    that share the threshold's 16-bit prefix are collected
//                    into LDS and ranked exactly by (key desc, position asc);
//                    only if more than HEAVY_CAP keys share it do two more
//                    radix passes over the full keys run, and a position pass
//                    where keys equal the threshold.  When the row's cuts of
//                    the previous half-sweep of this side are at hand, one
//                    counting pass over a 256-bin window of 16-bit keys around
//                    each previous threshold replaces the first two passes; it
//                    is exact, because the counts above and inside the window
//                    decide whether the new threshold lies inside (else the
//                    two passes run as before).
//   k_heavy_gram_x6  one wavefront per (row, chunk of `chunk` entries) builds
//                    the chunk's part of X*^T X and X*^T y (eq. core_ui) with
//                    the row's cut, FP32 products from an exact three-way
//                    bf16 split on 32x32x16 bf16 MFMA tiles, and stores it to
//                    scratch (column-major: element (a, b) at b * 64 + a).
//   k_heavy_solve    one wavefront per row sums its partial systems in chunk
//                    order (deterministic), adds lambda n_i, and solves it
//                    (blocked elimination without row exchanges under growth
//                    and multiplier bounds, else pivoted LU).
//
// BF16 precision modes run k_heavy_gram_x6 with one product per tile (the
// operands' bf16 roundings, FP32 accumulation) and add one step of iterative
// refinement: k_heavy_resid forms the partial residuals X*^T (y - X u) of
// each chunk in FP32 or FP64 from the fp32 data (the next 64 rows' gathers in
// flight while a block is reduced), and a
// second k_heavy_solve subtracts lambda n_i u, solves A d = rho with the LU
// factors the first solve kept (in the row's first partial slot) and returns
// u + d.
//
// Fold-in answers (check mode) add k_heavy_check / k_heavy_check_reduce,
// the relative residual of a candidate answer from per-chunk shares, before
// the Gram; rows whose candidate passes are skipped by the later kernels.
#include <type_traits>

#include "rowops.hpp"

namespace coreals {

namespace {

// Eight waves per heavy row and 32 gathers in flight per wave: the passes are
// bound by the latency of the row gathers, so they need many loads in flight.
constexpr int HS_THREADS = 512;
constexpr int HS_WAVES = HS_THREADS / 64;
constexpr int HS_BATCH = 32;

struct HeavySelLds {
    // Narrow rows (n < 65536): bins 2j, 2j+1 of column a share word [j][a] as
    // two 16-bit counters.  Wide rows: word [d - dlo][a] is the 32-bit count of
    // digit d within the half range [dlo, dlo + 128) being counted.
    // the candidate lists are used only after the last counting pass
    union {
        uint32_t hist[128][64];
        struct {
            int ckey[64][HEAVY_CAP + 1];  // padded: column a's list starts in bank a
            int cpos[64][HEAVY_CAP + 1];
        };
    };
    int ccnt[64];
    int prefix[64];
    int rem[64];
    int ceq[64];
    int cum[64];
    int found[64];
    int done[64];
    int T[64];
    int K[64];
    int wlo[64];  // hint pass: the window's lowest 16-bit key
    int flag;
};

// Rows the heavy-row selection cuts: heavy, with something to drop and
// something to keep (s = 0 keeps nothing and needs no cut).
__device__ __forceinline__ bool is_heavy_core(int n, int s, int heavy_n) {
    return class_of(n, s, heavy_n) == CLS_HEAVY && s < n && s > 0;
}

// Factor-row gathers of the selection passes: lane a reads entry a of one
// factor row per load instruction, as raw bits (every test below masks the
// sign).  Padded lanes (a >= n_f) read column n_f - 1 and are never used.
// With a buffer resource (factor matrices below 2^31 bytes) the row offset is
// a scalar operand of the load, so a gather costs one readlane and one scalar
// multiply; otherwise each lane forms a 64-bit address.
template <bool BUF>
struct RowGather;

template <>
struct RowGather<true> {
    __amdgpu_buffer_rsrc_t rs;
    int voff, stride;
    __device__ RowGather(const float *other, int nf, int lane)
        : rs(__builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(other), (short)0, 0x7FFFFFFF, 0x00020000)),
          voff(4 * min(lane, nf - 1)), stride(4 * nf) {}
    __device__ __forceinline__ int bits(int col) const {
        return __builtin_amdgcn_raw_buffer_load_b32(rs, voff, col * stride, 0);
    }
    // a different row per lane
    __device__ __forceinline__ int bits_lane(int col) const {
        return __builtin_amdgcn_raw_buffer_load_b32(rs, voff + col * stride, 0, 0);
    }
};

template <>
struct RowGather<false> {
    const float *p;
    int stride;
    __device__ RowGather(const float *other, int nf, int lane) : p(other + min(lane, nf - 1)), stride(nf) {}
    __device__ __forceinline__ int bits(int col) const { return __float_as_int(p[(size_t)col * stride]); }
};

// The same gathers from the 16-bit key copy (bits 30..15 of each entry, the
// digits of the first two passes): half the bytes of a factor row.
struct KeyGather16 {
    __amdgpu_buffer_rsrc_t rs;
    int voff, stride;
    __device__ KeyGather16(const uint16_t *key16, int nf, int lane)
        : rs(__builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(key16), (short)0, 0x7FFFFFFF, 0x00020000)),
          voff(2 * min(lane, nf - 1)), stride(2 * nf) {}
    __device__ __forceinline__ int bits(int col) const {
        return (int)__builtin_amdgcn_raw_buffer_load_b16(rs, voff, col * stride, 0);
    }
};

// Wave w's chunks of 64 positions (w*64, w*64 + HS_WAVES*64, ...): the next
// chunk's column indices load while the current chunk is gathered.  f(colv,
// c0, m): lane j of colv holds the column of position c0 + j (0 past m).
template <class F>
__device__ __forceinline__ void for_chunks(const int32_t *idx, int64_t beg, int n, int w, int lane, F &&f) {
    int c0 = w * 64;
    if (c0 >= n) return;
    int colv = lane < n - c0 ? idx[beg + c0 + lane] : 0;
    for (;;) {
        const int c1 = c0 + HS_WAVES * 64;
        int next = 0;
        if (c1 < n) next = lane < n - c1 ? idx[beg + c1 + lane] : 0;
        f(colv, c0, min(64, n - c0));
        if (c1 >= n) break;
        colv = next;
        c0 = c1;
    }
}

// One chunk: HS_BATCH gathers in flight, then g(bits, j) for each position
// j < m of the batch, in order.  The bound is uniform: full chunks run without
// tests, and in the last chunk positions past m gather column 0 (a valid row)
// and are skipped.
template <class RG, class G>
__device__ __forceinline__ void gather_chunk(const RG &R, int colv, int m, G &&g) {
    if (m == 64) {
#pragma unroll 1
        for (int j0 = 0; j0 < 64; j0 += HS_BATCH) {
            int b[HS_BATCH];
#pragma unroll
            for (int j = 0; j < HS_BATCH; ++j) b[j] = R.bits(__builtin_amdgcn_readlane(colv, j0 + j));
#pragma unroll
            for (int j = 0; j < HS_BATCH; ++j) g(b[j], j0 + j);
        }
    } else {
#pragma unroll 1
        for (int j0 = 0; j0 < m; j0 += HS_BATCH) {
            int b[HS_BATCH];
#pragma unroll
            for (int j = 0; j < HS_BATCH; ++j) b[j] = R.bits(__builtin_amdgcn_readlane(colv, (j0 + j) & 63));
#pragma unroll
            for (int j = 0; j < HS_BATCH; ++j)
                if (j0 + j < m) g(b[j], j0 + j);
        }
    }
}

// One counting pass over the row: for keys whose bits above `shift` equal the
// column's prefix, count digit d = bits [shift, shift + width).  Narrow rows:
// bins 2j, 2j+1 share word j as two 16-bit counters (the increment is 1 or
// 1 << 16 by the digit's low bit).  Wide rows count only d in [dlo, dhi).
// Columns already resolved count too, into their own words, which no pick
// reads again.  The gathered values hold key bits KOFF.. (shift and hmask are
// given in those units; KOFF = 15 for the 16-bit key copy).
template <bool WIDE, bool FIRST, int WIDTH, int KOFF, class RG>
__device__ __forceinline__ void heavy_hist_pass(HeavySelLds &S, const int32_t *idx, const RG &R, int64_t beg,
                                                int n, int shift, int hmask, int dlo, int dhi, int w, int lane) {
    const int pre = S.prefix[lane] >> KOFF;
    for_chunks(idx, beg, n, w, lane, [&](int colv, int, int m) {
        gather_chunk(R, colv, m, [&](int b, int) {
            const unsigned u = (unsigned)b;
            if constexpr (FIRST) {
                // every key counts by its exponent byte, bits 30..23; the
                // barrier keeps each count next to its load's wait (clustered,
                // the counts of a batch would hold twice the registers)
                atomicAdd(&S.hist[__builtin_amdgcn_ubfe(u, 24 - KOFF, 7)][lane],
                          __umul24(__builtin_amdgcn_ubfe(u, 23 - KOFF, 1), 0xFFFFu) + 1u);
                __builtin_amdgcn_sched_barrier(0);
            } else if constexpr (WIDE) {
                const int d = (int)__builtin_amdgcn_ubfe(u, shift, WIDTH);
                if ((b & hmask) == pre && d >= dlo && d < dhi) atomicAdd(&S.hist[d - dlo][lane], 1u);
            } else {
                if ((b & hmask) == pre)
                    atomicAdd(&S.hist[__builtin_amdgcn_ubfe(u, shift + 1, WIDTH - 1)][lane],
                              __umul24(__builtin_amdgcn_ubfe(u, shift, 1), 0xFFFFu) + 1u);
            }
        });
    });
}

// Hint pass: for keys whose 16-bit key k16 is at least the column's window
// start wlo, count bin min(k16 - wlo, 255) (packed 16-bit counters, as in the
// narrow passes); bin 255 gathers every key at or above wlo + 255.
template <int KOFF, class RG>
__device__ __forceinline__ void heavy_hint_pass(HeavySelLds &S, const int32_t *idx, const RG &R, int64_t beg, int n,
                                                int w, int lane) {
    const int wlo = S.wlo[lane];
    for_chunks(idx, beg, n, w, lane, [&](int colv, int, int m) {
        gather_chunk(R, colv, m, [&](int b, int) {
            const int k16 = (int)__builtin_amdgcn_ubfe((unsigned)b, 15 - KOFF, 16);
            const int d = min(k16 - wlo, 255);
            if (d >= 0) atomicAdd(&S.hist[d >> 1][lane], (d & 1) ? 0x10000u : 1u);
        });
    });
}

// Column a after the hint pass: the rem-th largest key lies in bin d < 255
// (a hit: its 16-bit key is wlo + d, as two narrow passes would have fixed
// it) or outside the window (a miss: returns false).
__device__ __forceinline__ bool heavy_pick_hint(HeavySelLds &S, int a) {
    if (S.done[a]) return true;
    const int rem = S.rem[a];
    int cum = 0, dsel = -1, hsel = 0;
    // eight words (sixteen bins) per batch, their LDS reads in flight together;
    // word j holds bin 2j in its low and bin 2j + 1 in its high half
    for (int w0 = 127; w0 >= 0 && dsel < 0; w0 -= 8) {
        uint32_t wv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) wv[q] = S.hist[w0 - q][a];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int hi = (int)(wv[q] >> 16), lo = (int)(wv[q] & 0xFFFFu);
            if (dsel < 0) {
                if (cum + hi >= rem) {
                    dsel = 2 * (w0 - q) + 1;
                    hsel = hi;
                } else {
                    cum += hi;
                    if (cum + lo >= rem) {
                        dsel = 2 * (w0 - q);
                        hsel = lo;
                    } else {
                        cum += lo;
                    }
                }
            }
        }
    }
    if (dsel < 0 || dsel == 255) return false;
    S.rem[a] = rem - cum;
    S.prefix[a] = (S.wlo[a] + dsel) << 15;
    S.ceq[a] = hsel;
    if (hsel == S.rem[a]) {  // every key with this prefix is kept
        S.done[a] = 1;
        S.T[a] = S.prefix[a];
        S.K[a] = 0x7FFFFFFF;
    }
    return true;
}

// Column a: walk digits dhi-1 .. dlo from the top; if the rem-th largest key
// falls in this range, fix the digit, else carry the running count.
__device__ __forceinline__ void heavy_pick(HeavySelLds &S, int a, int shift, int dlo, int dhi, bool wide) {
    if (S.done[a] || S.found[a]) return;
    int cum = S.cum[a], dsel = -1, below = 0, hsel = 0;
    const int rem = S.rem[a];
    // unrolled so that the LDS reads of several digits are in flight together
#pragma unroll 16
    for (int d = dhi - 1; d >= dlo; --d) {
        const int h = wide ? (int)S.hist[d - dlo][a] : (int)((S.hist[d >> 1][a] >> ((d & 1) << 4)) & 0xFFFFu);
        if (cum < rem && cum + h >= rem) {
            dsel = d;
            below = cum;
            hsel = h;
        }
        cum += h;
    }
    if (dsel < 0) {
        S.cum[a] = cum;
        return;
    }
    S.found[a] = 1;
    S.rem[a] = rem - below;
    S.prefix[a] |= dsel << shift;
    S.ceq[a] = hsel;
    if (hsel == S.rem[a]) {  // every key with this prefix is kept
        S.done[a] = 1;
        S.T[a] = S.prefix[a];
        S.K[a] = 0x7FFFFFFF;
    }
}

// Four workgroups per CU (the LDS allows four): at most 64 VGPRs.  K16: the
// first two passes and the candidate collection read the 16-bit key copy.
template <bool BUF, bool K16>
__global__ __launch_bounds__(HS_THREADS) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_heavy_select(
    HeavyArgs a, int64_t row_begin) {
    __shared__ HeavySelLds S;
    const int tid = threadIdx.x;
    const int w = wave_index();
    const int lane = tid & 63;
    const int nf = a.nf;
    // lane a ranks column col_base + a (ranks above 64: two launches, one per
    // half of the columns)
    const int col = a.col_base + lane;
    const RowGather<BUF> R(a.other, nf, col);
    const KeyGather16 R16(a.key16, nf, col);
    __shared__ int64_t next_t;
    int64_t t = blockIdx.x;
    for (;;) {
        // rows of very different degree: workgroups take the next row from a
        // counter when one is given, else a grid-stride order
        if (a.queue) {
            if (tid == 0) next_t = (int64_t)atomicAdd(a.queue, 1u);
            __syncthreads();
            t = next_t;
            __syncthreads();
        }
        if (t >= a.count) break;
        const int64_t i = a.rows ? (int64_t)a.rows[t] : row_begin + t;
        const int64_t beg = a.ptr[i];
        const int n = (int)(a.ptr[i + 1] - beg);
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        if (!is_heavy_core(n, s, a.heavy_n)) {  // uniform over the workgroup
            if (!a.queue) t += gridDim.x;
            continue;
        }
        const bool wide = n >= 65536;
        if (tid < 64) {
            // padded columns (a >= n_f, all-zero keys) get the cut of a column
            // of equal keys: the first s positions
            const bool pad = a.col_base + tid >= nf;
            S.prefix[tid] = 0;
            S.rem[tid] = s;
            S.done[tid] = pad ? 1 : 0;
            S.ccnt[tid] = 0;
            S.T[tid] = 0;
            S.K[tid] = pad ? s - 1 : 0x7FFFFFFF;
        }
        int hmask = 0;
        bool collected = false, all_done = false;
        int pass0 = 0;
        if (a.hint && !wide) {
            // the previous cuts of this row, where every live column has one
            if (tid == 0) S.flag = 0;
            __syncthreads();
            if (tid < 64) {
                const int h = a.cutT[t * a.cstride + a.col_base + tid];
                const int p16 = max(0, h) >> 15;
                S.wlo[tid] = min(max(p16 - 127, 0), 65535 - 254);
                if (!S.done[tid] && h < 0) atomicOr(&S.flag, 1);
            }
            for (int q = tid; q < 128 * 64; q += HS_THREADS) (&S.hist[0][0])[q] = 0u;
            __syncthreads();
            if (!S.flag) {
                if (K16)
                    heavy_hint_pass<15>(S, a.idx, R16, beg, n, w, lane);
                else
                    heavy_hint_pass<0>(S, a.idx, R, beg, n, w, lane);
                __syncthreads();
                if (tid < 64 && !heavy_pick_hint(S, tid)) atomicOr(&S.flag, 4);
                __syncthreads();
                if (S.flag & 4) {
                    // some threshold left its window: the two first passes
                    if (tid < 64) {
                        const bool pad = a.col_base + tid >= nf;
                        S.prefix[tid] = 0;
                        S.rem[tid] = s;
                        S.done[tid] = pad ? 1 : 0;
                        S.T[tid] = 0;
                        S.K[tid] = pad ? s - 1 : 0x7FFFFFFF;
                    }
                } else {
                    if (tid == 0) S.flag = 0;
                    __syncthreads();
                    if (tid < 64 && !S.done[tid]) {
                        atomicOr(&S.flag, 2);
                        if (S.ceq[tid] > HEAVY_CAP) atomicOr(&S.flag, 1);
                    }
                    __syncthreads();
                    const int f = S.flag;
                    hmask = 0xFFFF << 15;
                    pass0 = 2;
                    if (tid == 0) atomicAdd(&a.stats[ST_HINTED], 1ull);
                    if (!(f & 2)) all_done = true;
                    else if (!(f & 1)) collected = true;
                }
            }
            __syncthreads();
        }
        for (int pass = pass0; pass < 4 && !all_done && !collected; ++pass) {
            const int shift = pass < 3 ? 23 - 8 * pass : 0;
            const int width = pass < 3 ? 8 : 7;
            const int nd = 1 << width;
            if (tid < 64) {
                S.cum[tid] = 0;
                S.found[tid] = 0;
            }
            // narrow rows: one sub-pass over all digits; wide rows: upper half
            // first, the lower half only for columns not yet resolved
            const int nsub = wide ? 2 : 1;
            for (int sub = 0; sub < nsub; ++sub) {
                const int dlo = wide ? (sub == 0 ? nd / 2 : 0) : 0;
                const int dhi = wide ? (sub == 0 ? nd : nd / 2) : nd;
                for (int q = tid; q < 128 * 64; q += HS_THREADS) (&S.hist[0][0])[q] = 0u;
                __syncthreads();
                if (K16 && pass < 2) {
                    // the digits of the first two passes lie in bits 30..15
                    const int sh = shift - 15, hm = hmask >> 15;
                    if (wide)
                        heavy_hist_pass<true, false, 8, 15>(S, a.idx, R16, beg, n, sh, hm, dlo, dhi, w, lane);
                    else if (pass == 0)
                        heavy_hist_pass<false, true, 8, 15>(S, a.idx, R16, beg, n, sh, hm, dlo, dhi, w, lane);
                    else
                        heavy_hist_pass<false, false, 8, 15>(S, a.idx, R16, beg, n, sh, hm, dlo, dhi, w, lane);
                } else if (wide && pass < 3)
                    heavy_hist_pass<true, false, 8, 0>(S, a.idx, R, beg, n, shift, hmask, dlo, dhi, w, lane);
                else if (wide)
                    heavy_hist_pass<true, false, 7, 0>(S, a.idx, R, beg, n, shift, hmask, dlo, dhi, w, lane);
                else if (pass == 0)
                    heavy_hist_pass<false, true, 8, 0>(S, a.idx, R, beg, n, shift, hmask, dlo, dhi, w, lane);
                else if (pass < 3)
                    heavy_hist_pass<false, false, 8, 0>(S, a.idx, R, beg, n, shift, hmask, dlo, dhi, w, lane);
                else
                    heavy_hist_pass<false, false, 7, 0>(S, a.idx, R, beg, n, shift, hmask, dlo, dhi, w, lane);
                __syncthreads();
                if (tid < 64) heavy_pick(S, tid, shift, dlo, dhi, wide);
                __syncthreads();
            }
            if (tid == 0) S.flag = 0;
            __syncthreads();
            // bit 1: some column still open; bit 0: some open column has more
            // than HEAVY_CAP keys on its prefix
            if (tid < 64 && !S.done[tid]) {
                atomicOr(&S.flag, 2);
                if (S.ceq[tid] > HEAVY_CAP) atomicOr(&S.flag, 1);
            }
            __syncthreads();
            const int f = S.flag;
            hmask |= ((1 << width) - 1) << shift;
            if (!(f & 2)) {
                all_done = true;
                break;
            }
            if (pass == 1 && !(f & 1)) {
                collected = true;  // few keys share the 16-bit prefix: rank them in LDS
                break;
            }
        }
        if (all_done) {
            // every cut was fixed by a prefix alone
        } else if (collected) {
            const bool act = !S.done[lane];
            if constexpr (K16 && BUF) {
                // candidates share the 16-bit key: note their positions and
                // columns, then fetch their full keys (about n / 1000 per
                // column, so mostly one load per thread)
                const int pre16 = S.prefix[lane] >> 15;
                for_chunks(a.idx, beg, n, w, lane, [&](int colv, int c0, int m) {
                    gather_chunk(R16, colv, m, [&](int b, int j) {
                        if (act && b == pre16) {
                            const int slot = atomicAdd(&S.ccnt[lane], 1);
                            if (slot < HEAVY_CAP) {
                                S.ckey[lane][slot] = __builtin_amdgcn_readlane(colv, j);
                                S.cpos[lane][slot] = c0 + j;
                            }
                        }
                    });
                });
                __syncthreads();
                const int mc = act ? min(S.ccnt[lane], HEAVY_CAP) : 0;
#pragma unroll 1
                for (int x = w; x < mc; x += HS_WAVES) S.ckey[lane][x] = R.bits_lane(S.ckey[lane][x]) & KEYMASK;
            } else {
                const int pre = S.prefix[lane];
                for_chunks(a.idx, beg, n, w, lane, [&](int colv, int c0, int m) {
                    gather_chunk(R, colv, m, [&](int b, int j) {
                        if (act && (b & hmask) == pre) {
                            const int slot = atomicAdd(&S.ccnt[lane], 1);
                            if (slot < HEAVY_CAP) {
                                S.ckey[lane][slot] = b & KEYMASK;
                                S.cpos[lane][slot] = c0 + j;
                            }
                        }
                    });
                });
            }
            __syncthreads();
            // candidate x of column c is ranked by thread (c, x); exactly one
            // candidate per column has the wanted rank, so T and K get one writer
            for (int q = tid; q < 64 * HEAVY_CAP; q += HS_THREADS) {
                const int c = q & 63, x = q >> 6;
                const int m = min(S.ccnt[c], HEAVY_CAP);
                if (S.done[c] || x >= m) continue;
                const int kx = S.ckey[c][x], px = S.cpos[c][x];
                int rank = 0;
                for (int y = 0; y < m; ++y) {
                    const int ky = S.ckey[c][y], py = S.cpos[c][y];
                    rank += (ky > kx) || (ky == kx && py < px);
                }
                if (rank == S.rem[c] - 1) {  // rank from the top, 0-based
                    S.T[c] = kx;
                    S.K[c] = px;
                }
            }
        } else {
            // all 31 bits resolved: T is the key itself.  Where more keys than
            // needed equal T, the kept ones are the first `need` positions:
            // the positions of the keys equal to T are collected by all waves
            // (batched gathers) and ranked.
            if (tid < 64) {
                if (!S.done[tid]) S.T[tid] = S.prefix[tid];
                S.ccnt[tid] = 0;
            }
            __syncthreads();  // every thread has read the flag of the last pass
            if (tid == 0) S.flag = 0;
            __syncthreads();
            const bool tie = !S.done[lane] && S.ceq[lane] > S.rem[lane];
            if (w == 0) {
                const uint64_t any_tie = __ballot(tie);
                if (lane == 0 && any_tie != 0ull) S.flag = 1;
            }
            __syncthreads();
            if (S.flag) {
                const int T = S.T[lane];
                for_chunks(a.idx, beg, n, w, lane, [&](int colv, int c0, int m) {
                    gather_chunk(R, colv, m, [&](int b, int j) {
                        if (tie && (b & KEYMASK) == T) {
                            const int slot = atomicAdd(&S.ccnt[lane], 1);
                            if (slot < HEAVY_CAP) S.cpos[lane][slot] = c0 + j;
                        }
                    });
                });
                __syncthreads();
                for (int q = tid; q < 64 * HEAVY_CAP; q += HS_THREADS) {
                    const int c = q & 63, x = q >> 6;
                    const bool tie_c = !S.done[c] && S.ceq[c] > S.rem[c];
                    const int m = S.ccnt[c];
                    if (!tie_c || m > HEAVY_CAP || x >= m) continue;
                    const int px = S.cpos[c][x];
                    int rank = 0;
                    for (int y = 0; y < m; ++y) rank += S.cpos[c][y] < px;
                    if (rank == S.rem[c] - 1) S.K[c] = px;
                }
                __syncthreads();
                if (w == 0) {
                    // more equal keys than the lists hold: one wave walks the row
                    const bool over = tie && S.ccnt[lane] > HEAVY_CAP;
                    if (__ballot(over) != 0ull) {
                        const int need = S.rem[lane];
                        int cnt = 0, K = 0x7FFFFFFF;
                        for (int c0 = 0; c0 < n; c0 += 64) {
                            const int m = min(64, n - c0);
                            const int colv = lane < m ? a.idx[beg + c0 + lane] : 0;
                            for (int j = 0; j < m; ++j) {
                                const int key = R.bits(__builtin_amdgcn_readlane(colv, j)) & KEYMASK;
                                if (over && key == T) {
                                    ++cnt;
                                    if (cnt == need) K = c0 + j;
                                }
                            }
                        }
                        if (over) S.K[lane] = K;
                    }
                }
            }
        }
        __syncthreads();
        if (tid < 64) {
            a.cutT[t * a.cstride + a.col_base + tid] = S.T[tid];
            a.cutK[t * a.cstride + a.col_base + tid] = S.K[tid];
        }
        __syncthreads();
        if (!a.queue) t += gridDim.x;
    }
}

__global__ __launch_bounds__(WPB * 64) void k_heavy_solve(HeavyArgs a, int64_t slot_begin, int64_t slot_end,
                                                          int64_t pair_base) {
    __shared__ WaveLds lds[WPB];
    const int w = wave_index();
    const int lane0 = threadIdx.x & 63;
    WaveLds &L = lds[w];
    const bool vec4 = (a.nf == NF) && ((reinterpret_cast<uintptr_t>(a.other) & 15) == 0);
    for (int64_t slot = slot_begin + (int64_t)blockIdx.x * WPB + w; slot < slot_end;
         slot += (int64_t)gridDim.x * WPB) {
        const int lane = opaque_lane(lane0);
        const int64_t i = a.rows[slot];
        if (a.path && a.path[i] == 0) continue;  // fold-in answer accepted
        if (a.pass && a.flag[slot] != a.pass) continue;
        const int64_t beg = a.ptr[i];
        const int n = (int)(a.ptr[i + 1] - beg);
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        // UNIF: lambda times the sample size (the subsample's own system)
        const float lamn = (float)((double)a.lam * (double)(a.unif ? s : n));
        // the first pair's partial slot holds the kept LU factors between the
        // two solves (its partial system has been summed by then)
        // (fast variant: every row's sketch is a core system)
        float *fac = a.partials + (a.pair_off[slot] - pair_base) * (int64_t)(NF + 1) * 64;
        float A[NF];
        float rhs;
        auto build = [&]() {
            rhs = 0.f;
#pragma unroll
            for (int b = 0; b < NF; ++b) A[b] = 0.f;
            for (int64_t p = a.pair_off[slot]; p < a.pair_off[slot + 1]; ++p) {
                const float *src = a.partials + (p - pair_base) * (int64_t)(NF + 1) * 64;
#pragma unroll
                for (int b = 0; b < NF; ++b) A[b] += src[b * 64 + lane];
                rhs += src[NF * 64 + lane];
            }
            if (a.implicit) finish_system_implicit(A, rhs, a.G, a.lam, lane, a.nf);
            else finish_system(A, rhs, lamn, lane, a.nf);
        };
        build();
        float u = 0.f;
        const bool core = !a.unif && (a.gpos || s < n);
        bool ok;
        if (a.keep) {
            // a refinement step follows: keep the factors for it
            float rs = 0.f;  // |A|_inf, for the condition estimate
#pragma unroll
            for (int b = 0; b < NF; ++b) rs += fabsf(A[b]);
            const float anorm = __int_as_float(wave_max_key(__float_as_int(rs)));
            int my_step;
            float r[1] = {rhs};
            ok = lu_keep(A, r, lane, a.nf, system_tol(A, a.nf), my_step, L);
            int need64 = 0;        // bit 16 of the kept step: FP64 residual for this row
            bool regram = false;   // ALS_PREC_AUTO: Gram again with FP32 products
            if (ok) {
                u = lu_back(A, r, lane, my_step, L);
                if (a.fp64res == RES_PER_ROW) {
                    float e[1] = {lane < a.nf ? kappa_probe(lane) : 0.f};
                    fwd_all_u<1>(std::make_integer_sequence<int, NF>{}, A, e, my_step);
                    const float z = lu_back(A, e, lane, my_step, L);
                    const float kest =
                        anorm * __int_as_float(wave_max_key(__float_as_int(fabsf(z)))) * (1.f / 3.f);
                    need64 = ((double)a.lam < FP64_LAMBDA && kest > KAPPA_FP64) ? 1 : 0;
                    regram = a.pass == 0 && kest > KAPPA_BF16;
                } else if (a.fp64res == RES_FP64) {
                    need64 = 1;
                }
                if (!regram)
#pragma unroll
                    for (int b = 0; b < NF; ++b) fac[b * 64 + lane] = A[b];
            }
            fac[NF * 64 + lane] = __int_as_float(ok && !regram ? (my_step | (need64 << 16)) : -1);
            if (lane == 0 && a.pass == 0) {
                a.flag[slot] = regram ? 2 : 0;
                if (regram) atomicAdd(&a.stats[ST_FP32GRAM], 1ull);
            }
        } else {
            // elimination without row exchanges first (bounds as for light
            // rows); when rejected, the system is summed again for the
            // pivoted LU, which decides singularity
            ok = solve_unpivoted<WaveLds, true>(A, rhs, lane, a.nf, system_tol(A, a.nf), u, L);
            if (!ok) {
                if (lane == 0) atomicAdd(&a.stats[ST_PIVOTED], 1ull);
                build();
                ok = solve<true, WaveLds, true>(A, rhs, lane, a.nf, system_tol(A, a.nf), u, L);
            }
        }
        if (!ok) {
            u = 0.f;
            if (a.unif && lane == 0) atomicAdd(&a.stats[ST_FALLBACK], 1ull);  // singular sample system
            if (core) {
                // singular core system: full-data update of eq. (U)
                if (lane == 0) atomicAdd(&a.stats[ST_FALLBACK], 1ull);
                RowCtx r{a.idx, a.val, a.other, beg, n, a.nf, vec4, -1};
                Cut full{0, 0, false, true};
                if (a.implicit) {
                    gram_range_sparse<WaveLds, true>(L, r, full, 0, n, lane, A, rhs, a.alpha);
                    finish_system_implicit(A, rhs, a.G, a.lam, lane, a.nf);
                } else {
                    gram(L, r, full, lane, A, rhs);
                    finish_system(A, rhs, lamn, lane, a.nf);
                }
                ok = solve<true, WaveLds, true>(A, rhs, lane, a.nf, system_tol(A, a.nf), u, L);
                if (!ok) u = 0.f;
            }
        }
        if (lane < a.nf) a.out[i * a.nf + lane] = u;
    }
}

// Refinement step of a heavy row, with the LU factors its first solve kept:
// u + A^-1 (rho - lambda n u), rho = sum of the chunk residuals.
__global__ __launch_bounds__(WPB * 64) void k_heavy_refine(HeavyArgs a, int64_t slot_begin, int64_t slot_end,
                                                           int64_t pair_base) {
    __shared__ WaveLds lds[WPB];
    const int w = wave_index();
    const int lane0 = threadIdx.x & 63;
    WaveLds &L = lds[w];
    for (int64_t slot = slot_begin + (int64_t)blockIdx.x * WPB + w; slot < slot_end;
         slot += (int64_t)gridDim.x * WPB) {
        const int lane = opaque_lane(lane0);
        const int64_t i = a.rows[slot];
        if (a.path && a.path[i] == 0) continue;  // fold-in answer accepted
        const int n = (int)(a.ptr[i + 1] - a.ptr[i]);
        const float *fac = a.partials + (a.pair_off[slot] - pair_base) * (int64_t)(NF + 1) * 64;
        const int kept_step = __float_as_int(fac[NF * 64 + lane]);
        if (kept_step < 0) continue;  // the first solve used the full-data fallback
        const int my_step = kept_step & 0xFFFF;
        const bool need64 = (kept_step >> 16) & 1;
        float A[NF];
#pragma unroll
        for (int b = 0; b < NF; ++b) A[b] = fac[b * 64 + lane];
        const float u0 = lane < a.nf ? a.out[i * a.nf + lane] : 0.f;
        double rho = 0.0, bsum = 0.0;
        for (int64_t p = a.pair_off[slot]; p < a.pair_off[slot + 1]; ++p) {
            rho += a.resid[(p - pair_base) * 128 + lane];
            bsum += a.resid[(p - pair_base) * 128 + 64 + lane];
        }
        rho -= (double)a.lam * (double)n * (double)u0;
        if (lane >= a.nf) rho = 0.0;
        // relative residual |b - A u0| / |b| of the first solution
        const double rel = rel_residual(rho, bsum, lane, a.nf);
        if (lane == 0 && rel <= 1e300)
            atomicMax(&a.stats[ST_MAXRES], (unsigned long long)__double_as_longlong(rel));
        float r[1] = {(float)rho};
        fwd_all_u<1>(std::make_integer_sequence<int, NF>{}, A, r, my_step);
        const float d = lu_back(A, r, lane, my_step, L);
        if (need64 && lane == 0) atomicAdd(&a.stats[ST_FP64RES], 1ull);
        if (lane < a.nf) a.out[i * a.nf + lane] = u0 + d;
    }
}

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr uint32_t GF_NONE = 0x80000000u;  // a buffer offset past any factor matrix

// Partial system of a (row, chunk) pair, A = X*^T X and b = X*^T y over the
// chunk's entries, on bf16 MFMA tiles with FP32 accuracy.  Each operand value
// splits exactly as x = h + m + l: h is x rounded to nearest bfloat16, m is
// x - h (exact in FP32) rounded to nearest, l = x - h - m, itself a bfloat16
// number (the 24 significant bits of x leave at most 8 for it); |m| <=
// 2^-8 |x|, |l| <= 2^-16 |x|.  The product x x' is h h' + h m' + m h' + m m' +
// h l' + l h' up to terms below 2^-23 |x x'| of either sign, and bf16 products
// are exact in FP32, so six 32x32x16 bf16 MFMAs per tile and 16 entries
// (together 3/8 of the matrix-core time of the eight 32x32x2 FP32 MFMAs they
// replace) give FP32 products with FP32 accumulation; no refinement step is
// needed.  (Truncated parts would drop terms up to 2^-20 |x x'|, all of one
// sign on the diagonal: a bias that long rows accumulate.)
// A = X*^T (masked by the row's cut), B = X.  Lane (i, h) holds entries
// 8h .. 8h + 7 of a 16-entry step for column i of its tile, which is its slot
// in both the A operand (32 x 16) and the B operand (16 x 32); it loads them
// straight from memory (columns i and 32 + i of each entry's factor row: two
// 128-byte segments per load instruction).  Column indices and ratings of a
// 64-entry block are parked in LDS so that each lane reads its own with one LDS
// load; the cut test is one 64-bit compare of (key, -position).  Entries past
// the chunk and padded columns (a >= n_f) read zeros: with BUF their buffer
// offsets lie beyond the factor matrix, where buffer loads return 0.
// BUF: buffer loads with 32-bit offsets (factor matrices below 2^24 rows and
// 2^31 bytes); else 64-bit addresses, clamped rows and explicit zeros.
constexpr int GX_STEPS = 1;  // 16-entry MFMA steps per gather batch

typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

// Two values rounded to nearest bfloat16 (one v_cvt_pk_bf16_f32), packed with
// the first in the low half.
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

// GPOS (fast variant): one cut per column for every row (cstride 0), its tie
// rule applied to the entry's row index in `other` instead of its position.
// UNIF: entries outside the row's uniform draw are zeroed (both operands and
// the right-hand side), every remaining entry kept.
// IMPL (implicit feedback): the kept operand is weighted by alpha y_k and the
// right-hand side sums x_ka (1 + alpha y_k).
// ONE (BF16 precision modes): the products of the operands' bf16 roundings
// only, one MFMA per tile; a refinement step follows.
template <bool BUF, bool GPOS, bool UNIF, bool IMPL = false, bool ONE = false>
__global__ __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_heavy_gram_x6(
    HeavyArgs a, int64_t pair_begin, int64_t pair_end) {
    __shared__ int s_col[WPB][64];
    __shared__ float s_y[WPB][64];
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    const int m = lane & 31, h = lane >> 5;
    const int nf = a.nf;
    const uint32_t off0 = m < nf ? 4 * m : GF_NONE, off1 = 32 + m < nf ? 4 * (32 + m) : GF_NONE;
    const int stride = 4 * nf;
    // padding column: past the matrix (BUF) or -1
    const int rows = BUF ? (int)a.other_rows : -1;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float *>(a.other), (short)0, BUF ? (int)(a.other_rows * nf * 4) : 0, 0x00020000);
    const float *col0p = a.other + min(m, nf - 1), *col1p = a.other + min(32 + m, nf - 1);
    const bool live0 = m < nf, live1 = 32 + m < nf;
    for (int64_t p = pair_begin + (int64_t)blockIdx.x * WPB + w; p < pair_end; p += (int64_t)gridDim.x * WPB) {
        const int64_t slot = a.pair_slot[p];
        const int chunk = a.pair_chunk[p];
        const int64_t i = a.rows[slot];
        if (a.path && a.path[i] == 0) continue;  // fold-in answer accepted
        if (a.pass && a.flag[slot] != a.pass) continue;
        const int64_t beg = a.ptr[i];
        const int n = (int)(a.ptr[i + 1] - beg);
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        // kept(k) <=> (key, ~k) >= (T, ~K) as unsigned 64-bit pairs; every
        // entry is kept with (T, K) = (0, INT_MAX), none with s = 0
        int T0 = 0, K0 = 0x7FFFFFFF, T1 = 0, K1 = 0x7FFFFFFF;
        const uint32_t uT = UNIF ? a.uT[i] : 0u;
        const int uK = UNIF ? a.uK[i] : 0;
        if (!UNIF && (GPOS || s < n)) {
            const int64_t cb = slot * (int64_t)a.cstride;
            T0 = a.cutT[cb + m];
            K0 = a.cutK[cb + m];
            T1 = a.cutT[cb + 32 + m];
            K1 = a.cutK[cb + 32 + m];
        }
        if (!UNIF && !GPOS && s == 0) {
            T0 = T1 = 0x7FFFFFFF;
            K0 = K1 = -1;
        }
        const uint64_t b0 = ((uint64_t)(uint32_t)T0 << 32) | (uint32_t)~K0;
        const uint64_t b1 = ((uint64_t)(uint32_t)T1 << 32) | (uint32_t)~K1;
        f32x16 acc[2][2];
#pragma unroll
        for (int ta = 0; ta < 2; ++ta)
#pragma unroll
            for (int tb = 0; tb < 2; ++tb)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[ta][tb][q] = 0.f;
        float racc0 = 0.f, racc1 = 0.f;
        const int kb = chunk * a.chunk;
        const int ke = min(n, kb + a.chunk);
        int colv = kb + lane < ke ? a.idx[beg + kb + lane] : rows;
        float yv = kb + lane < ke ? a.val[beg + kb + lane] : 0.f;
        for (int k0 = kb; k0 < ke; k0 += 64) {
            wave_sync();  // the previous block's LDS reads are done
            s_col[w][lane] = colv;
            s_y[w][lane] = yv;
            wave_sync();
            const int k1 = k0 + 64;
            colv = rows;
            yv = 0.f;
            if (k1 < ke) {
                colv = k1 + lane < ke ? a.idx[beg + k1 + lane] : rows;
                yv = k1 + lane < ke ? a.val[beg + k1 + lane] : 0.f;
            }
#pragma unroll 1
            for (int e0 = k0; e0 < min(ke, k1); e0 += 16 * GX_STEPS) {
                const int j0 = e0 - k0;
                float x0[GX_STEPS][8], x1[GX_STEPS][8];
                int cols[GX_STEPS][8];
#pragma unroll
                for (int st = 0; st < GX_STEPS; ++st)
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int col = s_col[w][j0 + 16 * st + 8 * h + e];
                        cols[st][e] = col;
                        if constexpr (BUF) {
                            const uint32_t off = __umul24((unsigned)col, (unsigned)stride);
                            x0[st][e] =
                                __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)(off + off0), 0, 0));
                            x1[st][e] =
                                __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)(off + off1), 0, 0));
                        } else {
                            const size_t ro = (size_t)max(col, 0) * nf;
                            const float u0 = col0p[ro], u1 = col1p[ro];
                            x0[st][e] = (col >= 0 && live0) ? u0 : 0.f;
                            x1[st][e] = (col >= 0 && live1) ? u1 : 0.f;
                        }
                    }
                // every gather of the batch is issued before the first use
                __builtin_amdgcn_sched_barrier(0);
                if constexpr (UNIF) {
#pragma unroll
                    for (int st = 0; st < GX_STEPS; ++st)
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const int pos = e0 + 16 * st + 8 * h + e;
                            const uint32_t key = unif_key(a.seed, i, a.n_cols, cols[st][e]);
                            const bool kp = key < uT || (key == uT && pos <= uK);
                            x0[st][e] = kp ? x0[st][e] : 0.f;
                            x1[st][e] = kp ? x1[st][e] : 0.f;
                        }
                }
#pragma unroll
                for (int st = 0; st < GX_STEPS; ++st) {
                    const uint32_t nkb = ~(uint32_t)(e0 + 16 * st + 8 * h);  // ~k of the lane's first entry
                    uint32_t ph[2][4], pm[2][4], pl[2][4], mk[2][4];
                    uint32_t wh[2][4], wm[2][4], wl[2][4];  // IMPL: parts of the weighted operand
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const uint64_t bt = t ? b1 : b0;
#pragma unroll
                        for (int e2 = 0; e2 < 4; ++e2) {
                            float xv[2], xw[2];
                            uint32_t km[2];
#pragma unroll
                            for (int o = 0; o < 2; ++o) {
                                const int e = 2 * e2 + o;
                                const float x = t ? x1[st][e] : x0[st][e];
                                xv[o] = x;
                                const uint32_t u = __float_as_uint(x);
                                const uint32_t tie = GPOS ? ~(uint32_t)cols[st][e] : nkb - (uint32_t)e;
                                const uint64_t key = ((uint64_t)(u & 0x7FFFFFFFu) << 32) | tie;
                                const bool kp = key >= bt;
                                km[o] = kp ? 0xFFFFu : 0u;
                                const float y = s_y[w][j0 + 16 * st + 8 * h + e];
                                if constexpr (IMPL) {
                                    // X*^T W X: the kept operand carries the weight
                                    const float yc = fmaf(a.alpha, y, 1.f);
                                    if (t) racc1 = fmaf(kp ? x : 0.f, yc, racc1);
                                    else racc0 = fmaf(kp ? x : 0.f, yc, racc0);
                                    xw[o] = x * (a.alpha * y);
                                } else {
                                    if (t) racc1 = fmaf(kp ? x : 0.f, y, racc1);
                                    else racc0 = fmaf(kp ? x : 0.f, y, racc0);
                                }
                            }
                            // x = h + m + l, each part rounded to nearest from
                            // the exact remainder of the previous ones
                            const uint32_t qh = pack_bf16(xv[0], xv[1]);
                            const float r0 = xv[0] - __uint_as_float(qh << 16);
                            const float r1 = xv[1] - __uint_as_float(qh & 0xFFFF0000u);
                            const uint32_t qm = pack_bf16(r0, r1);
                            const float s0 = r0 - __uint_as_float(qm << 16);
                            const float s1 = r1 - __uint_as_float(qm & 0xFFFF0000u);
                            ph[t][e2] = qh;
                            pm[t][e2] = qm;
                            pl[t][e2] = pack_bf16(s0, s1);
                            mk[t][e2] = km[0] | (km[1] << 16);
                            if constexpr (IMPL) {
                                const uint32_t gh = pack_bf16(xw[0], xw[1]);
                                const float g0 = xw[0] - __uint_as_float(gh << 16);
                                const float g1 = xw[1] - __uint_as_float(gh & 0xFFFF0000u);
                                const uint32_t gm = pack_bf16(g0, g1);
                                wh[t][e2] = gh;
                                wm[t][e2] = gm;
                                wl[t][e2] = pack_bf16(g0 - __uint_as_float(gm << 16), g1 - __uint_as_float(gm & 0xFFFF0000u));
                            }
                        }
                    }
                    // B operands (all entries) and A operands (kept entries only)
                    bf16x8 bh[2], bm[2], bl[2], ah[2], am[2], al[2];
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        uint32_t qh[4], qm[4], ql[4];
#pragma unroll
                        for (int e2 = 0; e2 < 4; ++e2) {
                            qh[e2] = (IMPL ? wh[t][e2] : ph[t][e2]) & mk[t][e2];
                            qm[e2] = (IMPL ? wm[t][e2] : pm[t][e2]) & mk[t][e2];
                            ql[e2] = (IMPL ? wl[t][e2] : pl[t][e2]) & mk[t][e2];
                        }
                        bh[t] = __builtin_bit_cast(bf16x8, ph[t]);
                        bm[t] = __builtin_bit_cast(bf16x8, pm[t]);
                        bl[t] = __builtin_bit_cast(bf16x8, pl[t]);
                        ah[t] = __builtin_bit_cast(bf16x8, qh);
                        am[t] = __builtin_bit_cast(bf16x8, qm);
                        al[t] = __builtin_bit_cast(bf16x8, ql);
                    }
                    // six products per tile, the four tiles interleaved so that
                    // consecutive MFMAs are independent
#define GX_MFMA(A, B)                                                                             \
    _Pragma("unroll") for (int ta = 0; ta < 2; ++ta) _Pragma("unroll") for (int tb = 0; tb < 2; ++tb) \
        acc[ta][tb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[ta], B[tb], acc[ta][tb], 0, 0, 0);
                    if constexpr (ONE) {
                        GX_MFMA(ah, bh)
                    } else {
                        GX_MFMA(al, bh)
                        GX_MFMA(ah, bl)
                        GX_MFMA(am, bm)
                        GX_MFMA(am, bh)
                        GX_MFMA(ah, bm)
                        GX_MFMA(ah, bh)
                    }
#undef GX_MFMA
                }
            }
        }
        racc0 += __shfl_xor(racc0, 32);
        racc1 += __shfl_xor(racc1, 32);
        float *dst = a.partials + (p - pair_begin) * (int64_t)(NF + 1) * 64;
#pragma unroll
        for (int ta = 0; ta < 2; ++ta)
#pragma unroll
            for (int tb = 0; tb < 2; ++tb)
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int row = 8 * (q >> 2) + 4 * h + (q & 3);
                    dst[(32 * tb + m) * 64 + 32 * ta + row] = acc[ta][tb][q];
                }
        if (h == 0) {
            dst[NF * 64 + m] = racc0;
            dst[NF * 64 + 32 + m] = racc1;
        }
    }
}

// Partial refinement residual of one (row, chunk) pair: rho_a = sum over kept
// k of x_ka (y_k - x_k . u), with u the row's current solution (in `out`).
// Lane k forms y_k - x_k . u for the staged rows, lane a then accumulates its
// column.  FP64 accumulates in double throughout.
// The accumulation type is chosen per row: FP64 when the row's first solve
// asked for it (bit 16 of its kept pivot step), FP32 otherwise.
template <typename acc_t>
__device__ __forceinline__ void heavy_resid_pair(const HeavyArgs &a, WaveLds &L, RowCtx &r, const Cut &c, int chunk,
                                                 int n, int64_t p, int64_t pair_begin, int lane) {
    acc_t acc = 0;
    double bs = 0.0;  // the chunk's share of b = X*^T y
    const int kb = chunk * a.chunk;
    const int ke = min(n, kb + a.chunk);
    // 64-row blocks: with float4 rows, the next block's gathers are in flight
    // while this one is reduced, and the indices of the one after
    const bool pipe = r.vec4;
    int colA = 0;
    float yA = 0.f;
    float4 v[CK / 4];
    auto load_idx = [&](int k0, int &col, float &yv) {
        col = 0;
        yv = 0.f;
        if (k0 + lane < ke) {
            col = r.idx[r.beg + k0 + lane];
            yv = r.val[r.beg + k0 + lane];
        }
    };
    // gathers of the block whose indices lane j holds (row j of the block)
    auto gather = [&](int col) {
#pragma unroll
        for (int t = 0; t < CK / 4; ++t) {
            const int c = __shfl(col, t * 4 + (lane >> 4));
            v[t] = *reinterpret_cast<const float4 *>(r.other + (size_t)c * NF + (lane & 15) * 4);
        }
    };
    float ycur = 0.f;
    if (pipe) {
        int c0;
        load_idx(kb, c0, ycur);
        gather(c0);
        load_idx(kb + CK, colA, yA);
    }
    for (int k0 = kb; k0 < ke; k0 += CK) {
        const int mrows = min(CK, ke - k0);
        if (pipe) {
            wave_sync();
            L.y[lane] = ycur;
#pragma unroll
            for (int t = 0; t < CK / 4; ++t) {
                const int kk = t * 4 + (lane >> 4);
                *reinterpret_cast<float4 *>(&L.X[kk][(lane & 15) * 4]) =
                    kk < mrows ? v[t] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
            wave_sync();
            ycur = yA;
            if (k0 + CK < ke) {
                gather(colA);
                load_idx(k0 + 2 * CK, colA, yA);
            }
        } else {
            stage(L, r, k0, lane);
        }
        acc_t rk = 0;
        if (lane < mrows) {
            acc_t dot = 0;
#pragma unroll
            for (int b4 = 0; b4 < NF / 4; ++b4) {
                const float4 xr = *reinterpret_cast<const float4 *>(&L.X[lane][4 * b4]);
                dot += (acc_t)xr.x * (acc_t)L.urhs[4 * b4 + 0];
                dot += (acc_t)xr.y * (acc_t)L.urhs[4 * b4 + 1];
                dot += (acc_t)xr.z * (acc_t)L.urhs[4 * b4 + 2];
                dot += (acc_t)xr.w * (acc_t)L.urhs[4 * b4 + 3];
            }
            rk = (acc_t)L.y[lane] - dot;
        }
        L.rres[lane] = (double)rk;
        wave_sync();
        // all CK rows, unrolled and without branches (unkept and past-the-end
        // rows add zero), so that the LDS reads of a batch are in flight together
#pragma unroll 16
        for (int kk = 0; kk < CK; ++kk) {
            const float x = L.X[kk][lane];
            const float xm = (kk < mrows && kept(c, key_of(x), k0 + kk)) ? x : 0.f;
            acc += (acc_t)xm * (acc_t)L.rres[kk];
            bs += (double)xm * (double)L.y[kk];
        }
        wave_sync();
    }
    a.resid[(p - pair_begin) * 128 + lane] = (double)acc;
    a.resid[(p - pair_begin) * 128 + 64 + lane] = bs;
}

__global__ __launch_bounds__(WPB * 64) void k_heavy_resid(HeavyArgs a, int64_t pair_begin, int64_t pair_end) {
    __shared__ WaveLds lds[WPB];
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    WaveLds &L = lds[w];
    const bool vec4 = (a.nf == NF) && ((reinterpret_cast<uintptr_t>(a.other) & 15) == 0);
    for (int64_t p = pair_begin + (int64_t)blockIdx.x * WPB + w; p < pair_end; p += (int64_t)gridDim.x * WPB) {
        const int64_t slot = a.pair_slot[p];
        const int chunk = a.pair_chunk[p];
        const int64_t i = a.rows[slot];
        if (a.path && a.path[i] == 0) continue;  // fold-in answer accepted
        // the row's kept pivot step (first pair's slot): -1 = no refinement
        const float *fac = a.partials + (a.pair_off[slot] - pair_begin) * (int64_t)(NF + 1) * 64;
        const int kept_step = __builtin_amdgcn_readfirstlane(__float_as_int(fac[NF * 64]));
        if (kept_step < 0) continue;
        const int64_t beg = a.ptr[i];
        const int n = (int)(a.ptr[i + 1] - beg);
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        RowCtx r{a.idx, a.val, a.other, beg, n, a.nf, vec4, -1};
        Cut c;
        if (s == n) c = Cut{0, 0, false, true};
        else if (s == 0) c = Cut{0, 0, true, false};
        else c = Cut{a.cutT[slot * 64 + lane], a.cutK[slot * 64 + lane], false, false};
        wave_sync();
        L.urhs[lane] = lane < a.nf ? a.out[i * a.nf + lane] : 0.f;
        if ((kept_step >> 16) & 1) heavy_resid_pair<double>(a, L, r, c, chunk, n, p, pair_begin, lane);
        else heavy_resid_pair<float>(a, L, r, c, chunk, n, p, pair_begin, lane);
    }
}

// Fold-in check, part 1: per (row, chunk) pair, the chunk's share of
// b_a = sum over kept k of x_ka y_k and of X*^T (y - X g) for the candidate g
// (FP64 sums), into resid[pair][0..63] and resid[pair][64..127].
__global__ __launch_bounds__(WPB * 64) void k_heavy_check(HeavyArgs a, int64_t pair_begin, int64_t pair_end) {
    __shared__ WaveLds lds[WPB];
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    WaveLds &L = lds[w];
    const bool vec4 = (a.nf == NF) && ((reinterpret_cast<uintptr_t>(a.other) & 15) == 0);
    for (int64_t p = pair_begin + (int64_t)blockIdx.x * WPB + w; p < pair_end; p += (int64_t)gridDim.x * WPB) {
        const int64_t slot = a.pair_slot[p];
        const int chunk = a.pair_chunk[p];
        const int64_t i = a.rows[slot];
        const int64_t beg = a.ptr[i];
        const int n = (int)(a.ptr[i + 1] - beg);
        const int s = (int)budget_of(n, a.num, a.den, a.min_keep);
        RowCtx r{a.idx, a.val, a.other, beg, n, a.nf, vec4, -1};
        Cut c;
        if (s == n) c = Cut{0, 0, false, true};
        else if (s == 0) c = Cut{0, 0, true, false};
        else c = Cut{a.cutT[slot * 64 + lane], a.cutK[slot * 64 + lane], false, false};
        wave_sync();
        L.urhs[lane] = lane < a.nf ? a.guess[i * a.nf + lane] : 0.f;
        wave_sync();
        const int kb = chunk * a.chunk;
        const int ke = min(n, kb + a.chunk);
        double rho, bsum;
        resid_range(L, r, c, kb, ke, lane, rho, bsum);
        double *dst = a.resid + (p - pair_begin) * 128;
        dst[lane] = rho;
        dst[64 + lane] = bsum;
    }
}

// Fold-in check, part 2: one wavefront per heavy row sums its chunk shares in
// chunk order, subtracts lambda n_i g, and accepts g (path 0, copied to out)
// when |b - A g| / |b| <= tol; otherwise marks the row for the exact solve.
__global__ __launch_bounds__(WPB * 64) void k_heavy_check_reduce(HeavyArgs a, int64_t slot_begin, int64_t slot_end,
                                                                 int64_t pair_base) {
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    for (int64_t slot = slot_begin + (int64_t)blockIdx.x * WPB + w; slot < slot_end;
         slot += (int64_t)gridDim.x * WPB) {
        const int64_t i = a.rows[slot];
        const int n = (int)(a.ptr[i + 1] - a.ptr[i]);
        double rho = 0.0, bsum = 0.0;
        for (int64_t p = a.pair_off[slot]; p < a.pair_off[slot + 1]; ++p) {
            rho += a.resid[(p - pair_base) * 128 + lane];
            bsum += a.resid[(p - pair_base) * 128 + 64 + lane];
        }
        const float g = lane < a.nf ? a.guess[i * a.nf + lane] : 0.f;
        rho -= (double)a.lam * (double)n * (double)g;
        const double rel = rel_residual(rho, bsum, lane, a.nf);
        const bool accept = rel <= (double)a.tol;
        if (lane == 0) {
            a.rho[i] = (float)rel;
            a.path[i] = accept ? 0 : 1;
            if (!accept) atomicAdd(&a.stats[ST_FOLDIN_EXACT], 1ull);
        }
        if (accept && lane < a.nf) a.out[i * a.nf + lane] = g;
    }
}

unsigned blocks_for(int64_t items, int per_block, int64_t cap) {
    int64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_heavy_gram_bf16(const HeavyArgs &a, int64_t pair_begin, int64_t pair_end, hipStream_t s) {
    if (pair_end <= pair_begin) return hipSuccess;
    const bool buf = a.other_rows > 0 && a.other_rows < (1 << 24) &&
                     a.other_rows * (int64_t)a.nf * 4 <= (int64_t)0x7FFFFFFF;
    const dim3 grid(blocks_for(pair_end - pair_begin, WPB, 65536));
    if (buf)
        hipLaunchKernelGGL((k_heavy_gram_x6<true, false, false, false, true>), grid, dim3(WPB * 64), 0, s, a,
                           pair_begin, pair_end);
    else
        hipLaunchKernelGGL((k_heavy_gram_x6<false, false, false, false, true>), grid, dim3(WPB * 64), 0, s, a,
                           pair_begin, pair_end);
    return hipGetLastError();
}

hipError_t launch_heavy_resid(const HeavyArgs &a, int64_t pair_begin, int64_t pair_end, hipStream_t s) {
    if (pair_end <= pair_begin) return hipSuccess;
    hipLaunchKernelGGL(k_heavy_resid, dim3(blocks_for(pair_end - pair_begin, WPB, 65536)), dim3(WPB * 64), 0, s, a,
                       pair_begin, pair_end);
    return hipGetLastError();
}

hipError_t launch_heavy_check(const HeavyArgs &a, int64_t pair_begin, int64_t pair_end, hipStream_t s) {
    if (pair_end <= pair_begin) return hipSuccess;
    if (!a.guess) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_heavy_check, dim3(blocks_for(pair_end - pair_begin, WPB, 65536)), dim3(WPB * 64), 0, s, a,
                       pair_begin, pair_end);
    return hipGetLastError();
}

hipError_t launch_heavy_check_reduce(const HeavyArgs &a, int64_t slot_begin, int64_t slot_end, int64_t pair_base,
                                     hipStream_t s) {
    if (slot_end <= slot_begin) return hipSuccess;
    if (!a.guess || !a.path || !a.rho) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_heavy_check_reduce, dim3(blocks_for(slot_end - slot_begin, WPB, 65536)), dim3(WPB * 64), 0,
                       s, a, slot_begin, slot_end, pair_base);
    return hipGetLastError();
}

// key16[i] = bits 30..15 of other[i] (exponent and top mantissa byte of |x|);
// eight entries per thread, 16-byte accesses when `other` is 16-byte aligned.
template <bool VEC>
__global__ __launch_bounds__(256) void k_key16(const float *other, int64_t count, uint16_t *key16) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x * 8;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8; i < count; i += step) {
        if (VEC && i + 8 <= count) {
            const uint4 x = *reinterpret_cast<const uint4 *>(other + i);
            const uint4 y = *reinterpret_cast<const uint4 *>(other + i + 4);
            uint4 o;
            o.x = ((x.x >> 15) & 0xFFFFu) | (((x.y >> 15) & 0xFFFFu) << 16);
            o.y = ((x.z >> 15) & 0xFFFFu) | (((x.w >> 15) & 0xFFFFu) << 16);
            o.z = ((y.x >> 15) & 0xFFFFu) | (((y.y >> 15) & 0xFFFFu) << 16);
            o.w = ((y.z >> 15) & 0xFFFFu) | (((y.w >> 15) & 0xFFFFu) << 16);
            *reinterpret_cast<uint4 *>(key16 + i) = o;
        } else {
            for (int64_t k = i; k < i + 8 && k < count; ++k)
                key16[k] = (uint16_t)((__float_as_uint(other[k]) >> 15) & 0xFFFFu);
        }
    }
}

hipError_t launch_key16(const float *other, int64_t count, uint16_t *key16, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count + 2047) / 2048, 16384);
    if ((reinterpret_cast<uintptr_t>(other) & 15) == 0 && (reinterpret_cast<uintptr_t>(key16) & 15) == 0)
        hipLaunchKernelGGL(k_key16<true>, dim3(blocks), dim3(256), 0, s, other, count, key16);
    else
        hipLaunchKernelGGL(k_key16<false>, dim3(blocks), dim3(256), 0, s, other, count, key16);
    return hipGetLastError();
}

hipError_t launch_heavy_select(const HeavyArgs &a, int64_t row_begin, hipStream_t s) {
    if (a.count <= 0) return hipSuccess;
    // buffer loads address the factor matrix with 32-bit offsets
    const bool buf = a.other_rows > 0 && a.other_rows * (int64_t)a.nf * 4 <= (int64_t)0x7FFFFFFF;
    const dim3 grid(blocks_for(a.count, 1, 8192));
    if (buf && a.key16)
        hipLaunchKernelGGL((k_heavy_select<true, true>), grid, dim3(HS_THREADS), 0, s, a, row_begin);
    else if (buf)
        hipLaunchKernelGGL((k_heavy_select<true, false>), grid, dim3(HS_THREADS), 0, s, a, row_begin);
    else
        hipLaunchKernelGGL((k_heavy_select<false, false>), grid, dim3(HS_THREADS), 0, s, a, row_begin);
    return hipGetLastError();
}

hipError_t launch_heavy_gram(const HeavyArgs &a, int64_t pair_begin, int64_t pair_end, hipStream_t s) {
    if (pair_end <= pair_begin) return hipSuccess;
    // buffer offsets are 24-bit products row * 4 n_f plus 32-bit sums
    const bool buf = a.other_rows > 0 && a.other_rows < (1 << 24) &&
                     a.other_rows * (int64_t)a.nf * 4 <= (int64_t)0x7FFFFFFF;
    const dim3 grid(blocks_for(pair_end - pair_begin, WPB, 65536));
    if (buf && a.implicit)
        hipLaunchKernelGGL((k_heavy_gram_x6<true, false, false, true>), grid, dim3(WPB * 64), 0, s, a, pair_begin,
                           pair_end);
    else if (a.implicit)
        hipLaunchKernelGGL((k_heavy_gram_x6<false, false, false, true>), grid, dim3(WPB * 64), 0, s, a, pair_begin,
                           pair_end);
    else if (buf && a.unif)
        hipLaunchKernelGGL((k_heavy_gram_x6<true, false, true>), grid, dim3(WPB * 64), 0, s, a, pair_begin, pair_end);
    else if (buf && a.gpos)
        hipLaunchKernelGGL((k_heavy_gram_x6<true, true, false>), grid, dim3(WPB * 64), 0, s, a, pair_begin, pair_end);
    else if (buf)
        hipLaunchKernelGGL((k_heavy_gram_x6<true, false, false>), grid, dim3(WPB * 64), 0, s, a, pair_begin,
                           pair_end);
    else if (a.unif)
        hipLaunchKernelGGL((k_heavy_gram_x6<false, false, true>), grid, dim3(WPB * 64), 0, s, a, pair_begin,
                           pair_end);
    else if (a.gpos)
        hipLaunchKernelGGL((k_heavy_gram_x6<false, true, false>), grid, dim3(WPB * 64), 0, s, a, pair_begin,
                           pair_end);
    else
        hipLaunchKernelGGL((k_heavy_gram_x6<false, false, false>), grid, dim3(WPB * 64), 0, s, a, pair_begin,
                           pair_end);
    return hipGetLastError();
}

hipError_t launch_heavy_solve(const HeavyArgs &a, int64_t slot_begin, int64_t slot_end, int64_t pair_base,
                              hipStream_t s) {
    if (slot_end <= slot_begin) return hipSuccess;
    if (a.refine)
        hipLaunchKernelGGL(k_heavy_refine, dim3(blocks_for(slot_end - slot_begin, WPB, 65536)), dim3(WPB * 64), 0, s,
                           a, slot_begin, slot_end, pair_base);
    else
        hipLaunchKernelGGL(k_heavy_solve, dim3(blocks_for(slot_end - slot_begin, WPB, 65536)), dim3(WPB * 64), 0, s,
                           a, slot_begin, slot_end, pair_base);
    return hipGetLastError();
}

}  // namespace coreals
