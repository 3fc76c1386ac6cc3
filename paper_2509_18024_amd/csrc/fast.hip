// Global sketch of the fast variant of Core-ALS (gfx950).
//
// The fast variant (Section 3, the paragraph after Algorithm 2) applies CES
// once per half-sweep to the whole factor matrix of the other side instead of
// to every row's slice.  For each column a of `other` (n_other x n_f, n_f <=
// 64) this computes the cut (T_a, K_a) of its s = budget(n_other) entries of
// largest |x|: an entry (j, a) is kept iff key > T_a, or key == T_a and
// j <= K_a, with key the bit pattern of |x| (ties keep the smaller row j).
// The half-sweep kernels then test every entry against its column's cut.
//
// The cut is an exact radix select over all n_other rows, all columns at once:
// four passes over the 31-bit key (8, 8, 8, 7 bits, most significant first)
// and, only for columns where more keys equal the threshold than are needed,
// passes over the bits of the row index (smallest first).  Each pass is a
// histogram kernel (a block counts its rows' digits in LDS, lane a = column a,
// and adds its counts to a global histogram) and a one-block pick kernel that
// fixes each open column's digit.  A column is finished as soon as every key
// sharing its prefix is kept; the histogram kernels return at once when every
// column is finished.
#include "rowops.hpp"

namespace coreals {

namespace {

constexpr int GS_THREADS = 256;  // four waves: lane = column, waves over rows
constexpr int GS_BLOCKS = 1024;

struct GlobalSel {
    uint32_t hist[64 * 256];  // [column][digit] counts of the current pass
    int32_t prefix[64];       // key bits fixed so far (key passes)
    int32_t iprefix[64];      // row-index bits fixed so far (index passes)
    int32_t rem[64];          // entries still to keep among those on the prefix
    int32_t done[64];
    int32_t all_done;
};

// Counts of the digit [shift, shift + width) of every entry whose fixed bits
// match its column's prefix.  INDEX: the entry's key must equal the column's
// full key T (prefix) and the digit is taken from the row index j, whose bits
// above shift + width must match iprefix.
template <bool INDEX>
__global__ __launch_bounds__(GS_THREADS) void k_gsel_hist(const float *other, int64_t n_other, int nf,
                                                          GlobalSel *st, int shift, int width) {
    __shared__ uint32_t h[256][64];
    if (st->all_done) return;  // uniform
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    for (int q = tid; q < 256 * 64; q += GS_THREADS) (&h[0][0])[q] = 0u;
    const bool live = lane < nf && !st->done[lane];
    const int pre = st->prefix[lane];
    const int ipre = st->iprefix[lane];
    // key passes: bits above shift + width must match the prefix
    const int hmask = INDEX ? 0 : (int)(0x7FFFFFFFu & ~((1u << (shift + width)) - 1u));
    __syncthreads();
    const int64_t per = (n_other + gridDim.x - 1) / gridDim.x;
    const int64_t j0 = (int64_t)blockIdx.x * per;
    const int64_t j1 = min(n_other, j0 + per);
    if (live) {
        const float *col = other + lane;
        // eight rows per wave in flight: all loads of a batch before its counts
        constexpr int B = 8, STEP = GS_THREADS / 64;
        for (int64_t jb = j0 + w; jb < j1; jb += B * STEP) {
            int key[B];
#pragma unroll
            for (int t = 0; t < B; ++t) {
                const int64_t j = jb + t * STEP;
                key[t] = j < j1 ? (__float_as_int(col[j * nf]) & KEYMASK) : -1;
            }
#pragma unroll
            for (int t = 0; t < B; ++t) {
                const int64_t j = jb + t * STEP;
                if (key[t] < 0) continue;
                if constexpr (INDEX) {
                    const int64_t hi = j >> (shift + width);
                    if (key[t] == pre && hi == (int64_t)(ipre >> (shift + width)))
                        atomicAdd(&h[(j >> shift) & ((1 << width) - 1)][lane], 1u);
                } else {
                    if ((key[t] & hmask) == pre) atomicAdd(&h[(key[t] >> shift) & ((1 << width) - 1)][lane], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int q = tid; q < 256 * 64; q += GS_THREADS) {
        const int d = q >> 6, a = q & 63;
        const uint32_t v = h[d][a];
        if (v) atomicAdd(&st->hist[a * 256 + d], v);
    }
}

// Fix the digit of every open column.  Key passes walk digits from the top
// (largest keys first); index passes walk them from 0 (smallest rows first).
// A column finishes when every entry on its new prefix is kept: then
// (T, K) = (prefix - 1, -1) during the key passes (keep keys >= prefix), or
// (T, iprefix + 2^shift - 1) during the index passes.  The histogram is
// cleared for the next pass.
template <bool INDEX>
__global__ __launch_bounds__(64) void k_gsel_pick(GlobalSel *st, int nf, int shift, int width, int32_t *T,
                                                  int32_t *K) {
    __shared__ int open;
    const int a = threadIdx.x;
    if (a == 0) open = 0;
    __syncthreads();
    if (a < nf && !st->done[a] && !st->all_done) {
        const int nd = 1 << width;
        const int rem = st->rem[a];
        int cum = 0;
        for (int t = 0; t < nd; ++t) {
            const int d = INDEX ? t : nd - 1 - t;
            const int hc = (int)st->hist[a * 256 + d];
            if (cum + hc >= rem) {
                const int r2 = rem - cum;
                st->rem[a] = r2;
                if constexpr (INDEX) {
                    st->iprefix[a] |= d << shift;
                    if (hc == r2) {  // every row on this index prefix is kept
                        st->done[a] = 1;
                        T[a] = st->prefix[a];
                        K[a] = st->iprefix[a] | ((1 << shift) - 1);
                    }
                } else {
                    st->prefix[a] |= d << shift;
                    if (hc == r2) {  // every key on this prefix is kept
                        st->done[a] = 1;
                        T[a] = st->prefix[a] - 1;
                        K[a] = -1;
                    }
                }
                break;
            }
            cum += hc;
        }
    }
    if (a < 64)
        for (int d = 0; d < 256; ++d) st->hist[a * 256 + d] = 0u;
    if (a < nf && !st->done[a]) atomicAdd(&open, 1);
    __syncthreads();
    if (a == 0 && open == 0) st->all_done = 1;
}

// Start: s = budget(n_other) per column; s = 0 keeps nothing, s = n_other
// everything (no pass needed).
__global__ __launch_bounds__(64) void k_gsel_init(GlobalSel *st, int nf, int64_t n_other, int64_t s, int32_t *T,
                                                  int32_t *K) {
    __shared__ int open;
    const int a = threadIdx.x;
    if (a == 0) open = 0;
    __syncthreads();
    for (int d = 0; d < 256; ++d) st->hist[a * 256 + d] = 0u;
    st->prefix[a] = 0;
    st->iprefix[a] = 0;
    st->rem[a] = (int)s;
    bool done = a >= nf;
    if (done) {
        T[a] = -1;  // padded columns: every (zero) entry counts as kept
        K[a] = -1;
    } else if (s <= 0) {
        T[a] = 0x7FFFFFFF;  // no key exceeds it; K = -1: nothing kept
        K[a] = -1;
        done = true;
    } else if (s >= n_other) {
        T[a] = -1;  // every key exceeds it
        K[a] = -1;
        done = true;
    }
    st->done[a] = done ? 1 : 0;
    if (!done) atomicAdd(&open, 1);
    __syncthreads();
    if (a == 0) st->all_done = open == 0 ? 1 : 0;
}

}  // namespace

size_t global_select_state_bytes() { return sizeof(GlobalSel); }

hipError_t launch_global_select(const float *other, int64_t n_other, int nf, uint32_t num, uint32_t den,
                                int32_t min_keep, void *state, int32_t *T, int32_t *K, hipStream_t s) {
    if (nf < 1 || nf > 64 || n_other >= (int64_t)1 << 31) return hipErrorInvalidValue;
    GlobalSel *st = static_cast<GlobalSel *>(state);
    const int64_t sg = budget_of(n_other, num, den, min_keep);
    hipLaunchKernelGGL(k_gsel_init, dim3(1), dim3(64), 0, s, st, nf, n_other, sg, T, K);
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(GS_BLOCKS, (n_other + 255) / 256));
    const int shifts[4] = {23, 15, 7, 0}, widths[4] = {8, 8, 8, 7};
    for (int p = 0; p < 4; ++p) {
        hipLaunchKernelGGL(k_gsel_hist<false>, dim3(blocks), dim3(GS_THREADS), 0, s, other, n_other, nf, st,
                           shifts[p], widths[p]);
        hipLaunchKernelGGL(k_gsel_pick<false>, dim3(1), dim3(64), 0, s, st, nf, shifts[p], widths[p], T, K);
    }
    // ties at the full key: the smallest row indices, 8 bits at a time
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < n_other) ++bits;
    for (int top = bits; top > 0; top -= 8) {
        const int width = std::min(8, top), shift = top - width;
        hipLaunchKernelGGL(k_gsel_hist<true>, dim3(blocks), dim3(GS_THREADS), 0, s, other, n_other, nf, st, shift,
                           width);
        hipLaunchKernelGGL(k_gsel_pick<true>, dim3(1), dim3(64), 0, s, st, nf, shift, width, T, K);
    }
    return hipGetLastError();
}

}  // namespace coreals
