// Problem setup on the device: validation of R, the column view (CSC) built by
// a stable LSD radix sort of the entries by column, and the degree-class
// schedule of each half-sweep.  All one-off work of als_init.
#include "internal.hpp"

namespace coreals {

namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 8;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// --------------------------------------------------------------------------
// validation: one thread per row
// --------------------------------------------------------------------------
__global__ void k_validate(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *ptr,
                           const int32_t *idx, const float *val, int check_values, int *flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        if (ptr[0] != 0 || ptr[n_rows] != nnz) atomicOr(flags, 1);
    }
    for (; i < n_rows; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t b = ptr[i], e = ptr[i + 1];
        if (e < b || b < 0 || e > nnz) {
            atomicOr(flags, 1);
            continue;
        }
        int bad = 0;
        int prev = -1;
        for (int64_t t = b; t < e; ++t) {
            int c = idx[t];
            if (c < 0 || c >= n_cols || c <= prev) bad |= 2;
            prev = c;
            if (check_values) {
                float v = val[t];
                if (!(fabsf(v) <= 3.402823466e38f)) bad |= 4;
            }
        }
        if (bad) atomicOr(flags, bad);
    }
}

// --------------------------------------------------------------------------
// exclusive scan of int64 (three kernels)
// --------------------------------------------------------------------------
__device__ int64_t block_exclusive_scan(int64_t v, int64_t *sh, int64_t &total) {
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SC_THREADS; off <<= 1) {
        int64_t add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int64_t incl = sh[t];
    total = sh[SC_THREADS - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_tile(const int64_t *in, int64_t *out, int64_t n, int64_t *tile_sums) {
    __shared__ int64_t sh[SC_THREADS];
    int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
    int64_t loc[SC_ITEMS];
    int64_t sum = 0;
#pragma unroll
    for (int j = 0; j < SC_ITEMS; ++j) {
        int64_t e = base + j;
        loc[j] = e < n ? in[e] : 0;
        sum += loc[j];
    }
    int64_t total;
    int64_t run = block_exclusive_scan(sum, sh, total);
#pragma unroll
    for (int j = 0; j < SC_ITEMS; ++j) {
        int64_t e = base + j;
        if (e < n) out[e] = run;
        run += loc[j];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_sums(int64_t *sums, int64_t nt) {
    __shared__ int64_t sh[SC_THREADS];
    int64_t carry = 0;
    for (int64_t base = 0; base < nt; base += SC_THREADS) {
        int64_t e = base + threadIdx.x;
        int64_t v = e < nt ? sums[e] : 0;
        int64_t total;
        int64_t ex = block_exclusive_scan(v, sh, total);
        if (e < nt) sums[e] = ex + carry;
        carry += total;
        __syncthreads();
    }
}

__global__ void k_scan_add(int64_t *out, int64_t n, const int64_t *tile_sums) {
    int64_t e = (int64_t)blockIdx.x * SC_TILE + threadIdx.x;
    int64_t add = tile_sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < SC_ITEMS; ++j, e += SC_THREADS)
        if (e < n) out[e] += add;
}

size_t scan_temp_bytes(int64_t n) { return align256(sizeof(int64_t) * (size_t)((n + SC_TILE - 1) / SC_TILE + 1)); }

hipError_t exclusive_scan(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nt = (n + SC_TILE - 1) / SC_TILE;
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nt), dim3(SC_THREADS), 0, s, in, out, n, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SC_THREADS), 0, s, tmp, nt);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nt), dim3(SC_THREADS), 0, s, out, n, tmp);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// stable LSD radix sort of (uint32 key, int32 payload), 8-bit digits
// --------------------------------------------------------------------------
__global__ void k_rs_hist(const uint32_t *keys, int64_t n, int shift, int64_t *counts, int64_t nb) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
        int64_t e = base + (int64_t)r * RS_THREADS + threadIdx.x;
        if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255u], 1);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_rs_scatter(const uint32_t *kin, const int32_t *vin, uint32_t *kout, int32_t *vout,
                             int64_t n, int shift, const int64_t *offsets, int64_t nb) {
    __shared__ int64_t run[256];
    __shared__ int wcnt[RS_THREADS / 64][256];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    run[tid] = offsets[(int64_t)tid * nb + blockIdx.x];
    for (int q = 0; q < RS_THREADS / 64; ++q) wcnt[q][tid] = 0;
    __syncthreads();
    const uint64_t lanemask_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < RS_ITEMS; ++r) {
        int64_t e = (int64_t)blockIdx.x * RS_TILE + (int64_t)r * RS_THREADS + tid;
        bool valid = e < n;
        uint32_t k = valid ? kin[e] : 0u;
        int32_t v = valid ? vin[e] : 0;
        int d = (int)((k >> shift) & 255u);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bb : ~bb;
        }
        int rank = __popcll(peers & lanemask_lt);
        int leader = __ffsll((unsigned long long)peers) - 1;
        if (valid && lane == leader) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int64_t off = run[d] + rank;
            for (int q = 0; q < w; ++q) off += wcnt[q][d];
            kout[off] = k;
            vout[off] = v;
        }
        __syncthreads();
        int tot = 0;
        for (int q = 0; q < RS_THREADS / 64; ++q) {
            tot += wcnt[q][tid];
            wcnt[q][tid] = 0;
        }
        run[tid] += tot;
        __syncthreads();
    }
}

size_t radix_temp_bytes(int64_t n) {
    int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    size_t cnt = align256(sizeof(int64_t) * (size_t)(256 * nb + 1));
    return 2 * cnt + scan_temp_bytes(256 * nb + 1);
}

// Sorts (k0, v0) by the low `bits` bits of the key; the result ends in
// (k0, v0) (ping-pong through k1, v1).
hipError_t radix_sort(uint32_t *k0, int32_t *v0, uint32_t *k1, int32_t *v1, int64_t n, int bits,
                      void *temp, hipStream_t s) {
    if (n <= 1) return hipSuccess;
    int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    size_t cnt_bytes = align256(sizeof(int64_t) * (size_t)(256 * nb + 1));
    int64_t *counts = (int64_t *)temp;
    int64_t *offs = (int64_t *)((char *)temp + cnt_bytes);
    int64_t *stmp = (int64_t *)((char *)temp + 2 * cnt_bytes);
    uint32_t *ki = k0, *ko = k1;
    int32_t *vi = v0, *vo = v1;
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(RS_THREADS), 0, s, ki, n, shift, counts, nb);
        hipError_t e = exclusive_scan(counts, offs, 256 * nb, stmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(RS_THREADS), 0, s, ki, vi, ko, vo, n,
                           shift, offs, nb);
        uint32_t *tk = ki; ki = ko; ko = tk;
        int32_t *tv = vi; vi = vo; vo = tv;
    }
    if (ki != k0) {
        hipError_t e = hipMemcpyAsync(k0, ki, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(v0, vi, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

int bits_for(int64_t maxval) {
    int b = 0;
    while (b < 32 && (int64_t(1) << b) <= maxval) ++b;
    return b < 1 ? 1 : b;
}

// --------------------------------------------------------------------------
// CSC build helpers
// --------------------------------------------------------------------------
__global__ void k_row_of(int64_t n_rows, const int64_t *ptr, int32_t *row_of) {
    // one wave per row
    int lane = threadIdx.x & 63;
    int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = w; i < n_rows; i += nw)
        for (int64_t e = ptr[i] + lane; e < ptr[i + 1]; e += 64) row_of[e] = (int32_t)i;
}

__global__ void k_csc_keys(int64_t nnz, const int32_t *col_idx, uint32_t *keys, int32_t *vals,
                           unsigned long long *colcount) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        int c = col_idx[e];
        keys[e] = (uint32_t)c;
        vals[e] = (int32_t)e;
        atomicAdd(&colcount[c], 1ull);
    }
}

__global__ void k_csc_gather(int64_t nnz, const int32_t *perm, const int32_t *row_of, const float *val,
                             int32_t *row_idx, float *val_t) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nnz;
         t += (int64_t)gridDim.x * blockDim.x) {
        int32_t e = perm[t];
        row_idx[t] = row_of[e];
        val_t[t] = val[e];
    }
}

// --------------------------------------------------------------------------
// schedule: rows ordered by (class, degree descending)
// --------------------------------------------------------------------------
__global__ void k_sched_keys(int64_t n_rows, const int64_t *ptr, uint32_t num, uint32_t den,
                             int32_t min_keep, int32_t heavy_n, uint32_t *keys, int32_t *vals,
                             unsigned long long *class_count, unsigned long long *max_deg) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_rows;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t n = ptr[i + 1] - ptr[i];
        int64_t s = budget_of(n, num, den, min_keep);
        int cls = class_of(n, s, heavy_n);
        int64_t nc = n < 0x7FFFFFF ? n : 0x7FFFFFF;
        keys[i] = ((uint32_t)cls << 27) | (uint32_t)(0x7FFFFFF - nc);
        vals[i] = (int32_t)i;
        atomicAdd(&class_count[cls], 1ull);
        atomicMax(max_deg, (unsigned long long)n);
    }
}

__global__ void k_sel_sizes(const int64_t *ptr, int64_t row_begin, int64_t cnt, int32_t nf, uint32_t num,
                            uint32_t den, int32_t min_keep, int64_t *sizes) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= cnt;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (t == cnt) {
            sizes[t] = 0;
        } else {
            int64_t i = row_begin + t;
            int64_t n = ptr[i + 1] - ptr[i];
            sizes[t] = (int64_t)nf * budget_of(n, num, den, min_keep);
        }
    }
}

unsigned grid_for(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > 65535 * 4) g = 65535 * 4;
    return (unsigned)g;
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
    for (int q = threadIdx.x; q < n; q += blockDim.x) p[q] = 0ull;
}

}  // namespace

// Clears counters with a kernel (safe inside a captured HIP graph).
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

size_t csc_temp_bytes(int64_t nnz, int64_t n_cols) {
    size_t n = (size_t)(nnz > 0 ? nnz : 1);
    size_t b = 0;
    b += 4 * align256(sizeof(uint32_t) * n);                  // keys x2, vals x2
    b += align256(sizeof(int32_t) * n);                       // row_of
    b += align256(sizeof(int64_t) * (size_t)(n_cols + 1));    // column counts
    b += scan_temp_bytes(n_cols + 1);
    b += radix_temp_bytes(nnz);
    return b;
}

size_t perm_temp_bytes(int64_t n_rows) {
    size_t n = (size_t)(n_rows > 0 ? n_rows : 1);
    size_t b = 0;
    b += 4 * align256(sizeof(uint32_t) * n);
    b += align256(sizeof(int64_t) * (size_t)(NCLASS + 2));
    b += radix_temp_bytes(n_rows);
    b += align256(sizeof(int64_t) * (n + 1)) + scan_temp_bytes(n_rows + 1);
    return b;
}

hipError_t launch_validate(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *ptr,
                           const int32_t *idx, const float *val, int check_values, int *err_flags,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for(n_rows + 1, 256)), dim3(256), 0, s, n_rows, n_cols, nnz,
                       ptr, idx, val, check_values, err_flags);
    return hipGetLastError();
}

hipError_t build_csc(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                     const int32_t *col_idx, const float *val, int64_t *col_ptr, int32_t *row_idx,
                     float *val_t, void *temp, hipStream_t s) {
    size_t n = (size_t)(nnz > 0 ? nnz : 1);
    char *p = (char *)temp;
    uint32_t *k0 = (uint32_t *)p; p += align256(sizeof(uint32_t) * n);
    uint32_t *k1 = (uint32_t *)p; p += align256(sizeof(uint32_t) * n);
    int32_t *v0 = (int32_t *)p; p += align256(sizeof(int32_t) * n);
    int32_t *v1 = (int32_t *)p; p += align256(sizeof(int32_t) * n);
    int32_t *row_of = (int32_t *)p; p += align256(sizeof(int32_t) * n);
    int64_t *colcount = (int64_t *)p; p += align256(sizeof(int64_t) * (size_t)(n_cols + 1));
    int64_t *stmp = (int64_t *)p; p += scan_temp_bytes(n_cols + 1);
    void *rtmp = p;

    hipError_t e = hipMemsetAsync(colcount, 0, sizeof(int64_t) * (size_t)(n_cols + 1), s);
    if (e != hipSuccess) return e;
    if (nnz > 0) {
        hipLaunchKernelGGL(k_row_of, dim3(grid_for(n_rows * 64, 256)), dim3(256), 0, s, n_rows, row_ptr, row_of);
        hipLaunchKernelGGL(k_csc_keys, dim3(grid_for(nnz, 256)), dim3(256), 0, s, nnz, col_idx, k0, v0,
                           (unsigned long long *)colcount);
        e = radix_sort(k0, v0, k1, v1, nnz, bits_for(n_cols - 1), rtmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_csc_gather, dim3(grid_for(nnz, 256)), dim3(256), 0, s, nnz, v0, row_of, val,
                           row_idx, val_t);
    }
    e = exclusive_scan(colcount, col_ptr, n_cols + 1, stmp, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t build_schedule(int64_t n_rows, const int64_t *ptr, uint32_t num, uint32_t den, int32_t min_keep,
                          int32_t heavy_n, int32_t *perm, int64_t *class_count_dev, int64_t *max_deg_dev, void *temp,
                          hipStream_t s) {
    size_t n = (size_t)(n_rows > 0 ? n_rows : 1);
    char *p = (char *)temp;
    uint32_t *k0 = (uint32_t *)p; p += align256(sizeof(uint32_t) * n);
    uint32_t *k1 = (uint32_t *)p; p += align256(sizeof(uint32_t) * n);
    int32_t *v1 = (int32_t *)p; p += align256(sizeof(int32_t) * n);
    p += align256(sizeof(int32_t) * n);
    p += align256(sizeof(int64_t) * (size_t)(NCLASS + 2));
    void *rtmp = p;
    hipError_t e = hipMemsetAsync(class_count_dev, 0, sizeof(int64_t) * NCLASS, s);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(max_deg_dev, 0, sizeof(int64_t), s);
    if (e != hipSuccess) return e;
    if (n_rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sched_keys, dim3(grid_for(n_rows, 256)), dim3(256), 0, s, n_rows, ptr, num, den,
                       min_keep, heavy_n, k0, perm, (unsigned long long *)class_count_dev,
                       (unsigned long long *)max_deg_dev);
    return radix_sort(k0, perm, k1, v1, n_rows, 31, rtmp, s);
}

hipError_t launch_select_sizes(const int64_t *ptr, int64_t row_begin, int64_t row_end, int32_t nf, uint32_t num,
                               uint32_t den, int32_t min_keep, int64_t *sel_ptr, void *temp, hipStream_t s) {
    int64_t cnt = row_end - row_begin;
    int64_t *sizes = (int64_t *)temp;
    int64_t *stmp = (int64_t *)((char *)temp + align256(sizeof(int64_t) * (size_t)(cnt + 1)));
    hipLaunchKernelGGL(k_sel_sizes, dim3(grid_for(cnt + 1, 256)), dim3(256), 0, s, ptr, row_begin, cnt, nf, num,
                       den, min_keep, sizes);
    return exclusive_scan(sizes, sel_ptr, cnt + 1, stmp, s);
}

}  // namespace coreals
