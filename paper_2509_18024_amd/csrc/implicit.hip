// Implicit-feedback Core-ALS (gfx950): the Gram of the other side's factor
// matrix, and the light-row launches.
//
// Implicit ALS (Hu, Koren and Volinsky, 2008) treats every observed entry as
// a preference 1 with confidence 1 + alpha r and every other entry as a
// preference 0 with confidence 1; a row's system splits into the Gram of the
// whole other factor matrix, G = Y^T Y (the same for every row of a
// half-sweep), plus the observed part, which the core-elements sketch
// subsamples (Section 3, last paragraph):
//     (G + X*^T W X + lambda E) u = X*^T (1 + alpha r),   W = diag(alpha r).
// The row kernels are those of the explicit method with the weighted Gram
// (gram_range_sparse<.., true>, the heavy-row Gram with IMPL) and
// finish_system_implicit.
//
//   k_gram_part    each block sums X_j^T X_j over its share of the rows in
//                  FP64 (64 rows staged in LDS at a time, 16 outputs per
//                  thread), one partial Gram per block;
//   k_gram_reduce  the partials in block order (deterministic), rounded to
//                  FP32 for the row systems.
#include "rowops.hpp"

namespace coreals {

namespace {

constexpr int GG_BLOCKS = 256;
constexpr int GG_THREADS = 256;

__global__ __launch_bounds__(GG_THREADS) void k_gram_part(const float *other, int64_t n_other, int nf,
                                                          double *part) {
    __shared__ float X[64][NF + 1];
    const int tid = threadIdx.x;
    const int a = tid >> 2, c0 = (tid & 3) * 16;  // outputs (a, c0 .. c0 + 15)
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    const int64_t per = (n_other + gridDim.x - 1) / gridDim.x;
    const int64_t j0 = (int64_t)blockIdx.x * per;
    const int64_t j1 = min(n_other, j0 + per);
    for (int64_t jb = j0; jb < j1; jb += 64) {
        __syncthreads();
        for (int q = tid; q < 64 * NF; q += GG_THREADS) {
            const int r = q / NF, col = q % NF;
            X[r][col] = (jb + r < j1 && col < nf) ? other[(jb + r) * nf + col] : 0.f;
        }
        __syncthreads();
        const int m = (int)min((int64_t)64, j1 - jb);
        for (int r = 0; r < m; ++r) {
            const double xa = (double)X[r][a];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] = fma(xa, (double)X[r][c0 + q], acc[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) part[(int64_t)blockIdx.x * NF * NF + a * NF + c0 + q] = acc[q];
}

__global__ __launch_bounds__(GG_THREADS) void k_gram_reduce(const double *part, int nb, float *G) {
    const int t = blockIdx.x * GG_THREADS + threadIdx.x;
    if (t >= NF * NF) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(int64_t)b * NF * NF + t];
    G[t] = (float)s;
}

}  // namespace

int implicit_gram_blocks() { return GG_BLOCKS; }

hipError_t launch_global_gram(const float *other, int64_t n_other, int nf, double *partials, float *G,
                              hipStream_t s) {
    if (nf < 1 || nf > NF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gram_part, dim3(GG_BLOCKS), dim3(GG_THREADS), 0, s, other, n_other, nf, partials);
    hipLaunchKernelGGL(k_gram_reduce, dim3((NF * NF + GG_THREADS - 1) / GG_THREADS), dim3(GG_THREADS), 0, s,
                       partials, GG_BLOCKS, G);
    return hipGetLastError();
}

}  // namespace coreals
