// Objective of Section 2.1 (weighted-lambda penalty) with SSE, RMSE and ReMSE
// (Section 5.1).  FP32 products, FP64 accumulation, fixed grid and fixed
// reduction order, so repeated calls give bit-identical results.
#include "internal.hpp"

namespace coreals {

namespace {

constexpr int OBJ_THREADS = 256;
constexpr int OBJ_BLOCKS = 1024;

__device__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = OBJ_THREADS / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// One wave per user row: residuals of the row's entries (lanes over entries)
// and the row's penalty term n_i |u_i|^2.
__global__ __launch_bounds__(OBJ_THREADS) void k_obj_rows(int64_t n_u, int32_t nf, const int64_t *row_ptr,
                                                          const int32_t *col_idx, const float *val,
                                                          const float *U, const float *M, double *part) {
    __shared__ double sh[OBJ_THREADS];
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * OBJ_THREADS + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * OBJ_THREADS) >> 6;
    const bool vec4 = (nf % 4 == 0) && ((reinterpret_cast<uintptr_t>(U) & 15) == 0) &&
                      ((reinterpret_cast<uintptr_t>(M) & 15) == 0);
    double sse = 0.0, rr = 0.0, pen = 0.0;
    for (int64_t i = wave; i < n_u; i += nwaves) {
        const int64_t b = row_ptr[i], e = row_ptr[i + 1];
        const float *u = U + i * nf;
        for (int c = lane; c < nf; c += 64) pen += (double)(e - b) * (double)u[c] * (double)u[c];
        for (int64_t t = b + lane; t < e; t += 64) {
            const float *m = M + (int64_t)col_idx[t] * nf;
            float pred = 0.f;
            if (vec4) {
                for (int c = 0; c < nf; c += 4) {
                    const float4 uu = *reinterpret_cast<const float4 *>(u + c);
                    const float4 mm = *reinterpret_cast<const float4 *>(m + c);
                    pred = fmaf(uu.x, mm.x, pred);
                    pred = fmaf(uu.y, mm.y, pred);
                    pred = fmaf(uu.z, mm.z, pred);
                    pred = fmaf(uu.w, mm.w, pred);
                }
            } else {
                for (int c = 0; c < nf; ++c) pred = fmaf(u[c], m[c], pred);
            }
            const double y = (double)val[t];
            const double r = y - (double)pred;
            sse += r * r;
            rr += y * y;
        }
    }
    sse = block_sum(sse, sh);
    rr = block_sum(rr, sh);
    pen = block_sum(pen, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 0] = sse;
        part[blockIdx.x * 4 + 1] = rr;
        part[blockIdx.x * 4 + 2] = pen;
        part[blockIdx.x * 4 + 3] = 0.0;
    }
}

// Item penalty n_j |m_j|^2 (n_j from the column pointer of the CSC).
__global__ __launch_bounds__(OBJ_THREADS) void k_obj_items(int64_t n_m, int32_t nf, const int64_t *col_ptr,
                                                           const float *M, double *part) {
    __shared__ double sh[OBJ_THREADS];
    double pen = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * OBJ_THREADS + threadIdx.x; j < n_m;
         j += (int64_t)gridDim.x * OBJ_THREADS) {
        const double d = (double)(col_ptr[j + 1] - col_ptr[j]);
        double nrm = 0.0;
        for (int c = 0; c < nf; ++c) {
            const double v = (double)M[j * nf + c];
            nrm += v * v;
        }
        pen += d * nrm;
    }
    pen = block_sum(pen, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = pen;
}

__global__ __launch_bounds__(OBJ_THREADS) void k_obj_final(const double *rows, const double *items, int nb,
                                                           int64_t nnz, double lam, double *out) {
    __shared__ double sh[OBJ_THREADS];
    double sse = 0.0, rr = 0.0, pu = 0.0, pm = 0.0;
    for (int b = threadIdx.x; b < nb; b += OBJ_THREADS) {
        sse += rows[b * 4 + 0];
        rr += rows[b * 4 + 1];
        pu += rows[b * 4 + 2];
        pm += items[b];
    }
    sse = block_sum(sse, sh);
    rr = block_sum(rr, sh);
    pu = block_sum(pu, sh);
    pm = block_sum(pm, sh);
    if (threadIdx.x == 0) {
        out[0] = sse + lam * (pu + pm);
        out[1] = sse;
        out[2] = nnz > 0 ? sqrt(sse / (double)nnz) : 0.0;
        out[3] = rr > 0.0 ? sqrt(sse) / sqrt(rr) : 0.0;
    }
}

}  // namespace

int objective_blocks() { return OBJ_BLOCKS; }

hipError_t launch_objective(int64_t n_u, int64_t n_m, int32_t nf, const int64_t *row_ptr, const int32_t *col_idx,
                            const float *val, const int64_t *col_ptr, const float *U, const float *M, double lam,
                            double *partials, double *out4, hipStream_t s) {
    double *prow = partials;
    double *pitem = partials + 4 * OBJ_BLOCKS;
    int64_t nnz = 0;
    hipLaunchKernelGGL(k_obj_rows, dim3(OBJ_BLOCKS), dim3(OBJ_THREADS), 0, s, n_u, nf, row_ptr, col_idx, val, U, M,
                       prow);
    hipLaunchKernelGGL(k_obj_items, dim3(OBJ_BLOCKS), dim3(OBJ_THREADS), 0, s, n_m, nf, col_ptr, M, pitem);
    hipError_t e = hipMemcpyAsync(&nnz, row_ptr + n_u, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_obj_final, dim3(1), dim3(OBJ_THREADS), 0, s, prow, pitem, OBJ_BLOCKS, nnz, lam, out4);
    return hipGetLastError();
}

}  // namespace coreals
