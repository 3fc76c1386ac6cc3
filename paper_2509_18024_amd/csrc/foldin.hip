// Learned fold-in of new users (gfx950).  A small MLP maps the rating-weighted
// mean of a user's item factors to that user's factor row; the answer is kept
// when the relative residual of the user's own regression (the system a users
// half-sweep solves: eq. core_ui, eq. (U) when r = 1) is within a tolerance,
// and that regression is solved exactly otherwise.
//
//   k_bag          one wavefront per user: b = (1/d) sum_k r_k M[j_k]; lane f
//                  holds feature f, item rows are gathered eight at a time
//   k_gemm         C = A B on MFMA, one 32x32 tile per wavefront: bf16
//                  operands with FP32 accumulation (v_mfma_f32_32x32x16_bf16)
//                  or FP32 operands (v_mfma_f32_32x32x2_f32); strided operand
//                  views, so transposed products need no copies; epilogues:
//                  bias, bias + GELU (keeping the pre-activation), times the
//                  GELU derivative, and split-K partial slabs
//   k_loss         mean squared error and its gradient with respect to the output
//   k_wgrad        fixed-order sum of the split-K slabs into weight and bias
//                  gradients (the bias gradient is the product with a column of ones)
//   k_adamw        AdamW on the FP32 master weights
#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace coreals;

struct foldin_model {
    foldin_cfg cfg{};
    int nf = 0, H = 0, Bmax = 0;
    int64_t P = 0;
    hipStream_t stream = nullptr;
    float *theta = nullptr, *mom = nullptr, *vel = nullptr, *grad = nullptr;
    float *X0 = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *OUT = nullptr;
    float *D3 = nullptr, *D2 = nullptr, *D1 = nullptr;
    float *part = nullptr;
    double *loss_part = nullptr;
    double *loss_acc = nullptr;
    int32_t *perm = nullptr;
    int64_t step = 0;
    std::string err;
};

namespace {

constexpr int G_WAVES = 4;         // waves per GEMM workgroup (2 x 2 tiles of 32 x 32)
constexpr int KSPLIT = 256;        // batch rows per split-K slab of a weight gradient
constexpr int LOSS_BLOCKS = 256;
constexpr int FOLDIN_MAX_HIDDEN = 1024;

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

enum Epi : int { E_BIAS = 0, E_BIAS_GELU = 1, E_GELU_BWD = 2, E_PARTIAL = 3 };

struct GemmArgs {
    const float *A;
    int64_t a_m, a_k;  // A(m, k) = A[m * a_m + k * a_k]
    const float *B;
    int64_t b_k, b_n;  // B(k, n) = B[k * b_k + n * b_n]
    int M, N, K;
    int ones_n;        // column n == ones_n reads B(k, n) = 1; -1: none
    const float *bias; // [N] or nullptr
    float *out;
    int64_t ldo;       // out[m * ldo + n] (E_PARTIAL: slab z at out + z * M * ldo)
    float *zout;       // E_BIAS_GELU: pre-activation, same layout as out
    const float *zin;  // E_GELU_BWD: pre-activation, same layout as out
};

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad_f(float z) {
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

__device__ __forceinline__ float load_a(const GemmArgs &g, int m, int k, bool ok) {
    const float v = g.A[(int64_t)m * g.a_m + (int64_t)k * g.a_k];
    return ok ? v : 0.f;
}

// The ones column has no storage: its load reads column 0 (in range) and is
// replaced by 1.
__device__ __forceinline__ float load_b(const GemmArgs &g, int k, int n, bool ok, bool ones) {
    const float v = g.B[(int64_t)k * g.b_k + (int64_t)(ones ? 0 : n) * g.b_n];
    return ok ? (ones ? 1.f : v) : 0.f;
}

// One 32 x 32 tile of C per wavefront; blockIdx.z selects the split-K slab.
// Out-of-range rows, columns and k read clamped (valid) addresses and are
// zeroed, so every load is unconditional.  Output lane l holds column l % 32
// and rows 8 (r / 4) + 4 (l / 32) + r % 4 of accumulator r.
template <bool BF16, int EPI>
__global__ __launch_bounds__(G_WAVES * 64) void k_gemm(GemmArgs g, int k_per_split) {
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    const int l = lane & 31, h = lane >> 5;
    const int m0 = blockIdx.y * 64 + 32 * (w & 1);
    const int n0 = blockIdx.x * 64 + 32 * (w >> 1);
    if (m0 >= g.M || n0 >= g.N) return;
    const int kb = blockIdx.z * k_per_split;
    const int ke = min(g.K, kb + k_per_split);
    const int mrow = m0 + l, ncol = n0 + l;
    const bool mok = mrow < g.M, nok = ncol < g.N;
    const int mr = mok ? mrow : g.M - 1;
    const int nc = nok ? ncol : g.N - 1;
    const bool ones = ncol == g.ones_n;
    f32x16 acc;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.f;
    if constexpr (BF16) {
        for (int k0 = kb; k0 < ke; k0 += 16) {
            bf16x8 av, bv;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + 8 * h + e;
                const bool kok = k < ke;
                const int kc = kok ? k : ke - 1;
                av[e] = (__bf16)load_a(g, mr, kc, mok && kok);
                bv[e] = (__bf16)load_b(g, kc, nc, nok && kok, ones);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
    } else {
        for (int k0 = kb; k0 < ke; k0 += 2) {
            const int k = k0 + h;
            const bool kok = k < ke;
            const int kc = kok ? k : ke - 1;
            const float av = load_a(g, mr, kc, mok && kok);
            const float bv = load_b(g, kc, nc, nok && kok, ones);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
        }
    }
    if (!nok) return;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int row = m0 + 8 * (q >> 2) + 4 * h + (q & 3);
        if (row >= g.M) continue;
        const int64_t o = (int64_t)row * g.ldo + ncol;
        float v = acc[q];
        if constexpr (EPI == E_BIAS) {
            if (g.bias) v += g.bias[ncol];
            g.out[o] = v;
        } else if constexpr (EPI == E_BIAS_GELU) {
            v += g.bias[ncol];
            g.zout[o] = v;
            g.out[o] = gelu_f(v);
        } else if constexpr (EPI == E_GELU_BWD) {
            g.out[o] = v * gelu_grad_f(g.zin[o]);
        } else {
            g.out[(int64_t)blockIdx.z * g.M * g.ldo + o] = v;
        }
    }
}

// Embedding bag: out[b] = (1/d) sum_k r_k M[j_k] for row rows[b] (or
// row_begin + b); zero for a row without ratings.
__global__ __launch_bounds__(WPB * 64) void k_bag(const int64_t *ptr, const int32_t *items, const float *vals,
                                                  const int32_t *rows, int64_t row_begin, int64_t nrows,
                                                  const float *M, int nf, float *out) {
    const int w = wave_index();
    const int lane = threadIdx.x & 63;
    const int lc = min(lane, nf - 1);
    for (int64_t b = (int64_t)blockIdx.x * WPB + w; b < nrows; b += (int64_t)gridDim.x * WPB) {
        const int64_t i = rows ? (int64_t)rows[b] : row_begin + b;
        const int64_t beg = ptr[i];
        const int n = (int)(ptr[i + 1] - beg);
        float acc = 0.f;
        for (int k0 = 0; k0 < n; k0 += 64) {
            const int m = min(64, n - k0);
            const int j = lane < m ? items[beg + k0 + lane] : 0;
            const float r = lane < m ? vals[beg + k0 + lane] : 0.f;
            for (int kk = 0; kk < m; kk += 8) {
                float v[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int jj = __builtin_amdgcn_readlane(j, (kk + e) & 63);
                    v[e] = M[(int64_t)jj * nf + lc];
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float rr = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(r), (kk + e) & 63));
                    if (kk + e < m) acc = fmaf(rr, v[e], acc);
                }
            }
        }
        if (lane < nf) out[b * nf + lane] = n > 0 ? acc / (float)n : 0.f;
    }
}

// d_out = 2 (out - target) / (B n_f); per-block FP64 partial sums of squares.
__global__ __launch_bounds__(256) void k_loss(const float *out, const float *target, const int32_t *rows,
                                              int64_t row_begin, int64_t B, int nf, float *dout, double *part) {
    __shared__ double red[256];
    const int64_t total = B * nf;
    const float scale = 2.f / (float)total;
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t b = e / nf;
        const int f = (int)(e - b * nf);
        const int64_t i = rows ? (int64_t)rows[b] : row_begin + b;
        const float d = out[e] - target[i * nf + f];
        dout[e] = scale * d;
        s += (double)d * (double)d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss = sum of partials / (B n_f), in a fixed order; optionally added to an
// epoch accumulator and stored as float.
__global__ void k_loss_final(const double *part, int nparts, double total, float *loss_out, double *acc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int q = 0; q < nparts; ++q) s += part[q];
    const double L = s / total;
    if (loss_out) loss_out[0] = (float)L;
    if (acc) acc[0] += L;
}

__global__ void k_zero_d(double *p, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

// Weight gradient [M x (N - 1)] and bias gradient [M] from S slabs of the
// augmented product [M x N] (last column = sum over the batch).
__global__ __launch_bounds__(256) void k_wgrad(const float *part, int S, int M, int N, float *gW, float *gc) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)M * N) return;
    const int m = (int)(t / N), n = (int)(t - (int64_t)m * N);
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += part[(int64_t)z * M * N + t];
    if (n < N - 1) gW[(int64_t)m * (N - 1) + n] = s;
    else gc[m] = s;
}

__global__ __launch_bounds__(256) void k_adamw(float *theta, float *mom, float *vel, const float *grad, int64_t P,
                                               float lr, float b1, float b2, float eps, float wd, float c1, float c2) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= P) return;
    const float g = grad[t];
    const float m = b1 * mom[t] + (1.f - b1) * g;
    const float v = b2 * vel[t] + (1.f - b2) * g * g;
    mom[t] = m;
    vel[t] = v;
    const float mh = m * c1, vh = v * c2;
    theta[t] = theta[t] - lr * (mh / (sqrtf(vh) + eps) + wd * theta[t]);
}

inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct FoldinLayout {
    size_t theta, mom, vel, grad, X0, Z1, H1, Z2, H2, OUT, D3, D2, D1, part, loss_part, loss_acc, perm, total;
};

int64_t param_count(int nf, int H) { return (int64_t)H * nf + H + (int64_t)H * H + H + (int64_t)nf * H + nf; }

int max_splits(int Bmax) { return (Bmax + KSPLIT - 1) / KSPLIT; }

FoldinLayout foldin_layout(const foldin_cfg &c) {
    FoldinLayout L{};
    const int64_t P = param_count(c.n_f, c.hidden);
    const int64_t B = c.max_batch, F = c.n_f, H = c.hidden;
    const int64_t W = std::max(F, H);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += a256(bytes ? bytes : 1);
        return o;
    };
    L.theta = take(sizeof(float) * P);
    L.mom = take(sizeof(float) * P);
    L.vel = take(sizeof(float) * P);
    L.grad = take(sizeof(float) * P);
    L.X0 = take(sizeof(float) * B * F);
    L.Z1 = take(sizeof(float) * B * H);
    L.H1 = take(sizeof(float) * B * H);
    L.Z2 = take(sizeof(float) * B * H);
    L.H2 = take(sizeof(float) * B * H);
    L.OUT = take(sizeof(float) * B * F);
    L.D3 = take(sizeof(float) * B * F);
    L.D2 = take(sizeof(float) * B * H);
    L.D1 = take(sizeof(float) * B * H);
    L.part = take(sizeof(float) * (size_t)max_splits((int)B) * W * (W + 1));
    L.loss_part = take(sizeof(double) * LOSS_BLOCKS);
    L.loss_acc = take(sizeof(double) * 2);
    L.perm = take(sizeof(int32_t) * (size_t)std::max<int64_t>(c.max_train_rows, 0));
    L.total = off;
    return L;
}

bool cfg_ok(const foldin_cfg *c) {
    return c && c->n_f >= 1 && c->n_f <= NF && c->hidden >= 1 && c->hidden <= FOLDIN_MAX_HIDDEN && c->max_batch >= 1 &&
           c->max_batch <= (1 << 20) && (c->precision == FOLDIN_BF16 || c->precision == FOLDIN_FP32) &&
           c->max_train_rows >= 0 && c->max_train_rows <= INT32_MAX;
}

als_status mfail(foldin_model *m, als_status st, const std::string &msg) {
    if (m) m->err = msg;
    return st;
}

#define MHIP(m, expr)                                                                                \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return mfail((m), ALS_E_DEVICE, std::string("HIP error: ") + hipGetErrorString(e_)); \
    } while (0)

hipError_t gemm(const foldin_model *m, int epi, const GemmArgs &g, int splits, int k_per_split, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipSuccess;
    dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64), (unsigned)splits);
    dim3 block(G_WAVES * 64);
    const bool bf = m->cfg.precision == FOLDIN_BF16;
#define GEMM_LAUNCH(B16, E) hipLaunchKernelGGL((k_gemm<B16, E>), grid, block, 0, s, g, k_per_split)
    switch (epi) {
        case E_BIAS: if (bf) GEMM_LAUNCH(true, E_BIAS); else GEMM_LAUNCH(false, E_BIAS); break;
        case E_BIAS_GELU: if (bf) GEMM_LAUNCH(true, E_BIAS_GELU); else GEMM_LAUNCH(false, E_BIAS_GELU); break;
        case E_GELU_BWD: if (bf) GEMM_LAUNCH(true, E_GELU_BWD); else GEMM_LAUNCH(false, E_GELU_BWD); break;
        default: if (bf) GEMM_LAUNCH(true, E_PARTIAL); else GEMM_LAUNCH(false, E_PARTIAL); break;
    }
#undef GEMM_LAUNCH
    return hipGetLastError();
}

struct Params {
    float *W1, *c1, *W2, *c2, *W3, *c3;
};

Params views(float *base, int F, int H) {
    Params p;
    p.W1 = base;
    p.c1 = p.W1 + (int64_t)H * F;
    p.W2 = p.c1 + H;
    p.c2 = p.W2 + (int64_t)H * H;
    p.W3 = p.c2 + H;
    p.c3 = p.W3 + (int64_t)F * H;
    return p;
}

// Forward pass of B <= Bmax rows (rows[b] or row_begin + b); output to out
// (row-major [B x n_f]) or to the model's OUT buffer when out is nullptr.
hipError_t forward_batch(foldin_model *m, hipStream_t s, const float *M, const int64_t *ptr, const int32_t *items,
                         const float *vals, const int32_t *rows, int64_t row_begin, int B, float *out) {
    const int F = m->nf, H = m->H;
    Params p = views(m->theta, F, H);
    unsigned bag_blocks = (unsigned)std::min<int64_t>((B + WPB - 1) / WPB, 65536);
    hipLaunchKernelGGL(k_bag, dim3(bag_blocks), dim3(WPB * 64), 0, s, ptr, items, vals, rows, row_begin,
                       (int64_t)B, M, F, m->X0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    GemmArgs g{};
    g.ones_n = -1;
    // layer 1: Z1 = X0 W1^T + c1, H1 = GELU(Z1)
    g.A = m->X0; g.a_m = F; g.a_k = 1;
    g.B = p.W1; g.b_k = 1; g.b_n = F;
    g.M = B; g.N = H; g.K = F;
    g.bias = p.c1; g.out = m->H1; g.ldo = H; g.zout = m->Z1;
    if ((e = gemm(m, E_BIAS_GELU, g, 1, F, s)) != hipSuccess) return e;
    // layer 2
    g.A = m->H1; g.a_m = H; g.a_k = 1;
    g.B = p.W2; g.b_k = 1; g.b_n = H;
    g.M = B; g.N = H; g.K = H;
    g.bias = p.c2; g.out = m->H2; g.ldo = H; g.zout = m->Z2;
    if ((e = gemm(m, E_BIAS_GELU, g, 1, H, s)) != hipSuccess) return e;
    // layer 3 (linear)
    g.A = m->H2; g.a_m = H; g.a_k = 1;
    g.B = p.W3; g.b_k = 1; g.b_n = H;
    g.M = B; g.N = F; g.K = H;
    g.bias = p.c3; g.out = out ? out : m->OUT; g.ldo = F; g.zout = nullptr;
    return gemm(m, E_BIAS, g, 1, H, s);
}

// Weight and bias gradient of one layer: gW[Mo x Ki] = D^T X, gc = sum_b D,
// D [B x Mo] and X [B x Ki] row-major, as split-K slabs then a fixed-order sum.
hipError_t layer_wgrad(foldin_model *m, hipStream_t s, const float *D, int Mo, const float *X, int Ki, int B,
                       float *gW, float *gc) {
    GemmArgs g{};
    g.A = D; g.a_m = 1; g.a_k = Mo;
    g.B = X; g.b_k = Ki; g.b_n = 1;
    g.M = Mo; g.N = Ki + 1; g.K = B;
    g.ones_n = Ki;
    g.out = m->part; g.ldo = Ki + 1;
    const int S = max_splits(B);
    hipError_t e = gemm(m, E_PARTIAL, g, S, KSPLIT, s);
    if (e != hipSuccess) return e;
    const int64_t tot = (int64_t)Mo * (Ki + 1);
    hipLaunchKernelGGL(k_wgrad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, m->part, S, Mo, Ki + 1, gW, gc);
    return hipGetLastError();
}

// Forward and backward of one batch; gradient into m->grad, batch loss into
// loss_out (device float, optional) and added to acc (device double, optional).
hipError_t grad_batch(foldin_model *m, hipStream_t s, const float *M, const int64_t *ptr, const int32_t *items,
                      const float *vals, const int32_t *rows, int64_t row_begin, int B, const float *target,
                      float *loss_out, double *acc) {
    const int F = m->nf, H = m->H;
    hipError_t e = forward_batch(m, s, M, ptr, items, vals, rows, row_begin, B, nullptr);
    if (e != hipSuccess) return e;
    const int64_t total = (int64_t)B * F;
    const int nb = (int)std::min<int64_t>(LOSS_BLOCKS, (total + 255) / 256);
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, s, m->OUT, target, rows, row_begin, (int64_t)B, F, m->D3,
                       m->loss_part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, m->loss_part, nb, (double)total, loss_out, acc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    Params p = views(m->theta, F, H);
    Params gp = views(m->grad, F, H);
    // layer 3
    if ((e = layer_wgrad(m, s, m->D3, F, m->H2, H, B, gp.W3, gp.c3)) != hipSuccess) return e;
    GemmArgs g{};
    g.ones_n = -1;
    g.A = m->D3; g.a_m = F; g.a_k = 1;
    g.B = p.W3; g.b_k = H; g.b_n = 1;
    g.M = B; g.N = H; g.K = F;
    g.out = m->D2; g.ldo = H; g.zin = m->Z2;
    if ((e = gemm(m, E_GELU_BWD, g, 1, F, s)) != hipSuccess) return e;
    // layer 2
    if ((e = layer_wgrad(m, s, m->D2, H, m->H1, H, B, gp.W2, gp.c2)) != hipSuccess) return e;
    g.A = m->D2; g.a_m = H; g.a_k = 1;
    g.B = p.W2; g.b_k = H; g.b_n = 1;
    g.M = B; g.N = H; g.K = H;
    g.out = m->D1; g.ldo = H; g.zin = m->Z1;
    if ((e = gemm(m, E_GELU_BWD, g, 1, H, s)) != hipSuccess) return e;
    // layer 1
    return layer_wgrad(m, s, m->D1, H, m->X0, F, B, gp.W1, gp.c1);
}

hipError_t adamw_step(foldin_model *m, hipStream_t s, const float *grad) {
    m->step += 1;
    const double t = (double)m->step;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)m->cfg.beta1, t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)m->cfg.beta2, t)));
    hipLaunchKernelGGL(k_adamw, dim3((unsigned)((m->P + 255) / 256)), dim3(256), 0, s, m->theta, m->mom, m->vel,
                       grad, m->P, m->cfg.lr, m->cfg.beta1, m->cfg.beta2, m->cfg.eps, m->cfg.weight_decay, c1, c2);
    return hipGetLastError();
}

// splitmix64 (Steele, Lea and Flood, 2014): the seeded stream that shuffles
// the training rows of each epoch.
uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int64_t foldin_param_count(int32_t n_f, int32_t hidden) {
    if (n_f < 1 || hidden < 1) return 0;
    return param_count(n_f, hidden);
}

size_t foldin_workspace_size(const foldin_cfg *cfg) {
    if (!cfg_ok(cfg)) return 0;
    return foldin_layout(*cfg).total;
}

als_status foldin_create(const foldin_cfg *cfg, const float *params, foldin_model **out) {
    if (!out) return ALS_E_ARG;
    *out = nullptr;
    if (!cfg_ok(cfg) || !params) return ALS_E_ARG;
    FoldinLayout L = foldin_layout(*cfg);
    if (!cfg->workspace || cfg->workspace_bytes < L.total) return ALS_E_NOMEM;
    foldin_model *m = new (std::nothrow) foldin_model();
    if (!m) return ALS_E_NOMEM;
    m->cfg = *cfg;
    m->nf = cfg->n_f;
    m->H = cfg->hidden;
    m->Bmax = cfg->max_batch;
    m->P = param_count(cfg->n_f, cfg->hidden);
    m->stream = reinterpret_cast<hipStream_t>(cfg->stream);
    char *base = reinterpret_cast<char *>(cfg->workspace);
    m->theta = reinterpret_cast<float *>(base + L.theta);
    m->mom = reinterpret_cast<float *>(base + L.mom);
    m->vel = reinterpret_cast<float *>(base + L.vel);
    m->grad = reinterpret_cast<float *>(base + L.grad);
    m->X0 = reinterpret_cast<float *>(base + L.X0);
    m->Z1 = reinterpret_cast<float *>(base + L.Z1);
    m->H1 = reinterpret_cast<float *>(base + L.H1);
    m->Z2 = reinterpret_cast<float *>(base + L.Z2);
    m->H2 = reinterpret_cast<float *>(base + L.H2);
    m->OUT = reinterpret_cast<float *>(base + L.OUT);
    m->D3 = reinterpret_cast<float *>(base + L.D3);
    m->D2 = reinterpret_cast<float *>(base + L.D2);
    m->D1 = reinterpret_cast<float *>(base + L.D1);
    m->part = reinterpret_cast<float *>(base + L.part);
    m->loss_part = reinterpret_cast<double *>(base + L.loss_part);
    m->loss_acc = reinterpret_cast<double *>(base + L.loss_acc);
    m->perm = reinterpret_cast<int32_t *>(base + L.perm);
    hipError_t e = hipMemcpyAsync(m->theta, params, sizeof(float) * m->P, hipMemcpyDeviceToDevice, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->mom, 0, sizeof(float) * m->P, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->vel, 0, sizeof(float) * m->P, m->stream);
    if (e != hipSuccess) {
        delete m;
        return ALS_E_DEVICE;
    }
    *out = m;
    return ALS_OK;
}

als_status foldin_get_params(foldin_model *m, float *params) {
    if (!m) return ALS_E_STATE;
    if (!params) return mfail(m, ALS_E_ARG, "params is NULL");
    MHIP(m, hipMemcpyAsync(params, m->theta, sizeof(float) * m->P, hipMemcpyDeviceToDevice, m->stream));
    return ALS_OK;
}

als_status foldin_set_params(foldin_model *m, const float *params) {
    if (!m) return ALS_E_STATE;
    if (!params) return mfail(m, ALS_E_ARG, "params is NULL");
    MHIP(m, hipMemcpyAsync(m->theta, params, sizeof(float) * m->P, hipMemcpyDeviceToDevice, m->stream));
    MHIP(m, hipMemsetAsync(m->mom, 0, sizeof(float) * m->P, m->stream));
    MHIP(m, hipMemsetAsync(m->vel, 0, sizeof(float) * m->P, m->stream));
    m->step = 0;
    return ALS_OK;
}

als_status foldin_forward(foldin_model *m, const float *M, const int64_t *ptr, const int32_t *items,
                          const float *vals, const int32_t *rows, int64_t n, float *U_out) {
    if (!m) return ALS_E_STATE;
    if (n < 0) return mfail(m, ALS_E_ARG, "negative row count");
    if (n == 0) return ALS_OK;
    if (!M || !ptr || !U_out) return mfail(m, ALS_E_ARG, "NULL pointer");
    for (int64_t b0 = 0; b0 < n; b0 += m->Bmax) {
        const int B = (int)std::min<int64_t>(m->Bmax, n - b0);
        MHIP(m, forward_batch(m, m->stream, M, ptr, items, vals, rows ? rows + b0 : nullptr, rows ? 0 : b0, B,
                              U_out + b0 * m->nf));
    }
    return ALS_OK;
}

als_status foldin_grad(foldin_model *m, const float *M, const int64_t *ptr, const int32_t *items, const float *vals,
                       const int32_t *rows, int64_t n, const float *target, float *grad, float *loss) {
    if (!m) return ALS_E_STATE;
    if (n < 1 || n > m->Bmax) return mfail(m, ALS_E_ARG, "batch must have 1..max_batch rows");
    if (!M || !ptr || !target) return mfail(m, ALS_E_ARG, "NULL pointer");
    MHIP(m, grad_batch(m, m->stream, M, ptr, items, vals, rows, 0, (int)n, target, loss, nullptr));
    if (grad) MHIP(m, hipMemcpyAsync(grad, m->grad, sizeof(float) * m->P, hipMemcpyDeviceToDevice, m->stream));
    return ALS_OK;
}

als_status foldin_adamw(foldin_model *m, const float *grad) {
    if (!m) return ALS_E_STATE;
    MHIP(m, adamw_step(m, m->stream, grad ? grad : m->grad));
    return ALS_OK;
}

als_status foldin_train(foldin_model *m, const float *M, const int64_t *ptr, const int32_t *items,
                        const float *vals, int64_t n_rows, const float *target, int32_t epochs, int32_t batch,
                        uint64_t seed, float *loss_per_epoch) {
    if (!m) return ALS_E_STATE;
    if (n_rows < 1 || n_rows > m->cfg.max_train_rows)
        return mfail(m, ALS_E_ARG, "n_rows must be in 1..max_train_rows");
    if (batch < 1 || batch > m->Bmax) return mfail(m, ALS_E_ARG, "batch must be in 1..max_batch");
    if (epochs < 0) return mfail(m, ALS_E_ARG, "negative epoch count");
    if (!M || !ptr || !target) return mfail(m, ALS_E_ARG, "NULL pointer");
    hipStream_t s = m->stream;
    std::vector<int32_t> perm((size_t)n_rows);
    for (int ep = 0; ep < epochs; ++ep) {
        // Fisher-Yates shuffle of the training rows
        uint64_t state = seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(ep + 1));
        for (int64_t i = 0; i < n_rows; ++i) perm[i] = (int32_t)i;
        for (int64_t i = n_rows - 1; i > 0; --i) {
            const int64_t j = (int64_t)(splitmix64(state) % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        MHIP(m, hipMemcpyAsync(m->perm, perm.data(), sizeof(int32_t) * n_rows, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_zero_d, dim3(1), dim3(64), 0, s, m->loss_acc, 2);
        MHIP(m, hipGetLastError());
        int64_t nb = 0;
        for (int64_t b0 = 0; b0 < n_rows; b0 += batch, ++nb) {
            const int B = (int)std::min<int64_t>(batch, n_rows - b0);
            MHIP(m, grad_batch(m, s, M, ptr, items, vals, m->perm + b0, 0, B, target, nullptr, m->loss_acc));
            MHIP(m, adamw_step(m, s, m->grad));
        }
        double acc = 0.0;
        MHIP(m, hipMemcpyAsync(&acc, m->loss_acc, sizeof(double), hipMemcpyDeviceToHost, s));
        MHIP(m, hipStreamSynchronize(s));  // also keeps perm alive until its copy is done
        if (loss_per_epoch) loss_per_epoch[ep] = (float)(acc / (double)nb);
    }
    return ALS_OK;
}

als_status foldin_answer(als_ctx *q, foldin_model *m, const float *M, double tol, float *U_new, int32_t *path,
                         float *rho, foldin_answer_stats *st) {
    if (!m) return ALS_E_STATE;
    if (!q) return mfail(m, ALS_E_STATE, "query context is NULL");
    if (q->p.n_f != m->nf) return mfail(m, ALS_E_ARG, "query context and model differ in n_f");
    if (!M || !U_new || !path || !rho) return mfail(m, ALS_E_ARG, "NULL pointer");
    if (!(tol >= 0.0)) return mfail(m, ALS_E_ARG, "tol must be >= 0");
    const int64_t n = q->p.n_u;
    hipStream_t s = q->stream;
    for (int64_t b0 = 0; b0 < n; b0 += m->Bmax) {
        const int B = (int)std::min<int64_t>(m->Bmax, n - b0);
        MHIP(m, forward_batch(m, s, M, q->p.row_ptr, q->p.col_idx, q->p.val, nullptr, b0, B, U_new + b0 * m->nf));
    }
    CheckArgs chk{U_new, (float)tol, path, rho};
    als_status rs = enqueue_checked_users(q, M, U_new, chk);
    if (rs != ALS_OK) return mfail(m, rs, std::string("exact fallback: ") + als_last_error(q));
    if (st) {
        unsigned long long h[NSTATS];
        rs = read_stats(q, h);
        if (rs != ALS_OK) return mfail(m, rs, std::string("stats: ") + als_last_error(q));
        st->n_rows = n;
        st->n_exact = (int64_t)h[ST_FOLDIN_EXACT] + (int64_t)h[ST_EMPTY];
        st->n_mlp = n - st->n_exact;
        st->n_empty = (int64_t)h[ST_EMPTY];
        st->n_singular_fallback = (int64_t)h[ST_FALLBACK];
    }
    return ALS_OK;
}

void foldin_destroy(foldin_model *m) { delete m; }

const char *foldin_last_error(const foldin_model *m) { return m ? m->err.c_str() : "model is NULL"; }

}  // extern "C"
