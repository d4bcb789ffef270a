// Price surrogate: an ensemble of MLPs (n_in -> width x depth SiLU -> 1) trained and run on the
// GPU with BF16 weights/activations and FP32 accumulation (gfx950 v_mfma_f32_16x16x32_bf16),
// FP32 master weights and Adam.
//
// Layer l (1..depth): Z_l = A_{l-1} W_l^T + b_l (FP32), A_l = bf16(SiLU(Z_l)); A_0 = bf16(x)
// with the input padded to a multiple of 32 features. Head: y = A_depth . w_h + b_h (FP32).
// Loss: mean squared error. Backward: dZ_l = bf16(dA_l * SiLU'(Z_l)); dW_l = dZ_l^T A_{l-1},
// db_l = sum_b dZ_l, dA_{l-1} = dZ_l W_l, all with FP32 accumulation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ttfp.h"

namespace {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_grad(float z)
{
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------------------------- GEMM
// C[M x N] = A[M x K] B[N x K]^T, A and B bf16 with K contiguous (leading dimensions lda, ldb).
// A 256-thread workgroup computes a 64 x 64 tile of C; each wave a 32 x 32 quadrant as 2 x 2
// MFMA 16x16x32 tiles. Operand fragments are read straight from global memory: lane l holds
// row (l % 16) and k-block (l / 16) of 8 consecutive k values; the accumulator holds rows
// 4 (l / 16) + j, column l % 16.
// mode 0: C = acc + bias, plus A_out = bf16(SiLU(C)) (forward layer, Z stored in C)
// mode 1: C = acc (plain store)
// mode 2: atomicAdd(C, acc) (split-K over blockIdx.z)
__global__ __launch_bounds__(256) void k_gemm_bt(int M, int N, int K, const bf16 *__restrict__ A, int lda,
                                                 const bf16 *__restrict__ B, int ldb, float *__restrict__ C, int ldc,
                                                 int mode, const float *__restrict__ bias, bf16 *__restrict__ Aout,
                                                 int ldo, int kchunk)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int r16 = lane & 15, kb = lane >> 4;
    int kbeg = 0, kend = K;
    if (mode == 2) {
        kbeg = blockIdx.z * kchunk;
        kend = min(K, kbeg + kchunk);
    }
    f32x4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bool kvec = ((lda % 8) == 0) && ((ldb % 8) == 0);
    for (int k0 = kbeg; k0 < kend; k0 += 32) {
        bf16x8 fa[2], fb[2];
        const int kk = k0 + kb * 8;
        for (int t = 0; t < 2; ++t) {
            const int row = m0 + t * 16 + r16;
            const int col = n0 + t * 16 + r16;
            if (kvec && kk + 8 <= kend && row < M) {
                fa[t] = *reinterpret_cast<const bf16x8 *>(A + (size_t)row * lda + kk);
            } else {
                for (int j = 0; j < 8; ++j)
                    fa[t][j] = (row < M && kk + j < kend) ? A[(size_t)row * lda + kk + j] : (bf16)0.0f;
            }
            if (kvec && kk + 8 <= kend && col < N) {
                fb[t] = *reinterpret_cast<const bf16x8 *>(B + (size_t)col * ldb + kk);
            } else {
                for (int j = 0; j < 8; ++j)
                    fb[t][j] = (col < N && kk + j < kend) ? B[(size_t)col * ldb + kk + j] : (bf16)0.0f;
            }
        }
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int j = 0; j < 4; ++j) {
                const int row = m0 + a * 16 + kb * 4 + j;
                const int col = n0 + b * 16 + r16;
                if (row >= M || col >= N) continue;
                float v = acc[a][b][j];
                if (mode == 0) {
                    v += bias[col];
                    C[(size_t)row * ldc + col] = v;
                    Aout[(size_t)row * ldo + col] = (bf16)silu(v);
                } else if (mode == 1) {
                    C[(size_t)row * ldc + col] = v;
                } else {
                    atomicAdd(&C[(size_t)row * ldc + col], v);
                }
            }
}

// x (FP32, B x n_in) -> A_0 (bf16, B x kin, zero padded) and its transpose (kin x B)
__global__ void k_input(int Bn, int n_in, int kin, const float *x, bf16 *a0, bf16 *a0t)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)Bn * kin) return;
    const int b = (int)(e / kin), k = (int)(e % kin);
    const bf16 v = (bf16)(k < n_in ? x[(size_t)b * n_in + k] : 0.0f);
    a0[e] = v;
    a0t[(size_t)k * Bn + b] = v;
}

// activations transposed (for the weight gradient GEMM)
__global__ void k_transpose_bf16(int R, int Cc, const bf16 *src, bf16 *dst)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)R * Cc) return;
    const int r = (int)(e / Cc), c = (int)(e % Cc);
    dst[(size_t)c * R + r] = src[e];
}

// head: y = A . w + b (one wave per row)
__global__ void k_head_fwd(int Bn, int W, const bf16 *A, const bf16 *w, const float *bh, float *y)
{
    const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= Bn) return;
    float s = 0.f;
    for (int k = lane; k < W; k += 64) s += (float)A[(size_t)b * W + k] * (float)w[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) y[b] = s + bh[0];
}

// loss[0] = sum_b (y_b - t_b)^2, one workgroup
__global__ __launch_bounds__(1024) void k_sumsq(int Bn, const float *y, const float *t, float *loss)
{
    __shared__ float part[16];
    float s = 0.f;
    for (int b = threadIdx.x; b < Bn; b += blockDim.x) {
        const float r = y[b] - t[b];
        s += r * r;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float tot = 0.f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += part[w];
        loss[0] = tot;
    }
}

// out[k] += sum over this block's rows b of X[b, k] (times wgt[b] when given): column sums
// of a row-major B x W matrix, one partial per block of 256 rows
__global__ __launch_bounds__(256) void k_colsum(int Bn, int W, const bf16 *X, const float *wgt, float *out)
{
    const int r0 = blockIdx.x * 256, r1 = min(Bn, r0 + 256);
    for (int k = threadIdx.x; k < W; k += blockDim.x) {
        float s = 0.f;
        for (int b = r0; b < r1; ++b) s += (wgt ? wgt[b] : 1.0f) * (float)X[(size_t)b * W + k];
        atomicAdd(&out[k], s);
    }
}

// head backward: dy = 2 (y - t) / B; dZ = bf16(dy w * SiLU'(Z)) (and its transpose)
__global__ void k_head_bwd(int Bn, int W, const float *y, const float *tgt, const bf16 *w, const float *Z, float *dy_out,
                           bf16 *dZ, bf16 *dZt)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)Bn * W) return;
    const int b = (int)(e / W), k = (int)(e % W);
    const float dy = 2.0f * (y[b] - tgt[b]) / (float)Bn;
    if (k == 0) dy_out[b] = dy;
    const bf16 q = (bf16)(dy * (float)w[k] * silu_grad(Z[e]));
    dZ[e] = q;
    dZt[(size_t)k * Bn + b] = q;
}

// hidden backward: dZ = bf16(dA * SiLU'(Z)) (and its transpose)
__global__ void k_act_bwd(int Bn, int W, const float *dA, const float *Z, bf16 *dZ, bf16 *dZt)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)Bn * W) return;
    const int b = (int)(e / W), k = (int)(e % W);
    const bf16 q = (bf16)(dA[e] * silu_grad(Z[e]));
    dZ[e] = q;
    dZt[(size_t)k * Bn + b] = q;
}

// sum of a vector into out[0] (one workgroup)
__global__ __launch_bounds__(1024) void k_sum(int n, const float *v, float *out)
{
    __shared__ float part[16];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += v[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float tot = 0.f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += part[w];
        out[0] += tot;
    }
}

// Adam on FP32 master weights; refresh the BF16 copies (row-major and transposed)
struct LayerRef {
    int out, in, kin;         // kin: padded input width used by the BF16 copy
    size_t w_off, b_off;      // offsets into the FP32 parameter vector
    size_t bw_off, bt_off;    // offsets into the BF16 weight / transposed buffers
};

__global__ void k_adam(long long n, float *p, const float *g, float *m1, float *m2, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    p[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

__global__ void k_cast_weights(int out, int in, int kin, const float *w, bf16 *bw, bf16 *bt)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= out * kin) return;
    const int o = e / kin, k = e % kin;
    const bf16 v = (bf16)(k < in ? w[(size_t)o * in + k] : 0.0f);
    bw[e] = v;                             // out x kin
    bt[(size_t)k * out + o] = v;           // kin x out
}

// ------------------------------------------------------------------ fused ensemble inference
// All layers of every model of the ensemble for 64 rows of the batch in one workgroup: the
// activations stay in LDS (bf16, ping-pong), wave w computes output columns [64 w, 64 w + 64)
// of a layer as 4 x 4 MFMA 16x16x32 tiles (its slice of W streamed from L2 once per workgroup),
// the head is a per-row dot product, and the models' prices (control variate + scale * y) give
// the ensemble mean, spread (standard deviation) and the gate factor * spread <= gate * |mean|.
constexpr int ENS_ROWS = 64;
constexpr int ENS_MAXW = 256;
struct EnsembleDesc {
    int n_in, kin, width, depth, n_models;
    const bf16 *bw[16];                 // per model: bf16 weights (layers one after another)
    const float *p[16];                 // per model: FP32 parameters (biases, head bias)
    long long bw_off[17], b_off[17];    // per layer
};
__global__ __launch_bounds__(256) void k_mlp_ensemble(EnsembleDesc D, int Bn, const float *x, const float *cv, const float *scale,
                                                      float factor, float gate, float *mean, float *spread, int *ok)
{
    __shared__ bf16 act[2][ENS_ROWS][ENS_MAXW + 8];
    __shared__ float ys[16][ENS_ROWS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r16 = lane & 15, kb = lane >> 4;
    const int row0 = blockIdx.x * ENS_ROWS;
    const int W = D.width;
    for (int m = 0; m < D.n_models; ++m) {
        // input rows, bf16, zero padded to kin features
        for (int e = tid; e < ENS_ROWS * D.kin; e += 256) {
            const int r = e / D.kin, k = e % D.kin;
            const int b = row0 + r;
            act[0][r][k] = (bf16)((b < Bn && k < D.n_in) ? x[(size_t)b * D.n_in + k] : 0.0f);
        }
        __syncthreads();
        int cur = 0;
        for (int l = 0; l < D.depth; ++l) {
            const int K = l == 0 ? D.kin : W;
            const bf16 *Wl = D.bw[m] + D.bw_off[l];                 // W x K row-major
            const float *bl = D.p[m] + D.b_off[l];
            f32x4 acc[4][4];
            for (int a = 0; a < 4; ++a)
                for (int c = 0; c < 4; ++c) acc[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};
            const int c0 = wave * 64;
            for (int k0 = 0; k0 < K; k0 += 32) {
                const int kk = k0 + kb * 8;
                bf16x8 fa[4], fb[4];
                for (int a = 0; a < 4; ++a) fa[a] = *reinterpret_cast<const bf16x8 *>(&act[cur][16 * a + r16][kk]);
                for (int c = 0; c < 4; ++c) {
                    const int col = c0 + 16 * c + r16;
                    if (col < W) fb[c] = *reinterpret_cast<const bf16x8 *>(Wl + (size_t)col * K + kk);
                    else
                        for (int j = 0; j < 8; ++j) fb[c][j] = (bf16)0.0f;
                }
                for (int a = 0; a < 4; ++a)
                    for (int c = 0; c < 4; ++c) acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[c], acc[a][c], 0, 0, 0);
            }
            for (int a = 0; a < 4; ++a)
                for (int c = 0; c < 4; ++c)
                    for (int j = 0; j < 4; ++j) {
                        const int r = 16 * a + 4 * kb + j, col = c0 + 16 * c + r16;
                        if (col < W) act[cur ^ 1][r][col] = (bf16)silu(acc[a][c][j] + bl[col]);
                    }
            __syncthreads();
            cur ^= 1;
        }
        // head: y = A . w_h + b_h, four threads per row
        {
            const bf16 *wh = D.bw[m] + D.bw_off[D.depth];
            const float bh = D.p[m][D.b_off[D.depth]];
            const int r = tid >> 2, part = tid & 3;
            float sacc = 0.f;
            for (int k = part; k < W; k += 4) sacc += (float)act[cur][r][k] * (float)wh[k];
            sacc += __shfl_xor(sacc, 1, 64);
            sacc += __shfl_xor(sacc, 2, 64);
            if (part == 0) ys[m][r] = sacc + bh;
        }
        __syncthreads();
    }
    // ensemble statistics and the gate
    if (tid < ENS_ROWS) {
        const int b = row0 + tid;
        if (b < Bn) {
            const float c = cv[b], sc = scale[b];
            float mu = 0.f;
            for (int m = 0; m < D.n_models; ++m) mu += c + sc * ys[m][tid];
            mu /= (float)D.n_models;
            float var = 0.f;
            for (int m = 0; m < D.n_models; ++m) {
                const float dv = c + sc * ys[m][tid] - mu;
                var += dv * dv;
            }
            const float sd = D.n_models > 1 ? sqrtf(var / (float)(D.n_models - 1)) : 0.f;
            mean[b] = mu;
            spread[b] = sd;
            ok[b] = factor * sd <= gate * fabsf(mu) ? 1 : 0;
        }
    }
}

// Control variate of the call on the maximum: max_j of the single-asset Black-Scholes calls
// (a lower bound of the price). One thread per option; S0 and sigma are B x d row-major.
__global__ void k_bs_max_call(int Bn, int d, const float *S0, const float *sigma, const float *K, const float *T,
                              const float *r, float *out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= Bn) return;
    const double k = K[b], t = T[b], rr = r[b], disc = exp(-rr * t);
    double best = 0.0;
    for (int j = 0; j < d; ++j) {
        const double s = S0[(size_t)b * d + j], v = sigma[(size_t)b * d + j] * sqrt(t);
        const double d1 = (log(s / k) + (rr + 0.5 * sigma[(size_t)b * d + j] * sigma[(size_t)b * d + j]) * t) / v;
        const double c = s * 0.5 * erfc(-d1 * 0.7071067811865476) - k * disc * 0.5 * erfc(-(d1 - v) * 0.7071067811865476);
        best = fmax(best, c);
    }
    out[b] = (float)best;
}

}  // namespace

// =================================================================================== host
struct ttfp_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_in = 0, width = 0, depth = 0, n_models = 0, max_batch = 0, kin = 0;
    long long n_params = 0;
    std::vector<LayerRef> layers;     // depth hidden layers + head
    // per model
    std::vector<float *> P, G, M1, M2;
    std::vector<bf16 *> BW, BT;
    std::vector<long long> step;
    // activations (shared by models)
    bf16 *a0 = nullptr, *a0t = nullptr;
    std::vector<float *> Z;           // depth x (B x width)
    std::vector<bf16 *> Aact, Aactt;  // depth x (B x width) and transposes
    float *dA = nullptr;              // B x width
    float *dy = nullptr;              // B
    bf16 *dZ = nullptr, *dZt = nullptr;
    float *y = nullptr, *loss = nullptr;
    size_t bw_total = 0;
    std::string err;
};

namespace {
#define MCHK(expr)                                                             \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) {                                                \
            m->err = std::string(#expr) + ": " + hipGetErrorString(e_);        \
            return TTFP_EDEVICE;                                               \
        }                                                                      \
    } while (0)

unsigned cdivu(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

int refresh_bf16(ttfp_mlp *m, int model)
{
    for (const LayerRef &L : m->layers) {
        hipLaunchKernelGGL(k_cast_weights, dim3(cdivu((long long)L.out * L.kin, 256)), dim3(256), 0, m->stream, L.out, L.in, L.kin,
                           m->P[model] + L.w_off, m->BW[model] + L.bw_off, m->BT[model] + L.bt_off);
    }
    MCHK(hipGetLastError());
    return TTFP_OK;
}

// forward through the hidden layers and the head; Z / A of every layer kept for backward
int forward(ttfp_mlp *m, int model, int Bn, const float *x, const float *tgt)
{
    hipStream_t st = m->stream;
    hipLaunchKernelGGL(k_input, dim3(cdivu((long long)Bn * m->kin, 256)), dim3(256), 0, st, Bn, m->n_in, m->kin, x, m->a0, m->a0t);
    const bf16 *in = m->a0;
    int ldin = m->kin;
    for (int l = 0; l < m->depth; ++l) {
        const LayerRef &L = m->layers[l];
        dim3 grid(cdivu(L.out, 64), cdivu(Bn, 64), 1);
        hipLaunchKernelGGL(k_gemm_bt, grid, dim3(256), 0, st, Bn, L.out, L.kin, in, ldin, m->BW[model] + L.bw_off, L.kin,
                           m->Z[l], L.out, 0, m->P[model] + L.b_off, m->Aact[l], L.out, 0);
        in = m->Aact[l];
        ldin = L.out;
    }
    const LayerRef &H = m->layers[m->depth];
    hipLaunchKernelGGL(k_head_fwd, dim3(cdivu(Bn, 4)), dim3(256), 0, st, Bn, m->width, in, m->BW[model] + H.bw_off,
                       m->P[model] + H.b_off, m->y);
    if (tgt) hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(1024), 0, st, Bn, m->y, tgt, m->loss);
    MCHK(hipGetLastError());
    return TTFP_OK;
}

// gradient of the mean squared error into G[model]
int backward(ttfp_mlp *m, int model, int Bn, const float *tgt)
{
    hipStream_t st = m->stream;
    float *g = m->G[model];
    MCHK(hipMemsetAsync(g, 0, sizeof(float) * m->n_params, st));
    const LayerRef &H = m->layers[m->depth];
    const int W = m->width, D = m->depth;
    hipLaunchKernelGGL(k_head_bwd, dim3(cdivu((long long)Bn * W, 256)), dim3(256), 0, st, Bn, W, m->y, tgt, m->BW[model] + H.bw_off,
                       m->Z[D - 1], m->dy, m->dZ, m->dZt);
    // head weight and bias gradients, bias gradient of the last hidden layer
    hipLaunchKernelGGL(k_colsum, dim3(cdivu(Bn, 256)), dim3(256), 0, st, Bn, W, m->Aact[D - 1], m->dy, g + H.w_off);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, st, Bn, m->dy, g + H.b_off);
    hipLaunchKernelGGL(k_colsum, dim3(cdivu(Bn, 256)), dim3(256), 0, st, Bn, W, m->dZ, nullptr, g + m->layers[D - 1].b_off);
    for (int l = D - 1; l >= 0; --l) {
        const LayerRef &L = m->layers[l];
        // dW_l = dZ^T A_{l-1}: (out x B) (in x B)^T, split over the batch
        const bf16 *At = (l == 0) ? m->a0t : m->Aactt[l - 1];
        if (l > 0)
            hipLaunchKernelGGL(k_transpose_bf16, dim3(cdivu((long long)Bn * W, 256)), dim3(256), 0, st, Bn, W, m->Aact[l - 1],
                               m->Aactt[l - 1]);
        const int kchunk = 1024;
        dim3 gw(cdivu(L.kin, 64), cdivu(L.out, 64), cdivu(Bn, kchunk));
        // the FP32 weight block is out x in (ldc = in); for the first layer the padded input
        // columns >= in are never stored (N = in)
        hipLaunchKernelGGL(k_gemm_bt, gw, dim3(256), 0, st, L.out, L.in, Bn, m->dZt, Bn, At, Bn, g + L.w_off, L.in, 2,
                           nullptr, nullptr, 0, kchunk);
        if (l > 0) {
            const LayerRef &Lp = m->layers[l - 1];
            // dA_{l-1} = dZ_l W_l : (B x out) (in x out)^T
            dim3 gd(cdivu(L.in, 64), cdivu(Bn, 64), 1);
            hipLaunchKernelGGL(k_gemm_bt, gd, dim3(256), 0, st, Bn, L.in, L.out, m->dZ, L.out, m->BT[model] + L.bt_off, L.out,
                               m->dA, L.in, 1, nullptr, nullptr, 0, 0);
            hipLaunchKernelGGL(k_act_bwd, dim3(cdivu((long long)Bn * W, 256)), dim3(256), 0, st, Bn, W, m->dA, m->Z[l - 1], m->dZ,
                               m->dZt);
            hipLaunchKernelGGL(k_colsum, dim3(cdivu(Bn, 256)), dim3(256), 0, st, Bn, W, m->dZ, nullptr, g + Lp.b_off);
        }
    }
    MCHK(hipGetLastError());
    return TTFP_OK;
}

int check_model(ttfp_mlp *m, int model, int Bn)
{
    if (model < 0 || model >= m->n_models) { m->err = "model out of range"; return TTFP_EINVAL; }
    if (Bn < 1 || Bn > m->max_batch) { m->err = "batch out of range"; return TTFP_EINVAL; }
    return TTFP_OK;
}
}  // namespace

extern "C" {

int ttfp_mlp_create(ttfp_mlp **out, int device, void *stream, int n_in, int width, int depth, int n_models, int max_batch,
                    uint64_t seed)
{
    if (!out) return TTFP_EINVAL;
    *out = nullptr;
    if (n_in < 1 || n_in > 1024 || width < 16 || width > 4096 || (width % 16) || depth < 1 || depth > 16 || n_models < 1 ||
        n_models > 16 || max_batch < 1 || max_batch > (1 << 22))
        return TTFP_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return TTFP_EDEVICE;
    ttfp_mlp *m = new (std::nothrow) ttfp_mlp();
    if (!m) return TTFP_ENOMEM;
    m->device = device;
    m->stream = (hipStream_t)stream;
    m->n_in = n_in;
    m->width = width;
    m->depth = depth;
    m->n_models = n_models;
    m->max_batch = max_batch;
    m->kin = (n_in + 31) / 32 * 32;
    size_t off = 0, boff = 0;
    for (int l = 0; l <= depth; ++l) {
        LayerRef L;
        L.in = l == 0 ? n_in : width;
        L.kin = l == 0 ? m->kin : width;
        L.out = l == depth ? 1 : width;
        L.w_off = off;
        off += (size_t)L.out * L.in;
        L.b_off = off;
        off += L.out;
        L.bw_off = boff;
        L.bt_off = boff;                     // transposed copy lives in BT at the same offset
        boff += (size_t)L.out * L.kin;
        m->layers.push_back(L);
    }
    m->n_params = (long long)off;
    m->bw_total = boff;
    // He-style initialisation from a counter-based generator (host), biases zero
    std::vector<float> init(off, 0.0f);
    const size_t Bsz = (size_t)max_batch;
    hipError_t e = hipSuccess;
    for (int md = 0; md < n_models; ++md) {
        uint64_t s = seed * 0x9E3779B97F4A7C15ull + (uint64_t)md * 0xD1B54A32D192ED03ull + 1;
        auto next = [&s]() {
            s += 0x9E3779B97F4A7C15ull;
            uint64_t z = s;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            return (double)(z >> 11) * (1.0 / 9007199254740992.0);
        };
        for (const LayerRef &L : m->layers) {
            const double sc = std::sqrt(6.0 / L.in);       // uniform(-sc, sc)
            for (size_t i = 0; i < (size_t)L.out * L.in; ++i) init[L.w_off + i] = (float)((2.0 * next() - 1.0) * sc);
            for (int i = 0; i < L.out; ++i) init[L.b_off + i] = 0.0f;
        }
        float *P = nullptr, *G = nullptr, *A1 = nullptr, *A2 = nullptr;
        bf16 *BW = nullptr, *BT = nullptr;
        e = e ? e : hipMalloc(&P, sizeof(float) * off);
        e = e ? e : hipMalloc(&G, sizeof(float) * off);
        e = e ? e : hipMalloc(&A1, sizeof(float) * off);
        e = e ? e : hipMalloc(&A2, sizeof(float) * off);
        e = e ? e : hipMalloc(&BW, sizeof(bf16) * boff);
        e = e ? e : hipMalloc(&BT, sizeof(bf16) * boff);
        e = e ? e : hipMemcpy(P, init.data(), sizeof(float) * off, hipMemcpyHostToDevice);
        e = e ? e : hipMemset(A1, 0, sizeof(float) * off);
        e = e ? e : hipMemset(A2, 0, sizeof(float) * off);
        m->P.push_back(P);
        m->G.push_back(G);
        m->M1.push_back(A1);
        m->M2.push_back(A2);
        m->BW.push_back(BW);
        m->BT.push_back(BT);
        m->step.push_back(0);
    }
    e = e ? e : hipMalloc(&m->a0, sizeof(bf16) * Bsz * m->kin);
    e = e ? e : hipMalloc(&m->a0t, sizeof(bf16) * Bsz * m->kin);
    for (int l = 0; l < depth; ++l) {
        float *z = nullptr;
        bf16 *a = nullptr, *at = nullptr;
        e = e ? e : hipMalloc(&z, sizeof(float) * Bsz * width);
        e = e ? e : hipMalloc(&a, sizeof(bf16) * Bsz * width);
        e = e ? e : hipMalloc(&at, sizeof(bf16) * Bsz * width);
        m->Z.push_back(z);
        m->Aact.push_back(a);
        m->Aactt.push_back(at);
    }
    e = e ? e : hipMalloc(&m->dA, sizeof(float) * Bsz * width);
    e = e ? e : hipMalloc(&m->dy, sizeof(float) * Bsz);
    e = e ? e : hipMalloc(&m->dZ, sizeof(bf16) * Bsz * width);
    e = e ? e : hipMalloc(&m->dZt, sizeof(bf16) * Bsz * width);
    e = e ? e : hipMalloc(&m->y, sizeof(float) * Bsz);
    e = e ? e : hipMalloc(&m->loss, sizeof(float));
    if (e) {
        *out = m;
        ttfp_mlp_destroy(m);
        *out = nullptr;
        return TTFP_ENOMEM;
    }
    for (int md = 0; md < n_models; ++md)
        if (refresh_bf16(m, md)) return TTFP_EDEVICE;
    if (hipStreamSynchronize(m->stream) != hipSuccess) return TTFP_EDEVICE;
    *out = m;
    return TTFP_OK;
}

int ttfp_mlp_destroy(ttfp_mlp *m)
{
    if (!m) return TTFP_EINVAL;
    (void)hipSetDevice(m->device);
    for (auto p : m->P) (void)hipFree(p);
    for (auto p : m->G) (void)hipFree(p);
    for (auto p : m->M1) (void)hipFree(p);
    for (auto p : m->M2) (void)hipFree(p);
    for (auto p : m->BW) (void)hipFree(p);
    for (auto p : m->BT) (void)hipFree(p);
    for (auto p : m->Z) (void)hipFree(p);
    for (auto p : m->Aact) (void)hipFree(p);
    for (auto p : m->Aactt) (void)hipFree(p);
    (void)hipFree(m->a0);
    (void)hipFree(m->a0t);
    (void)hipFree(m->dA);
    (void)hipFree(m->dy);
    (void)hipFree(m->dZ);
    (void)hipFree(m->dZt);
    (void)hipFree(m->y);
    (void)hipFree(m->loss);
    delete m;
    return TTFP_OK;
}

int ttfp_mlp_n_params(const ttfp_mlp *m, int64_t *n)
{
    if (!m || !n) return TTFP_EINVAL;
    *n = m->n_params;
    return TTFP_OK;
}

int ttfp_mlp_get_params(ttfp_mlp *m, int model, float *params)
{
    if (!m || !params || model < 0 || model >= m->n_models) return TTFP_EINVAL;
    MCHK(hipStreamSynchronize(m->stream));
    MCHK(hipMemcpy(params, m->P[model], sizeof(float) * m->n_params, hipMemcpyDeviceToHost));
    return TTFP_OK;
}

int ttfp_mlp_set_params(ttfp_mlp *m, int model, const float *params)
{
    if (!m || !params || model < 0 || model >= m->n_models) return TTFP_EINVAL;
    MCHK(hipStreamSynchronize(m->stream));
    MCHK(hipMemcpy(m->P[model], params, sizeof(float) * m->n_params, hipMemcpyHostToDevice));
    MCHK(hipMemset(m->M1[model], 0, sizeof(float) * m->n_params));
    MCHK(hipMemset(m->M2[model], 0, sizeof(float) * m->n_params));
    m->step[model] = 0;
    return refresh_bf16(m, model);
}

int ttfp_mlp_forward(ttfp_mlp *m, int model, int batch, const float *x_dev, float *y_dev)
{
    if (!m || !x_dev || !y_dev) return TTFP_EINVAL;
    int rc = check_model(m, model, batch);
    if (rc) return rc;
    MCHK(hipSetDevice(m->device));
    rc = forward(m, model, batch, x_dev, nullptr);
    if (rc) return rc;
    MCHK(hipMemcpyAsync(y_dev, m->y, sizeof(float) * batch, hipMemcpyDeviceToDevice, m->stream));
    return TTFP_OK;
}

int ttfp_mlp_grad(ttfp_mlp *m, int model, int batch, const float *x_dev, const float *t_dev, float *grad, float *loss)
{
    if (!m || !x_dev || !t_dev) return TTFP_EINVAL;
    int rc = check_model(m, model, batch);
    if (rc) return rc;
    MCHK(hipSetDevice(m->device));
    rc = forward(m, model, batch, x_dev, t_dev);
    if (!rc) rc = backward(m, model, batch, t_dev);
    if (rc) return rc;
    MCHK(hipStreamSynchronize(m->stream));
    if (grad) MCHK(hipMemcpy(grad, m->G[model], sizeof(float) * m->n_params, hipMemcpyDeviceToHost));
    if (loss) {
        float l = 0.f;
        MCHK(hipMemcpy(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost));
        *loss = l / batch;
    }
    return TTFP_OK;
}

int ttfp_mlp_train_step(ttfp_mlp *m, int model, int batch, const float *x_dev, const float *t_dev, float lr, float *loss)
{
    if (!m || !x_dev || !t_dev || !(lr > 0)) return TTFP_EINVAL;
    int rc = check_model(m, model, batch);
    if (rc) return rc;
    MCHK(hipSetDevice(m->device));
    rc = forward(m, model, batch, x_dev, t_dev);
    if (!rc) rc = backward(m, model, batch, t_dev);
    if (rc) return rc;
    const long long st = ++m->step[model];
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)st), c2 = 1.0f - std::pow(b2, (float)st);
    hipLaunchKernelGGL(k_adam, dim3(cdivu(m->n_params, 256)), dim3(256), 0, m->stream, m->n_params, m->P[model], m->G[model],
                       m->M1[model], m->M2[model], lr, b1, b2, 1e-8f, c1, c2);
    MCHK(hipGetLastError());
    rc = refresh_bf16(m, model);
    if (rc) return rc;
    if (loss) {
        float l = 0.f;
        MCHK(hipMemcpyAsync(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MCHK(hipStreamSynchronize(m->stream));
        *loss = l / batch;
    }
    return TTFP_OK;
}

int ttfp_mlp_predict(ttfp_mlp *m, int batch, const float *x_dev, const float *cv_dev, const float *scale_dev, float factor,
                     float gate, float *mean_dev, float *spread_dev, int32_t *ok_dev)
{
    if (!m || !x_dev || !cv_dev || !scale_dev || !mean_dev || !spread_dev || !ok_dev) return TTFP_EINVAL;
    if (batch < 1) { m->err = "batch out of range"; return TTFP_EINVAL; }
    if (m->width > ENS_MAXW || m->kin > ENS_MAXW || (m->width % 32)) {
        m->err = "the fused ensemble kernel needs width <= 256, a multiple of 32";
        return TTFP_EINVAL;
    }
    MCHK(hipSetDevice(m->device));
    EnsembleDesc D;
    std::memset(&D, 0, sizeof D);
    D.n_in = m->n_in;
    D.kin = m->kin;
    D.width = m->width;
    D.depth = m->depth;
    D.n_models = m->n_models;
    for (int md = 0; md < m->n_models; ++md) {
        D.bw[md] = m->BW[md];
        D.p[md] = m->P[md];
    }
    for (int l = 0; l <= m->depth; ++l) {
        D.bw_off[l] = (long long)m->layers[l].bw_off;
        D.b_off[l] = (long long)m->layers[l].b_off;
    }
    hipLaunchKernelGGL(k_mlp_ensemble, dim3(cdivu(batch, ENS_ROWS)), dim3(256), 0, m->stream, D, batch, x_dev, cv_dev, scale_dev,
                       factor, gate, mean_dev, spread_dev, (int *)ok_dev);
    MCHK(hipGetLastError());
    return TTFP_OK;
}

int ttfp_mlp_control_variate(ttfp_mlp *m, int batch, int d, const float *S0_dev, const float *sigma_dev, const float *K_dev,
                             const float *T_dev, const float *r_dev, float *cv_dev)
{
    if (!m || !S0_dev || !sigma_dev || !K_dev || !T_dev || !r_dev || !cv_dev || batch < 1 || d < 1) return TTFP_EINVAL;
    MCHK(hipSetDevice(m->device));
    hipLaunchKernelGGL(k_bs_max_call, dim3(cdivu(batch, 256)), dim3(256), 0, m->stream, batch, d, S0_dev, sigma_dev, K_dev, T_dev,
                       r_dev, cv_dev);
    MCHK(hipGetLastError());
    return TTFP_OK;
}

const char *ttfp_mlp_last_error(const ttfp_mlp *m) { return m ? m->err.c_str() : "no model"; }

}  // extern "C"
