// The learned surrogate: a multilayer perceptron from the retrieval parameters to the
// binned spectrum, trained and evaluated on the matrix cores in BF16 with FP32
// accumulation (v_mfma_f32_16x16x32_bf16), FP32 master weights and Adam.
//
// The paper motivates machine-learning surrogates for retrievals and notes that they
// did not reproduce the posterior exactly (Sec. 1); here the surrogate only screens
// proposals (stage 1 of delayed acceptance) and the exact forward model decides, so the
// posterior is unchanged.
//
// Layer i: z_i = h_i W_i^T + b_i (W_i is [out][in], row-major), h_{i+1} = silu(z_i) for
// hidden layers, the last layer is linear. Backward: dz_L = d loss / d out;
// gW_i = dz_i^T h_i, gb_i = sum_rows dz_i, dz_{i-1} = (dz_i W_i) * silu'(z_{i-1}).
#include <cmath>

#include "bm_internal.h"

namespace bm {

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    // round to nearest even; NaN stays NaN
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// ---- GEMM: C[M][N] = sum_k A(m, k) B(k, n) -------------------------------------------------
// A(m, k) = A[m * lda + k] (trans_a = 0) or A[k * lda + m] (trans_a = 1); B(k, n) =
// B[n * ldb + k] (trans_b = 0: B holds rows of length K, as W[out][in]) or B[k * ldb + n].
// Block tile BM x BN x TK with 4 waves in a 2 x 2 layout, each wave (BM/2) x (BN/2) of
// 16 x 16 MFMA tiles. Operand tiles are double-buffered in LDS: the next tile's global
// loads are in flight while the matrix cores work on the current one. Each thread moves
// groups of 8 consecutive elements of an operand row (one 16-byte load each when the
// layout allows it). The k loop is latency-bound for small products (one load round
// trip per TK slice), so the small tiles take TK = 128; the matrix cores step through a
// slice 32 k at a time, in the same k order for every TK.
constexpr int kPad = 8;

struct GemmArgs {
    int M, N, K;
    const uint16_t* A;
    int lda, trans_a;
    const uint16_t* B;
    int ldb, trans_b;
    int mode;                 // BM_GEMM_* epilogue
    const float* bias;        // [N]
    const float* aux;         // [M][ldaux] pre-activations for silu'
    int ldaux;
    float* out_f32;           // [M][ldo]
    int ldo;
    uint16_t* out_bf16;       // [M][ldob]
    int ldob;
    float beta;               // out_f32 = beta * out_f32 + result (accumulating modes)
    int vec_a, vec_b;         // 16-byte operand loads allowed (alignment and extents)
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 8 elements of one operand for tile rows [r0, r0 + R) x k-slice [k0, k0 + TK): chunk t of
// the tile. Non-transposed: row r = t / (TK / 8), k = 8 (t % (TK / 8)) .. +7 (contiguous in
// memory). Transposed: k = t / (R / 8), rows 8 (t % (R / 8)) .. +7 (contiguous in memory).
// Thread t of the 256 holds chunks t, t + 256, ...
template <int R, int TK>
struct TileChunk {
    static constexpr int kChunks = R * TK / 8;
    static constexpr int kPer = (kChunks + 255) / 256;
    u32x4 v[kPer];
    __device__ __forceinline__ static u32x4 load_one(const uint16_t* __restrict__ X, int ld, int trans, int vec,
                                                    int rows, int K, int r0, int k0, int t) {
        u32x4 out = u32x4{0u, 0u, 0u, 0u};
        if (t >= kChunks) return out;
        uint16_t e[8];
        if (!trans) {
            const int r = r0 + t / (TK / 8), k = k0 + 8 * (t % (TK / 8));
            if (r >= rows) return out;
            const uint16_t* p = X + (size_t)r * ld + k;
            if (vec) {
                if (k < K) out = *reinterpret_cast<const u32x4*>(p);  // K % 8 == 0: all 8 or none
                return out;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) e[i] = (k + i < K) ? p[i] : (uint16_t)0;
        } else {
            const int k = k0 + t / (R / 8), r = r0 + 8 * (t % (R / 8));
            if (k >= K) return out;
            const uint16_t* p = X + (size_t)k * ld + r;
            if (vec) {
                if (r < rows) out = *reinterpret_cast<const u32x4*>(p);  // rows % 8 == 0
                return out;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) e[i] = (r + i < rows) ? p[i] : (uint16_t)0;
        }
        return u32x4{(uint32_t)e[0] | ((uint32_t)e[1] << 16), (uint32_t)e[2] | ((uint32_t)e[3] << 16),
                     (uint32_t)e[4] | ((uint32_t)e[5] << 16), (uint32_t)e[6] | ((uint32_t)e[7] << 16)};
    }
    __device__ __forceinline__ void load(const uint16_t* __restrict__ X, int ld, int trans, int vec, int rows,
                                         int K, int r0, int k0, int t) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) v[u] = load_one(X, ld, trans, vec, rows, K, r0, k0, t + 256 * u);
    }
    // into the LDS tile [R][TK + kPad] (row-major in k)
    __device__ __forceinline__ void store(uint16_t (*S)[TK + kPad], int trans, int t0) const {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int t = t0 + 256 * u;
            if (t >= kChunks) continue;
            if (!trans) {
                *reinterpret_cast<u32x4*>(&S[t / (TK / 8)][8 * (t % (TK / 8))]) = v[u];
            } else {
                const int k = t / (R / 8), r = 8 * (t % (R / 8));
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    S[r + 2 * i][k] = (uint16_t)(v[u][i] & 0xffffu);
                    S[r + 2 * i + 1][k] = (uint16_t)(v[u][i] >> 16);
                }
            }
        }
    }
};

template <int BM, int BN, int TK>
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
    constexpr int WM = BM / 2, WN = BN / 2;          // wave tile
    constexpr int TI = WM / 16, TJ = WN / 16;        // MFMA tiles per wave
    static_assert(TK % 32 == 0, "k slices of whole MFMA steps");
    // slices of 512 or more hold the whole of k (one load round trip, launched only when
    // K <= TK) and need no second buffer
    constexpr int kBuf = TK >= 512 ? 1 : 2;
    __shared__ __align__(16) uint16_t As[kBuf][BM][TK + kPad];
    __shared__ __align__(16) uint16_t Bs[kBuf][BN][TK + kPad];
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
    f32x4 acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nk = (g.K + TK - 1) / TK;
    TileChunk<BM, TK> ca;
    TileChunk<BN, TK> cb;
    ca.load(g.A, g.lda, g.trans_a, g.vec_a, g.M, g.K, m0, 0, tid);
    cb.load(g.B, g.ldb, g.trans_b, g.vec_b, g.N, g.K, n0, 0, tid);
    ca.store(As[0], g.trans_a, tid);
    cb.store(Bs[0], g.trans_b, tid);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & (kBuf - 1);
        if (kBuf == 2 && kt + 1 < nk) {
            ca.load(g.A, g.lda, g.trans_a, g.vec_a, g.M, g.K, m0, (kt + 1) * TK, tid);
            cb.load(g.B, g.ldb, g.trans_b, g.vec_b, g.N, g.K, n0, (kt + 1) * TK, tid);
        }
        // operands: lane holds 8 consecutive k of row (lane % 16); k offset 8 (lane / 16)
#pragma unroll
        for (int kk = 0; kk < TK; kk += 32) {
            const int kq = kk + 8 * (lane >> 4);
            bf16x8 a[TI], b[TJ];
#pragma unroll
            for (int i = 0; i < TI; ++i)
                a[i] = *reinterpret_cast<const bf16x8*>(&As[cur][wm + 16 * i + (lane & 15)][kq]);
#pragma unroll
            for (int j = 0; j < TJ; ++j)
                b[j] = *reinterpret_cast<const bf16x8*>(&Bs[cur][wn + 16 * j + (lane & 15)][kq]);
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (kBuf == 2 && kt + 1 < nk) {
            ca.store(As[cur ^ (kBuf - 1)], g.trans_a, tid);
            cb.store(Bs[cur ^ (kBuf - 1)], g.trans_b, tid);
        }
        __syncthreads();
    }
    // epilogue: lane holds C[4 (lane / 16) + r][lane % 16] of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int n = n0 + wn + 16 * j + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][r];
                switch (g.mode) {
                    case BM_GEMM_STORE:
                        g.out_f32[(size_t)m * g.ldo + n] =
                            (g.beta != 0.f ? g.beta * g.out_f32[(size_t)m * g.ldo + n] : 0.f) + v;
                        break;
                    case BM_GEMM_BIAS_SILU: {
                        const float z = v + g.bias[n];
                        if (g.out_f32) g.out_f32[(size_t)m * g.ldo + n] = z;
                        g.out_bf16[(size_t)m * g.ldob + n] = f2bf(silu(z));
                        break;
                    }
                    case BM_GEMM_BIAS:
                        g.out_f32[(size_t)m * g.ldo + n] = v + g.bias[n];
                        break;
                    case BM_GEMM_SILU_GRAD:
                        g.out_bf16[(size_t)m * g.ldob + n] = f2bf(v * silu_grad(g.aux[(size_t)m * g.ldaux + n]));
                        break;
                }
            }
}

// column sums of a bf16 matrix [M][N] (bias gradients): 64 columns per workgroup, four
// row groups per column summed in a fixed order
__global__ void __launch_bounds__(256) k_colsum_bf16(const uint16_t* __restrict__ x, int M, int N,
                                                     float* __restrict__ out, float beta) {
    __shared__ float part[4][64];
    const int c = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    float s = 0.f;
    if (n < N) {
#pragma unroll 8
        for (int m = grp; m < M; m += 4) s += bf2f(x[(size_t)m * N + n]);
    }
    part[grp][c] = s;
    __syncthreads();
    if (grp == 0 && n < N) {
        const float tot = (part[0][c] + part[1][c]) + (part[2][c] + part[3][c]);
        out[n] = (beta != 0.f ? beta * out[n] : 0.f) + tot;
    }
}

// network input: h0[b][j] = bf16((theta_j - lo_j) / (hi_j - lo_j)), zero padding to dims[0]
__global__ void k_mlp_input(const double* __restrict__ params, int stride, const int32_t* __restrict__ rows, int B,
                            int P, const double* __restrict__ lo, const double* __restrict__ hi, int d0,
                            uint16_t* __restrict__ h0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * d0) return;
    const int b = i / d0, j = i % d0;
    const int64_t r = rows ? rows[b] : b;
    float v = 0.f;
    if (j < P) v = (float)((params[r * stride + j] - lo[j]) / (hi[j] - lo[j]));
    h0[i] = f2bf(v);
}

// mean-squared-error loss and its gradient wrt the (linear) output, as the last layer's dz
__global__ void k_mse_grad(const float* __restrict__ out, const double* __restrict__ target,
                           const int32_t* __restrict__ rows, const double* __restrict__ mean,
                           const double* __restrict__ scale, int B, int N, uint16_t* __restrict__ dz,
                           float* __restrict__ row_loss) {
    __shared__ float part[256];
    const int b = blockIdx.x;
    const int64_t r = rows ? rows[b] : b;
    float s = 0.f;
    const float gscale = 2.0f / ((float)B * (float)N);
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        double t = target[r * N + n];
        if (mean) t = (t - mean[n]) / scale[n];
        const float d = out[(size_t)b * N + n] - (float)t;
        s += d * d;
        dz[(size_t)b * N + n] = f2bf(gscale * d);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) row_loss[b] = part[0];
}

// Adam (Kingma & Ba 2015) on FP32 master weights, refreshing the BF16 copy
__global__ void k_adam(float* __restrict__ w, uint16_t* __restrict__ w16, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (w16) w16[i] = f2bf(wi);
}

__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// surrogate chi^2: the standardised output back to depths, then chi^2 against the data
__global__ void k_surrogate_chi2(const float* __restrict__ out, int B, int N, const double* __restrict__ mean,
                                 const double* __restrict__ scale, const double* __restrict__ data,
                                 const double* __restrict__ err, double* __restrict__ chi2) {
    __shared__ double part[256];
    const int b = blockIdx.x;
    double s = 0.0;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const double pred = mean[n] + scale[n] * (double)out[(size_t)b * N + n];
        const double d = (pred - data[n]) / err[n];
        s += d * d;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) chi2[b] = part[0];
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

static int launch_gemm(GemmArgs a, hipStream_t st) {
    if (a.M < 0 || a.N < 0 || a.K < 0) return BM_ESHAPE;
    if (a.M == 0 || a.N == 0) return BM_OK;
    // 16-byte operand loads: rows of 8-element multiples, aligned base
    a.vec_a = aligned16(a.A) && a.lda % 8 == 0 && (a.trans_a ? a.M % 8 == 0 : a.K % 8 == 0);
    a.vec_b = aligned16(a.B) && a.ldb % 8 == 0 && (a.trans_b ? a.N % 8 == 0 : a.K % 8 == 0);
    // 64 x 64 tiles when they fill the chip, 32 x 32 tiles (4x the workgroups) otherwise
    const long tiles64 = (long)((a.N + 63) / 64) * ((a.M + 63) / 64);
    if (tiles64 >= 256) {
        dim3 grid((a.N + 63) / 64, (a.M + 63) / 64);
        hipLaunchKernelGGL((k_gemm_bf16<64, 64, 32>), grid, dim3(256), 0, st, a);
    } else {
        // small products: few workgroups, so each takes deep k slices (fewer round trips):
        // the whole of k at once up to 512, else 128-deep slices
        dim3 grid((a.N + 31) / 32, (a.M + 31) / 32);
        if (a.K > 128 && a.K <= 512)
            hipLaunchKernelGGL((k_gemm_bf16<32, 32, 512>), grid, dim3(256), 0, st, a);
        else if (a.K > 64)
            hipLaunchKernelGGL((k_gemm_bf16<32, 32, 128>), grid, dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_gemm_bf16<32, 32, 32>), grid, dim3(256), 0, st, a);
    }
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

static int check_mlp(const bm_mlp* n, int B) {
    if (!n || n->n_layers < 1 || n->n_layers > BM_MLP_MAX_LAYERS) return BM_EINVAL;
    if (B < 0 || B > n->max_batch) return BM_ESHAPE;
    for (int i = 0; i <= n->n_layers; ++i)
        if (n->dims[i] < 1) return BM_ESHAPE;
    for (int i = 0; i < n->n_layers; ++i) {
        if (!n->w16[i] || !n->b32[i] || !n->h[i]) return BM_EINVAL;
        if (i < n->n_layers - 1 && !n->z[i]) return BM_EINVAL;
    }
    return BM_OK;
}

}  // namespace bm

using namespace bm;

extern "C" int bm_gemm_bf16(int M, int N, int K, const void* A, int lda, int trans_a, const void* B, int ldb,
                            int trans_b, int mode, const float* bias, const float* aux, int ldaux, float* out_f32,
                            int ldo, void* out_bf16, int ldob, float beta, void* stream) {
    if (!A || !B) return BM_EINVAL;
    if (mode < BM_GEMM_STORE || mode > BM_GEMM_SILU_GRAD) return BM_EINVAL;
    if ((mode == BM_GEMM_STORE || mode == BM_GEMM_BIAS) && !out_f32) return BM_EINVAL;
    if ((mode == BM_GEMM_BIAS_SILU || mode == BM_GEMM_BIAS) && !bias) return BM_EINVAL;
    if ((mode == BM_GEMM_BIAS_SILU || mode == BM_GEMM_SILU_GRAD) && !out_bf16) return BM_EINVAL;
    if (mode == BM_GEMM_SILU_GRAD && !aux) return BM_EINVAL;
    GemmArgs a{M, N, K, (const uint16_t*)A, lda, trans_a, (const uint16_t*)B, ldb, trans_b, mode, bias, aux, ldaux,
               out_f32, ldo, (uint16_t*)out_bf16, ldob, beta};
    return launch_gemm(a, (hipStream_t)stream);
}

extern "C" int bm_mlp_set_input(const bm_mlp* net, const double* params, int param_stride, const int32_t* rows,
                                int B, int P, const double* lo, const double* hi, void* stream) {
    int st = check_mlp(net, B);
    if (st != BM_OK) return st;
    if (!params || !lo || !hi) return BM_EINVAL;
    if (P < 1 || P > net->dims[0] || param_stride < P) return BM_ESHAPE;
    if (B == 0) return BM_OK;
    const int n = B * net->dims[0];
    hipLaunchKernelGGL(k_mlp_input, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, param_stride, rows,
                       B, P, lo, hi, net->dims[0], (uint16_t*)net->h[0]);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

extern "C" int bm_mlp_forward(const bm_mlp* net, int B, float* out, void* stream) {
    int st = check_mlp(net, B);
    if (st != BM_OK) return st;
    if (!out) return BM_EINVAL;
    const int L = net->n_layers;
    for (int i = 0; i < L; ++i) {
        const int K = net->dims[i], N = net->dims[i + 1];
        const bool last = (i == L - 1);
        if (!last && !net->h[i + 1]) return BM_EINVAL;
        GemmArgs a{B, N, K, (const uint16_t*)net->h[i], K, 0, (const uint16_t*)net->w16[i], K, 0,
                   last ? BM_GEMM_BIAS : BM_GEMM_BIAS_SILU, net->b32[i], nullptr, 0,
                   last ? out : net->z[i], N, last ? nullptr : (uint16_t*)net->h[i + 1], N, 0.f};
        st = launch_gemm(a, (hipStream_t)stream);
        if (st != BM_OK) return st;
    }
    return BM_OK;
}

extern "C" int bm_mlp_loss_grad(const bm_mlp* net, int B, const float* out, const double* target,
                                const int32_t* rows, const double* mean, const double* scale, float* row_loss,
                                void* stream) {
    int st = check_mlp(net, B);
    if (st != BM_OK) return st;
    if (!out || !target || !row_loss || !net->dz[0]) return BM_EINVAL;
    if ((mean == nullptr) != (scale == nullptr)) return BM_EINVAL;
    if (B == 0) return BM_OK;
    hipLaunchKernelGGL(k_mse_grad, dim3(B), dim3(256), 0, (hipStream_t)stream, out, target, rows, mean, scale,
                       B, net->dims[net->n_layers], (uint16_t*)net->dz[0], row_loss);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

extern "C" int bm_mlp_backward(const bm_mlp* net, int B, void* stream) {
    int st = check_mlp(net, B);
    if (st != BM_OK) return st;
    const int L = net->n_layers;
    for (int i = 0; i < L; ++i)
        if (!net->gw[i] || !net->gb[i]) return BM_EINVAL;
    if (!net->dz[0] || !net->dz[1]) return BM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int cur = 0;  // dz of layer i lives in dz[cur]
    for (int i = L - 1; i >= 0; --i) {
        const int K = net->dims[i], N = net->dims[i + 1];
        const uint16_t* dz = (const uint16_t*)net->dz[cur];
        // gW_i [N][K] = dz^T [N][B] h_i [B][K]
        GemmArgs gw{N, K, B, dz, N, 1, (const uint16_t*)net->h[i], K, 1, BM_GEMM_STORE, nullptr, nullptr, 0,
                    net->gw[i], K, nullptr, 0, 0.f};
        st = launch_gemm(gw, s);
        if (st != BM_OK) return st;
        hipLaunchKernelGGL(k_colsum_bf16, dim3((N + 63) / 64), dim3(256), 0, s, dz, B, N, net->gb[i], 0.f);
        BM_CHECK_HIP(hipGetLastError());
        if (i > 0) {
            // dz_{i-1} [B][K] = (dz [B][N] W_i [N][K]) * silu'(z_{i-1})
            GemmArgs dx{B, K, N, dz, N, 0, (const uint16_t*)net->w16[i], K, 1, BM_GEMM_SILU_GRAD, nullptr,
                        net->z[i - 1], K, nullptr, 0, (uint16_t*)net->dz[1 - cur], K, 0.f};
            st = launch_gemm(dx, s);
            if (st != BM_OK) return st;
            cur = 1 - cur;
        }
    }
    return BM_OK;
}

extern "C" int bm_adam_step(const bm_mlp* net, float lr, float beta1, float beta2, float eps, int step,
                            void* stream) {
    int st = check_mlp(net, 0);
    if (st != BM_OK) return st;
    if (step < 1) return BM_EINVAL;
    // bias corrections in double: 1 - beta^t cancels badly in float for beta near 1
    const float c1 = (float)(1.0 - std::pow((double)beta1, step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, step));
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < net->n_layers; ++i) {
        if (!net->w32[i] || !net->gw[i] || !net->mw[i] || !net->vw[i] || !net->gb[i] || !net->mb[i] || !net->vb[i])
            return BM_EINVAL;
        const int64_t nw = (int64_t)net->dims[i + 1] * net->dims[i];
        const int64_t nb = net->dims[i + 1];
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, net->w32[i],
                           (uint16_t*)net->w16[i], net->gw[i], net->mw[i], net->vw[i], nw, lr, beta1, beta2, eps, c1,
                           c2);
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, net->b32[i],
                           (uint16_t*)nullptr, net->gb[i], net->mb[i], net->vb[i], nb, lr, beta1, beta2, eps, c1, c2);
        BM_CHECK_HIP(hipGetLastError());
    }
    return BM_OK;
}

extern "C" int bm_mlp_sync_bf16(const bm_mlp* net, void* stream) {
    int st = check_mlp(net, 0);
    if (st != BM_OK) return st;
    for (int i = 0; i < net->n_layers; ++i) {
        if (!net->w32[i]) return BM_EINVAL;
        const int64_t nw = (int64_t)net->dims[i + 1] * net->dims[i];
        hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                           net->w32[i], (uint16_t*)net->w16[i], nw);
        BM_CHECK_HIP(hipGetLastError());
    }
    return BM_OK;
}

extern "C" int bm_surrogate_chi2(const float* out, int B, int N, const double* mean, const double* scale,
                                 const double* data, const double* err, double* chi2, void* stream) {
    if (!out || !mean || !scale || !data || !err || !chi2) return BM_EINVAL;
    if (B < 0 || N < 1) return BM_ESHAPE;
    if (B == 0) return BM_OK;
    hipLaunchKernelGGL(k_surrogate_chi2, dim3(B), dim3(256), 0, (hipStream_t)stream, out, B, N, mean, scale, data,
                       err, chi2);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}
