// Learned surrogate of the batched shock tubes (C ABI in include/lbm.h):
// BF16-MFMA forward/backward kernels with FP32 accumulation, Adam, and the
// admission check / equilibrium lift / merge used for the plain-scheme
// fallback.
//
// Matrix products use v_mfma_f32_32x32x16_bf16 (gfx950).  Operand layout
// (lane l of a wave): A fragment = 8 BF16 of row (l & 31), k = 8 (l >> 5) ..
// +7; B fragment = 8 BF16 of column (l & 31) at the same k; the 16 FP32
// results of lane l sit at column (l & 31), rows 8 (i >> 2) + 4 (l >> 5) +
// (i & 3) for i = 0..15.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <string>

#include "launch.hpp"
#include "lbm.h"
#include "lbm_device.hpp"

namespace lbmx {
namespace sur {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int C = 64, HID = 128, NB = 4, TAPS = 5, FIN = 16, FOUT = 12;
constexpr int PATCH = 4;
constexpr double OUT_SCALE = 0.1;
// Feature normalisation (rho, u, T, gamma): (v - mu) / sd.
__device__ constexpr double kMu[4] = {0.5, 0.0, 1.0, 1.4};
__device__ constexpr double kSd[4] = {0.5, 0.5, 0.5, 0.3};

// FP32 parameter offsets
constexpr int P_WE = 0, P_BE = 1024, P_BLK = 1088, BLK = 16960;
constexpr int B_KC = 0, B_BC = 320, B_W1 = 384, B_B1 = 8576, B_W2 = 8704, B_B2 = 16896;
constexpr int P_WH = P_BLK + NB * BLK, P_BH = P_WH + FOUT * C, NPARAMS = P_BH + FOUT;
static_assert(NPARAMS == LBM_SUR_NPARAMS, "parameter count");
// BF16 copies (element offsets)
constexpr int Q_WE = 0, Q_BLK = 1024, QBLK = 49152;  // per block: W1, W1t, W2, W2t, W2f, W1f
constexpr int Q_W1 = 0, Q_W1T = 8192, Q_W2 = 16384, Q_W2T = 24576, Q_W2F = 32768, Q_W1F = 40960;
constexpr int Q_WHP = Q_BLK + NB * QBLK;   // [32][64], rows >= 12 zero
constexpr int Q_WHTP = Q_WHP + 32 * C;     // [64][16], cols >= 12 zero
constexpr int QTOTAL = Q_WHTP + C * 16;

// Hidden order of the second MLP product in the fused forward kernel: the
// output of the first product (hidden x tokens) leaves lane half h holding,
// within each 16-wide hidden chunk, offsets {4h..4h+3, 8+4h..8+4h+3}; used
// directly as the A operand, its k slot 8h + e therefore means hidden offset
// 4h + e (+4 for e >= 4).
__host__ __device__ constexpr int w2p_hidden(int kk) {
    const int q = kk / 16, s = kk % 16, h = s / 8, e = s % 8;
    return 16 * q + 4 * h + e + (e >= 4 ? 4 : 0);
}
// The fused forward kernel's weight operands in fragment order: fragment f
// is 64 lanes x 8 BF16 = 1 KB contiguous, lane l at 16 l bytes, so that each
// operand load of a wave reads whole cache lines.
//   W1f  fragment 4 h + s (hidden tile h, k step s): lane 32 hl + n holds
//        W1[32 h + n][16 s + 8 hl .. +7]
//   W2f  fragment 2 q + o (hidden chunk q, output tile o): lane 32 hl + n
//        holds W2[32 o + n][w2p_hidden(16 q + 8 hl + e)], e = 0..7

// Round-to-nearest-even FP32 -> BF16 (NaN kept quiet).
__device__ __forceinline__ __bf16 to_bf16(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    uint16_t h;
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) h = (uint16_t)((u >> 16) | 0x40);
    else h = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    return __builtin_bit_cast(__bf16, h);
}
__device__ __forceinline__ float from_bf16(__bf16 b) {
    return __builtin_bit_cast(float, ((uint32_t)__builtin_bit_cast(uint16_t, b)) << 16);
}

__device__ __forceinline__ float gelu(float z) {
    const float k = 0.7978845608028654f;  // sqrt(2/pi)
    return 0.5f * z * (1.0f + tanhf(k * (z + 0.044715f * z * z * z)));
}
__device__ __forceinline__ float gelu_grad(float z) {
    const float k = 0.7978845608028654f;
    const float t = tanhf(k * (z + 0.044715f * z * z * z));
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * k * (1.0f + 3.0f * 0.044715f * z * z);
}

// ---------------------------------------------------------------------------
// GEMM: C[M][N] = A[M][K] Bt[N][K]^T (+ epilogue), A FP32 (rounded to BF16 on
// load) or BF16, Bt BF16.  Workgroup = 4 waves = 128 rows x all N columns;
// K is staged in LDS at once (rows padded by 8 elements).
// ---------------------------------------------------------------------------
enum { EPI_BIAS = 1, EPI_GELU = 2, EPI_RES = 4, EPI_F32 = 8, EPI_BF16 = 16 };

struct GemmArgs {
    int M, nvalid;
    const void *A;
    const __bf16 *Bt;
    const float *bias;   // [nvalid]
    const float *R;      // residual [M][N] FP32
    float *out;          // [M][N] FP32
    __bf16 *out_bf;      // [M][N] BF16
    float *pre;          // [M][N] FP32 pre-activation (GELU)
};

template <int N, int K, bool AF32, int EPI>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    constexpr int KP = K + 8;
    __shared__ __attribute__((aligned(16))) __bf16 As[128 * KP];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[N * KP];
    const int row0 = blockIdx.x * 128;
    for (int e = threadIdx.x; e < 128 * (K / 8); e += 256) {
        const int r = e / (K / 8), k8 = (e % (K / 8)) * 8;
        const int gr = row0 + r;
        bf16x8 v;
        if (gr < g.M) {
            if constexpr (AF32) {
                const float *a = reinterpret_cast<const float *>(g.A) + (size_t)gr * K + k8;
                const float4 p = *reinterpret_cast<const float4 *>(a);
                const float4 q = *reinterpret_cast<const float4 *>(a + 4);
                v[0] = to_bf16(p.x); v[1] = to_bf16(p.y); v[2] = to_bf16(p.z); v[3] = to_bf16(p.w);
                v[4] = to_bf16(q.x); v[5] = to_bf16(q.y); v[6] = to_bf16(q.z); v[7] = to_bf16(q.w);
            } else {
                v = *reinterpret_cast<const bf16x8 *>(reinterpret_cast<const __bf16 *>(g.A) +
                                                      (size_t)gr * K + k8);
            }
        } else {
            for (int j = 0; j < 8; ++j) v[j] = to_bf16(0.0f);
        }
        *reinterpret_cast<bf16x8 *>(&As[r * KP + k8]) = v;
    }
    for (int e = threadIdx.x; e < N * (K / 8); e += 256) {
        const int n = e / (K / 8), k8 = (e % (K / 8)) * 8;
        *reinterpret_cast<bf16x8 *>(&Bs[n * KP + k8]) =
            *reinterpret_cast<const bf16x8 *>(g.Bt + (size_t)n * K + k8);
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    f32x16 acc[N / 32];
#pragma unroll
    for (int t = 0; t < N / 32; ++t)
        for (int i = 0; i < 16; ++i) acc[t][i] = 0.0f;
#pragma unroll
    for (int kk = 0; kk < K; kk += 16) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&As[(w * 32 + (l & 31)) * KP + kk + (l >> 5) * 8]);
#pragma unroll
        for (int t = 0; t < N / 32; ++t) {
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&Bs[(t * 32 + (l & 31)) * KP + kk + (l >> 5) * 8]);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < N / 32; ++t) {
        const int col = t * 32 + (l & 31);
        const float bias = ((EPI & EPI_BIAS) && col < g.nvalid) ? g.bias[col] : 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int row = row0 + w * 32 + 8 * (i >> 2) + 4 * (l >> 5) + (i & 3);
            if (row >= g.M) continue;
            const size_t o = (size_t)row * N + col;
            float v = acc[t][i] + bias;
            if constexpr (EPI & EPI_GELU) {
                g.pre[o] = v;
                v = gelu(v);
            }
            if constexpr (EPI & EPI_RES) v += g.R[o];
            if constexpr (EPI & EPI_F32) g.out[o] = v;
            if constexpr (EPI & EPI_BF16) g.out_bf[o] = to_bf16(v);
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient: G[n][k] = sum_m A[m][n] B[m][k] over a 128-row chunk per
// workgroup (partials [chunk][Nv][Kv]); optional bias gradient partial
// sum_m A[m][n] ([chunk][Nv]).  A, B FP32 (rounded to BF16) or BF16 with row
// lengths NA, KB; N, K are the padded MFMA sizes (multiples of 32).
// ---------------------------------------------------------------------------
struct WgArgs {
    int M, Nv, Kv;
    const void *A;
    const void *B;
    float *part;   // [gridDim.x][Nv][Kv]
    float *bpart;  // [gridDim.x][Nv] or NULL
};

template <int N, int K, int NA, int KB, bool AF32, bool BF32>
__global__ void __launch_bounds__(256) k_wgrad(WgArgs g) {
    constexpr int MP = 128 + 8;
    __shared__ __attribute__((aligned(16))) __bf16 At[N * MP];
    __shared__ __attribute__((aligned(16))) __bf16 Bt[K * MP];
    const int m0 = blockIdx.x * 128;
    for (int e = threadIdx.x; e < N * 128; e += 256) {
        const int m = e & 127, n = e >> 7;
        __bf16 v = to_bf16(0.0f);
        if (n < NA && m0 + m < g.M) {
            if constexpr (AF32) v = to_bf16(reinterpret_cast<const float *>(g.A)[(size_t)(m0 + m) * NA + n]);
            else v = reinterpret_cast<const __bf16 *>(g.A)[(size_t)(m0 + m) * NA + n];
        }
        At[n * MP + m] = v;
    }
    for (int e = threadIdx.x; e < K * 128; e += 256) {
        const int m = e & 127, k = e >> 7;
        __bf16 v = to_bf16(0.0f);
        if (k < KB && m0 + m < g.M) {
            if constexpr (BF32) v = to_bf16(reinterpret_cast<const float *>(g.B)[(size_t)(m0 + m) * KB + k]);
            else v = reinterpret_cast<const __bf16 *>(g.B)[(size_t)(m0 + m) * KB + k];
        }
        Bt[k * MP + m] = v;
    }
    __syncthreads();
    if (g.bpart) {
        for (int n = threadIdx.x; n < g.Nv; n += 256) {
            float s = 0.0f;
            for (int m = 0; m < 128; ++m) s += from_bf16(At[n * MP + m]);
            g.bpart[(size_t)blockIdx.x * g.Nv + n] = s;
        }
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    constexpr int TN = N / 32, TK = K / 32, TT = TN * TK;
    for (int t = w; t < TT; t += 4) {
        const int tn = t / TK, tk = t % TK;
        f32x16 acc;
        for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
#pragma unroll
        for (int mm = 0; mm < 128; mm += 16) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&At[(tn * 32 + (l & 31)) * MP + mm + (l >> 5) * 8]);
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&Bt[(tk * 32 + (l & 31)) * MP + mm + (l >> 5) * 8]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        const int k = tk * 32 + (l & 31);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int n = tn * 32 + 8 * (i >> 2) + 4 * (l >> 5) + (i & 3);
            if (n < g.Nv && k < g.Kv) g.part[((size_t)blockIdx.x * g.Nv + n) * g.Kv + k] = acc[i];
        }
    }
}

// out[j] (= or +=) sum_c part[c][j] in a fixed order: thread group k of a
// workgroup sums the chunks c = k (mod 16) in ascending order, then the 16
// group sums are added in group order.  A workgroup covers 64 outputs.
constexpr int RED_J = 64, RED_K = 16;
__global__ void __launch_bounds__(RED_J * RED_K) k_reduce_parts(const float *part, int nch, int len, float *out,
                                                              int accumulate) {
    __shared__ float red[RED_K][RED_J];
    const int jl = threadIdx.x % RED_J, k = threadIdx.x / RED_J;
    const int j = blockIdx.x * RED_J + jl;
    float s = 0.0f;
    if (j < len) {
        int c = k;
        for (; c + 3 * RED_K < nch; c += 4 * RED_K) {  // four loads in flight, same order
            const float v0 = part[(size_t)c * len + j], v1 = part[(size_t)(c + RED_K) * len + j];
            const float v2 = part[(size_t)(c + 2 * RED_K) * len + j], v3 = part[(size_t)(c + 3 * RED_K) * len + j];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; c < nch; c += RED_K) s += part[(size_t)c * len + j];
    }
    red[k][jl] = s;
    __syncthreads();
    if (k == 0 && j < len) {
        float t = red[0][jl];
        for (int q = 1; q < RED_K; ++q) t += red[q][jl];
        out[j] = accumulate ? out[j] + t : t;
    }
}

// ---------------------------------------------------------------------------
// Tokens, convolution, head output, loss, GELU backward
// ---------------------------------------------------------------------------
struct Shape {
    int B, L, T, M;  // tubes, nodes per tube, tokens per tube, tokens
};

// X[b*T + t][p*4 + c] = bf16((field_c(b, 4t+p) - mu_c) / sd_c); c = 3 is gamma_b.
__global__ void __launch_bounds__(256) k_patchify(Shape s, const double *x, const double *gamma,
                                                  __bf16 *X) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= s.M * FIN) return;
    const int tok = e / FIN, f = e % FIN, p = f / 4, c = f % 4;
    const int b = tok / s.T, t = tok % s.T;
    const size_t node = (size_t)b * s.L + t * PATCH + p;
    const double v = c < 3 ? x[(size_t)c * s.B * s.L + node] : gamma[b];
    X[e] = to_bf16((float)((v - kMu[c]) / kSd[c]));
}

// Hc = H + bc + sum_k kc[c][k] H[t+k-2] (zero padding at tube ends).
__global__ void __launch_bounds__(256) k_conv_fwd(Shape s, const float *H, const float *kc,
                                                  const float *bc, float *Hc) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= s.M * C) return;
    const int tok = e / C, c = e % C, t = tok % s.T;
    float v = H[e] + bc[c];
#pragma unroll
    for (int k = 0; k < TAPS; ++k) {
        const int tt = t + k - 2;
        if (tt >= 0 && tt < s.T) v += kc[c * TAPS + k] * H[(size_t)(tok + k - 2) * C + c];
    }
    Hc[e] = v;
}

// dH = dHc + sum_k kc[c][k] dHc[t-k+2]; partials of dkc and dbc per 64-row
// workgroup: part[wg][c][0..4] taps, [5] bias.
__global__ void __launch_bounds__(256) k_conv_bwd(Shape s, const float *dHc, const float *H,
                                                  const float *kc, float *dH, float *part) {
    __shared__ float red[4][C][6];
    const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int r0 = blockIdx.x * 64 + q * 16;
    float acc[6] = {0, 0, 0, 0, 0, 0};
    for (int r = r0; r < r0 + 16 && r < s.M; ++r) {
        const int t = r % s.T;
        const float d = dHc[(size_t)r * C + c];
        float v = d;
#pragma unroll
        for (int k = 0; k < TAPS; ++k) {
            const int tt = t - k + 2;
            if (tt >= 0 && tt < s.T) v += kc[c * TAPS + k] * dHc[(size_t)(r - k + 2) * C + c];
            const int th = t + k - 2;
            if (th >= 0 && th < s.T) acc[k] += d * H[(size_t)(r + k - 2) * C + c];
        }
        acc[5] += d;
        dH[(size_t)r * C + c] = v;
    }
    for (int k = 0; k < 6; ++k) red[q][c][k] = acc[k];
    __syncthreads();
    if (q == 0)
        for (int k = 0; k < 6; ++k)
            part[((size_t)blockIdx.x * C + c) * 6 + k] = red[0][c][k] + red[1][c][k] + red[2][c][k] + red[3][c][k];
}

// y_c(node 4t+p) = x_c(node) + 0.1 Y[tok][p*3 + c]
__global__ void __launch_bounds__(256) k_head_out(Shape s, const double *x, const float *Y, double *y) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= 3 * s.B * s.L) return;
    const int c = e / (s.B * s.L), node = e % (s.B * s.L);
    const int b = node / s.L, l = node % s.L, t = l / PATCH, p = l % PATCH;
    y[e] = x[e] + OUT_SCALE * (double)Y[(size_t)(b * s.T + t) * 32 + p * 3 + c];
}

// dY = 2 (Y - (target - x)/0.1) / (M*12) as BF16 [M][16] (cols >= 12 zero);
// loss partial per workgroup.
__global__ void __launch_bounds__(256) k_loss(Shape s, const double *x, const double *target,
                                              const float *Y, __bf16 *dY, float *lpart) {
    __shared__ float red[256];
    const int e = blockIdx.x * 256 + threadIdx.x;
    float sq = 0.0f;
    if (e < s.M * 16) {
        const int tok = e / 16, j = e % 16;
        float d = 0.0f;
        if (j < FOUT) {
            const int p = j / 3, c = j % 3, b = tok / s.T, t = tok % s.T;
            const size_t idx = (size_t)c * s.B * s.L + (size_t)b * s.L + t * PATCH + p;
            const float tn = (float)((target[idx] - x[idx]) / OUT_SCALE);
            const float diff = Y[(size_t)tok * 32 + j] - tn;
            sq = diff * diff;
            d = 2.0f * diff / ((float)s.M * FOUT);
        }
        dY[e] = to_bf16(d);
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_loss_final(const float *lpart, int n, int count, float *loss) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += lpart[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (float)count;
}

// [c][6] partial sums -> kc[c][5], bc[c] gradients
__global__ void __launch_bounds__(64) k_conv_scatter(const float *src, float *kcg, float *bcg) {
    const int c = threadIdx.x;
    for (int t = 0; t < TAPS; ++t) kcg[c * TAPS + t] = src[c * 6 + t];
    bcg[c] = src[c * 6 + 5];
}

// dZ1 = bf16(dA1 * gelu'(Z1))
__global__ void __launch_bounds__(256) k_gelu_bwd(int n, const float *dA1, const float *Z1, __bf16 *dZ1) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < n) dZ1[e] = to_bf16(dA1[e] * gelu_grad(Z1[e]));
}

// ---------------------------------------------------------------------------
// Parameters: BF16 copies (with transposes and zero padding), Adam
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_pack(const float *P, __bf16 *Q) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= QTOTAL) return;
    float v = 0.0f;
    if (e < Q_BLK) {
        v = P[P_WE + e];
    } else if (e < Q_WHP) {
        const int b = (e - Q_BLK) / QBLK, r = (e - Q_BLK) % QBLK;
        const float *blk = P + P_BLK + b * BLK;
        if (r < Q_W1T) v = blk[B_W1 + r];                                        // W1 [128][64]
        else if (r < Q_W2) { const int i = r - Q_W1T, k = i / HID, n = i % HID;  // W1t [64][128]
            v = blk[B_W1 + n * C + k]; }
        else if (r < Q_W2T) v = blk[B_W2 + (r - Q_W2)];                          // W2 [64][128]
        else if (r < Q_W2F) { const int i = r - Q_W2T, k = i / C, n = i % C;     // W2t [128][64]
            v = blk[B_W2 + n * HID + k]; }
        else {                                                                   // W2f, W1f
            const bool w1 = r >= Q_W1F;
            const int i = r - (w1 ? Q_W1F : Q_W2F), f = i / 512, ln = (i / 8) % 64, e = i % 8;
            const int n = ln % 32, hl = ln / 32;
            if (w1) v = blk[B_W1 + (32 * (f / 4) + n) * C + 16 * (f % 4) + 8 * hl + e];
            else v = blk[B_W2 + (32 * (f % 2) + n) * HID + w2p_hidden(16 * (f / 2) + 8 * hl + e)];
        }
    } else if (e < Q_WHTP) {
        const int i = e - Q_WHP, n = i / C, k = i % C;                           // Whp [32][64]
        v = n < FOUT ? P[P_WH + n * C + k] : 0.0f;
    } else {
        const int i = e - Q_WHTP, k = i / 16, n = i % 16;                        // Whtp [64][16]
        v = n < FOUT ? P[P_WH + n * C + k] : 0.0f;
    }
    Q[e] = to_bf16(v);
}

__global__ void __launch_bounds__(256) k_adam(int n, float *p, float *m, float *v, const float *gr,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float g = gr[e];
    const float mm = b1 * m[e] + (1.0f - b1) * g;
    const float vv = b2 * v[e] + (1.0f - b2) * g * g;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// ---------------------------------------------------------------------------
// Fused inference: one workgroup (4 waves) carries a tile of 128 consecutive
// tokens of one tube through the embedding, the four blocks and the head,
// with the residual stream in LDS (FP32, 35 KB).  Each block's depthwise
// convolution needs two tokens on each side, so the tile carries 8 halo
// tokens per side and writes the middle 112.
// Wave w owns rows 32w..32w+31.  The first MLP product is formed transposed,
// Z1^T = W1 Hc^T, one 32-wide hidden tile at a time, so that each lane's
// accumulators (one token, 16 hidden units) become, after bias, GELU and
// BF16 rounding, the A operand of the second product in registers (hidden
// order as in W2f); at most 168 registers per lane keep three waves on each
// SIMD.  Rounding points are those of the layer-wise kernels: the inputs,
// Hc, GELU(Z1) and H4.
// ---------------------------------------------------------------------------
constexpr int FNW = 4;                  // waves per workgroup, 32 token rows each (6: 131 vs 94 us)
constexpr int FR = 32 * FNW;            // token rows per tile
constexpr int FHALO = 2 * NB;           // halo rows per side
constexpr int FOUTR = FR - 2 * FHALO;   // output rows per tile
constexpr int HS = C + 4;               // FP32 row stride in LDS

struct FwdArgs {
    int B, L, T, ntile;
    const double *x, *gamma;
    const int32_t *active;  // NULL, or [B]: tubes with active[b] == 0 are skipped
    const float *P;
    const __bf16 *Q;
    double *y;
};

// GELU (tanh form) as z / (1 + exp(-2a)), a = sqrt(2/pi) (z + 0.044715 z^3),
// which equals 0.5 z (1 + tanh a); hardware exp2 and reciprocal.
__device__ __forceinline__ float gelu_fast(float z) {
    constexpr float c0 = -2.0f * 0.7978845608028654f * 1.4426950408889634f;  // -2 sqrt(2/pi) log2(e)
    constexpr float c1 = c0 * 0.044715f;
    const float e = __builtin_amdgcn_exp2f(z * fmaf(c1, z * z, c0));
    return z * __builtin_amdgcn_rcpf(1.0f + e);
}

__device__ __forceinline__ bf16x8 ld_frag(const __bf16 *p) {
    return *reinterpret_cast<const bf16x8 *>(p);
}

// Eight BF16 of the FP32 row p[0..7] (an MFMA operand fragment).
__device__ __forceinline__ bf16x8 frag_from_f32(const float *p) {
    const float4 u = *reinterpret_cast<const float4 *>(p);
    const float4 v = *reinterpret_cast<const float4 *>(p + 4);
    bf16x8 f;
    f[0] = (__bf16)u.x; f[1] = (__bf16)u.y; f[2] = (__bf16)u.z; f[3] = (__bf16)u.w;
    f[4] = (__bf16)v.x; f[5] = (__bf16)v.y; f[6] = (__bf16)v.z; f[7] = (__bf16)v.w;
    return f;
}

__global__ void __launch_bounds__(64 * FNW, 3) k_fwd_fused(FwdArgs a) {
    // Rows -2, -1, FR and FR + 1 stay zero: the convolution window of the
    // edge rows reads them unconditionally.
    __shared__ __attribute__((aligned(16))) float Hs[(FR + 4) * HS];
    float *const Hf = Hs + 2 * HS;
    // Copies of each wave's first two and last two rows, the only rows its
    // neighbours' convolution windows read, double-buffered by block parity:
    // a wave may then overwrite its own rows without waiting for the
    // neighbours' reads.
    __shared__ __attribute__((aligned(16))) float Hh[2][FNW][4][HS];
    for (int e = threadIdx.x; e < 4 * HS; e += 64 * FNW) Hs[e < 2 * HS ? e : (FR + 2) * HS + e - 2 * HS] = 0.0f;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, n32 = l & 31, hl = l >> 5;
    const int b = blockIdx.x / a.ntile, tile = blockIdx.x % a.ntile;
    if (a.active && !a.active[b]) return;  // workgroup-uniform
    // First MLP biases of every block, read from LDS when each hidden tile's
    // accumulators start (a global load there would stall the tile's MFMAs).
    __shared__ __attribute__((aligned(16))) float B1s[NB * HID];
    for (int e = threadIdx.x; e < NB * HID; e += 64 * FNW) B1s[e] = a.P[P_BLK + (e / HID) * BLK + B_B1 + e % HID];
    const int t0 = tile * FOUTR - FHALO;  // token of row 0
    const int r0 = 32 * w;
    const size_t BL = (size_t)a.B * a.L;
    auto in_tube = [&](int r) { return t0 + r >= 0 && t0 + r < a.T; };
    const bool full = t0 >= 0 && t0 + FR <= a.T;  // every row of the tile inside the tube
    // Row r0 + 8 (i >> 2) + 4 hl + (i & 3) of an accumulator element i is a
    // boundary row for i = 0, 1 (hl = 0: rows 0, 1) and i = 14, 15 (hl = 1:
    // rows 30, 31); keep its copy in slot 0..3.
    auto keep_edge = [&](int par, int i, int ch, float v) {
        if (i < 2 && hl == 0) Hh[par][w][i][ch] = v;
        if (i >= 14 && hl == 1) Hh[par][w][i - 12][ch] = v;
    };

    // Embedding H0 = X We^T + be; rows outside the tube are zero (padding).
    {
        bf16x8 xa;
        const int t = t0 + r0 + n32;
        const bool in = t >= 0 && t < a.T;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int p = 2 * hl + e / 4, c = e % 4;
            double v = 0.0;
            if (in) v = c < 3 ? a.x[(size_t)c * BL + (size_t)b * a.L + 4 * t + p] : a.gamma[b];
            xa[e] = (__bf16)(float)((v - kMu[c]) / kSd[c]);
        }
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const int ch = 32 * ct + n32;
            f32x16 acc;
            for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa, ld_frag(a.Q + Q_WE + ch * FIN + 8 * hl), acc, 0, 0, 0);
            const float be = a.P[P_BE + ch];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int r = r0 + 8 * (i >> 2) + 4 * hl + (i & 3);
                const float v = in_tube(r) ? acc[i] + be : 0.0f;
                Hf[r * HS + ch] = v;
                keep_edge(0, i, ch, v);
            }
        }
    }

    // Weight fragments of the next hidden tile: those of block 0's first
    // tile are issued here, every later tile's as soon as the products of
    // the one before have read the registers (for a block's first tile, at
    // the end of the previous block), so their latency overlaps other work.
    bf16x8 w1[4], w2[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) w1[s] = ld_frag(a.Q + Q_BLK + Q_W1F + s * 512 + 8 * l);
#pragma unroll
    for (int f = 0; f < 4; ++f) w2[f] = ld_frag(a.Q + Q_BLK + Q_W2F + f * 512 + 8 * l);
    for (int k = 0; k < NB; ++k) {
        const float *blk = a.P + P_BLK + k * BLK;
        const __bf16 *qb = a.Q + Q_BLK + k * QBLK;
        // the block's convolution taps and second bias, loaded before the
        // barrier so that the wait there hides their latency
        const int c = l;
        float kc[TAPS];
#pragma unroll
        for (int q = 0; q < TAPS; ++q) kc[q] = blk[B_KC + c * TAPS + q];
        const float bc = blk[B_BC + c];
        float b2[2];
#pragma unroll
        for (int ot = 0; ot < 2; ++ot) b2[ot] = blk[B_B2 + 32 * ot + n32];
        __syncthreads();  // H of every row and its edge copies written
        const int par = k & 1;
        // Depthwise convolution: lane = channel, the wave's 32 rows.
        float hc[32];
        {
            const float kc2 = kc[2] + 1.0f;  // the residual folded into the centre tap
            float win[36];
            // rows r0-2, r0-1 and r0+32, r0+33 from the neighbours' edge
            // copies (the zero rows at the tile's ends)
            const float *lo = w == 0 ? Hf - 2 * HS : &Hh[par][w - 1][2][0];
            const float *hi = w == FNW - 1 ? Hf + FR * HS : &Hh[par][w + 1][0][0];
            win[0] = lo[c];
            win[1] = lo[HS + c];
#pragma unroll
            for (int m = 2; m < 34; ++m) win[m] = Hf[(r0 + m - 2) * HS + c];
            win[34] = hi[c];
            win[35] = hi[HS + c];
#pragma unroll
            for (int m = 0; m < 32; ++m) {
                float v = fmaf(kc2, win[m + 2], bc);
#pragma unroll
                for (int q = 0; q < TAPS; ++q)
                    if (q != 2) v = fmaf(kc[q], win[m + q], v);
                hc[m] = v;
            }
        }
        // no other wave reads these rows in this block (edge copies above)
#pragma unroll
        for (int m = 0; m < 32; ++m) Hf[(r0 + m) * HS + l] = hc[m];
        // MLP on the wave's rows.  B operand of Z1^T: token n32, channels
        // 16 s + 8 hl .. +7, rounded from the rows the wave just wrote.
        bf16x8 hb[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) hb[s] = frag_from_f32(&Hf[(r0 + n32) * HS + 16 * s + 8 * hl]);
        f32x16 acc2[2];
#pragma unroll
        for (int ot = 0; ot < 2; ++ot)
            for (int i = 0; i < 16; ++i) acc2[ot][i] = b2[ot];
#pragma unroll
        for (int h = 0; h < 4; ++h) {  // 32-wide hidden tiles
            f32x16 acc1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 bv = *reinterpret_cast<const float4 *>(&B1s[k * HID + 32 * h + 8 * q + 4 * hl]);
                acc1[4 * q] = bv.x;
                acc1[4 * q + 1] = bv.y;
                acc1[4 * q + 2] = bv.z;
                acc1[4 * q + 3] = bv.w;
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1[s], hb[s], acc1, 0, 0, 0);
            // next tile: (k, h + 1), or block k + 1's first
            const __bf16 *qn = h < 3 ? qb + (4 * (h + 1)) * 512 : qb + QBLK;
            if (h < 3 || k + 1 < NB) {
#pragma unroll
                for (int s = 0; s < 4; ++s) w1[s] = ld_frag(qn + Q_W1F + s * 512 + 8 * l);
            }
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {  // 16-wide hidden chunk 2 h + cc
                bf16x8 af;
#pragma unroll
                for (int e = 0; e < 8; ++e) af[e] = (__bf16)gelu_fast(acc1[8 * cc + e]);
#pragma unroll
                for (int ot = 0; ot < 2; ++ot)
                    acc2[ot] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, w2[2 * cc + ot], acc2[ot], 0, 0, 0);
            }
            if (h < 3 || k + 1 < NB) {
#pragma unroll
                for (int f = 0; f < 4; ++f) w2[f] = ld_frag(qn + Q_W2F + f * 512 + 8 * l);
            }
        }
        // H' = Hc + (b2 + A1 W2^T) on the wave's rows (zero outside the tube).
#pragma unroll
        for (int ot = 0; ot < 2; ++ot) {
            const int ch = 32 * ot + n32;
            float hv[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) hv[i] = Hf[(r0 + 8 * (i >> 2) + 4 * hl + (i & 3)) * HS + ch];
            if (full) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const float v = hv[i] + acc2[ot][i];
                    Hf[(r0 + 8 * (i >> 2) + 4 * hl + (i & 3)) * HS + ch] = v;
                    keep_edge(par ^ 1, i, ch, v);
                }
            } else {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int r = r0 + 8 * (i >> 2) + 4 * hl + (i & 3);
                    const float v = in_tube(r) ? hv[i] + acc2[ot][i] : 0.0f;
                    Hf[r * HS + ch] = v;
                    keep_edge(par ^ 1, i, ch, v);
                }
            }
        }
    }

    // Head: Y = bf16(H4) Wh^T + bh on the wave's rows; y = x + 0.1 Y.
    f32x16 acc;
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const bf16x8 ha = frag_from_f32(&Hf[(r0 + n32) * HS + 16 * s + 8 * hl]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ha, ld_frag(a.Q + Q_WHP + n32 * C + 16 * s + 8 * hl), acc, 0,
                                                      0, 0);
    }
    if (n32 < FOUT) {
        const int p = n32 / 3, c = n32 % 3;
        const float bh = a.P[P_BH + n32];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = r0 + 8 * (i >> 2) + 4 * hl + (i & 3);
            if (r < FHALO || r >= FR - FHALO || !in_tube(r)) continue;
            const size_t idx = (size_t)c * BL + (size_t)b * a.L + 4 * (t0 + r) + p;
            a.y[idx] = a.x[idx] + OUT_SCALE * (double)(acc[i] + bh);
        }
    }
}

// ---------------------------------------------------------------------------
// Admission check, lift, merge
// ---------------------------------------------------------------------------
struct CheckArgs {
    int B, L;
    const double *x, *y, *gamma;
    double tol_m, tol_p, tol_e;
    double max_mach;  // bound on |u| / sqrt(T) of y (0: none)
    int32_t *accept;
};

// One workgroup of kChkT threads per tube: FP64 totals of x and y in a
// fixed order.
constexpr int kChkT = 1024;
__global__ void __launch_bounds__(kChkT) k_check(CheckArgs a) {
    __shared__ double red[kChkT][7];
    __shared__ int bad_s;
    const int b = blockIdx.x;
    const double n = 2.0 / (a.gamma[b] - 1.0) - 1.0;
    const size_t BL = (size_t)a.B * a.L;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};  // Mx, Px, Ex, My, Py, Ey, Tmax
    int bad = 0;
    for (int l = threadIdx.x; l < a.L; l += kChkT) {
        const size_t i = (size_t)b * a.L + l;
        const double rx = a.x[i], ux = a.x[BL + i], Tx = a.x[2 * BL + i];
        const double ry = a.y[i], uy = a.y[BL + i], Ty = a.y[2 * BL + i];
        acc[0] += rx;
        acc[1] += rx * ux;
        acc[2] += rx * (0.5 * ux * ux + 0.5 * (1.0 + n) * Tx);
        acc[3] += ry;
        acc[4] += ry * uy;
        acc[5] += ry * (0.5 * uy * uy + 0.5 * (1.0 + n) * Ty);
        acc[6] = fmax(acc[6], Tx);
        if (!__builtin_isfinite(ry) || !__builtin_isfinite(uy) || !__builtin_isfinite(Ty) || ry <= 0.0 ||
            Ty <= 0.0)
            bad = 1;
        // the envelope where the fourth-order equilibria stay positive
        // (|u| <= ~0.91 sqrt(T) on D1Q7): a prediction outside it is rejected
        else if (a.max_mach > 0.0 && uy * uy > a.max_mach * a.max_mach * Ty)
            bad = 1;
    }
    if (threadIdx.x == 0) bad_s = 0;
    for (int k = 0; k < 7; ++k) red[threadIdx.x][k] = acc[k];
    __syncthreads();
    if (bad) atomicOr(&bad_s, 1);
    for (int h = kChkT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 7; ++k)
                red[threadIdx.x][k] = k == 6 ? fmax(red[threadIdx.x][k], red[threadIdx.x + h][k])
                                             : red[threadIdx.x][k] + red[threadIdx.x + h][k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double Mx = red[0][0], Px = red[0][1], Ex = red[0][2];
        const double My = red[0][3], Py = red[0][4], Ey = red[0][5], Tm = red[0][6];
        // An open tube exchanges mass, momentum and energy with the outside
        // only through its two ends (the balance laws of Sec. II integrated
        // over the tube): over the K steps of a call each total changes by
        // (K / r) (F(first node) - F(last node)) with the equilibrium fluxes
        // F = (rho u, rho (u^2 + T), rho u (u^2/2 + (3 + n) T / 2)) in lattice
        // units (a population moves c = xi / r nodes per step), the end
        // states taken as the mean of x and y.
        double F[3] = {0.0, 0.0, 0.0};
        for (int side = 0; side < 2; ++side) {
            const size_t i = (size_t)b * a.L + (side ? a.L - 1 : 0);
            for (int q = 0; q < 2; ++q) {
                const double *v = q ? a.y : a.x;
                const double r = v[i], u = v[BL + i], T = v[2 * BL + i];
                const double sg = side ? -0.5 : 0.5;
                F[0] += sg * r * u;
                F[1] += sg * r * (u * u + T);
                F[2] += sg * r * u * (0.5 * u * u + 0.5 * (3.0 + n) * T);
            }
        }
        const double kt = (double)LBM_SUR_K / kR;
        bool ok = !bad_s && __builtin_isfinite(My) && __builtin_isfinite(Ey);
        ok = ok && fabs(My - Mx - kt * F[0]) <= a.tol_m * fabs(Mx);
        ok = ok && fabs(Py - Px - kt * F[1]) <= a.tol_p * fabs(Mx) * sqrt(Tm > 0.0 ? Tm : 0.0);
        ok = ok && fabs(Ey - Ex - kt * F[2]) <= a.tol_e * fabs(Ex);
        a.accept[b] = ok ? 1 : 0;
    }
}

// Equilibrium populations of x for rejected tubes without live populations;
// nsteps of the rejected tubes (accepted tubes' entries stay as they are).  A batch tube whose node range is not [b L, (b+1) L)
// gets nothing written and 0 steps (the host checks the batch's size and
// type; the ranges live in device memory).
__global__ void __launch_bounds__(256) k_lift(int B, int L, const double *x, const int32_t *accept,
                                              const int32_t *valid, const int64_t *offsets, float *f0,
                                              float *g0, int64_t *nsteps, int64_t steps) {
    const size_t BL = (size_t)B * L;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < (size_t)B && !accept[i]) {
        const bool fits = offsets[i] == (int64_t)i * L && offsets[i + 1] == (int64_t)(i + 1) * L;
        nsteps[i] = fits ? steps : 0;
    }
    if (i >= BL) return;
    const int b = (int)(i / L);
    if (accept[b] || valid[b]) return;
    if (offsets[b] != (int64_t)b * L || offsets[b + 1] != (int64_t)(b + 1) * L) return;
    const double uu[3] = {x[BL + i], 0.0, 0.0};
    const FeqCoef<double> fc = feq_coef<double, 1>(x[i], uu, x[2 * BL + i]);
    static_for<0, 7>([&](auto I) {
        constexpr int k = decltype(I)::value;
        f0[(size_t)k * BL + i] = (float)feq_dir<double, 1, k>(fc);
    });
    const GeqCoef<double> gc = geq_coef<double>(x[2 * BL + i]);
    static_for<0, 7>([&](auto J) {
        constexpr int j = decltype(J)::value;
        g0[(size_t)j * BL + i] = (float)geq_dir<double, j>(gc);
    });
}

__global__ void __launch_bounds__(256) k_merge(int B, int L, const int32_t *accept, const double *y,
                                               const double *z, double *out, int32_t *valid) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t BL = (size_t)B * L;
    if (e >= 3 * BL) return;
    const int b = (int)((e % BL) / L);
    out[e] = accept[b] ? y[e] : z[e];
    if (e < BL && e % L == 0) valid[b] = accept[b] ? 0 : 1;
}

}  // namespace sur
}  // namespace lbmx

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {
using namespace lbmx::sur;

lbm_status sfail(lbm_status s, const std::string &m) {
    lbmx::set_error(m.c_str());
    return s;
}

// Carves 256-byte aligned pieces out of the workspace.  With no workspace
// (sizing only) the pieces are offsets from address 0, formed as integers.
struct WS {
    size_t off = 0;
    uintptr_t base;
    explicit WS(void *b) : base((uintptr_t)b) {}
    template <typename T> T *take(size_t n) {
        off = (off + 255) / 256 * 256;
        T *p = reinterpret_cast<T *>(base + off);
        off += n * sizeof(T);
        return p;
    }
};

struct Bufs {
    __bf16 *X, *dY, *dZ1, *A1[NB];
    float *H[NB + 1], *Hc[NB], *Z1[NB], *Y, *dH, *dA1, *dHc, *part, *bpart, *lpart;
};

size_t nchunk128(int M) { return (size_t)(M + 127) / 128; }

Bufs carve(const lbm_sur_desc *d, size_t *bytes) {
    const int M = d->batch * d->length / PATCH;
    WS w(d->workspace);
    Bufs b;
    b.X = w.take<__bf16>((size_t)M * FIN);
    for (int i = 0; i <= NB; ++i) b.H[i] = w.take<float>((size_t)M * C);
    for (int i = 0; i < NB; ++i) {
        b.Hc[i] = w.take<float>((size_t)M * C);
        b.Z1[i] = w.take<float>((size_t)M * HID);
        b.A1[i] = w.take<__bf16>((size_t)M * HID);
    }
    b.Y = w.take<float>((size_t)M * 32);
    b.dY = w.take<__bf16>((size_t)M * 16);
    b.dH = w.take<float>((size_t)M * C);
    b.dA1 = w.take<float>((size_t)M * HID);
    b.dZ1 = w.take<__bf16>((size_t)M * HID);
    b.dHc = w.take<float>((size_t)M * C);
    const size_t nch = nchunk128(M);
    b.part = w.take<float>(nch * HID * HID > (size_t)(M / 64 + 1) * C * 6 ? nch * HID * HID
                                                                          : (size_t)(M / 64 + 1) * C * 6);
    b.bpart = w.take<float>(nch * HID);
    b.lpart = w.take<float>((size_t)M * 16 / 256 + 1);
    *bytes = w.off + 256;
    return b;
}

lbm_status svalidate(const lbm_sur_desc *d) {
    if (!d) return sfail(LBM_EINVAL, "surrogate descriptor is NULL");
    if (d->abi_version != LBM_ABI_VERSION) return sfail(LBM_EINVAL, "abi_version mismatch");
    if (d->batch < 1 || d->length < 128 || d->length % 128)
        return sfail(LBM_EINVAL, "batch >= 1 and length a positive multiple of 128 required");
    if ((long long)d->batch * d->length >= (1LL << 31)) return sfail(LBM_EINVAL, "batch * length too large");
    return LBM_OK;
}

unsigned nblk(size_t n) { return (unsigned)((n + 255) / 256); }
unsigned nred(size_t n) { return (unsigned)((n + RED_J - 1) / RED_J); }

template <int N, int K, bool AF32, int EPI>
void gemm(hipStream_t s, int M, int nvalid, const void *A, const __bf16 *Bt, const float *bias,
          const float *R, float *out, __bf16 *out_bf, float *pre) {
    GemmArgs g{M, nvalid, A, Bt, bias, R, out, out_bf, pre};
    hipLaunchKernelGGL((k_gemm<N, K, AF32, EPI>), dim3((M + 127) / 128), dim3(256), 0, s, g);
}

template <int N, int K, int NA, int KB, bool AF32, bool BF32>
void wgrad(hipStream_t s, int M, int Nv, int Kv, const void *A, const void *B, float *part, float *bpart,
           float *gW, float *gb) {
    const int nch = (int)nchunk128(M);
    WgArgs g{M, Nv, Kv, A, B, part, gb ? bpart : nullptr};
    hipLaunchKernelGGL((k_wgrad<N, K, NA, KB, AF32, BF32>), dim3(nch), dim3(256), 0, s, g);
    hipLaunchKernelGGL(k_reduce_parts, dim3(nred((size_t)Nv * Kv)), dim3(RED_J * RED_K), 0, s, part, nch, Nv * Kv, gW, 0);
    if (gb) hipLaunchKernelGGL(k_reduce_parts, dim3(nred(Nv)), dim3(RED_J * RED_K), 0, s, bpart, nch, Nv, gb, 0);
}

// Forward through the network; keeps every activation needed by backward.
void forward(const lbm_sur_desc *d, const Bufs &b, const double *x, const double *gamma, hipStream_t s) {
    const Shape sh{d->batch, d->length, d->length / PATCH, d->batch * d->length / PATCH};
    const int M = sh.M;
    const float *P = d->params;
    const __bf16 *Q = (const __bf16 *)d->params_bf16;
    hipLaunchKernelGGL(k_patchify, dim3(nblk((size_t)M * FIN)), dim3(256), 0, s, sh, x, gamma, b.X);
    gemm<64, 16, false, EPI_BIAS | EPI_F32>(s, M, C, b.X, Q + Q_WE, P + P_BE, nullptr, b.H[0], nullptr, nullptr);
    for (int k = 0; k < NB; ++k) {
        const float *blk = P + P_BLK + k * BLK;
        const __bf16 *qb = Q + Q_BLK + k * QBLK;
        hipLaunchKernelGGL(k_conv_fwd, dim3(nblk((size_t)M * C)), dim3(256), 0, s, sh, b.H[k], blk + B_KC,
                           blk + B_BC, b.Hc[k]);
        gemm<128, 64, true, EPI_BIAS | EPI_GELU | EPI_BF16>(s, M, HID, b.Hc[k], qb + Q_W1, blk + B_B1, nullptr,
                                                            nullptr, b.A1[k], b.Z1[k]);
        gemm<64, 128, false, EPI_BIAS | EPI_RES | EPI_F32>(s, M, C, b.A1[k], qb + Q_W2, blk + B_B2, b.Hc[k],
                                                           b.H[k + 1], nullptr, nullptr);
    }
    gemm<32, 64, true, EPI_BIAS | EPI_F32>(s, M, FOUT, b.H[NB], Q + Q_WHP, P + P_BH, nullptr, b.Y, nullptr,
                                           nullptr);
}

}  // namespace

extern "C" {

size_t lbm_sur_bf16_bytes(void) { return (size_t)QTOTAL * 2; }

size_t lbm_sur_workspace_bytes(const lbm_sur_desc *desc) {
    if (!desc || desc->batch < 1 || desc->length < 128) return 0;
    lbm_sur_desc d = *desc;
    d.workspace = nullptr;
    size_t bytes = 0;
    carve(&d, &bytes);
    return bytes;
}

lbm_status lbm_sur_pack(const lbm_sur_desc *d, void *stream) {
    lbm_status st = svalidate(d);
    if (st) return st;
    if (!d->params || !d->params_bf16) return sfail(LBM_EINVAL, "params and params_bf16 required");
    hipLaunchKernelGGL(k_pack, dim3(nblk(QTOTAL)), dim3(256), 0, (hipStream_t)stream, d->params,
                       (__bf16 *)d->params_bf16);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : sfail(LBM_ELAUNCH, hipGetErrorString(e));
}

lbm_status lbm_sur_forward(const lbm_sur_desc *d, const double *x, const double *gamma,
                           const int32_t *active, double *y, void *stream) {
    lbm_status st = svalidate(d);
    if (st) return st;
    if (!d->params || !d->params_bf16 || !d->workspace || !x || !gamma || !y)
        return sfail(LBM_EINVAL, "NULL argument");
    if (x == y) return sfail(LBM_EINVAL, "y may not alias x");
    hipStream_t s = (hipStream_t)stream;
    const int T = d->length / PATCH, ntile = (T + FOUTR - 1) / FOUTR;
    FwdArgs fa{d->batch, d->length, T, ntile, x, gamma, active, d->params, (const __bf16 *)d->params_bf16, y};
    hipLaunchKernelGGL(k_fwd_fused, dim3((unsigned)(d->batch * ntile)), dim3(64 * FNW), 0, s, fa);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : sfail(LBM_ELAUNCH, hipGetErrorString(e));
}

lbm_status lbm_sur_backward(const lbm_sur_desc *d, const double *x, const double *gamma,
                            const double *target, float *grads, float *loss, void *stream) {
    lbm_status st = svalidate(d);
    if (st) return st;
    if (!d->params || !d->params_bf16 || !d->workspace || !x || !gamma || !target || !grads || !loss)
        return sfail(LBM_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    size_t bytes;
    const Bufs b = carve(d, &bytes);
    forward(d, b, x, gamma, s);
    const Shape sh{d->batch, d->length, d->length / PATCH, d->batch * d->length / PATCH};
    const int M = sh.M;
    const __bf16 *Q = (const __bf16 *)d->params_bf16;
    const float *P = d->params;
    const unsigned nl = nblk((size_t)M * 16);
    hipLaunchKernelGGL(k_loss, dim3(nl), dim3(256), 0, s, sh, x, target, b.Y, b.dY, b.lpart);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, b.lpart, (int)nl, M * FOUT, loss);
    // head
    wgrad<32, 64, 16, 64, false, true>(s, M, FOUT, C, b.dY, b.H[NB], b.part, b.bpart, grads + P_WH, grads + P_BH);
    gemm<64, 16, false, EPI_F32>(s, M, C, b.dY, Q + Q_WHTP, nullptr, nullptr, b.dH, nullptr, nullptr);
    for (int k = NB - 1; k >= 0; --k) {
        const float *blk = P + P_BLK + k * BLK;
        float *gblk = grads + P_BLK + k * BLK;
        const __bf16 *qb = Q + Q_BLK + k * QBLK;
        // dA1 = dO W2 ; dZ1 = dA1 gelu'(Z1)
        gemm<128, 64, true, EPI_F32>(s, M, HID, b.dH, qb + Q_W2T, nullptr, nullptr, b.dA1, nullptr, nullptr);
        hipLaunchKernelGGL(k_gelu_bwd, dim3(nblk((size_t)M * HID)), dim3(256), 0, s, M * HID, b.dA1, b.Z1[k],
                           b.dZ1);
        wgrad<64, 128, 64, 128, true, false>(s, M, C, HID, b.dH, b.A1[k], b.part, b.bpart, gblk + B_W2,
                                             gblk + B_B2);
        wgrad<128, 64, 128, 64, false, true>(s, M, HID, C, b.dZ1, b.Hc[k], b.part, b.bpart, gblk + B_W1,
                                             gblk + B_B1);
        // dHc = dO + dZ1 W1 ; dH = dHc + conv^T(dHc)
        gemm<64, 128, false, EPI_RES | EPI_F32>(s, M, C, b.dZ1, qb + Q_W1T, nullptr, b.dH, b.dHc, nullptr,
                                                nullptr);
        const unsigned nc = (unsigned)((M + 63) / 64);
        hipLaunchKernelGGL(k_conv_bwd, dim3(nc), dim3(256), 0, s, sh, b.dHc, b.H[k], blk + B_KC, b.dH, b.part);
        // taps and bias of the convolution: part[wg][c][6] -> [c][6] -> kc, bc
        hipLaunchKernelGGL(k_reduce_parts, dim3(nred(C * 6)), dim3(RED_J * RED_K), 0, s, b.part, (int)nc, C * 6, b.bpart, 0);
        hipLaunchKernelGGL(k_conv_scatter, dim3(1), dim3(64), 0, s, b.bpart, gblk + B_KC, gblk + B_BC);
    }
    wgrad<64, 32, 64, 16, true, false>(s, M, C, FIN, b.dH, b.X, b.part, b.bpart, grads + P_WE, grads + P_BE);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : sfail(LBM_ELAUNCH, hipGetErrorString(e));
}

lbm_status lbm_sur_adam(const lbm_sur_desc *d, float *params, float *m, float *v, const float *grads, float lr,
                        float beta1, float beta2, float eps, int64_t step, void *stream) {
    lbm_status st = svalidate(d);
    if (st) return st;
    if (!params || !m || !v || !grads || step < 1) return sfail(LBM_EINVAL, "bad Adam arguments");
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_adam, dim3(nblk(NPARAMS)), dim3(256), 0, s, NPARAMS, params, m, v, grads, lr, beta1,
                       beta2, eps, c1, c2);
    hipLaunchKernelGGL(k_pack, dim3(nblk(QTOTAL)), dim3(256), 0, s, params, (__bf16 *)d->params_bf16);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : sfail(LBM_ELAUNCH, hipGetErrorString(e));
}

lbm_status lbm_sur_check(const lbm_sur_desc *d, const double *x, const double *y, const double *gamma,
                         double tol_mass, double tol_mom, double tol_energy, double max_mach,
                         int32_t *accept, void *stream) {
    lbm_status st = svalidate(d);
    if (st) return st;
    if (!x || !y || !gamma || !accept) return sfail(LBM_EINVAL, "NULL argument");
    if (!(max_mach >= 0.0)) return sfail(LBM_EINVAL, "max_mach must be >= 0");
    CheckArgs a{d->batch, d->length, x, y, gamma, tol_mass, tol_mom, tol_energy, max_mach, accept};
    hipLaunchKernelGGL(k_check, dim3(d->batch), dim3(kChkT), 0, (hipStream_t)stream, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : sfail(LBM_ELAUNCH, hipGetErrorString(e));
}

lbm_status lbm_sur_lift(const lbm_sur_desc *d, const double *x, const int32_t *accept, const int32_t *valid,
                        const lbm_batch_desc *batch, int64_t steps, void *stream) {
    lbm_status st = svalidate(d);
    if (st) return st;
    if (!x || !accept || !valid || !batch) return sfail(LBM_EINVAL, "NULL argument");
    if (steps < 0) return sfail(LBM_EINVAL, "steps must be >= 0");
    if (batch->abi_version != LBM_ABI_VERSION) return sfail(LBM_EINVAL, "batch abi_version mismatch");
    if (batch->dtype != LBM_F32) return sfail(LBM_EINVAL, "the fallback batch must hold FP32 populations");
    if (batch->num_instances != d->batch || batch->total_nodes != (int64_t)d->batch * d->length)
        return sfail(LBM_EINVAL, "the fallback batch must have one tube of the surrogate's length per surrogate tube");
    if (!batch->f[0] || !batch->g[0] || !batch->nsteps || !batch->offsets)
        return sfail(LBM_EINVAL, "fallback batch buffers must not be NULL");
    const size_t BL = (size_t)d->batch * d->length;
    // nsteps is an input of lbm_batch_step; lift is what sets it
    hipLaunchKernelGGL(k_lift, dim3(nblk(BL > (size_t)d->batch ? BL : d->batch)), dim3(256), 0, (hipStream_t)stream,
                       d->batch, d->length, x, accept, valid, batch->offsets, (float *)batch->f[0],
                       (float *)batch->g[0], const_cast<int64_t *>(batch->nsteps), steps);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : sfail(LBM_ELAUNCH, hipGetErrorString(e));
}

lbm_status lbm_sur_merge(const lbm_sur_desc *d, const int32_t *accept, const double *y, const double *z,
                         double *out, int32_t *valid, void *stream) {
    lbm_status st = svalidate(d);
    if (st) return st;
    if (!accept || !y || !z || !out || !valid) return sfail(LBM_EINVAL, "NULL argument");
    const size_t n = (size_t)3 * d->batch * d->length;
    hipLaunchKernelGGL(k_merge, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, d->batch, d->length, accept,
                       y, z, out, valid);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : sfail(LBM_ELAUNCH, hipGetErrorString(e));
}

}  // extern "C"
