// rsi_mlp.hip -- the learned surrogate: Fourier-feature MLP trained and evaluated with
// bfloat16 MFMA GEMMs (gfx950 v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// Every GEMM of training is written in one "NT" form, C[M][N] = A[M][K] . B[N][K]^T, with
// both operands contiguous along the reduction dimension, so that each lane of a wave
// loads its 8 bfloat16 MFMA operands with one 16-byte load:
//   forward   Z_l  = H_{l-1} [B][K]  . W_l   [N][K]^T
//   input grad dH  = dZ_l    [B][N]  . W_l^T [K][N]^T      (transposed weight copy)
//   weight grad dW = dZ_l^T  [N][B]  . H^T   [K][B]^T      (transposed activations)
// The epilogues fuse bias + SiLU (forward) and the SiLU derivative (input gradient) and
// write the row-major and the transposed bfloat16 copies the next GEMM needs.  Weight
// gradients are split over the batch and reduced in a fixed order (deterministic).
//
// MFMA 16x16x32 bf16 operand layout (lane l, i = 0..7 / e = 0..3):
//   A[l % 16][8 (l / 16) + i],  B[8 (l / 16) + i][l % 16],  D[4 (l / 16) + e][l % 16].
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <vector>

#include "../../include/rsi_mlp.h"
#include "rsi_internal.h"

namespace rsi {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTileM = 64, kTileN = 64, kTileK = 32;
constexpr int kMaxLayers = 16;

__device__ inline float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ inline float silu_grad_f(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

enum { EPI_FWD = 0, EPI_FWD_INFER = 1, EPI_DX = 2, EPI_DW = 3 };

struct GemmArgs {
    const bf16 *A;
    int64_t lda;
    const bf16 *B;
    int64_t ldb;
    int64_t M, N, K, k_per_split;
    const float *bias;  // EPI_FWD*: [N]
    float *Z;           // EPI_FWD: pre-activation out; EPI_DX: previous pre-activation in
    int64_t ldz;
    bf16 *H;            // EPI_FWD*: activation out; EPI_DX: previous dZ out
    int64_t ldh;
    bf16 *HT;           // optional transposed copy [N][M]
    int64_t ldht;
    float *P;           // EPI_DW: partials [split][M][N]
};

template <int EPI>
__global__ void __launch_bounds__(256) gemm_nt_kernel(GemmArgs g) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t m0 = (int64_t)blockIdx.x * kTileM + (wave >> 1) * 32;
    const int64_t n0 = (int64_t)blockIdx.y * kTileN + (wave & 1) * 32;
    const int64_t kb = (int64_t)blockIdx.z * g.k_per_split;
    const int64_t ke = (kb + g.k_per_split < g.K) ? kb + g.k_per_split : g.K;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const bf16 *pa0 = g.A + (m0 + r) * g.lda + kq, *pa1 = pa0 + 16 * g.lda;
    const bf16 *pb0 = g.B + (n0 + r) * g.ldb + kq, *pb1 = pb0 + 16 * g.ldb;
    for (int64_t k = kb; k < ke; k += kTileK) {
        const bf16x8 a0 = *reinterpret_cast<const bf16x8 *>(pa0 + k);
        const bf16x8 a1 = *reinterpret_cast<const bf16x8 *>(pa1 + k);
        const bf16x8 b0 = *reinterpret_cast<const bf16x8 *>(pb0 + k);
        const bf16x8 b1 = *reinterpret_cast<const bf16x8 *>(pb1 + k);
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
    const int cn = lane & 15, cm = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t n = n0 + 16 * j + cn;
            const int64_t mb = m0 + 16 * i + cm;
            if constexpr (EPI == EPI_DW) {
                float *p = g.P + (int64_t)blockIdx.z * g.M * g.N;
#pragma unroll
                for (int e = 0; e < 4; ++e) p[(mb + e) * g.N + n] = acc[i][j][e];
            } else {
                bf16x4 hv;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t m = mb + e;
                    float v;
                    if constexpr (EPI == EPI_DX) {
                        v = acc[i][j][e] * silu_grad_f(g.Z[m * g.ldz + n]);
                    } else {
                        const float z = acc[i][j][e] + g.bias[n];
                        if constexpr (EPI == EPI_FWD) g.Z[m * g.ldz + n] = z;
                        v = silu_f(z);
                    }
                    const bf16 h = (bf16)v;
                    g.H[m * g.ldh + n] = h;
                    hv[e] = h;
                }
                if (g.HT) *reinterpret_cast<bf16x4 *>(g.HT + n * g.ldht + mb) = hv;
            }
        }
}

// Fourier features of the normalised query: h0 = [sin 2 pi u, cos 2 pi u], u = B v.
struct Box {
    double lo[5], inv[5];  // v = 2 (q - lo) * inv - 1, inv = 1 / (hi - lo)
};

__global__ void __launch_bounds__(256) features_kernel(int64_t n, int64_t Mp, int m,
                                                       const float *__restrict__ q, Box box,
                                                       const float *__restrict__ Bff,
                                                       bf16 *__restrict__ H0, int64_t ld) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= Mp * m) return;
    const int64_t b = g / m;
    const int j = (int)(g - b * m);
    // u and its reduction to one revolution in FP64: the bf16 features then round the
    // same values the FP64 reference rounds (|u| reaches tens of revolutions)
    double u = 0.0;
    if (b < n) {
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const double v = 2.0 * ((double)q[b * 5 + c] - box.lo[c]) * box.inv[c] - 1.0;
            u = fma((double)Bff[j * 5 + c], v, u);
        }
    }
    const float ph = (float)(u - floor(u));  // sin(2 pi u): revolutions
    H0[b * ld + j] = (bf16)__builtin_amdgcn_sinf(ph);
    H0[b * ld + m + j] = (bf16)__builtin_amdgcn_cosf(ph);
}

// bf16 transpose [R][C] -> [C][R] through LDS, 64 x 64 tiles.
__global__ void __launch_bounds__(256) transpose_bf16_kernel(const bf16 *__restrict__ in, int64_t R,
                                                             int64_t C, bf16 *__restrict__ out) {
    __shared__ bf16 tile[64][66];
    const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int rr = ty; rr < 64; rr += 4) tile[rr][tx] = in[(r0 + rr) * C + c0 + tx];
    __syncthreads();
    for (int cc = ty; cc < 64; cc += 4) out[(c0 + cc) * R + r0 + tx] = tile[tx][cc];
}

// Output layer (FP32), loss and its gradient, one wave per row.  Training when t != NULL:
// dZ_L = bf16((dy Wo) * silu'(Z_L)), per-block partial sums of dWo, dbo and the loss.
__global__ void __launch_bounds__(256) head_kernel(int64_t n, int W, const bf16 *__restrict__ H,
                                                   const float *__restrict__ Z,
                                                   const float *__restrict__ Wo,
                                                   const float *__restrict__ bo,
                                                   const float *__restrict__ t, float *__restrict__ y,
                                                   bf16 *__restrict__ dZ, float *__restrict__ part) {
    constexpr int kMaxPerLane = 16;  // W <= 1024
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int per = W / 64;
    float gw0[kMaxPerLane], gw1[kMaxPerLane];
    for (int q = 0; q < per; ++q) gw0[q] = gw1[q] = 0.0f;
    float gb0 = 0.0f, gb1 = 0.0f, loss = 0.0f;
    for (int rr = 0; rr < 16; ++rr) {
        const int64_t row = (int64_t)blockIdx.x * 64 + wave * 16 + rr;
        float hv[kMaxPerLane];
        float y0 = 0.0f, y1 = 0.0f;
        for (int q = 0; q < per; ++q) {
            const int f = lane + 64 * q;
            hv[q] = (float)H[row * W + f];
            y0 = fmaf(Wo[f], hv[q], y0);
            y1 = fmaf(Wo[W + f], hv[q], y1);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            y0 += __shfl_xor(y0, off);
            y1 += __shfl_xor(y1, off);
        }
        y0 += bo[0];
        y1 += bo[1];
        if (row < n && lane == 0 && y) {
            y[2 * row] = y0;
            y[2 * row + 1] = y1;
        }
        if (!t) continue;
        float d0 = 0.0f, d1 = 0.0f;
        if (row < n) {
            const float e0 = y0 - t[2 * row], e1 = y1 - t[2 * row + 1];
            d0 = e0 / (float)n;
            d1 = e1 / (float)n;
            loss += 0.5f * (e0 * e0 + e1 * e1) / (float)n;
        }
        gb0 += d0;
        gb1 += d1;
        for (int q = 0; q < per; ++q) {
            const int f = lane + 64 * q;
            gw0[q] = fmaf(d0, hv[q], gw0[q]);
            gw1[q] = fmaf(d1, hv[q], gw1[q]);
            const float dh = d0 * Wo[f] + d1 * Wo[W + f];
            dZ[row * W + f] = (bf16)(dh * silu_grad_f(Z[row * W + f]));
        }
    }
    if (!t) return;
    // block partials: [2W] weight grads, [2] bias grads, [1] loss (fixed-order sums)
    __shared__ float sh[4][2 * 1024 + 3];
    for (int q = 0; q < per; ++q) {
        sh[wave][lane + 64 * q] = gw0[q];
        sh[wave][W + lane + 64 * q] = gw1[q];
    }
    if (lane == 0) {
        sh[wave][2 * W] = gb0;
        sh[wave][2 * W + 1] = gb1;
        sh[wave][2 * W + 2] = loss;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 2 * W + 3; idx += 256)
        part[(int64_t)blockIdx.x * (2 * W + 3) + idx] =
            ((sh[0][idx] + sh[1][idx]) + sh[2][idx]) + sh[3][idx];
}

// Fixed-order column sums: out[c] = sum_r in[r * ld + c] (r < R), accumulated in FP64.
__global__ void __launch_bounds__(256) colsum_kernel(const float *__restrict__ in, int64_t R, int64_t C,
                                                     int64_t ld, float *__restrict__ out) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= C) return;
    double s = 0.0;
    for (int64_t r = 0; r < R; ++r) s += (double)in[r * ld + c];
    out[c] = (float)s;
}

// Bias gradient, first level: part[chunk][c] = sum of dZ[r][c] over the chunk's rows.
constexpr int kBiasRows = 1024;
__global__ void __launch_bounds__(256) bias_partial_kernel(const bf16 *__restrict__ dZ, int64_t Mp, int W,
                                                           float *__restrict__ part) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= W) return;
    const int64_t r0 = (int64_t)blockIdx.y * kBiasRows;
    const int64_t r1 = (r0 + kBiasRows < Mp) ? r0 + kBiasRows : Mp;
    float s = 0.0f;
    for (int64_t r = r0; r < r1; ++r) s += (float)dZ[r * W + c];
    part[(int64_t)blockIdx.y * W + c] = s;
}

__global__ void __launch_bounds__(256) adam_kernel(int64_t P, float *__restrict__ p,
                                                   const float *__restrict__ g, float *__restrict__ m,
                                                   float *__restrict__ v, float lr, float c1,
                                                   float c2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= P) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// bf16 copies of one weight matrix [O][I]: row-major and transposed.
__global__ void __launch_bounds__(256) cast_weight_kernel(const float *__restrict__ Wf, int O, int I,
                                                          bf16 *__restrict__ Wb, bf16 *__restrict__ WTb) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (int64_t)O * I) return;
    const int o = (int)(k / I), i = (int)(k - (int64_t)o * I);
    const bf16 v = (bf16)Wf[k];
    Wb[k] = v;
    WTb[(int64_t)i * O + o] = v;
}

// Carrier: the phase of the tilted piston's plane wave refracted at the plane z = depth.
// Its horizontal slowness C = sin(tilt)/c1 is conserved (eq. 15), so
//     psi = 2 pi f (C x + eta1 depth + eta2 z_below),  eta_i = sqrt(1/c_i^2 - C^2),
// with eta2 = 0 past the critical angle (no propagating phase below the plane).  Near
// the interface the beam of the piston is close to this plane wave (the interface lies
// within the piston's near field a^2/lambda at these frequencies), so the envelope
// field * e^{-i psi} varies slowly across the beam.
__global__ void __launch_bounds__(256) carrier_kernel(int64_t n, const float *__restrict__ q, double c1,
                                                      double c2, int mode, double scale,
                                                      const float2 *__restrict__ in, float2 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double x = (double)q[5 * i], zb = (double)q[5 * i + 1], f = (double)q[5 * i + 2],
                 h1 = (double)q[5 * i + 3], tilt = (double)q[5 * i + 4];
    const double C = sin(tilt) / c1;
    const double eta1 = sqrt(fmax(1.0 / (c1 * c1) - C * C, 0.0));
    const double eta2 = sqrt(fmax(1.0 / (c2 * c2) - C * C, 0.0));
    double ph = f * (C * x + eta1 * h1 + eta2 * zb);  // revolutions
    ph -= floor(ph);
    double sn, cs;
    sincospi(2.0 * ph, &sn, &cs);
    const float2 a = in[i];
    if (mode == 0) {  // envelope = field * e^{-i psi} / scale
        out[i] = make_float2((float)((a.x * cs + a.y * sn) / scale), (float)((a.y * cs - a.x * sn) / scale));
    } else {          // field = envelope * e^{+i psi} * scale
        out[i] = make_float2((float)((a.x * cs - a.y * sn) * scale), (float)((a.y * cs + a.x * sn) * scale));
    }
}

}  // namespace rsi

// ---------------------------------------------------------------------------
// The network object.
// ---------------------------------------------------------------------------
struct rsi_mlp {
    int m = 0, F = 0, W = 0, L = 0;
    int64_t max_batch = 0, Mp_max = 0;
    rsi::Box box{};
    int64_t P = 0;
    std::vector<int64_t> offW, offb;  // per layer, into the flat parameter vector
    std::vector<int> in_dim;
    int64_t offWo = 0, offbo = 0;
    int64_t step = 0;
    rsi::DeviceBuffer Bff, params, grads, adam_m, adam_v;
    std::vector<std::unique_ptr<rsi::DeviceBuffer>> Wb, WTb;  // bf16 weights and transposes
    std::vector<std::unique_ptr<rsi::DeviceBuffer>> H, Z;    // activations [L+1], pre-acts [L]
    rsi::DeviceBuffer HT, dZ[2], dZT, dwpart, headpart, lossbuf;
    int dw_splits = 1;
};

namespace rsi {

static int64_t pad64(int64_t n) { return (n + 63) / 64 * 64; }

static rsi_status gemm(int epi, const GemmArgs &g, int splits, hipStream_t s) {
    const dim3 grid((unsigned)(g.M / kTileM), (unsigned)(g.N / kTileN), (unsigned)splits);
    switch (epi) {
        case EPI_FWD: hipLaunchKernelGGL(gemm_nt_kernel<EPI_FWD>, grid, dim3(256), 0, s, g); break;
        case EPI_FWD_INFER: hipLaunchKernelGGL(gemm_nt_kernel<EPI_FWD_INFER>, grid, dim3(256), 0, s, g); break;
        case EPI_DX: hipLaunchKernelGGL(gemm_nt_kernel<EPI_DX>, grid, dim3(256), 0, s, g); break;
        default: hipLaunchKernelGGL(gemm_nt_kernel<EPI_DW>, grid, dim3(256), 0, s, g); break;
    }
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

static rsi_status transpose(const bf16 *in, int64_t R, int64_t C, bf16 *out, hipStream_t s) {
    hipLaunchKernelGGL(transpose_bf16_kernel, dim3((unsigned)(R / 64), (unsigned)(C / 64)), dim3(256), 0, s,
                       in, R, C, out);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

static rsi_status refresh_bf16(rsi_mlp *net, hipStream_t s) {
    for (int l = 0; l < net->L; ++l) {
        const int O = net->W, I = net->in_dim[l];
        const int64_t cnt = (int64_t)O * I;
        hipLaunchKernelGGL(cast_weight_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                           net->params.as<float>() + net->offW[l], O, I, net->Wb[l]->as<bf16>(),
                           net->WTb[l]->as<bf16>());
        RSI_HIP(hipGetLastError());
    }
    return RSI_OK;
}

// Forward through the hidden layers (training keeps Z and nothing else is needed).
static rsi_status forward_hidden(rsi_mlp *net, int64_t n, const float *q, bool train, hipStream_t s) {
    const int64_t Mp = pad64(n);
    const int64_t tot = Mp * net->m;
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, Mp, net->m,
                       q, net->box, net->Bff.as<float>(), net->H[0]->as<bf16>(), (int64_t)net->F);
    RSI_HIP(hipGetLastError());
    for (int l = 0; l < net->L; ++l) {
        GemmArgs g{};
        g.A = net->H[l]->as<bf16>();
        g.lda = net->in_dim[l];
        g.B = net->Wb[l]->as<bf16>();
        g.ldb = net->in_dim[l];
        g.M = Mp;
        g.N = net->W;
        g.K = net->in_dim[l];
        g.k_per_split = g.K;
        g.bias = net->params.as<float>() + net->offb[l];
        g.Z = train ? net->Z[l]->as<float>() : nullptr;
        g.ldz = net->W;
        g.H = net->H[l + 1]->as<bf16>();
        g.ldh = net->W;
        g.HT = nullptr;
        RSI_TRY(gemm(train ? EPI_FWD : EPI_FWD_INFER, g, 1, s));
    }
    return RSI_OK;
}

static rsi_status backward(rsi_mlp *net, int64_t n, const float *t, float *grad, float *loss,
                           hipStream_t s) {
    const int64_t Mp = pad64(n);
    const int W = net->W;
    const unsigned hb = (unsigned)(Mp / 64);
    const float *params = net->params.as<float>();
    hipLaunchKernelGGL(head_kernel, dim3(hb), dim3(256), 0, s, n, W, net->H[net->L]->as<bf16>(),
                       net->Z[net->L - 1]->as<float>(), params + net->offWo, params + net->offbo, t,
                       (float *)nullptr, net->dZ[0].as<bf16>(), net->headpart.as<float>());
    RSI_HIP(hipGetLastError());
    // head partials [hb][2W + 3] -> dWo, dbo (columns 0..2W+1) and the loss (column 2W+2)
    {
        const int64_t C = 2 * W + 3;
        float *lossdst = loss ? loss : net->lossbuf.as<float>();
        hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((C - 1 + 255) / 256)), dim3(256), 0, s,
                           net->headpart.as<float>(), (int64_t)hb, C - 1, C, grad + net->offWo);
        RSI_HIP(hipGetLastError());
        hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(256), 0, s, net->headpart.as<float>() + (C - 1),
                           (int64_t)hb, (int64_t)1, C, lossdst);
        RSI_HIP(hipGetLastError());
    }
    int cur = 0;
    for (int l = net->L - 1; l >= 0; --l) {
        const int I = net->in_dim[l];
        // transposes for the weight gradient: dZ^T [W][Mp], H_{l}^T [I][Mp]
        RSI_TRY(transpose(net->dZ[cur].as<bf16>(), Mp, W, net->dZT.as<bf16>(), s));
        RSI_TRY(transpose(net->H[l]->as<bf16>(), Mp, I, net->HT.as<bf16>(), s));
        int splits = net->dw_splits;
        while (splits > 1 && (Mp % ((int64_t)splits * kTileK) != 0)) splits >>= 1;
        GemmArgs g{};
        g.A = net->dZT.as<bf16>();
        g.lda = Mp;
        g.B = net->HT.as<bf16>();
        g.ldb = Mp;
        g.M = W;
        g.N = I;
        g.K = Mp;
        g.k_per_split = Mp / splits;
        g.P = net->dwpart.as<float>();
        RSI_TRY(gemm(EPI_DW, g, splits, s));
        const int64_t C = (int64_t)W * I;
        hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, s,
                           net->dwpart.as<float>(), (int64_t)splits, C, C, grad + net->offW[l]);
        RSI_HIP(hipGetLastError());
        // bias gradient: chunked column sums of dZ, then a fixed-order sum of the chunks
        // (the weight partials are consumed above, so their buffer is reused here)
        const int64_t nch = (Mp + kBiasRows - 1) / kBiasRows;
        hipLaunchKernelGGL(bias_partial_kernel, dim3((unsigned)((W + 255) / 256), (unsigned)nch), dim3(256),
                           0, s, net->dZ[cur].as<bf16>(), Mp, W, net->dwpart.as<float>());
        RSI_HIP(hipGetLastError());
        hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, s,
                           net->dwpart.as<float>(), nch, (int64_t)W, (int64_t)W, grad + net->offb[l]);
        RSI_HIP(hipGetLastError());
        if (l == 0) break;
        GemmArgs d{};
        d.A = net->dZ[cur].as<bf16>();
        d.lda = W;
        d.B = net->WTb[l]->as<bf16>();
        d.ldb = W;
        d.M = Mp;
        d.N = I;
        d.K = W;
        d.k_per_split = W;
        d.Z = net->Z[l - 1]->as<float>();
        d.ldz = W;
        d.H = net->dZ[cur ^ 1].as<bf16>();
        d.ldh = I;
        d.HT = nullptr;
        RSI_TRY(gemm(EPI_DX, d, 1, s));
        cur ^= 1;
    }
    return RSI_OK;
}

static rsi_status check_batch(const rsi_mlp *net, int64_t n, const void *q) {
    if (!net) return RSI_ERR_NULL;
    if (n < 0 || n > net->max_batch) return RSI_ERR_SIZE;
    if (n > 0 && !q) return RSI_ERR_NULL;
    return RSI_OK;
}

}  // namespace rsi

using namespace rsi;

extern "C" {

rsi_status rsi_mlp_create(rsi_mlp **out, int n_ff, int width, int depth, const float *B,
                          const float *lo, const float *hi, int64_t max_batch) {
    if (!out || !B || !lo || !hi) return RSI_ERR_NULL;
    *out = nullptr;
    const int F = 2 * n_ff;
    if (n_ff <= 0 || F % 64 || F > 1024 || width <= 0 || width % 64 || width > 1024 || depth < 1 ||
        depth > kMaxLayers)
        return RSI_ERR_ARG;
    if (max_batch <= 0 || max_batch > (int64_t(1) << 26)) return RSI_ERR_SIZE;
    for (int c = 0; c < 5; ++c)
        if (!(hi[c] > lo[c])) return RSI_ERR_ARG;
    std::unique_ptr<rsi_mlp> net(new rsi_mlp);
    net->m = n_ff;
    net->F = F;
    net->W = width;
    net->L = depth;
    net->max_batch = max_batch;
    net->Mp_max = pad64(max_batch);
    for (int c = 0; c < 5; ++c) {
        net->box.lo[c] = lo[c];
        net->box.inv[c] = 1.0 / ((double)hi[c] - (double)lo[c]);
    }
    int64_t o = 0;
    for (int l = 0; l < depth; ++l) {
        const int I = l == 0 ? F : width;
        net->in_dim.push_back(I);
        net->offW.push_back(o);
        o += (int64_t)width * I;
        net->offb.push_back(o);
        o += width;
    }
    net->offWo = o;
    o += 2 * (int64_t)width;
    net->offbo = o;
    o += 2;
    net->P = o;
    const int64_t Mp = net->Mp_max;
    const int maxdim = F > width ? F : width;
    RSI_TRY(net->Bff.alloc(sizeof(float) * n_ff * 5));
    RSI_HIP(hipMemcpy(net->Bff.as<void>(), B, sizeof(float) * n_ff * 5, hipMemcpyHostToDevice));
    for (auto *b : {&net->params, &net->grads, &net->adam_m, &net->adam_v}) {
        RSI_TRY(b->alloc(sizeof(float) * net->P));
        RSI_HIP(hipMemset(b->as<void>(), 0, sizeof(float) * net->P));
    }
    for (int l = 0; l < depth; ++l) {
        net->Wb.emplace_back(new DeviceBuffer);
        net->WTb.emplace_back(new DeviceBuffer);
        RSI_TRY(net->Wb.back()->alloc(sizeof(bf16) * width * net->in_dim[l]));
        RSI_TRY(net->WTb.back()->alloc(sizeof(bf16) * width * net->in_dim[l]));
        net->Z.emplace_back(new DeviceBuffer);
        RSI_TRY(net->Z.back()->alloc(sizeof(float) * Mp * width));
    }
    for (int l = 0; l <= depth; ++l) {
        net->H.emplace_back(new DeviceBuffer);
        RSI_TRY(net->H.back()->alloc(sizeof(bf16) * Mp * (l == 0 ? F : width)));
    }
    RSI_TRY(net->HT.alloc(sizeof(bf16) * Mp * maxdim));
    RSI_TRY(net->dZ[0].alloc(sizeof(bf16) * Mp * maxdim));
    RSI_TRY(net->dZ[1].alloc(sizeof(bf16) * Mp * maxdim));
    RSI_TRY(net->dZT.alloc(sizeof(bf16) * Mp * maxdim));
    // weight-gradient split over the batch: about 1024 rows per split, at most 128 splits
    int splits = 1;
    while (splits < 128 && Mp / (splits * 2) >= 1024) splits *= 2;
    net->dw_splits = splits;
    const size_t bias_chunks = (size_t)((Mp + kBiasRows - 1) / kBiasRows);
    const size_t dw_elems = (size_t)splits * width * maxdim;
    RSI_TRY(net->dwpart.alloc(sizeof(float) * std::max(dw_elems, bias_chunks * width)));
    RSI_TRY(net->headpart.alloc(sizeof(float) * (size_t)(Mp / 64) * (2 * width + 3)));
    RSI_TRY(net->lossbuf.alloc(sizeof(float) * 4));
    RSI_TRY(refresh_bf16(net.get(), nullptr));
    RSI_HIP(hipDeviceSynchronize());
    *out = net.release();
    return RSI_OK;
}

rsi_status rsi_mlp_destroy(rsi_mlp *net) {
    if (!net) return RSI_OK;
    RSI_HIP(hipDeviceSynchronize());
    delete net;
    return RSI_OK;
}

int64_t rsi_mlp_num_params(const rsi_mlp *net) { return net ? net->P : 0; }

rsi_status rsi_mlp_set_params(rsi_mlp *net, const float *hp) {
    if (!net || !hp) return RSI_ERR_NULL;
    RSI_HIP(hipMemcpy(net->params.as<void>(), hp, sizeof(float) * net->P, hipMemcpyHostToDevice));
    RSI_HIP(hipMemset(net->adam_m.as<void>(), 0, sizeof(float) * net->P));
    RSI_HIP(hipMemset(net->adam_v.as<void>(), 0, sizeof(float) * net->P));
    net->step = 0;
    RSI_TRY(refresh_bf16(net, nullptr));
    RSI_HIP(hipDeviceSynchronize());
    return RSI_OK;
}

rsi_status rsi_mlp_get_params(const rsi_mlp *net, float *hp) {
    if (!net || !hp) return RSI_ERR_NULL;
    RSI_HIP(hipDeviceSynchronize());
    RSI_HIP(hipMemcpy(hp, net->params.as<void>(), sizeof(float) * net->P, hipMemcpyDeviceToHost));
    return RSI_OK;
}

rsi_status rsi_mlp_forward(rsi_mlp *net, int64_t n, const float *q, float *y, void *stream) {
    RSI_TRY(check_batch(net, n, q));
    if (n == 0) return RSI_OK;
    if (!y) return RSI_ERR_NULL;
    hipStream_t s = as_stream(stream);
    RSI_TRY(forward_hidden(net, n, q, false, s));
    const int64_t Mp = pad64(n);
    const float *params = net->params.as<float>();
    hipLaunchKernelGGL(head_kernel, dim3((unsigned)(Mp / 64)), dim3(256), 0, s, n, net->W,
                       net->H[net->L]->as<bf16>(), (const float *)nullptr, params + net->offWo,
                       params + net->offbo, (const float *)nullptr, y, (bf16 *)nullptr, (float *)nullptr);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

rsi_status rsi_mlp_gradients(rsi_mlp *net, int64_t n, const float *q, const float *t, float *grad,
                             float *loss, void *stream) {
    RSI_TRY(check_batch(net, n, q));
    if (n == 0) return RSI_ERR_SIZE;
    if (!t || !grad) return RSI_ERR_NULL;
    hipStream_t s = as_stream(stream);
    RSI_TRY(forward_hidden(net, n, q, true, s));
    return backward(net, n, t, grad, loss, s);
}

rsi_status rsi_mlp_train_step(rsi_mlp *net, int64_t n, const float *q, const float *t, float lr,
                              float *loss, void *stream) {
    RSI_TRY(check_batch(net, n, q));
    if (n == 0) return RSI_ERR_SIZE;
    if (!t) return RSI_ERR_NULL;
    if (!(lr > 0.0f)) return RSI_ERR_ARG;
    hipStream_t s = as_stream(stream);
    RSI_TRY(forward_hidden(net, n, q, true, s));
    RSI_TRY(backward(net, n, t, net->grads.as<float>(), loss, s));
    net->step += 1;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)net->step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)net->step));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((net->P + 255) / 256)), dim3(256), 0, s, net->P,
                       net->params.as<float>(), net->grads.as<float>(), net->adam_m.as<float>(),
                       net->adam_v.as<float>(), lr, c1, c2);
    RSI_HIP(hipGetLastError());
    return refresh_bf16(net, s);
}

static const uint32_t kMagic = 0x524d4c50u;  // "RMLP"

rsi_status rsi_mlp_save(const rsi_mlp *net, const char *path) {
    if (!net || !path) return RSI_ERR_NULL;
    RSI_HIP(hipDeviceSynchronize());
    std::vector<float> buf((size_t)net->P * 3);
    RSI_HIP(hipMemcpy(buf.data(), net->params.as<void>(), sizeof(float) * net->P, hipMemcpyDeviceToHost));
    RSI_HIP(hipMemcpy(buf.data() + net->P, net->adam_m.as<void>(), sizeof(float) * net->P, hipMemcpyDeviceToHost));
    RSI_HIP(hipMemcpy(buf.data() + 2 * net->P, net->adam_v.as<void>(), sizeof(float) * net->P, hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) return RSI_ERR_ARG;
    const int32_t dims[4] = {net->m, net->W, net->L, 0};
    const int64_t hdr[2] = {net->P, net->step};
    bool ok = std::fwrite(&kMagic, 4, 1, f) == 1 && std::fwrite(dims, 4, 4, f) == 4 &&
              std::fwrite(hdr, 8, 2, f) == 2 && std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? RSI_OK : RSI_ERR_ARG;
}

rsi_status rsi_mlp_load(rsi_mlp *net, const char *path) {
    if (!net || !path) return RSI_ERR_NULL;
    FILE *f = std::fopen(path, "rb");
    if (!f) return RSI_ERR_ARG;
    uint32_t magic = 0;
    int32_t dims[4] = {0, 0, 0, 0};
    int64_t hdr[2] = {0, 0};
    bool ok = std::fread(&magic, 4, 1, f) == 1 && std::fread(dims, 4, 4, f) == 4 &&
              std::fread(hdr, 8, 2, f) == 2;
    ok = ok && magic == kMagic && dims[0] == net->m && dims[1] == net->W && dims[2] == net->L &&
         hdr[0] == net->P && hdr[1] >= 0;
    std::vector<float> buf;
    if (ok) {
        buf.resize((size_t)net->P * 3);
        ok = std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    }
    std::fclose(f);
    if (!ok) return RSI_ERR_ARG;
    RSI_HIP(hipDeviceSynchronize());
    RSI_HIP(hipMemcpy(net->params.as<void>(), buf.data(), sizeof(float) * net->P, hipMemcpyHostToDevice));
    RSI_HIP(hipMemcpy(net->adam_m.as<void>(), buf.data() + net->P, sizeof(float) * net->P, hipMemcpyHostToDevice));
    RSI_HIP(hipMemcpy(net->adam_v.as<void>(), buf.data() + 2 * net->P, sizeof(float) * net->P, hipMemcpyHostToDevice));
    net->step = hdr[1];
    RSI_TRY(refresh_bf16(net, nullptr));
    RSI_HIP(hipDeviceSynchronize());
    return RSI_OK;
}

rsi_status rsi_surrogate_carrier(int64_t n, const float *q, rsi_medium m1, rsi_medium m2, int mode,
                                 const float *in, float *out, void *stream) {
    if (n < 0) return RSI_ERR_SIZE;
    if (mode != 0 && mode != 1) return RSI_ERR_ARG;
    if (!(m1.c > 0.0) || !(m2.c > 0.0) || !(m1.rho > 0.0) || !(m2.rho > 0.0)) return RSI_ERR_ARG;
    if (n == 0) return RSI_OK;
    if (!q || !in || !out) return RSI_ERR_NULL;
    hipLaunchKernelGGL(carrier_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream), n,
                       q, m1.c, m2.c, mode, m1.rho * m1.c, reinterpret_cast<const float2 *>(in),
                       reinterpret_cast<float2 *>(out));
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

}  // extern "C"
