// rsi_mlp.hip -- the learned surrogate: Fourier-feature MLP trained and evaluated with
// bfloat16 MFMA GEMMs (gfx950 v_mfma_f32_32x32x16_bf16, FP32 accumulation).
//
// The forward and input-gradient GEMMs are written in the "NT" form, C[M][N] = A[M][K] .
// B[N][K]^T, with both operands contiguous along the reduction dimension, so that each lane
// of a wave reads its 8 bfloat16 MFMA operands with one 16-byte LDS read:
//   forward   Z_l  = H_{l-1} [B][K]  . W_l   [N][K]^T
//   input grad dH  = dZ_l    [B][N]  . W_l^T [K][N]^T      (transposed weight copy)
// The weight gradient dW = dZ_l^T . H_{l-1} contracts over the batch, along the rows of both
// row-major tensors; its kernel transposes its operand tiles as it reads them from LDS.  The
// epilogues fuse bias + SiLU (forward) and the SiLU derivative (input gradient) and write
// bfloat16 row-major.  Weight gradients are split over the batch and reduced in a fixed
// order (deterministic).
//
// MFMA 32x32x16 bf16 operand layout (lane l, i = 0..7 / v = 0..15; checked on gfx950 with
// small-integer operands):
//   A[l % 32][8 (l / 32) + i],  B[8 (l / 32) + i][l % 32],
//   D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
// The 32x32x16 form is used throughout: measured on MI355X with independent chains and no
// memory traffic, it sustains 2.12 PFLOP/s against 1.17 for v_mfma_f32_16x16x32_bf16.
// Every GEMM and the fused inference kernel accumulate K in the same order (steps of 16),
// so the fused and the layer-by-layer forward give the same bits.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <memory>
#include <vector>

#include "../../include/rsi_mlp.h"
#include "rsi_internal.h"

namespace rsi {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// One 32x32x16 bf16 MFMA step: acc += A (32 x 16) . B (16 x 32).
__device__ __forceinline__ f32x16 mfma32(const bf16x8 &a, const bf16x8 &b, const f32x16 &acc) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
}
// Row of element v of a 32 x 32 accumulator fragment held by lane l (its column is l % 32).
__device__ __forceinline__ int frag_row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

constexpr int kTileK = 32;  // K step of the GEMM (one MFMA)
constexpr int kMaxLayers = 16;

// SiLU and its derivative with the hardware reciprocal (1 ulp in FP32; the results are
// rounded to bfloat16 next).  exp(-z) = inf for very negative z gives s = 0 as it should.
__device__ inline float sigmoid_f(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ inline float silu_f(float z) { return z * sigmoid_f(z); }
__device__ inline float silu_grad_f(float z) {
    const float s = sigmoid_f(z);
    return s * (1.0f + z * (1.0f - s));
}

enum { EPI_FWD = 0, EPI_FWD_INFER = 1, EPI_DX = 2 };

struct GemmArgs {
    const bf16 *A;
    int64_t lda;
    const bf16 *B;
    int64_t ldb;
    int64_t M, N, K, k_per_split;
    const float *bias;  // EPI_FWD*: [N]
    float *Z;           // EPI_FWD: pre-activation out; EPI_DX: previous pre-activation in
    int64_t ldz;        // row pitch of Z, or 0: Z in the tile-native order (see below)
    bf16 *H;            // EPI_FWD*: activation out; EPI_DX: previous dZ out
    int64_t ldh;
    float *P;           // weight gradient (gemm_dw_rowmajor_kernel): partials [split][M][N]
};

// NT GEMM on one workgroup tile BM x BN: four waves in a 2 x 2 grid, each computing a
// (BM/2) x (BN/2) block as (BM/64) x (BN/64) MFMA fragments of 32 x 32.  K advances in
// steps of 32 (two MFMAs of K = 16): both operand slices are staged in LDS (rows padded to
// 40 bfloat16 = 80 bytes, so the lanes that read one 16-byte column chunk of consecutive
// rows hit disjoint bank quadruples), double-buffered, with the global loads of step k+1
// issued before the MFMAs of step k.  Bounded to 128 VGPRs (no spill), so that four
// workgroups share a CU (at the compiler's own 156-176 registers only two did: a training
// step took 1.005 ms against 0.930 with four).
template <int EPI, int BM, int BN>
__global__ void __launch_bounds__(256, 3) gemm_nt_kernel(GemmArgs g) {
    constexpr int BK = 32, LDK = BK + 8;
    constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 32, FN = WN / 32;
    constexpr int CA = BM * BK / 8 / 256, CB = BN * BK / 8 / 256;  // 16-byte chunks per thread
    static_assert(CA >= 1 && CB >= 1, "tile too small for 256 threads");
    // operand buffers, reused after the K loop as the staging tile of the bf16 output
    constexpr int LDT = BN + 8;  // staging row pitch (bf16)
    constexpr int kOps = 2 * (BM + BN) * LDK * 2, kStage = BM * LDT * 2;
    __shared__ __attribute__((aligned(16))) char smem[kOps > kStage ? kOps : kStage];
    auto sA = reinterpret_cast<bf16 (*)[BM][LDK]>(smem);
    auto sB = reinterpret_cast<bf16 (*)[BN][LDK]>(smem + 2 * BM * LDK * 2);
    auto st = reinterpret_cast<bf16 (*)[LDT]>(smem);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
    const int64_t kb = (int64_t)blockIdx.z * g.k_per_split;
    const int64_t ke = (kb + g.k_per_split < g.K) ? kb + g.k_per_split : g.K;
    const int nk = (int)((ke - kb) / BK);
    bf16x8 ra[CA], rb[CB];
    auto gload = [&](int64_t k) {
#pragma unroll
        for (int i = 0; i < CA; ++i) {
            const int c = tid + 256 * i;
            ra[i] = *reinterpret_cast<const bf16x8 *>(g.A + (m0 + (c >> 2)) * g.lda + k + (c & 3) * 8);
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int c = tid + 256 * i;
            rb[i] = *reinterpret_cast<const bf16x8 *>(g.B + (n0 + (c >> 2)) * g.ldb + k + (c & 3) * 8);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < CA; ++i) {
            const int c = tid + 256 * i;
            *reinterpret_cast<bf16x8 *>(&sA[buf][c >> 2][(c & 3) * 8]) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int c = tid + 256 * i;
            *reinterpret_cast<bf16x8 *>(&sB[buf][c >> 2][(c & 3) * 8]) = rb[i];
        }
    };
    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
    const int r = lane & 31, kq = (lane >> 5) * 8;
    if (nk > 0) {
        gload(kb);
        sstore(0);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) gload(kb + (int64_t)(kt + 1) * BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            bf16x8 af[FM], bfr[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                af[i] = *reinterpret_cast<const bf16x8 *>(&sA[buf][wm * WM + 32 * i + r][ks + kq]);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                bfr[j] = *reinterpret_cast<const bf16x8 *>(&sB[buf][wn * WN + 32 * j + r][ks + kq]);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = mfma32(af[i], bfr[j], acc[i][j]);
        }
        // the other buffer was last read before the barrier that ended step kt - 1
        if (kt + 1 < nk) sstore(buf ^ 1);
        __syncthreads();
    }
    const int cn = lane & 31;
    // Tile-native order of Z: fragment (i, j) of wave w holds 16 values per lane, stored as
    // four 16-byte chunks at ((tile * 4 + w) * FM * FN + i * FN + j) * 1024 + lane * 16, so
    // the forward GEMM writes and the input-gradient GEMM of the same shape reads it with
    // fully coalesced accesses.
    const int64_t tile = (int64_t)blockIdx.x * gridDim.y + blockIdx.y;
    auto znat = [&](int i, int j) { return ((tile * 4 + wave) * (FM * FN) + i * FN + j) * 1024 + lane * 16; };
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int nl = wn * WN + 32 * j + cn, mbl = wm * WM + 32 * i;
            const int64_t n = n0 + nl;
            f32x16 zin;
            if constexpr (EPI == EPI_DX) {
                if (g.ldz == 0) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const f32x4 z4 = *reinterpret_cast<const f32x4 *>(g.Z + znat(i, j) + 4 * c);
#pragma unroll
                        for (int e = 0; e < 4; ++e) zin[4 * c + e] = z4[e];
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < 16; ++v) zin[v] = g.Z[(m0 + mbl + frag_row(v, lane)) * g.ldz + n];
                }
            }
            f32x16 zout;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                float val;
                if constexpr (EPI == EPI_DX) {
                    val = acc[i][j][v] * silu_grad_f(zin[v]);
                } else {
                    const float z = acc[i][j][v] + g.bias[n];
                    zout[v] = z;
                    val = silu_f(z);
                }
                st[mbl + frag_row(v, lane)][nl] = (bf16)val;
            }
            if constexpr (EPI == EPI_FWD) {
                if (g.ldz == 0) {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        *reinterpret_cast<f32x4 *>(g.Z + znat(i, j) + 4 * c) =
                            f32x4{zout[4 * c], zout[4 * c + 1], zout[4 * c + 2], zout[4 * c + 3]};
                } else {
#pragma unroll
                    for (int v = 0; v < 16; ++v) g.Z[(m0 + mbl + frag_row(v, lane)) * g.ldz + n] = zout[v];
                }
            }
        }
    __syncthreads();
    // row-major output in 16-byte chunks
    for (int c = tid; c < BM * BN / 8; c += 256) {
        const int row = c / (BN / 8), c8 = (c - row * (BN / 8)) * 8;
        *reinterpret_cast<bf16x8 *>(g.H + (m0 + row) * g.ldh + n0 + c8) =
            *reinterpret_cast<const bf16x8 *>(&st[row][c8]);
    }
}

// Weight gradient from the row-major tensors: P[split][m][n] = sum over the split's rows k
// of A[k][m] B[k][n] (A = dZ [rows][M], B = H [rows][N]), the contraction running along the
// rows of both.  Tiles of 32 rows are copied to LDS as they are (16-byte loads and stores),
// and each MFMA operand -- 8 consecutive k of one m -- is read with two transposing LDS reads
// (ds_read_b64_tr_b16): within a group of 16 lanes, lane j points at row kb + j / 4, columns
// c + 4 (j % 4) .. + 3, and lane i receives rows kb .. kb + 3 of column c + i.  The operands,
// and so the products and their order, are those of an NT GEMM over transposed copies of dZ
// and H, without those copies being written.
// Row pitch of the LDS tiles: 32 mod 64 elements (an odd multiple of 16 banks), so one read's
// 8 rows x 64 bytes cover the 64 banks twice (the minimum for 512 bytes).
typedef short s16x4 __attribute__((ext_vector_type(4)));
template <int BM, int BN>
__global__ void __launch_bounds__(256, 3) gemm_dw_rowmajor_kernel(GemmArgs g) {
    constexpr int BK = 32, PA = BM + 32, PB = BN + 32;
    constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 32, FN = WN / 32;
    constexpr int CA = BM * BK / 8 / 256, CB = BN * BK / 8 / 256;  // 16-byte chunks per thread
    static_assert(CA >= 1 && CB >= 1, "tile too small for 256 threads");
    static_assert(PA % 64 == 32 && PB % 64 == 32, "row pitch 32 mod 64");
    __shared__ __attribute__((aligned(16))) bf16 sA[2][BK][PA];
    __shared__ __attribute__((aligned(16))) bf16 sB[2][BK][PB];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
    const int64_t kb = (int64_t)blockIdx.z * g.k_per_split;
    const int64_t ke = (kb + g.k_per_split < g.K) ? kb + g.k_per_split : g.K;
    const int nk = (int)((ke - kb) / BK);
    bf16x8 ra[CA], rb[CB];
    auto gload = [&](int64_t k) {
#pragma unroll
        for (int i = 0; i < CA; ++i) {
            const int c = tid + 256 * i;
            ra[i] = *reinterpret_cast<const bf16x8 *>(g.A + (k + c / (BM / 8)) * g.lda + m0 + (c % (BM / 8)) * 8);
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int c = tid + 256 * i;
            rb[i] = *reinterpret_cast<const bf16x8 *>(g.B + (k + c / (BN / 8)) * g.ldb + n0 + (c % (BN / 8)) * 8);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < CA; ++i) {
            const int c = tid + 256 * i;
            *reinterpret_cast<bf16x8 *>(&sA[buf][c / (BM / 8)][(c % (BM / 8)) * 8]) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int c = tid + 256 * i;
            *reinterpret_cast<bf16x8 *>(&sB[buf][c / (BN / 8)][(c % (BN / 8)) * 8]) = rb[i];
        }
    };
    // lane's place in its group of 16: the row offset and the column offset of its read
    const int grp = lane >> 4, jr = (lane & 15) >> 2, jc = 4 * (lane & 3);
    const int colg = 16 * (grp & 1), kq = 8 * (grp >> 1);
    auto tread = [&](const bf16 *p) {
        const s16x4 v = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
            (__attribute__((address_space(3))) s16x4 *)(p));
        return v;
    };
    auto operand = [&](const bf16 *tile, int pitch, int col, int ks) {
        // rows ks + kq .. + 7 of column col + lane % 32
        const bf16 *p = tile + (ks + kq + jr) * pitch + col + colg + jc;
        const bf16x4 lo = __builtin_bit_cast(bf16x4, tread(p));
        const bf16x4 hi = __builtin_bit_cast(bf16x4, tread(p + 4 * pitch));
        return (bf16x8)__builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    };
    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
    if (nk > 0) {
        gload(kb);
        sstore(0);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) gload(kb + (int64_t)(kt + 1) * BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            bf16x8 af[FM], bfr[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) af[i] = operand(&sA[buf][0][0], PA, wm * WM + 32 * i, ks);
#pragma unroll
            for (int j = 0; j < FN; ++j) bfr[j] = operand(&sB[buf][0][0], PB, wn * WN + 32 * j, ks);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = mfma32(af[i], bfr[j], acc[i][j]);
        }
        // the other buffer was last read before the barrier that ended step kt - 1
        if (kt + 1 < nk) sstore(buf ^ 1);
        __syncthreads();
    }
    const int cn = lane & 31;
    float *p = g.P + (int64_t)blockIdx.z * g.M * g.N;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int64_t n = n0 + wn * WN + 32 * j + cn;
            const int64_t mb = m0 + wm * WM + 32 * i;
#pragma unroll
            for (int v = 0; v < 16; ++v) p[(mb + frag_row(v, lane)) * g.N + n] = acc[i][j][v];
        }
}

// Fourier features of the normalised query: h0 = [sin 2 pi u, cos 2 pi u], u = B v.
struct Box {
    double lo[5], inv[5];  // v = 2 (q - lo) * inv - 1, inv = 1 / (hi - lo)
};

// One thread: 8 consecutive features of one row.  Block = 64 rows (x) x 4 chunks of 8
// features (y); grid.y covers the m/32 groups of chunks.  Writes the row-major features
// (16-byte stores).  Rows past n get u = 0.
__global__ void __launch_bounds__(256) features_kernel(int64_t n, int64_t Mp, int m,
                                                       const float *__restrict__ q, Box box,
                                                       const float *__restrict__ Bff,
                                                       bf16 *__restrict__ H0, int64_t ld) {
    const int64_t b = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int j0 = (blockIdx.y * 4 + threadIdx.y) * 8;
    if (b >= Mp || j0 >= m) return;
    // the 8 features' 40 matrix entries loaded before any FMA (rows past n have v = 0, so
    // their u is +0 as when the sum is skipped)
    float bf[40];
#pragma unroll
    for (int k = 0; k < 40; ++k) bf[k] = Bff[j0 * 5 + k];
    // v and u = B v, and u's reduction to one revolution, in FP64: the bf16 features then
    // round the same values the FP64 reference rounds (|u| reaches tens of revolutions)
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const bool live = b < n;
    if (live)
#pragma unroll
        for (int c = 0; c < 5; ++c) v[c] = 2.0 * ((double)q[b * 5 + c] - box.lo[c]) * box.inv[c] - 1.0;
    bf16x8 hs, hc;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        double u = 0.0;
#pragma unroll
        for (int c = 0; c < 5; ++c) u = fma((double)bf[t * 5 + c], v[c], u);
        const float ph = (float)(u - floor(u));  // sin(2 pi u): revolutions
        hs[t] = (bf16)__builtin_amdgcn_sinf(ph);
        hc[t] = (bf16)__builtin_amdgcn_cosf(ph);
    }
    *reinterpret_cast<bf16x8 *>(H0 + b * ld + j0) = hs;
    *reinterpret_cast<bf16x8 *>(H0 + b * ld + m + j0) = hc;
}

// Fused inference: features, every hidden layer and the head for a tile of BM rows in
// one workgroup, the activations kept in LDS between layers (bf16, rows padded by 8 so the
// 16 lanes that read one MFMA fragment hit disjoint banks) and the weights streamed from
// L2 straight into MFMA operands, from a copy in fragment order (one contiguous 1 KB block
// per MFMA operand).  Four waves split each layer's W output columns.  The MFMA takes the
// weights as its A operand and the activations as B, so each lane ends with four
// consecutive output columns of one row per four accumulator elements and stores them as
// one 8-byte write.  The arithmetic is that of the unfused path step for step -- the same
// bf16 features, the same products summed over K in the same order, bias + SiLU in FP32
// rounded to bf16, the head's FMAs in feature order -- so the two give the same bits; only
// the HBM round trips of the activations are gone.
struct FusedArgs {
    const float *q;
    int64_t n;
    Box box;
    const float *Bff;
    int m;  // Fourier frequencies (F = 2m features)
    int L;
    const bf16 *Wl[kMaxLayers];  // bf16 weights in MFMA fragment order (cast_weight_kernel)
    const float *bl[kMaxLayers];
    int in_dim[kMaxLayers];
    const float *Wo, *bo;
    float *y;
};

// Two workgroups per CU (the register budget that leaves: about 200 VGPRs at width 256, no
// spill); a single wave per SIMD left every load wait exposed (122 against 81 us for 65536
// rows of a 5 x 256 net).  On gfx950 the VALU work of one wave does not hide behind the
// MFMAs of the other wave on its SIMD: a micro-benchmark of this MFMA pattern runs 2.0
// PFLOP/s without an epilogue and 1.43 with a SiLU after every layer, also when the two waves
// are in opposite phases or keep their accumulators in AGPRs.  So every instruction besides
// the MFMAs costs time, and the kernel is written to issue few: the small operands sit in
// LDS, the first K step of a layer adds into the constant 0 instead of cleared registers.
// Measured on the 7 x 256 net at 65536 rows: 103 us with row-major weights and one-element
// activation stores, 91 us with the weights in fragment order, 84-86 us with the transposed
// output as well, 74-79 us with the LDS operands and the constant-0 first step.  Timing
// copies with one part removed (79.6 us with all parts): LDS operand reads 3.3 us, weight
// loads 4.3 (both 11.2), barriers 1.3, features 3.6, head 1.2, SiLU 9.7.  Not kept,
// measured: 8 waves per workgroup (64 rows each, 4 waves per SIMD) 91-138 us; 256-row tiles
// 117 us; LDS operand reads half a step ahead of their MFMAs, a start delay for every other
// workgroup, and a warm-up load of all weights into L2, no change; two 64-row tiles per
// workgroup taking turns (one tile's MFMAs interleaved with the other's bias + SiLU, each
// tile streaming the weights) 88 us; two activation buffers (one barrier per layer) 101 us
// at 64 rows (LDS then allows two workgroups per CU instead of four; 64-row tiles with one
// buffer: 84 us).
// BM rows per workgroup: 128 when the grid still fills the chip, 32 or 64 for calls of a
// few thousand rows, where one workgroup's latency is the call's time.
template <int W, int BM>
__global__ void __launch_bounds__(256, 2) mlp_infer_fused_kernel(FusedArgs a) {
    // waves split the W output columns into CG groups and the BM rows into RG groups, each
    // wave a (BM/RG) x (W/CG) block of 32 x 32 fragments; waves past CG * RG (width 64 with
    // 32-row tiles) only take part in the features, the barriers and the head
    constexpr int LDA = W + 8, TPR = 256 / BM;
    constexpr int CG = (W / 32 < 4) ? W / 32 : 4;
    constexpr int RG = (BM / 32 < 4 / CG) ? BM / 32 : 4 / CG;
    constexpr int WN = W / CG, WMr = BM / RG, FN = WN / 32, FM = WMr / 32;
    static_assert(FN >= 1 && FM >= 1, "fragments of 32 x 32");
    static_assert(BM == 32 || BM == 64 || BM == 128, "32, 64 or 128 rows");
    __shared__ __attribute__((aligned(16))) bf16 act[BM][LDA];
    // small operands every wave reads at the same addresses, staged once so that no
    // per-iteration global load stalls a phase: the Fourier matrix in FP64 while the features
    // are computed, then the head's weights and biases; and the current layer's biases
    constexpr int NSIDE = W / 2 * 5, NBF = (NSIDE + 255) / 256, NWO = (2 * W + 2 + 255) / 256;
    __shared__ __attribute__((aligned(16))) double side[NSIDE];
    __shared__ __attribute__((aligned(16))) float bias_s[W];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t r0 = (int64_t)blockIdx.x * BM;
    const bool mma = wave < CG * RG;
    const int wc = wave % CG, wr = wave / CG;
    const int r = lane & 31, kq = (lane >> 5) * 8;
    // B fragments straight from L2, from the weights in fragment order: the operand of one
    // MFMA (32 columns x 16 inputs) is 1 KB, lane l's 16 bytes at l * 16, so a wave's load
    // is one contiguous block; blocks of a 32-column group follow each other along K
    // (32 x K elements per group).  Two register sets take turns (no copies between them);
    // every K step issues the loads of the step after it, the last step of a layer those
    // of the next layer's first step (the last layer's re-reads its final slice), and the
    // first layer's first slice is loaded before the features.  The loop body is
    // straight-line, so each step's MFMAs wait only for the loads issued one step earlier.
    auto wrow = [&](int l) { return a.Wl[l] + (int64_t)wc * FN * 32 * a.in_dim[l] + 8 * lane; };
    bf16x8 b0[2][FN], b1[2][FN];
    auto load = [&](bf16x8 (&b)[2][FN], const bf16 *p, int64_t ld) {  // p: slice start, ld: K
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int j = 0; j < FN; ++j)
                b[s][j] = *reinterpret_cast<const bf16x8 *>(p + (int64_t)32 * j * ld + 512 * s);
    };
    // Every global load below is unconditional (indices clamped into their arrays), so
    // that the compiler can count the loads still in flight instead of draining them all.
    // (Rows past n compute u = +0, as they do in features_kernel; their outputs are
    // dropped.)  m <= W / 2: the features fit the width.
    const int row = tid & (BM - 1), part = tid / BM;
    const int64_t b = r0 + row;
    const bool live = b < a.n;
    float bff[NBF], wo[NWO], qv[5];
#pragma unroll
    for (int t = 0; t < NBF; ++t) bff[t] = a.Bff[min(tid + 256 * t, 5 * a.m - 1)];
#pragma unroll
    for (int c = 0; c < 5; ++c) qv[c] = a.q[(live ? b : a.n - 1) * 5 + c];
#pragma unroll
    for (int t = 0; t < NWO; ++t) {
        const int i = min(tid + 256 * t, 2 * W + 1);
        wo[t] = i < 2 * W ? a.Wo[i] : a.bo[i - 2 * W];
    }
    float bcur = a.bl[0][tid & (W - 1)];  // biases of the layer about to run
    if (mma) load(b0, wrow(0), a.in_dim[0]);
#pragma unroll
    for (int t = 0; t < NBF; ++t)
        if (tid + 256 * t < NSIDE) side[tid + 256 * t] = (double)bff[t];
    __syncthreads();
    {
        // features as in features_kernel: TPR threads per row, each a share of the frequencies
        double v[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) v[c] = live ? 2.0 * ((double)qv[c] - a.box.lo[c]) * a.box.inv[c] - 1.0 : 0.0;
        const int mh = a.m / TPR;  // m is a multiple of 32
#pragma unroll 4
        for (int j = part * mh; j < (part + 1) * mh; ++j) {
            double u = 0.0;
#pragma unroll
            for (int c = 0; c < 5; ++c) u = fma(side[j * 5 + c], v[c], u);
            const float ph = (float)(u - floor(u));
            act[row][j] = (bf16)__builtin_amdgcn_sinf(ph);
            act[row][a.m + j] = (bf16)__builtin_amdgcn_cosf(ph);
        }
    }
    __syncthreads();
    for (int l = 0; l < a.L; ++l) {
        const int K = a.in_dim[l];
        // this layer's biases, loaded a layer ahead (the previous layer's readers are past
        // the barrier that ended it), and the next layer's load; the wait for them here is
        // the wait for this layer's first weights.  Before the first layer the head's weights
        // and biases take the place of the Fourier matrix, which the features are done with.
        if (tid < W) bias_s[tid] = bcur;
        bcur = a.bl[min(l + 1, a.L - 1)][tid & (W - 1)];
        if (l == 0) {
            float *wos = reinterpret_cast<float *>(side);  // Wo [2][W], then bo [2]
#pragma unroll
            for (int t = 0; t < NWO; ++t)
                if (tid + 256 * t < 2 * W + 2) wos[tid + 256 * t] = wo[t];
        }
        f32x16 acc[FM][FN];  // set by the first K step (waves without MFMA work never read it)
        if (mma) {
            const bf16 *Wl = wrow(l);
            const bool more = l + 1 < a.L;
            const bf16 *Wn = more ? wrow(l + 1) : Wl + 32 * (K - 32);
            const int64_t Kn = more ? a.in_dim[l + 1] : K;
            // first: the layer's first K step, whose MFMAs take the constant 0 as their
            // accumulator input (no register clearing; the same sums)
            auto step = [&](const bf16x8 (&b)[2][FN], int k, auto first) {
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int i = 0; i < FM; ++i) {
                        const bf16x8 af =
                            *reinterpret_cast<const bf16x8 *>(&act[wr * WMr + 32 * i + r][k + 16 * s + kq]);
#pragma unroll
                        for (int j = 0; j < FN; ++j) {
                            if constexpr (decltype(first)::value)
                                acc[i][j] = mfma32(b[s][j], af, s == 0 ? f32x16{} : acc[i][j]);
                            else
                                acc[i][j] = mfma32(b[s][j], af, acc[i][j]);
                        }
                    }
            };
            // (the scheduling barriers keep the compiler from sinking the loads below the MFMAs)
            for (int k0 = 0; k0 < K; k0 += 64) {  // K is a multiple of 64
                load(b1, Wl + 32 * (k0 + 32), K);
                __builtin_amdgcn_sched_barrier(0);
                if (k0 == 0) step(b0, k0, std::true_type{});
                else step(b0, k0, std::false_type{});
                __builtin_amdgcn_sched_barrier(0);
                const bool last = k0 + 64 >= K;
                load(b0, last ? Wn : Wl + 32 * (k0 + 64), last ? Kn : K);
                __builtin_amdgcn_sched_barrier(0);
                step(b1, k0 + 32, std::false_type{});
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        __syncthreads();  // every wave has read this layer's input
        if (mma) {
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // the transposed fragment: lane l holds row l % 32 and, for q, the four
                    // consecutive columns 8 q + 4 (l / 32) .. + 3 (elements 4 q .. 4 q + 3)
                    const int n = wc * WN + 32 * j + 8 * q + 4 * (lane >> 5);
                    const float4 bias = *reinterpret_cast<const float4 *>(&bias_s[n]);
#pragma unroll
                    for (int i = 0; i < FM; ++i) {
                        bf16x4 h;
                        h[0] = (bf16)silu_f(acc[i][j][4 * q + 0] + bias.x);
                        h[1] = (bf16)silu_f(acc[i][j][4 * q + 1] + bias.y);
                        h[2] = (bf16)silu_f(acc[i][j][4 * q + 2] + bias.z);
                        h[3] = (bf16)silu_f(acc[i][j][4 * q + 3] + bias.w);
                        *reinterpret_cast<bf16x4 *>(&act[wr * WMr + 32 * i + r][n]) = h;
                    }
                }
        }
        __syncthreads();
    }
    // head as in head_kernel: one (row, output) per thread, FMAs in feature order
    if (tid >= 2 * BM) return;
    const int hrow = tid >> 1, k = tid & 1;
    const float *wos = reinterpret_cast<const float *>(side);  // Wo [2][W], then bo [2]
    float yk = 0.0f;
    for (int f = 0; f < W; f += 8) {  // 16-byte LDS reads, the FMAs still in feature order
        const bf16x8 h = *reinterpret_cast<const bf16x8 *>(&act[hrow][f]);
        const float4 w0 = *reinterpret_cast<const float4 *>(&wos[k * W + f]);
        const float4 w1 = *reinterpret_cast<const float4 *>(&wos[k * W + f + 4]);
        const float w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) yk = fmaf(w[e], (float)h[e], yk);
    }
    yk += wos[2 * W + k];
    if (r0 + hrow < a.n) a.y[2 * (r0 + hrow) + k] = yk;
}

// Output layer (FP32), one thread per row: y = Wo h + bo.  Training (t != NULL): the
// row's loss and output gradient dy = (y - t)/n go to dyl [Mp][3] (0 for padding rows)
// and dZ_L = bf16((dy Wo) * silu'(Z_L)), row-major.  Wo is read through the constant address
// space (scalar loads: every lane uses the same weights).
typedef const __attribute__((address_space(4))) float *ConstF;

__global__ void __launch_bounds__(256) head_kernel(int64_t n, int64_t Mp, int W,
                                                   const bf16 *__restrict__ H,
                                                   const float *__restrict__ Z, const float *Wo_,
                                                   const float *bo_, const float *__restrict__ t,
                                                   float *__restrict__ y, bf16 *__restrict__ dZ,
                                                   float *__restrict__ dyl) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= Mp) return;
    const ConstF Wo = (ConstF)Wo_, bo = (ConstF)bo_;
    const bf16 *h = H + row * W;
    float y0 = 0.0f, y1 = 0.0f;
    for (int f0 = 0; f0 < W; f0 += 64) {  // W is a multiple of 64: 8 loads ahead of their FMAs
        bf16x8 hb[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) hb[k] = *reinterpret_cast<const bf16x8 *>(h + f0 + 8 * k);
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int f = f0 + 8 * k;
                y0 = fmaf(Wo[f + u], (float)hb[k][u], y0);
                y1 = fmaf(Wo[W + f + u], (float)hb[k][u], y1);
            }
    }
    y0 += bo[0];
    y1 += bo[1];
    const bool live = row < n;
    if (live && y) {
        y[2 * row] = y0;
        y[2 * row + 1] = y1;
    }
    if (!t) return;
    float d0 = 0.0f, d1 = 0.0f, loss = 0.0f;
    if (live) {
        const float e0 = y0 - t[2 * row], e1 = y1 - t[2 * row + 1];
        d0 = e0 / (float)n;
        d1 = e1 / (float)n;
        loss = 0.5f * (e0 * e0 + e1 * e1) / (float)n;
    }
    dyl[3 * row] = d0;
    dyl[3 * row + 1] = d1;
    dyl[3 * row + 2] = loss;
    const float *z = Z + row * W;
    bf16 *dz = dZ + row * W;
    for (int f0 = 0; f0 < W; f0 += 32) {  // 32 pre-activations loaded ahead of their use
        f32x4 zb[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) zb[k] = *reinterpret_cast<const f32x4 *>(z + f0 + 4 * k);
#pragma unroll
        for (int k8 = 0; k8 < 4; ++k8) {
            const int f = f0 + 8 * k8;
            bf16x8 o;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float dh = d0 * Wo[f + u] + d1 * Wo[W + f + u];
                o[u] = (bf16)(dh * silu_grad_f(zb[2 * k8 + u / 4][u % 4]));
            }
            *reinterpret_cast<bf16x8 *>(dz + f) = o;
        }
    }
}

// Head gradients, first level, over the rows of chunk blockIdx.x (kHeadRows rows):
// part[chunk][c] for c < 2W = sum of dy_k h_f (c = k W + f), then dy_0, dy_1 and the loss.
// The chunk's dy and losses are staged in LDS; a thread covers 8 features (16-byte
// loads) of every 4th row, and the 4 row groups are added in a fixed order.
constexpr int kHeadRows = 256;
__global__ void __launch_bounds__(256) head_grad_kernel(int64_t Mp, int W, const bf16 *__restrict__ H,
                                                        const float *__restrict__ dyl, float *__restrict__ part) {
    __shared__ float sdy[kHeadRows * 3];
    __shared__ float sacc[4][2 * 1024];
    const int64_t r0 = (int64_t)blockIdx.x * kHeadRows;
    const int rows = (int)((Mp - r0 < kHeadRows) ? Mp - r0 : kHeadRows);
    for (int i = threadIdx.x; i < rows * 3; i += 256) sdy[i] = dyl[3 * r0 + i];
    __syncthreads();
    const int nfc = W / 8, tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int fc = tx; fc < nfc; fc += 64) {
        float a0[8], a1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a0[u] = a1[u] = 0.0f;
        // rows ty, ty + 4, ... in order, eight rows' loads issued ahead of their FMAs
        int r = ty;
        for (; r + 28 < rows; r += 32) {
            bf16x8 hb[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) hb[k] = *reinterpret_cast<const bf16x8 *>(H + (r0 + r + 4 * k) * W + 8 * fc);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float d0 = sdy[3 * (r + 4 * k)], d1 = sdy[3 * (r + 4 * k) + 1];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    a0[u] = fmaf(d0, (float)hb[k][u], a0[u]);
                    a1[u] = fmaf(d1, (float)hb[k][u], a1[u]);
                }
            }
        }
        for (; r < rows; r += 4) {
            const bf16x8 h = *reinterpret_cast<const bf16x8 *>(H + (r0 + r) * W + 8 * fc);
            const float d0 = sdy[3 * r], d1 = sdy[3 * r + 1];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                a0[u] = fmaf(d0, (float)h[u], a0[u]);
                a1[u] = fmaf(d1, (float)h[u], a1[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            sacc[ty][8 * fc + u] = a0[u];
            sacc[ty][W + 8 * fc + u] = a1[u];
        }
    }
    __syncthreads();
    const int C = 2 * W + 3;
    float *out = part + (int64_t)blockIdx.x * C;
    for (int c = threadIdx.x; c < 2 * W; c += 256) {
        float v = sacc[0][c];
        for (int g = 1; g < 4; ++g) v += sacc[g][c];
        out[c] = v;
    }
    if (threadIdx.x < 3) {
        float v = 0.0f;
        for (int r = 0; r < rows; ++r) v += sdy[3 * r + threadIdx.x];
        out[2 * W + threadIdx.x] = v;
    }
}

// Fixed-order column sums: out[c] = sum_r in[r * ld + c] (r < R), in FP64.  A block covers
// 64 columns with 4 row groups (rows = g mod 4) whose sums are added in order.
__global__ void __launch_bounds__(256) colsum_kernel(const float *__restrict__ in, int64_t R, int64_t C,
                                                     int64_t ld, float *__restrict__ out) {
    __shared__ double sh[4][64];
    const int cx = threadIdx.x & 63, ry = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * 64 + cx;
    double acc = 0.0;
    if (c < C) {
        int64_t r = ry;
        for (; r + 60 < R; r += 64) {  // 16 rows of the group loaded ahead of their additions
            float x[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) x[u] = in[(r + 4 * u) * ld + c];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc += (double)x[u];
        }
        for (; r < R; r += 4) acc += (double)in[r * ld + c];
    }
    sh[ry][cx] = acc;
    __syncthreads();
    if (ry == 0 && c < C) out[c] = (float)(((sh[0][cx] + sh[1][cx]) + sh[2][cx]) + sh[3][cx]);
}

// Bias-gradient segments: the batch is cut into kRowSumSegs interleaved segments whose sums
// are added in order (bias_node_kernel, bias_tree_kernel, then the column sums).
constexpr int kRowSumSegs = 16;

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
                                                          bf16 *__restrict__ Wb, bf16 *__restrict__ WTb,
                                                          bf16 *__restrict__ Wf32) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (int64_t)O * I) return;
    const int o = (int)(k / I), i = (int)(k - (int64_t)o * I);
    const bf16 v = (bf16)Wf[k];
    Wb[k] = v;
    WTb[(int64_t)i * O + o] = v;
    // fragment order for the fused inference kernel: the B operand of one 32x32x16 MFMA
    // (32 output columns x 16 inputs) as 64 lanes x 8 contiguous values, lane = o % 32 +
    // 32 ((i % 16) / 8), blocks ordered by input slice within each 32-column group
    const int c = o >> 5, t = i >> 4, lane = (o & 31) + 32 * ((i & 15) >> 3);
    Wf32[(((int64_t)c * (I >> 4) + t) * 64 + lane) * 8 + (i & 7)] = v;
}

// Bias gradient from the row-major dZ [rows][W], for each column o and segment sg: 256
// leaves t, each the sum in order of the 8-row chunks (sg * 256 + t) * 8 + 2048 kRowSumSegs i,
// meet in the halving tree sh[t] += sh[t + w], w = 128 .. 1 (the order of a reduction with one
// workgroup per row of a transposed copy of dZ, 256 threads each summing its chunks).
// Here a thread takes the 8 leaves t5 + 32 i of one column and adds them as the tree's first
// three levels do (w = 128, 64, 32), giving node [kRowSumSegs][32][W]; bias_tree_kernel
// finishes the last five levels.  Block (64 columns, 4 values of t5); grid (W / 64,
// kRowSumSegs, 8).
__global__ void __launch_bounds__(256) bias_node_kernel(const bf16 *__restrict__ dZ, int64_t rows, int W,
                                                        float *__restrict__ node) {
    const int o = blockIdx.x * 64 + threadIdx.x, sg = blockIdx.y, t5 = blockIdx.z * 4 + threadIdx.y;
    constexpr int64_t kStride = (int64_t)kRowSumSegs * 256 * 8;
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = 0.0f;
    for (int64_t c = 0; c < rows; c += kStride) {
        bf16 x[8][8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t k = ((int64_t)sg * 256 + t5 + 32 * i) * 8 + c;
            const int64_t kl = k < rows ? k : rows - 8;  // loads unconditional, so all are in flight
#pragma unroll
            for (int u = 0; u < 8; ++u) x[i][u] = dZ[(kl + u) * W + o];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t k = ((int64_t)sg * 256 + t5 + 32 * i) * 8 + c;
            if (k < rows)
#pragma unroll
                for (int u = 0; u < 8; ++u) v[i] += (float)x[i][u];
        }
    }
    const float a0 = v[0] + v[4], a1 = v[1] + v[5], a2 = v[2] + v[6], a3 = v[3] + v[7];  // w = 128
    node[((int64_t)sg * 32 + t5) * W + o] = (a0 + a2) + (a1 + a3);                     // w = 64, 32
}

// The tree's last levels (w = 16 .. 1) over node [kRowSumSegs][32][W] -> part [kRowSumSegs][W],
// for every layer in one launch (layer blockIdx.z: node and part at its offsets); grid
// (W / 64, kRowSumSegs, layers), 64 threads.
__global__ void __launch_bounds__(64) bias_tree_kernel(const float *__restrict__ node_all, int W,
                                                       float *__restrict__ part_all) {
    const int o = blockIdx.x * 64 + threadIdx.x, sg = blockIdx.y;
    const float *node = node_all + (int64_t)blockIdx.z * kRowSumSegs * 32 * W;
    float *part = part_all + (int64_t)blockIdx.z * kRowSumSegs * W;
    float n[32];
#pragma unroll
    for (int t = 0; t < 32; ++t) n[t] = node[((int64_t)sg * 32 + t) * W + o];
#pragma unroll
    for (int w = 16; w > 0; w >>= 1)
#pragma unroll
        for (int t = 0; t < w; ++t) n[t] += n[t + w];
    part[(int64_t)sg * W + o] = n[0];
}

// One training step's Adam update fused with the reductions that finish its gradients:
// parameter i reads the partial sums the backward kernels left for it (weight-gradient
// splits, bias-gradient segments, head chunks) and adds them in colsum_kernel's order, so
// the update equals that of separate colsum, adam and weight-cast launches bit for bit; a
// weight's new value then goes to its three bf16 copies as cast_weight_kernel writes them.
struct AdamArgs {
    int64_t P;
    float *p, *m, *v;
    float lr, c1, c2;
    int L, W;
    int64_t offW[kMaxLayers], offb[kMaxLayers];
    int in_dim[kMaxLayers];
    const float *dw[kMaxLayers];  // [splits][W][in_dim[l]] weight-gradient partials
    const float *bp[kMaxLayers];  // [kRowSumSegs][W] bias-gradient segments
    bf16 *Wb[kMaxLayers], *WTb[kMaxLayers], *Wfr[kMaxLayers];
    int64_t splits;
    const float *head;  // [chunks][2W + 3]: dWo, dbo, loss
    int64_t chunks, offWo;
};

// colsum_kernel's sum of one column: rows r = g mod 4 in order, in FP64, then the four
// groups.  Rows are loaded 16 at a time ahead of their additions (one thread walks the whole
// column, so the loads in flight are what hides the memory latency).
__device__ inline float colsum_at(const float *__restrict__ in, int64_t R, int64_t ld, int64_t c) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t r = 0;
    for (; r + 16 <= R; r += 16) {
        float x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) x[u] = in[(r + u) * ld + c];
#pragma unroll
        for (int u = 0; u < 16; u += 4) {
            a0 += (double)x[u];
            a1 += (double)x[u + 1];
            a2 += (double)x[u + 2];
            a3 += (double)x[u + 3];
        }
    }
    for (; r < R; ++r) {
        const double x = (double)in[r * ld + c];
        const int gq = (int)(r & 3);
        if (gq == 0) a0 += x;
        else if (gq == 1) a1 += x;
        else if (gq == 2) a2 += x;
        else a3 += x;
    }
    return (float)(((a0 + a1) + a2) + a3);
}

__global__ void __launch_bounds__(256) adam_fused_kernel(AdamArgs a) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.P) return;
    float g;
    int lw = -1;  // the layer whose weight i is, or -1
    int64_t e = 0;
    if (i >= a.offWo) {
        g = colsum_at(a.head, a.chunks, 2 * (int64_t)a.W + 3, i - a.offWo);
    } else {
        int l = 0;
        while (l + 1 < a.L && i >= a.offW[l + 1]) ++l;
        if (i < a.offb[l]) {
            lw = l;
            e = i - a.offW[l];
            g = colsum_at(a.dw[l], a.splits, (int64_t)a.W * a.in_dim[l], e);
        } else {
            g = colsum_at(a.bp[l], kRowSumSegs, a.W, i - a.offb[l]);
        }
    }
    const float mi = 0.9f * a.m[i] + 0.1f * g;
    const float vi = 0.999f * a.v[i] + 0.001f * g * g;
    a.m[i] = mi;
    a.v[i] = vi;
    const float pn = a.p[i] - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + 1e-8f);
    a.p[i] = pn;
    if (lw >= 0) {
        const int I = a.in_dim[lw], o = (int)(e / I), ii = (int)(e - (int64_t)o * I);
        const bf16 bv = (bf16)pn;
        a.Wb[lw][e] = bv;
        a.WTb[lw][(int64_t)ii * a.W + o] = bv;
        const int c = o >> 5, t = ii >> 4, lane = (o & 31) + 32 * ((ii & 15) >> 3);
        a.Wfr[lw][(((int64_t)c * (I >> 4) + t) * 64 + lane) * 8 + (ii & 7)] = bv;
    }
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

// Ray-model frame: every block first forms s = RMS of the n_ref reference values (a few
// hundred loads, fixed order), then maps its points.
__global__ void __launch_bounds__(256) ray_frame_kernel(int64_t n, const float2 *__restrict__ pr,
                                                        int64_t n_ref, const float2 *__restrict__ ref,
                                                        double sigma, double clip, int mode,
                                                        const float2 *__restrict__ in,
                                                        float2 *__restrict__ out) {
    __shared__ double part[256];
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < n_ref; k += 256) {
        const float2 v = ref[k];
        acc += (double)v.x * v.x + (double)v.y * v.y;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    const double s = sqrt(part[0] / (double)n_ref);
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float2 p = pr[i], a = in[i];
    const double mag = fmax(sqrt((double)p.x * p.x + (double)p.y * p.y), 1e-30 * s);
    const double ux = p.x / mag, uy = p.y / mag, ss = s * sigma;
    if (mode == 0) {  // (in - p_ray) conj(u) / (s sigma)
        const double dx = (double)a.x - p.x, dy = (double)a.y - p.y;
        double yr = (dx * ux + dy * uy) / ss, yi = (dy * ux - dx * uy) / ss;
        const double ym = sqrt(yr * yr + yi * yi);
        if (clip > 0.0 && ym > clip) {
            yr *= clip / ym;
            yi *= clip / ym;
        }
        out[i] = make_float2((float)yr, (float)yi);
    } else {          // p_ray + s sigma in u
        out[i] = make_float2((float)(p.x + ss * (a.x * ux - a.y * uy)),
                             (float)(p.y + ss * (a.x * uy + a.y * ux)));
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
    std::vector<std::unique_ptr<rsi::DeviceBuffer>> Wfr;      // bf16 weights in MFMA fragment order
    std::vector<std::unique_ptr<rsi::DeviceBuffer>> H, Z;    // activations [L+1], pre-acts [L]
    rsi::DeviceBuffer dZ[2], dwpart, headpart, bpart, bnode, dyl, lossbuf;
    std::vector<int64_t> dwoff;  // per layer, into dwpart (each layer keeps its partials)
    int dw_splits = 1;
};

namespace rsi {

static int64_t pad64(int64_t n) { return (n + 63) / 64 * 64; }

template <int BM, int BN>
static void launch_gemm(int epi, const GemmArgs &g, int splits, hipStream_t s) {
    const dim3 grid((unsigned)(g.M / BM), (unsigned)(g.N / BN), (unsigned)splits);
    switch (epi) {
        case EPI_FWD: hipLaunchKernelGGL((gemm_nt_kernel<EPI_FWD, BM, BN>), grid, dim3(256), 0, s, g); break;
        case EPI_FWD_INFER:
            hipLaunchKernelGGL((gemm_nt_kernel<EPI_FWD_INFER, BM, BN>), grid, dim3(256), 0, s, g);
            break;
        default: hipLaunchKernelGGL((gemm_nt_kernel<EPI_DX, BM, BN>), grid, dim3(256), 0, s, g); break;
    }
}

// Tile: 128 rows / columns where the dimension allows it (M, N are multiples of 64 and
// the K range of every split a multiple of 32, checked by the callers' padding).
static rsi_status gemm(int epi, const GemmArgs &g, int splits, hipStream_t s) {
    if (g.M % 64 || g.N % 64 || g.k_per_split % 32 || (g.K % g.k_per_split)) return RSI_ERR_SIZE;
    const bool bm = g.M % 128 == 0, bn = g.N % 128 == 0;
    if (bm && bn) launch_gemm<128, 128>(epi, g, splits, s);
    else if (bm) launch_gemm<128, 64>(epi, g, splits, s);
    else if (bn) launch_gemm<64, 128>(epi, g, splits, s);
    else launch_gemm<64, 64>(epi, g, splits, s);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

// The weight-gradient GEMM on row-major operands (gemm_dw_rowmajor_kernel), tiles as gemm().
static rsi_status gemm_dw(const GemmArgs &g, int splits, hipStream_t s) {
    if (g.M % 64 || g.N % 64 || g.k_per_split % 32 || (g.K % g.k_per_split)) return RSI_ERR_SIZE;
    const bool bm = g.M % 128 == 0, bn = g.N % 128 == 0;
    const dim3 grid((unsigned)(g.M / (bm ? 128 : 64)), (unsigned)(g.N / (bn ? 128 : 64)), (unsigned)splits);
    if (bm && bn) hipLaunchKernelGGL((gemm_dw_rowmajor_kernel<128, 128>), grid, dim3(256), 0, s, g);
    else if (bm) hipLaunchKernelGGL((gemm_dw_rowmajor_kernel<128, 64>), grid, dim3(256), 0, s, g);
    else if (bn) hipLaunchKernelGGL((gemm_dw_rowmajor_kernel<64, 128>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((gemm_dw_rowmajor_kernel<64, 64>), grid, dim3(256), 0, s, g);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

static rsi_status refresh_bf16(rsi_mlp *net, hipStream_t s) {
    for (int l = 0; l < net->L; ++l) {
        const int O = net->W, I = net->in_dim[l];
        const int64_t cnt = (int64_t)O * I;
        hipLaunchKernelGGL(cast_weight_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                           net->params.as<float>() + net->offW[l], O, I, net->Wb[l]->as<bf16>(),
                           net->WTb[l]->as<bf16>(), net->Wfr[l]->as<bf16>());
        RSI_HIP(hipGetLastError());
    }
    return RSI_OK;
}

// Forward through the hidden layers (training keeps Z and nothing else is needed).
static rsi_status forward_hidden(rsi_mlp *net, int64_t n, const float *q, bool train, hipStream_t s) {
    const int64_t Mp = pad64(n);
    // m is a multiple of 32: m / 32 groups of 4 chunks of 8 features
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)(Mp / 64), (unsigned)(net->m / 32)), dim3(64, 4), 0, s,
                       n, Mp, net->m, q, net->box, net->Bff.as<float>(), net->H[0]->as<bf16>(),
                       (int64_t)net->F);
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
        g.ldz = (l + 1 == net->L) ? net->W : 0;  // tile-native except for the head's input
        g.H = net->H[l + 1]->as<bf16>();
        g.ldh = net->W;
        RSI_TRY(gemm(train ? EPI_FWD : EPI_FWD_INFER, g, 1, s));
    }
    return RSI_OK;
}

// The gradients into grad, or (grad == NULL) only their partial sums -- per-layer weight
// splits, bias segments, head chunks -- for the fused Adam step to add; the loss is summed
// either way.  Returns the number of weight-gradient splits used.
static rsi_status backward(rsi_mlp *net, int64_t n, const float *t, float *grad, float *loss,
                           hipStream_t s, int *splits_used = nullptr) {
    const int64_t Mp = pad64(n);
    const int W = net->W;
    const float *params = net->params.as<float>();
    hipLaunchKernelGGL(head_kernel, dim3((unsigned)((Mp + 255) / 256)), dim3(256), 0, s, n, Mp, W,
                       net->H[net->L]->as<bf16>(), net->Z[net->L - 1]->as<float>(), params + net->offWo,
                       params + net->offbo, t, (float *)nullptr, net->dZ[0].as<bf16>(), net->dyl.as<float>());
    RSI_HIP(hipGetLastError());
    // head partials [chunks][2W + 3] -> dWo, dbo (columns 0..2W+1) and the loss (column 2W+2)
    {
        const int64_t C = 2 * W + 3, chunks = (Mp + kHeadRows - 1) / kHeadRows;
        hipLaunchKernelGGL(head_grad_kernel, dim3((unsigned)chunks), dim3(256), 0, s, Mp, W,
                           net->H[net->L]->as<bf16>(), net->dyl.as<float>(), net->headpart.as<float>());
        RSI_HIP(hipGetLastError());
        float *lossdst = loss ? loss : net->lossbuf.as<float>();
        if (grad) {
            hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((C - 1 + 63) / 64)), dim3(256), 0, s,
                               net->headpart.as<float>(), chunks, C - 1, C, grad + net->offWo);
            RSI_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(256), 0, s, net->headpart.as<float>() + (C - 1), chunks,
                           (int64_t)1, C, lossdst);
        RSI_HIP(hipGetLastError());
    }
    int cur = 0;
    for (int l = net->L - 1; l >= 0; --l) {
        const int I = net->in_dim[l];
        // the weight gradient and the bias gradient read dZ_l [Mp][W] and H_l [Mp][I] as the
        // epilogues that produced them wrote them (row-major)
        int splits = net->dw_splits;
        while (splits > 1 && (Mp % ((int64_t)splits * kTileK) != 0)) splits >>= 1;
        if (splits_used) *splits_used = splits;
        float *dwp = net->dwpart.as<float>() + net->dwoff[l];
        GemmArgs g{};
        g.A = net->dZ[cur].as<bf16>();
        g.lda = W;
        g.B = net->H[l]->as<bf16>();
        g.ldb = I;
        g.M = W;
        g.N = I;
        g.K = Mp;
        g.k_per_split = Mp / splits;
        g.P = dwp;
        RSI_TRY(gemm_dw(g, splits, s));
        const int64_t C = (int64_t)W * I;
        if (grad) {
            hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((C + 63) / 64)), dim3(256), 0, s, dwp,
                               (int64_t)splits, C, C, grad + net->offW[l]);
            RSI_HIP(hipGetLastError());
        }
        // bias gradient: column sums of dZ, in kRowSumSegs segments added in order
        // (the trees' last levels run for all layers after the loop)
        hipLaunchKernelGGL(bias_node_kernel, dim3((unsigned)(W / 64), (unsigned)kRowSumSegs, 8u), dim3(64, 4), 0, s,
                           net->dZ[cur].as<bf16>(), Mp, W,
                           net->bnode.as<float>() + (int64_t)l * kRowSumSegs * 32 * W);
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
        d.ldz = 0;  // written tile-native by the forward GEMM of the same shape
        d.H = net->dZ[cur ^ 1].as<bf16>();
        d.ldh = I;
        RSI_TRY(gemm(EPI_DX, d, 1, s));
        cur ^= 1;
    }
    hipLaunchKernelGGL(bias_tree_kernel, dim3((unsigned)(W / 64), (unsigned)kRowSumSegs, (unsigned)net->L), dim3(64),
                       0, s, net->bnode.as<float>(), W, net->bpart.as<float>());
    RSI_HIP(hipGetLastError());
    if (grad)
        for (int l = 0; l < net->L; ++l) {
            hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((W + 63) / 64)), dim3(256), 0, s,
                               net->bpart.as<float>() + (int64_t)l * kRowSumSegs * W, (int64_t)kRowSumSegs,
                               (int64_t)W, (int64_t)W, grad + net->offb[l]);
            RSI_HIP(hipGetLastError());
        }
    return RSI_OK;
}

static rsi_status check_batch(const rsi_mlp *net, int64_t n, const void *q) {
    if (!net) return RSI_ERR_NULL;
    if (n < 0 || n > net->max_batch) return RSI_ERR_SIZE;
    if (n > 0 && !q) return RSI_ERR_NULL;
    return RSI_OK;
}

template <int BM>
static void launch_fused(int W, dim3 grid, dim3 block, hipStream_t s, const FusedArgs &a) {
    if (W == 256) hipLaunchKernelGGL((mlp_infer_fused_kernel<256, BM>), grid, block, 0, s, a);
    else if (W == 128) hipLaunchKernelGGL((mlp_infer_fused_kernel<128, BM>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((mlp_infer_fused_kernel<64, BM>), grid, block, 0, s, a);
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
        net->Wfr.emplace_back(new DeviceBuffer);
        RSI_TRY(net->Wb.back()->alloc(sizeof(bf16) * width * net->in_dim[l]));
        RSI_TRY(net->WTb.back()->alloc(sizeof(bf16) * width * net->in_dim[l]));
        RSI_TRY(net->Wfr.back()->alloc(sizeof(bf16) * width * net->in_dim[l]));
        net->Z.emplace_back(new DeviceBuffer);
        RSI_TRY(net->Z.back()->alloc(sizeof(float) * Mp * width));
    }
    for (int l = 0; l <= depth; ++l) {
        net->H.emplace_back(new DeviceBuffer);
        RSI_TRY(net->H.back()->alloc(sizeof(bf16) * Mp * (l == 0 ? F : width)));
    }
    for (int k = 0; k < 2; ++k) {
        RSI_TRY(net->dZ[k].alloc(sizeof(bf16) * Mp * maxdim));
    }
    // weight-gradient split over the batch: at least 256 rows per split, at most 128
    // splits (measured best for 256 x 256 weights at a batch of 65536: 512 workgroups of
    // 512-row K ranges, a training step 0.809 ms against 0.836 with 64 splits and 0.887
    // with 256, where the partials' traffic outgrows what the extra workgroups gain)
    int max_splits = 128;
    if (const char *e = std::getenv("RSI_MLP_DW_SPLITS")) {  // tuning sweeps: a power of two
        const int v = std::atoi(e);
        if (v >= 1 && v <= 4096 && (v & (v - 1)) == 0) max_splits = v;
    }
    int splits = 1;
    while (splits < max_splits && Mp / (splits * 2) >= 256) splits *= 2;
    net->dw_splits = splits;
    // every layer's partials stay until the fused Adam step adds them
    size_t dw_elems = 0;
    for (int l = 0; l < depth; ++l) {
        net->dwoff.push_back((int64_t)dw_elems);
        dw_elems += (size_t)splits * width * net->in_dim[l];
    }
    RSI_TRY(net->dwpart.alloc(sizeof(float) * dw_elems));
    RSI_TRY(net->headpart.alloc(sizeof(float) * (size_t)((Mp + kHeadRows - 1) / kHeadRows) * (2 * width + 3)));
    RSI_TRY(net->bpart.alloc(sizeof(float) * kRowSumSegs * (size_t)width * depth));
    RSI_TRY(net->bnode.alloc(sizeof(float) * kRowSumSegs * 32 * (size_t)width * depth));
    RSI_TRY(net->dyl.alloc(sizeof(float) * 3 * (size_t)Mp));
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
    // one fused launch when the features fit the hidden width (RSI_MLP_FUSED=0: layer by layer)
    const char *fe = std::getenv("RSI_MLP_FUSED");
    const bool fused = !(fe && fe[0] == '0' && fe[1] == 0);
    if (fused && net->F <= net->W && (net->W == 64 || net->W == 128 || net->W == 256)) {
        FusedArgs a{};
        a.q = q;
        a.n = n;
        a.box = net->box;
        a.Bff = net->Bff.as<float>();
        a.m = net->m;
        a.L = net->L;
        const float *params = net->params.as<float>();
        for (int l = 0; l < net->L; ++l) {
            a.Wl[l] = net->Wfr[l]->as<bf16>();
            a.bl[l] = params + net->offb[l];
            a.in_dim[l] = net->in_dim[l];
        }
        a.Wo = params + net->offWo;
        a.bo = params + net->offbo;
        a.y = y;
        // 128-row tiles while they give two workgroups per CU, 64 down to 128 workgroups,
        // 32 below (15625 rows: 57, 41 and 50 us for 128, 64 and 32; RSI_MLP_FUSED_ROWS:
        // 32, 64 or 128 forces one)
        int rows = n >= 128 * 512 ? 128 : n >= 64 * 128 ? 64 : 32;
        if (const char *fr = std::getenv("RSI_MLP_FUSED_ROWS")) {
            const int v = std::atoi(fr);
            if (v == 32 || v == 64 || v == 128) rows = v;
        }
        const dim3 grid((unsigned)((n + rows - 1) / rows)), block(256);
        if (rows == 128) launch_fused<128>(net->W, grid, block, s, a);
        else if (rows == 64) launch_fused<64>(net->W, grid, block, s, a);
        else launch_fused<32>(net->W, grid, block, s, a);
        RSI_HIP(hipGetLastError());
        return RSI_OK;
    }
    RSI_TRY(forward_hidden(net, n, q, false, s));
    const int64_t Mp = pad64(n);
    const float *params = net->params.as<float>();
    hipLaunchKernelGGL(head_kernel, dim3((unsigned)((Mp + 255) / 256)), dim3(256), 0, s, n, Mp, net->W,
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
    // RSI_MLP_ADAM_FUSED=0: the gradients summed by colsum_kernel, then adam_kernel and the
    // weight casts as separate launches (the same arithmetic in the same order)
    const char *fe = std::getenv("RSI_MLP_ADAM_FUSED");
    if (fe && fe[0] == '0' && fe[1] == 0) {
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
    int splits = 1;
    RSI_TRY(backward(net, n, t, nullptr, loss, s, &splits));
    net->step += 1;
    AdamArgs a{};
    a.P = net->P;
    a.p = net->params.as<float>();
    a.m = net->adam_m.as<float>();
    a.v = net->adam_v.as<float>();
    a.lr = lr;
    a.c1 = (float)(1.0 - std::pow(0.9, (double)net->step));
    a.c2 = (float)(1.0 - std::pow(0.999, (double)net->step));
    a.L = net->L;
    a.W = net->W;
    for (int l = 0; l < net->L; ++l) {
        a.offW[l] = net->offW[l];
        a.offb[l] = net->offb[l];
        a.in_dim[l] = net->in_dim[l];
        a.dw[l] = net->dwpart.as<float>() + net->dwoff[l];
        a.bp[l] = net->bpart.as<float>() + (int64_t)l * kRowSumSegs * net->W;
        a.Wb[l] = net->Wb[l]->as<bf16>();
        a.WTb[l] = net->WTb[l]->as<bf16>();
        a.Wfr[l] = net->Wfr[l]->as<bf16>();
    }
    a.splits = splits;
    a.head = net->headpart.as<float>();
    a.chunks = (pad64(n) + kHeadRows - 1) / kHeadRows;
    a.offWo = net->offWo;
    hipLaunchKernelGGL(adam_fused_kernel, dim3((unsigned)((net->P + 255) / 256)), dim3(256), 0, s, a);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
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

rsi_status rsi_surrogate_ray_frame(int64_t n, const float *p_ray, int64_t n_ref, const float *ref,
                                   double sigma, double clip, int mode, const float *in,
                                   float *out, void *stream) {
    if (n < 0 || n_ref < 0) return RSI_ERR_SIZE;
    if (mode != 0 && mode != 1) return RSI_ERR_ARG;
    if (!(sigma > 0.0) || !std::isfinite(sigma) || !std::isfinite(clip)) return RSI_ERR_ARG;
    if (n == 0) return RSI_OK;
    if (n_ref < 1 || (n + 255) / 256 > 0x7fffffff) return RSI_ERR_SIZE;
    if (!p_ray || !ref || !in || !out) return RSI_ERR_NULL;
    hipLaunchKernelGGL(ray_frame_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream),
                       n, reinterpret_cast<const float2 *>(p_ray), n_ref,
                       reinterpret_cast<const float2 *>(ref), sigma, clip, mode,
                       reinterpret_cast<const float2 *>(in), reinterpret_cast<float2 *>(out));
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

}  // extern "C"
