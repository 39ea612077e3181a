// rsi_device.h -- device-side building blocks of the pair sum, shared by the one-shot
// kernels (rsi_pairsum.hip) and the persistent batched kernels (rsi_batched.hip).
//
// Pair sum (eqs. 3 and 7 under eq. 16):
//   phi(P_i) = sum_j s'_j K(P_i, Q_j),  s'_j = -(1/2pi) w_j s_j (folded at preparation)
//   monopole K = e^{ikr}/r,  dipole K = cos(theta)(ik - 1/r) e^{ikr}/r.
#pragma once

#include "rsi_internal.h"

namespace rsi {

constexpr int kSub = 64;  // sources per FP32 partial block before the compensated fold

// Sources per iteration of the FP32 inner loop (independent pair chains per wave).
#ifndef RSI_SRC_UNROLL
#define RSI_SRC_UNROLL 1
#endif

// The phase argument p_ref + (r - r_ref + psi lambda)/lambda lies within 1 + R/lambda + 1/4
// revolutions of zero (|r - r_ref| <= |Q_j - C| <= R, the set's half diagonal).
// v_sin_f32 / v_cos_f32 take revolutions and reduce arguments up to 256 in magnitude
// themselves (measured on gfx950: max abs error 1.22e-7 over [-256, 256], the same as
// over [-1, 1]), so below that bound the explicit fract is dropped.  The FMA result is
// rounded at the argument's magnitude in both cases, so the values are the same.
__device__ __forceinline__ bool phase_in_sin_range(double radius, double inv_lam) {
    return radius * inv_lam < 250.0;
}

// Per-target constants of the FP32 path (see rsi_pairsum.hip for the derivation).
template <int KIND, int TPL>
struct TargetsF {
    float dmx[TPL], dmy[TPL], dmz[TPL];  // -2 (P - C)
    float rr2[TPL], rr[TPL], p0[TPL];    // r_ref^2, r_ref, frac(r_ref f / c)
    float ht[TPL];                       // n.(P - C) (dipole)
};

// FP64 set-up of TPL targets per lane: tbase + u * kBlock, u < TPL.  Targets past the
// end repeat the last one (their results are never stored).
template <int KIND, int TPL>
__device__ __forceinline__ void setup_targets_f32(TargetsF<KIND, TPL> &T, const double *tx,
                                                  const double *ty, const double *tz,
                                                  int64_t n_tgt, int64_t tbase, double ax,
                                                  double ay, double az, double inv_lam,
                                                  double nx, double ny, double nz) {
#pragma unroll
    for (int u = 0; u < TPL; ++u) {
        int64_t i = tbase + (int64_t)u * kBlock;
        if (i >= n_tgt) i = n_tgt - 1;
        const double dx = tx[i] - ax, dy = ty[i] - ay, dz = tz[i] - az;
        const double rr2 = dx * dx + dy * dy + dz * dz;
        const double rr = sqrt(rr2);
        double ph = rr * inv_lam;  // reference phase in revolutions, reduced in FP64
        ph -= floor(ph);
        T.dmx[u] = (float)(-2.0 * dx);
        T.dmy[u] = (float)(-2.0 * dy);
        T.dmz[u] = (float)(-2.0 * dz);
        T.rr2[u] = (float)rr2;
        T.rr[u] = (float)rr;
        T.p0[u] = (float)ph;
        T.ht[u] = (float)(nx * dx + ny * dy + nz * dz);
    }
}

// Accumulators of one lane's field point.  Monopole: A1 = sum a_j e^{i phi_j}/r_j.
// Dipole: A1 = sum a_j c_j e^{i phi_j}/r_j^2 and A2 = sum a_j c_j e^{i phi_j}/r_j^3 with
// c_j = n.(P - Q_j) (1 for planar sources, whose c_j is the field point's height and is
// applied once at the end), so that the field is c (ik A1 - A2): the factor (ik - 1/r)
// of eq. 7 splits into a per-target constant ik and one more power of 1/r.
struct AccF {
    float r1, i1, r2, i2;
};

// One source against the lane's TPL targets.  `s` is wave-uniform (SGPRs).  PLANAR:
// every source lies in the plane z = C_z with normal +z (interface samples), so
// e_z = 0 and n.e_j = 0, and the z terms drop out.
//
// The source strength enters as a signed magnitude a_j and a phase offset psi_j held as
// the path length psi_j lambda, which is added to r - r_ref by the FMA that finishes
// the path difference; the complex multiply by the strength disappears.
template <int KIND, int TPL, bool PLANAR, bool FRACT, class Rec>
__device__ __forceinline__ void pair_f32(const TargetsF<KIND, TPL> &T, const Rec &s,
                                         float ilam, AccF (&A)[TPL]) {
#pragma unroll
    for (int u = 0; u < TPL; ++u) {
        float t = T.dmx[u] * s.ex;
        t = fmaf(T.dmy[u], s.ey, t);
        if constexpr (!PLANAR) t = fmaf(T.dmz[u], s.ez, t);
        const float q = t + s.es2;                           // r^2 - r_ref^2
        const float r2 = T.rr2[u] + q;
        // |r^2|: the source modifier of v_rsq is free; r^2 < 0 only by rounding for a
        // field point on a source, which the FP32 path excludes
        const float ir = __builtin_amdgcn_rsqf(fabsf(r2));    // 1/r
        const float den = fmaf(r2, ir, T.rr[u]);              // r + r_ref
        const float d = fmaf(q, __builtin_amdgcn_rcpf(den), s.psil);  // r - r_ref + psi lambda
        float ph = fmaf(d, ilam, T.p0[u]);  // revolutions
        if constexpr (FRACT) ph = __builtin_amdgcn_fractf(ph);
        const float cs = __builtin_amdgcn_cosf(ph);
        const float sn = __builtin_amdgcn_sinf(ph);
        const float m0 = ir * s.a;                            // a / r
        if constexpr (KIND == RSI_MONOPOLE) {
            A[u].r1 = fmaf(m0, cs, A[u].r1);
            A[u].i1 = fmaf(m0, sn, A[u].i1);
        } else {
            float m1 = m0 * ir;                               // a / r^2
            if constexpr (!PLANAR) m1 *= T.ht[u] - s.h;       // times n.(P - Q)
            const float m2 = m1 * ir;
            A[u].r1 = fmaf(m1, cs, A[u].r1);
            A[u].i1 = fmaf(m1, sn, A[u].i1);
            A[u].r2 = fmaf(m2, cs, A[u].r2);
            A[u].i2 = fmaf(m2, sn, A[u].i2);
        }
    }
}

// Source records are read through the constant address space: no kernel writes them,
// and loads from that space may go through the scalar cache, so a wave-uniform record
// index gives s_load even when the pointer itself came from memory (batched items).
typedef const __attribute__((address_space(4))) SrcRecF *SrcRecConstPtr;

// Sum of sources [j0, j1): FP32 blocks of kSub sources folded into a Kahan-compensated
// running sum (mre, mim with compensation cre, cim).  For the dipole each block is
// combined to ik A1 - A2 before the fold, and the planar height is applied at the end.
template <int KIND, int TPL, bool PLANAR, bool FRACT>
__device__ __forceinline__ void sum_range_f32(const TargetsF<KIND, TPL> &T,
                                              const SrcRecF *recs, int64_t j0,
                                              int64_t j1, float ilam, float k,
                                              float (&mre)[TPL], float (&mim)[TPL]) {
    const SrcRecConstPtr rec = (SrcRecConstPtr)recs;
    float cre[TPL], cim[TPL];
#pragma unroll
    for (int u = 0; u < TPL; ++u) mre[u] = mim[u] = cre[u] = cim[u] = 0.0f;
    for (int64_t jb = j0; jb < j1; jb += kSub) {
        const int64_t je = (jb + kSub < j1) ? jb + kSub : j1;
        AccF A[TPL];
#pragma unroll
        for (int u = 0; u < TPL; ++u) A[u].r1 = A[u].i1 = A[u].r2 = A[u].i2 = 0.0f;
        if (je - jb == kSub) {
#pragma unroll RSI_SRC_UNROLL
            for (int jj = 0; jj < kSub; ++jj) pair_f32<KIND, TPL, PLANAR, FRACT>(T, rec[jb + jj], ilam, A);
        } else {
            for (int64_t j = jb; j < je; ++j) pair_f32<KIND, TPL, PLANAR, FRACT>(T, rec[j], ilam, A);
        }
#pragma unroll
        for (int u = 0; u < TPL; ++u) {
            float br = A[u].r1, bi = A[u].i1;
            if constexpr (KIND == RSI_DIPOLE) {  // ik A1 - A2
                br = fmaf(-k, A[u].i1, -A[u].r2);
                bi = fmaf(k, A[u].r1, -A[u].i2);
            }
            float y = br - cre[u];
            float t = mre[u] + y;
            cre[u] = (t - mre[u]) - y;
            mre[u] = t;
            y = bi - cim[u];
            t = mim[u] + y;
            cim[u] = (t - mim[u]) - y;
            mim[u] = t;
        }
    }
    if constexpr (KIND == RSI_DIPOLE && PLANAR) {
#pragma unroll
        for (int u = 0; u < TPL; ++u) {
            mre[u] *= T.ht[u];
            mim[u] *= T.ht[u];
        }
    }
}

// Few field points: the 64 lanes of a wave take every 64th source of [j0, j1) for the
// same field point (records by vector loads), each lane folds its blocks as above, and
// the lane sums are combined by a fixed shuffle tree (bitwise repeatable).
template <int KIND, bool PLANAR, bool FRACT>
__device__ __forceinline__ void sum_lanes_f32(const TargetsF<KIND, 1> &T,
                                              const SrcRecF *__restrict__ rec, int64_t j0,
                                              int64_t j1, float ilam, float k, float &mre,
                                              float &mim) {
    const int lane = threadIdx.x & 63;
    float cre = 0.0f, cim = 0.0f;
    mre = mim = 0.0f;
    for (int64_t jb = j0 + lane; jb < j1; jb += 64 * kSub) {
        const int64_t je = (jb + 64 * kSub < j1) ? jb + 64 * kSub : j1;
        AccF A[1];
        A[0].r1 = A[0].i1 = A[0].r2 = A[0].i2 = 0.0f;
        for (int64_t j = jb; j < je; j += 64) {
            const SrcRecF s = rec[j];
            pair_f32<KIND, 1, PLANAR, FRACT>(T, s, ilam, A);
        }
        float br = A[0].r1, bi = A[0].i1;
        if constexpr (KIND == RSI_DIPOLE) {  // ik A1 - A2
            br = fmaf(-k, A[0].i1, -A[0].r2);
            bi = fmaf(k, A[0].r1, -A[0].i2);
        }
        float y = br - cre;
        float t = mre + y;
        cre = (t - mre) - y;
        mre = t;
        y = bi - cim;
        t = mim + y;
        cim = (t - mim) - y;
        mim = t;
    }
    if constexpr (KIND == RSI_DIPOLE && PLANAR) {
        mre *= T.ht[0];
        mim *= T.ht[0];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        mre += __shfl_xor(mre, off);
        mim += __shfl_xor(mim, off);
    }
}

// FP64: sources [j0, j1) against one target, same operations as the definition.
template <int KIND>
__device__ __forceinline__ void sum_range_f64(double px, double py, double pz,
                                              const SrcRecD *__restrict__ rec, int64_t j0,
                                              int64_t j1, double inv_lam, double k, double nx,
                                              double ny, double nz, double &mre, double &mim) {
    double cre = 0.0, cim = 0.0;
    mre = mim = 0.0;
    for (int64_t jb = j0; jb < j1; jb += kSub) {
        const int64_t je = (jb + kSub < j1) ? jb + kSub : j1;
        double are = 0.0, aim = 0.0;
        for (int64_t j = jb; j < je; ++j) {
            const SrcRecD s = rec[j];
            const double dx = px - s.x, dy = py - s.y, dz = pz - s.z;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r < kRMin) continue;  // singular pair: contributes nothing
            const double ir = 1.0 / r;
            double ph = r * inv_lam;
            ph -= rint(ph);  // k r in revolutions, reduced to [-1/2, 1/2]
            double sn, cs;
            sincospi(2.0 * ph, &sn, &cs);
            double gr, gi;
            if constexpr (KIND == RSI_MONOPOLE) {
                gr = cs * ir;
                gi = sn * ir;
            } else {
                const double g2 = (nx * dx + ny * dy + nz * dz) * ir * ir;
                const double al = -g2 * ir, be = g2 * k;
                gr = al * cs - be * sn;
                gi = al * sn + be * cs;
            }
            are += s.sre * gr - s.sim * gi;
            aim += s.sre * gi + s.sim * gr;
        }
        double y = are - cre, t = mre + y;
        cre = (t - mre) - y;
        mre = t;
        y = aim - cim;
        t = mim + y;
        cim = (t - mim) - y;
        mim = t;
    }
}

}  // namespace rsi
