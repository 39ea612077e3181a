// rsi_ray.hip -- the ray-tracing model of Sec. 2.2: eq. (12) under the estimator of
// eq. (16), with the conserved slowness of eq. (14) found per (sample, field point).
//
//   phi(P) = -(v0 / 2pi) sum_j w_j T_j e^{i omega t_j} / A_j
//
// Only the transducer is sampled.  The ray from sample Q_j to field point P crosses the
// planes z = zif[0] < ... < zif[n-1]; layer l (l = 0..n) has slowness S_l = 1/c_l and the
// ray's vertical extent in it is h_l (h_0 = zif[0] - z_j, inner layers their thickness,
// h_n = z_P - zif[n-1]).  With eta_l(C) = sqrt(S_l^2 - C^2) (so c_l eta_l = cos theta_l)
// the horizontal slowness C solves eq. (14) through the stack,
//   F(C) = C S1(C) - rho = 0,   S1 = sum_l h_l / eta_l,   rho = horizontal |P - Q_j|,
// and then
//   t   = C rho + sum_l h_l eta_l                 (= sum_l D_l / c_l, D_l = h_l S_l / eta_l)
//   A   = eta_0 sqrt(S1 S3),   S3 = sum_l h_l S_l^2 / eta_l^3 = F'(C)
//         (eq. 12's two spreading factors: sum_l (c_l/c_0) D_l = S_0 S1 and
//          sum_l (c_l/c_0)(cos^2 theta_0 / cos^2 theta_l) D_l = (eta_0^2 / S_0) S3)
//   T   = prod_l 2 rho_l eta_l / (rho_{l+1} eta_l + rho_l eta_{l+1})   (eq. 11 per plane)
// F is increasing and convex in C on [0, min_l S_l), so Newton steps from the right
// never leave the interval and a step from the left is only kept inside it.
//
// FP32 path.  Per field point, once and in FP64: the reference ray from the anchor C_A
// of the transducer samples (bounding-box centre) to P -- its root C_0, the eta_l^0 =
// eta_l(C_0), the travel time t_0 and the reference phases frac(f_q t_0) in revolutions.
// Per pair, in FP32, with e = Q_j - C_A:
//   q    = |e_h|^2 - 2 (P - C_A)_h . e_h        ( = rho^2 - rho_0^2 )
//   drho = q / (rho + rho_0)                    ( = rho - rho_0, no cancellation )
//   C    = Newton from the linear predictor C_0 + (drho + e_z C_0/eta_0^0) / F'_0
//   dt   = C_0 drho - e_z eta_0^0 + (C - C_0) [rho - (C + C_0) sum_l h_l / (eta_l + eta_l^0)]
// dt = t - t_0 exactly (the two terms are t(C_0) on the pair's geometry minus t_0, and
// t(C) - t(C_0) on the pair's geometry); none of it cancels, and t is stationary in C at
// the root, so the root's rounding enters the phase only at second order.  The phase is
// frac(f_q t_0) + f_q dt revolutions.  Sums run in FP32 blocks of 64 sources folded into a
// Kahan-compensated total; source ranges may be split across workgroups and the partial
// sums are reduced in a fixed order.
//
// FP64 path: every pair in FP64 -- the root by Newton inside a shrinking bracket to the
// last bit, t from the formula above, phase reduced to revolutions and evaluated with
// sincospi.
//
// Pairs whose source is on or below the first plane, or whose field point is on or above
// the last plane, contribute nothing.  With no plane the model is eq. (3), the monopole
// pair sum of rsi_pairsum.hip.
#include <cfloat>
#include <cmath>
#include <cstdlib>
#include <type_traits>

#include "rsi_device.h"

namespace rsi {
namespace {

constexpr int kRayMaxIf = 8;               // planes per call
constexpr int kRayMaxL = kRayMaxIf + 1;    // layers
constexpr int kRayFB = 8;                  // frequencies per launch
constexpr int kRaySub = 64;                // sources per FP32 block before the fold
constexpr int kRayMaxIt = 12;              // FP32 Newton evaluations per pair (bound)

// One transducer sample of the FP32 path (read with wave-uniform scalar loads).
struct alignas(32) RayRecF {
    float ex, ey, ez, eh2;   // offset from the anchor; |horizontal offset|^2
    float a;                 // -(1/2pi) w_j v0 2 rho_0 S_f (see ray_pair_f32)
    float h0, hf0, hf0S2;    // h_0 = zif[0] - z_j (positive: samples below it have a = 0),
                             // S_f h_0 and S_f h_0 S_0^2
};
// FP64 path: absolute position and folded strength.
struct alignas(32) RayRecD {
    double x, y, z, a;
};
typedef const __attribute__((address_space(4))) RayRecF *RayRecFPtr;
typedef const __attribute__((address_space(4))) RayRecD *RayRecDPtr;

// Layer constants, passed by value (kernel arguments, read with scalar loads).
struct RayStack {
    double S2d[kRayMaxL];    // S_l^2
    double hd[kRayMaxL];     // thickness of inner layer l (1 <= l <= n-1)
    double rhod[kRayMaxL];   // densities
    double zif0, zlast;      // first and last plane
    double Smind;            // min_l S_l
    float S2[kRayMaxL], h[kRayMaxL], hf[kRayMaxL], hfS2[kRayMaxL], rho[kRayMaxL], rho2[kRayMaxL];
    float dS2[kRayMaxL];     // S_l^2 - S_f^2 >= 0, S_f the smallest slowness (fastest layer)
    float Sf;                // S_f
};
struct RayFreqs {
    double f[kRayFB];
    float ff[kRayFB];
    int n;                   // valid entries (the rest repeat the last)
};

// Anchor = centre of the samples' bounding box; radius = its half diagonal.
__device__ inline void ray_anchor(const double *__restrict__ partials, double &ax, double &ay,
                                  double &az, double &radius) {
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    for (int b = 0; b < kBBoxBlocks; ++b)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fmin(lo[k], partials[b * 6 + k]);
            hi[k] = fmax(hi[k], partials[b * 6 + 3 + k]);
        }
    ax = 0.5 * (lo[0] + hi[0]);
    ay = 0.5 * (lo[1] + hi[1]);
    az = 0.5 * (lo[2] + hi[2]);
    const double sx = hi[0] - lo[0], sy = hi[1] - lo[1], sz = hi[2] - lo[2];
    radius = 0.5 * sqrt(sx * sx + sy * sy + sz * sz);
}

// A sample on or below the first plane has no ray: its strength is zero (decided here
// in FP64, as in the definition).
__global__ void __launch_bounds__(256) ray_prep_f32_kernel(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ w, double v0, double zif0,
    double rho0, double S20, double Sf, const double *__restrict__ partials,
    double *__restrict__ anchor_out, RayRecF *__restrict__ rec) {
    double ax, ay, az, radius;
    ray_anchor(partials, ax, ay, az, radius);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        anchor_out[0] = ax;
        anchor_out[1] = ay;
        anchor_out[2] = az;
        anchor_out[3] = radius;
    }
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const float ex = (float)(x[j] - ax), ey = (float)(y[j] - ay), ez = (float)(z[j] - az);
    const double dex = ex, dey = ey;  // the rounded offset is the sample's position
    RayRecF r;
    r.ex = ex;
    r.ey = ey;
    r.ez = ez;
    r.eh2 = (float)(dex * dex + dey * dey);
    const double h0 = zif0 - z[j];
    const double hp = fmax(h0, 1e-12);  // a masked sample keeps the iteration finite
    r.a = h0 > 0.0 ? (float)(-w[j] * v0 * 2.0 * rho0 * Sf / kTwoPi) : 0.0f;
    r.h0 = (float)hp;
    r.hf0 = (float)(hp * Sf);
    r.hf0S2 = (float)(hp * Sf * S20);
    rec[j] = r;
}

__global__ void __launch_bounds__(256) ray_prep_f64_kernel(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ w, double v0,
    const double *__restrict__ partials, double *__restrict__ anchor_out,
    RayRecD *__restrict__ rec) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double ax, ay, az, radius;
        ray_anchor(partials, ax, ay, az, radius);
        anchor_out[0] = ax;
        anchor_out[1] = ay;
        anchor_out[2] = az;
        anchor_out[3] = 0.0;
    }
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    RayRecD r;
    r.x = x[j];
    r.y = y[j];
    r.z = z[j];
    r.a = -w[j] * v0 / kTwoPi;
    rec[j] = r;
}

// Root of F(C) = C sum_l h_l / eta_l(C) - rho on [0, Smin), h_l > 0: Newton inside a
// bracket that every evaluation shrinks, bisection when a step leaves it.  Ends when
// the step no longer moves C or the bracket is one ulp wide.
template <int L>
__device__ double ray_root_f64(double rho, const double (&h)[L], const RayStack &st,
                               double C) {
    double lo = 0.0, hi = st.Smind * (1.0 - 0x1p-50);  // eta_l > 0 everywhere in the bracket
    if (!(C >= lo && C < hi)) C = 0.5 * hi;
    for (int it = 0; it < 200; ++it) {
        double S1 = 0.0, S3 = 0.0;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const double e2 = st.S2d[l] - C * C;
            const double ie = 1.0 / sqrt(e2);
            const double g = h[l] * ie;
            S1 += g;
            S3 += g * ie * ie * st.S2d[l];
        }
        const double F = C * S1 - rho;
        if (F > 0.0) hi = C;
        else lo = C;
        double Cn = C - F / S3;
        if (!(Cn >= lo && Cn <= hi)) Cn = 0.5 * (lo + hi);
        const bool done = Cn == C || hi - lo <= 0x1p-52 * hi;
        C = Cn;
        if (done) break;
    }
    return C;
}

// Straight-line guess in the first medium, kept inside the interval.
__device__ inline double ray_guess(double rho, double H, const RayStack &st) {
    const double g = sqrt(st.S2d[0]) * rho / sqrt(rho * rho + H * H + 1e-300);
    return fmin(g, 0.9 * st.Smind);
}

// Per-target constants of the FP32 path.
// The pair's iteration runs in v = tan(theta_f), theta_f the angle in the fastest layer
// (slowness S_f), on F(v) = S_f v sum_l h_l q_l(v) - rho, q_l = (S_l^2 + (S_l^2 - S_f^2) v^2)^(-1/2).
// Its start: the pair's F at the reference root v_0 is exactly -R with
// R = drho + e_z tan(theta_0) (the reference ray solves the reference equation, and the
// sample sits e_z deeper, shortening h_0 by e_z), and its derivatives at v_0 are the
// reference's with h_0 lowered by e_z.  Series reversion of F(v_0 + delta) = 0 to third order:
//   d = R / F1,  delta = d - a d^2 + (2 a^2 - b) d^3,  a = F2 / (2 F1),  b = F3 / (6 F1),
// with 1/F1 = (1/F1_0)(1 + e_z g1 / F1_0), F2 = F2_0 - e_z g2 (g1, g2 the h_0-derivatives
// of F1 and F2).
template <int L, int NF>
struct RayTgtF {
    float dmx, dmy;         // -2 (P - C_A) horizontal
    float rho0, rho02;      // reference horizontal distance, squared
    float C0, c0e0;         // reference root, C_0 / eta_0^0 (= tan(theta_0))
    float v0;               // reference root in v
    float iF1, k1;          // 1/F1_0 and g1 / F1_0^2
    float F2h, g2h, b3;     // F2_0 / 2, g2 / 2, F3_0 / (6 F1_0)
    float hn, hfn, hfnS2;   // h_n of the field point (> 0), S_f h_n and S_f h_n S_n^2
    float eta0[L];
    float S2[L];            // S_l^2 (lane copies: the iteration's FMA takes one SGPR operand)
    float ph0[NF];          // frac(f_q t_0)
    bool valid;             // field point below the last plane
};

template <int L, int NF>
__device__ __forceinline__ void ray_setup_f32(RayTgtF<L, NF> &T, double px, double py,
                                              double pz, double ax, double ay, double az,
                                              const RayStack &st, const RayFreqs &fr) {
    const double dx = px - ax, dy = py - ay;
    const double rho0 = sqrt(dx * dx + dy * dy);
    double h[L], hc[L];
    h[0] = st.zif0 - az;
#pragma unroll
    for (int l = 1; l < L - 1; ++l) h[l] = st.hd[l];
    h[L - 1] = pz - st.zlast;
    double H = 0.0;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        hc[l] = fmax(h[l], 1e-12);  // the root needs positive extents
        H += hc[l];
    }
    const double C0 = ray_root_f64<L>(rho0, hc, st, ray_guess(rho0, H, st));
    // t_0 with the true extents: dt = t - t_0 holds for any C_0 and any h_0^0.  The
    // derivatives of F for the start use the clamped extents (well posed).  In v:
    // q_l(v_0) = sqrt(S_f^2 - C_0^2) / (S_f eta_l), and with p_l = h_l S_l^2 q_l^3,
    //   F1 = S_f sum p_l,  F2 = -3 S_f v_0 sum p_l k_l,  F3 = -3 S_f sum p_l k_l (1 - 5 v_0^2 k_l),
    // k_l = (S_l^2 - S_f^2) q_l^2.
    const double C02 = C0 * C0, Sf = st.Smind, Sf2 = Sf * Sf;
    const double cf = sqrt(Sf2 - C02), v0 = C0 / cf;
    double t0 = C0 * rho0, F1 = 0.0, F2 = 0.0, F3 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const double eta = sqrt(st.S2d[l] - C02);
        T.eta0[l] = (float)eta;
        t0 += h[l] * eta;
        const double ql = cf / (Sf * eta);
        const double kl = (st.S2d[l] - Sf2) * ql * ql;
        const double p1 = st.S2d[l] * ql * ql * ql;  // per unit extent
        F1 += hc[l] * p1;
        F2 += hc[l] * p1 * kl;
        F3 += hc[l] * p1 * kl * (1.0 - 5.0 * v0 * v0 * kl);
        if (l == 0) {
            g1 = Sf * p1;
            g2 = -3.0 * Sf * v0 * p1 * kl;
        }
    }
    F1 *= Sf;
    F2 *= -3.0 * Sf * v0;
    F3 *= -3.0 * Sf;
    const double iF1 = 1.0 / F1;
    T.dmx = (float)(-2.0 * dx);
    T.dmy = (float)(-2.0 * dy);
    T.rho0 = (float)rho0;
    T.rho02 = (float)(rho0 * rho0);
    T.C0 = (float)C0;
    T.c0e0 = (float)(C0 / T.eta0[0]);
    T.v0 = (float)v0;
    T.iF1 = (float)iF1;
    T.k1 = (float)(g1 * iF1 * iF1);
    T.F2h = (float)(0.5 * F2);
    T.g2h = (float)(0.5 * g2);
    T.b3 = (float)(F3 * iF1 / 6.0);
    T.hn = (float)hc[L - 1];  // positive, so the pair's iteration stays well posed
    T.hfn = (float)(hc[L - 1] * st.Smind);
    T.hfnS2 = (float)(hc[L - 1] * st.Smind * st.S2d[L - 1]);
    T.valid = h[L - 1] > 0.0;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        T.S2[l] = st.S2[l];
        asm volatile("" : "+v"(T.S2[l]));  // keep a lane copy: the FMA below takes one SGPR
    }
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        double p = t0 * fr.f[q];
        p -= floor(p);
        T.ph0[q] = (float)p;
    }
}

// One transducer sample against the lane's field point.  `s` is wave-uniform (SGPRs).
// FRACT: reduce the phase to [0, 1) before v_sin / v_cos (needed only when the argument
// can exceed their own range: |f dt| <= f |Q_j - C_A| / c_0, the travel time changing with
// the sample's position at most at the first medium's slowness).
template <int L, int NF, bool FRACT, class Rec>
__device__ __forceinline__ void ray_pair_f32(const RayTgtF<L, NF> &T, const Rec &s,
                                             const RayStack &st, const float (&ff)[NF],
                                             float (&ar)[NF], float (&ai)[NF]) {
    const float q = fmaf(T.dmy, s.ey, fmaf(T.dmx, s.ex, s.eh2));  // rho^2 - rho_0^2
    const float r2 = fmaxf(T.rho02 + q, 0.0f);
    const float rho = __builtin_amdgcn_sqrtf(r2);
    const float drho = q * __builtin_amdgcn_rcpf(fmaxf(rho + T.rho0, FLT_MIN));
    // extents, and S_f h and S_f h S^2 per layer (the sample's own from its record)
    float h[L], hf[L], hfS2[L];
    h[0] = s.h0;
    hf[0] = s.hf0;
    hfS2[0] = s.hf0S2;
#pragma unroll
    for (int l = 1; l < L - 1; ++l) {
        h[l] = st.h[l];
        hf[l] = st.hf[l];
        hfS2[l] = st.hfS2[l];
    }
    h[L - 1] = T.hn;
    hf[L - 1] = T.hfn;
    hfS2[L - 1] = T.hfnS2;
    // start: third-order series reversion about the reference root (in v)
    const float R = fmaf(s.ez, T.c0e0, drho);
    const float iF1 = fmaf(s.ez, T.k1, T.iF1);
    const float d = R * iF1;
    const float a = fmaf(-s.ez, T.g2h, T.F2h) * iF1;
    const float u = fmaf(a + a, a, -T.b3);
    float v = fmaxf(fmaf(d, fmaf(fmaf(u, d, -a), d, 1.0f), T.v0), 0.0f);
    // Newton in v: every layer's tan(theta_l) = S_f v q_l, so
    //   F(v) = v Q1 - rho,  Q1 = S_f sum h_l q_l,   F'(v) = Q3,  Q3 = S_f sum h_l S_l^2 q_l^3,
    // the fastest layer's term is linear (no pole at grazing), nothing cancels, and F is
    // concave and increasing on [0, inf) with F(0) = -rho <= 0: a step from the right lands
    // at or left of the root (clamped at 0), steps from the left rise monotonically.
    // Iterate until |F| is within a few units of its FP32 rounding (the phase is stationary
    // in the root; the amplitude moves by ~1e-6 relative).
    const float tolF = fmaf(4e-6f, rho, 1e-9f);
    float e2[L], qs[L], Q1, Q3;
    for (int it = 0;; ++it) {
        const float vv = v * v;
        Q1 = 0.0f;
        Q3 = 0.0f;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            e2[l] = fmaf(st.dS2[l], vv, T.S2[l]);
            qs[l] = __builtin_amdgcn_rsqf(e2[l]);
            Q1 = fmaf(hf[l], qs[l], Q1);
            Q3 = fmaf(hfS2[l] * qs[l], qs[l] * qs[l], Q3);
        }
        const float F = fmaf(v, Q1, -rho);
        if (fabsf(F) <= tolF || it == kRayMaxIt) break;
        v = fmaxf(fmaf(-F, __builtin_amdgcn_rcpf(Q3), v), 0.0f);
    }
    // back to C and eta_l: with w = 1 + v^2, C = S_f v / sqrt(w), eta_l = sqrt(e2_l / w)
    const float rw = __builtin_amdgcn_rsqf(fmaf(v, v, 1.0f));
    const float C = st.Sf * v * rw;
    float eta[L];
#pragma unroll
    for (int l = 0; l < L; ++l) eta[l] = e2[l] * qs[l] * rw;
    // sum_l h_l / (eta_l + eta_l^0)
    float hsum;
    if constexpr (L <= 5) {
        float num = h[0], den = eta[0] + T.eta0[0];
#pragma unroll
        for (int l = 1; l < L; ++l) {
            const float dl = eta[l] + T.eta0[l];
            num = fmaf(num, dl, h[l] * den);
            den *= dl;
        }
        hsum = num * __builtin_amdgcn_rcpf(den);
    } else {
        hsum = 0.0f;
#pragma unroll
        for (int l = 0; l < L; ++l) hsum = fmaf(h[l], __builtin_amdgcn_rcpf(eta[l] + T.eta0[l]), hsum);
    }
    const float B = fmaf(-(C + T.C0), hsum, rho);
    const float dt = fmaf(C - T.C0, B, fmaf(T.C0, drho, -s.ez * T.eta0[0]));
    // T / A = prod(2 rho_l eta_l) / (eta_0 sqrt(S1 S3) prod(den_l)),
    // den_l = rho_{l+1} eta_l + rho_l eta_{l+1}; the first factor 2 rho_0 eta_0 / eta_0 is
    // the constant 2 rho_0, folded into the sample's strength a.  S1 = sum h_l/eta_l =
    // sqrt(w) Q1 / S_f and S3 = sum h_l S_l^2/eta_l^3 = w^(3/2) Q3 / S_f, so
    // S1 S3 = w^2 Q1 Q3 / S_f^2 (the S_f is in a as well).
    const float w = fmaf(v, v, 1.0f);
    float num = s.a, den2 = (w * w) * (Q1 * Q3);
#pragma unroll
    for (int l = 0; l < L - 1; ++l) {
        const float dn = fmaf(st.rho[l + 1], eta[l], st.rho[l] * eta[l + 1]);
        if (l > 0) num *= st.rho2[l] * eta[l];
        den2 *= dn * dn;
    }
    const float m = num * __builtin_amdgcn_rsqf(den2);
#pragma unroll
    for (int q2 = 0; q2 < NF; ++q2) {
        float ph = fmaf(dt, ff[q2], T.ph0[q2]);  // revolutions
        if constexpr (FRACT) ph = __builtin_amdgcn_fractf(ph);
        ar[q2] = fmaf(m, __builtin_amdgcn_cosf(ph), ar[q2]);
        ai[q2] = fmaf(m, __builtin_amdgcn_sinf(ph), ai[q2]);
    }
}

template <int L, int NF, bool FRACT>
__device__ __forceinline__ void ray_sum_f32(const RayTgtF<L, NF> &T, const RayRecF *recs,
                                            int64_t j0, int64_t j1, const RayStack &st,
                                            const float (&ff)[NF], float (&mre)[NF],
                                            float (&mim)[NF]) {
    const RayRecFPtr rec = (RayRecFPtr)recs;
    float cre[NF], cim[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) mre[q] = mim[q] = cre[q] = cim[q] = 0.0f;
    for (int64_t jb = j0; jb < j1; jb += kRaySub) {
        const int64_t je = (jb + kRaySub < j1) ? jb + kRaySub : j1;
        float ar[NF], ai[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) ar[q] = ai[q] = 0.0f;
        if (je - jb == kRaySub) {  // full block: constant trip count
            for (int jj = 0; jj < kRaySub; ++jj)
                ray_pair_f32<L, NF, FRACT>(T, rec[jb + jj], st, ff, ar, ai);
        } else {
            for (int64_t j = jb; j < je; ++j) ray_pair_f32<L, NF, FRACT>(T, rec[j], st, ff, ar, ai);
        }
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            float y = ar[q] - cre[q];
            float t = mre[q] + y;
            cre[q] = (t - mre[q]) - y;
            mre[q] = t;
            y = ai[q] - cim[q];
            t = mim[q] + y;
            cim[q] = (t - mim[q]) - y;
            mim[q] = t;
        }
    }
}

// grid (target tiles of kBlock, source splits); out [split][fr.n][n_tgt].  inv_lam0 =
// the block's highest frequency over c_0 (bounds the phase argument with the anchor radius).
template <int L, int NF>
__global__ void __launch_bounds__(kBlock) ray_f32_kernel(
    const RayRecF *__restrict__ recs, int64_t n_src, int64_t chunk,
    const double *__restrict__ tx, const double *__restrict__ ty, const double *__restrict__ tz,
    int64_t n_tgt, const double *__restrict__ anchor, RayStack st, RayFreqs fr, double inv_lam0,
    float2 *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool in = i < n_tgt;
    if (!in) i = n_tgt - 1;
    RayTgtF<L, NF> T;
    ray_setup_f32<L, NF>(T, tx[i], ty[i], tz[i], anchor[0], anchor[1], anchor[2], st, fr);
    float ff[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) ff[q] = fr.ff[q];
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = (j0 + chunk < n_src) ? j0 + chunk : n_src;
    float mre[NF], mim[NF];
    if (phase_in_sin_range(anchor[3], inv_lam0))
        ray_sum_f32<L, NF, false>(T, recs, j0, j1, st, ff, mre, mim);
    else
        ray_sum_f32<L, NF, true>(T, recs, j0, j1, st, ff, mre, mim);
    if (!in) return;
    float2 *o = out + (int64_t)blockIdx.y * fr.n * n_tgt;
#pragma unroll
    for (int q = 0; q < NF; ++q)
        if (q < fr.n) o[(int64_t)q * n_tgt + i] = T.valid ? make_float2(mre[q], mim[q]) : make_float2(0.0f, 0.0f);
}

// Few field points: one wave per (field point, source range).  Lanes take every 64th
// sample (vector loads; the sample records stay in L2), and the 64 lane sums are combined
// by a fixed shuffle tree, so results are still bitwise repeatable.  grid (n_tgt, splits),
// out [split][fr.n][n_tgt].
template <int L, int NF, bool FRACT>
__device__ __forceinline__ void ray_sum_lanes_f32(const RayTgtF<L, NF> &T,
                                                  const RayRecF *__restrict__ rec, int64_t j0,
                                                  int64_t j1, const RayStack &st,
                                                  const float (&ff)[NF], float (&mre)[NF],
                                                  float (&mim)[NF]) {
    float cre[NF], cim[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) mre[q] = mim[q] = cre[q] = cim[q] = 0.0f;
    const int lane = threadIdx.x & 63;
    for (int64_t jb = j0 + lane; jb < j1; jb += 64 * kRaySub) {
        const int64_t je = (jb + 64 * kRaySub < j1) ? jb + 64 * kRaySub : j1;
        float ar[NF], ai[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) ar[q] = ai[q] = 0.0f;
        for (int64_t j = jb; j < je; j += 64) {
            const RayRecF r = rec[j];
            ray_pair_f32<L, NF, FRACT>(T, r, st, ff, ar, ai);
        }
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            float y = ar[q] - cre[q];
            float t = mre[q] + y;
            cre[q] = (t - mre[q]) - y;
            mre[q] = t;
            y = ai[q] - cim[q];
            t = mim[q] + y;
            cim[q] = (t - mim[q]) - y;
            mim[q] = t;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            mre[q] += __shfl_xor(mre[q], off);
            mim[q] += __shfl_xor(mim[q], off);
        }
    }
}

template <int L, int NF>
__global__ void __launch_bounds__(64) ray_f32_few_kernel(
    const RayRecF *__restrict__ recs, int64_t n_src, int64_t chunk,
    const double *__restrict__ tx, const double *__restrict__ ty, const double *__restrict__ tz,
    int64_t n_tgt, const double *__restrict__ anchor, RayStack st, RayFreqs fr, double inv_lam0,
    float2 *__restrict__ out) {
    const int64_t i = blockIdx.x;
    RayTgtF<L, NF> T;
    ray_setup_f32<L, NF>(T, tx[i], ty[i], tz[i], anchor[0], anchor[1], anchor[2], st, fr);
    float ff[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) ff[q] = fr.ff[q];
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = (j0 + chunk < n_src) ? j0 + chunk : n_src;
    float mre[NF], mim[NF];
    if (phase_in_sin_range(anchor[3], inv_lam0))
        ray_sum_lanes_f32<L, NF, false>(T, recs, j0, j1, st, ff, mre, mim);
    else
        ray_sum_lanes_f32<L, NF, true>(T, recs, j0, j1, st, ff, mre, mim);
    if (threadIdx.x != 0) return;
    float2 *o = out + (int64_t)blockIdx.y * fr.n * n_tgt;
#pragma unroll
    for (int q = 0; q < NF; ++q)
        if (q < fr.n) o[(int64_t)q * n_tgt + i] = T.valid ? make_float2(mre[q], mim[q]) : make_float2(0.0f, 0.0f);
}

template <int L, int NF>
__global__ void __launch_bounds__(kBlock) ray_f64_kernel(
    const RayRecD *__restrict__ recs, int64_t n_src, int64_t chunk,
    const double *__restrict__ tx, const double *__restrict__ ty, const double *__restrict__ tz,
    int64_t n_tgt, const double *__restrict__ anchor, RayStack st, RayFreqs fr,
    double2 *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool in = i < n_tgt;
    if (!in) i = n_tgt - 1;
    const double px = tx[i], py = ty[i], pz = tz[i];
    double h[L];
    h[0] = fmax(st.zif0 - anchor[2], 1e-12);
#pragma unroll
    for (int l = 1; l < L - 1; ++l) h[l] = st.hd[l];
    const double hn = pz - st.zlast;
    h[L - 1] = fmax(hn, 1e-12);
    double H = 0.0;
#pragma unroll
    for (int l = 0; l < L; ++l) H += h[l];
    const double ax = px - anchor[0], ay = py - anchor[1];
    const double rho0 = sqrt(ax * ax + ay * ay);
    const double Cst = ray_root_f64<L>(rho0, h, st, ray_guess(rho0, H, st));
    h[L - 1] = hn;
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = (j0 + chunk < n_src) ? j0 + chunk : n_src;
    const RayRecDPtr rec = (RayRecDPtr)recs;
    double mre[NF], mim[NF], cre[NF], cim[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) mre[q] = mim[q] = cre[q] = cim[q] = 0.0;
    for (int64_t jb = j0; jb < j1; jb += kRaySub) {
        const int64_t je = (jb + kRaySub < j1) ? jb + kRaySub : j1;
        double ar[NF], ai[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) ar[q] = ai[q] = 0.0;
        for (int64_t j = jb; j < je; ++j) {
            const double sx = rec[j].x, sy = rec[j].y, sz = rec[j].z, sa = rec[j].a;
            h[0] = st.zif0 - sz;
            if (!(h[0] > 0.0 && hn > 0.0)) continue;  // no ray: contributes nothing
            const double dx = px - sx, dy = py - sy;
            const double rho = sqrt(dx * dx + dy * dy);
            const double C = ray_root_f64<L>(rho, h, st, Cst);
            double S1 = 0.0, S3 = 0.0, t = C * rho, eta[L];
#pragma unroll
            for (int l = 0; l < L; ++l) {
                const double e2 = st.S2d[l] - C * C;
                eta[l] = sqrt(e2);
                S1 += h[l] / eta[l];
                S3 += h[l] * st.S2d[l] / (eta[l] * e2);
                t += h[l] * eta[l];
            }
            double m = sa / (eta[0] * sqrt(S1 * S3));
#pragma unroll
            for (int l = 0; l < L - 1; ++l)
                m *= 2.0 * st.rhod[l] * eta[l] / (st.rhod[l + 1] * eta[l] + st.rhod[l] * eta[l + 1]);
#pragma unroll
            for (int q = 0; q < NF; ++q) {
                double ph = t * fr.f[q];
                ph -= rint(ph);
                double sn, cs;
                sincospi(2.0 * ph, &sn, &cs);
                ar[q] += m * cs;
                ai[q] += m * sn;
            }
        }
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            double y = ar[q] - cre[q];
            double t = mre[q] + y;
            cre[q] = (t - mre[q]) - y;
            mre[q] = t;
            y = ai[q] - cim[q];
            t = mim[q] + y;
            cim[q] = (t - mim[q]) - y;
            mim[q] = t;
        }
    }
    if (!in) return;
    double2 *o = out + (int64_t)blockIdx.y * fr.n * n_tgt;
#pragma unroll
    for (int q = 0; q < NF; ++q)
        if (q < fr.n) o[(int64_t)q * n_tgt + i] = make_double2(mre[q], mim[q]);
}

// Fixed-order sum of the split partials [ns][n] into out [n].
template <typename T2>
__global__ void __launch_bounds__(256) ray_reduce_kernel(const T2 *__restrict__ partial, int ns,
                                                         int64_t n, T2 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < ns; ++s) {
        const T2 v = partial[(int64_t)s * n + i];
        re += (double)v.x;
        im += (double)v.y;
    }
    T2 r;
    r.x = re;
    r.y = im;
    out[i] = r;
}

template <typename T2>
__global__ void __launch_bounds__(256) ray_zero_kernel(int64_t n, T2 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        T2 z;
        z.x = 0;
        z.y = 0;
        out[i] = z;
    }
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

template <int L, int NF>
void launch_ray_f32(dim3 grid, hipStream_t s, const RayRecF *rec, int64_t n_src, int64_t chunk,
                    const Targets &t, const double *anchor, const RayStack &st,
                    const RayFreqs &fr, float2 *dst) {
    double fmax = 0.0;
    for (int q = 0; q < fr.n; ++q) fmax = fr.f[q] > fmax ? fr.f[q] : fmax;
    hipLaunchKernelGGL((ray_f32_kernel<L, NF>), grid, dim3(kBlock), 0, s, rec, n_src, chunk, t.x,
                       t.y, t.z, t.n, anchor, st, fr, fmax * sqrt(st.S2d[0]), dst);
}

template <int L, int NF>
void launch_ray_f32_few(dim3 grid, hipStream_t s, const RayRecF *rec, int64_t n_src,
                        int64_t chunk, const Targets &t, const double *anchor,
                        const RayStack &st, const RayFreqs &fr, float2 *dst) {
    double fmax = 0.0;
    for (int q = 0; q < fr.n; ++q) fmax = fr.f[q] > fmax ? fr.f[q] : fmax;
    hipLaunchKernelGGL((ray_f32_few_kernel<L, NF>), grid, dim3(64), 0, s, rec, n_src, chunk, t.x,
                       t.y, t.z, t.n, anchor, st, fr, fmax * sqrt(st.S2d[0]), dst);
}

template <int L, int NF>
void launch_ray_f64(dim3 grid, hipStream_t s, const RayRecD *rec, int64_t n_src, int64_t chunk,
                    const Targets &t, const double *anchor, const RayStack &st,
                    const RayFreqs &fr, double2 *dst) {
    hipLaunchKernelGGL((ray_f64_kernel<L, NF>), grid, dim3(kBlock), 0, s, rec, n_src, chunk, t.x,
                       t.y, t.z, t.n, anchor, st, fr, dst);
}

template <int NF, class Rec, class T2>
void dispatch_ray(int L, bool few, dim3 grid, hipStream_t s, const Rec *rec, int64_t n_src,
                  int64_t chunk, const Targets &t, const double *anchor, const RayStack &st,
                  const RayFreqs &fr, T2 *dst) {
#define RSI_RAY_CASE(LL)                                                                   \
    case LL:                                                                               \
        if constexpr (std::is_same<T2, float2>::value) {                                   \
            if (few)                                                                       \
                launch_ray_f32_few<LL, NF>(grid, s, rec, n_src, chunk, t, anchor, st, fr, dst); \
            else                                                                           \
                launch_ray_f32<LL, NF>(grid, s, rec, n_src, chunk, t, anchor, st, fr, dst); \
        } else {                                                                           \
            launch_ray_f64<LL, NF>(grid, s, rec, n_src, chunk, t, anchor, st, fr, dst);    \
        }                                                                                  \
        break;
    switch (L) {
        RSI_RAY_CASE(2)
        RSI_RAY_CASE(3)
        RSI_RAY_CASE(4)
        RSI_RAY_CASE(5)
        RSI_RAY_CASE(6)
        RSI_RAY_CASE(7)
        RSI_RAY_CASE(8)
        RSI_RAY_CASE(9)
        default:
            break;
    }
#undef RSI_RAY_CASE
}

rsi_status validate_ray(const rsi_transducer *xd, const double *zif, int n_if,
                        const rsi_medium *media, const rsi_points *tgt, const double *freqs,
                        int n_freq, rsi_precision prec, void *out) {
    if (!xd || !media || !tgt) return RSI_ERR_NULL;
    if (n_if < 0 || n_freq < 0 || xd->pts.n < 0 || tgt->n < 0) return RSI_ERR_SIZE;
    if (n_if > kRayMaxIf) return RSI_ERR_SIZE;
    if (n_if > 0 && !zif) return RSI_ERR_NULL;
    if (n_freq > 0 && !freqs) return RSI_ERR_NULL;
    if (prec != RSI_FP32 && prec != RSI_FP64) return RSI_ERR_ARG;
    if (!std::isfinite(xd->v0)) return RSI_ERR_ARG;
    for (int l = 0; l <= n_if; ++l)
        if (!(media[l].c > 0.0) || !(media[l].rho > 0.0) || !std::isfinite(media[l].c) ||
            !std::isfinite(media[l].rho))
            return RSI_ERR_ARG;
    for (int l = 0; l < n_if; ++l) {
        if (!std::isfinite(zif[l])) return RSI_ERR_ARG;
        if (l > 0 && !(zif[l] > zif[l - 1])) return RSI_ERR_ARG;
    }
    for (int q = 0; q < n_freq; ++q)
        if (!(freqs[q] > 0.0) || !std::isfinite(freqs[q])) return RSI_ERR_ARG;
    if (tgt->n == 0 || n_freq == 0) return RSI_OK;
    if (!out || !tgt->x || !tgt->y || !tgt->z) return RSI_ERR_NULL;
    if (xd->pts.n > 0 && (!xd->pts.x || !xd->pts.y || !xd->pts.z || !xd->w)) return RSI_ERR_NULL;
    return RSI_OK;
}

RayStack make_stack(const double *zif, int n_if, const rsi_medium *media) {
    RayStack st{};
    const int L = n_if + 1;
    double Smin = 1.0 / media[0].c;
    for (int l = 0; l < L; ++l) {
        const double S = 1.0 / media[l].c;
        st.S2d[l] = S * S;
        st.rhod[l] = media[l].rho;
        st.S2[l] = (float)(S * S);
        st.rho[l] = (float)media[l].rho;
        st.rho2[l] = (float)(2.0 * media[l].rho);
        Smin = S < Smin ? S : Smin;
    }
    for (int l = 1; l < L - 1; ++l) {
        st.hd[l] = zif[l] - zif[l - 1];
        st.h[l] = (float)st.hd[l];
        st.hf[l] = (float)(st.hd[l] * Smin);
        st.hfS2[l] = (float)(st.hd[l] * Smin * st.S2d[l]);
    }
    st.zif0 = zif[0];
    st.zlast = zif[n_if - 1];
    st.Smind = Smin;
    for (int l = 0; l < L; ++l) st.dS2[l] = (float)(st.S2d[l] - Smin * Smin);
    st.Sf = (float)Smin;
    return st;
}

RayFreqs freq_block(const double *freqs, int q0, int nb) {
    RayFreqs fr{};
    fr.n = nb;
    for (int q = 0; q < kRayFB; ++q) {
        const double f = freqs[q0 + (q < nb ? q : nb - 1)];
        fr.f[q] = f;
        fr.ff[q] = (float)f;
    }
    return fr;
}

}  // namespace
}  // namespace rsi

using namespace rsi;

extern "C" rsi_status rsi_ray_field(const rsi_transducer *xd, const double *zif, int n_if,
                                    const rsi_medium *media, const rsi_points *tgt,
                                    const double *freqs, int n_freq, rsi_precision prec,
                                    void *out, void *stream) {
    RSI_TRY(validate_ray(xd, zif, n_if, media, tgt, freqs, n_freq, prec, out));
    if (tgt->n == 0 || n_freq == 0) return RSI_OK;
    hipStream_t s = as_stream(stream);
    {
        std::vector<DevSpan> in;
        add_points(in, xd->pts);
        in.push_back({xd->w, xd->pts.n});
        add_points(in, *tgt);
        RSI_TRY(check_finite(s, in));
    }
    Scratch scratch(s);
    const Targets t{tgt->x, tgt->y, tgt->z, tgt->n};
    const int64_t n_src = xd->pts.n, n_out = (int64_t)n_freq * tgt->n;
    if (n_src == 0) {
        if (prec == RSI_FP32)
            hipLaunchKernelGGL(ray_zero_kernel<float2>, dim3(blocks_of(n_out)), dim3(256), 0, s, n_out,
                               static_cast<float2 *>(out));
        else
            hipLaunchKernelGGL(ray_zero_kernel<double2>, dim3(blocks_of(n_out)), dim3(256), 0, s, n_out,
                               static_cast<double2 *>(out));
        RSI_HIP(hipGetLastError());
        return RSI_OK;
    }
    double *partials = nullptr;
    RSI_TRY(scratch.alloc(&partials, kBBoxBlocks * 6));
    RSI_TRY(bbox_partials(xd->pts, partials, s));
    if (n_if == 0) {
        // one medium: eq. (12) is eq. (3), the monopole pair sum (with its own shape rule)
        const PairShape sh = default_shape(n_src, tgt->n, prec == RSI_FP32 ? kFewWaves / 8 : 0);
        const int64_t nslots = partial_slots(sh, n_src, tgt->n);
        const double c0 = media[0].c;
        if (prec == RSI_FP32) {
            SrcSetF set;
            float2 *partial = nullptr;
            RSI_TRY(scratch.alloc(&set.rec, (size_t)n_src));
            RSI_TRY(scratch.alloc(&set.anchor, 4));
            if (nslots > 0) RSI_TRY(scratch.alloc(&partial, (size_t)nslots));
            RSI_TRY(prep_sources_f32(xd->pts, xd->w, nullptr, xd->v0, nullptr, partials,
                                     c0 / freqs[0], Cplx{1.0, 0.0}, set, s));
            for (int q = 0; q < n_freq; ++q)
                RSI_TRY(pairsum_f32(set, t, RSI_MONOPOLE, nullptr, c0, freqs[q], sh, partial,
                                    static_cast<float2 *>(out) + (int64_t)q * tgt->n, s));
            return RSI_OK;
        }
        SrcSetD set;
        double2 *partial = nullptr;
        RSI_TRY(scratch.alloc(&set.rec, (size_t)n_src));
        if (nslots > 0) RSI_TRY(scratch.alloc(&partial, (size_t)nslots));
        RSI_TRY(prep_sources_f64(xd->pts, xd->w, nullptr, xd->v0, Cplx{1.0, 0.0}, set, s));
        for (int q = 0; q < n_freq; ++q)
            RSI_TRY(pairsum_f64(set, t, RSI_MONOPOLE, nullptr, c0, freqs[q], sh, partial,
                                static_cast<double2 *>(out) + (int64_t)q * tgt->n, s));
        return RSI_OK;
    }
    // ray pairs cost ~6x an RSI pair: splits of >= 1024 sources keep enough waves for the
    // one-point-per-lane launch down to ~10^4 field points (measured best of 256 .. 4096)
    static const int ray_min_chunk = env_int("RSI_RAY_MIN_CHUNK", 1024);
    const PairShape sh = default_shape(n_src, tgt->n, prec == RSI_FP32 ? kFewWaves / 2 : 0, ray_min_chunk);
    const RayStack st = make_stack(zif, n_if, media);
    const int L = n_if + 1;
    // FP32 with too few field points to give every CU 32 waves one per lane: one wave per
    // (point, source range) instead (PairShape::few)
    const int64_t chunk = sh.chunk > 0 ? sh.chunk : n_src;
    bool few = prec == RSI_FP32 && sh.few;
    if (const char *e = std::getenv("RSI_RAY_FEW"))  // tuning/testing override: 0 or 1
        if (prec == RSI_FP32 && (e[0] == '0' || e[0] == '1') && e[1] == 0) few = e[0] == '1';
    const int64_t ns = (n_src + chunk - 1) / chunk;
    if (ns > 65535) return RSI_ERR_SIZE;
    const int64_t bx = few ? tgt->n : (tgt->n + kBlock - 1) / kBlock;
    if (bx > 0x7fffffff) return RSI_ERR_SIZE;
    const dim3 grid((unsigned)bx, (unsigned)ns);
    double *anchor = nullptr;
    RSI_TRY(scratch.alloc(&anchor, 4));
    const int nfb_max = n_freq < kRayFB ? n_freq : kRayFB;
    if (prec == RSI_FP32) {
        RayRecF *rec = nullptr;
        float2 *partial = nullptr;
        RSI_TRY(scratch.alloc(&rec, (size_t)n_src));
        if (ns > 1) RSI_TRY(scratch.alloc(&partial, (size_t)(ns * nfb_max * tgt->n)));
        hipLaunchKernelGGL(ray_prep_f32_kernel, dim3(blocks_of(n_src)), dim3(256), 0, s, n_src,
                           xd->pts.x, xd->pts.y, xd->pts.z, xd->w, xd->v0, zif[0], media[0].rho,
                           st.S2d[0], st.Smind, partials, anchor, rec);
        RSI_HIP(hipGetLastError());
        for (int q0 = 0; q0 < n_freq; q0 += kRayFB) {
            const int nb = n_freq - q0 < kRayFB ? n_freq - q0 : kRayFB;
            const RayFreqs fr = freq_block(freqs, q0, nb);
            float2 *o = static_cast<float2 *>(out) + (int64_t)q0 * tgt->n;
            float2 *dst = ns > 1 ? partial : o;
            if (nb == 1) dispatch_ray<1>(L, few, grid, s, rec, n_src, chunk, t, anchor, st, fr, dst);
            else dispatch_ray<kRayFB>(L, few, grid, s, rec, n_src, chunk, t, anchor, st, fr, dst);
            RSI_HIP(hipGetLastError());
            if (ns > 1) {
                const int64_t n = (int64_t)nb * tgt->n;
                hipLaunchKernelGGL(ray_reduce_kernel<float2>, dim3(blocks_of(n)), dim3(256), 0, s,
                                   partial, (int)ns, n, o);
                RSI_HIP(hipGetLastError());
            }
        }
        return RSI_OK;
    }
    RayRecD *rec = nullptr;
    double2 *partial = nullptr;
    RSI_TRY(scratch.alloc(&rec, (size_t)n_src));
    if (ns > 1) RSI_TRY(scratch.alloc(&partial, (size_t)(ns * nfb_max * tgt->n)));
    hipLaunchKernelGGL(ray_prep_f64_kernel, dim3(blocks_of(n_src)), dim3(256), 0, s, n_src,
                       xd->pts.x, xd->pts.y, xd->pts.z, xd->w, xd->v0, partials, anchor, rec);
    RSI_HIP(hipGetLastError());
    for (int q0 = 0; q0 < n_freq; q0 += kRayFB) {
        const int nb = n_freq - q0 < kRayFB ? n_freq - q0 : kRayFB;
        const RayFreqs fr = freq_block(freqs, q0, nb);
        double2 *o = static_cast<double2 *>(out) + (int64_t)q0 * tgt->n;
        double2 *dst = ns > 1 ? partial : o;
        if (nb == 1) dispatch_ray<1>(L, false, grid, s, rec, n_src, chunk, t, anchor, st, fr, dst);
        else dispatch_ray<kRayFB>(L, false, grid, s, rec, n_src, chunk, t, anchor, st, fr, dst);
        RSI_HIP(hipGetLastError());
        if (ns > 1) {
            const int64_t n = (int64_t)nb * tgt->n;
            hipLaunchKernelGGL(ray_reduce_kernel<double2>, dim3(blocks_of(n)), dim3(256), 0, s,
                               partial, (int)ns, n, o);
            RSI_HIP(hipGetLastError());
        }
    }
    return RSI_OK;
}
