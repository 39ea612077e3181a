// rsi_chain.hip -- interface transmission (eqs. 7, 8, 11, 14, 15), the chained model
// transducer -> interface 1 -> ... -> field (Sec. 2.1 applied once per interface), and
// the pressure conversion.
#include <cmath>
#include <cstdlib>

#include "rsi_device.h"

namespace rsi {

constexpr int kMaxInterfaces = 32;

struct Layers {
    int m;                         // interface index (1-based) the coefficients are for
    double h[kMaxInterfaces];      // vertical thickness of each layer above interface m
    double c[kMaxInterfaces + 1];  // speeds of media 0..m
    double rho[kMaxInterfaces + 1];
    double c_max;                  // fastest of media 0..m-1
    double C_global;               // slowness of the beam axis (RSI_T_GLOBAL)
    double xc, yc;                 // transducer face centre (horizontal)
};

// Slowness C of the refracted ray reaching horizontal distance `rho_h` through the
// layers (eqs. 14-15): sum_l h_l C c_l / sqrt(1 - C^2 c_l^2) = rho_h.  Newton steps
// on a shrinking bracket [lo, hi] of 0 <= C < 1/c_max; bisection whenever a step
// leaves the bracket.
__device__ double ray_slowness_dev(const Layers &L, double rho_h) {
    if (rho_h <= 0.0) return 0.0;
    double lo = 0.0, hi = 1.0 / L.c_max;
    // start from the straight line through the whole stack, scaled into the bracket
    double H = 0.0;
    for (int l = 0; l < L.m; ++l) H += L.h[l];
    double C = (rho_h / sqrt(rho_h * rho_h + H * H)) / L.c_max;
    for (int it = 0; it < 200; ++it) {
        double f = -rho_h, df = 0.0;
        for (int l = 0; l < L.m; ++l) {
            const double sc = C * L.c[l];
            const double q = 1.0 - sc * sc;
            const double sq = sqrt(q);
            f += L.h[l] * sc / sq;
            df += L.h[l] * L.c[l] / (q * sq);
        }
        if (f < 0.0) lo = C; else hi = C;
        double Cn = C - f / df;
        if (!(Cn > lo && Cn < hi)) Cn = 0.5 * (lo + hi);
        if (fabs(Cn - C) <= 1e-17 * fabs(C) || Cn == lo || Cn == hi) {
            C = Cn;
            break;
        }
        C = Cn;
    }
    return C;
}

__device__ inline void cos_of_sine(double s, double &re, double &im) {
    if (s <= 1.0) {
        re = sqrt(1.0 - s * s);
        im = 0.0;
    } else {  // past the critical angle: the branch decaying away from the plane
        re = 0.0;
        im = sqrt(s * s - 1.0);
    }
}

// Transmission (REFLECT = false, eq. 11) or reflection (REFLECT = true, eq. 8)
// coefficient of interface L.m at each sample, for the incidence angle of `tmode`.
template <bool REFLECT>
__global__ void __launch_bounds__(256) coefficient_kernel(int tmode, Layers L, int64_t n,
                                                          const double *__restrict__ qx,
                                                          const double *__restrict__ qy,
                                                          double2 *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    if (tmode == RSI_T_UNITY) {  // display mode: media matched, T = 1, R = 0
        out[j] = make_double2(REFLECT ? 0.0 : 1.0, 0.0);
        return;
    }
    double C = L.C_global;
    if (tmode == RSI_T_LOCAL) {
        const double ex = qx[j] - L.xc, ey = qy[j] - L.yc;
        C = ray_slowness_dev(L, sqrt(ex * ex + ey * ey));
    }
    const int m = L.m;
    const double c1 = L.c[m - 1], c2 = L.c[m], r1 = L.rho[m - 1], r2 = L.rho[m];
    double a_re, a_im, b_re, b_im;
    cos_of_sine(C * c1, a_re, a_im);  // incidence
    cos_of_sine(C * c2, b_re, b_im);  // refraction (eq. 15)
    const double dre = r2 * c2 * a_re + r1 * c1 * b_re, dim = r2 * c2 * a_im + r1 * c1 * b_im;
    double nre, nim;
    if constexpr (REFLECT) {
        // eq. (8): R = (rho2 c2 cos a1 - rho1 c1 cos a2) / (rho2 c2 cos a1 + rho1 c1 cos a2)
        nre = r2 * c2 * a_re - r1 * c1 * b_re;
        nim = r2 * c2 * a_im - r1 * c1 * b_im;
    } else {
        // eq. (11): T = 2 rho1 c2 cos a1 / (rho2 c2 cos a1 + rho1 c1 cos a2)
        nre = 2.0 * r1 * c2 * a_re;
        nim = 2.0 * r1 * c2 * a_im;
    }
    const double d2 = dre * dre + dim * dim;
    out[j] = make_double2((nre * dre + nim * dim) / d2, (nim * dre - nre * dim) / d2);
}

static rsi_status make_layers(rsi_tmode tmode, int m, const double *zif, const rsi_medium *media,
                              const double *xc, const double *axis, Layers &L) {
    if (m < 1 || m > kMaxInterfaces) return RSI_ERR_SIZE;
    if (!zif || !media) return RSI_ERR_NULL;
    for (int l = 0; l <= m; ++l)
        if (!(media[l].c > 0.0) || !(media[l].rho > 0.0)) return RSI_ERR_ARG;
    L = Layers{};
    L.m = m;
    if (tmode == RSI_T_LOCAL) {
        if (!xc) return RSI_ERR_NULL;
        L.h[0] = zif[0] - xc[2];
        if (!(L.h[0] > 0.0)) return RSI_ERR_ARG;  // the source must lie above interface 1
        L.xc = xc[0];
        L.yc = xc[1];
    }
    for (int l = 1; l < m; ++l) {
        L.h[l] = zif[l] - zif[l - 1];
        if (!(L.h[l] > 0.0)) return RSI_ERR_ARG;
    }
    L.c_max = 0.0;
    for (int l = 0; l <= m; ++l) {
        L.c[l] = media[l].c;
        L.rho[l] = media[l].rho;
        if (l < m && L.c[l] > L.c_max) L.c_max = L.c[l];
    }
    if (tmode == RSI_T_GLOBAL) {
        if (!axis) return RSI_ERR_NULL;
        const double an = sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
        if (!(an > 0.0)) return RSI_ERR_ARG;
        L.C_global = sqrt(axis[0] * axis[0] + axis[1] * axis[1]) / an / media[0].c;
    }
    return RSI_OK;
}

rsi_status coefficient_device(bool reflect, rsi_tmode tmode, int m, const double *zif,
                              const rsi_medium *media, const double *xc, const double *axis,
                              int64_t n, const double *qx, const double *qy, double *out,
                              hipStream_t s) {
    if (tmode != RSI_T_GLOBAL && tmode != RSI_T_LOCAL && tmode != RSI_T_UNITY) return RSI_ERR_ARG;
    if (n < 0) return RSI_ERR_SIZE;
    Layers L;
    RSI_TRY(make_layers(tmode, m, zif, media, xc, axis, L));
    if (n == 0) return RSI_OK;
    if (!out || (tmode == RSI_T_LOCAL && (!qx || !qy))) return RSI_ERR_NULL;
    const dim3 g((unsigned)((n + 255) / 256));
    if (reflect)
        hipLaunchKernelGGL(coefficient_kernel<true>, g, dim3(256), 0, s, (int)tmode, L, n, qx, qy,
                           reinterpret_cast<double2 *>(out));
    else
        hipLaunchKernelGGL(coefficient_kernel<false>, g, dim3(256), 0, s, (int)tmode, L, n, qx, qy,
                           reinterpret_cast<double2 *>(out));
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

rsi_status transmission_device(rsi_tmode tmode, int m, const double *zif,
                               const rsi_medium *media, const double *xc, const double *axis,
                               int64_t n, const double *qx, const double *qy, double *out,
                               hipStream_t s) {
    return coefficient_device(false, tmode, m, zif, media, xc, axis, n, qx, qy, out, s);
}

// out += add (complex, n elements)
template <typename T2>
__global__ void __launch_bounds__(256) add_kernel(int64_t n, const T2 *__restrict__ add, T2 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    T2 v = out[i];
    const T2 a = add[i];
    v.x += a.x;
    v.y += a.y;
    out[i] = v;
}

static rsi_status add_into(bool fp32, int64_t n, const void *add, void *out, hipStream_t s) {
    if (n == 0) return RSI_OK;
    const dim3 g((unsigned)((n + 255) / 256));
    if (fp32)
        hipLaunchKernelGGL(add_kernel<float2>, g, dim3(256), 0, s, n, static_cast<const float2 *>(add),
                           static_cast<float2 *>(out));
    else
        hipLaunchKernelGGL(add_kernel<double2>, g, dim3(256), 0, s, n, static_cast<const double2 *>(add),
                           static_cast<double2 *>(out));
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

template <typename T2>
__global__ void __launch_bounds__(256) pressure_kernel(int64_t n, const T2 *__restrict__ phi,
                                                       double scale, T2 *__restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const T2 v = phi[i];
    T2 r;
    r.x = -scale * (double)v.y;  // i omega rho phi
    r.y = scale * (double)v.x;
    p[i] = r;
}

// ---------------------------------------------------------------------------
// Chain orchestration.
// ---------------------------------------------------------------------------
rsi_status validate_chain(const rsi_transducer *xd, const rsi_interface *ifaces, int n_if,
                                 const rsi_medium *media, const rsi_points *tgt,
                                 const double *freqs, int n_freq, rsi_tmode tmode,
                                 rsi_precision prec, uint32_t flags, void *out) {
    if ((flags & ~(uint32_t)(RSI_CHAIN_OMNI | RSI_CHAIN_ABOVE)) != 0) return RSI_ERR_ARG;
    if ((flags & RSI_CHAIN_ABOVE) && n_if < 1) return RSI_ERR_ARG;
    if (!xd || !media || !tgt || (n_if > 0 && !ifaces) || (n_freq > 0 && !freqs))
        return RSI_ERR_NULL;
    if (n_if < 0 || n_if > kMaxInterfaces || n_freq < 0) return RSI_ERR_SIZE;
    if (prec != RSI_FP32 && prec != RSI_FP64) return RSI_ERR_ARG;
    if (tmode != RSI_T_GLOBAL && tmode != RSI_T_LOCAL && tmode != RSI_T_UNITY) return RSI_ERR_ARG;
    for (int l = 0; l <= n_if; ++l)
        if (!(media[l].c > 0.0) || !(media[l].rho > 0.0)) return RSI_ERR_ARG;
    for (int f = 0; f < n_freq; ++f)
        if (!(freqs[f] > 0.0) || !std::isfinite(freqs[f])) return RSI_ERR_ARG;
    if (xd->pts.n < 0 || tgt->n < 0) return RSI_ERR_SIZE;
    for (int m = 0; m < n_if; ++m) {
        if (ifaces[m].pts.n < 0) return RSI_ERR_SIZE;
        if (m > 0 && !(ifaces[m].z > ifaces[m - 1].z)) return RSI_ERR_ARG;
        if (ifaces[m].pts.n > 0 &&
            (!ifaces[m].pts.x || !ifaces[m].pts.y || !ifaces[m].pts.z || !ifaces[m].w))
            return RSI_ERR_NULL;
    }
    if (n_if > 0 && tmode == RSI_T_LOCAL && !(ifaces[0].z > xd->centre[2])) return RSI_ERR_ARG;
    if (xd->pts.n > 0 && (!xd->pts.x || !xd->pts.y || !xd->pts.z || !xd->w)) return RSI_ERR_NULL;
    if (tgt->n > 0 && n_freq > 0 && (!out || !tgt->x || !tgt->y || !tgt->z)) return RSI_ERR_NULL;
    return RSI_OK;
}

rsi_status alloc_chain(const AllocFn &alloc, const rsi_transducer *xd, const rsi_interface *ifaces,
                       int n_if, const rsi_points *tgt, const double *freqs, int n_freq,
                       rsi_precision prec, uint32_t flags, ChainWork &W) {
    static const bool mf_enabled = [] {
        const char *v = std::getenv("RSI_MULTIFREQ");  // "0" disables the batched stages
        return !(v && v[0] == '0');
    }();
    W.flags = flags;
    const bool above = (flags & RSI_CHAIN_ABOVE) != 0;
    W.multifreq = mf_enabled && prec == RSI_FP32 && uniform_grid(freqs, n_freq, W.f0, W.df);
    W.tco.assign(n_if, nullptr);
    W.bbox.assign(n_if + 1, nullptr);
    W.setf.assign(n_if + 1, SrcSetF{});
    W.setd.assign(n_if + 1, SrcSetD{});
    int64_t nmax = 1, nslot = 0;
    auto slots = [&](int64_t ns, int64_t nt) {
        const PairShape sh = default_shape(ns, nt, prec == RSI_FP32 ? kFewWaves / 8 : 0);
        const int64_t ps = partial_slots(sh, ns, nt);
        if (ps > nslot) nslot = ps;
    };
    for (int m = 0; m <= n_if; ++m) {
        const rsi_points &sp = (m == 0) ? xd->pts : ifaces[m - 1].pts;
        const rsi_points &tp = (m == n_if) ? *tgt : ifaces[m].pts;
        slots(sp.n, tp.n);
        if (above && m == n_if - 1) slots(sp.n, tgt->n);  // incident field at the points
        if (m < n_if && ifaces[m].pts.n > nmax) nmax = ifaces[m].pts.n;
        if (prec == RSI_FP32) {
            RSI_TRY(alloc((void **)&W.setf[m].rec, sizeof(SrcRecF) * (size_t)(sp.n > 0 ? sp.n : 1)));
            RSI_TRY(alloc((void **)&W.setf[m].anchor, sizeof(double) * 4));
            RSI_TRY(alloc((void **)&W.bbox[m], sizeof(double) * kBBoxBlocks * 6));
        } else {
            RSI_TRY(alloc((void **)&W.setd[m].rec, sizeof(SrcRecD) * (size_t)(sp.n > 0 ? sp.n : 1)));
        }
    }
    for (int m = 0; m < n_if; ++m)
        RSI_TRY(alloc((void **)&W.tco[m], sizeof(double) * 2 * (size_t)(ifaces[m].pts.n > 0 ? ifaces[m].pts.n : 1)));
    const size_t esz = prec == RSI_FP32 ? sizeof(float2) : sizeof(double2);
    const size_t nf = W.multifreq ? (size_t)n_freq : 1;
    if (above) {
        const int64_t nl = ifaces[n_if - 1].pts.n;
        RSI_TRY(alloc((void **)&W.rco, sizeof(double) * 2 * (size_t)(nl > 0 ? nl : 1)));
        RSI_TRY(alloc(&W.above, esz * (size_t)(tgt->n > 0 ? tgt->n : 1) * nf));
    }
    RSI_TRY(alloc(&W.field[0], esz * (size_t)nmax * nf));
    RSI_TRY(alloc(&W.field[1], esz * (size_t)nmax * nf));
    if (W.multifreq) {
        const size_t nf_pad = (size_t)mf_pad(n_freq);
        RSI_TRY(alloc((void **)&W.S, sizeof(float2) * (size_t)nmax * nf_pad));
        W.partial = nullptr;  // the multi-frequency stages write their outputs directly
        return RSI_OK;
    }
    RSI_TRY(alloc(&W.partial, esz * (size_t)(nslot > 0 ? nslot : 1)));
    return RSI_OK;
}

// Enqueue the whole chain on `s` using the workspace W (flags as given to alloc_chain).
rsi_status enqueue_chain(const rsi_transducer *xd, const rsi_interface *ifaces, int n_if,
                                const rsi_medium *media, const rsi_points *tgt,
                                const double *freqs, int n_freq, rsi_tmode tmode,
                                rsi_precision prec, void *out, ChainWork &W, hipStream_t s) {
    static const double nz[3] = {0.0, 0.0, 1.0};
    const bool omni = (W.flags & RSI_CHAIN_OMNI) != 0, above = (W.flags & RSI_CHAIN_ABOVE) != 0;
    const bool fp32 = prec == RSI_FP32;
    // interface sources: the dipole of eq. 7, or omnidirectional sources (the monopole
    // sum of strengths times ik); the reflection radiates along -z: the dipole sum with
    // the strengths negated (the kernel is linear in the normal), omni unchanged
    const rsi_kernel ikind = omni ? RSI_MONOPOLE : RSI_DIPOLE;
    std::vector<double> zif(n_if > 0 ? n_if : 1);
    for (int m = 0; m < n_if; ++m) zif[m] = ifaces[m].z;
    // geometry of every source set, once for all frequencies
    for (int m = 0; m <= n_if; ++m) {
        const rsi_points &sp = (m == 0) ? xd->pts : ifaces[m - 1].pts;
        const double *w = (m == 0) ? xd->w : ifaces[m - 1].w;
        if (fp32) {
            if (sp.n > 0) {
                RSI_TRY(bbox_partials(sp, W.bbox[m], s));
                // real strengths (v0, or zero until set per frequency): no wavelength needed
                RSI_TRY(prep_sources_f32(sp, w, nullptr, m == 0 ? xd->v0 : 0.0, m == 0 ? nullptr : nz,
                                         W.bbox[m], 0.0, Cplx{1.0, 0.0}, W.setf[m], s));
            } else {
                W.setf[m].n = 0;
            }
        } else {
            RSI_TRY(prep_sources_f64(sp, w, nullptr, m == 0 ? xd->v0 : 0.0, Cplx{1.0, 0.0}, W.setd[m], s));
        }
    }
    const int n_tr = above ? n_if - 1 : n_if;  // interfaces that transmit
    for (int m = 1; m <= n_tr; ++m)
        RSI_TRY(transmission_device(tmode, m, zif.data(), media, xd->centre, xd->axis,
                                    ifaces[m - 1].pts.n, ifaces[m - 1].pts.x, ifaces[m - 1].pts.y,
                                    W.tco[m - 1], s));
    if (above)
        RSI_TRY(coefficient_device(true, tmode, n_if, zif.data(), media, xd->centre, xd->axis,
                                   ifaces[n_if - 1].pts.n, ifaces[n_if - 1].pts.x,
                                   ifaces[n_if - 1].pts.y, W.rco, s));
    const Targets T_out{tgt->x, tgt->y, tgt->z, tgt->n};
    if (W.multifreq) {
        // every stage once for all frequencies; fields are [n_freq][n].  Stage m > 0 reads
        // field[cur] and writes field[cur ^ 1]; the field at the last transmitting
        // stage's targets ends in field[cur].
        int cur = 0;
        for (int m = 0; m <= n_tr; ++m) {
            const bool last = (m == n_tr);
            const rsi_points &tp = (last && !above) ? *tgt : ifaces[m].pts;
            const Targets t{tp.x, tp.y, tp.z, tp.n};
            float2 *dst = (last && !above) ? static_cast<float2 *>(out)
                                           : static_cast<float2 *>(W.field[m == 0 ? 0 : cur ^ 1]);
            const float2 *S = nullptr;  // stage 0: the transducer's shared real strengths
            rsi_kernel kind = RSI_MONOPOLE;
            if (m > 0) {
                // strengths T phi (times ik for omnidirectional sources)
                RSI_TRY(strength_multifreq(W.setf[m].n, n_freq, ifaces[m - 1].w,
                                           static_cast<const float2 *>(W.field[cur]), W.tco[m - 1],
                                           omni ? 0.0 : 1.0, omni ? 1.0 : 0.0, media[m].c, W.f0, W.df,
                                           W.S, s));
                S = W.S;
                kind = ikind;
            }
            RSI_TRY(pairsum_multifreq_f32(W.setf[m], S, t, kind, m > 0, media[m].c, W.f0, W.df, n_freq,
                                          dst, s));
            if (last && above)  // incident field at the points, from the same sources
                RSI_TRY(pairsum_multifreq_f32(W.setf[m], S, T_out, kind, m > 0, media[m].c, W.f0, W.df,
                                              n_freq, static_cast<float2 *>(out), s));
            if (m > 0) cur ^= 1;
        }
        if (above) {
            // reflection at interface n_if back into medium n_if - 1
            RSI_TRY(strength_multifreq(W.setf[n_if].n, n_freq, ifaces[n_if - 1].w,
                                       static_cast<const float2 *>(W.field[cur]), W.rco,
                                       omni ? 0.0 : -1.0, omni ? 1.0 : 0.0, media[n_if - 1].c, W.f0,
                                       W.df, W.S, s));
            RSI_TRY(pairsum_multifreq_f32(W.setf[n_if], W.S, T_out, ikind, true, media[n_if - 1].c, W.f0,
                                          W.df, n_freq, static_cast<float2 *>(W.above), s));
            RSI_TRY(add_into(true, (int64_t)n_freq * tgt->n, W.above, out, s));
        }
        return RSI_OK;
    }
    const size_t esz = fp32 ? sizeof(float2) : sizeof(double2);
    for (int f = 0; f < n_freq; ++f) {
        char *out_f = static_cast<char *>(out) + esz * (size_t)f * (size_t)tgt->n;
        const double k_of = kTwoPi * freqs[f];  // k = k_of / c
        int cur = 0;
        // one pair sum of source set m (medium mm, kernel kind) onto t into dst
        auto psum = [&](int m, int mm, rsi_kernel kind, const Targets &t, void *dst) -> rsi_status {
            const rsi_points &sp = (m == 0) ? xd->pts : ifaces[m - 1].pts;
            const PairShape sh = default_shape(sp.n, t.n, fp32 ? kFewWaves / 8 : 0);
            if (fp32)
                // interface samples lie on their plane (ABI contract): planar kernel
                return pairsum_f32(W.setf[m], t, kind, m == 0 ? nullptr : nz, media[mm].c, freqs[f], sh,
                                   static_cast<float2 *>(W.partial), static_cast<float2 *>(dst), s, m > 0);
            return pairsum_f64(W.setd[m], t, kind, m == 0 ? nullptr : nz, media[mm].c, freqs[f], sh,
                               static_cast<double2 *>(W.partial), static_cast<double2 *>(dst), s);
        };
        // strengths of interface set m from the field at its samples with coefficient c
        // and stage factor F
        auto strengths = [&](int m, const double *coef, Cplx F, double c_stage) -> rsi_status {
            if (fp32)
                return set_strength_f32(W.setf[m], ifaces[m - 1].w, W.field[cur], false, coef,
                                        c_stage / freqs[f], F, s);
            return set_strength_f64(W.setd[m], ifaces[m - 1].w, static_cast<const double *>(W.field[cur]),
                                    coef, F, s);
        };
        for (int m = 0; m <= n_tr; ++m) {
            const bool last = (m == n_tr);
            const rsi_points &tp = (last && !above) ? *tgt : ifaces[m].pts;
            const Targets t{tp.x, tp.y, tp.z, tp.n};
            // stage m reads field[cur] (m > 0) and writes field[cur ^ 1], or the output
            void *dst = (last && !above) ? (void *)out_f : W.field[m == 0 ? 0 : cur ^ 1];
            const rsi_kernel kind = m == 0 ? RSI_MONOPOLE : ikind;
            if (m > 0)
                RSI_TRY(strengths(m, W.tco[m - 1],
                                  omni ? Cplx{0.0, k_of / media[m].c} : Cplx{1.0, 0.0}, media[m].c));
            RSI_TRY(psum(m, m, kind, t, dst));
            if (last && above) RSI_TRY(psum(m, m, kind, T_out, out_f));  // incident field
            if (m > 0) cur ^= 1;
        }
        if (above) {
            // reflection at interface n_if back into medium n_if - 1 (field at its samples
            // in field[cur])
            const int ml = n_if - 1;
            RSI_TRY(strengths(n_if, W.rco,
                              omni ? Cplx{0.0, k_of / media[ml].c} : Cplx{-1.0, 0.0}, media[ml].c));
            RSI_TRY(psum(n_if, ml, ikind, T_out, W.above));
            RSI_TRY(add_into(fp32, tgt->n, W.above, out_f, s));
        }
    }
    return RSI_OK;
}

}  // namespace rsi

using namespace rsi;

std::vector<DevSpan> rsi::chain_inputs(const rsi_transducer *xd, const rsi_interface *ifaces,
                                       int n_if, const rsi_points *tgt) {
    std::vector<DevSpan> in;
    add_points(in, xd->pts);
    in.push_back({xd->w, xd->pts.n});
    for (int m = 0; m < n_if; ++m) {
        add_points(in, ifaces[m].pts);
        in.push_back({ifaces[m].w, ifaces[m].pts.n});
    }
    add_points(in, *tgt);
    return in;
}

extern "C" {

rsi_status rsi_transmission(rsi_tmode tmode, int m, const double *zif, const rsi_medium *media,
                            const double *xc, const double *axis, int64_t n, const double *qx,
                            const double *qy, double *out, void *stream) {
    return transmission_device(tmode, m, zif, media, xc, axis, n, qx, qy, out, as_stream(stream));
}

rsi_status rsi_to_pressure(int64_t n, const void *phi, rsi_precision prec, double rho,
                           double freq, void *p, void *stream) {
    if (n < 0) return RSI_ERR_SIZE;
    if (prec != RSI_FP32 && prec != RSI_FP64) return RSI_ERR_ARG;
    if (!(rho > 0.0) || !(freq > 0.0)) return RSI_ERR_ARG;
    if (n == 0) return RSI_OK;
    if (!phi || !p) return RSI_ERR_NULL;
    const double scale = kTwoPi * freq * rho;
    const dim3 g((unsigned)((n + 255) / 256));
    if (prec == RSI_FP32)
        hipLaunchKernelGGL(pressure_kernel<float2>, g, dim3(256), 0, as_stream(stream), n,
                           static_cast<const float2 *>(phi), scale, static_cast<float2 *>(p));
    else
        hipLaunchKernelGGL(pressure_kernel<double2>, g, dim3(256), 0, as_stream(stream), n,
                           static_cast<const double2 *>(phi), scale, static_cast<double2 *>(p));
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

rsi_status rsi_reflection(rsi_tmode tmode, int m, const double *zif, const rsi_medium *media,
                          const double *xc, const double *axis, int64_t n, const double *qx,
                          const double *qy, double *out, void *stream) {
    return coefficient_device(true, tmode, m, zif, media, xc, axis, n, qx, qy, out, as_stream(stream));
}

rsi_status rsi_chain_ex(const rsi_transducer *xd, const rsi_interface *ifaces, int n_if,
                        const rsi_medium *media, const rsi_points *tgt, const double *freqs,
                        int n_freq, rsi_tmode tmode, rsi_precision prec, uint32_t flags, void *out,
                        void *stream) {
    RSI_TRY(validate_chain(xd, ifaces, n_if, media, tgt, freqs, n_freq, tmode, prec, flags, out));
    if (tgt->n == 0 || n_freq == 0) return RSI_OK;
    hipStream_t s = as_stream(stream);
    RSI_TRY(check_finite(s, chain_inputs(xd, ifaces, n_if, tgt)));
    Scratch scratch(s);
    ChainWork W;
    RSI_TRY(alloc_chain([&](void **p, size_t bytes) { return scratch.alloc((char **)p, bytes); },
                        xd, ifaces, n_if, tgt, freqs, n_freq, prec, flags, W));
    return enqueue_chain(xd, ifaces, n_if, media, tgt, freqs, n_freq, tmode, prec, out, W, s);
}

rsi_status rsi_chain(const rsi_transducer *xd, const rsi_interface *ifaces, int n_if,
                     const rsi_medium *media, const rsi_points *tgt, const double *freqs,
                     int n_freq, rsi_tmode tmode, rsi_precision prec, void *out, void *stream) {
    return rsi_chain_ex(xd, ifaces, n_if, media, tgt, freqs, n_freq, tmode, prec, 0u, out, stream);
}

}  // extern "C"
