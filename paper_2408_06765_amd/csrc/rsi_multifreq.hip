// rsi_multifreq.hip -- one pair sum (a stage of the chain, or rsi_propagate_multifreq)
// for many frequencies in one launch (multi-frequency superposition, Sec. 4), FP32 path.
//
// On a uniform grid f_q = f_0 + q df the phase of a pair is linear in q:
//     r f_q / c = r f_b / c + (q - q_b) r df / c,
// so e^{i k_q r} advances by the same unit phasor e^{i dk r} from one frequency to the
// next, and e_q = e^{i k_q r} obeys e_{q+1} = 2 cos(dk r) e_q - e_{q-1}.  The geometry of a
// pair (q, 1/r, r - r_ref) and two phasors (block start and step) are evaluated once per
// block of 16 or 32 frequencies; each further frequency costs two FMAs of that
// recurrence, the dipole factor (three operations) and the complex multiply-accumulate
// with that frequency's strength (four).  The recurrence depends on the step only through
// its cosine, whose rounding moves the step angle by up to about sqrt(2 ulp) where
// sin(dk r) ~ 0; over 16 frequencies this stays at a few 1e-6 of the field (float32
// emulation on the stack's last stage: 3.3e-6 worst frequency against 1.0e-6 for a complex
// rotation), and a block of 32 restarts it at its 17th frequency to stay there.
// The strengths of one source for a frequency block are contiguous (source-major,
// frequency-minor), so a wave reads them with wave-uniform loads.  SHARED_S: one real
// strength per source for every frequency (the transducer stage), taken from the record's
// signed magnitude; its phase offset is zero for real strengths.
#include <algorithm>
#include <cmath>

#include "rsi_device.h"

namespace rsi {

// Per-target constants of a multi-frequency block (FP32, from the FP64 set-up).
struct TargetMF {
    float dmx, dmy, dmz;  // -2 (P - C)
    float rr2, rr;        // r_ref^2, r_ref
    float p0b, p0d;       // frac(r_ref f_b / c), frac(r_ref df / c)
    float p0h;            // frac(r_ref f_h / c), f_h = f_b + 16 df (blocks of 32)
    float ht;             // (P - C).z: n.(P - Q) for planar sources with n = +z
};

// Per-block (wave-uniform) constants.
struct BlockMF {
    float ilb, ild, ilh;  // f_b / c, df / c, f_h / c
    float kb, dk;         // 2 pi f_b / c, 2 pi df / c
};

// Sum over sources [j0, j1) for the NB frequencies of one block into mre, mim.  FRACT:
// reduce the phase arguments with v_fract; without it they go to v_sin / v_cos as they
// are, which the caller allows only while they stay inside the hardware's own reduction
// range.
template <int KIND, bool PLANAR, bool SHARED_S, bool FRACT, int NB>
__device__ __forceinline__ void multifreq_sum(const TargetMF &T, const BlockMF &B,
                                              const SrcRecF *__restrict__ rec,
                                              const float2 *__restrict__ S, int64_t j0, int64_t j1,
                                              int nf_pad, int q0, float (&mre)[NB],
                                              float (&mim)[NB]) {
    // plain FP32 running sums over the launch's chunk of sources: with one register pair
    // per frequency the block reaches 32 frequencies at 4 waves per SIMD; the rounding of
    // the sum over a chunk of 8192 sources stays below that of the recurrence (float32
    // emulation of the volume stage: the same worst frequency as 64-source block sums)
#pragma unroll
    for (int q = 0; q < NB; ++q) mre[q] = mim[q] = 0.0f;
    const int cnt = (int)(j1 - j0);  // chunks are far below 2^31 sources
    const SrcRecF *blk = rec + j0;
    const float2 *Sb = SHARED_S ? nullptr : S + j0 * nf_pad + q0;  // S is NULL when shared
    for (int jj = 0; jj < cnt; ++jj) {  // 32-bit count: the loop test stays scalar
        const SrcRecF s = blk[jj];
        // the block's strengths up front: wave-uniform loads, all in flight at once
        float2 sv[NB];
        if constexpr (!SHARED_S) {
#pragma unroll
            for (int q = 0; q < NB; ++q) sv[q] = Sb[(int64_t)jj * nf_pad + q];
        }
        float t = T.dmx * s.ex;
        t = fmaf(T.dmy, s.ey, t);
        if constexpr (!PLANAR) t = fmaf(T.dmz, s.ez, t);
        const float qq = t + s.es2;
        const float r2 = T.rr2 + qq;
        const float ir = __builtin_amdgcn_rsqf(fabsf(r2));
        const float dr = qq * __builtin_amdgcn_rcpf(fmaf(r2, ir, T.rr));
        float phb = fmaf(dr, B.ilb, T.p0b), phd = fmaf(dr, B.ild, T.p0d);
        if constexpr (FRACT) {
            phb = __builtin_amdgcn_fractf(phb);
            phd = __builtin_amdgcn_fractf(phd);
        }
        const float cd = __builtin_amdgcn_cosf(phd), sd = __builtin_amdgcn_sinf(phd);
        float amp = ir;  // monopole: e^{ikr}/r
        float kr = 0.0f, dkr = 0.0f;
        if constexpr (KIND == RSI_DIPOLE) {
            // (cos(theta)/r)(ik - 1/r) = -(cos(theta)/r^2)(1 - i k r): the real factor goes
            // into the amplitude, k_q r = k_b r + q dk r is carried by one add per frequency
            const float hh = PLANAR ? T.ht : T.ht - s.h;
            amp = -hh * ir * ir * ir;
            const float r = r2 * ir;
            kr = B.kb * r;
            dkr = B.dk * r;
        }
        if constexpr (SHARED_S) amp *= s.a;  // one real strength for every frequency
        // e_q = amp e^{i k_q r}: e_0 and e_1 from the two phasors, then the two-term
        // recurrence e_{q+1} = 2 cos(dk r) e_q - e_{q-1} (2 FMAs per frequency); a block of
        // 32 restarts it at its 17th frequency from a third phasor, which keeps the drift
        // of the recurrence at that of a block of 16
        float er = __builtin_amdgcn_cosf(phb) * amp, ei = __builtin_amdgcn_sinf(phb) * amp;
        float nr = fmaf(er, cd, -ei * sd), ni = fmaf(er, sd, ei * cd);
        const float tc = cd + cd;
        float hr = 0.0f, hi = 0.0f;  // e_16 (blocks of 32)
        if constexpr (NB > 16) {
            float phh = fmaf(dr, B.ilh, T.p0h);
            if constexpr (FRACT) phh = __builtin_amdgcn_fractf(phh);
            hr = __builtin_amdgcn_cosf(phh) * amp;
            hi = __builtin_amdgcn_sinf(phh) * amp;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            float gr = er, gi = ei;
            if constexpr (KIND == RSI_DIPOLE) {  // (1 - i k_q r) e_q
                gr = fmaf(kr, ei, er);
                gi = fmaf(-kr, er, ei);
                kr += dkr;
            }
            if constexpr (SHARED_S) {
                mre[q] += gr;
                mim[q] += gi;
            } else {
                mre[q] = fmaf(sv[q].x, gr, mre[q]);
                mre[q] = fmaf(-sv[q].y, gi, mre[q]);
                mim[q] = fmaf(sv[q].x, gi, mim[q]);
                mim[q] = fmaf(sv[q].y, gr, mim[q]);
            }
            if (q == 15 && NB > 16) {  // e_16, e_17 from the third phasor
                er = hr;
                ei = hi;
                nr = fmaf(er, cd, -ei * sd);
                ni = fmaf(er, sd, ei * cd);
            } else if (q + 2 < NB) {  // e_{q+2} from e_{q+1} and e_q
                const float tr = fmaf(tc, nr, -er), ti = fmaf(tc, ni, -ei);
                er = nr;
                ei = ni;
                nr = tr;
                ni = ti;
            } else {
                er = nr;
                ei = ni;
            }
        }
    }
}

// Sources [j0, j1) of one launch; `accumulate`: add to what `out` holds (the sum of the
// earlier source chunks, from earlier launches on the same stream) instead of storing.
template <int KIND, bool PLANAR, bool SHARED_S, int NB>
__global__ void __launch_bounds__(kBlock) multifreq_f32_kernel(
    const SrcRecF *__restrict__ rec, const float2 *__restrict__ S, int64_t j0, int64_t j1,
    int nf_pad, const double *__restrict__ tx, const double *__restrict__ ty,
    const double *__restrict__ tz, int64_t n_tgt, const double *__restrict__ anchor, double f0,
    double df, int n_freq, double inv_c, int accumulate, float2 *__restrict__ out) {
    const int q0 = blockIdx.y * NB;
    const double fb = f0 + q0 * df, fh = fb + 16 * df;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < n_tgt;
    if (!valid) i = n_tgt - 1;
    // per target, in FP64: reference distance and the reference phases
    const double dx = tx[i] - anchor[0], dy = ty[i] - anchor[1], dz = tz[i] - anchor[2];
    const double rr2d = dx * dx + dy * dy + dz * dz, rrd = sqrt(rr2d);
    double pb = rrd * fb * inv_c, pd = rrd * df * inv_c, ph = rrd * fh * inv_c;
    pb -= floor(pb);
    pd -= floor(pd);
    ph -= floor(ph);
    TargetMF T;
    T.dmx = (float)(-2.0 * dx);
    T.dmy = (float)(-2.0 * dy);
    T.dmz = (float)(-2.0 * dz);
    T.rr2 = (float)rr2d;
    T.rr = (float)rrd;
    T.p0b = (float)pb;
    T.p0d = (float)pd;
    T.p0h = (float)ph;
    T.ht = (float)dz;  // n = +z for the interface (dipole) stages
    BlockMF B;
    B.ilb = (float)(fb * inv_c);
    B.ild = (float)(df * inv_c);
    B.ilh = (float)(fh * inv_c);
    B.kb = (float)(kTwoPi * fb * inv_c);
    B.dk = (float)(kTwoPi * df * inv_c);
    float mre[NB], mim[NB];
    // |r - r_ref| <= R (the set's half diagonal), so every phase argument stays within
    // 1 + R f / c revolutions for the largest of the frequencies it is taken at
    const double fmax = NB > 16 ? (fh > df ? fh : df) : (fb > df ? fb : df);
    if (phase_in_sin_range(anchor[3], fmax * inv_c))
        multifreq_sum<KIND, PLANAR, SHARED_S, false, NB>(T, B, rec, S, j0, j1, nf_pad, q0, mre, mim);
    else
        multifreq_sum<KIND, PLANAR, SHARED_S, true, NB>(T, B, rec, S, j0, j1, nf_pad, q0, mre, mim);
    if (!valid) return;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        if (q0 + q >= n_freq) continue;
        float2 &o = out[(int64_t)(q0 + q) * n_tgt + i];
        if (accumulate) {
            const float2 p = o;
            o = make_float2(p.x + mre[q], p.y + mim[q]);
        } else {
            o = make_float2(mre[q], mim[q]);
        }
    }
}

// S[j][q] = -(1/2pi) w_j T_j phi_q(Q_j) F_q for q < n_freq, 0 for the padding, with the
// stage factor F_q = Fa + i Fb k_q (1; ik_q for omnidirectional sources; -1 for a dipole
// radiating along -z), k_q = 2 pi (f0 + q df) / c.
__global__ void __launch_bounds__(256) strength_multifreq_kernel(
    int64_t n, int n_freq, int nf_pad, const double *__restrict__ w,
    const float2 *__restrict__ field /* [n_freq][n] */, const double *__restrict__ tco,
    double Fa, double Fb, double c, double f0, double df, float2 *__restrict__ S) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= n * nf_pad) return;
    const int64_t j = g / nf_pad;
    const int q = (int)(g - j * nf_pad);
    float2 r = make_float2(0.0f, 0.0f);
    if (q < n_freq) {
        const float2 f = field[(int64_t)q * n + j];
        const double tre = tco[2 * j], tim = tco[2 * j + 1];
        const double scale = -w[j] / kTwoPi;
        const double sre = tre * f.x - tim * f.y, sim = tre * f.y + tim * f.x;
        const double Fi = Fb * kTwoPi * (f0 + q * df) / c;
        r.x = (float)(scale * (sre * Fa - sim * Fi));
        r.y = (float)(scale * (sre * Fi + sim * Fa));
    }
    S[g] = r;
}

// S[j][q] = -(1/2pi) w_j v_q(j) (Fa + i Fb k_q) for q < n_freq, 0 for the padding, with the
// caller's complex FP64 strengths v [n_freq][n] (v = 1 when vel is NULL),
// k_q = 2 pi (f0 + q df) / c.
__global__ void __launch_bounds__(256) strength_vel_multifreq_kernel(
    int64_t n, int n_freq, int nf_pad, const double *__restrict__ w, const double *__restrict__ vel,
    double Fa, double Fb, double c, double f0, double df, float2 *__restrict__ S) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= n * nf_pad) return;
    const int64_t j = g / nf_pad;
    const int q = (int)(g - j * nf_pad);
    float2 r = make_float2(0.0f, 0.0f);
    if (q < n_freq) {
        double vre = 1.0, vim = 0.0;
        if (vel) {
            vre = vel[2 * ((int64_t)q * n + j)];
            vim = vel[2 * ((int64_t)q * n + j) + 1];
        }
        const double scale = -w[j] / kTwoPi;
        const double Fi = Fb * kTwoPi * (f0 + q * df) / c;
        r.x = (float)(scale * (vre * Fa - vim * Fi));
        r.y = (float)(scale * (vre * Fi + vim * Fa));
    }
    S[g] = r;
}

__global__ void __launch_bounds__(256) zero_f2_kernel(int64_t n, float2 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = make_float2(0.0f, 0.0f);
}

bool uniform_grid(const double *freqs, int n, double &f0, double &df) {
    if (n < 2) return false;
    f0 = freqs[0];
    df = (freqs[n - 1] - freqs[0]) / (n - 1);
    if (!(df > 0.0)) return false;
    for (int q = 0; q < n; ++q)
        if (std::fabs(freqs[q] - (f0 + q * df)) > 1e-9 * std::fabs(freqs[n - 1])) return false;
    return true;
}

int mf_block(int n_freq) {
    static const int forced = env_int("RSI_MF_BLOCK", 0);
    if (forced == 16 || forced == 32) return forced;
    // a block of 32 costs 0.88 of two blocks of 16 per pair-frequency (measured on the
    // volume stage); it pays unless its padding outweighs that
    const int p16 = (n_freq + 15) / 16 * 16, p32 = (n_freq + 31) / 32 * 32;
    return 0.88 * p32 < p16 ? 32 : 16;
}

int mf_pad(int n_freq) {
    const int nb = mf_block(n_freq);
    return (n_freq + nb - 1) / nb * nb;
}

rsi_status strength_multifreq(int64_t n, int n_freq, const double *w, const float2 *field,
                              const double *tco, double Fa, double Fb, double c, double f0,
                              double df, float2 *S, hipStream_t s) {
    if (n == 0) return RSI_OK;
    const int nf_pad = mf_pad(n_freq);
    const int64_t total = n * nf_pad;
    hipLaunchKernelGGL(strength_multifreq_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256),
                       0, s, n, n_freq, nf_pad, w, field, tco, Fa, Fb, c, f0, df, S);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

rsi_status pairsum_multifreq_f32(const SrcSetF &set, const float2 *S, const Targets &t,
                                 rsi_kernel kind, bool planar_z, double c, double f0, double df,
                                 int n_freq, float2 *out, hipStream_t s) {
    if (t.n == 0 || n_freq == 0) return RSI_OK;
    const int nb = mf_block(n_freq);
    const int nf_pad = mf_pad(n_freq);
    const int nfb = nf_pad / nb;
    const int64_t bx = (t.n + kBlock - 1) / kBlock;
    if (bx > 0x7fffffff || nfb > 65535) return RSI_ERR_SIZE;
    const dim3 grid((unsigned)bx, (unsigned)nfb);
    const double inv_c = 1.0 / c;
    const bool shared = (S == nullptr);
    if (kind != RSI_MONOPOLE && !planar_z) return RSI_ERR_UNSUPPORTED;  // interface stages are planar (+z)
    // One launch per chunk of sources, each adding to the output in chunk order (the sum
    // stays deterministic).  A chunk's records and strengths (288 B per source for a block
    // of 32 frequencies: 2.4 MB for 8192 sources) fit one XCD's 4 MB L2, and the
    // workgroups in flight at any time all read the same chunk, because they are
    // dispatched in order and every target tile of a chunk comes before the next chunk.
    // Without chunks every workgroup streams the whole source set at its own pace and the
    // L2 misses on nearly every record.  Measured on 2^18 sources x 2^18 points x 64
    // frequencies: 992, 1005, 1038, 1047 ms for chunks of 8192, 16384, 32768, 65536
    // sources, 1011 ms for one launch.
    static const int64_t chunk = std::max<int64_t>(kSub, (int64_t)env_int("RSI_MF_CHUNK", 8192) / kSub * kSub);
    const int64_t n_src = set.n > 0 ? set.n : 0;
    int64_t j0 = 0;
    do {
        const int64_t j1 = (n_src - j0 > chunk) ? j0 + chunk : n_src;
        const int acc = j0 > 0 ? 1 : 0;
#define RSI_MF_LAUNCH(K, P, SH)                                                                   \
    do {                                                                                          \
        if (nb == 32)                                                                             \
            hipLaunchKernelGGL((multifreq_f32_kernel<K, P, SH, 32>), grid, dim3(kBlock), 0, s,     \
                               set.rec, S, j0, j1, nf_pad, t.x, t.y, t.z, t.n, set.anchor, f0, df, \
                               n_freq, inv_c, acc, out);                                          \
        else                                                                                      \
            hipLaunchKernelGGL((multifreq_f32_kernel<K, P, SH, 16>), grid, dim3(kBlock), 0, s,     \
                               set.rec, S, j0, j1, nf_pad, t.x, t.y, t.z, t.n, set.anchor, f0, df, \
                               n_freq, inv_c, acc, out);                                          \
    } while (0)
        if (kind == RSI_MONOPOLE) {
            if (shared) {
                if (planar_z) RSI_MF_LAUNCH(RSI_MONOPOLE, true, true);
                else RSI_MF_LAUNCH(RSI_MONOPOLE, false, true);
            } else {
                if (planar_z) RSI_MF_LAUNCH(RSI_MONOPOLE, true, false);
                else RSI_MF_LAUNCH(RSI_MONOPOLE, false, false);
            }
        } else {
            if (shared) RSI_MF_LAUNCH(RSI_DIPOLE, true, true);
            else RSI_MF_LAUNCH(RSI_DIPOLE, true, false);
        }
#undef RSI_MF_LAUNCH
        RSI_HIP(hipGetLastError());
        j0 = j1;
    } while (j0 < n_src);
    return RSI_OK;
}

}  // namespace rsi

using namespace rsi;

extern "C" rsi_status rsi_propagate_multifreq(const rsi_points *src, const double *src_w,
                                              const double *src_vel, const double *normal,
                                              const rsi_points *tgt, rsi_medium medium,
                                              const double *freqs, int n_freq, rsi_kernel kind,
                                              rsi_precision prec, uint32_t flags, void *out,
                                              void *stream) {
    if (n_freq < 0) return RSI_ERR_SIZE;
    if (n_freq == 0) return RSI_OK;
    if (!freqs) return RSI_ERR_NULL;
    for (int q = 0; q < n_freq; ++q)
        if (!(freqs[q] > 0.0) || !std::isfinite(freqs[q])) return RSI_ERR_ARG;
    // the per-source strengths check of the single-frequency call does not apply: NULL
    // strengths mean 1 here
    static const double one[2] = {1.0, 0.0};
    RSI_TRY(validate_propagate(src, src_w, src_vel ? src_vel : one, normal, tgt, medium, freqs[0], kind,
                               prec, flags, out));
    if (tgt->n == 0) return RSI_OK;
    if ((int64_t)n_freq * tgt->n > ((int64_t)1 << 38)) return RSI_ERR_SIZE;
    hipStream_t s = as_stream(stream);
    {
        std::vector<DevSpan> in;
        add_points(in, *src);
        in.push_back({src_w, src->n});
        if (src_vel) in.push_back({src_vel, 2 * (int64_t)n_freq * src->n});
        add_points(in, *tgt);
        RSI_TRY(check_finite(s, in));
    }
    const bool planar = (flags & RSI_FLAG_PLANAR_Z) != 0;
    // a dipole along -z is the +z dipole with the strengths negated (linear in the normal)
    bool z_normal = false;
    double sign = 1.0;
    if (kind == RSI_DIPOLE) {
        z_normal = normal[0] == 0.0 && normal[1] == 0.0;
        sign = normal[2] < 0.0 ? -1.0 : 1.0;
    }
    const rsi_kernel kk = kind == RSI_OMNI ? RSI_MONOPOLE : kind;
    const Targets t{tgt->x, tgt->y, tgt->z, tgt->n};
    Scratch scratch(s);
    double f0 = 0.0, df = 0.0;
    if (prec == RSI_FP32 && uniform_grid(freqs, n_freq, f0, df) && (kind != RSI_DIPOLE || (planar && z_normal))) {
        const int nf_pad = mf_pad(n_freq);
        if (nf_pad / mf_block(n_freq) > 65535) return RSI_ERR_SIZE;
        SrcSetF set;
        double *partials = nullptr;
        float2 *S = nullptr;
        // one real strength shared by every frequency when the strengths are all 1 and the
        // kernel has no per-frequency factor; otherwise per-frequency strengths
        const bool shared = !src_vel && kind != RSI_OMNI;
        if (src->n > 0) {
            RSI_TRY(scratch.alloc(&set.rec, (size_t)src->n));
            RSI_TRY(scratch.alloc(&set.anchor, 4));
            RSI_TRY(scratch.alloc(&partials, kBBoxBlocks * 6));
            if (!shared) RSI_TRY(scratch.alloc(&S, (size_t)src->n * nf_pad));
            RSI_TRY(bbox_partials(*src, partials, s));
            RSI_TRY(prep_sources_f32(*src, src_w, nullptr, shared ? sign : 0.0, kind == RSI_DIPOLE ? normal : nullptr,
                                     partials, 0.0, Cplx{1.0, 0.0}, set, s));
            if (!shared) {
                const int64_t total = src->n * (int64_t)nf_pad;
                hipLaunchKernelGGL(strength_vel_multifreq_kernel, dim3((unsigned)((total + 255) / 256)),
                                   dim3(256), 0, s, src->n, n_freq, nf_pad, src_w, src_vel,
                                   kind == RSI_OMNI ? 0.0 : sign, kind == RSI_OMNI ? 1.0 : 0.0, medium.c,
                                   f0, df, S);
                RSI_HIP(hipGetLastError());
            }
        }
        if (src->n == 0) {
            const int64_t total = (int64_t)n_freq * tgt->n;
            hipLaunchKernelGGL(zero_f2_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total,
                               static_cast<float2 *>(out));
            RSI_HIP(hipGetLastError());
            return RSI_OK;
        }
        return pairsum_multifreq_f32(set, S, t, kk, planar, medium.c, f0, df, n_freq,
                                     static_cast<float2 *>(out), s);
    }
    // one pair sum per frequency, strengths of frequency q from src_vel + q n
    const PairShape sh = default_shape(src->n, tgt->n, prec == RSI_FP32 ? kFewWaves / 8 : 0);
    const int64_t nslots = partial_slots(sh, src->n, tgt->n);
    const size_t esz = prec == RSI_FP32 ? sizeof(float2) : sizeof(double2);
    SrcSetF setf;
    SrcSetD setd;
    double *partials = nullptr;
    void *partial = nullptr;
    if (src->n > 0) {
        if (prec == RSI_FP32) {
            RSI_TRY(scratch.alloc(&setf.rec, (size_t)src->n));
            RSI_TRY(scratch.alloc(&setf.anchor, 4));
            RSI_TRY(scratch.alloc(&partials, kBBoxBlocks * 6));
            RSI_TRY(bbox_partials(*src, partials, s));
        } else {
            RSI_TRY(scratch.alloc(&setd.rec, (size_t)src->n));
        }
    }
    if (nslots > 0) RSI_TRY(scratch.alloc((char **)&partial, esz * (size_t)nslots));
    for (int q = 0; q < n_freq; ++q) {
        const double *vq = src_vel ? src_vel + 2 * (int64_t)q * src->n : nullptr;
        const Cplx F = kind == RSI_OMNI ? Cplx{0.0, kTwoPi * freqs[q] / medium.c} : Cplx{1.0, 0.0};
        char *out_q = static_cast<char *>(out) + esz * (size_t)q * (size_t)tgt->n;
        if (prec == RSI_FP32) {
            if (src->n > 0)
                RSI_TRY(prep_sources_f32(*src, src_w, vq, 1.0, normal, partials, medium.c / freqs[q], F,
                                         setf, s));
            RSI_TRY(pairsum_f32(setf, t, kk, normal, medium.c, freqs[q], sh, static_cast<float2 *>(partial),
                                reinterpret_cast<float2 *>(out_q), s, planar));
        } else {
            if (src->n > 0) RSI_TRY(prep_sources_f64(*src, src_w, vq, 1.0, F, setd, s));
            RSI_TRY(pairsum_f64(setd, t, kk, normal, medium.c, freqs[q], sh, static_cast<double2 *>(partial),
                                reinterpret_cast<double2 *>(out_q), s));
        }
    }
    return RSI_OK;
}
