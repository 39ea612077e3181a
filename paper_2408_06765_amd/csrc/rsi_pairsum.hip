// rsi_pairsum.hip -- the RSI pair sum (eqs. 3 and 7 under the estimator of eq. 16).
//
//   phi(P_i) = -(1/2pi) sum_j w_j s_j K(P_i, Q_j)
//   monopole K = e^{ikr}/r,  dipole K = cos(theta)(ik - 1/r) e^{ikr}/r.
//
// Layout and precision (FP32 path)
//   * Sources are prepared once per set into 32-byte records: the offset e_j of the
//     source from the set's anchor C (bounding-box centre) in FP32, |e_j|^2, the folded
//     strength -(1/2pi) w_j s_j, and n.e_j for the dipole.  All lanes of a wave walk
//     the same source at the same time, so the records are read with wave-uniform
//     (scalar) loads into SGPRs and broadcast to every lane for free: no LDS traffic
//     and no VGPRs spent on source data.
//   * Field points are coalesced, TPL per lane.  For each target the kernel computes,
//     once and in FP64, D = P - C, r_ref = |D| and the reference phase
//     frac(r_ref f / c) in revolutions.  Per pair it then needs only FP32:
//         q  = |e|^2 - 2 D.e              ( = r^2 - r_ref^2 )
//         r  = sqrt(r_ref^2 + q)          (via rsqrt, amplitude only)
//         dr = q / (r + r_ref)            ( = r - r_ref, free of cancellation )
//         phase = frac(p_ref + dr f / c)  (revolutions, fed to v_sin/v_cos directly)
//     so the large part of k r never passes through FP32.
//   * Sums run in FP32: per 64-source block, then folded into a Kahan-compensated
//     running sum.  Source ranges may be split across workgroups (split-K); partial
//     sums are reduced in a fixed order, so results are bitwise repeatable.
//
// FP64 path: absolute coordinates, r from sqrt, phase reduced to revolutions and
// evaluated with sincospi, pairs closer than 1e-12 m skipped -- the same operations
// as the definition, in FP64.
#include <cfloat>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <string>

#include "rsi_device.h"

namespace rsi {

// ---------------------------------------------------------------------------
// Anchor: bounding-box centre of the source set, from per-block partial extents.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) bbox_kernel(const double *__restrict__ x,
                                                   const double *__restrict__ y,
                                                   const double *__restrict__ z, int64_t n,
                                                   double *__restrict__ partials) {
    double v[6] = {DBL_MAX, DBL_MAX, DBL_MAX, -DBL_MAX, -DBL_MAX, -DBL_MAX};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const double a = x[i], b = y[i], c = z[i];
        v[0] = fmin(v[0], a); v[1] = fmin(v[1], b); v[2] = fmin(v[2], c);
        v[3] = fmax(v[3], a); v[4] = fmax(v[4], b); v[5] = fmax(v[5], c);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) v[k] = fmin(v[k], __shfl_xor(v[k], off));
#pragma unroll
        for (int k = 3; k < 6; ++k) v[k] = fmax(v[k], __shfl_xor(v[k], off));
    }
    __shared__ double sh[4][6];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int k = 0; k < 6; ++k) sh[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        double r = sh[0][k];
        for (int w = 1; w < 4; ++w) r = (k < 3) ? fmin(r, sh[w][k]) : fmax(r, sh[w][k]);
        partials[blockIdx.x * 6 + k] = r;
    }
}

// Anchor C = centre of the bounding box, and its half diagonal, which bounds |Q_j - C|.
__device__ inline void anchor_from_partials(const double *__restrict__ partials, double &ax,
                                            double &ay, double &az, double &radius) {
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

rsi_status bbox_partials(const rsi_points &pts, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(bbox_kernel, dim3(kBBoxBlocks), dim3(256), 0, s, pts.x, pts.y, pts.z,
                       pts.n, partials);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

// ---------------------------------------------------------------------------
// Source preparation.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) prep_f32_kernel(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ w, const double *__restrict__ vel,
    double v0, double nx, double ny, double nz, double lam, double fre, double fim,
    const double *__restrict__ partials, double *__restrict__ anchor_out, SrcRecF *__restrict__ rec) {
    double ax, ay, az, radius;
    anchor_from_partials(partials, ax, ay, az, radius);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        anchor_out[0] = ax;
        anchor_out[1] = ay;
        anchor_out[2] = az;
        anchor_out[3] = radius;
    }
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const float ex = (float)(x[j] - ax), ey = (float)(y[j] - ay), ez = (float)(z[j] - az);
    const double dex = ex, dey = ey, dez = ez;  // the rounded offset is the source position
    double sre = v0, sim = 0.0;
    if (vel) {
        sre = vel[2 * j];
        sim = vel[2 * j + 1];
    }
    const double scale = -w[j] / kTwoPi;
    SrcRecF r;
    r.ex = ex;
    r.ey = ey;
    r.ez = ez;
    r.es2 = (float)(dex * dex + dey * dey + dez * dez);
    polar_strength(scale * (sre * fre - sim * fim), scale * (sre * fim + sim * fre), lam, r.a, r.psil);
    r.h = (float)(nx * dex + ny * dey + nz * dez);
    r.pad = 0.0f;
    rec[j] = r;
}

// s_j = T_j phi_j (interface strength, eq. 7; R_j phi_j for a reflection) times the
// stage factor F (1; ik for omnidirectional sources; -1 for a dipole radiating along
// -z), folded with -(1/2pi) w_j.
template <typename FieldT>
__global__ void __launch_bounds__(256) strength_f32_kernel(int64_t n, const double *__restrict__ w,
                                                           const FieldT *__restrict__ field,
                                                           const double *__restrict__ tco,
                                                           double lam, double Fre, double Fim,
                                                           SrcRecF *__restrict__ rec) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const double fre = field[2 * j], fim = field[2 * j + 1];
    double sre = fre, sim = fim;
    if (tco) {
        const double tre = tco[2 * j], tim = tco[2 * j + 1];
        sre = tre * fre - tim * fim;
        sim = tre * fim + tim * fre;
    }
    const double scale = -w[j] / kTwoPi;
    float a, psil;
    polar_strength(scale * (sre * Fre - sim * Fim), scale * (sre * Fim + sim * Fre), lam, a, psil);
    rec[j].a = a;
    rec[j].psil = psil;
}

__global__ void __launch_bounds__(256) prep_f64_kernel(int64_t n, const double *__restrict__ x,
                                                       const double *__restrict__ y,
                                                       const double *__restrict__ z,
                                                       const double *__restrict__ w,
                                                       const double *__restrict__ vel, double v0,
                                                       double Fre, double Fim,
                                                       SrcRecD *__restrict__ rec) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    double sre = v0, sim = 0.0;
    if (vel) {
        sre = vel[2 * j];
        sim = vel[2 * j + 1];
    }
    const double scale = -w[j] / kTwoPi;
    SrcRecD r;
    r.x = x[j];
    r.y = y[j];
    r.z = z[j];
    r.pad0 = 0.0;
    r.sre = scale * (sre * Fre - sim * Fim);
    r.sim = scale * (sre * Fim + sim * Fre);
    r.pad1 = r.pad2 = 0.0;
    rec[j] = r;
}

__global__ void __launch_bounds__(256) strength_f64_kernel(int64_t n, const double *__restrict__ w,
                                                           const double *__restrict__ field,
                                                           const double *__restrict__ tco,
                                                           double Fre, double Fim,
                                                           SrcRecD *__restrict__ rec) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const double fre = field[2 * j], fim = field[2 * j + 1];
    double sre = fre, sim = fim;
    if (tco) {
        const double tre = tco[2 * j], tim = tco[2 * j + 1];
        sre = tre * fre - tim * fim;
        sim = tre * fim + tim * fre;
    }
    const double scale = -w[j] / kTwoPi;
    rec[j].sre = scale * (sre * Fre - sim * Fim);
    rec[j].sim = scale * (sre * Fim + sim * Fre);
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

static void unit_normal(const double *normal, double &nx, double &ny, double &nz) {
    nx = ny = nz = 0.0;
    if (!normal) return;
    const double l = sqrt(normal[0] * normal[0] + normal[1] * normal[1] + normal[2] * normal[2]);
    if (l > 0.0) {
        nx = normal[0] / l;
        ny = normal[1] / l;
        nz = normal[2] / l;
    }
}

rsi_status prep_sources_f32(const rsi_points &pts, const double *w, const double *vel,
                            double v0, const double *normal, const double *partials,
                            double lam, Cplx F, SrcSetF &set, hipStream_t s) {
    double nx, ny, nz;
    unit_normal(normal, nx, ny, nz);
    set.n = pts.n;
    if (pts.n == 0) return RSI_OK;
    hipLaunchKernelGGL(prep_f32_kernel, dim3(blocks_for(pts.n)), dim3(256), 0, s, pts.n, pts.x,
                       pts.y, pts.z, w, vel, v0, nx, ny, nz, lam, F.re, F.im, partials, set.anchor, set.rec);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

rsi_status set_strength_f32(SrcSetF &set, const double *w, const void *field, bool field_fp64,
                            const double *tco, double lam, Cplx F, hipStream_t s) {
    if (set.n == 0) return RSI_OK;
    if (field_fp64)
        hipLaunchKernelGGL(strength_f32_kernel<double>, dim3(blocks_for(set.n)), dim3(256), 0, s,
                           set.n, w, static_cast<const double *>(field), tco, lam, F.re, F.im, set.rec);
    else
        hipLaunchKernelGGL(strength_f32_kernel<float>, dim3(blocks_for(set.n)), dim3(256), 0, s,
                           set.n, w, static_cast<const float *>(field), tco, lam, F.re, F.im, set.rec);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

rsi_status prep_sources_f64(const rsi_points &pts, const double *w, const double *vel,
                            double v0, Cplx F, SrcSetD &set, hipStream_t s) {
    set.n = pts.n;
    if (pts.n == 0) return RSI_OK;
    hipLaunchKernelGGL(prep_f64_kernel, dim3(blocks_for(pts.n)), dim3(256), 0, s, pts.n, pts.x,
                       pts.y, pts.z, w, vel, v0, F.re, F.im, set.rec);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

rsi_status set_strength_f64(SrcSetD &set, const double *w, const double *field,
                            const double *tco, Cplx F, hipStream_t s) {
    if (set.n == 0) return RSI_OK;
    hipLaunchKernelGGL(strength_f64_kernel, dim3(blocks_for(set.n)), dim3(256), 0, s, set.n, w,
                       field, tco, F.re, F.im, set.rec);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

// ---------------------------------------------------------------------------
// FP32 pair-sum kernel: grid (target tiles of kBlock*TPL, source splits).
// ---------------------------------------------------------------------------
template <int KIND, int TPL, bool PLANAR>
__global__ void __launch_bounds__(kBlock) pairsum_f32_kernel(
    const SrcRecF *__restrict__ rec, int64_t n_src, int64_t chunk,
    const double *__restrict__ tx, const double *__restrict__ ty, const double *__restrict__ tz,
    int64_t n_tgt, const double *__restrict__ anchor, double inv_lam, float k, double nx,
    double ny, double nz, float2 *__restrict__ out) {
    TargetsF<KIND, TPL> T;
    const int64_t tbase = (int64_t)blockIdx.x * (kBlock * TPL) + threadIdx.x;
    setup_targets_f32<KIND, TPL>(T, tx, ty, tz, n_tgt, tbase, anchor[0], anchor[1], anchor[2],
                                 inv_lam, nx, ny, nz);
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = (j0 + chunk < n_src) ? j0 + chunk : n_src;
    float mre[TPL], mim[TPL];
    if (phase_in_sin_range(anchor[3], inv_lam))
        sum_range_f32<KIND, TPL, PLANAR, false>(T, rec, j0, j1, (float)inv_lam, k, mre, mim);
    else
        sum_range_f32<KIND, TPL, PLANAR, true>(T, rec, j0, j1, (float)inv_lam, k, mre, mim);
    float2 *o = out + (int64_t)blockIdx.y * n_tgt;
#pragma unroll
    for (int u = 0; u < TPL; ++u) {
        const int64_t i = tbase + (int64_t)u * kBlock;
        if (i < n_tgt) o[i] = make_float2(mre[u], mim[u]);
    }
}

// ---------------------------------------------------------------------------
// FP32 pair-sum kernel for few field points: grid (field points, source splits) of one
// wave each; the wave's lanes share the field point and split its sources.
// ---------------------------------------------------------------------------
template <int KIND, bool PLANAR>
__global__ void __launch_bounds__(64) pairsum_f32_few_kernel(
    const SrcRecF *__restrict__ rec, int64_t n_src, int64_t chunk,
    const double *__restrict__ tx, const double *__restrict__ ty, const double *__restrict__ tz,
    int64_t n_tgt, const double *__restrict__ anchor, double inv_lam, float k, double nx,
    double ny, double nz, float2 *__restrict__ out) {
    TargetsF<KIND, 1> T;
    const int64_t i = blockIdx.x;
    setup_targets_f32<KIND, 1>(T, tx, ty, tz, n_tgt, i, anchor[0], anchor[1], anchor[2], inv_lam,
                               nx, ny, nz);
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = (j0 + chunk < n_src) ? j0 + chunk : n_src;
    float mre, mim;
    if (phase_in_sin_range(anchor[3], inv_lam))
        sum_lanes_f32<KIND, PLANAR, false>(T, rec, j0, j1, (float)inv_lam, k, mre, mim);
    else
        sum_lanes_f32<KIND, PLANAR, true>(T, rec, j0, j1, (float)inv_lam, k, mre, mim);
    if (threadIdx.x == 0) out[(int64_t)blockIdx.y * n_tgt + i] = make_float2(mre, mim);
}

// ---------------------------------------------------------------------------
// FP64 pair-sum kernel (one target per lane).
// ---------------------------------------------------------------------------
template <int KIND>
__global__ void __launch_bounds__(kBlock) pairsum_f64_kernel(
    const SrcRecD *__restrict__ rec, int64_t n_src, int64_t chunk,
    const double *__restrict__ tx, const double *__restrict__ ty, const double *__restrict__ tz,
    int64_t n_tgt, double inv_lam, double k, double nx, double ny, double nz,
    double2 *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < n_tgt;
    if (!valid) i = n_tgt - 1;
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = (j0 + chunk < n_src) ? j0 + chunk : n_src;
    double mre, mim;
    sum_range_f64<KIND>(tx[i], ty[i], tz[i], rec, j0, j1, inv_lam, k, nx, ny, nz, mre, mim);
    if (valid) out[(int64_t)blockIdx.y * n_tgt + i] = make_double2(mre, mim);
}

// ---------------------------------------------------------------------------
// Split-K reduction (fixed order) and zero fill.
// ---------------------------------------------------------------------------
template <typename T2>
__global__ void __launch_bounds__(256) reduce_splits_kernel(const T2 *__restrict__ partial,
                                                            int n_split, int64_t n,
                                                            T2 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < n_split; ++s) {
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
__global__ void __launch_bounds__(256) zero_kernel(int64_t n, T2 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        T2 z;
        z.x = 0;
        z.y = 0;
        out[i] = z;
    }
}

// Optional overrides of the default launch shape, for tuning sweeps:
// RSI_PAIRSUM_TPL (1, 2 or 4 targets per lane) and RSI_PAIRSUM_MIN_WG (workgroup goal).
int env_int(const char *name, int dflt) {
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    char *end = nullptr;
    const long x = std::strtol(v, &end, 10);
    return (end && *end == 0 && x > 0 && x < (1L << 30)) ? (int)x : dflt;
}

PairShape default_shape(int64_t n_src, int64_t n_tgt, int64_t few_below, int64_t min_chunk) {
    static const int tpl_env = env_int("RSI_PAIRSUM_TPL", 1);
    static const int min_wg = env_int("RSI_PAIRSUM_MIN_WG", 32768);
    PairShape sh;
    sh.tpl = (tpl_env == 2 || tpl_env == 4) ? tpl_env : 1;
    const int64_t bx = (n_tgt + kBlock * sh.tpl - 1) / (kBlock * sh.tpl);
    // aim for >= min_wg workgroups (128 per CU: small items balance the CUs at the end
    // of the launch) while keeping >= min_chunk sources per split
    if (min_chunk < kSub) min_chunk = kSub;
    int64_t splits = (min_wg + bx - 1) / (bx > 0 ? bx : 1);
    const int64_t max_splits = (n_src + min_chunk - 1) / min_chunk;
    if (splits > max_splits) splits = max_splits;
    if (splits < 1) splits = 1;
    int64_t chunk = (n_src + splits - 1) / splits;
    chunk = (chunk + kSub - 1) / kSub * kSub;
    sh.chunk = chunk > 0 ? chunk : kSub;
    // too few field points to fill the CUs one point per lane: one wave per (point, split)
    // instead, about 64 waves per CU with >= 4 sources per lane (RSI_PAIRSUM_FEW = 0 or 1
    // forces either launch, for tuning and tests)
    bool few = 4 * bx * splits < few_below;
    if (const char *e = std::getenv("RSI_PAIRSUM_FEW"))
        if ((e[0] == '0' || e[0] == '1') && e[1] == 0) few = e[0] == '1';
    if (few_below <= 0) few = false;
    if (few && n_tgt > 0) {
        int64_t fs = (kFewWaves + n_tgt - 1) / n_tgt;
        const int64_t fmax = (n_src + 255) / 256;
        if (fs > fmax) fs = fmax;
        if (fs < 1) fs = 1;
        if (fs > 65535) fs = 65535;
        int64_t fc = (n_src + fs - 1) / fs;
        fc = (fc + kSub - 1) / kSub * kSub;
        sh.chunk = fc > 0 ? fc : kSub;
        sh.tpl = 1;
        sh.few = true;
    }
    return sh;
}

static int64_t n_splits(const PairShape &sh, int64_t n_src) {
    if (n_src <= 0) return 1;
    const int64_t chunk = sh.chunk > 0 ? sh.chunk : n_src;
    return (n_src + chunk - 1) / chunk;
}

int64_t partial_slots(const PairShape &sh, int64_t n_src, int64_t n_tgt) {
    const int64_t ns = n_splits(sh, n_src);
    return ns > 1 ? ns * n_tgt : 0;
}

template <int KIND>
static void launch_f32_few(dim3 grid, hipStream_t s, const SrcSetF &set, int64_t chunk,
                           const Targets &t, double inv_lam, float k, double nx, double ny,
                           double nz, bool planar, float2 *dst) {
    if (planar)
        hipLaunchKernelGGL((pairsum_f32_few_kernel<KIND, true>), grid, dim3(64), 0, s, set.rec, set.n,
                           chunk, t.x, t.y, t.z, t.n, set.anchor, inv_lam, k, nx, ny, nz, dst);
    else
        hipLaunchKernelGGL((pairsum_f32_few_kernel<KIND, false>), grid, dim3(64), 0, s, set.rec, set.n,
                           chunk, t.x, t.y, t.z, t.n, set.anchor, inv_lam, k, nx, ny, nz, dst);
}

template <int KIND, int TPL>
static void launch_f32(dim3 grid, hipStream_t s, const SrcSetF &set, int64_t chunk,
                       const Targets &t, double inv_lam, float k, double nx, double ny,
                       double nz, bool planar, float2 *dst) {
    if (planar)
        hipLaunchKernelGGL((pairsum_f32_kernel<KIND, TPL, true>), grid, dim3(kBlock), 0, s, set.rec,
                           set.n, chunk, t.x, t.y, t.z, t.n, set.anchor, inv_lam, k, nx, ny, nz, dst);
    else
        hipLaunchKernelGGL((pairsum_f32_kernel<KIND, TPL, false>), grid, dim3(kBlock), 0, s, set.rec,
                           set.n, chunk, t.x, t.y, t.z, t.n, set.anchor, inv_lam, k, nx, ny, nz, dst);
}

rsi_status pairsum_f32(const SrcSetF &set, const Targets &t, rsi_kernel kind,
                       const double *normal, double c, double freq, const PairShape &sh,
                       float2 *partial, float2 *out, hipStream_t s, bool planar_z) {
    if (t.n == 0) return RSI_OK;
    if (set.n == 0) {
        hipLaunchKernelGGL(zero_kernel<float2>, dim3(blocks_for(t.n)), dim3(256), 0, s, t.n, out);
        RSI_HIP(hipGetLastError());
        return RSI_OK;
    }
    double nx, ny, nz;
    unit_normal(normal, nx, ny, nz);
    const int tpl = (sh.tpl == 1 || sh.tpl == 4) ? sh.tpl : 2;
    const int64_t chunk = sh.chunk > 0 ? sh.chunk : set.n;
    const int64_t ns = n_splits(sh, set.n);
    if (ns > 65535) return RSI_ERR_SIZE;
    const int64_t bx = sh.few ? t.n : (t.n + (int64_t)kBlock * tpl - 1) / ((int64_t)kBlock * tpl);
    if (bx > 0x7fffffff) return RSI_ERR_SIZE;
    const dim3 grid((unsigned)bx, (unsigned)ns);
    float2 *dst = ns > 1 ? partial : out;
    if (ns > 1 && !partial) return RSI_ERR_WORKSPACE;
    const double inv_lam = freq / c;
    const float k = (float)(kTwoPi * freq / c);
    if (sh.few) {
        if (kind == RSI_MONOPOLE) launch_f32_few<RSI_MONOPOLE>(grid, s, set, chunk, t, inv_lam, k, nx, ny, nz, planar_z, dst);
        else launch_f32_few<RSI_DIPOLE>(grid, s, set, chunk, t, inv_lam, k, nx, ny, nz, planar_z, dst);
    } else if (kind == RSI_MONOPOLE) {
        if (tpl == 1) launch_f32<RSI_MONOPOLE, 1>(grid, s, set, chunk, t, inv_lam, k, nx, ny, nz, planar_z, dst);
        else if (tpl == 2) launch_f32<RSI_MONOPOLE, 2>(grid, s, set, chunk, t, inv_lam, k, nx, ny, nz, planar_z, dst);
        else launch_f32<RSI_MONOPOLE, 4>(grid, s, set, chunk, t, inv_lam, k, nx, ny, nz, planar_z, dst);
    } else {
        if (tpl == 1) launch_f32<RSI_DIPOLE, 1>(grid, s, set, chunk, t, inv_lam, k, nx, ny, nz, planar_z, dst);
        else if (tpl == 2) launch_f32<RSI_DIPOLE, 2>(grid, s, set, chunk, t, inv_lam, k, nx, ny, nz, planar_z, dst);
        else launch_f32<RSI_DIPOLE, 4>(grid, s, set, chunk, t, inv_lam, k, nx, ny, nz, planar_z, dst);
    }
    RSI_HIP(hipGetLastError());
    if (ns > 1) {
        hipLaunchKernelGGL(reduce_splits_kernel<float2>, dim3(blocks_for(t.n)), dim3(256), 0, s,
                           partial, (int)ns, t.n, out);
        RSI_HIP(hipGetLastError());
    }
    return RSI_OK;
}

rsi_status pairsum_f64(const SrcSetD &set, const Targets &t, rsi_kernel kind,
                       const double *normal, double c, double freq, const PairShape &sh,
                       double2 *partial, double2 *out, hipStream_t s) {
    if (t.n == 0) return RSI_OK;
    if (set.n == 0) {
        hipLaunchKernelGGL(zero_kernel<double2>, dim3(blocks_for(t.n)), dim3(256), 0, s, t.n, out);
        RSI_HIP(hipGetLastError());
        return RSI_OK;
    }
    double nx, ny, nz;
    unit_normal(normal, nx, ny, nz);
    const int64_t chunk = sh.chunk > 0 ? sh.chunk : set.n;
    const int64_t ns = n_splits(sh, set.n);
    if (ns > 65535) return RSI_ERR_SIZE;
    const int64_t bx = (t.n + kBlock - 1) / kBlock;
    if (bx > 0x7fffffff) return RSI_ERR_SIZE;
    const dim3 grid((unsigned)bx, (unsigned)ns);
    double2 *dst = ns > 1 ? partial : out;
    if (ns > 1 && !partial) return RSI_ERR_WORKSPACE;
    const double inv_lam = freq / c, k = kTwoPi * freq / c;
    if (kind == RSI_MONOPOLE)
        hipLaunchKernelGGL(pairsum_f64_kernel<RSI_MONOPOLE>, grid, dim3(kBlock), 0, s, set.rec,
                           set.n, chunk, t.x, t.y, t.z, t.n, inv_lam, k, nx, ny, nz, dst);
    else
        hipLaunchKernelGGL(pairsum_f64_kernel<RSI_DIPOLE>, grid, dim3(kBlock), 0, s, set.rec,
                           set.n, chunk, t.x, t.y, t.z, t.n, inv_lam, k, nx, ny, nz, dst);
    RSI_HIP(hipGetLastError());
    if (ns > 1) {
        hipLaunchKernelGGL(reduce_splits_kernel<double2>, dim3(blocks_for(t.n)), dim3(256), 0, s,
                           partial, (int)ns, t.n, out);
        RSI_HIP(hipGetLastError());
    }
    return RSI_OK;
}

}  // namespace rsi

using namespace rsi;

rsi_status rsi::validate_propagate(const rsi_points *src, const double *src_w,
                                   const double *src_vel, const double *normal,
                                   const rsi_points *tgt, rsi_medium medium, double freq,
                                   rsi_kernel kind, rsi_precision prec, uint32_t flags, void *out) {
    if ((flags & ~(uint32_t)RSI_FLAG_PLANAR_Z) != 0) return RSI_ERR_ARG;
    const bool planar = (flags & RSI_FLAG_PLANAR_Z) != 0;
    if (!src || !tgt) return RSI_ERR_NULL;
    if (kind != RSI_MONOPOLE && kind != RSI_DIPOLE && kind != RSI_OMNI) return RSI_ERR_ARG;
    if (prec != RSI_FP32 && prec != RSI_FP64) return RSI_ERR_ARG;
    if (!(freq > 0.0) || !(medium.c > 0.0) || !std::isfinite(freq) || !std::isfinite(medium.c))
        return RSI_ERR_ARG;
    if (src->n < 0 || tgt->n < 0) return RSI_ERR_SIZE;
    if (tgt->n == 0) return RSI_OK;
    if (!out || !tgt->x || !tgt->y || !tgt->z) return RSI_ERR_NULL;
    if (src->n > 0 && (!src->x || !src->y || !src->z || !src_w || !src_vel)) return RSI_ERR_NULL;
    if (kind == RSI_DIPOLE) {
        if (!normal) return RSI_ERR_NULL;
        const double l2 = normal[0] * normal[0] + normal[1] * normal[1] + normal[2] * normal[2];
        if (!(l2 > 0.0) || !std::isfinite(l2)) return RSI_ERR_ARG;
        if (planar && (normal[0] != 0.0 || normal[1] != 0.0)) return RSI_ERR_ARG;
    }
    return RSI_OK;
}

namespace {

// Workspace of a one-shot pair sum drawn from the stream-ordered allocator.
struct PoolWorkspace {
    Scratch scratch;
    explicit PoolWorkspace(hipStream_t s) : scratch(s) {}
    template <class T>
    rsi_status alloc(T **p, size_t count) { return scratch.alloc(p, count); }
    size_t left() const { return SIZE_MAX; }
};

// Workspace carved out of a fixed device array: 256-byte aligned pieces, no allocation.
struct ArenaWorkspace {
    char *base;
    size_t cap, used = 0;
    static size_t piece(size_t bytes) { return (bytes + 255) / 256 * 256; }
    template <class T>
    rsi_status alloc(T **p, size_t count) {
        const size_t bytes = piece(sizeof(T) * (count > 0 ? count : 1));
        if (bytes > cap - used) {
            *p = nullptr;
            set_last_error_text("rsi_propagate_noalloc: the call needs more than the " +
                                std::to_string((long long)cap) + "-byte scratch array");
            return RSI_ERR_SIZE;
        }
        *p = reinterpret_cast<T *>(base + used);
        used += bytes;
        return RSI_OK;
    }
    size_t left() const { return cap - used; }
};

// Lower the split count of `sh` until its partials ([splits][n_tgt] of elem bytes) fit
// in `bytes`; one split needs no partials.  Sources per split stay a multiple of kSub.
void fit_partials(PairShape &sh, int64_t n_src, int64_t n_tgt, size_t elem, size_t bytes) {
    if (partial_slots(sh, n_src, n_tgt) * (int64_t)elem <= (int64_t)bytes) return;
    const int64_t most = (int64_t)(bytes / 256 * 256 / elem) / (n_tgt > 0 ? n_tgt : 1);
    int64_t chunk = n_src;
    if (most >= 2) chunk = ((n_src + most - 1) / most + kSub - 1) / kSub * kSub;
    while (chunk < n_src && partial_slots(PairShape{sh.tpl, chunk, sh.few}, n_src, n_tgt) * (int64_t)elem >
                                (int64_t)(bytes / 256 * 256))
        chunk += kSub;
    sh.chunk = chunk < n_src ? chunk : (n_src > 0 ? n_src : kSub);
}

// The pair sum of rsi_propagate_ex after validation, its workspace taken from `ws`
// (records, anchor and extents first, then the split partials, whose split count is
// lowered to what is left when `fit` is set).
template <class Workspace>
rsi_status propagate_impl(const rsi_points *src, const double *src_w, const double *src_vel,
                          const double *normal, const rsi_points *tgt, rsi_medium medium,
                          double freq, rsi_kernel kind, rsi_precision prec, uint32_t flags,
                          void *out, hipStream_t s, Workspace &ws, bool fit) {
    const bool planar = (flags & RSI_FLAG_PLANAR_Z) != 0;
    {
        std::vector<DevSpan> in;
        add_points(in, *src);
        in.push_back({src_w, src->n});
        in.push_back({src_vel, 2 * src->n});
        add_points(in, *tgt);
        int *flag = nullptr;
        if (fit) RSI_TRY(ws.alloc(&flag, 1));
        RSI_TRY(check_finite(s, in, flag));
    }
    const Targets t{tgt->x, tgt->y, tgt->z, tgt->n};
    // RSI_OMNI = the monopole sum of strengths times ik
    const Cplx F = kind == RSI_OMNI ? Cplx{0.0, kTwoPi * freq / medium.c} : Cplx{1.0, 0.0};
    const rsi_kernel kk = kind == RSI_OMNI ? RSI_MONOPOLE : kind;
    PairShape sh = default_shape(src->n, tgt->n, prec == RSI_FP32 ? kFewWaves / 8 : 0);
    if (prec == RSI_FP32) {
        SrcSetF set;
        double *partials = nullptr;
        float2 *partial = nullptr;
        if (src->n > 0) {
            RSI_TRY(ws.alloc(&set.rec, (size_t)src->n));
            RSI_TRY(ws.alloc(&set.anchor, 4));
            RSI_TRY(ws.alloc(&partials, kBBoxBlocks * 6));
        }
        if (fit) fit_partials(sh, src->n, tgt->n, sizeof(float2), ws.left());
        const int64_t nslots = partial_slots(sh, src->n, tgt->n);
        if (nslots > 0) RSI_TRY(ws.alloc(&partial, (size_t)nslots));
        if (src->n > 0) {
            RSI_TRY(bbox_partials(*src, partials, s));
            RSI_TRY(prep_sources_f32(*src, src_w, src_vel, 0.0, normal, partials, medium.c / freq, F,
                                     set, s));
        }
        return pairsum_f32(set, t, kk, normal, medium.c, freq, sh, partial,
                           static_cast<float2 *>(out), s, planar);
    }
    SrcSetD set;
    double2 *partial = nullptr;
    if (src->n > 0) RSI_TRY(ws.alloc(&set.rec, (size_t)src->n));
    if (fit) fit_partials(sh, src->n, tgt->n, sizeof(double2), ws.left());
    const int64_t nslots = partial_slots(sh, src->n, tgt->n);
    if (nslots > 0) RSI_TRY(ws.alloc(&partial, (size_t)nslots));
    if (src->n > 0) RSI_TRY(prep_sources_f64(*src, src_w, src_vel, 0.0, F, set, s));
    return pairsum_f64(set, t, kk, normal, medium.c, freq, sh, partial,
                       static_cast<double2 *>(out), s);
}

}  // namespace

extern "C" rsi_status rsi_propagate_ex(const rsi_points *src, const double *src_w,
                                       const double *src_vel, const double *normal,
                                       const rsi_points *tgt, rsi_medium medium, double freq,
                                       rsi_kernel kind, rsi_precision prec, uint32_t flags,
                                       void *out, void *stream) {
    RSI_TRY(validate_propagate(src, src_w, src_vel, normal, tgt, medium, freq, kind, prec, flags, out));
    if (tgt->n == 0) return RSI_OK;
    hipStream_t s = as_stream(stream);
    PoolWorkspace ws(s);
    return propagate_impl(src, src_w, src_vel, normal, tgt, medium, freq, kind, prec, flags, out, s,
                          ws, false);
}

// The fixed workspace of rsi_propagate_noalloc: one copy per device, reserved when the
// library's code object is loaded there.  Host code never uses its name as an address:
// the per-device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[RSI_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<char *> g_scratch_addr;  // indexed by device

// Device address of `scratch` on the current device, looked up once per device with that
// device current.
rsi_status scratch_address(char **addr) {
    int dev = 0;
    RSI_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_addr.size() <= dev) g_scratch_addr.resize(dev + 1, nullptr);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        RSI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_last_error_text("hipGetSymbolAddress(scratch) returned NULL");
            return RSI_ERR_DEVICE;
        }
        g_scratch_addr[dev] = static_cast<char *>(p);
    }
    *addr = g_scratch_addr[dev];
    return RSI_OK;
}
}  // namespace

extern "C" rsi_status rsi_propagate_noalloc(const rsi_points *src, const double *src_w,
                                            const double *src_vel, const double *normal,
                                            const rsi_points *tgt, rsi_medium medium, double freq,
                                            rsi_kernel kind, rsi_precision prec, uint32_t flags,
                                            void *out, void *stream) {
    RSI_TRY(validate_propagate(src, src_w, src_vel, normal, tgt, medium, freq, kind, prec, flags, out));
    if (tgt->n == 0) return RSI_OK;
    // the records alone must fit (the flag, anchor and extents take 4 KiB)
    const int64_t rec_bytes = prec == RSI_FP32 ? (int64_t)sizeof(SrcRecF) : (int64_t)sizeof(SrcRecD);
    const int64_t fixed = prec == RSI_FP32 ? 256 + 256 + (int64_t)ArenaWorkspace::piece(kBBoxBlocks * 6 * 8)
                                           : 256;
    if (src->n > (RSI_NOALLOC_SCRATCH_BYTES - fixed) / rec_bytes) {
        set_last_error_text("rsi_propagate_noalloc: " + std::to_string((long long)src->n) +
                            " sources need " + std::to_string((long long)(src->n * rec_bytes + fixed)) +
                            " bytes of scratch; the array holds " +
                            std::to_string((long long)RSI_NOALLOC_SCRATCH_BYTES));
        return RSI_ERR_SIZE;
    }
    hipStream_t s = as_stream(stream);
    char *base = nullptr;
    RSI_TRY(scratch_address(&base));
    ArenaWorkspace ws{base, (size_t)RSI_NOALLOC_SCRATCH_BYTES};
    return propagate_impl(src, src_w, src_vel, normal, tgt, medium, freq, kind, prec, flags, out, s,
                          ws, true);
}

extern "C" rsi_status rsi_propagate(const rsi_points *src, const double *src_w,
                                    const double *src_vel, const double *normal,
                                    const rsi_points *tgt, rsi_medium medium, double freq,
                                    rsi_kernel kind, rsi_precision prec, void *out,
                                    void *stream) {
    return rsi_propagate_ex(src, src_w, src_vel, normal, tgt, medium, freq, kind, prec, 0u, out,
                            stream);
}
