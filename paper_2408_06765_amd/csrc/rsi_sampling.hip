// rsi_sampling.hip -- sample points on the radiating surfaces (Sec. 2.3, eqs. 16-18)
// and the small ABI utilities (status strings, last error, version, the input check).
//
// The paper draws its QMC points from a Halton sequence; this library uses a
// two-dimensional Sobol sequence with a hash-based nested uniform (Owen) scramble,
// which keeps the (0, m, 2)-net property of every power-of-two prefix.  Each point is
// computed from its index alone, so any range of points is one independent launch.
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "rsi_internal.h"

namespace rsi {

static thread_local std::string g_last_error;
static int g_check_finite = [] {
    const char *e = std::getenv("RSI_CHECK_FINITE");
    return (e && e[0] == '1' && e[1] == 0) ? 1 : 0;
}();

// Sets *flag when a value of a[0, n) is not finite (lanes that see one store 1).
__global__ void __launch_bounds__(256) nonfinite_kernel(const double *__restrict__ a, int64_t n,
                                                         int *__restrict__ flag) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        bad = bad || !isfinite(a[i]);
    if (bad) flag[0] = 1;
}

__global__ void __launch_bounds__(64) clear_flag_kernel(int *__restrict__ flag) {
    if (threadIdx.x == 0) flag[0] = 0;
}

rsi_status check_finite(hipStream_t s, const std::vector<DevSpan> &arrays, int *flag) {
    if (!__atomic_load_n(&g_check_finite, __ATOMIC_RELAXED)) return RSI_OK;
    Scratch scratch(s);
    if (!flag) RSI_TRY(scratch.alloc(&flag, 1));
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(64), 0, s, flag);
    RSI_HIP(hipGetLastError());
    for (const DevSpan &a : arrays) {
        if (!a.p || a.n <= 0) continue;
        const int64_t blocks = (a.n + 255) / 256;
        hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, s,
                           a.p, a.n, flag);
        RSI_HIP(hipGetLastError());
    }
    int host = 0;
    RSI_HIP(hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    RSI_HIP(hipStreamSynchronize(s));
    return host ? RSI_ERR_NONFINITE : RSI_OK;
}

void set_last_error(const char *what, hipError_t e) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
}

void set_last_error_text(const std::string &text) { g_last_error = text; }

// Coordinate seeds: MurmurHash3 32-bit finaliser of seed + golden-ratio step.
__host__ __device__ inline uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

__host__ __device__ inline uint32_t coord_seed(uint32_t seed, uint32_t d) {
    return fmix32(seed + 0x9e3779b9u * (d + 1u));
}

// Burley (JCGT 2020) hash-based Laine-Karras permutation on the bit-reversed value:
// a nested uniform scramble of the binary digits (higher digits permute lower ones).
__device__ inline uint32_t nested_uniform_scramble(uint32_t x, uint32_t seed) {
    x = __builtin_bitreverse32(x);
    x += seed;
    x ^= x * 0x6c50b47cu;
    x ^= x * 0xb82f1e52u;
    x ^= x * 0xc7afe638u;
    x ^= x * 0x8d22f6e6u;
    return __builtin_bitreverse32(x);
}

// Unscrambled Sobol coordinates of point `idx` (< 2^32).  Coordinate 0 has direction
// numbers 2^(31-b): the bit reversal of the index.  Coordinate 1 (polynomial x + 1)
// has v_0 = 2^31, v_b = v_{b-1} ^ (v_{b-1} >> 1).
__device__ inline void sobol_pair(uint32_t idx, uint32_t &x0, uint32_t &x1) {
    x0 = __builtin_bitreverse32(idx);
    uint32_t v = 0x80000000u, acc = 0u;
    while (idx) {
        if (idx & 1u) acc ^= v;
        v ^= v >> 1;
        idx >>= 1;
    }
    x1 = acc;
}

__device__ inline void scrambled_pair(uint32_t idx, uint32_t s0, uint32_t s1, uint32_t &u0,
                                      uint32_t &u1) {
    uint32_t x0, x1;
    sobol_pair(idx, x0, x1);
    u0 = nested_uniform_scramble(x0, s0);
    u1 = nested_uniform_scramble(x1, s1);
}

__global__ void __launch_bounds__(256) sobol2d_kernel(uint32_t s0, uint32_t s1, int64_t first,
                                                      int64_t n, uint32_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t u0, u1;
    scrambled_pair((uint32_t)(first + i), s0, s1, u0, u1);
    reinterpret_cast<uint2 *>(out)[i] = make_uint2(u0, u1);
}

// 2^-32: maps a 32-bit digit string onto [0, 1) exactly in FP64.
constexpr double kU32 = 1.0 / 4294967296.0;

// Halton sequence (the paper's choice, Sec. 2.3): the radical inverse of the index in
// base b, as the integer of mirrored digits over b^K followed by one IEEE division
// (the correctly rounded value; exact integers below 2^53 for indices below 2^40).
__device__ inline double radical_inverse(uint64_t index, uint64_t base) {
    uint64_t num = 0, den = 1;
    while (index) {
        const uint64_t q = index / base;
        num = num * base + (index - q * base);
        den *= base;
        index = q;
    }
    return (double)num / (double)den;
}

// Where the two unit coordinates of sample i come from: scrambled Sobol points with
// the coordinate seeds s0, s1 (seq 0), or Halton points of index first + i (seq 1).
struct UnitSource {
    int seq;
    uint32_t s0, s1;
    int64_t first;
};

__device__ inline void unit_pair(const UnitSource &u, int64_t i, double &u0, double &u1) {
    if (u.seq == RSI_SEQ_HALTON) {
        u0 = radical_inverse((uint64_t)(u.first + i), 2);
        u1 = radical_inverse((uint64_t)(u.first + i), 3);
    } else {
        uint32_t a, b;
        scrambled_pair((uint32_t)i, u.s0, u.s1, a, b);
        u0 = (double)a * kU32;
        u1 = (double)b * kU32;
    }
}

__global__ void __launch_bounds__(256) halton2d_kernel(int64_t first, int64_t n, double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    reinterpret_cast<double2 *>(out)[i] =
        make_double2(radical_inverse((uint64_t)(first + i), 2), radical_inverse((uint64_t)(first + i), 3));
}

__global__ void __launch_bounds__(256) disc_kernel(UnitSource us, int64_t n, double radius,
                                                   double cx, double cy, double cz, double ct,
                                                   double st, double wj, double *x, double *y,
                                                   double *z, double *w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double u0, u1;
    unit_pair(us, i, u0, u1);
    // eq. (18): area-uniform radius and uniform angle
    const double r = radius * sqrt(u0);
    double sn, cs;
    sincospi(2.0 * u1, &sn, &cs);
    const double xi = r * cs, eta = r * sn;
    x[i] = cx + xi * ct;  // rotation by `tilt` about +y, then translation
    y[i] = cy + eta;
    z[i] = cz - xi * st;
    w[i] = wj;
}

__global__ void __launch_bounds__(256) square_kernel(UnitSource us, int64_t n, double cx,
                                                     double cy, double z0, double h, double wj,
                                                     double *x, double *y, double *z, double *w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double u0, u1;
    unit_pair(us, i, u0, u1);
    // eq. (17): uniform on the square [cx - h, cx + h] x [cy - h, cy + h]
    x[i] = cx + h * (2.0 * u0 - 1.0);
    y[i] = cy + h * (2.0 * u1 - 1.0);
    z[i] = z0;
    w[i] = wj;
}

// Spherical cap (focused transducer, Sec. 3.3): height above the apex uniform in u0
// (area-uniform), azimuth 2 pi u1; in the cap frame (R sin a cos p, R sin a sin p,
// R (1 - cos a)), then tilted about +y and translated like the flat disc.
__global__ void __launch_bounds__(256) cap_kernel(UnitSource us, int64_t n, double R, double ca,
                                                  double cx, double cy, double cz, double ct,
                                                  double st, double wj, double *x, double *y,
                                                  double *z, double *w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double u0, u1;
    unit_pair(us, i, u0, u1);
    // t = 1 - cos(a); sin(a) = sqrt(t (2 - t)) has no cancellation near the apex
    const double t = u0 * (1.0 - ca);
    const double sal = sqrt(t * (2.0 - t));
    double sn, cs;
    sincospi(2.0 * u1, &sn, &cs);
    const double xi = R * sal * cs, eta = R * sal * sn, zeta = R * t;
    x[i] = cx + xi * ct + zeta * st;
    y[i] = cy + eta;
    z[i] = cz - xi * st + zeta * ct;
    w[i] = wj;
}

// Gaussian apodisation (Sec. 4): w *= exp(-rho^2 / width^2), rho the distance from the
// axis line through the centre.
__global__ void __launch_bounds__(256) apodise_kernel(int64_t n, const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      const double *__restrict__ z, double cx,
                                                      double cy, double cz, double ax, double ay,
                                                      double az, double inv_w2, double *w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double dx = x[i] - cx, dy = y[i] - cy, dz = z[i] - cz;
    const double along = dx * ax + dy * ay + dz * az;
    const double rho2 = dx * dx + dy * dy + dz * dz - along * along;
    w[i] *= exp(-rho2 * inv_w2);
}

static unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace rsi

using namespace rsi;

extern "C" {

const char *rsi_status_string(rsi_status s) {
    switch (s) {
        case RSI_OK: return "RSI_OK";
        case RSI_ERR_NULL: return "RSI_ERR_NULL";
        case RSI_ERR_ARG: return "RSI_ERR_ARG";
        case RSI_ERR_SIZE: return "RSI_ERR_SIZE";
        case RSI_ERR_DEVICE: return "RSI_ERR_DEVICE";
        case RSI_ERR_WORKSPACE: return "RSI_ERR_WORKSPACE";
        case RSI_ERR_NONFINITE: return "RSI_ERR_NONFINITE";
        case RSI_ERR_UNSUPPORTED: return "RSI_ERR_UNSUPPORTED";
        default: break;
    }
    return "RSI_UNKNOWN_STATUS";
}

const char *rsi_last_error(void) { return g_last_error.c_str(); }

int rsi_version(void) { return (1 << 16) | 2; }

int rsi_set_check_finite(int enable) {
    return __atomic_exchange_n(&g_check_finite, enable ? 1 : 0, __ATOMIC_RELAXED);
}

rsi_status rsi_sobol2d(uint32_t seed, int64_t first, int64_t n, uint32_t *out, void *stream) {
    if (first < 0 || n < 0 || first + n > (int64_t(1) << 32)) return RSI_ERR_SIZE;
    if (n == 0) return RSI_OK;
    if (!out) return RSI_ERR_NULL;
    hipLaunchKernelGGL(sobol2d_kernel, dim3(grid_for(n)), dim3(256), 0, as_stream(stream),
                       coord_seed(seed, 0), coord_seed(seed, 1), first, n, out);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

static rsi_status unit_source(rsi_sequence seq, uint32_t seed, int64_t n, UnitSource &us) {
    if (seq != RSI_SEQ_SOBOL && seq != RSI_SEQ_HALTON) return RSI_ERR_ARG;
    if (n < 0 || n > (int64_t(1) << 32)) return RSI_ERR_SIZE;
    us.seq = (int)seq;
    us.s0 = coord_seed(seed, 0);
    us.s1 = coord_seed(seed, 1);
    us.first = (int64_t)seed + 1;  // Halton: start after the origin point
    return RSI_OK;
}

rsi_status rsi_halton2d(int64_t first, int64_t n, double *out, void *stream) {
    if (first < 0 || n < 0 || first + n > (int64_t(1) << 40)) return RSI_ERR_SIZE;
    if (n == 0) return RSI_OK;
    if (!out) return RSI_ERR_NULL;
    hipLaunchKernelGGL(halton2d_kernel, dim3(grid_for(n)), dim3(256), 0, as_stream(stream), first, n, out);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

rsi_status rsi_sample_disc_ex(rsi_sequence seq, uint32_t seed, int64_t n, double radius,
                              const double *centre, double tilt, double *x, double *y, double *z,
                              double *w, void *stream) {
    UnitSource us;
    RSI_TRY(unit_source(seq, seed, n, us));
    if (!(radius > 0.0)) return RSI_ERR_ARG;
    if (n == 0) return RSI_OK;
    if (!centre || !x || !y || !z || !w) return RSI_ERR_NULL;
    const double wj = kPi * radius * radius / (double)n;
    hipLaunchKernelGGL(disc_kernel, dim3(grid_for(n)), dim3(256), 0, as_stream(stream), us, n, radius,
                       centre[0], centre[1], centre[2], cos(tilt), sin(tilt), wj, x, y, z, w);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

rsi_status rsi_sample_disc(uint32_t seed, int64_t n, double radius, const double *centre,
                           double tilt, double *x, double *y, double *z, double *w,
                           void *stream) {
    return rsi_sample_disc_ex(RSI_SEQ_SOBOL, seed, n, radius, centre, tilt, x, y, z, w, stream);
}

rsi_status rsi_sample_square_ex(rsi_sequence seq, uint32_t seed, int64_t n, double cx, double cy,
                                double z0, double half_width, double *x, double *y, double *z,
                                double *w, void *stream) {
    UnitSource us;
    RSI_TRY(unit_source(seq, seed, n, us));
    if (!(half_width > 0.0)) return RSI_ERR_ARG;
    if (n == 0) return RSI_OK;
    if (!x || !y || !z || !w) return RSI_ERR_NULL;
    const double wj = 4.0 * half_width * half_width / (double)n;
    hipLaunchKernelGGL(square_kernel, dim3(grid_for(n)), dim3(256), 0, as_stream(stream), us, n, cx, cy, z0,
                       half_width, wj, x, y, z, w);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

rsi_status rsi_sample_square(uint32_t seed, int64_t n, double cx, double cy, double z0,
                             double half_width, double *x, double *y, double *z, double *w,
                             void *stream) {
    return rsi_sample_square_ex(RSI_SEQ_SOBOL, seed, n, cx, cy, z0, half_width, x, y, z, w, stream);
}

rsi_status rsi_sample_cap(rsi_sequence seq, uint32_t seed, int64_t n, double radius,
                          double curvature, const double *centre, double tilt, double *x, double *y,
                          double *z, double *w, void *stream) {
    UnitSource us;
    RSI_TRY(unit_source(seq, seed, n, us));
    if (!(radius > 0.0) || !(curvature >= radius) || !std::isfinite(curvature)) return RSI_ERR_ARG;
    if (n == 0) return RSI_OK;
    if (!centre || !x || !y || !z || !w) return RSI_ERR_NULL;
    const double sa = radius / curvature, ca = sqrt(1.0 - sa * sa);
    const double wj = 2.0 * kPi * curvature * curvature * (1.0 - ca) / (double)n;
    hipLaunchKernelGGL(cap_kernel, dim3(grid_for(n)), dim3(256), 0, as_stream(stream), us, n, curvature, ca,
                       centre[0], centre[1], centre[2], cos(tilt), sin(tilt), wj, x, y, z, w);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

rsi_status rsi_apodise(int64_t n, const double *x, const double *y, const double *z,
                       const double *centre, const double *axis, double width, double *w,
                       void *stream) {
    if (n < 0) return RSI_ERR_SIZE;
    if (!(width > 0.0)) return RSI_ERR_ARG;
    if (!centre || !axis) return RSI_ERR_NULL;
    const double an = sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
    if (!(an > 0.0)) return RSI_ERR_ARG;
    if (n == 0) return RSI_OK;
    if (!x || !y || !z || !w) return RSI_ERR_NULL;
    hipLaunchKernelGGL(apodise_kernel, dim3(grid_for(n)), dim3(256), 0, as_stream(stream), n, x, y, z,
                       centre[0], centre[1], centre[2], axis[0] / an, axis[1] / an, axis[2] / an,
                       1.0 / (width * width), w);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

}  // extern "C"
