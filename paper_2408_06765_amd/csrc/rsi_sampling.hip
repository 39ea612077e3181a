// rsi_sampling.hip -- sample points on the radiating surfaces (Sec. 2.3, eqs. 16-18)
// and the small ABI utilities (status strings, last error, version).
//
// The paper draws its QMC points from a Halton sequence; this library uses a
// two-dimensional Sobol sequence with a hash-based nested uniform (Owen) scramble,
// which keeps the (0, m, 2)-net property of every power-of-two prefix.  Each point is
// computed from its index alone, so any range of points is one independent launch.
#include <cstring>

#include "rsi_internal.h"

namespace rsi {

static thread_local std::string g_last_error;

void set_last_error(const char *what, hipError_t e) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
}

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

__global__ void __launch_bounds__(256) disc_kernel(uint32_t s0, uint32_t s1, int64_t n,
                                                   double radius, double cx, double cy,
                                                   double cz, double ct, double st, double wj,
                                                   double *x, double *y, double *z,
                                                   double *w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t u0, u1;
    scrambled_pair((uint32_t)i, s0, s1, u0, u1);
    // eq. (18): area-uniform radius and uniform angle
    const double r = radius * sqrt((double)u0 * kU32);
    double sn, cs;
    sincospi(2.0 * ((double)u1 * kU32), &sn, &cs);
    const double xi = r * cs, eta = r * sn;
    x[i] = cx + xi * ct;  // rotation by `tilt` about +y, then translation
    y[i] = cy + eta;
    z[i] = cz - xi * st;
    w[i] = wj;
}

__global__ void __launch_bounds__(256) square_kernel(uint32_t s0, uint32_t s1, int64_t n,
                                                     double cx, double cy, double z0,
                                                     double h, double wj, double *x,
                                                     double *y, double *z, double *w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t u0, u1;
    scrambled_pair((uint32_t)i, s0, s1, u0, u1);
    // eq. (17): uniform on the square [cx - h, cx + h] x [cy - h, cy + h]
    x[i] = cx + h * (2.0 * ((double)u0 * kU32) - 1.0);
    y[i] = cy + h * (2.0 * ((double)u1 * kU32) - 1.0);
    z[i] = z0;
    w[i] = wj;
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
    }
    return "RSI_UNKNOWN_STATUS";
}

const char *rsi_last_error(void) { return g_last_error.c_str(); }

int rsi_version(void) { return (1 << 16) | 1; }

rsi_status rsi_sobol2d(uint32_t seed, int64_t first, int64_t n, uint32_t *out, void *stream) {
    if (first < 0 || n < 0 || first + n > (int64_t(1) << 32)) return RSI_ERR_SIZE;
    if (n == 0) return RSI_OK;
    if (!out) return RSI_ERR_NULL;
    hipLaunchKernelGGL(sobol2d_kernel, dim3(grid_for(n)), dim3(256), 0, as_stream(stream),
                       coord_seed(seed, 0), coord_seed(seed, 1), first, n, out);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

rsi_status rsi_sample_disc(uint32_t seed, int64_t n, double radius, const double *centre,
                           double tilt, double *x, double *y, double *z, double *w,
                           void *stream) {
    if (n < 0 || n > (int64_t(1) << 32)) return RSI_ERR_SIZE;
    if (!(radius > 0.0)) return RSI_ERR_ARG;
    if (n == 0) return RSI_OK;
    if (!centre || !x || !y || !z || !w) return RSI_ERR_NULL;
    const double wj = kPi * radius * radius / (double)n;
    hipLaunchKernelGGL(disc_kernel, dim3(grid_for(n)), dim3(256), 0, as_stream(stream),
                       coord_seed(seed, 0), coord_seed(seed, 1), n, radius, centre[0],
                       centre[1], centre[2], cos(tilt), sin(tilt), wj, x, y, z, w);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

rsi_status rsi_sample_square(uint32_t seed, int64_t n, double cx, double cy, double z0,
                             double half_width, double *x, double *y, double *z, double *w,
                             void *stream) {
    if (n < 0 || n > (int64_t(1) << 32)) return RSI_ERR_SIZE;
    if (!(half_width > 0.0)) return RSI_ERR_ARG;
    if (n == 0) return RSI_OK;
    if (!x || !y || !z || !w) return RSI_ERR_NULL;
    const double wj = 4.0 * half_width * half_width / (double)n;
    hipLaunchKernelGGL(square_kernel, dim3(grid_for(n)), dim3(256), 0, as_stream(stream),
                       coord_seed(seed, 0), coord_seed(seed, 1), n, cx, cy, z0, half_width, wj,
                       x, y, z, w);
    RSI_HIP(hipGetLastError());
    return RSI_OK;
}

}  // extern "C"
