// rsi_internal.h -- shared internals of librsi (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <functional>
#include <string>
#include <vector>

#include "../../include/rsi.h"

namespace rsi {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
// Pairs closer than this contribute nothing in the FP64 path (the kernel is
// singular on the radiating surface).
constexpr double kRMin = 1.0e-12;

// Threads per workgroup of the pair-sum kernels (four wave64s).
constexpr int kBlock = 256;

void set_last_error(const char *what, hipError_t e);
void set_last_error_text(const std::string &text);

#define RSI_HIP(call)                                                   \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) {                                         \
            ::rsi::set_last_error(#call, e_);                           \
            return RSI_ERR_DEVICE;                                      \
        }                                                               \
    } while (0)

#define RSI_TRY(call)                                                   \
    do {                                                                \
        rsi_status s_ = (call);                                         \
        if (s_ != RSI_OK) return s_;                                    \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Debug check of device inputs (rsi_set_check_finite): RSI_ERR_NONFINITE if any of the
// given arrays (device pointer, element count; null pointers and empty arrays skipped)
// holds a NaN or an infinity; RSI_OK at once when the check is off.  Synchronises s.
// flag: a device int the check may use, or NULL to take one from the stream-ordered
// allocator.
struct DevSpan {
    const double *p;
    int64_t n;
};
rsi_status check_finite(hipStream_t s, const std::vector<DevSpan> &arrays, int *flag = nullptr);
inline void add_points(std::vector<DevSpan> &v, const rsi_points &p) {
    v.push_back({p.x, p.n});
    v.push_back({p.y, p.n});
    v.push_back({p.z, p.n});
}

// Stream-ordered scratch allocations released together (hipFreeAsync) on scope exit.
class Scratch {
public:
    explicit Scratch(hipStream_t s) : stream_(s) {}
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
    ~Scratch() {
        for (void *p : ptrs_) (void)hipFreeAsync(p, stream_);
    }
    template <class T>
    rsi_status alloc(T **p, size_t count) {
        *p = nullptr;
        if (count == 0) count = 1;
        hipError_t e = hipMallocAsync(reinterpret_cast<void **>(p), sizeof(T) * count, stream_);
        if (e != hipSuccess) {
            set_last_error("hipMallocAsync", e);
            return RSI_ERR_WORKSPACE;
        }
        ptrs_.push_back(*p);
        return RSI_OK;
    }

private:
    hipStream_t stream_;
    std::vector<void *> ptrs_;
};

// Device memory that lives as long as its owner (plans).
class DeviceBuffer {
public:
    DeviceBuffer() = default;
    DeviceBuffer(const DeviceBuffer &) = delete;
    DeviceBuffer &operator=(const DeviceBuffer &) = delete;
    ~DeviceBuffer() { release(); }
    rsi_status alloc(size_t bytes) {
        release();
        if (bytes == 0) bytes = 16;
        hipError_t e = hipMalloc(&ptr_, bytes);
        if (e != hipSuccess) {
            ptr_ = nullptr;
            set_last_error("hipMalloc", e);
            return RSI_ERR_WORKSPACE;
        }
        bytes_ = bytes;
        return RSI_OK;
    }
    void release() {
        if (ptr_) (void)hipFree(ptr_);
        ptr_ = nullptr;
        bytes_ = 0;
    }
    template <class T>
    T *as() const { return reinterpret_cast<T *>(ptr_); }
    size_t bytes() const { return bytes_; }

private:
    void *ptr_ = nullptr;
    size_t bytes_ = 0;
};

// ---------------------------------------------------------------------------
// FP32 source records.  One record per source, read by wave-uniform (scalar)
// loads: offsets from the set's anchor, |offset|^2, the folded strength
// s'_j = -(1/2pi) w_j s_j in polar form, and the normal offset n.e_j used by the
// dipole.  The strength is s'_j = a e^{2 pi i psi} with psi in (-1/4, 1/4]
// revolutions and a signed, stored as a and the length psi lambda (metres, lambda =
// c / f of the stage), so a real strength of either sign has psil = 0 at every
// frequency.
// ---------------------------------------------------------------------------
struct alignas(32) SrcRecF {
    float ex, ey, ez, es2;
    float a, psil, h, pad;
};

// Polar form of a folded strength (sre + i sim) for wavelength lam.
__device__ inline void polar_strength(double sre, double sim, double lam, float &a,
                                      float &psil) {
    double m = hypot(sre, sim);
    double psi = atan2(sim, sre) / kTwoPi;  // (-1/2, 1/2]
    if (psi > 0.25) {
        psi -= 0.5;
        m = -m;
    } else if (psi <= -0.25) {
        psi += 0.5;
        m = -m;
    }
    a = (float)m;
    psil = (float)(psi * lam);
}

// FP64 source records: absolute coordinates and folded strength.
struct alignas(64) SrcRecD {
    double x, y, z, pad0;
    double sre, sim, pad1, pad2;
};

// A prepared source set on the device.
struct SrcSetF {
    SrcRecF *rec = nullptr;   // [n]
    double *anchor = nullptr; // [4]: anchor x, y, z (device)
    int64_t n = 0;
};
struct SrcSetD {
    SrcRecD *rec = nullptr;
    int64_t n = 0;
};

struct Targets {
    const double *x, *y, *z;
    int64_t n;
};

// Launch shape of one pair sum.
struct PairShape {
    int tpl = 2;          // targets per lane (1, 2 or 4)
    int64_t chunk = 0;    // sources per split (0: all)
    bool few = false;     // FP32: one wave per (field point, split), sources across its lanes
};

// --- rsi_pairsum.hip ---------------------------------------------------------
rsi_status bbox_partials(const rsi_points &pts, double *partials /*[kBBoxBlocks*6]*/,
                         hipStream_t s);
constexpr int kBBoxBlocks = 64;
// Strengths are folded as -(1/2pi) w_j s_j F with a stage factor F (1; ik for RSI_OMNI
// sources; -1 for a dipole radiating along -z).  lam = c / f of the stage: needed only
// for complex strengths (vel != NULL or F not real).
struct Cplx {
    double re, im;
};
rsi_status prep_sources_f32(const rsi_points &pts, const double *w, const double *vel,
                            double v0, const double *normal, const double *partials,
                            double lam, Cplx F, SrcSetF &set, hipStream_t s);
rsi_status set_strength_f32(SrcSetF &set, const double *w, const void *field, bool field_fp64,
                            const double *tco, double lam, Cplx F, hipStream_t s);
rsi_status prep_sources_f64(const rsi_points &pts, const double *w, const double *vel,
                            double v0, Cplx F, SrcSetD &set, hipStream_t s);
rsi_status set_strength_f64(SrcSetD &set, const double *w, const double *field,
                            const double *tco, Cplx F, hipStream_t s);
// Waves a few-field-point launch aims for (64 per CU).  default_shape switches to it when
// the launch with one field point per lane would have fewer than `few_below` waves: the
// RSI pair sum (short pairs, scalar records) from below 8 waves per CU, the ray model
// (long, divergent pairs) from below 32.  few_below = 0: never (the FP64 paths, which
// have one launch only; their source splits then follow the one-point-per-lane rule).
constexpr int64_t kFewWaves = 16384;
// min_chunk: fewest sources per split (the RSI pair sum keeps 4096; the ray model, whose
// pairs cost ~6x more, splits finer).
PairShape default_shape(int64_t n_src, int64_t n_tgt, int64_t few_below = kFewWaves / 8,
                        int64_t min_chunk = 4096);
// Integer environment override (tuning knobs): the value if it parses as 1 .. 2^30 - 1.
int env_int(const char *name, int dflt);
int64_t partial_slots(const PairShape &sh, int64_t n_src, int64_t n_tgt);
// planar_z: every source lies on the plane z = const through the set's anchor (normal
// +z); the kernel then drops the z terms (interface samples, by the ABI contract).
rsi_status pairsum_f32(const SrcSetF &set, const Targets &t, rsi_kernel kind,
                       const double *normal, double c, double freq, const PairShape &sh,
                       float2 *partial, float2 *out, hipStream_t s, bool planar_z = false);
// Argument checks shared by the single-frequency and multi-frequency pair-sum entry
// points (freq: the first frequency); RSI_OK also for tgt->n == 0.
rsi_status validate_propagate(const rsi_points *src, const double *src_w, const double *src_vel,
                              const double *normal, const rsi_points *tgt, rsi_medium medium,
                              double freq, rsi_kernel kind, rsi_precision prec, uint32_t flags,
                              void *out);
rsi_status pairsum_f64(const SrcSetD &set, const Targets &t, rsi_kernel kind,
                       const double *normal, double c, double freq, const PairShape &sh,
                       double2 *partial, double2 *out, hipStream_t s);

// --- rsi_multifreq.hip -------------------------------------------------------
// True when freqs[0..n) is a uniform grid f0 + q df (n >= 2, df > 0).
bool uniform_grid(const double *freqs, int n, double &f0, double &df);
// Frequencies per block of the multi-frequency kernel for a grid of n_freq (16 or 32;
// RSI_MF_BLOCK forces one), and n_freq rounded up to it: the row length of the strengths.
int mf_block(int n_freq);
int mf_pad(int n_freq);
// S [n][mf_pad(n_freq)] of -(1/2pi) w T phi from field [n_freq][n].
// S[j][q] = -(1/2pi) w_j T_j field_q(Q_j) (Fa + i Fb k_q), k_q = 2 pi (f0 + q df) / c
rsi_status strength_multifreq(int64_t n, int n_freq, const double *w, const float2 *field,
                              const double *tco, double Fa, double Fb, double c, double f0,
                              double df, float2 *S, hipStream_t s);
// One stage for all frequencies; S == nullptr: the record strengths serve every frequency.
rsi_status pairsum_multifreq_f32(const SrcSetF &set, const float2 *S, const Targets &t,
                                 rsi_kernel kind, bool planar_z, double c, double f0, double df,
                                 int n_freq, float2 *out, hipStream_t s);

// --- rsi_chain.hip -----------------------------------------------------------
// Workspace of a chain: shared by the one-shot call and the chain plan.
struct ChainWork {
    std::vector<double *> tco;   // complex FP64 transmission coefficients per interface
    std::vector<double *> bbox;  // partial extents per source set
    std::vector<SrcSetF> setf;   // [0]: transducer, [m]: interface m
    std::vector<SrcSetD> setd;
    void *field[2] = {nullptr, nullptr};
    void *partial = nullptr;
    float2 *S = nullptr;      // multi-frequency strengths
    bool multifreq = false;   // FP32 on a uniform frequency grid: one launch per stage
    double f0 = 0.0, df = 0.0;
    uint32_t flags = 0;       // RSI_CHAIN_*
    double *rco = nullptr;    // RSI_CHAIN_ABOVE: reflection coefficients of the last interface
    void *above = nullptr;    // RSI_CHAIN_ABOVE: reflected field at the points
};
using AllocFn = std::function<rsi_status(void **, size_t)>;
rsi_status validate_chain(const rsi_transducer *xd, const rsi_interface *ifaces, int n_if,
                          const rsi_medium *media, const rsi_points *tgt, const double *freqs,
                          int n_freq, rsi_tmode tmode, rsi_precision prec, uint32_t flags,
                          void *out);
rsi_status alloc_chain(const AllocFn &alloc, const rsi_transducer *xd,
                       const rsi_interface *ifaces, int n_if, const rsi_points *tgt,
                       const double *freqs, int n_freq, rsi_precision prec, uint32_t flags,
                       ChainWork &W);
// The device inputs of a chain, for check_finite.
std::vector<DevSpan> chain_inputs(const rsi_transducer *xd, const rsi_interface *ifaces, int n_if,
                                  const rsi_points *tgt);
rsi_status enqueue_chain(const rsi_transducer *xd, const rsi_interface *ifaces, int n_if,
                         const rsi_medium *media, const rsi_points *tgt, const double *freqs,
                         int n_freq, rsi_tmode tmode, rsi_precision prec, void *out,
                         ChainWork &W, hipStream_t s);
rsi_status coefficient_device(bool reflect, rsi_tmode tmode, int m, const double *zif,
                              const rsi_medium *media, const double *xc, const double *axis,
                              int64_t n, const double *qx, const double *qy, double *out,
                              hipStream_t s);
rsi_status transmission_device(rsi_tmode tmode, int m, const double *zif,
                               const rsi_medium *media, const double *xc, const double *axis,
                               int64_t n, const double *qx, const double *qy, double *out,
                               hipStream_t s);

}  // namespace rsi
