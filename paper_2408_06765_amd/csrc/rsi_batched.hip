// rsi_batched.hip -- batching: many independent pair sums in one persistent launch,
// plans that capture a chain or a batch into a hipGraph, and the autotuner that picks
// the launch shape of the batched kernel.
//
// The batched work is cut into items (instance, target tile, source chunk).  Items are
// sorted by cost (largest first) on the host and pulled by the workgroups of a
// persistent grid from a device counter, so instances that differ by orders of
// magnitude in size share one launch without a tail of idle CUs.  Every item writes
// its partial sum to a fixed slot, and a final kernel adds the chunks of each target in
// chunk order: the result does not depend on which workgroup ran which item.
#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <memory>
#include <sstream>

#include <sys/stat.h>

#include "rsi_device.h"

namespace rsi {

struct InstDev {
    const SrcRecF *recf;
    const SrcRecD *recd;
    const double *anchor;
    const double *tx, *ty, *tz;
    int64_t n_tgt;
    double inv_lam, k, nx, ny, nz;
    int32_t kind, n_chunks;
    void *out;
    void *partial;  // [n_chunks][n_tgt] when n_chunks > 1
};

struct PrepDev {
    const double *x, *y, *z, *w, *vel;
    double v0, nx, ny, nz;
    double lam;       // c / f of the instance (phase offset of complex strengths)
    double Fre, Fim;  // strength factor: 1, or ik for RSI_OMNI
    int64_t n;
    double *partials;  // [kBBoxBlocks * 6]
    double *anchor;    // [4]
    SrcRecF *recf;
    SrcRecD *recd;
};

struct WorkItem {
    int32_t inst, chunk;
    int64_t tbase;
    int64_t j0, j1;
};

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
__global__ void reset_counter_kernel(unsigned *counter) { *counter = 0u; }

__global__ void __launch_bounds__(256) bbox_batched_kernel(const PrepDev *__restrict__ P) {
    const PrepDev p = P[blockIdx.y];
    double v[6] = {1.0e300, 1.0e300, 1.0e300, -1.0e300, -1.0e300, -1.0e300};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < p.n;
         i += (int64_t)gridDim.x * 256) {
        const double a = p.x[i], b = p.y[i], c = p.z[i];
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
        p.partials[blockIdx.x * 6 + k] = r;
    }
}

__device__ inline int find_segment(const int64_t *__restrict__ starts, int n, int64_t key) {
    int lo = 0, hi = n - 1;  // largest s with starts[s] <= key
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= key) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <bool FP64>
__global__ void __launch_bounds__(256) prep_batched_kernel(const PrepDev *__restrict__ P,
                                                           const int64_t *__restrict__ block_start,
                                                           int n_inst) {
    const int inst = find_segment(block_start, n_inst, (int64_t)blockIdx.x);
    const PrepDev p = P[inst];
    const int64_t j = ((int64_t)blockIdx.x - block_start[inst]) * 256 + threadIdx.x;
    double sre = p.v0, sim = 0.0;
    if constexpr (FP64) {
        if (j >= p.n) return;
        if (p.vel) {
            sre = p.vel[2 * j];
            sim = p.vel[2 * j + 1];
        }
        const double scale = -p.w[j] / kTwoPi;
        SrcRecD r;
        r.x = p.x[j];
        r.y = p.y[j];
        r.z = p.z[j];
        r.pad0 = 0.0;
        r.sre = scale * (sre * p.Fre - sim * p.Fim);
        r.sim = scale * (sre * p.Fim + sim * p.Fre);
        r.pad1 = r.pad2 = 0.0;
        p.recd[j] = r;
    } else {
        double lo[3] = {1.0e300, 1.0e300, 1.0e300}, hi[3] = {-1.0e300, -1.0e300, -1.0e300};
        for (int b = 0; b < kBBoxBlocks; ++b)
            for (int k = 0; k < 3; ++k) {
                lo[k] = fmin(lo[k], p.partials[b * 6 + k]);
                hi[k] = fmax(hi[k], p.partials[b * 6 + 3 + k]);
            }
        const double ax = 0.5 * (lo[0] + hi[0]), ay = 0.5 * (lo[1] + hi[1]),
                     az = 0.5 * (lo[2] + hi[2]);
        if (j == 0) {
            const double sx = hi[0] - lo[0], sy = hi[1] - lo[1], sz = hi[2] - lo[2];
            p.anchor[0] = ax;
            p.anchor[1] = ay;
            p.anchor[2] = az;
            p.anchor[3] = 0.5 * sqrt(sx * sx + sy * sy + sz * sz);  // bounds |Q_j - C|
        }
        if (j >= p.n) return;
        if (p.vel) {
            sre = p.vel[2 * j];
            sim = p.vel[2 * j + 1];
        }
        const float ex = (float)(p.x[j] - ax), ey = (float)(p.y[j] - ay), ez = (float)(p.z[j] - az);
        const double dex = ex, dey = ey, dez = ez;
        const double scale = -p.w[j] / kTwoPi;
        SrcRecF r;
        r.ex = ex;
        r.ey = ey;
        r.ez = ez;
        r.es2 = (float)(dex * dex + dey * dey + dez * dez);
        polar_strength(scale * (sre * p.Fre - sim * p.Fim), scale * (sre * p.Fim + sim * p.Fre), p.lam, r.a,
                       r.psil);
        r.h = (float)(p.nx * dex + p.ny * dey + p.nz * dez);
        r.pad = 0.0f;
        p.recf[j] = r;
    }
}

template <int KIND, int TPL>
__device__ __forceinline__ void run_item_f32(const InstDev &I, const WorkItem &w) {
    TargetsF<KIND, TPL> T;
    const int64_t tbase = w.tbase + threadIdx.x;
    setup_targets_f32<KIND, TPL>(T, I.tx, I.ty, I.tz, I.n_tgt, tbase, I.anchor[0], I.anchor[1],
                                 I.anchor[2], I.inv_lam, I.nx, I.ny, I.nz);
    float mre[TPL], mim[TPL];
    if (phase_in_sin_range(I.anchor[3], I.inv_lam))
        sum_range_f32<KIND, TPL, false, false>(T, I.recf, w.j0, w.j1, (float)I.inv_lam, (float)I.k,
                                               mre, mim);
    else
        sum_range_f32<KIND, TPL, false, true>(T, I.recf, w.j0, w.j1, (float)I.inv_lam, (float)I.k,
                                              mre, mim);
    float2 *o = I.n_chunks > 1 ? static_cast<float2 *>(I.partial) + (int64_t)w.chunk * I.n_tgt
                               : static_cast<float2 *>(I.out);
#pragma unroll
    for (int u = 0; u < TPL; ++u) {
        const int64_t i = tbase + (int64_t)u * kBlock;
        if (i < I.n_tgt) o[i] = make_float2(mre[u], mim[u]);
    }
}

// Persistent kernel: every workgroup pulls items until the counter passes n_items, so
// each wave reaches the exit test after a finite number of items.
template <int TPL>
__global__ void __launch_bounds__(kBlock) batched_f32_kernel(const InstDev *__restrict__ insts,
                                                             const WorkItem *__restrict__ items,
                                                             int n_items, unsigned *counter) {
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);  // the same for every lane
        __syncthreads();
        if (it >= n_items) break;
        const WorkItem w = items[it];
        const InstDev I = insts[w.inst];
        if (I.kind == RSI_MONOPOLE) run_item_f32<RSI_MONOPOLE, TPL>(I, w);
        else run_item_f32<RSI_DIPOLE, TPL>(I, w);
    }
}

__global__ void __launch_bounds__(kBlock) batched_f64_kernel(const InstDev *__restrict__ insts,
                                                             const WorkItem *__restrict__ items,
                                                             int n_items, unsigned *counter) {
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= n_items) break;
        const WorkItem w = items[it];
        const InstDev I = insts[w.inst];
        int64_t i = w.tbase + threadIdx.x;
        const bool valid = i < I.n_tgt;
        if (!valid) i = I.n_tgt - 1;
        double mre, mim;
        if (I.kind == RSI_MONOPOLE)
            sum_range_f64<RSI_MONOPOLE>(I.tx[i], I.ty[i], I.tz[i], I.recd, w.j0, w.j1, I.inv_lam,
                                        I.k, I.nx, I.ny, I.nz, mre, mim);
        else
            sum_range_f64<RSI_DIPOLE>(I.tx[i], I.ty[i], I.tz[i], I.recd, w.j0, w.j1, I.inv_lam,
                                      I.k, I.nx, I.ny, I.nz, mre, mim);
        double2 *o = I.n_chunks > 1 ? static_cast<double2 *>(I.partial) + (int64_t)w.chunk * I.n_tgt
                                    : static_cast<double2 *>(I.out);
        if (valid) o[i] = make_double2(mre, mim);
    }
}

// Fixed-order sum of the chunk partials of every split instance.
template <typename T2>
__global__ void __launch_bounds__(256) batched_reduce_kernel(const InstDev *__restrict__ insts,
                                                             const int64_t *__restrict__ seg_start,
                                                             const int32_t *__restrict__ seg_inst,
                                                             int n_seg, int64_t total) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= total) return;
    const int s = find_segment(seg_start, n_seg, g);
    const InstDev I = insts[seg_inst[s]];
    const int64_t i = g - seg_start[s];
    const T2 *p = static_cast<const T2 *>(I.partial);
    double re = 0.0, im = 0.0;
    for (int c = 0; c < I.n_chunks; ++c) {
        const T2 v = p[(int64_t)c * I.n_tgt + i];
        re += (double)v.x;
        im += (double)v.y;
    }
    T2 r;
    r.x = re;
    r.y = im;
    static_cast<T2 *>(I.out)[i] = r;
}

// ---------------------------------------------------------------------------
// Host side: batch tables.
// ---------------------------------------------------------------------------
struct BatchShape {
    int tpl = 1;
    int64_t chunk = 16384;
};

struct BatchTables {
    std::vector<InstDev> inst;
    std::vector<PrepDev> prep;
    std::vector<WorkItem> items;
    std::vector<int64_t> prep_block_start;  // [n_inst]
    int64_t prep_blocks = 0;
    std::vector<int64_t> seg_start;  // reduce segments
    std::vector<int32_t> seg_inst;
    int64_t reduce_total = 0;
    size_t rec_bytes = 0, partial_bytes = 0, bbox_doubles = 0, anchor_doubles = 0;
};

struct BatchBuffers {
    DeviceBuffer inst, prep, items, block_start, seg_start, seg_inst, counter;
    DeviceBuffer rec, partial, bbox, anchor;
};

// The device inputs of a batch, for check_finite.
static std::vector<DevSpan> instance_inputs(const rsi_instance *inst, int n_inst) {
    std::vector<DevSpan> in;
    for (int i = 0; i < n_inst; ++i) {
        add_points(in, inst[i].src);
        in.push_back({inst[i].w, inst[i].src.n});
        in.push_back({inst[i].vel, 2 * inst[i].src.n});
        add_points(in, inst[i].tgt);
    }
    return in;
}

static rsi_status validate_instances(const rsi_instance *inst, int n_inst, rsi_precision prec) {
    if (n_inst < 0) return RSI_ERR_SIZE;
    if (n_inst > 0 && !inst) return RSI_ERR_NULL;
    if (prec != RSI_FP32 && prec != RSI_FP64) return RSI_ERR_ARG;
    for (int i = 0; i < n_inst; ++i) {
        const rsi_instance &a = inst[i];
        if (a.kind != RSI_MONOPOLE && a.kind != RSI_DIPOLE && a.kind != RSI_OMNI) return RSI_ERR_ARG;
        if (!(a.freq > 0.0) || !(a.medium.c > 0.0) || !std::isfinite(a.freq)) return RSI_ERR_ARG;
        if (a.src.n < 0 || a.tgt.n < 0) return RSI_ERR_SIZE;
        if (a.tgt.n > 0 && (!a.out || !a.tgt.x || !a.tgt.y || !a.tgt.z)) return RSI_ERR_NULL;
        if (a.src.n > 0 && (!a.src.x || !a.src.y || !a.src.z || !a.w)) return RSI_ERR_NULL;
        if (a.kind == RSI_DIPOLE) {
            const double l2 = a.normal[0] * a.normal[0] + a.normal[1] * a.normal[1] +
                              a.normal[2] * a.normal[2];
            if (!(l2 > 0.0)) return RSI_ERR_ARG;
        }
    }
    return RSI_OK;
}

// Host tables for one shape; device addresses are filled in by bind_tables.
static rsi_status build_tables(const rsi_instance *inst, int n_inst, rsi_precision prec,
                               const BatchShape &sh, BatchTables &T) {
    const int tpl = prec == RSI_FP64 ? 1 : sh.tpl;
    const int64_t tile = (int64_t)kBlock * tpl;
    const int64_t chunk = sh.chunk > 0 ? (sh.chunk + kSub - 1) / kSub * kSub : kSub;
    T = BatchTables{};
    T.inst.resize(n_inst);
    T.prep.resize(n_inst);
    T.prep_block_start.resize(n_inst);
    size_t rec_off = 0, part_off = 0;
    std::vector<std::pair<double, WorkItem>> costed;
    for (int i = 0; i < n_inst; ++i) {
        const rsi_instance &a = inst[i];
        InstDev &d = T.inst[i];
        std::memset(&d, 0, sizeof(d));
        d.n_tgt = a.tgt.n;
        d.tx = a.tgt.x;
        d.ty = a.tgt.y;
        d.tz = a.tgt.z;
        d.inv_lam = a.freq / a.medium.c;
        d.k = kTwoPi * a.freq / a.medium.c;
        const double l = std::sqrt(a.normal[0] * a.normal[0] + a.normal[1] * a.normal[1] +
                                   a.normal[2] * a.normal[2]);
        if (a.kind == RSI_DIPOLE && l > 0.0) {
            d.nx = a.normal[0] / l;
            d.ny = a.normal[1] / l;
            d.nz = a.normal[2] / l;
        }
        d.kind = a.kind == RSI_OMNI ? RSI_MONOPOLE : a.kind;  // omni: monopole of strengths x ik
        d.out = a.out;
        const int64_t nchunks = a.src.n > 0 ? (a.src.n + chunk - 1) / chunk : 1;
        d.n_chunks = (int32_t)nchunks;
        // record offsets (bytes) and partial offsets (elements) relative to their buffers
        d.recf = reinterpret_cast<const SrcRecF *>(rec_off);
        d.recd = reinterpret_cast<const SrcRecD *>(rec_off);
        d.anchor = reinterpret_cast<const double *>((size_t)i * 4 * sizeof(double));
        rec_off += (size_t)std::max<int64_t>(a.src.n, 1) *
                   (prec == RSI_FP32 ? sizeof(SrcRecF) : sizeof(SrcRecD));
        rec_off = (rec_off + 255) / 256 * 256;
        if (nchunks > 1 && a.tgt.n > 0) {
            d.partial = reinterpret_cast<void *>(part_off);
            part_off += (size_t)nchunks * (size_t)a.tgt.n;
            T.seg_start.push_back(T.reduce_total);
            T.seg_inst.push_back(i);
            T.reduce_total += a.tgt.n;
        }
        PrepDev &p = T.prep[i];
        std::memset(&p, 0, sizeof(p));
        p.x = a.src.x;
        p.y = a.src.y;
        p.z = a.src.z;
        p.w = a.w;
        p.vel = a.vel;
        p.v0 = a.v0;
        p.lam = a.medium.c / a.freq;
        p.Fre = a.kind == RSI_OMNI ? 0.0 : 1.0;
        p.Fim = a.kind == RSI_OMNI ? d.k : 0.0;
        p.nx = d.nx;
        p.ny = d.ny;
        p.nz = d.nz;
        p.n = a.src.n;
        T.prep_block_start[i] = T.prep_blocks;
        T.prep_blocks += std::max<int64_t>((a.src.n + 255) / 256, 1);
        if (a.tgt.n == 0) continue;
        const int64_t ntiles = (a.tgt.n + tile - 1) / tile;
        for (int64_t c = 0; c < nchunks; ++c) {
            const int64_t j0 = std::min(a.src.n, c * chunk), j1 = std::min(a.src.n, (c + 1) * chunk);
            for (int64_t t = 0; t < ntiles; ++t) {
                WorkItem w{};
                w.inst = i;
                w.chunk = (int32_t)c;
                w.tbase = t * tile;
                w.j0 = j0;
                w.j1 = j1;
                const int64_t nt = std::min(tile, a.tgt.n - t * tile);
                // cost: pairs, plus the per-target set-up that every item pays
                costed.push_back({(double)(j1 - j0) * (double)nt + 64.0 * (double)nt, w});
            }
        }
    }
    if (costed.size() > 0x7fffffff) return RSI_ERR_SIZE;
    std::stable_sort(costed.begin(), costed.end(),
                     [](const auto &a, const auto &b) { return a.first > b.first; });
    T.items.reserve(costed.size());
    for (auto &c : costed) T.items.push_back(c.second);
    T.rec_bytes = rec_off;
    T.partial_bytes = part_off * (prec == RSI_FP32 ? sizeof(float2) : sizeof(double2));
    T.bbox_doubles = (size_t)n_inst * kBBoxBlocks * 6;
    T.anchor_doubles = (size_t)n_inst * 4;
    return RSI_OK;
}

template <class T>
static rsi_status upload(DeviceBuffer &buf, const std::vector<T> &v) {
    RSI_TRY(buf.alloc(sizeof(T) * std::max<size_t>(v.size(), 1)));
    if (!v.empty()) RSI_HIP(hipMemcpy(buf.as<void>(), v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return RSI_OK;
}

// Allocate the device buffers, turn offsets into addresses and upload the tables.
static rsi_status bind_tables(BatchTables &T, rsi_precision prec, BatchBuffers &B) {
    RSI_TRY(B.rec.alloc(T.rec_bytes));
    RSI_TRY(B.partial.alloc(T.partial_bytes));
    RSI_TRY(B.bbox.alloc(sizeof(double) * std::max<size_t>(T.bbox_doubles, 1)));
    RSI_TRY(B.anchor.alloc(sizeof(double) * std::max<size_t>(T.anchor_doubles, 1)));
    RSI_TRY(B.counter.alloc(sizeof(unsigned)));
    char *rec = B.rec.as<char>();
    char *part = B.partial.as<char>();
    const size_t esz = prec == RSI_FP32 ? sizeof(float2) : sizeof(double2);
    for (size_t i = 0; i < T.inst.size(); ++i) {
        InstDev &d = T.inst[i];
        const size_t off = reinterpret_cast<size_t>(d.recf);
        d.recf = reinterpret_cast<const SrcRecF *>(rec + off);
        d.recd = reinterpret_cast<const SrcRecD *>(rec + off);
        d.anchor = B.anchor.as<double>() + i * 4;
        if (d.n_chunks > 1 && d.n_tgt > 0)
            d.partial = part + reinterpret_cast<size_t>(d.partial) * esz;
        else
            d.partial = nullptr;
        PrepDev &p = T.prep[i];
        p.partials = B.bbox.as<double>() + i * kBBoxBlocks * 6;
        p.anchor = const_cast<double *>(d.anchor);
        p.recf = const_cast<SrcRecF *>(d.recf);
        p.recd = const_cast<SrcRecD *>(d.recd);
    }
    RSI_TRY(upload(B.inst, T.inst));
    RSI_TRY(upload(B.prep, T.prep));
    RSI_TRY(upload(B.items, T.items));
    RSI_TRY(upload(B.block_start, T.prep_block_start));
    RSI_TRY(upload(B.seg_start, T.seg_start));
    RSI_TRY(upload(B.seg_inst, T.seg_inst));
    return RSI_OK;
}

// Persistent grid: as many workgroups as can be resident at once (compute units times
// the kernel's occupancy), so every SIMD holds as many waves as its registers allow;
// fewer waves leave the transcendental latency of the low-ILP one-target-per-lane loop
// exposed.
template <class K>
static int persistent_blocks(K kernel) {
    int dev = 0, cus = 256, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 4;
    return std::max(cus, 1) * per_cu;
}

static rsi_status enqueue_batched(const BatchTables &T, const BatchBuffers &B, rsi_precision prec,
                                  int tpl, hipStream_t s) {
    const int n_inst = (int)T.inst.size();
    if (n_inst == 0) return RSI_OK;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, B.counter.as<unsigned>());
    RSI_HIP(hipGetLastError());
    if (prec == RSI_FP32) {
        hipLaunchKernelGGL(bbox_batched_kernel, dim3(kBBoxBlocks, n_inst), dim3(256), 0, s,
                           B.prep.as<const PrepDev>());
        RSI_HIP(hipGetLastError());
        hipLaunchKernelGGL(prep_batched_kernel<false>, dim3((unsigned)T.prep_blocks), dim3(256), 0, s,
                           B.prep.as<const PrepDev>(), B.block_start.as<const int64_t>(), n_inst);
    } else {
        hipLaunchKernelGGL(prep_batched_kernel<true>, dim3((unsigned)T.prep_blocks), dim3(256), 0, s,
                           B.prep.as<const PrepDev>(), B.block_start.as<const int64_t>(), n_inst);
    }
    RSI_HIP(hipGetLastError());
    const int n_items = (int)T.items.size();
    if (n_items > 0) {
        const InstDev *I = B.inst.as<const InstDev>();
        const WorkItem *W = B.items.as<const WorkItem>();
        unsigned *ctr = B.counter.as<unsigned>();
        auto launch = [&](auto kernel) {
            const int grid = (int)std::min<int64_t>(persistent_blocks(kernel), n_items);
            hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, I, W, n_items, ctr);
        };
        if (prec == RSI_FP64) launch(batched_f64_kernel);
        else if (tpl == 1) launch(batched_f32_kernel<1>);
        else if (tpl == 4) launch(batched_f32_kernel<4>);
        else launch(batched_f32_kernel<2>);
        RSI_HIP(hipGetLastError());
    }
    if (T.reduce_total > 0) {
        const dim3 g((unsigned)((T.reduce_total + 255) / 256));
        if (prec == RSI_FP32)
            hipLaunchKernelGGL(batched_reduce_kernel<float2>, g, dim3(256), 0, s,
                               B.inst.as<const InstDev>(), B.seg_start.as<const int64_t>(),
                               B.seg_inst.as<const int32_t>(), (int)T.seg_inst.size(), T.reduce_total);
        else
            hipLaunchKernelGGL(batched_reduce_kernel<double2>, g, dim3(256), 0, s,
                               B.inst.as<const InstDev>(), B.seg_start.as<const int64_t>(),
                               B.seg_inst.as<const int32_t>(), (int)T.seg_inst.size(), T.reduce_total);
        RSI_HIP(hipGetLastError());
    }
    return RSI_OK;
}

// ---------------------------------------------------------------------------
// Autotune cache: one line per workload key, "key tpl chunk ms".
// ---------------------------------------------------------------------------
static std::string cache_path() {
    if (const char *p = std::getenv("RSI_AUTOTUNE_CACHE")) return p;
    const char *home = std::getenv("HOME");
    return std::string(home ? home : ".") + "/.cache/rsi_autotune.txt";
}

static std::string workload_key(const rsi_instance *inst, int n_inst, rsi_precision prec) {
    double pairs = 0.0;
    int64_t max_src = 0, max_tgt = 0;
    int kinds = 0;
    for (int i = 0; i < n_inst; ++i) {
        pairs += (double)inst[i].src.n * (double)inst[i].tgt.n;
        max_src = std::max(max_src, inst[i].src.n);
        max_tgt = std::max(max_tgt, inst[i].tgt.n);
        kinds |= 1 << inst[i].kind;
    }
    char dev[64] = "gpu";
    hipDeviceProp_t prop;
    int d = 0;
    if (hipGetDevice(&d) == hipSuccess && hipGetDeviceProperties(&prop, d) == hipSuccess)
        std::snprintf(dev, sizeof(dev), "%s", prop.gcnArchName);
    for (char *c = dev; *c; ++c)
        if (*c == ' ' || *c == ':') *c = '_';
    std::ostringstream os;
    os << "batched/" << dev << "/p" << (int)prec << "/k" << kinds << "/n" << n_inst << "/lp"
       << (int)std::lround(std::log2(std::max(pairs, 1.0)) * 4) << "/ms"
       << (int)std::lround(std::log2((double)std::max<int64_t>(max_src, 1)))
       << "/mt" << (int)std::lround(std::log2((double)std::max<int64_t>(max_tgt, 1)));
    return os.str();
}

static bool cache_lookup(const std::string &key, BatchShape &sh) {
    std::ifstream f(cache_path());
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        int tpl = 0;
        long long chunk = 0;
        double ms = 0.0;
        if (!(is >> k >> tpl >> chunk >> ms)) continue;  // corrupt line: ignored
        if (k != key || (tpl != 1 && tpl != 2 && tpl != 4) || chunk < kSub || chunk > (1LL << 32))
            continue;
        sh.tpl = tpl;
        sh.chunk = chunk;
        found = true;  // the last valid entry wins
    }
    return found;
}

static void cache_store(const std::string &key, const BatchShape &sh, double ms) {
    const std::string path = cache_path();
    const size_t slash = path.find_last_of('/');
    if (slash != std::string::npos) {
        // create the parent directory if needed (one level is enough for the default path)
        (void)mkdir(path.substr(0, slash).c_str(), 0755);
    }
    std::ofstream f(path, std::ios::app);
    if (f) f << key << ' ' << sh.tpl << ' ' << sh.chunk << ' ' << ms << '\n';
}

static BatchShape default_batch_shape(const rsi_instance *inst, int n_inst) {
    BatchShape sh;
    double pairs = 0.0;
    for (int i = 0; i < n_inst; ++i) pairs += (double)inst[i].src.n * (double)inst[i].tgt.n;
    sh.tpl = 1;
    // small items balance the CUs (measured best on a 256-instance scan: 4096 sources)
    sh.chunk = 4096;
    (void)pairs;
    return sh;
}

}  // namespace rsi

// ---------------------------------------------------------------------------
// Plans.
// ---------------------------------------------------------------------------
struct rsi_plan {
    int type = 0;  // 0: chain, 1: batched
    std::vector<std::unique_ptr<rsi::DeviceBuffer>> bufs;
    rsi::ChainWork W;
    rsi::BatchTables T;
    rsi::BatchBuffers B;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~rsi_plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace rsi {

// Capture `body` (which enqueues on the given stream) into plan->graph / plan->exec.
template <class F>
static rsi_status capture(rsi_plan *plan, F &&body) {
    hipStream_t cs = nullptr;
    RSI_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        set_last_error("hipStreamBeginCapture", e);
        return RSI_ERR_DEVICE;
    }
    const rsi_status st = body(cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (st != RSI_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) {
        set_last_error("hipStreamEndCapture", e);
        return RSI_ERR_DEVICE;
    }
    plan->graph = g;
    RSI_HIP(hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0));
    return RSI_OK;
}

}  // namespace rsi

using namespace rsi;

extern "C" {

rsi_status rsi_plan_create_chain_ex(rsi_plan **plan, const rsi_transducer *xd,
                                    const rsi_interface *ifaces, int n_if, const rsi_medium *media,
                                    const rsi_points *tgt, const double *freqs, int n_freq,
                                    rsi_tmode tmode, rsi_precision prec, uint32_t flags, void *out) {
    if (!plan) return RSI_ERR_NULL;
    *plan = nullptr;
    RSI_TRY(validate_chain(xd, ifaces, n_if, media, tgt, freqs, n_freq, tmode, prec, flags, out));
    RSI_TRY(check_finite(nullptr, chain_inputs(xd, ifaces, n_if, tgt)));
    std::unique_ptr<rsi_plan> p(new rsi_plan);
    p->type = 0;
    auto alloc = [&](void **ptr, size_t bytes) -> rsi_status {
        p->bufs.emplace_back(new DeviceBuffer);
        RSI_TRY(p->bufs.back()->alloc(bytes));
        *ptr = p->bufs.back()->as<void>();
        return RSI_OK;
    };
    RSI_TRY(alloc_chain(alloc, xd, ifaces, n_if, tgt, freqs, n_freq, prec, flags, p->W));
    // copies of the host descriptors: the captured graph keeps only device pointers and
    // kernel arguments, so nothing here needs to outlive the call
    if (tgt->n > 0 && n_freq > 0) {
        RSI_TRY(capture(p.get(), [&](hipStream_t cs) {
            return enqueue_chain(xd, ifaces, n_if, media, tgt, freqs, n_freq, tmode, prec, out,
                                 p->W, cs);
        }));
    }
    *plan = p.release();
    return RSI_OK;
}

rsi_status rsi_plan_create_chain(rsi_plan **plan, const rsi_transducer *xd,
                                 const rsi_interface *ifaces, int n_if, const rsi_medium *media,
                                 const rsi_points *tgt, const double *freqs, int n_freq,
                                 rsi_tmode tmode, rsi_precision prec, void *out) {
    return rsi_plan_create_chain_ex(plan, xd, ifaces, n_if, media, tgt, freqs, n_freq, tmode, prec, 0u,
                                    out);
}

rsi_status rsi_plan_create_batched(rsi_plan **plan, const rsi_instance *inst, int n_inst,
                                   rsi_precision prec) {
    if (!plan) return RSI_ERR_NULL;
    *plan = nullptr;
    RSI_TRY(validate_instances(inst, n_inst, prec));
    RSI_TRY(check_finite(nullptr, instance_inputs(inst, n_inst)));
    std::unique_ptr<rsi_plan> p(new rsi_plan);
    p->type = 1;
    BatchShape sh = default_batch_shape(inst, n_inst);
    (void)cache_lookup(workload_key(inst, n_inst, prec), sh);
    RSI_TRY(build_tables(inst, n_inst, prec, sh, p->T));
    RSI_TRY(bind_tables(p->T, prec, p->B));
    if (n_inst > 0) {
        RSI_TRY(capture(p.get(), [&](hipStream_t cs) {
            return enqueue_batched(p->T, p->B, prec, sh.tpl, cs);
        }));
    }
    *plan = p.release();
    return RSI_OK;
}

rsi_status rsi_plan_execute(rsi_plan *plan, void *stream) {
    if (!plan) return RSI_ERR_NULL;
    if (!plan->exec) return RSI_OK;  // empty plan
    RSI_HIP(hipGraphLaunch(plan->exec, as_stream(stream)));
    return RSI_OK;
}

rsi_status rsi_plan_destroy(rsi_plan *plan) {
    if (!plan) return RSI_OK;
    // the graph may still run on the caller's stream: wait for the device before freeing
    RSI_HIP(hipDeviceSynchronize());
    delete plan;
    return RSI_OK;
}

rsi_status rsi_propagate_batched(const rsi_instance *inst, int n_inst, rsi_precision prec,
                                 void *stream) {
    RSI_TRY(validate_instances(inst, n_inst, prec));
    if (n_inst == 0) return RSI_OK;
    RSI_TRY(check_finite(as_stream(stream), instance_inputs(inst, n_inst)));
    BatchShape sh = default_batch_shape(inst, n_inst);
    (void)cache_lookup(workload_key(inst, n_inst, prec), sh);
    BatchTables T;
    BatchBuffers B;
    RSI_TRY(build_tables(inst, n_inst, prec, sh, T));
    RSI_TRY(bind_tables(T, prec, B));
    hipStream_t s = as_stream(stream);
    RSI_TRY(enqueue_batched(T, B, prec, sh.tpl, s));
    // the work list lives in this call's buffers: wait before releasing them
    RSI_HIP(hipStreamSynchronize(s));
    return RSI_OK;
}

rsi_status rsi_autotune_batched(const rsi_instance *inst, int n_inst, rsi_precision prec) {
    RSI_TRY(validate_instances(inst, n_inst, prec));
    if (n_inst == 0) return RSI_OK;
    const int tpls[] = {1, 2, 4};
    const int64_t chunks[] = {4096, 16384, 65536};
    BatchShape best;
    double best_ms = 1e300;
    hipStream_t s = nullptr;
    RSI_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    RSI_HIP(hipEventCreate(&e0));
    RSI_HIP(hipEventCreate(&e1));
    rsi_status st = RSI_OK;
    for (int tpl : tpls) {
        if (prec == RSI_FP64 && tpl != 1) continue;
        for (int64_t chunk : chunks) {
            BatchShape sh;
            sh.tpl = tpl;
            sh.chunk = chunk;
            BatchTables T;
            BatchBuffers B;
            st = build_tables(inst, n_inst, prec, sh, T);
            if (st == RSI_OK) st = bind_tables(T, prec, B);
            if (st == RSI_OK) st = enqueue_batched(T, B, prec, tpl, s);  // warm-up
            if (st == RSI_OK && hipEventRecord(e0, s) != hipSuccess) st = RSI_ERR_DEVICE;
            for (int rep = 0; rep < 3 && st == RSI_OK; ++rep) st = enqueue_batched(T, B, prec, tpl, s);
            if (st == RSI_OK && hipEventRecord(e1, s) != hipSuccess) st = RSI_ERR_DEVICE;
            if (st == RSI_OK && hipEventSynchronize(e1) != hipSuccess) st = RSI_ERR_DEVICE;
            float ms = 0.0f;
            if (st == RSI_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = RSI_ERR_DEVICE;
            if (st != RSI_OK) break;
            if (ms / 3.0 < best_ms) {
                best_ms = ms / 3.0;
                best = sh;
            }
        }
        if (st != RSI_OK) break;
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    if (st != RSI_OK) return st;
    cache_store(workload_key(inst, n_inst, prec), best, best_ms);
    return RSI_OK;
}

}  // extern "C"
