/*
 * rsi.h -- C ABI of librsi: the Rayleigh-Sommerfeld integral (RSI) quasi-Monte-Carlo
 * beam model on MI355X (gfx950).
 *
 * Paper: "Efficient numerical frameworks for modelling ultrasonic beams propagating
 * across interfaces" (Lello de Almeida, Png, Lan).  The library evaluates the QMC
 * estimator (eq. 16) of the piston integral (eq. 3) and of the interface integral
 * (eq. 7) at arbitrary field points, and chains them transducer -> interface 1 ->
 * ... -> field (Sec. 2.1; Sec. 2.2 for the interface count as the bottleneck).
 *
 * Conventions shared by every entry point
 *  - SI units; time dependence exp(-i omega t); the returned field is the velocity
 *    potential phi (v = grad phi); rsi_to_pressure gives p = i omega rho phi.
 *  - Complex numbers are interleaved (re, im) pairs of the stated precision.
 *  - Every array argument is a DEVICE pointer owned by the caller, unless the
 *    comment says "host".  Point sets are structure-of-arrays FP64.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null stream)
 *    and returns after enqueueing.  Calls on distinct streams may run concurrently.
 *    One-shot calls take their temporary workspace from the stream-ordered
 *    allocator (hipMallocAsync/hipFreeAsync) on `stream`; plans own theirs.
 *  - Errors are reported as rsi_status; no C++ exception crosses the ABI.  An
 *    argument error is detected before anything is enqueued.  n = 0 is valid and
 *    enqueues nothing (a zero-length output has nothing to write).
 *  - Precision: RSI_FP64 computes every operation in FP64 and excludes pairs closer
 *    than 1e-12 m, exactly as the FP64 reference does.  RSI_FP32 keeps FP64 for the
 *    per-target reference distance and the reduction of the phase k r to
 *    revolutions, and runs the per-pair arithmetic and the accumulation in FP32.  It
 *    does not test for close pairs (the kernel is singular on the radiating surface,
 *    Sec. 3.2; a test per pair costs 8 % of the single-frequency pair sum): the squared
 *    distance of a pair carries an absolute rounding error of a few 2^-24 s^2, with
 *    s = |P - C| + R (C the centre of the sources' bounding box, R its half diagonal),
 *    so the term of a source at distance r from field point P is off by about
 *    3e-7 (s/r)^2 relative.  Field points farther than 1e-3 s from every source get a
 *    finite value; nearer ones, and a field point on a source, may get a non-finite one.
 */
#ifndef RSI_H
#define RSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Every enum below carries two range markers (never valid arguments) so that its type
 * spans the whole int range: a C caller may pass any int where an enum is expected, and
 * the library then answers RSI_ERR_ARG (or "RSI_UNKNOWN_STATUS") with well-defined code. */
#define RSI_ENUM_RANGE_(prefix) prefix##RANGE_MIN_ = -2147483647 - 1, prefix##RANGE_MAX_ = 2147483647

typedef enum {
    RSI_OK = 0,
    RSI_ERR_NULL = 1,        /* a required pointer is NULL                          */
    RSI_ERR_ARG = 2,         /* a scalar argument is out of range (freq <= 0, ...)  */
    RSI_ERR_SIZE = 3,        /* a count is negative or exceeds a documented limit   */
    RSI_ERR_DEVICE = 4,      /* a HIP runtime call failed (message via last_error) */
    RSI_ERR_WORKSPACE = 5,   /* workspace allocation failed                         */
    RSI_ERR_NONFINITE = 6,   /* non-finite input (only with the finite check on)   */
    RSI_ERR_UNSUPPORTED = 7, /* the combination of options is not implemented       */
    RSI_ENUM_RANGE_(RSI_STATUS_)
} rsi_status;

typedef enum { RSI_MONOPOLE = 0, RSI_DIPOLE = 1, RSI_OMNI = 2, RSI_ENUM_RANGE_(RSI_KERNEL_) } rsi_kernel;
typedef enum { RSI_FP32 = 0, RSI_FP64 = 1, RSI_ENUM_RANGE_(RSI_PRECISION_) } rsi_precision;
typedef enum { RSI_T_GLOBAL = 0, RSI_T_LOCAL = 1, RSI_T_UNITY = 2, RSI_ENUM_RANGE_(RSI_TMODE_) } rsi_tmode;
typedef enum { RSI_SEQ_SOBOL = 0, RSI_SEQ_HALTON = 1, RSI_ENUM_RANGE_(RSI_SEQUENCE_) } rsi_sequence;

typedef struct { double c, rho; } rsi_medium;            /* m/s, kg/m^3             */

typedef struct {                                          /* device SoA, FP64, metres */
    const double *x, *y, *z;
    int64_t n;
} rsi_points;

typedef struct {                                          /* the radiating piston     */
    rsi_points pts;          /* face samples (eq. 18)                                */
    const double *w;         /* device quadrature weights (area / N, eq. 16)         */
    double v0;               /* normal velocity amplitude (eq. 3)                    */
    double centre[3];        /* face centre, for the incidence angles of RSI_T_*    */
    double axis[3];          /* unit beam axis (RSI_T_GLOBAL uses its inclination)  */
} rsi_transducer;

typedef struct {                                          /* one planar interface     */
    rsi_points pts;          /* samples on the plane z = `z` (eq. 17)                */
    const double *w;         /* device quadrature weights                            */
    double z;                /* plane depth; normal +z; planes strictly increasing   */
} rsi_interface;

/* One independent pair sum for rsi_propagate_batched / rsi_plan_create_batched. */
typedef struct {
    rsi_points src;          /* sources                                               */
    const double *w;         /* weights                                               */
    const double *vel;       /* complex FP64 strength per source, or NULL: all = v0   */
    double v0;               /* used when vel == NULL                                 */
    double normal[3];        /* dipole normal (ignored for RSI_MONOPOLE)              */
    rsi_points tgt;          /* field points                                          */
    rsi_medium medium;
    double freq;             /* Hz                                                    */
    rsi_kernel kind;
    void *out;               /* complex [tgt.n], FP32 or FP64 per the call's precision */
} rsi_instance;

typedef struct rsi_plan rsi_plan;                         /* opaque                   */

/* Human-readable status name; never NULL. */
const char *rsi_status_string(rsi_status s);

/* Text of the last HIP error seen by this thread (empty if none); never NULL. */
const char *rsi_last_error(void);

/* ABI version: (major << 16) | minor. */
int rsi_version(void);

/* Input check for debugging: with enable != 0 the pair-sum entry points (rsi_propagate,
 * rsi_propagate_ex, rsi_propagate_multifreq, rsi_propagate_noalloc, rsi_chain, rsi_chain_ex,
 * rsi_ray_field, rsi_propagate_batched and the plan constructors) scan their device inputs -- coordinates, weights, complex strengths,
 * interface samples, field points -- and return RSI_ERR_NONFINITE, launching nothing, if
 * any value is NaN or infinite.  The scan costs one pass over the inputs and a stream
 * synchronisation, so it is off by default and must not be used on a stream under graph
 * capture.  Setting the environment variable RSI_CHECK_FINITE=1 turns it on at load.
 * Process-wide; returns the previous setting. */
int rsi_set_check_finite(int enable);

/* ------------------------------------------------------------------------------
 * a1. Sampling (Sec. 2.3, eqs. 16-18).
 * ------------------------------------------------------------------------------ */

/* Scrambled two-dimensional Sobol points `first .. first+n-1` as uint32 pairs,
 * out[2i+d] = coordinate d.  Coordinate 0: van der Corput direction numbers;
 * coordinate 1: primitive polynomial x+1.  Each coordinate is Owen-scrambled by the
 * hash-based Laine-Karras permutation of Burley (JCGT 2020) with a per-coordinate
 * seed fmix32(seed + 0x9e3779b9 * (d + 1)) (MurmurHash3 finaliser).  The first 2^m
 * points of any seed form a (0, m, 2)-net.  Replaces the Halton sequence of Sec. 2.3.
 * out: device uint32[2n].  RSI_ERR_SIZE if first < 0, n < 0 or first + n > 2^32. */
rsi_status rsi_sobol2d(uint32_t seed, int64_t first, int64_t n, uint32_t *out, void *stream);

/* Piston face samples, eq. (18): radius a sqrt(u0), angle 2 pi u1 on the disc, the
 * disc tilted by `tilt` radians about +y (axis becomes (sin tilt, 0, cos tilt)) and
 * translated to centre (host double[3]).  w = pi a^2 / n.  Outputs: device
 * double[n] each.  RSI_ERR_ARG if radius <= 0. */
rsi_status rsi_sample_disc(uint32_t seed, int64_t n, double radius, const double *centre,
                           double tilt, double *x, double *y, double *z, double *w,
                           void *stream);

/* Interface patch samples, eq. (17): x = cx + h (2 u0 - 1), y = cy + h (2 u1 - 1),
 * z = z0, w = (2h)^2 / n.  RSI_ERR_ARG if half_width <= 0. */
rsi_status rsi_sample_square(uint32_t seed, int64_t n, double cx, double cy, double z0,
                             double half_width, double *x, double *y, double *z, double *w,
                             void *stream);

/* Halton points (the paper's sequence, Sec. 2.3) of indices first .. first+n-1:
 * out[2i+d] = radical inverse of the index in base 2 (d = 0) or 3 (d = 1), the integer
 * of mirrored digits over b^K rounded once (bit-identical to that fraction rounded to
 * FP64).  out: device double[2n].  RSI_ERR_SIZE unless 0 <= first, first + n <= 2^40. */
rsi_status rsi_halton2d(int64_t first, int64_t n, double *out, void *stream);

/* rsi_sample_disc / rsi_sample_square with a choice of sequence: RSI_SEQ_SOBOL (the
 * scrambled Sobol points of `seed`, identical to the functions above) or RSI_SEQ_HALTON
 * (Halton points of indices seed+1 .. seed+n: the origin point is skipped).
 * RSI_ERR_ARG for an unknown sequence. */
rsi_status rsi_sample_disc_ex(rsi_sequence seq, uint32_t seed, int64_t n, double radius,
                              const double *centre, double tilt, double *x, double *y, double *z,
                              double *w, void *stream);
rsi_status rsi_sample_square_ex(rsi_sequence seq, uint32_t seed, int64_t n, double cx, double cy,
                                double z0, double half_width, double *x, double *y, double *z,
                                double *w, void *stream);

/* Focused transducer (Sec. 3.3): n area-uniform samples on a spherical cap of aperture
 * radius `radius` and radius of curvature `curvature` (>= radius), apex at `centre`
 * (host double[3]), concave towards its axis (sin tilt, 0, cos tilt) so that the
 * geometric focus lies at centre + curvature * axis.  Height above the apex uniform in
 * u0, azimuth 2 pi u1; w = 2 pi R^2 (1 - cos a_max) / n with sin a_max = radius/R.
 * The cap radiates with eq. (3) like the flat piston (rsi_transducer.pts / .w).
 * RSI_ERR_ARG if radius <= 0 or curvature < radius. */
rsi_status rsi_sample_cap(rsi_sequence seq, uint32_t seed, int64_t n, double radius,
                          double curvature, const double *centre, double tilt, double *x, double *y,
                          double *z, double *w, void *stream);

/* Gaussian apodisation of a transducer (Sec. 4: the face velocity modulated by the
 * position of each source), folded into the quadrature weights: w[i] *= exp(-rho_i^2 /
 * width^2), rho_i the distance of sample i from the line through `centre` along `axis`
 * (host double[3] each; axis need not be unit).  w: device double[n], updated in place.
 * RSI_ERR_ARG if width <= 0 or axis = 0. */
rsi_status rsi_apodise(int64_t n, const double *x, const double *y, const double *z,
                       const double *centre, const double *axis, double width, double *w,
                       void *stream);

/* ------------------------------------------------------------------------------
 * a2. Interface transmission (eqs. 7, 8, 11, 15).
 * ------------------------------------------------------------------------------ */

/* Velocity-potential transmission coefficient at each sample of interface m
 * (1-based) of the stack `zif` (host double[m], planes z = zif[l], normal +z) with
 * media (host rsi_medium[m+1], medium 0 holds the transducer):
 *     T = 2 rho1 c2 cos a1 / (rho2 c2 cos a1 + rho1 c1 cos a2)        (eq. 11)
 *       = (rho1/rho2)(1 + R12)                                        (eqs. 7-8)
 * with sin a2 = (c2/c1) sin a1 (eq. 15) and cos a2 = +i sqrt(sin^2 a2 - 1) past the
 * critical angle.  The incidence angle a1 is, per tmode:
 *   RSI_T_GLOBAL: the inclination of `axis` (host double[3]) from +z, Snell-chained
 *                 through the layers above (one value per interface);
 *   RSI_T_LOCAL:  the angle of the refracted ray from `xc` (host double[3]) to the
 *                 sample, whose conserved slowness C solves
 *                 sum_l h_l C c_l / sqrt(1 - C^2 c_l^2) = horizontal distance
 *                 (eqs. 14-15; a straight line for m = 1);
 *   RSI_T_UNITY:  T = 1 (the impedance-matched display mode of Sec. 3.1).
 * qx, qy: device double[n] sample coordinates; out: device complex FP64 [n]. */
rsi_status rsi_transmission(rsi_tmode tmode, int m, const double *zif,
                            const rsi_medium *media, const double *xc, const double *axis,
                            int64_t n, const double *qx, const double *qy, double *out,
                            void *stream);

/* Velocity-potential reflection coefficient at each sample of interface m (eq. 8):
 *     R12 = (rho2 c2 cos a1 - rho1 c1 cos a2) / (rho2 c2 cos a1 + rho1 c1 cos a2),
 * same arguments, incidence angles and complex branch as rsi_transmission
 * (T = (rho1/rho2)(1 + R12) holds sample by sample); R = 0 for RSI_T_UNITY (the media
 * matched).  The reflected field of rsi_chain_ex(RSI_CHAIN_ABOVE) uses it. */
rsi_status rsi_reflection(rsi_tmode tmode, int m, const double *zif, const rsi_medium *media,
                          const double *xc, const double *axis, int64_t n, const double *qx,
                          const double *qy, double *out, void *stream);

/* ------------------------------------------------------------------------------
 * a3/a4. The pair sum (eqs. 3, 7; estimator eq. 16).
 * ------------------------------------------------------------------------------ */

/* phi(P_i) = -(1/2 pi) sum_j w_j s_j K(P_i, Q_j) for every target P_i, with
 *   RSI_MONOPOLE: K = e^{ikr}/r                                   (eq. 3, s = v0)
 *   RSI_DIPOLE:   K = cos(theta) (ik - 1/r) e^{ikr}/r,  cos(theta) = n.(P-Q)/r
 *                 (the first Rayleigh-Sommerfeld solution, eqs. 2 and 7, with the
 *                 overall sign that reproduces a field continued through a
 *                 transparent plane)
 *   RSI_OMNI:     K = ik e^{ikr}/r: an interface sample as an omnidirectional point
 *                 source, without the directivity cos(theta) and the near-field term
 *                 -1/r (the formulation Sec. 2.1 contrasts with eq. 2, attributed to
 *                 Zhang et al. 2022; kept for the ablation)
 * k = 2 pi freq / medium.c.  src_vel: device complex FP64 [src->n] (s_j, e.g.
 * T_j phi_in(Q_j)); normal: host double[3], required for RSI_DIPOLE (need not be
 * unit: it is normalised), ignored otherwise.  out: device complex [tgt->n] of the
 * call's precision (FP32: float pairs, FP64: double pairs), overwritten.
 * RSI_ERR_ARG if freq <= 0 or medium.c <= 0. */
rsi_status rsi_propagate(const rsi_points *src, const double *src_w, const double *src_vel,
                         const double *normal, const rsi_points *tgt, rsi_medium medium,
                         double freq, rsi_kernel kind, rsi_precision prec, void *out,
                         void *stream);

/* Flags of rsi_propagate_ex. */
enum {
    /* Every source has the same z (a horizontal interface patch).  The FP32 kernel then
     * drops the z terms of each pair; for RSI_DIPOLE the normal must be +-z.  Results
     * are unspecified if the sources do not share one z. */
    RSI_FLAG_PLANAR_Z = 1u
};

/* rsi_propagate with flags (a bitwise OR of RSI_FLAG_*; 0 is rsi_propagate).
 * RSI_ERR_ARG for unknown flags, or RSI_FLAG_PLANAR_Z with a dipole normal not
 * parallel to z.  FP64 ignores RSI_FLAG_PLANAR_Z (it evaluates every term). */
rsi_status rsi_propagate_ex(const rsi_points *src, const double *src_w, const double *src_vel,
                            const double *normal, const rsi_points *tgt, rsi_medium medium,
                            double freq, rsi_kernel kind, rsi_precision prec, uint32_t flags,
                            void *out, void *stream);

/* The pair sum of rsi_propagate_ex for many frequencies in one call (multi-frequency
 * superposition, Sec. 4): out[q][i] is phi at field point i for frequency freqs[q] (host
 * double[n_freq]) with the strengths src_vel[q][j] (device complex FP64 [n_freq][src->n],
 * frequency-major; NULL: 1 for every source and frequency); medium, kind, normal and flags
 * as in rsi_propagate_ex.  out: device complex [n_freq][tgt->n] of the call's precision.
 * With RSI_FP32 on a uniform grid (n_freq >= 2, f_q = f_0 + q df) and a monopole or
 * omnidirectional kernel, or a dipole with RSI_FLAG_PLANAR_Z (normal +z or -z), the call
 * is one multi-frequency launch: the pair geometry is evaluated once per block of 16 or
 * 32 frequencies and e^{ikr} is carried from one frequency to the next; every other case
 * (RSI_FP64, a non-uniform list, a dipole with any other normal) runs one pair sum per
 * frequency.  Errors: those of rsi_propagate_ex; RSI_ERR_ARG for a frequency <= 0 or not
 * finite; RSI_ERR_NULL for freqs == NULL with n_freq > 0; RSI_ERR_SIZE for n_freq < 0 or
 * n_freq * tgt->n > 2^38.  n_freq = 0 enqueues nothing. */
rsi_status rsi_propagate_multifreq(const rsi_points *src, const double *src_w,
                                   const double *src_vel, const double *normal,
                                   const rsi_points *tgt, rsi_medium medium, const double *freqs,
                                   int n_freq, rsi_kernel kind, rsi_precision prec, uint32_t flags,
                                   void *out, void *stream);

/* Size in bytes of the fixed device array that rsi_propagate_noalloc works in. */
#define RSI_NOALLOC_SCRATCH_BYTES (64LL << 20)

/* rsi_propagate_ex for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Arguments, results,
 * argument errors and the finite check are those of rsi_propagate_ex; the caller still
 * passes the inputs and the output.  The call allocates and frees nothing: its workspace
 * comes from one file-scope device array of RSI_NOALLOC_SCRATCH_BYTES (64 MiB) inside
 * the library, one copy per device, reserved when the library's code is loaded on that
 * device and held until the process ends.  Workspace, in 256-byte aligned pieces:
 *   FP32: 256 (finite-check flag) + 256 (anchor) + 3072 (extents) + 32 n_src (records)
 *         + 8 n_tgt per source split (partial sums);
 *   FP64: 256 (flag) + 64 n_src (records) + 16 n_tgt per source split.
 * When the partial sums of rsi_propagate_ex's launch would not fit, the call uses fewer
 * source splits (down to one, which needs none), so its results may differ from
 * rsi_propagate_ex's by rounding only.  RSI_ERR_SIZE, before anything is enqueued and
 * with rsi_last_error giving the sizes, if the records alone do not fit: more than
 * 2,097,040 sources in FP32 or 1,048,572 in FP64.
 * Every call on one device shares that device's array, and each call overwrites what the
 * previous one left there (nothing in it is assumed to start at zero).  Calls on one
 * stream are ordered and therefore safe; calls that overlap in time on one device (other
 * streams, other host threads, graphs replayed concurrently) race on the array and give
 * wrong results. */
rsi_status rsi_propagate_noalloc(const rsi_points *src, const double *src_w,
                                 const double *src_vel, const double *normal,
                                 const rsi_points *tgt, rsi_medium medium, double freq,
                                 rsi_kernel kind, rsi_precision prec, uint32_t flags, void *out,
                                 void *stream);

/* ------------------------------------------------------------------------------
 * a5. The chain (Sec. 2.1 repeated per interface, Sec. 3.4-3.5).
 * ------------------------------------------------------------------------------ */

/* For every frequency f of `freqs` (host double[n_freq]):
 *   phi_0 = monopole sum from the transducer (strength v0) onto interface 1;
 *   for m = 1..n_if: s_j = T_m(Q_j) phi_{m-1}(Q_j) (rsi_transmission with `tmode`),
 *     phi_m = dipole sum (normal +z, medium m) onto interface m+1, or onto `tgt`
 *     after the last interface.
 * n_if = 0 radiates the transducer straight onto tgt.  media: host rsi_medium
 * [n_if+1]; ifaces: host array of n_if descriptors with strictly increasing z.
 * out: device complex [n_freq][tgt->n] of the call's precision (FP32 chains keep
 * their interface fields in FP32).  With RSI_FP32 and n_freq > 1 on a uniform
 * frequency grid, each stage runs as one multi-frequency launch that evaluates the
 * pair geometry once and advances e^{ikr} across the frequencies by complex
 * rotation. */
rsi_status rsi_chain(const rsi_transducer *xd, const rsi_interface *ifaces, int n_if,
                     const rsi_medium *media, const rsi_points *tgt, const double *freqs,
                     int n_freq, rsi_tmode tmode, rsi_precision prec, void *out,
                     void *stream);

/* Flags of rsi_chain_ex and rsi_plan_create_chain_ex. */
enum {
    /* Interface samples radiate with RSI_OMNI instead of RSI_DIPOLE (the ablation of
     * the dipole and directivity terms, Sec. 2.1). */
    RSI_CHAIN_OMNI = 1u,
    /* The field points lie in medium n_if - 1, above the last interface (n_if >= 1).
     * out = incident + reflected field there: the incident field is the chain through
     * interfaces 1..n_if-1 evaluated at the points (the transducer's own field for
     * n_if = 1); the reflected field radiates the boundary values R(Q_j) phi_inc(Q_j)
     * of the last interface (rsi_reflection with `tmode`; the approximation
     * phi_r = R12 phi_i that also yields eq. 7) back into medium n_if - 1, i.e. the
     * interface kernel with normal -z (eqs. 4-5).  With the fields below the
     * interface from rsi_chain, p = i omega rho phi on both sides gives the pressure
     * continuity of eq. 6. */
    RSI_CHAIN_ABOVE = 2u
};

/* rsi_chain with flags (a bitwise OR of RSI_CHAIN_*; 0 is rsi_chain).  RSI_ERR_ARG
 * for unknown flags or RSI_CHAIN_ABOVE with n_if = 0. */
rsi_status rsi_chain_ex(const rsi_transducer *xd, const rsi_interface *ifaces, int n_if,
                        const rsi_medium *media, const rsi_points *tgt, const double *freqs,
                        int n_freq, rsi_tmode tmode, rsi_precision prec, uint32_t flags,
                        void *out, void *stream);

/* ------------------------------------------------------------------------------
 * Ray tracing (Sec. 2.2): the single-surface-integral model.
 * ------------------------------------------------------------------------------ */

/* For every frequency f of `freqs` (host double[n_freq]) and every field point P:
 *   phi(P) = -(v0 / 2 pi) sum_j w_j T_j e^{i 2 pi f t_j} / A_j      (eq. 12 under eq. 16)
 * over the transducer samples Q_j of `xd` alone: no interface is sampled.  The ray
 * from Q_j to P crosses the planes z = zif[0] < ... < zif[n_if-1] (host double[n_if],
 * normal +z; layer l = 0..n_if is media[l], host rsi_medium[n_if+1]) with the
 * horizontal slowness C that solves eq. (14) through the stack,
 *   sum_l h_l C / sqrt(S_l^2 - C^2) = |P - Q_j| (horizontal),   S_l = 1 / c_l,
 * h_l its vertical extent in layer l (h_0 = zif[0] - z_j, h_last = z_P - zif[n_if-1]).
 * With eta_l = sqrt(S_l^2 - C^2) (c_l eta_l = cos theta_l, eq. 15):
 *   t_j = C rho + sum_l h_l eta_l, the travel time (phase sum_l k_l D_l);
 *   A_j = eta_0 sqrt((sum_l h_l / eta_l)(sum_l h_l S_l^2 / eta_l^3)), eq. (12)'s
 *         spreading, extended to several planes by the stationary-phase evaluation
 *         of the layered angular spectrum (eq. 10);
 *   T_j = prod over the planes of eq. (11) at the ray's angles (real: a ray is never
 *         past a critical angle).
 * Pairs whose sample is on or below the first plane, or whose field point is on or
 * above the last plane, contribute nothing.  n_if = 0: one medium, where eq. (12) is
 * eq. (3) (the monopole pair sum of rsi_propagate).  xd->centre and xd->axis are not
 * used.  out: device complex [n_freq][tgt->n] of the call's precision.
 * Precision: RSI_FP64 solves every root to the last bit by Newton's method inside a
 * bisection bracket.  RSI_FP32 computes per field point, in FP64, the ray from the
 * centre of the samples' bounding box and its phase in revolutions; per pair it solves
 * the root by Newton's method in FP32 from that ray and forms the travel-time
 * difference to it in a cancellation-free form, so the large part of the phase never
 * passes through FP32.  Errors: RSI_ERR_SIZE for n_if > 8 or negative counts;
 * RSI_ERR_ARG for media with c or rho <= 0, planes not strictly increasing, a
 * frequency <= 0 or non-finite values. */
rsi_status rsi_ray_field(const rsi_transducer *xd, const double *zif, int n_if,
                         const rsi_medium *media, const rsi_points *tgt, const double *freqs,
                         int n_freq, rsi_precision prec, void *out, void *stream);

/* ------------------------------------------------------------------------------
 * a7. Batching: persistent launches, plans and graph replay.
 * ------------------------------------------------------------------------------ */

/* Evaluate n_inst independent pair sums (host rsi_instance[n_inst]) in ONE
 * persistent launch: the work is cut into (instance, target tile, source chunk)
 * items sorted by cost, pulled from a device work counter, and reduced per target in
 * a fixed order (bitwise repeatable).  Tile shapes come from the autotune cache when
 * it holds an entry for this workload, otherwise from built-in defaults. */
rsi_status rsi_propagate_batched(const rsi_instance *inst, int n_inst, rsi_precision prec,
                                 void *stream);

/* Plans: the whole chain (or batched launch) with its workspace allocated once and
 * its kernels captured into a hipGraph; rsi_plan_execute replays the graph on
 * `stream`.  The plan binds the device pointers given at creation (inputs and
 * output) -- their contents may change between executions, their addresses may not.
 * A plan may be executed on one stream at a time. */
rsi_status rsi_plan_create_chain(rsi_plan **plan, const rsi_transducer *xd,
                                 const rsi_interface *ifaces, int n_if,
                                 const rsi_medium *media, const rsi_points *tgt,
                                 const double *freqs, int n_freq, rsi_tmode tmode,
                                 rsi_precision prec, void *out);
rsi_status rsi_plan_create_chain_ex(rsi_plan **plan, const rsi_transducer *xd,
                                    const rsi_interface *ifaces, int n_if,
                                    const rsi_medium *media, const rsi_points *tgt,
                                    const double *freqs, int n_freq, rsi_tmode tmode,
                                    rsi_precision prec, uint32_t flags, void *out);
rsi_status rsi_plan_create_batched(rsi_plan **plan, const rsi_instance *inst, int n_inst,
                                   rsi_precision prec);
rsi_status rsi_plan_execute(rsi_plan *plan, void *stream);
rsi_status rsi_plan_destroy(rsi_plan *plan);

/* Time the candidate tile shapes (targets per lane, split-K chunk) of the batched
 * launch for this instance list on the current device and store the fastest in the
 * autotune cache (file named by RSI_AUTOTUNE_CACHE, else ~/.cache/rsi_autotune.txt).
 * Synchronises the device; overwrites every inst[i].out.  A missing or corrupt cache
 * file is treated as empty. */
rsi_status rsi_autotune_batched(const rsi_instance *inst, int n_inst, rsi_precision prec);

/* ------------------------------------------------------------------------------
 * a8. Output.
 * ------------------------------------------------------------------------------ */

/* p = i omega rho phi with omega = 2 pi freq; phi and p: device complex [n] of the
 * given precision (may alias). */
rsi_status rsi_to_pressure(int64_t n, const void *phi, rsi_precision prec, double rho,
                           double freq, void *p, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RSI_H */
