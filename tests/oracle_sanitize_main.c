/*
 * Driver for the reference library under the sanitizers (test infrastructure): calls every
 * entry point of oracle/rsi_oracle.c on small inputs -- sampling, apodisation, the three
 * pair-sum kinds, transmission and reflection, the chain in each mode, the ray model --
 * and checks return codes and that every output is finite.  Built and run by
 * tests/test_oracle_sanitize.py with AddressSanitizer + UndefinedBehaviorSanitizer and
 * with ThreadSanitizer (OpenMP threads).  Prints "ok" on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_sobol2d(uint32_t seed, int64_t first, int64_t n, uint32_t *out);
int orc_halton2d(int64_t first, int64_t n, double *out);
int orc_sample_disc_ex(int seq, uint32_t seed, int64_t n, double radius, const double centre[3],
                       double tilt, double *x, double *y, double *z, double *w);
int orc_sample_square_ex(int seq, uint32_t seed, int64_t n, double cx, double cy, double z0,
                         double half_width, double *x, double *y, double *z, double *w);
int orc_sample_cap(int seq, uint32_t seed, int64_t n, double radius, double curvature,
                   const double centre[3], double tilt, double *x, double *y, double *z,
                   double *w);
int orc_apodise(int64_t n, const double *x, const double *y, const double *z,
                const double centre[3], const double axis[3], double width, double *w);
int orc_propagate(int kind, int64_t n_src, const double *sx, const double *sy,
                  const double *sz, const double *sw, const double *s, const double *normal,
                  int64_t n_tgt, const double *tx, const double *ty, const double *tz, double c,
                  double freq, double *out);
int orc_transmission(int tmode, int m, const double *zif, const double *c, const double *rho,
                     const double xc[3], const double axis[3], int64_t n, const double *qx,
                     const double *qy, double *out);
int orc_reflection(int tmode, int m, const double *zif, const double *c, const double *rho,
                   const double xc[3], const double axis[3], int64_t n, const double *qx,
                   const double *qy, double *out);
int orc_chain_ex(int64_t n_xd, const double *xx, const double *xy, const double *xz,
                 const double *xw, double v0, const double xc[3], const double axis[3],
                 int n_if, const int64_t *n_q, const double *const *qx,
                 const double *const *qy, const double *const *qz,
                 const double *const *qw, const double *zif, const double *c,
                 const double *rho, int64_t n_tgt, const double *tx, const double *ty,
                 const double *tz, int n_freq, const double *freqs, int tmode, int flags,
                 double *out);
int orc_ray_field(int64_t n_xd, const double *xx, const double *xy, const double *xz,
                  const double *xw, double v0, int n_if, const double *zif, const double *c,
                  const double *rho, int64_t n_tgt, const double *tx, const double *ty,
                  const double *tz, int n_freq, const double *freqs, double *out);

static int failures = 0;

static void expect(int cond, const char *what) {
    if (!cond) {
        printf("FAILED: %s\n", what);
        ++failures;
    }
}

static void expect_finite(const double *a, int64_t n, const char *what) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) {
            printf("FAILED: %s[%ld] not finite\n", what, (long)i);
            ++failures;
            return;
        }
}

static double *alloc(int64_t n) {
    double *p = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!p) exit(2);
    return p;
}

int main(void) {
    enum { NX = 257, NQ = 301, NT = 67, NF = 3 };
    const double zero[3] = {0.0, 0.0, 0.0}, axis[3] = {0.0, 0.0, 1.0};
    const double tilt = 0.15, a = 6.35e-3;

    uint32_t *sob = malloc(sizeof(uint32_t) * 2 * NX);
    double *hal = alloc(2 * NX);
    expect(orc_sobol2d(7, 11, NX, sob) == 0, "sobol2d");
    expect(orc_halton2d(3, NX, hal) == 0, "halton2d");
    expect_finite(hal, 2 * NX, "halton2d");

    double *xx = alloc(NX), *xy = alloc(NX), *xz = alloc(NX), *xw = alloc(NX);
    expect(orc_sample_disc_ex(0, 1, NX, a, zero, tilt, xx, xy, xz, xw) == 0, "sample_disc");
    expect(orc_sample_disc_ex(1, 1, NX, a, zero, tilt, xx, xy, xz, xw) == 0, "sample_disc halton");
    double *cx = alloc(NX), *cy = alloc(NX), *cz = alloc(NX), *cw = alloc(NX);
    expect(orc_sample_cap(0, 2, NX, a, 0.033, zero, 0.0, cx, cy, cz, cw) == 0, "sample_cap");
    expect(orc_apodise(NX, cx, cy, cz, zero, axis, a, cw) == 0, "apodise");
    expect_finite(cw, NX, "apodise");

    const double zif[2] = {0.02, 0.022};
    const double c[3] = {1480.0, 5900.0, 2700.0}, rho[3] = {1000.0, 7800.0, 2700.0};
    double *qx[2], *qy[2], *qz[2], *qw[2];
    int64_t nq[2] = {NQ, NQ - 17};
    for (int m = 0; m < 2; ++m) {
        qx[m] = alloc(NQ); qy[m] = alloc(NQ); qz[m] = alloc(NQ); qw[m] = alloc(NQ);
        expect(orc_sample_square_ex(0, 3 + m, nq[m], 0.004, 0.0, zif[m], 0.012, qx[m], qy[m], qz[m],
                                    qw[m]) == 0, "sample_square");
    }
    double *tco = alloc(2 * NQ), *rco = alloc(2 * NQ);
    for (int tmode = 0; tmode < 3; ++tmode) {
        expect(orc_transmission(tmode, 2, zif, c, rho, zero, axis, nq[1], qx[1], qy[1], tco) == 0,
               "transmission");
        expect(orc_reflection(tmode, 1, zif, c, rho, zero, axis, nq[0], qx[0], qy[0], rco) == 0,
               "reflection");
        expect_finite(tco, 2 * nq[1], "transmission");
        expect_finite(rco, 2 * nq[0], "reflection");
    }

    double *tx = alloc(NT), *ty = alloc(NT), *tz = alloc(NT);
    for (int i = 0; i < NT; ++i) {
        tx[i] = 0.004 + 1e-4 * (i % 13);
        ty[i] = -2e-3 + 5e-5 * i;
        tz[i] = 0.03 + 1e-4 * (i % 7);
    }
    double *s = alloc(2 * NX), *out = alloc(2 * NT * NF);
    for (int j = 0; j < NX; ++j) {
        s[2 * j] = cos(0.1 * j);
        s[2 * j + 1] = sin(0.1 * j);
    }
    for (int kind = 0; kind < 3; ++kind) {
        expect(orc_propagate(kind, NX, xx, xy, xz, xw, s, axis, NT, tx, ty, tz, 1480.0, 2.0e6, out) == 0,
               "propagate");
        expect_finite(out, 2 * NT, "propagate");
    }

    const double freqs[NF] = {1.0e6, 2.0e6, 3.0e6};
    for (int flags = 0; flags < 4; ++flags) {
        const double *tzs = tz;
        double *above = NULL;
        if (flags & 2) {  /* reflected field: points above the last plane */
            above = alloc(NT);
            for (int i = 0; i < NT; ++i) above[i] = 0.019 - 1e-4 * (i % 5);
            tzs = above;
        }
        expect(orc_chain_ex(NX, xx, xy, xz, xw, 1.0, zero, axis, (flags & 2) ? 1 : 2, nq,
                            (const double *const *)qx, (const double *const *)qy,
                            (const double *const *)qz, (const double *const *)qw, zif, c, rho, NT, tx,
                            ty, tzs, NF, freqs, 1, flags, out) == 0, "chain_ex");
        expect_finite(out, 2 * NT * NF, "chain_ex");
        free(above);
    }

    expect(orc_ray_field(NX, xx, xy, xz, xw, 1.0, 2, zif, c, rho, NT, tx, ty, tz, NF, freqs, out) == 0,
           "ray_field");
    expect_finite(out, 2 * NT * NF, "ray_field");

    free(sob); free(hal); free(xx); free(xy); free(xz); free(xw);
    free(cx); free(cy); free(cz); free(cw);
    for (int m = 0; m < 2; ++m) { free(qx[m]); free(qy[m]); free(qz[m]); free(qw[m]); }
    free(tco); free(rco); free(tx); free(ty); free(tz); free(s); free(out);
    if (failures) return 1;
    printf("ok\n");
    return 0;
}
