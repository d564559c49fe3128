/*
 * HVOX reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct FP64 evaluation of the two sums the HVOX
 * method approximates (HVOX paper, Sect. 2, Eqs. 2 and 3, with unit
 * tesselation weights and the 2*pi convention for wavelength-normalised
 * baselines):
 *
 *   synthesis (sky -> vis):  V_k = sum_n I_n exp(-2 pi i <p_k, r_n>)
 *   analysis  (vis -> sky):  I_n = sum_k V_k exp(+2 pi i <p_k, r_n>)
 *
 * Direct evaluation costs O(N_vis * N_pix) (Sect. 2); it is the ground truth
 * the paper's accuracy study compares against (Sect. 5.2).
 *
 * Only the tests, the package's smoke check and the benchmark's CPU-baseline
 * leg may load this library.  It shares no code with the GPU library.
 *
 * Numerics:
 *  - the phase <p, r> is a compensated dot product (Dot2 of Ogita, Rump and
 *    Oishi 2005: error-free products and sums), reduced modulo 1 in
 *    double-double before cos/sin from libm, so arguments of 1e5 cycles keep
 *    ~1e-16 absolute phase accuracy;
 *  - sums use Neumaier compensated summation;
 *  - one output per OpenMP iteration: no atomics, deterministic.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <omp.h>

#define TWO_PI 6.283185307179586476925286766559

/* Test hook: deliberately wrong variants so that tests can show that the
 * oracle's pins detect plausible mistakes.  0 = correct. */
enum {
    FAULT_NONE = 0,
    FAULT_SIGN = 1,        /* exponent sign flipped                      */
    FAULT_NO_TWO_PI = 2,   /* exp(-i pi <p,r>) instead of exp(-2 pi i ..)  */
    FAULT_SWAP_XY = 3,     /* u paired with y, v with x (transposed use) */
    FAULT_DROP_LAST = 4,   /* last summand dropped                        */
    FAULT_NO_CONJ = 5      /* analysis uses the synthesis sign           */
};
static int g_fault = FAULT_NONE;

int hvox_oracle_set_fault(int kind) { int old = g_fault; g_fault = kind; return old; }

int hvox_oracle_max_threads(void) { return omp_get_max_threads(); }

static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static inline void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* fractional part in [-1/2, 1/2] of <p, r>, accurate to ~1e-16 absolute */
static double phase_frac(const double *p, const double *r)
{
    double a = p[0], b = p[1], c = p[2];
    if (g_fault == FAULT_SWAP_XY) { a = p[1]; b = p[0]; }
    double s, err, h, e, q;
    two_prod(a, r[0], &s, &err);
    two_prod(b, r[1], &h, &e);
    two_sum(s, h, &s, &q);
    err += q + e;
    two_prod(c, r[2], &h, &e);
    two_sum(s, h, &s, &q);
    err += q + e;
    double n = nearbyint(s);
    double f = (s - n) + err;          /* s - n is exact */
    f -= nearbyint(f);
    return f;
}

typedef struct { double re, im, cre, cim; } nsum;

static inline void nsum_add(nsum *acc, double x, double y)
{
    double t = acc->re + x;
    if (fabs(acc->re) >= fabs(x)) acc->cre += (acc->re - t) + x; else acc->cre += (x - t) + acc->re;
    acc->re = t;
    t = acc->im + y;
    if (fabs(acc->im) >= fabs(y)) acc->cim += (acc->im - t) + y; else acc->cim += (y - t) + acc->im;
    acc->im = t;
}

/* One output of sum_j c_j exp(sgn 2 pi i <a_out, b_j>) */
static void one_output(const double *a_out, const double *b, int64_t nb,
                       const double *c /* complex interleaved [nb] */,
                       double sgn, double *out)
{
    nsum acc = {0.0, 0.0, 0.0, 0.0};
    double scale = (g_fault == FAULT_NO_TWO_PI) ? 0.5 * TWO_PI : TWO_PI;
    int64_t n_end = (g_fault == FAULT_DROP_LAST && nb > 0) ? nb - 1 : nb;
    for (int64_t j = 0; j < n_end; ++j) {
        double f = phase_frac(a_out, b + 3 * j);
        double ang = sgn * scale * f;
        double cs = cos(ang), sn = sin(ang);
        double xr = c[2 * j], xi = c[2 * j + 1];
        nsum_add(&acc, xr * cs - xi * sn, xr * sn + xi * cs);
    }
    out[0] = acc.re + acc.cre;
    out[1] = acc.im + acc.cim;
}

/*
 * V[t][r] = sum_n I[t][n] exp(-2 pi i <uvw[rows[r]], xyz[n]>)
 * uvw: [n_vis][3], xyz: [n_pix][3], I: complex [ntrans][n_pix],
 * rows: NULL (all n_vis outputs) or nrows indices into [0, n_vis).
 * V: complex [ntrans][nrows or n_vis].  Returns 0, or -1 on bad arguments.
 */
int hvox_oracle_synthesis(const double *uvw, int64_t n_vis,
                          const double *xyz, int64_t n_pix,
                          const double *I, int32_t ntrans,
                          const int64_t *rows, int64_t nrows, double *V)
{
    if (!uvw || !xyz || !I || !V || n_vis < 0 || n_pix < 0 || ntrans < 1) return -1;
    int64_t nout = rows ? nrows : n_vis;
    double sgn = (g_fault == FAULT_SIGN) ? +1.0 : -1.0;
    for (int64_t r = 0; r < nout; ++r)
        if (rows && (rows[r] < 0 || rows[r] >= n_vis)) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nout; ++r) {
        int64_t k = rows ? rows[r] : r;
        for (int32_t t = 0; t < ntrans; ++t)
            one_output(uvw + 3 * k, xyz, n_pix, I + 2 * (int64_t)t * n_pix, sgn,
                       V + 2 * ((int64_t)t * nout + r));
    }
    return 0;
}

/*
 * Ipix[t][r] = sum_k V[t][k] exp(+2 pi i <uvw[k], xyz[rows[r]]>)
 * Same layout conventions as hvox_oracle_synthesis with roles swapped.
 */
int hvox_oracle_analysis(const double *uvw, int64_t n_vis,
                         const double *xyz, int64_t n_pix,
                         const double *V, int32_t ntrans,
                         const int64_t *rows, int64_t nrows, double *Ipix)
{
    if (!uvw || !xyz || !V || !Ipix || n_vis < 0 || n_pix < 0 || ntrans < 1) return -1;
    int64_t nout = rows ? nrows : n_pix;
    double sgn = (g_fault == FAULT_SIGN || g_fault == FAULT_NO_CONJ) ? -1.0 : +1.0;
    for (int64_t r = 0; r < nout; ++r)
        if (rows && (rows[r] < 0 || rows[r] >= n_pix)) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nout; ++r) {
        int64_t n = rows ? rows[r] : r;
        for (int32_t t = 0; t < ntrans; ++t)
            one_output(xyz + 3 * n, uvw, n_vis, V + 2 * (int64_t)t * n_vis, sgn,
                       Ipix + 2 * ((int64_t)t * nout + r));
    }
    return 0;
}
