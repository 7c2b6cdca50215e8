/*
 * sincos_oracle.c -- CPU oracle for the single-precision sine-cosine pair of
 * M. H. Mendenhall, "A Fast, Vectorizable Algorithm for Producing
 * Single-Precision Sine-Cosine Pairs" (2004).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU library
 * shares no code, header, table or constant with it; its constants are typed
 * here again from the paper's decimals.
 *
 * The method as Sec. II states it, and as this file computes it, one element
 * at a time, in binary32 with round-to-nearest and IEEE subnormals:
 *
 *   Reduction.  The angle theta is multiplied by 1/(2 pi) and reduced modulo
 *   1 by rounding to the nearest integer and subtracting, which leaves the
 *   fraction of a turn x in [-1/2, 1/2] (the subtraction is exact).
 *
 *   Series.  Power series give the sine and the cosine of a quarter of the
 *   reduced angle, 2 pi x / 4: an odd polynomial in x for the sine, an even
 *   one for the cosine, both evaluated by Horner's rule in x^2.  The first
 *   method's coefficients are a least-squares fit of sine and cosine, the
 *   second method's a fit of the angle alone (Sec. II, two coefficient sets).
 *
 *   Doubling.  Two angle doublings with eq. (1), sin 2u = 2 sin u cos u and
 *   cos 2u = cos^2 u - sin^2 u, carry the quarter angle to the whole circle.
 *   The stability analysis of Sec. II shows what one doubling does to a pair
 *   with magnitude a and angle error d: (a sin(u+d), a cos(u+d)) becomes
 *   (a^2 sin 2(u+d), a^2 cos 2(u+d)).  The relative angle error survives
 *   unchanged; only the magnitude is squared.  (The rejected eq. (2) uses
 *   cos 2u = 1 - 2 sin^2 u instead, which gives a^2 cos 2(u+d) + (1 - a^2):
 *   the magnitude error leaks into the angle.  It is kept as an ablation.)
 *
 *   Magnitude.  After n doublings the magnitude is a^(2^n).  The magnitude
 *   squared of the pair before the last doubling is that same number, so
 *   with |p|^2 = 1 + e read there, the final pair is rescaled by 1/(1 + e):
 *   to first order 1 - e = 2 - |p|^2 (first method, whose series keep e
 *   tiny), or the exact reciprocal 1/|p|^2 (second method, whose series do
 *   not).  Reading the factor one doubling early lets it be formed beside
 *   the last doubling instead of after it; the paper's sample implementation
 *   (Fig. 1) does the same, and the accuracy figures printed in Sec. II,
 *   which the tests pin, come from it.  The text's own form, (3 - s^2 - c^2)
 *   / 2 on the final pair, agrees to first order in e and is an ablation.
 *
 * Two arithmetic modes, selected per call:
 *   ORACLE_FUSED  every product that feeds a sum is fused into it, one
 *                 rounding (C99 fmaf), as on the paper's vector unit, which
 *                 has only fused multiply-add.  In a sum of two products
 *                 (c^2 - s^2, 2 - c^2 - s^2, s^2 + c^2) the cosine's square
 *                 is the inner term: rounded on its own in c^2 - s^2 and
 *                 s^2 + c^2, fused with the 2 in 2 - c^2 - s^2; the sine's
 *                 square is fused last.  This is the placement of Fig. 1,
 *                 the one the printed accuracy figures were measured with.
 *   ORACLE_SPLIT  the same expressions with every product and every sum
 *                 rounded on its own.  This file must be compiled with
 *                 -ffp-contract=off so that the compiler fuses nothing.
 *
 * Readings where the paper leaves a choice open:
 *   - A vector unit without a plain multiply writes a product as a
 *     multiply-add with a +0.0 addend.  Here a product is a product.  The
 *     two differ only in the sign of an exact-zero result; the reduced angle
 *     below is never -0 (x - rint(x) with round-to-nearest gives +0), so the
 *     pair is the same.
 *   - rint() rounds ties to even, as the vector unit's round does; the
 *     reduced angle lies in [-1/2, 1/2].
 *   - The negative multiply-subtract c - a*b is IEEE fusedMultiplyAdd(-a,b,c)
 *     in the fused mode; its exact-zero result is +0.
 *   - Method 2's coefficient ss2 is the value printed in the text of Sec. II
 *     (-0.6466386936); Fig. 1's -0.6466386396 is taken as a typo.
 *   - Method 2's reciprocal is the correctly rounded 1.0f / d.
 *   - Inputs with |theta| >= 2^23 / (1/(2 pi)) reduce to x = 0 and give
 *     (0, 1); +-Inf and NaN give (NaN, NaN).  Nothing special-cases them.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared
 *        -pthread sincos_oracle.c -lm
 */
#define _GNU_SOURCE
#include <fenv.h>
#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_FUSED 0
#define ORACLE_SPLIT 1
#define ORACLE_METHOD1 0 /* normalized least-squares series + 2 - |p|^2 fix */
#define ORACLE_METHOD2 1 /* arctan-fit series + reciprocal of |p|^2 */

/* ---------------------------------------------------------------------- */
/* Constants: the paper's decimals, each read as a C double and rounded to
 * binary32 once.                                                           */

static float reduction_constant(void)
{
    /* 1/(2 pi) with pi written to ten decimals, as the paper writes it. */
    return (float)(1.0 / (2.0 * 3.1415926536));
}

struct series_coeffs {
    float ss1, ss2, ss3, ss4; /* sin(pi x / 2) = x (ss1 + ss2 x^2 + ss3 x^4 + ss4 x^6) */
    float cc1, cc2, cc3;      /* cos(pi x / 2) = 1 + cc1 x^2 + cc2 x^4 + cc3 x^6       */
};

static struct series_coeffs method_coeffs(int method)
{
    struct series_coeffs k;
    if (method == ORACLE_METHOD2) {
        /* Sec. II, second method: fit of the angle, not of the magnitude. */
        k.ss1 = (float)1.5707963268;
        k.ss2 = (float)-0.6466386936;
        k.ss3 = (float)0.0679105987;
        k.ss4 = (float)-0.0011573807;
        k.cc1 = (float)-1.2341299769;
        k.cc2 = (float)0.2465220241;
        k.cc3 = (float)-0.0123926179;
    } else {
        /* Sec. II, first method: least-squares series of sin and cos. */
        k.ss1 = (float)1.5707963235;
        k.ss2 = (float)-0.645963615;
        k.ss3 = (float)0.0796819754;
        k.ss4 = (float)-0.0046075748;
        k.cc1 = (float)-1.2336977925;
        k.cc2 = (float)0.2536086171;
        k.cc3 = (float)-0.0204391631;
    }
    return k;
}

/* ---------------------------------------------------------------------- */
/* The two ways of evaluating a*b + c and c - a*b.                          */

static float mul_add(float a, float b, float c, int arith)
{
    if (arith == ORACLE_FUSED)
        return fmaf(a, b, c);
    float p = a * b;
    return p + c;
}

static float mul_sub_from(float a, float b, float c, int arith)
{
    if (arith == ORACLE_FUSED)
        return fmaf(-a, b, c);
    float p = a * b;
    return c - p;
}

/* Horner's rule in x2 over coef[0..n-1], highest power first:
 * coef[0] + coef[1] x2 + ... + coef[n-1] x2^(n-1).                         */
static float horner(float x2, const float *coef, int n, int arith)
{
    float p = coef[n - 1];
    for (int k = n - 2; k >= 0; k--)
        p = mul_add(x2, p, coef[k], arith);
    return p;
}

/* ---------------------------------------------------------------------- */
/* Reduction (Sec. II): the fraction of a turn, theta / (2 pi) less the
 * nearest integer.  The subtraction is exact (Sterbenz), so both arithmetic
 * modes agree.                                                             */
float oracle_reduce(float theta)
{
    float turns = theta * reduction_constant();
    float whole = rintf(turns);
    return turns - whole;
}

/* Series (Sec. II polynomials): *s ~ sin(pi x / 2), *c ~ cos(pi x / 2) for
 * the reduced angle x.                                                     */
void oracle_quarter_series(float x, int arith, int method, float *s, float *c)
{
    struct series_coeffs k = method_coeffs(method);
    const float sin_coef[4] = {k.ss1, k.ss2, k.ss3, k.ss4};
    const float cos_coef[4] = {1.0f, k.cc1, k.cc2, k.cc3};
    float x2 = x * x;
    *s = x * horner(x2, sin_coef, 4, arith);
    *c = horner(x2, cos_coef, 4, arith);
}

/* eq. (1): sin 2u = 2 sin u cos u, cos 2u = cos^2 u - sin^2 u.  The sine's
 * product is rounded before it is doubled (doubling a rounded product is
 * exact; rounding 2s * c instead would differ among subnormals).           */
void oracle_double_angle(float s, float c, int arith, float *s_out, float *c_out)
{
    float cos_sq = c * c;
    *c_out = mul_sub_from(s, s, cos_sq, arith);
    float sin_cos = s * c;
    *s_out = 2.0f * sin_cos;
}

/* The rejected eq. (2): sin 2u = 2 sin u cos u, cos 2u = 1 - 2 sin^2 u
 * (ablation only).                                                         */
void oracle_double_angle_eq2(float s, float c, int arith, float *s_out, float *c_out)
{
    float twice_sin = 2.0f * s;
    *c_out = mul_sub_from(twice_sin, s, 1.0f, arith);
    float sin_cos = s * c;
    *s_out = 2.0f * sin_cos;
}

/* Magnitude factor from a pair p whose squared magnitude 1 + e equals the
 * final pair's magnitude: 1 - e = 2 - |p|^2 (method 1), 1 / |p|^2 (method 2). */
float oracle_magnitude_factor(float s, float c, int arith, int method)
{
    if (method == ORACLE_METHOD2) {
        float cos_sq = c * c;
        float mag_sq = mul_add(s, s, cos_sq, arith);
        return 1.0f / mag_sq;
    }
    float two_less_cos_sq = mul_sub_from(c, c, 2.0f, arith);
    return mul_sub_from(s, s, two_less_cos_sq, arith);
}

/* Series, two doublings and the magnitude factor, on a reduced angle x in
 * [-1/2, 1/2].  The factor is read from the pair after the first doubling,
 * whose squared magnitude is the final magnitude.                          */
void oracle_pair_from_reduced(float x, int arith, int method, float *s, float *c)
{
    float qs, qc, hs, hc, fs, fc;
    oracle_quarter_series(x, arith, method, &qs, &qc); /* angle pi x / 2 */
    oracle_double_angle(qs, qc, arith, &hs, &hc);      /* angle pi x     */
    float m = oracle_magnitude_factor(hs, hc, arith, method);
    oracle_double_angle(hs, hc, arith, &fs, &fc);      /* angle 2 pi x   */
    *s = fs * m;
    *c = fc * m;
}

/* The sine-cosine pair of the angle theta (radians).                       */
void oracle_sincos_pair(float theta, int arith, int method, float *s, float *c)
{
    oracle_pair_from_reduced(oracle_reduce(theta), arith, method, s, c);
}

/* The same pair without the magnitude factor (the drift it removes).       */
void oracle_pair_unfixed(float x, int arith, int method, float *s, float *c)
{
    float qs, qc, hs, hc;
    oracle_quarter_series(x, arith, method, &qs, &qc);
    oracle_double_angle(qs, qc, arith, &hs, &hc);
    oracle_double_angle(hs, hc, arith, s, c);
}

/* ---------------------------------------------------------------------- */
/* Ablations of Sec. II (analysis only; the method is oracle_pair_from_reduced).
 *   ORACLE_VARIANT_LISTING    the method: factor 2 - |p|^2 read after doubling 1
 *   ORACLE_VARIANT_NO_FIX     no magnitude correction
 *   ORACLE_VARIANT_TEXT_FIX   the text's form: (3 - s^2 - c^2)/2 on the final pair
 *   ORACLE_VARIANT_EQ2        both doublings with the rejected eq. (2),
 *                             cos 2u = 1 - 2 sin^2 u, then the method's factor */
#define ORACLE_VARIANT_LISTING 0
#define ORACLE_VARIANT_NO_FIX 1
#define ORACLE_VARIANT_TEXT_FIX 2
#define ORACLE_VARIANT_EQ2 3

/* (3 - s^2 - c^2) / 2: one Newton step towards 1/|p| from |p|^2 = 1 + e. */
static float text_factor(float s, float c, int arith)
{
    float three_less_cos_sq = mul_sub_from(c, c, 3.0f, arith);
    float h = mul_sub_from(s, s, three_less_cos_sq, arith);
    return 0.5f * h;
}

void oracle_pair_variant(float x, int arith, int method, int variant, float *s, float *c)
{
    float qs, qc, hs, hc, fs, fc;
    oracle_quarter_series(x, arith, method, &qs, &qc);
    if (variant == ORACLE_VARIANT_EQ2) {
        oracle_double_angle_eq2(qs, qc, arith, &hs, &hc);
        float m = oracle_magnitude_factor(hs, hc, arith, method);
        oracle_double_angle_eq2(hs, hc, arith, &fs, &fc);
        *s = fs * m;
        *c = fc * m;
        return;
    }
    oracle_double_angle(qs, qc, arith, &hs, &hc);
    oracle_double_angle(hs, hc, arith, &fs, &fc);
    if (variant == ORACLE_VARIANT_NO_FIX) {
        *s = fs;
        *c = fc;
        return;
    }
    float m = variant == ORACLE_VARIANT_TEXT_FIX ? text_factor(fs, fc, arith)
                                                 : oracle_magnitude_factor(hs, hc, arith, method);
    *s = fs * m;
    *c = fc * m;
}

/* ---------------------------------------------------------------------- */
/* Ablation: the number of doublings against the series length (analysis
 * only).  Sec. II argues that each eq. (1) doubling keeps the relative angle
 * error and squares the magnitude, so a series over a smaller angle (shorter,
 * for the same fit error) can be followed by more doublings, at the price of
 * a magnitude drift and first-pair rounding that grow with 2^n.  Here the
 * series approximate sin and cos of 2 pi x / 2^n (n = ndoub; n = 2 is the
 * method, whose quarter angle is pi x / 2):
 *   s = x (ss[0] + ss[1] x2 + ... + ss[ns-1] x2^(ns-1))
 *   c = 1 + x2 (cc[0] + cc[1] x2 + ... + cc[nc-1] x2^(nc-1))
 * by Horner's rule in x2 as in the method.  Then n doublings with eq. (1).
 * With fix, the factor 2 - |p|^2 is read from the pair that precedes the
 * last doubling, whose squared magnitude is the final magnitude a^(2^n).
 * With no doubling at all (n = 0) there is no earlier pair: the text's
 * (3 - s^2 - c^2) / 2 is applied to the series pair itself.  With n = 2, the
 * first method's coefficients and fix, this is the method exactly.        */
void oracle_pair_general(float x, int arith, int ndoub, const float *ss, int ns,
                         const float *cc, int nc, int fix, float *s, float *c)
{
    float x2 = x * x;
    float ps = x * horner(x2, ss, ns, arith);
    float pc = mul_add(x2, horner(x2, cc, nc, arith), 1.0f, arith);
    float m = 1.0f;
    if (ndoub == 0 && fix)
        m = text_factor(ps, pc, arith);
    for (int d = 0; d < ndoub; d++) {
        if (fix && d == ndoub - 1)
            m = oracle_magnitude_factor(ps, pc, arith, ORACLE_METHOD1);
        float ds, dc;
        oracle_double_angle(ps, pc, arith, &ds, &dc);
        ps = ds;
        pc = dc;
    }
    *s = fix ? ps * m : ps;
    *c = fix ? pc * m : pc;
}

/* ---------------------------------------------------------------------- */
/* Array drivers.  A plain loop over elements; with threads > 1 the array is
 * cut into contiguous chunks, each run by the same scalar loop.  Each worker
 * first installs the default floating-point environment (round to nearest,
 * no flush-to-zero), whatever the host process has set.                    */

typedef void (*chunk_fn)(void *job, int64_t lo, int64_t hi);

struct chunk_task {
    chunk_fn fn;
    void *job;
    int64_t lo, hi;
};

static void *chunk_worker(void *arg)
{
    struct chunk_task *t = (struct chunk_task *)arg;
    fenv_t saved;
    fegetenv(&saved);
    fesetenv(FE_DFL_ENV);
    t->fn(t->job, t->lo, t->hi);
    fesetenv(&saved);
    return NULL;
}

static int run_chunks(chunk_fn fn, void *job, int64_t n, int threads)
{
    if (threads < 1)
        threads = 1;
    if (threads > 256)
        threads = 256;
    if ((int64_t)threads > n)
        threads = n > 0 ? (int)n : 1;
    struct chunk_task tasks[256];
    pthread_t tid[256];
    int64_t per = (n + threads - 1) / threads;
    int started = 0;
    for (int i = 0; i < threads; i++) {
        int64_t lo = (int64_t)i * per, hi = lo + per;
        if (lo > n)
            lo = n;
        if (hi > n)
            hi = n;
        tasks[i].fn = fn;
        tasks[i].job = job;
        tasks[i].lo = lo;
        tasks[i].hi = hi;
    }
    if (threads == 1) {
        chunk_worker(&tasks[0]);
        return 0;
    }
    for (int i = 0; i < threads; i++) {
        if (pthread_create(&tid[i], NULL, chunk_worker, &tasks[i]) != 0)
            break;
        started++;
    }
    for (int i = started; i < threads; i++) /* could not start: run here */
        chunk_worker(&tasks[i]);
    for (int i = 0; i < started; i++)
        pthread_join(tid[i], NULL);
    return 0;
}

struct pair_job {
    const float *x;
    float *s, *c;
    int arith, method;
};

static void pair_chunk(void *job, int64_t lo, int64_t hi)
{
    struct pair_job *j = (struct pair_job *)job;
    for (int64_t i = lo; i < hi; i++)
        oracle_sincos_pair(j->x[i], j->arith, j->method, &j->s[i], &j->c[i]);
}

/* s[i], c[i] = pair(x[i]) for 0 <= i < n.                                  */
int oracle_sincos_f32(const float *x, float *s, float *c, int64_t n, int arith, int method,
                      int threads)
{
    if (n < 0 || (n > 0 && (!x || !s || !c)))
        return -1;
    struct pair_job j = {x, s, c, arith, method};
    return run_chunks(pair_chunk, &j, n, threads);
}

/* Pair from already reduced angles (the reduced-angle error sweep).        */
struct reduced_job {
    const float *q;
    float *s, *c;
    int arith, method, fixed;
};

static void reduced_chunk(void *job, int64_t lo, int64_t hi)
{
    struct reduced_job *j = (struct reduced_job *)job;
    for (int64_t i = lo; i < hi; i++) {
        if (j->fixed)
            oracle_pair_from_reduced(j->q[i], j->arith, j->method, &j->s[i], &j->c[i]);
        else
            oracle_pair_unfixed(j->q[i], j->arith, j->method, &j->s[i], &j->c[i]);
    }
}

int oracle_pair_from_reduced_f32(const float *q, float *s, float *c, int64_t n, int arith,
                                 int method, int fixed, int threads)
{
    if (n < 0 || (n > 0 && (!q || !s || !c)))
        return -1;
    struct reduced_job j = {q, s, c, arith, method, fixed};
    return run_chunks(reduced_chunk, &j, n, threads);
}

/* The ablations over arrays of angles (step 1, then oracle_pair_variant or
 * oracle_pair_general on the reduced angle), for comparison with GPU
 * kernels that compute the same variants.                                  */
struct ablation_job {
    const float *x;
    float *s, *c;
    int arith, method, variant;       /* variant >= 0: oracle_pair_variant  */
    int ndoub, ns, nc, fix;           /* variant < 0: oracle_pair_general   */
    const float *ss, *cc;
};

static void ablation_chunk(void *job, int64_t lo, int64_t hi)
{
    struct ablation_job *j = (struct ablation_job *)job;
    for (int64_t i = lo; i < hi; i++) {
        const float x = oracle_reduce(j->x[i]);
        if (j->variant >= 0)
            oracle_pair_variant(x, j->arith, j->method, j->variant, &j->s[i], &j->c[i]);
        else
            oracle_pair_general(x, j->arith, j->ndoub, j->ss, j->ns, j->cc, j->nc, j->fix,
                                &j->s[i], &j->c[i]);
    }
}

int oracle_pair_variant_f32(const float *x, float *s, float *c, int64_t n, int arith, int method,
                            int variant, int threads)
{
    if (n < 0 || (n > 0 && (!x || !s || !c)) || variant < 0 || variant > 3)
        return -1;
    struct ablation_job j = {x, s, c, arith, method, variant, 0, 0, 0, 0, NULL, NULL};
    return run_chunks(ablation_chunk, &j, n, threads);
}

int oracle_pair_general_f32(const float *x, float *s, float *c, int64_t n, int arith, int ndoub,
                            const float *ss, int ns, const float *cc, int nc, int fix,
                            int threads)
{
    if (n < 0 || (n > 0 && (!x || !s || !c)) || !ss || !cc || ns < 1 || ns > 16 || nc < 1 ||
        nc > 16 || ndoub < 0 || ndoub > 8)
        return -1;
    struct ablation_job j = {x, s, c, arith, 0, -1, ndoub, ns, nc, fix, ss, cc};
    return run_chunks(ablation_chunk, &j, n, threads);
}

/* Reduction alone, elementwise.                                             */
int oracle_reduce_f32(const float *x, float *q, int64_t n)
{
    if (n < 0 || (n > 0 && (!x || !q)))
        return -1;
    for (int64_t i = 0; i < n; i++)
        q[i] = oracle_reduce(x[i]);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Error statistics against the double-precision system library, measured
 * as the paper measures them (Sec. II, method 1 results):
 *   vector error    sqrt((c - cos)^2 + (s - sin)^2)
 *   amplitude error |1 - sqrt(c^2 + s^2)|
 * over every binary32 reduced angle q whose bit pattern lies in
 * [bits_lo, bits_hi] with the given stride, the reference angle being
 * 2 pi q in double precision.  Negative q follow by symmetry.              */

struct err_stats {
    double max_vec, sum_sq_vec, max_amp;
    float argmax_vec, argmax_amp;
    int64_t count;
};

struct scan_job {
    uint32_t bits_lo, bits_hi, stride;
    int arith, method, variant;
    struct err_stats *per_chunk; /* one slot per chunk start */
    int64_t per;                 /* chunk length, to find the slot */
    /* oracle_pair_general's parameters when general != 0 */
    int general, ndoub, ns, nc, fix;
    const float *ss, *cc;
};

static void scan_chunk(void *job, int64_t lo, int64_t hi)
{
    struct scan_job *j = (struct scan_job *)job;
    struct err_stats st = {0.0, 0.0, 0.0, 0.0f, 0.0f, 0};
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t k = lo; k < hi; k++) {
        uint32_t bits = j->bits_lo + (uint32_t)k * j->stride;
        float q;
        memcpy(&q, &bits, sizeof q);
        float s, c;
        if (j->general)
            oracle_pair_general(q, j->arith, j->ndoub, j->ss, j->ns, j->cc, j->nc, j->fix, &s, &c);
        else if (j->variant == ORACLE_VARIANT_LISTING)
            oracle_pair_from_reduced(q, j->arith, j->method, &s, &c);
        else
            oracle_pair_variant(q, j->arith, j->method, j->variant, &s, &c);
        double a = two_pi * (double)q, rs, rc;
        sincos(a, &rs, &rc);
        double ds = (double)s - rs, dc = (double)c - rc;
        double ev = sqrt(ds * ds + dc * dc);
        double ea = fabs(1.0 - sqrt((double)s * s + (double)c * c));
        st.sum_sq_vec += ev * ev;
        if (ev > st.max_vec) {
            st.max_vec = ev;
            st.argmax_vec = q;
        }
        if (ea > st.max_amp) {
            st.max_amp = ea;
            st.argmax_amp = q;
        }
        st.count++;
    }
    j->per_chunk[lo / j->per] = st;
}

int oracle_error_scan_variant(uint32_t bits_lo, uint32_t bits_hi, uint32_t stride, int arith,
                              int method, int variant, int threads, double *out_max_vec,
                              double *out_rms_vec, double *out_max_amp, float *out_argmax_vec,
                              float *out_argmax_amp, int64_t *out_count);

/* fixed = 1: the method; fixed = 0: without step 4. */
int oracle_error_scan_reduced(uint32_t bits_lo, uint32_t bits_hi, uint32_t stride, int arith,
                              int method, int fixed, int threads, double *out_max_vec,
                              double *out_rms_vec, double *out_max_amp, float *out_argmax_vec,
                              float *out_argmax_amp, int64_t *out_count)
{
    return oracle_error_scan_variant(bits_lo, bits_hi, stride, arith, method,
                                     fixed ? ORACLE_VARIANT_LISTING : ORACLE_VARIANT_NO_FIX,
                                     threads, out_max_vec, out_rms_vec, out_max_amp,
                                     out_argmax_vec, out_argmax_amp, out_count);
}

static int run_scan(struct scan_job *j, int threads, double *out_max_vec, double *out_rms_vec,
                    double *out_max_amp, float *out_argmax_vec, float *out_argmax_amp,
                    int64_t *out_count)
{
    if (j->stride == 0 || j->bits_hi < j->bits_lo)
        return -1;
    int64_t n = (int64_t)((j->bits_hi - j->bits_lo) / j->stride) + 1;
    if (threads < 1)
        threads = 1;
    if (threads > 256)
        threads = 256;
    if ((int64_t)threads > n)
        threads = (int)n;
    struct err_stats slots[256];
    memset(slots, 0, sizeof slots);
    j->per_chunk = slots;
    j->per = (n + threads - 1) / threads;
    run_chunks(scan_chunk, j, n, threads);
    struct err_stats tot = {0.0, 0.0, 0.0, 0.0f, 0.0f, 0};
    for (int i = 0; i < threads; i++) {
        tot.sum_sq_vec += slots[i].sum_sq_vec;
        tot.count += slots[i].count;
        if (slots[i].max_vec > tot.max_vec) {
            tot.max_vec = slots[i].max_vec;
            tot.argmax_vec = slots[i].argmax_vec;
        }
        if (slots[i].max_amp > tot.max_amp) {
            tot.max_amp = slots[i].max_amp;
            tot.argmax_amp = slots[i].argmax_amp;
        }
    }
    *out_max_vec = tot.max_vec;
    *out_rms_vec = tot.count ? sqrt(tot.sum_sq_vec / (double)tot.count) : 0.0;
    *out_max_amp = tot.max_amp;
    *out_argmax_vec = tot.argmax_vec;
    *out_argmax_amp = tot.argmax_amp;
    *out_count = tot.count;
    return 0;
}

int oracle_error_scan_variant(uint32_t bits_lo, uint32_t bits_hi, uint32_t stride, int arith,
                              int method, int variant, int threads, double *out_max_vec,
                              double *out_rms_vec, double *out_max_amp, float *out_argmax_vec,
                              float *out_argmax_amp, int64_t *out_count)
{
    struct scan_job j;
    memset(&j, 0, sizeof j);
    j.bits_lo = bits_lo;
    j.bits_hi = bits_hi;
    j.stride = stride;
    j.arith = arith;
    j.method = method;
    j.variant = variant;
    return run_scan(&j, threads, out_max_vec, out_rms_vec, out_max_amp, out_argmax_vec,
                    out_argmax_amp, out_count);
}

/* The same statistics for oracle_pair_general (1 <= ns, nc <= 16,
 * 0 <= ndoub <= 16).                                                        */
int oracle_error_scan_general(uint32_t bits_lo, uint32_t bits_hi, uint32_t stride, int arith,
                              int ndoub, const float *ss, int ns, const float *cc, int nc,
                              int fix, int threads, double *out_max_vec, double *out_rms_vec,
                              double *out_max_amp, float *out_argmax_vec,
                              float *out_argmax_amp, int64_t *out_count)
{
    if (ns < 1 || ns > 16 || nc < 1 || nc > 16 || ndoub < 0 || ndoub > 16 || !ss || !cc)
        return -1;
    struct scan_job j;
    memset(&j, 0, sizeof j);
    j.bits_lo = bits_lo;
    j.bits_hi = bits_hi;
    j.stride = stride;
    j.arith = arith;
    j.general = 1;
    j.ndoub = ndoub;
    j.ns = ns;
    j.nc = nc;
    j.fix = fix;
    j.ss = ss;
    j.cc = cc;
    return run_scan(&j, threads, out_max_vec, out_rms_vec, out_max_amp, out_argmax_vec,
                    out_argmax_amp, out_count);
}

/* ---------------------------------------------------------------------- */
/* Adjoint of the pair (plain definition): d sin/dx = cos, d cos/dx = -sin,
 * so the gradient reaching x is gx = gs * c - gc * s, each product and the
 * difference rounded once in binary32.  A null gs or gc counts as zero.    */
int oracle_sincos_backward_f32(const float *s, const float *c, const float *gs, const float *gc,
                               float *gx, int64_t n)
{
    if (n < 0 || (n > 0 && (!s || !c || !gx)))
        return -1;
    for (int64_t i = 0; i < n; i++) {
        float a = gs ? gs[i] * c[i] : 0.0f;
        float b = gc ? gc[i] * s[i] : 0.0f;
        gx[i] = a - b;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Sinusoid model used for fitting (the application of Sec. II, second
 * paragraph: least-squares fits need a smooth function).  In binary32:
 *   theta_ik = fmaf(w_k, t_i, phi_k)
 *   y_i      = sum over k = 0..K-1, in that order, acc = fmaf(A_k, s_ik, acc)
 * with (s_ik, c_ik) the pair of theta_ik from steps 1-4.                   */

struct sinusoid_job {
    const float *t, *A, *w, *phi;
    int32_t K;
    float *y;
    int arith, method;
};

static void sinusoid_chunk(void *job, int64_t lo, int64_t hi)
{
    struct sinusoid_job *j = (struct sinusoid_job *)job;
    for (int64_t i = lo; i < hi; i++) {
        float acc = 0.0f;
        for (int32_t k = 0; k < j->K; k++) {
            float theta = fmaf(j->w[k], j->t[i], j->phi[k]);
            float s, c;
            oracle_sincos_pair(theta, j->arith, j->method, &s, &c);
            acc = fmaf(j->A[k], s, acc);
        }
        j->y[i] = acc;
    }
}

int oracle_sinusoid_forward_f32(const float *t, int64_t N, const float *A, const float *w,
                                const float *phi, int32_t K, float *y, int arith, int method,
                                int threads)
{
    if (N < 0 || K < 0 || (N > 0 && (!t || !y)) || (K > 0 && (!A || !w || !phi)))
        return -1;
    struct sinusoid_job j = {t, A, w, phi, K, y, arith, method};
    return run_chunks(sinusoid_chunk, &j, N, threads);
}

/* Gradients of L with dL/dy_i = g_i (g = y - y_obs for L = 1/2 sum r^2):
 *   gA_k   = sum_i g_i s_ik
 *   gphi_k = A_k sum_i g_i c_ik
 *   gw_k   = A_k sum_i g_i c_ik t_i
 * The pairs are the binary32 pairs of the binary32 theta_ik above; every
 * product and sum after that is done in double precision, in index order.
 * abs_* receive the same sums over absolute values of the terms, which bound
 * the rounding error of any other summation order.                          */
int oracle_sinusoid_adjoint_f64(const float *t, const float *g, int64_t N, const float *A,
                                const float *w, const float *phi, int32_t K, double *gA,
                                double *gw, double *gphi, double *abs_A, double *abs_w,
                                double *abs_phi, int arith, int method)
{
    if (N < 0 || K < 0 || (N > 0 && (!t || !g)) || (K > 0 && (!A || !w || !phi)))
        return -1;
    for (int32_t k = 0; k < K; k++) {
        double sa = 0, sp = 0, sw = 0, aa = 0, ap = 0, aw = 0;
        for (int64_t i = 0; i < N; i++) {
            float theta = fmaf(w[k], t[i], phi[k]);
            float s, c;
            oracle_sincos_pair(theta, arith, method, &s, &c);
            double ts = (double)g[i] * s;
            double tc = (double)g[i] * c;
            double tw = tc * (double)t[i];
            sa += ts;
            sp += tc;
            sw += tw;
            aa += fabs(ts);
            ap += fabs(tc);
            aw += fabs(tw);
        }
        gA[k] = sa;
        gphi[k] = (double)A[k] * sp;
        gw[k] = (double)A[k] * sw;
        if (abs_A)
            abs_A[k] = aa;
        if (abs_phi)
            abs_phi[k] = fabs((double)A[k]) * ap;
        if (abs_w)
            abs_w[k] = fabs((double)A[k]) * aw;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Huygens' principle (the author's application, Sec. IV): the field at
 * screen point i (xo_i, yo_i, L) from S point sources (xa_j, ya_j, 0) of
 * amplitude a_j and phase phi_j,
 *     U_i = sum_j (a_j / r_ij) exp(i (k (r_ij - L) + phi_j)),
 * with the obliquity factor taken as 1 and the path difference r - L
 * written as rho^2 / (r + L) so that no cancellation occurs.  Both
 * quotients, rho^2 / (r + L) and a / r, come from one reciprocal of
 * r (r + L) while that product is a normal binary32; outside that range
 * (r beyond about 2^63 or below about 2^-63) each is its own division.
 * In binary32, each operation rounded, for one block of sources
 * j = lo..hi-1 in order, accumulators from +0:
 *     dx = xo - xa;  dy = yo - ya;  rho2 = fmaf(dx, dx, dy * dy)
 *     r = sqrtf(rho2 + L2) with L2 = L * L;  e = r + L;  x = r * e
 *     if FLT_MIN <= x <= FLT_MAX:  g = 1 / x;  d = rho2 * (r * g);  w = a * (e * g)
 *     else:                        d = rho2 / e;  w = a / r
 *     theta = fmaf(k, d, phi);  (s, c) = the pair of theta
 *     re = fmaf(w, c, re);  im = fmaf(w, s, im)
 * (r g is 1 / e and e g is 1 / r up to rounding, so no intermediate grows
 * past the quotients themselves.)
 * The sum over all S sources splits them into `blocks` contiguous blocks of
 * ceil(S / blocks) sources (the last ones shorter or empty), sums each block
 * as above and adds the block sums in block order, (((B0 + B1) + B2) + ...),
 * re and im separately.  oracle_huygens_f32 is this with 4 blocks (the
 * order is not in the paper; four blocks let four GPU lanes share a point);
 * one block is the plain sum in source order.  src holds (xa, ya, a, phi)
 * per source.                                                               */
#define HUYGENS_BLOCKS 4

struct huygens_job {
    const float *xo, *yo, *src;
    int32_t S, blocks;
    float k, L;
    float *re, *im;
    int arith, method;
};

static void huygens_block_sum(const struct huygens_job *j, int64_t i, int32_t lo, int32_t hi,
                              float *re_out, float *im_out)
{
    const float L2 = j->L * j->L;
    float re = 0.0f, im = 0.0f;
    for (int32_t q = lo; q < hi; q++) {
        const float *sq = j->src + 4 * (int64_t)q;
        float dx = j->xo[i] - sq[0];
        float dy = j->yo[i] - sq[1];
        float dy2 = dy * dy;
        float rho2 = fmaf(dx, dx, dy2);
        float r = sqrtf(rho2 + L2);
        float e = r + j->L;
        float x = r * e;
        float d, w;
        if (x >= FLT_MIN && x <= FLT_MAX) {
            float g = 1.0f / x;
            d = rho2 * (r * g);
            w = sq[2] * (e * g);
        } else {
            d = rho2 / e;
            w = sq[2] / r;
        }
        float theta = fmaf(j->k, d, sq[3]);
        float sv, cv;
        oracle_sincos_pair(theta, j->arith, j->method, &sv, &cv);
        re = fmaf(w, cv, re);
        im = fmaf(w, sv, im);
    }
    *re_out = re;
    *im_out = im;
}

static void huygens_chunk(void *job, int64_t lo, int64_t hi)
{
    struct huygens_job *j = (struct huygens_job *)job;
    const int32_t per = (int32_t)(((int64_t)j->S + j->blocks - 1) / j->blocks);
    for (int64_t i = lo; i < hi; i++) {
        float re = 0.0f, im = 0.0f;
        for (int32_t b = 0; b < j->blocks; b++) {
            const int32_t first = (int32_t)(b * (int64_t)per < j->S ? b * (int64_t)per : j->S);
            const int32_t last = (int32_t)(first + (int64_t)per < j->S ? first + per : j->S);
            float bre, bim;
            huygens_block_sum(j, i, first, last, &bre, &bim);
            if (b == 0) {
                re = bre;
                im = bim;
            } else {
                re = re + bre;
                im = im + bim;
            }
        }
        j->re[i] = re;
        j->im[i] = im;
    }
}

int oracle_huygens_blocks_f32(const float *xo, const float *yo, int64_t P, const float *src,
                              int32_t S, int32_t blocks, float k, float L, float *re, float *im,
                              int arith, int method, int threads)
{
    if (P < 0 || S < 0 || blocks < 1 || (P > 0 && (!xo || !yo || !re || !im)) ||
        (S > 0 && !src))
        return -1;
    struct huygens_job j = {xo, yo, src, S, blocks, k, L, re, im, arith, method};
    return run_chunks(huygens_chunk, &j, P, threads);
}

int oracle_huygens_f32(const float *xo, const float *yo, int64_t P, const float *src, int32_t S,
                       float k, float L, float *re, float *im, int arith, int method, int threads)
{
    return oracle_huygens_blocks_f32(xo, yo, P, src, S, HUYGENS_BLOCKS, k, L, re, im, arith,
                                     method, threads);
}

/* Constants as the oracle rounds them, for the bit-pattern test.           */
void oracle_constants(int method, float *out8)
{
    struct series_coeffs k = method_coeffs(method);
    out8[0] = reduction_constant();
    out8[1] = k.ss1;
    out8[2] = k.ss2;
    out8[3] = k.ss3;
    out8[4] = k.ss4;
    out8[5] = k.cc1;
    out8[6] = k.cc2;
    out8[7] = k.cc3;
}
