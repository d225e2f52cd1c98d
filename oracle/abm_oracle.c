/*
 * Reference CPU oracle for the fractional Adams-Bashforth-Moulton (ABM)
 * predictor-corrector (Bonchis, Kaslik, Rosu, "HPC optimal parallel
 * communication algorithm for the simulation of fractional-order systems",
 * arXiv 1710.01133).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * What it computes (Section 2, "Preliminaries"):
 *   problem      D^alpha y = f(t, y), y(0) = x0, and y'(0) = x1 when
 *                1 < alpha <= 2 (the ceil(alpha) initial values of eq. fde)
 *   grid         t_n = n h, f_n = f(t_n, y_n) with the corrected y_n
 *   start term   T(t) = x0 (alpha <= 1),  x0 + t x1 (1 < alpha <= 2): the
 *                Taylor sum over k < ceil(alpha) in eq. abm
 *   predictor    yP_{n+1} = T(t_{n+1}) + h^alpha * sum_{k=0..n} b_{n-k} f_k      (eq. abm)
 *   corrector    y_{n+1}  = T(t_{n+1}) + h^alpha * ( c_n f_0 + sum_{k=1..n} a_{n-k} f_k
 *                                            + f(t_{n+1}, yP_{n+1}) / Gamma(alpha+2) )
 *   weights      b_n = ((n+1)^alpha - n^alpha) / Gamma(alpha+1)
 *                a_n = ((n+2)^(alpha+1) - 2 (n+1)^(alpha+1) + n^(alpha+1)) / Gamma(alpha+2)
 *                c_n = (n^(alpha+1) - (n-alpha)(n+1)^alpha) / Gamma(alpha+2)
 * Readings taken where the text is garbled:
 *   - b_n is printed with "+" between the two powers; the product-rectangle
 *     rule it comes from needs "-" (the tests pin this by quadrature and by
 *     the telescoping sum of b).
 *   - exactly one corrector evaluation per step (PECE), f_n uses corrected y_n.
 *   - systems are treated component by component; an incommensurate system
 *     (eq. sys.LRC with alpha_1 != alpha_2) applies to component i the
 *     scalar scheme of order alpha_i: its own weights, h^alpha_i,
 *     Gamma(alpha_i + 2) and start term, with f evaluated on the whole state.
 *
 * Arithmetic: the weights are evaluated from the literal formulas in
 * __float128 (113-bit significand), so the cancellation inside the
 * differences of powers costs nothing visible, then rounded once to double.
 * Gamma(alpha+1), Gamma(alpha+2) and h^alpha are taken in double (tgamma,
 * pow).  History sums run in double, ascending k, plain or (optionally)
 * Neumaier-compensated.  A second form (oracle_solve_quad) runs the whole
 * scheme in __float128: the oracle of the library's double-double mode.
 *
 * Right-hand sides (a fixed set, numbered here on their own):
 *   0 LINEAR   f = -lambda * y                          p = {lambda}
 *   1 DUFFING  f = (y2, -delta y2 - y1 - y1^3 + A cos(omega t))   p = {delta, A, omega}
 *   2 LORENZ   f = (s(y2-y1), y1(r-y3)-y2, y1 y2 - b y3)          p = {s, r, b}
 *   3 POLY     f = c0 + c1 t (each component)            p = {c0, c1}
 *   4 LCR      f = (y2 - g(y1), -sigma y2 - y1 + F sin(omega t))  (eq. sys.LRC)
 *              p = {sigma, omega, a, b, F}
 *              g(x) = b x - a + b (x <= -1), a x (|x| < 1), b x + a - b (x >= 1)
 *   5 DIAG     f = (-l1 y1 + m1, -l2 y2 + m2): two uncoupled scalar equations,
 *              a test system for per-component orders   p = {l1, l2, m1, m2}
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

static int rhs_dim(int rhs)
{
    switch (rhs) {
    case 0: return 1;
    case 1: return 2;
    case 2: return 3;
    case 3: return 1;
    case 4: return 2;
    case 5: return 2;
    default: return -1;
    }
}

/* Right-hand side f(t, y) for the fixed set above. */
static void rhs_eval(int rhs, const double *p, double t, const double *y, double *f)
{
    switch (rhs) {
    case 0:
        f[0] = -p[0] * y[0];
        break;
    case 1:
        f[0] = y[1];
        f[1] = -p[0] * y[1] - y[0] - y[0] * y[0] * y[0] + p[1] * cos(p[2] * t);
        break;
    case 2:
        f[0] = p[0] * (y[1] - y[0]);
        f[1] = y[0] * (p[1] - y[2]) - y[1];
        f[2] = y[0] * y[1] - p[2] * y[2];
        break;
    case 3:
        f[0] = p[0] + p[1] * t;
        break;
    case 4: {
        double x = y[0], g;
        if (x <= -1.0)
            g = p[3] * x - p[2] + p[3];
        else if (x >= 1.0)
            g = p[3] * x + p[2] - p[3];
        else
            g = p[2] * x;
        f[0] = y[1] - g;
        f[1] = -p[0] * y[1] - y[0] + p[4] * sin(p[1] * t);
        break;
    }
    case 5:
        f[0] = -p[0] * y[0] + p[2];
        f[1] = -p[1] * y[1] + p[3];
        break;
    }
}

/* Orders accepted: 0 < alpha <= 2 (at most one initial derivative). */
static int order_ok(double alpha)
{
    return alpha > 0.0 && alpha <= 2.0;
}

/*
 * Weights b_k, a_k, c_k for k = k0..k0+n-1 (Section 2, eq. abm and the
 * corrector weights below it), each from its literal formula in __float128,
 * rounded once to double and stored at index k-k0.  The Gamma factors are
 * taken in double and applied in quad.
 */
int oracle_weights_at(double alpha, int64_t k0, int64_t n, double *b, double *a, double *c)
{
    if (!order_ok(alpha) || n < 0 || k0 < 0)
        return ORC_EINVAL;
    const __float128 al = (__float128)alpha;
    const __float128 g1 = (__float128)tgamma(alpha + 1.0);
    const __float128 g2 = (__float128)tgamma(alpha + 2.0);
    /* every index is independent of the others */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const int64_t k = k0 + i;
        const __float128 kq = (__float128)k;
        const __float128 k1 = kq + 1, k2 = kq + 2;
        const __float128 pk0 = (k == 0) ? 0 : powq(kq, al);   /* k^alpha */
        const __float128 pk1 = powq(k1, al);                  /* (k+1)^alpha */
        const __float128 qk0 = (k == 0) ? 0 : powq(kq, al + 1);
        const __float128 qk1 = powq(k1, al + 1);
        const __float128 qk2 = powq(k2, al + 1);
        if (b) b[i] = (double)((pk1 - pk0) / g1);
        if (a) a[i] = (double)((qk2 - 2 * qk1 + qk0) / g2);
        if (c) c[i] = (double)((qk0 - (kq - al) * pk1) / g2);
    }
    return ORC_OK;
}

/* Weights for k = 0..n-1. */
int oracle_weights(double alpha, int64_t n, double *b, double *a, double *c)
{
    return oracle_weights_at(alpha, 0, n, b, a, c);
}

/* One ABM history sum for one component: plain ascending order, or
 * Neumaier-compensated when comp != 0. */
static double hist_sum(const double *w, const double *F, int d, int comp_idx,
                       int64_t k_lo, int64_t n, int comp)
{
    double s = 0.0, e = 0.0;
    for (int64_t k = k_lo; k <= n; ++k) {
        const double term = w[n - k] * F[k * d + comp_idx];
        if (comp) {
            const double t = s + term;
            if (fabs(s) >= fabs(term))
                e += (s - t) + term;
            else
                e += (term - t) + s;
            s = t;
        } else {
            s += term;
        }
    }
    return s + e;
}

/* The history sum sum_{k=k_lo..n} w[n-k] F[k] of one scalar sequence, with
 * the summation the solver uses (comp = 0 plain ascending, comp = 1
 * Neumaier-compensated); exported so that the tests can pin both variants on
 * ill-conditioned sums. */
double oracle_history_sum(const double *w, const double *F, int64_t k_lo, int64_t n, int comp)
{
    return hist_sum(w, F, 1, 0, k_lo, n, comp);
}

/* Weight tables and scalar factors of one component of order alpha. */
struct comp_tables {
    double *b, *a, *c;
    double ha, g2;
};

static void free_tables(struct comp_tables *T, int d)
{
    for (int i = 0; i < d; ++i) {
        free(T[i].b);
        free(T[i].a);
        free(T[i].c);
        T[i].b = T[i].a = T[i].c = NULL;
    }
}

/* Tables for n indices of every component (orders alphas[0..d-1]). */
static int make_tables(struct comp_tables *T, int d, const double *alphas, double h, int64_t n)
{
    for (int i = 0; i < d; ++i)
        T[i].b = T[i].a = T[i].c = NULL;
    for (int i = 0; i < d; ++i) {
        T[i].b = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        T[i].a = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        T[i].c = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        if (!T[i].b || !T[i].a || !T[i].c) {
            free_tables(T, d);
            return ORC_ENOMEM;
        }
        int rc = oracle_weights(alphas[i], n, T[i].b, T[i].a, T[i].c);
        if (rc != ORC_OK) {
            free_tables(T, d);
            return rc;
        }
        T[i].ha = pow(h, alphas[i]);
        T[i].g2 = tgamma(alphas[i] + 2.0);
    }
    return ORC_OK;
}

/* Start term of component i at time t (the Taylor sum of eq. abm). */
static double start_term(double alpha, double x0, const double *x1, int i, double t)
{
    return alpha > 1.0 ? x0 + t * x1[i] : x0;
}

static int orders_ok(int d, const double *alphas)
{
    for (int i = 0; i < d; ++i)
        if (!order_ok(alphas[i]))
            return 0;
    return 1;
}

/*
 * One trajectory of the fractional ABM scheme, general form.
 *   rhs, p      right-hand side and its parameters (table above)
 *   d           state dimension (must equal the dimension of rhs)
 *   alphas      order of each component (d values, each in (0, 2]); equal
 *               values give the commensurate scheme
 *   h, N        step size, number of steps
 *   x0          initial state, d doubles
 *   x1          initial first derivative, d doubles, read only for components
 *               of order above 1 (may be NULL when there are none)
 *   out_stride  0: write only y_N;  k>0: write y_s for s = 0, k, 2k, ... and y_N
 *   y_out       d doubles per written state, in that order
 *   comp        0: plain ascending sums; 1: Neumaier-compensated sums
 * Returns 0, or a negative code for invalid arguments / allocation failure.
 */
int oracle_solve_gen(int rhs, int d, const double *alphas, double h, int64_t N,
                     const double *x0, const double *x1, const double *p, int64_t out_stride,
                     double *y_out, int comp)
{
    if (rhs_dim(rhs) != d || !alphas || !orders_ok(d, alphas) || !(h > 0.0) ||
        !isfinite(h) || N < 1 || out_stride < 0 || !x0 || !p || !y_out)
        return ORC_EINVAL;
    for (int i = 0; i < d; ++i)
        if (alphas[i] > 1.0 && !x1)
            return ORC_EINVAL;
    struct comp_tables T[8];
    double *F = malloc(sizeof(double) * (size_t)(N + 1) * (size_t)d);
    if (!F)
        return ORC_ENOMEM;
    int rc = make_tables(T, d, alphas, h, N);
    if (rc != ORC_OK) {
        free(F);
        return rc;
    }
    double y[8], yp[8], fp[8], P[8], C[8];

    rhs_eval(rhs, p, 0.0, x0, F);   /* F_0 = f(t_0, y_0) */
    int64_t w = 0;
    if (out_stride > 0) {
        memcpy(y_out, x0, sizeof(double) * (size_t)d);
        w = 1;
    }
    for (int64_t s = 1; s <= N; ++s) {
        const int64_t n = s - 1;
        const double t = (double)s * h;
        for (int i = 0; i < d; ++i)
            P[i] = hist_sum(T[i].b, F, d, i, 0, n, comp);
        for (int i = 0; i < d; ++i)
            yp[i] = start_term(alphas[i], x0[i], x1, i, t) + T[i].ha * P[i];
        rhs_eval(rhs, p, t, yp, fp);
        for (int i = 0; i < d; ++i) {
            /* c_n f_0 first, then the a-weighted sum over k = 1..n */
            double hs = hist_sum(T[i].a, F, d, i, 1, n, comp);
            C[i] = T[i].c[n] * F[i] + hs;
            y[i] = start_term(alphas[i], x0[i], x1, i, t) + T[i].ha * (C[i] + fp[i] / T[i].g2);
        }
        rhs_eval(rhs, p, t, y, F + s * d);
        if (out_stride > 0 && (s % out_stride == 0 || s == N)) {
            memcpy(y_out + w * d, y, sizeof(double) * (size_t)d);
            ++w;
        }
    }
    if (out_stride == 0)
        memcpy(y_out, y, sizeof(double) * (size_t)d);
    free_tables(T, d);
    free(F);
    return ORC_OK;
}

/* One trajectory with one order for every component and no initial
 * derivative (0 < alpha <= 1, or alpha <= 2 with y'(0) = 0). */
int oracle_solve(int rhs, int d, double alpha, double h, int64_t N,
                 const double *x0, const double *p, int64_t out_stride,
                 double *y_out, int comp)
{
    if (rhs_dim(rhs) != d || !(alpha > 0.0 && alpha <= 1.0))
        return ORC_EINVAL;
    double al[8];
    for (int i = 0; i < d; ++i)
        al[i] = alpha;
    return oracle_solve_gen(rhs, d, al, h, N, x0, NULL, p, out_stride, y_out, comp);
}

/* sum_{k=k_lo..n} |w[n-k] F[k]| of one component: the size of the terms of
 * a history sum, which bounds what rounding inside the sum can change. */
static double hist_abs_sum(const double *w, const double *F, int d, int comp_idx,
                           int64_t k_lo, int64_t n)
{
    double s = 0.0;
    for (int64_t k = k_lo; k <= n; ++k)
        s += fabs(w[n - k] * F[k * d + comp_idx]);
    return s;
}

/*
 * Single steps recomputed from a given state history, for checking outputs of
 * a long run one by one.  y_hist holds y_0 .. y_{smax-1} (d doubles each,
 * smax = max over s_list); for every s in s_list the oracle forms
 * F_k = f(t_k, y_hist_k) for k < s and applies one predictor-corrector step
 * (the same formulas as oracle_solve_gen), writing y_s to y_out + i*d.
 * scale_out (may be NULL) receives, per listed step and component, the size
 * of the history terms entering y_s:
 *   h^alpha * ( sum_{k=0..n} |b_{n-k} F_k| + |c_n F_0| + sum_{k=1..n} |a_{n-k} F_k| ).
 * comp != 0 takes the two history sums Neumaier-compensated, so that the
 * recomputed step carries almost none of the rounding a plain sum of n terms
 * accumulates.
 */
int oracle_steps_from_states_gen(int rhs, int d, const double *alphas, double h,
                                 const double *x0, const double *x1, const double *p,
                                 const double *y_hist, const int64_t *s_list, int32_t ns,
                                 double *y_out, double *scale_out, int comp)
{
    if (rhs_dim(rhs) != d || !alphas || !orders_ok(d, alphas) || !(h > 0.0) || ns < 0)
        return ORC_EINVAL;
    for (int i = 0; i < d; ++i)
        if (alphas[i] > 1.0 && !x1)
            return ORC_EINVAL;
    int64_t smax = 0;
    for (int32_t i = 0; i < ns; ++i) {
        if (s_list[i] < 1)
            return ORC_EINVAL;
        if (s_list[i] > smax)
            smax = s_list[i];
    }
    if (smax == 0)
        return ORC_OK;
    struct comp_tables T[8];
    double *F = malloc(sizeof(double) * (size_t)smax * (size_t)d);
    if (!F)
        return ORC_ENOMEM;
    int rc = make_tables(T, d, alphas, h, smax);
    if (rc != ORC_OK) {
        free(F);
        return rc;
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < smax; ++k)
        rhs_eval(rhs, p, (double)k * h, y_hist + k * d, F + k * d);
    /* the listed steps are independent of each other */
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t j = 0; j < ns; ++j) {
        double yp[8], fp[8];
        const int64_t s = s_list[j], n = s - 1;
        const double t = (double)s * h;
        for (int i = 0; i < d; ++i)
            yp[i] = start_term(alphas[i], x0[i], x1, i, t) +
                    T[i].ha * hist_sum(T[i].b, F, d, i, 0, n, comp);
        rhs_eval(rhs, p, t, yp, fp);
        for (int i = 0; i < d; ++i) {
            double hs = hist_sum(T[i].a, F, d, i, 1, n, comp);
            y_out[j * d + i] = start_term(alphas[i], x0[i], x1, i, t) +
                               T[i].ha * ((T[i].c[n] * F[i] + hs) + fp[i] / T[i].g2);
            if (scale_out)
                scale_out[j * d + i] = T[i].ha * (hist_abs_sum(T[i].b, F, d, i, 0, n) +
                                                  fabs(T[i].c[n] * F[i]) +
                                                  hist_abs_sum(T[i].a, F, d, i, 1, n));
        }
    }
    free_tables(T, d);
    free(F);
    return ORC_OK;
}

int oracle_steps_from_states(int rhs, int d, double alpha, double h, const double *x0,
                             const double *p, const double *y_hist, const int64_t *s_list,
                             int32_t ns, double *y_out)
{
    if (rhs_dim(rhs) != d || !(alpha > 0.0 && alpha <= 1.0))
        return ORC_EINVAL;
    double al[8];
    for (int i = 0; i < d; ++i)
        al[i] = alpha;
    return oracle_steps_from_states_gen(rhs, d, al, h, x0, NULL, p, y_hist, s_list, ns, y_out,
                                        NULL, 0);
}

/* ---------------------------------------------------------------------
 * The scheme in quad precision: the oracle of the library's double-double
 * mode, the counterpart of the paper's long-double runs (Section "Memory
 * saving improves computing time": the same computation with a wider type).
 * Every quantity is __float128 (113-bit significand): the weights from their
 * literal formulas (not rounded to double), Gamma(alpha+1), Gamma(alpha+2) by
 * tgammaq, h^alpha by powq, t_s = s h (exact: s and h are integers and
 * doubles), the right-hand side with cosq / sinq, the history sums (plain
 * ascending) and the state.  Inputs are the same doubles as for the double
 * oracle; each written state leaves as d pairs (hi, lo) of doubles with
 * hi = (double)y and lo = (double)(y - hi).
 * --------------------------------------------------------------------- */

typedef __float128 quad;

static void rhs_eval_q(int rhs, const double *pd, quad t, const quad *y, quad *f)
{
    quad p[8];
    for (int i = 0; i < 8; ++i)
        p[i] = (quad)pd[i];
    switch (rhs) {
    case 0:
        f[0] = -p[0] * y[0];
        break;
    case 1:
        f[0] = y[1];
        f[1] = -p[0] * y[1] - y[0] - y[0] * y[0] * y[0] + p[1] * cosq(p[2] * t);
        break;
    case 2:
        f[0] = p[0] * (y[1] - y[0]);
        f[1] = y[0] * (p[1] - y[2]) - y[1];
        f[2] = y[0] * y[1] - p[2] * y[2];
        break;
    case 3:
        f[0] = p[0] + p[1] * t;
        break;
    case 4: {
        quad x = y[0], g;
        if (x <= -1)
            g = p[3] * x - p[2] + p[3];
        else if (x >= 1)
            g = p[3] * x + p[2] - p[3];
        else
            g = p[2] * x;
        f[0] = y[1] - g;
        f[1] = -p[0] * y[1] - y[0] + p[4] * sinq(p[1] * t);
        break;
    }
    case 5:
        f[0] = -p[0] * y[0] + p[2];
        f[1] = -p[1] * y[1] + p[3];
        break;
    }
}

/* Quad weights b_k, a_k, c_k for k = 0..n-1 of order alpha, with quad Gamma
 * factors.  For k <= 1 the literal formulas; beyond, the same differences of
 * powers rewritten exactly so that quad keeps its digits (the literal forms
 * lose about log10 k digits for b and 2 log10 k for a and c), with
 * u = 1/k, v = 1/(k+1), e = (1+u)^alpha - 1 = expm1(alpha log1p(u)):
 *   (k+1)^alpha - k^alpha                     = k^alpha e
 *   (k+2)^(a+1) - 2 (k+1)^(a+1) + k^(a+1)     = (k+1)^(a+1) ((1+v)^(a+1) - 1 + (1-v)^(a+1) - 1)
 *   k^(a+1) - (k - alpha)(k+1)^alpha          = k^(a+1) (alpha u (1 + e) - e)
 * (each loses about log10 k digits). */
static void weights_q(double alpha, int64_t n, quad *b, quad *a, quad *c)
{
    const quad al = (quad)alpha, be = al + 1;
    const quad g1 = tgammaq(al + 1), g2 = tgammaq(al + 2);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        const quad kq = (quad)k;
        if (k <= 1) {
            const quad pk0 = (k == 0) ? 0 : powq(kq, al);
            const quad pk1 = powq(kq + 1, al);
            const quad qk0 = (k == 0) ? 0 : powq(kq, be);
            const quad qk1 = powq(kq + 1, be);
            const quad qk2 = powq(kq + 2, be);
            b[k] = (pk1 - pk0) / g1;
            a[k] = (qk2 - 2 * qk1 + qk0) / g2;
            c[k] = (qk0 - (kq - al) * pk1) / g2;
        } else {
            const quad u = 1 / kq, v = 1 / (kq + 1);
            const quad e = expm1q(al * log1pq(u));
            b[k] = powq(kq, al) * e / g1;
            a[k] = powq(kq + 1, be) * (expm1q(be * log1pq(v)) + expm1q(be * log1pq(-v))) / g2;
            c[k] = powq(kq, be) * (al * u * (1 + e) - e) / g2;
        }
    }
}

struct comp_tables_q {
    quad *b, *a, *c;
    quad ha, g2;
};

static void free_tables_q(struct comp_tables_q *T, int d)
{
    for (int i = 0; i < d; ++i) {
        free(T[i].b);
        free(T[i].a);
        free(T[i].c);
        T[i].b = T[i].a = T[i].c = NULL;
    }
}

static int make_tables_q(struct comp_tables_q *T, int d, const double *alphas, double h,
                         int64_t n)
{
    for (int i = 0; i < d; ++i)
        T[i].b = T[i].a = T[i].c = NULL;
    for (int i = 0; i < d; ++i) {
        const size_t bytes = sizeof(quad) * (size_t)(n > 0 ? n : 1);
        T[i].b = malloc(bytes);
        T[i].a = malloc(bytes);
        T[i].c = malloc(bytes);
        if (!T[i].b || !T[i].a || !T[i].c) {
            free_tables_q(T, d);
            return ORC_ENOMEM;
        }
        weights_q(alphas[i], n, T[i].b, T[i].a, T[i].c);
        T[i].ha = powq((quad)h, (quad)alphas[i]);
        T[i].g2 = tgammaq((quad)alphas[i] + 2);
    }
    return ORC_OK;
}

static quad hist_sum_q(const quad *w, const quad *F, int d, int comp_idx, int64_t k_lo, int64_t n)
{
    quad s = 0;
    for (int64_t k = k_lo; k <= n; ++k)
        s += w[n - k] * F[k * d + comp_idx];
    return s;
}

static quad start_term_q(double alpha, double x0, const double *x1, int i, quad t)
{
    return alpha > 1.0 ? (quad)x0 + t * (quad)x1[i] : (quad)x0;
}

static void put_pair(double *dst, quad v)
{
    const double hi = (double)v;
    dst[0] = hi;
    dst[1] = (double)(v - (quad)hi);
}

/* Quad weights of order alpha for k = k0..k0+n-1, as (hi, lo) pairs. */
int oracle_weights_quad(double alpha, int64_t k0, int64_t n, double *b, double *a, double *c)
{
    if (!order_ok(alpha) || n < 0 || k0 < 0)
        return ORC_EINVAL;
    quad *w = malloc(sizeof(quad) * 3 * (size_t)(k0 + n > 0 ? k0 + n : 1));
    if (!w)
        return ORC_ENOMEM;
    quad *wb = w, *wa = w + (k0 + n), *wc = w + 2 * (k0 + n);
    weights_q(alpha, k0 + n, wb, wa, wc);
    for (int64_t i = 0; i < n; ++i) {
        if (b) put_pair(b + 2 * i, wb[k0 + i]);
        if (a) put_pair(a + 2 * i, wa[k0 + i]);
        if (c) put_pair(c + 2 * i, wc[k0 + i]);
    }
    free(w);
    return ORC_OK;
}

/*
 * One trajectory of the scheme in quad precision (arguments as for
 * oracle_solve_gen; no compensated variant).  y_out: 2d doubles per written
 * state, the (hi, lo) pair of each component.
 */
int oracle_solve_quad(int rhs, int d, const double *alphas, double h, int64_t N,
                      const double *x0, const double *x1, const double *p, int64_t out_stride,
                      double *y_out)
{
    if (rhs_dim(rhs) != d || !alphas || !orders_ok(d, alphas) || !(h > 0.0) ||
        !isfinite(h) || N < 1 || out_stride < 0 || !x0 || !p || !y_out)
        return ORC_EINVAL;
    for (int i = 0; i < d; ++i)
        if (alphas[i] > 1.0 && !x1)
            return ORC_EINVAL;
    struct comp_tables_q T[8];
    quad *F = malloc(sizeof(quad) * (size_t)(N + 1) * (size_t)d);
    if (!F)
        return ORC_ENOMEM;
    int rc = make_tables_q(T, d, alphas, h, N);
    if (rc != ORC_OK) {
        free(F);
        return rc;
    }
    quad y0[8], y[8], yp[8], fp[8];
    for (int i = 0; i < d; ++i)
        y0[i] = y[i] = (quad)x0[i];
    rhs_eval_q(rhs, p, 0, y0, F);
    int64_t w = 0;
    if (out_stride > 0) {
        for (int i = 0; i < d; ++i)
            put_pair(y_out + 2 * i, y0[i]);
        w = 1;
    }
    for (int64_t s = 1; s <= N; ++s) {
        const int64_t n = s - 1;
        const quad t = (quad)s * (quad)h;
        for (int i = 0; i < d; ++i)
            yp[i] = start_term_q(alphas[i], x0[i], x1, i, t) +
                    T[i].ha * hist_sum_q(T[i].b, F, d, i, 0, n);
        rhs_eval_q(rhs, p, t, yp, fp);
        for (int i = 0; i < d; ++i) {
            const quad C = T[i].c[n] * F[i] + hist_sum_q(T[i].a, F, d, i, 1, n);
            y[i] = start_term_q(alphas[i], x0[i], x1, i, t) + T[i].ha * (C + fp[i] / T[i].g2);
        }
        rhs_eval_q(rhs, p, t, y, F + s * d);
        if (out_stride > 0 && (s % out_stride == 0 || s == N)) {
            for (int i = 0; i < d; ++i)
                put_pair(y_out + 2 * (w * d + i), y[i]);
            ++w;
        }
    }
    if (out_stride == 0)
        for (int i = 0; i < d; ++i)
            put_pair(y_out + 2 * i, y[i]);
    free_tables_q(T, d);
    free(F);
    return ORC_OK;
}

/*
 * Single quad steps from a given state history: y_hist holds y_0..y_{smax-1}
 * as (hi, lo) pairs (2d doubles per state, the value hi + lo); for every s in
 * s_list one predictor-corrector step in quad from f_k = f(t_k, y_k), k < s,
 * written to y_out as (hi, lo) pairs.
 */
int oracle_steps_from_states_quad(int rhs, int d, const double *alphas, double h,
                                  const double *x0, const double *x1, const double *p,
                                  const double *y_hist, const int64_t *s_list, int32_t ns,
                                  double *y_out)
{
    if (rhs_dim(rhs) != d || !alphas || !orders_ok(d, alphas) || !(h > 0.0) || ns < 0)
        return ORC_EINVAL;
    for (int i = 0; i < d; ++i)
        if (alphas[i] > 1.0 && !x1)
            return ORC_EINVAL;
    int64_t smax = 0;
    for (int32_t i = 0; i < ns; ++i) {
        if (s_list[i] < 1)
            return ORC_EINVAL;
        if (s_list[i] > smax)
            smax = s_list[i];
    }
    if (smax == 0)
        return ORC_OK;
    struct comp_tables_q T[8];
    quad *F = malloc(sizeof(quad) * (size_t)smax * (size_t)d);
    if (!F)
        return ORC_ENOMEM;
    int rc = make_tables_q(T, d, alphas, h, smax);
    if (rc != ORC_OK) {
        free(F);
        return rc;
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < smax; ++k) {
        quad yk[8];
        for (int i = 0; i < d; ++i)
            yk[i] = (quad)y_hist[2 * (k * d + i)] + (quad)y_hist[2 * (k * d + i) + 1];
        rhs_eval_q(rhs, p, (quad)k * (quad)h, yk, F + k * d);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t j = 0; j < ns; ++j) {
        quad yp[8], fp[8];
        const int64_t s = s_list[j], n = s - 1;
        const quad t = (quad)s * (quad)h;
        for (int i = 0; i < d; ++i)
            yp[i] = start_term_q(alphas[i], x0[i], x1, i, t) +
                    T[i].ha * hist_sum_q(T[i].b, F, d, i, 0, n);
        rhs_eval_q(rhs, p, t, yp, fp);
        for (int i = 0; i < d; ++i) {
            const quad C = T[i].c[n] * F[i] + hist_sum_q(T[i].a, F, d, i, 1, n);
            put_pair(y_out + 2 * (j * d + i),
                     start_term_q(alphas[i], x0[i], x1, i, t) + T[i].ha * (C + fp[i] / T[i].g2));
        }
    }
    free_tables_q(T, d);
    free(F);
    return ORC_OK;
}

/*
 * A batch of independent trajectories, one per entry, run in parallel over
 * trajectories with OpenMP (each trajectory is the single-trajectory scheme
 * above, unchanged).  Arrays are per trajectory: rhs[i], d[i], h[i], N[i],
 * alphas[i*4 ...] (order of each component), x0[i*4 ...], x1[i*4 ...],
 * p[i*8 ...]; y_out[i] points at that trajectory's output.  status[i]
 * receives each trajectory's return code.
 */
int oracle_solve_batch_gen(int32_t B, const int32_t *rhs, const int32_t *d,
                           const double *alphas, const double *h, const int64_t *N,
                           const double *x0, const double *x1, const double *p,
                           int64_t out_stride, double *const *y_out, int32_t *status, int comp)
{
    if (B < 0)
        return ORC_EINVAL;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int32_t i = 0; i < B; ++i) {
        status[i] = oracle_solve_gen(rhs[i], d[i], alphas + 4 * (size_t)i, h[i], N[i],
                                     x0 + 4 * (size_t)i, x1 + 4 * (size_t)i, p + 8 * (size_t)i,
                                     out_stride, y_out[i], comp);
        bad |= (status[i] != ORC_OK);
    }
    return bad ? ORC_EINVAL : ORC_OK;
}

/* Number of OpenMP threads the batch entry point would use. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
