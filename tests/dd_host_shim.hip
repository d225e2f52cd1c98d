// Host build of the library's double-double arithmetic (csrc/dd.h) for the
// CPU test of its operations against 50-digit values: every function takes
// and returns (hi, lo) pairs through plain arrays.
#include "dd.h"

using abm::dd;

extern "C" {
void t_add(const double* x, const double* y, double* o) { const dd r = abm::dd_add(dd{x[0], x[1]}, dd{y[0], y[1]}); o[0] = r.hi; o[1] = r.lo; }
void t_mul(const double* x, const double* y, double* o) { const dd r = abm::dd_mul(dd{x[0], x[1]}, dd{y[0], y[1]}); o[0] = r.hi; o[1] = r.lo; }
void t_div(const double* x, const double* y, double* o) { const dd r = abm::dd_div(dd{x[0], x[1]}, dd{y[0], y[1]}); o[0] = r.hi; o[1] = r.lo; }
void t_div_d(const double* x, double y, double* o) { const dd r = abm::dd_div_d(dd{x[0], x[1]}, y); o[0] = r.hi; o[1] = r.lo; }
void t_exp(const double* x, double* o) { const dd r = abm::dd_exp(dd{x[0], x[1]}); o[0] = r.hi; o[1] = r.lo; }
void t_log(const double* x, double* o) { const dd r = abm::dd_log(dd{x[0], x[1]}); o[0] = r.hi; o[1] = r.lo; }
void t_pow(const double* x, double a, double* o) { const dd r = abm::dd_pow(dd{x[0], x[1]}, a); o[0] = r.hi; o[1] = r.lo; }
void t_gamma(const double* x, double* o) { const dd r = abm::dd_gamma(dd{x[0], x[1]}); o[0] = r.hi; o[1] = r.lo; }
void t_sincos(const double* x, double* o)
{
    dd s, c;
    abm::dd_sincos(dd{x[0], x[1]}, &s, &c);
    o[0] = s.hi;
    o[1] = s.lo;
    o[2] = c.hi;
    o[3] = c.lo;
}
}
