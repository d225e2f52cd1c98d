// K0: the ABM weight tables b_k, a_k, c_k (Section 2, eq. abm and the
// corrector weights after it) for k = 0..n-1, in double, on the device.
//
// The defining formulas are differences of nearby powers,
//   b_k Gamma(a+1) = (k+1)^a - k^a
//   a_k Gamma(a+2) = (k+2)^(a+1) - 2 (k+1)^(a+1) + k^(a+1)
//   c_k Gamma(a+2) = k^(a+1) - (k-a) (k+1)^a,
// whose direct evaluation in double loses about 2 log10(k) digits (a_k at
// k = 262144 would carry a relative error near 1e-6).  Here each difference is
// rewritten as a binomial series in u = 1/k (or 1/(k+1)) that has no
// cancellation:
//   (k+1)^a - k^a                  = k^(a-1)   * sum_{j>=1} C(a,j) u^(j-1)
//   (m+1)^b - 2 m^b + (m-1)^b      = 2 m^(b-2) * sum_{j>=1} C(b,2j) u^(2j-2),  m = k+1, b = a+1
//   k^(a+1) - (k-a)(k+1)^a         = k^(a-1)   * sum_{j>=2} -(C(a,j) - a C(a,j-1)) u^(j-2)
// The series are used for k >= 2 (u <= 1/2, terms fall at least like 2^-j)
// and the first indices are taken from short exact expressions.  Each result
// is within a few ulp of the exact weight; at a = 1 the series collapse to
// b = a = 1, c = 1/2 up to the rounding of the Gamma factors.
#include "abm_dev.h"
#include "abm_kernels.h"

namespace abm {

namespace {

// 2^a - 1 without losing digits for small a.
__device__ double two_pow_m1(double a)
{
    return (a >= 0.5) ? (exp2(a) - 1.0) : expm1(a * 0.69314718055994530942);
}

__device__ double series_b(double al, double u)
{
    // sum_{j>=1} C(al, j) u^(j-1)
    double coef = al;      // C(al, 1)
    double up = 1.0;       // u^(j-1)
    double s = 0.0;
    for (int j = 1; j < 200; ++j) {
        const double term = coef * up;
        s += term;
        if (fabs(term) <= 1e-18 * fabs(s)) break;
        coef *= (al - j) / (j + 1.0);  // C(al, j+1)
        up *= u;
    }
    return s;
}

__device__ double series_a(double be, double u)
{
    // sum_{j>=1} C(be, 2j) u^(2j-2)
    double c2 = be * (be - 1.0) * 0.5;   // C(be, 2)
    const double u2 = u * u;
    double up = 1.0;
    double s = 0.0;
    for (int j = 1; j < 200; ++j) {
        const double term = c2 * up;
        s += term;
        if (fabs(term) <= 1e-18 * fabs(s) || c2 == 0.0) break;
        // C(be, 2j+2) = C(be, 2j) (be-2j)(be-2j-1) / ((2j+1)(2j+2))
        c2 *= (be - 2.0 * j) * (be - 2.0 * j - 1.0) / ((2.0 * j + 1.0) * (2.0 * j + 2.0));
        up *= u2;
    }
    return s;
}

__device__ double series_c(double al, double u)
{
    // sum_{j>=2} -(C(al,j) - al C(al,j-1)) u^(j-2)
    double cj1 = al;                       // C(al, 1)
    double cj = al * (al - 1.0) * 0.5;     // C(al, 2)
    double up = 1.0;
    double s = 0.0;
    for (int j = 2; j < 200; ++j) {
        const double term = -(cj - al * cj1) * up;
        s += term;
        if (fabs(term) <= 1e-18 * fabs(s)) break;
        cj1 = cj;
        cj *= (al - j) / (j + 1.0);
        up *= u;
    }
    return s;
}

__global__ __launch_bounds__(256) void k_weights(double al, int64_t n,
                                                 const double* __restrict__ gam,
                                                 double* __restrict__ b, double* __restrict__ a,
                                                 double* __restrict__ c)
{
    const double g1inv = 1.0 / gam[0], g2inv = 1.0 / gam[1];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        double bk, ak, ck;
        if (k == 0) {
            bk = 1.0;
            ak = 2.0 * two_pow_m1(al);         // 2^(a+1) - 2
            ck = al;
        } else if (k == 1) {
            bk = two_pow_m1(al);               // 2^a - 1
            // 3^(a+1) - 2^(a+2) + 1: series in u = 1/2 around m = 2
            ak = exp2(al) * series_a(al + 1.0, 0.5);
            ck = al - (1.0 - al) * two_pow_m1(al);   // 1 - (1-a) 2^a
        } else {
            const double kd = (double)k;
            const double u = 1.0 / kd;
            const double m = kd + 1.0;
            // k^(a-1) as k^a / k: the exponent a is exact, a-1 would not be
            const double pk = pow(kd, al) / kd;
            const double pm = pow(m, al) / m;
            bk = pk * series_b(al, u);
            ak = 2.0 * pm * series_a(al + 1.0, 1.0 / m);
            ck = pk * series_c(al, u);
        }
        b[k] = bk * g1inv;
        a[k] = ak * g2inv;
        c[k] = ck * g2inv;
    }
}

// Gamma(alpha+1), Gamma(alpha+2) on the device, written to g[0], g[1].
__global__ void k_gammas(double al, double* g)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        g[0] = tgamma(al + 1.0);
        g[1] = tgamma(al + 2.0);
    }
}

// Reduced copies of b and a for the far field: float, and the bf16 split
// terms (see bf16_split3).  Any output pointer may be null.
__global__ __launch_bounds__(256) void k_weights_lowp(int64_t n, const double* __restrict__ b,
                                                      const double* __restrict__ a, float* b32,
                                                      float* a32, uint16_t* bh0, uint16_t* bh1,
                                                      uint16_t* bh2, uint16_t* ah0, uint16_t* ah1,
                                                      uint16_t* ah2)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const double bk = b[k], ak = a[k];
        if (b32) b32[k] = (float)bk;
        if (a32) a32[k] = (float)ak;
        if (bh0) {
            uint16_t t[3];
            bf16_split3(bk, t);
            bh0[k] = t[0];
            bh1[k] = t[1];
            if (bh2) bh2[k] = t[2];
            bf16_split3(ak, t);
            ah0[k] = t[0];
            ah1[k] = t[1];
            if (ah2) ah2[k] = t[2];
        }
    }
}

}  // namespace

hipError_t launch_weights_lowp(int64_t n, const double* b, const double* a, float* b32, float* a32,
                               uint16_t* const* bh, uint16_t* const* ah, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_weights_lowp, dim3((unsigned)blocks), dim3(256), 0, st, n, b, a, b32, a32,
                       bh[0], bh[1], bh[2], ah[0], ah[1], ah[2]);
    return hipGetLastError();
}

hipError_t launch_weights(double alpha, int64_t n, double* gam, double* b, double* a, double* c,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_gammas, dim3(1), dim3(64), 0, st, alpha, gam);
    if (n <= 0) return hipGetLastError();
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_weights, dim3((unsigned)blocks), dim3(256), 0, st, alpha, n, gam, b, a,
                       c);
    return hipGetLastError();
}

}  // namespace abm
