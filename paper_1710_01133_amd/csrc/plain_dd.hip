// The plain per-step method in double-double: the library's counterpart of
// the paper's long-double runs (Section "Memory saving improves computing
// time": the same computation in a wider type, at a higher cost).  Every
// quantity of the scheme is a double-double (dd.h, about 106 significant
// bits): the weights b_k, a_k, c_k, Gamma(alpha+1), Gamma(alpha+2), h^alpha,
// t_s = s h, the history f_k, both history sums, the state and the right-hand
// side (with the forcing cos / sin).  The sums and the update are those of the
// double kernels in plain.hip (Section 2, eq. abm and the corrector; the
// decomposition of Algorithm 1), with double-double operations:
//   * k_weights_dd: the cancellation-free binomial series of the double weight
//     kernel, u = 1/k, in double-double;
//   * k_plain_single_dd: one workgroup, weights stationary in registers, the
//     history in LDS (short histories);
//   * k_plain_dd: G cooperative workgroups, block-cyclic history slices in LDS,
//     one published partial per workgroup and step, the all-reduce pipelined
//     four steps ahead as in k_plain, and the update taken redundantly by
//     every workgroup.
// Tables and outputs are (hi, lo) pairs of doubles.
#include "abm_dev.h"
#include "abm_kernels.h"
#include "dd.h"

namespace abm {

namespace {

// ------------------------------------------------------------------ weights
// C(al, j) u^(j-1) summed over j >= 1 (al as a pair: al + 1 need not be a double)
__host__ __device__ dd series_b_dd(dd al, dd u)
{
    dd coef = al, up = dd_make(1.0), s = dd_make(0.0);
    for (int j = 1; j < 400; ++j) {
        const dd term = dd_mul(coef, up);
        s = dd_add(s, term);
        if (fabs(term.hi) <= 1e-34 * fabs(s.hi)) break;
        coef = dd_div(dd_mul(coef, dd_add_d(al, -(double)j)), dd_make(j + 1.0));   // C(al, j+1)
        up = dd_mul(up, u);
    }
    return s;
}

// C(be, 2j) u^(2j-2) summed over j >= 1
__host__ __device__ dd series_a_dd(dd be, dd u)
{
    dd c2 = dd_ldexp(dd_mul(be, dd_add_d(be, -1.0)), -1);   // C(be, 2)
    const dd u2 = dd_mul(u, u);
    dd up = dd_make(1.0), s = dd_make(0.0);
    for (int j = 1; j < 400; ++j) {
        const dd term = dd_mul(c2, up);
        s = dd_add(s, term);
        if (fabs(term.hi) <= 1e-34 * fabs(s.hi) || c2.hi == 0.0) break;
        // C(be, 2j+2) = C(be, 2j) (be-2j)(be-2j-1) / ((2j+1)(2j+2))
        c2 = dd_div(dd_mul(c2, dd_mul(dd_add_d(be, -2.0 * j), dd_add_d(be, -2.0 * j - 1.0))),
                    dd_make((2.0 * j + 1.0) * (2.0 * j + 2.0)));
        up = dd_mul(up, u2);
    }
    return s;
}

// -(C(al, j) - al C(al, j-1)) u^(j-2) summed over j >= 2
__host__ __device__ dd series_c_dd(dd al, dd u)
{
    dd cj1 = al;                                             // C(al, 1)
    dd cj = dd_ldexp(dd_mul(al, dd_add_d(al, -1.0)), -1);    // C(al, 2)
    dd up = dd_make(1.0), s = dd_make(0.0);
    for (int j = 2; j < 400; ++j) {
        const dd term = dd_neg(dd_mul(dd_sub(cj, dd_mul(al, cj1)), up));
        s = dd_add(s, term);
        if (fabs(term.hi) <= 1e-34 * fabs(s.hi)) break;
        cj1 = cj;
        cj = dd_div(dd_mul(cj, dd_add_d(al, -(double)j)), dd_make(j + 1.0));
        up = dd_mul(up, u);
    }
    return s;
}

// Gamma(alpha+1), Gamma(alpha+2)
__host__ __device__ inline void gammas_dd(double alpha, dd* g1, dd* g2)
{
    const dd z = dd_add_d(dd_make(alpha), 1.0);
    *g1 = dd_gamma(z);
    *g2 = dd_mul(z, *g1);                                    // Gamma(a+2) = (a+1) Gamma(a+1)
}

// b_k Gamma(alpha+1), a_k Gamma(alpha+2), c_k Gamma(alpha+2) (Section 2's
// weights before their Gamma factors) by the binomial series in u = 1/k
__host__ __device__ inline void weights_dd_at(double alpha, int64_t k, dd* bk, dd* ak, dd* ck)
{
    const dd al = dd_make(alpha);
    const dd be = dd_add_d(al, 1.0);
    if (k <= 1) {
        const dd t2m1 = dd_expm1_series(dd_mul_d(dd_ln2(), alpha));   // 2^a - 1
        if (k == 0) {
            *bk = dd_make(1.0);
            *ak = dd_ldexp(t2m1, 1);                                   // 2^(a+1) - 2
            *ck = al;
        } else {
            *bk = t2m1;
            // 3^(a+1) - 2^(a+2) + 1 = 2^a * series in u = 1/2 around m = 2
            *ak = dd_mul(dd_add_d(t2m1, 1.0), series_a_dd(be, dd_make(0.5)));
            *ck = dd_sub(al, dd_mul(dd_add_d(dd_neg(al), 1.0), t2m1));  // a - (1-a)(2^a - 1)
        }
    } else {
        const dd kd = dd_make((double)k);
        const dd m = dd_make((double)(k + 1));
        const dd u = dd_div(dd_make(1.0), kd);
        // k^(a-1) as k^a / k (a - 1 would round)
        const dd pk = dd_div(dd_pow(kd, alpha), kd);
        const dd pm = dd_div(dd_pow(m, alpha), m);
        *bk = dd_mul(pk, series_b_dd(al, u));
        *ak = dd_ldexp(dd_mul(pm, series_a_dd(be, dd_div(dd_make(1.0), m))), 1);
        *ck = dd_mul(pk, series_c_dd(al, u));
    }
}

__device__ __forceinline__ void put(double* t, int64_t k, dd v)
{
    t[2 * k] = v.hi;
    t[2 * k + 1] = v.lo;
}

// gam: Gamma(alpha+1), Gamma(alpha+2) as pairs (4 doubles)
__global__ void k_gammas_dd(double alpha, double* gam)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        dd g1, g2;
        gammas_dd(alpha, &g1, &g2);
        put(gam, 0, g1);
        put(gam, 1, g2);
    }
}

__global__ __launch_bounds__(256) void k_weights_dd(double alpha, int64_t n, const double* gam,
                                                    double* b, double* a, double* c)
{
    const dd g1 = dd{gam[0], gam[1]}, g2 = dd{gam[2], gam[3]};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        dd bk, ak, ck;
        weights_dd_at(alpha, k, &bk, &ak, &ck);
        put(b, k, dd_div(bk, g1));
        put(a, k, dd_div(ak, g2));
        put(c, k, dd_div(ck, g2));
    }
}

// ------------------------------------------------------------------ f(t, y)
// sin and cos of the forcing's phase at t (Duffing: omega t, LCR: omega t);
// zero for the unforced systems
template <int R>
__device__ __forceinline__ void forcing_dd(const double* __restrict__ p, dd t, dd* sn, dd* cs)
{
    if constexpr (R == ABM_RHS_DUFFING) {
        dd_sincos(dd_mul_d(t, p[2]), sn, cs);
    } else if constexpr (R == ABM_RHS_LCR) {
        dd_sincos(dd_mul_d(t, p[1]), sn, cs);
    } else {
        *sn = *cs = dd_make(0.0);
    }
}

// f(t, y) with the forcing's sin and cos at t given (one evaluation serves
// the predictor's and the corrector's right-hand side of a step)
template <int R, int D>
__device__ __forceinline__ void rhs_dd_sc(const double* __restrict__ p, dd t, dd sn, dd cs, const dd* y, dd* f)
{
    if constexpr (R == ABM_RHS_LINEAR) {
        f[0] = dd_mul_d(y[0], -p[0]);
    } else if constexpr (R == ABM_RHS_DUFFING) {
        f[0] = y[1];
        const dd cube = dd_mul(dd_mul(y[0], y[0]), y[0]);
        f[1] = dd_add(dd_sub(dd_sub(dd_mul_d(y[1], -p[0]), y[0]), cube), dd_mul_d(cs, p[1]));
    } else if constexpr (R == ABM_RHS_LORENZ) {
        f[0] = dd_mul_d(dd_sub(y[1], y[0]), p[0]);
        f[1] = dd_sub(dd_mul(y[0], dd_add_d(dd_neg(y[2]), p[1])), y[1]);
        f[2] = dd_sub(dd_mul(y[0], y[1]), dd_mul_d(y[2], p[2]));
    } else if constexpr (R == ABM_RHS_POLY) {
        f[0] = dd_add_d(dd_mul_d(t, p[1]), p[0]);
    } else if constexpr (R == ABM_RHS_LCR) {
        const dd x = y[0];
        dd g;
        if (dd_le(x, -1.0))
            g = dd_add_d(dd_add_d(dd_mul_d(x, p[3]), -p[2]), p[3]);
        else if (dd_ge(x, 1.0))
            g = dd_add_d(dd_add_d(dd_mul_d(x, p[3]), p[2]), -p[3]);
        else
            g = dd_mul_d(x, p[2]);
        f[0] = dd_sub(y[1], g);
        f[1] = dd_add(dd_sub(dd_mul_d(y[1], -p[0]), y[0]), dd_mul_d(sn, p[4]));
    } else if constexpr (R == ABM_RHS_DIAG) {
        f[0] = dd_add_d(dd_mul_d(y[0], -p[0]), p[2]);
        f[1] = dd_add_d(dd_mul_d(y[1], -p[1]), p[3]);
    }
    (void)t;
    (void)sn;
    (void)cs;
}

template <int R, int D>
__device__ __forceinline__ void rhs_dd(const double* __restrict__ p, dd t, const dd* y, dd* f)
{
    dd sn, cs;
    forcing_dd<R>(p, t, &sn, &cs);
    rhs_dd_sc<R, D>(p, t, sn, cs, y, f);
}

// ------------------------------------------------------------------ reductions
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ dd dpp_dd(dd v)
{
    return dd{dpp_f64<CTRL, ROWS>(v.hi), dpp_f64<CTRL, ROWS>(v.lo)};
}

// lane l's value (l the same in every lane)
__device__ __forceinline__ double readlane_d(double v, int l)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum of a full wave's pairs (the DPP order of the double kernels); every
// lane gets lane 63's total.
__device__ __forceinline__ dd wave_sum_dd(dd v)
{
    v = dd_add(v, dpp_dd<0xB1, 0xF>(v));
    v = dd_add(v, dpp_dd<0x4E, 0xF>(v));
    v = dd_add(v, dpp_dd<0x141, 0xF>(v));
    v = dd_add(v, dpp_dd<0x140, 0xF>(v));
    v = dd_add(v, dpp_dd<0x142, 0xA>(v));
    v = dd_add(v, dpp_dd<0x143, 0xC>(v));
    return dd{readlane_d(v.hi, 63), readlane_d(v.lo, 63)};
}

__device__ __forceinline__ dd ld(const double* t, int64_t k) { return dd{t[2 * k], t[2 * k + 1]}; }

// The forcing depends on t only: the updating wave evaluates it for 64 steps
// at a time, step s0 + l in lane l (s0 = 1, 65, 129, ..), and a step reads
// its lane's values; the same operations as one evaluation per step.
template <int R>
constexpr bool forced_dd() { return R == ABM_RHS_DUFFING || R == ABM_RHS_LCR; }

template <int R>
struct ForcingBlock {
    dd sn, cs;
    // call with every lane of the wave at each step s = 1, 2, ..
    __device__ __forceinline__ void step(const PlainArgs& A, int64_t s, int lane, dd* s_sn, dd* s_cs)
    {
        if constexpr (forced_dd<R>()) {
            const int j = (int)((s - 1) & 63);
            if (j == 0) forcing_dd<R>(A.p, two_prod((double)(s + lane), A.h), &sn, &cs);
            *s_sn = dd{readlane_d(sn.hi, j), readlane_d(sn.lo, j)};
            *s_cs = dd{readlane_d(cs.hi, j), readlane_d(cs.lo, j)};
        } else {
            *s_sn = *s_cs = dd_make(0.0);
        }
    }
};

// Index of the state written after step s (stride 0: the final state only), or -1.
__device__ __forceinline__ int64_t out_index(int64_t s, int64_t N, int64_t stride)
{
    if (stride == 0) return s == N ? 0 : -1;
    if (s % stride == 0) return s / stride;
    return s == N ? s / stride + 1 : -1;
}

// Step s's update (eq. abm and the corrector) from the totals P = tot[0..D),
// C = tot[D..2D) (every history term but c_n f_0) and the forcing's sin and
// cos at t_s: writes y and f_s.
template <int R, int D, bool PC>
__device__ __forceinline__ void update_dd(const PlainArgs& A, int64_t s, const dd* tot, const dd* ha,
                                          const dd* g2, const bool* deriv, const dd* cn, const dd* F0,
                                          dd sn, dd cs, dd* y, dd* fs)
{
    const dd td = two_prod((double)s, A.h);                 // t_s = s h, exactly
    dd base[D];
#pragma unroll
    for (int i = 0; i < D; ++i)
        base[i] = deriv[i] ? dd_add(dd_make(A.x0[i]), dd_mul_d(td, A.x1[i])) : dd_make(A.x0[i]);
    dd yP[D], fP[D];
#pragma unroll
    for (int i = 0; i < D; ++i) yP[i] = dd_add(base[i], dd_mul(ha[i], tot[i]));
    rhs_dd_sc<R, D>(A.p, td, sn, cs, yP, fP);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const dd corr = dd_add(dd_add(tot[D + i], dd_mul(cn[PC ? i : 0], F0[i])), dd_div(fP[i], g2[i]));
        y[i] = dd_add(base[i], dd_mul(ha[i], corr));
    }
    rhs_dd_sc<R, D>(A.p, td, sn, cs, y, fs);
}

// Scalar factors of each component: h^alpha, Gamma(alpha+2), start-term flag.
template <int D, bool PC>
__device__ __forceinline__ void factors_dd(const PlainArgs& A, dd* ha, dd* g2, bool* deriv)
{
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const int w = PC ? i : 0;
        ha[i] = dd_pow(dd_make(A.h), A.alpha[w]);
        g2[i] = ld(A.gam[w], 1);
        deriv[i] = A.alpha[w] > 1.0;
    }
}

template <int D>
__device__ __forceinline__ void write_out_dd(const PlainArgs& A, int64_t s, const dd* y)
{
    const int64_t w = out_index(s, A.N, A.out_stride);
    if (w >= 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            A.y_out[2 * (w * D + i)] = y[i].hi;
            A.y_out[2 * (w * D + i) + 1] = y[i].lo;
        }
    }
}

// ------------------------------------------------------------------ one workgroup
// As k_plain_single (plain.hip) with pairs: work thread u holds the pairs
// b_j, a_j, j = u + 448 q, the update wave adds the j = 0 terms.
constexpr int kSdThreads = 512;
constexpr int kSdWork = kSdThreads - kWave;                  // 448
constexpr int kSdWaves = kSdWork / kWave;                    // 7
constexpr size_t kSdLds = 160 * 1024;
// most weight pairs per thread that stay in registers: NJ tables max(d, 2) <= 18
constexpr int single_dd_max_nj(int d, int tables) { return 18 / (tables * (d > 2 ? d : 2)); }

size_t single_dd_lds(int64_t N, int d)
{
    return ((size_t)N * d * 2 + 2 * kSdWaves * 2 * d * 2) * sizeof(double);
}

template <int R, int D, bool PC, int NJ>
__global__ __launch_bounds__(kSdThreads) void k_plain_single_dd(PlainArgs A)
{
    extern __shared__ double sm[];
    dd* Fl = reinterpret_cast<dd*>(sm);                        // [N][D] f_0 .. f_{N-1}
    dd* red = Fl + (size_t)A.N * D;                            // [2][7][2D] by step parity
    constexpr int NW = PC ? D : 1;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int64_t N = A.N;

    dd wb[NJ][NW], wa[NJ][NW];
    dd ha[D], g2[D], F0[D], Fn[D], cn[NW], b0[NW], a0[NW];
    bool deriv[D];
    ForcingBlock<R> fb{};
    if (wid == 0) {
        factors_dd<D, PC>(A, ha, g2, deriv);
        dd x0[D];
#pragma unroll
        for (int i = 0; i < D; ++i) x0[i] = dd_make(A.x0[i]);
        rhs_dd<R, D>(A.p, dd_make(0.0), x0, F0);
#pragma unroll
        for (int i = 0; i < D; ++i) Fn[i] = F0[i];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            cn[w] = ld(A.c[w], 0);
            b0[w] = ld(A.b[w], 0);
            a0[w] = ld(A.a[w], 0);
        }
        if (lane == 0) {
#pragma unroll
            for (int i = 0; i < D; ++i) Fl[i] = F0[i];
            if (A.out_stride > 0) write_out_dd<D>(A, 0, x0);
        }
    } else {
        const int u = t - kWave;
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
            const int j = u + kSdWork * q;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                wb[q][w] = j < N ? ld(A.b[w], j) : dd_make(0.0);
                wa[q][w] = j < N ? ld(A.a[w], j) : dd_make(0.0);
            }
        }
    }
    __syncthreads();

    for (int64_t s = 1; s <= N; ++s) {
        const int64_t n = s - 1;
        dd* rp = red + (size_t)(s & 1) * kSdWaves * 2 * D;
        if (wid != 0) {
            const int u = t - kWave, nn = (int)n;
            dd P[D], C[D];
#pragma unroll
            for (int i = 0; i < D; ++i) P[i] = C[i] = dd_make(0.0);
#pragma unroll
            for (int q = 0; q < NJ; ++q) {
                const int j = u + kSdWork * q;
                if (j >= 1 && j <= nn) {
                    const dd* f = Fl + (nn - j) * D;
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        P[i] = dd_fma(wb[q][PC ? i : 0], f[i], P[i]);
                        if (j <= nn - 1) C[i] = dd_fma(wa[q][PC ? i : 0], f[i], C[i]);   // k = n-j >= 1
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const dd ps = wave_sum_dd(P[i]);
                const dd cs = wave_sum_dd(C[i]);
                if (lane == 0) {
                    rp[(wid - 1) * 2 * D + i] = ps;
                    rp[(wid - 1) * 2 * D + D + i] = cs;
                }
            }
        }
        __syncthreads();
        if (wid == 0) {
            dd tot[2 * D];
#pragma unroll
            for (int j = 0; j < 2 * D; ++j) {
                dd acc = rp[j];
#pragma unroll
                for (int w = 1; w < kSdWaves; ++w) acc = dd_add(acc, rp[w * 2 * D + j]);
                tot[j] = acc;
            }
#pragma unroll
            for (int i = 0; i < D; ++i) {
                tot[i] = dd_fma(b0[PC ? i : 0], Fn[i], tot[i]);
                if (n >= 1) tot[D + i] = dd_fma(a0[PC ? i : 0], Fn[i], tot[D + i]);
            }
            dd y[D], fs[D], sn, cs;
            fb.step(A, s, lane, &sn, &cs);
            update_dd<R, D, PC>(A, s, tot, ha, g2, deriv, cn, F0, sn, cs, y, fs);
            if (s < N) {
#pragma unroll
                for (int w = 0; w < NW; ++w) cn[w] = ld(A.c[w], s);
            }
#pragma unroll
            for (int i = 0; i < D; ++i) Fn[i] = fs[i];
            if (lane == 0) {
                if (s < N) {
#pragma unroll
                    for (int i = 0; i < D; ++i) Fl[(size_t)s * D + i] = fs[i];
                }
                bool bad = false;
#pragma unroll
                for (int i = 0; i < D; ++i) bad |= !dd_isfinite(y[i]);
                if (bad) raise_status(A.status, kStatusNonFinite);
                write_out_dd<D>(A, s, y);
            }
        }
    }
}

// ------------------------------------------------------------------ cooperative
constexpr int kCdCh = 256;                 // history indices per chunk (= work threads)
constexpr int kCdThreads = kCdCh + kWave;  // + the synchronising wave
constexpr int kCdWorkWaves = kCdCh / kWave;
constexpr int kCdPartStride = 16;          // doubles per partial slot (2D pairs, D <= 3)
constexpr int kCdLook = 4;                 // steps between a slice sum and its use
constexpr int kCdSlots = 8;                // partial slots, by step mod kCdSlots
constexpr int kCdGLanes = 4;               // workgroups per lane of the synchronising wave (G <= 256)
constexpr size_t kCdLds = 160 * 1024 - 256;

// pairs of LDS beside the history slice: the work-wave partials of kCdSlots
// steps, b_0 .. b_3, a_0 .. a_3 of each weight table and the gathered totals
// of two steps
constexpr size_t cd_extra_pairs(int d, int tables)
{
    return (size_t)kCdSlots * kCdWorkWaves * 2 * d + 2 * kCdLook * tables + 2 * 2 * d;
}
constexpr int kCdGather = kCdWorkWaves - 2;   // work waves 2 and 3 also gather the partials (G <= 64; above, wave 3 alone)

// As k_plain (plain.hip) with pairs, and the same pipelining of the
// all-reduce: the slice sums of step s+4 over the indices k <= s-1 are taken
// during step s and published right after it; the synchronising wave adds
// the kCdLook newest terms, b_3 f_{s-4} + .. + b_0 f_{s-1} (a_j likewise),
// from its own updates and takes the update.  The double-double sum over the
// workgroups' partials is moved off its path: after its own slice sums, work
// wave 3 adds up step s+1's partials (loaded during step s-1) into LDS for
// the synchronising wave's next step, checks the flags of step s+2 (loaded
// during step s-1), loads step s+2's partials and step s+3's flags; with at
// most 64 workgroups (one per lane) waves 2 and 3 share this, the predictor
// and the corrector sums.
// NLP > 0 (one weight table, at most NLP local chunks): the weights of the
// coming step are loaded into registers during the current one; NLP = 0:
// loaded in the step.
template <int R, int D, bool PC, int NLP>
__global__ __launch_bounds__(kCdThreads) void k_plain_dd(PlainArgs A)
{
    static_assert(NLP == 0 || !PC, "prefetched weights: one weight table");
    constexpr int NW = PC ? D : 1;
    extern __shared__ double sm[];
    dd* Fl = reinterpret_cast<dd*>(sm);                        // [nloc][256][D] history slice
    dd* red = Fl + (size_t)A.nloc * kCdCh * D;                 // [kCdSlots][4][2D] work-wave partials by step mod kCdSlots
    dd* wn = red + (size_t)kCdSlots * kCdWorkWaves * 2 * D;    // [kCdLook][NW] b_j, then [kCdLook][NW] a_j
    dd* gtot = wn + 2 * kCdLook * NW;                          // [2][2D] gathered totals by step parity
    __shared__ int s_abort;
    const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const bool sync_wave = wid == kCdWorkWaves;
    const int G = A.G, nloc = A.nloc;
    const int64_t N = A.N;

    dd ha[D], g2[D], F0[D];
    bool deriv[D];
    factors_dd<D, PC>(A, ha, g2, deriv);
    {
        dd x0[D];
#pragma unroll
        for (int i = 0; i < D; ++i) x0[i] = dd_make(A.x0[i]);
        rhs_dd<R, D>(A.p, dd_make(0.0), x0, F0);
        if (t == 0) s_abort = 0;
        if (sync_wave && lane == 0 && g == 0) {
#pragma unroll
            for (int i = 0; i < D; ++i) Fl[i] = F0[i];       // f_0: chunk 0, local chunk 0, thread 0
            if (A.out_stride > 0) write_out_dd<D>(A, 0, x0);
        }
    }
    // weights b_{m-k}, a_{m-k} of this thread's indices k for the slice sums
    // of step m+1 (index clamped at 0 where k > m: those are not used)
    constexpr int NLPR = NLP > 0 ? NLP : 1;
    dd wbp[NLPR], wap[NLPR];
    auto fetch = [&](int64_t m) {
#pragma unroll
        for (int l = 0; l < NLP; ++l) {
            const int64_t k = (int64_t)(g + l * G) * kCdCh + t;
            const int64_t idx = m - k < 0 ? 0 : m - k;
            wbp[l] = ld(A.b[0], idx);
            wap[l] = ld(A.a[0], idx);
        }
    };
    // synchronising wave: c_n of the coming step and the kCdLook newest
    // history rows (Fm[j] = f_{s-1-j}); gathering wave: per lane the loaded
    // partials (pl) and flags (fl) of workgroups lane, lane + 64, ..
    dd cn[NW], Fm[kCdLook][D];
    dd pl[kCdGLanes][2 * D];
    uint32_t fl[kCdGLanes];
    ForcingBlock<R> fb{};
#pragma unroll
    for (int r = 0; r < kCdGLanes; ++r) {
        fl[r] = 0u;
#pragma unroll
        for (int j = 0; j < 2 * D; ++j) pl[r][j] = dd_make(0.0);
    }
    if (!sync_wave) {
        if constexpr (NLP > 0) fetch(kCdLook);
    } else {
#pragma unroll
        for (int w = 0; w < NW; ++w) cn[w] = ld(A.c[w], 0);
        if (lane < kCdLook * NW) {
            const int j = lane / NW, w = lane % NW;
            wn[lane] = ld(A.b[w], j);
            wn[kCdLook * NW + lane] = ld(A.a[w], j);
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            Fm[0][i] = F0[i];
#pragma unroll
            for (int j = 1; j < kCdLook; ++j) Fm[j][i] = dd_make(0.0);
        }
    }
    __syncthreads();

    for (int64_t s = 1; s <= N; ++s) {
        const int64_t n = s - 1;
        // work-wave partials of step m in LDS slot m mod kCdSlots: written
        // during step m-kCdLook, read during step m (a single workgroup) or
        // published right after step m-kCdLook (several)
        if (sync_wave) {
            dd sn, cs;                                         // the forcing at t_s
            fb.step(A, s, lane, &sn, &cs);
            dd tot[2 * D];
            if (s <= kCdLook) {
#pragma unroll
                for (int j = 0; j < 2 * D; ++j) tot[j] = dd_make(0.0);   // no history before f_{s-kCdLook}
            } else if (G == 1) {
                const dd* rr = red + (size_t)(s % kCdSlots) * kCdWorkWaves * 2 * D;
#pragma unroll
                for (int j = 0; j < 2 * D; ++j)
                    tot[j] = dd_add(dd_add(dd_add(rr[j], rr[2 * D + j]), rr[4 * D + j]), rr[6 * D + j]);
            } else {
                const dd* gt = gtot + (s & 1) * 2 * D;        // gathered during step s-1
#pragma unroll
                for (int j = 0; j < 2 * D; ++j) tot[j] = gt[j];
            }
            // the kCdLook newest terms, oldest first: k = n-j with weights
            // b_j (k >= 0) and a_j (k >= 1); the k = 0 corrector term is
            // c_n f_0
#pragma unroll
            for (int j = kCdLook - 1; j >= 0; --j) {
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const int w = PC ? i : 0;
                    if (n >= j) tot[i] = dd_fma(wn[j * NW + w], Fm[j][i], tot[i]);
                    if (n >= j + 1) tot[D + i] = dd_fma(wn[(kCdLook + j) * NW + w], Fm[j][i], tot[D + i]);
                }
            }
            dd y[D], fs[D];
            update_dd<R, D, PC>(A, s, tot, ha, g2, deriv, cn, F0, sn, cs, y, fs);
#pragma unroll
            for (int i = 0; i < D; ++i) {
#pragma unroll
                for (int j = kCdLook - 1; j >= 1; --j) Fm[j][i] = Fm[j - 1][i];
                Fm[0][i] = fs[i];
            }
            if (s < N) {
#pragma unroll
                for (int w = 0; w < NW; ++w) cn[w] = ld(A.c[w], s);
            }
            if (lane == 0) {
                if (s < N) {
                    const int64_t cs = s / kCdCh;
                    if ((int)(cs % G) == g) {
                        dd* dst = Fl + ((size_t)(cs / G) * kCdCh + (s % kCdCh)) * D;
#pragma unroll
                        for (int i = 0; i < D; ++i) dst[i] = fs[i];
                    }
                }
                if (g == 0) {
                    bool bad = false;
#pragma unroll
                    for (int i = 0; i < D; ++i) bad |= !dd_isfinite(y[i]);
                    if (bad) raise_status(A.status, kStatusNonFinite);
                    write_out_dd<D>(A, s, y);
                }
            }
        } else {
            if (s + kCdLook <= N) {
                // slice sums of step s+4 over this thread's indices k <= s-1:
                // b_{s+3-k} f_k and, for k >= 1, a_{s+3-k} f_k
                dd* rw = red + (size_t)((s + kCdLook) % kCdSlots) * kCdWorkWaves * 2 * D;
                dd P[D], C[D];
#pragma unroll
                for (int i = 0; i < D; ++i) P[i] = C[i] = dd_make(0.0);
                if constexpr (NLP > 0) {
#pragma unroll
                    for (int l = 0; l < NLP; ++l) {
                        const int64_t k = (int64_t)(g + l * G) * kCdCh + t;
                        if (l < nloc && k <= n) {
                            const dd* f = Fl + ((size_t)l * kCdCh + t) * D;
#pragma unroll
                            for (int i = 0; i < D; ++i) {
                                P[i] = dd_fma(wbp[l], f[i], P[i]);
                                if (k >= 1) C[i] = dd_fma(wap[l], f[i], C[i]);   // k = 0: c_n
                            }
                        }
                    }
                    fetch(s + kCdLook);    // in flight while the step is synchronised
                } else {
                    for (int l = 0; l < nloc; ++l) {
                        const int64_t k = (int64_t)(g + l * G) * kCdCh + t;
                        if (k > n) break;               // later local chunks lie further out
                        const dd* f = Fl + ((size_t)l * kCdCh + t) * D;
#pragma unroll
                        for (int i = 0; i < D; ++i) {
                            const int w = PC ? i : 0;
                            P[i] = dd_fma(ld(A.b[w], s + kCdLook - 1 - k), f[i], P[i]);
                            if (k >= 1) C[i] = dd_fma(ld(A.a[w], s + kCdLook - 1 - k), f[i], C[i]);   // k = 0: c_n
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const dd ps = wave_sum_dd(P[i]);
                    const dd cs = wave_sum_dd(C[i]);
                    if (lane == 0) {
                        rw[wid * 2 * D + i] = ps;
                        rw[wid * 2 * D + D + i] = cs;
                    }
                }
            }
            // with one workgroup per lane (G <= 64) waves 2 and 3 share the
            // gathering, the predictor sums (wave 2) and the corrector sums
            // (wave 3); with more, the flag polls of a second wave cost more
            // than the halved sums save, and wave 3 gathers both
            const bool split = G <= kWave;
            if (G > 1 && (wid == kCdWorkWaves - 1 || (split && wid == kCdGather))) {
                const int v0 = split ? (wid - kCdGather) * D : 0;   // this wave's first value
                const int nv = split ? D : 2 * D;                   // and its count
                // step s+1's partials (loaded during step s-1), in a fixed
                // order, for the synchronising wave's next step
                if (s + 1 > kCdLook && s + 1 <= N) {
                    dd* gt = gtot + ((s + 1) & 1) * 2 * D + v0;
#pragma unroll
                    for (int j = 0; j < 2 * D; ++j) {
                        if (j >= nv) break;
                        dd acc = dd_make(0.0);
#pragma unroll
                        for (int r = 0; r < kCdGLanes; ++r)
                            if (lane + kWave * r < G) acc = dd_add(acc, pl[r][j]);
                        acc = wave_sum_dd(acc);
                        if (lane == 0) gt[j] = acc;
                    }
                }
                bool ok = true;
                if (s + 2 > kCdLook && s + 2 <= N) {
                    // every workgroup has published step s+2 (after its step
                    // s+2-kCdLook): checked on the flags loaded during step s-1
                    const uint32_t m2 = (uint32_t)(s + 2) + A.wait_bias;
#pragma unroll
                    for (int r = 0; r < kCdGLanes; ++r) {
                        const int q = lane + kWave * r;
                        if (q < G) {
                            uint32_t spins = 0;
                            while (fl[r] < m2) {
                                if (++spins > A.spin_limit) {
                                    ok = false;
                                    break;
                                }
                                spin_pause();
                                fl[r] = ld_relaxed(&A.flags[q]);
                            }
                        }
                    }
                    // the partials of step s+2, loaded with device-coherent
                    // loads issued after every flag load has returned s+2:
                    // each writer's release made its partials visible before
                    // its flag, so no acquire fence (which would invalidate
                    // this XCD's L2 every step) is needed
                    if (ok) {
                        const double* slot_base = A.part + (size_t)((s + 2) % kCdSlots) * G * kCdPartStride;
#pragma unroll
                        for (int r = 0; r < kCdGLanes; ++r) {
                            const int q = lane + kWave * r;
                            if (q < G) {
                                const double* sl = slot_base + (size_t)q * kCdPartStride + 2 * v0;
#pragma unroll
                                for (int j = 0; j < 2 * D; ++j)
                                    if (j < nv) pl[r][j] = dd{ld_relaxed(&sl[2 * j]), ld_relaxed(&sl[2 * j + 1])};
                            }
                        }
                    }
                }
                // the flags of step s+3, checked at step s+1
                if (s + 3 > kCdLook && s + 3 <= N) {
#pragma unroll
                    for (int r = 0; r < kCdGLanes; ++r)
                        if (lane + kWave * r < G) fl[r] = ld_relaxed(&A.flags[lane + kWave * r]);
                }
                if (__ballot(!ok) != 0) {
                    if (lane == 0) {
                        raise_status(A.status, kStatusTimeout);
                        s_abort = 1;
                        // the run is incomplete: its final state reads NaN
                        if (g == 0) {
                            const int64_t last = A.out_stride == 0 ? 0 : N / A.out_stride + (N % A.out_stride ? 1 : 0);
#pragma unroll
                            for (int i = 0; i < D; ++i) {
                                A.y_out[2 * (last * D + i)] = __builtin_nan("");
                                A.y_out[2 * (last * D + i) + 1] = __builtin_nan("");
                            }
                        }
                    }
                }
            }
        }
        // f_s is stored, step s+4's work-wave partials and step s+1's
        // gathered totals are in LDS
        __syncthreads();
        if (s_abort) return;
        // work wave 0 publishes the workgroup's slice sums of step s+4 and
        // raises its flag to s+4 (slots by step mod kCdSlots)
        if (G > 1 && t == 0 && s + kCdLook <= N) {
            const dd* rw = red + (size_t)((s + kCdLook) % kCdSlots) * kCdWorkWaves * 2 * D;
            double* slot = A.part + ((size_t)((s + kCdLook) % kCdSlots) * G + g) * kCdPartStride;
#pragma unroll
            for (int j = 0; j < 2 * D; ++j) {
                const dd v = dd_add(dd_add(dd_add(rw[j], rw[2 * D + j]), rw[4 * D + j]), rw[6 * D + j]);
                slot[2 * j] = v.hi;
                slot[2 * j + 1] = v.lo;
            }
            st_release(&A.flags[g], (uint32_t)(s + kCdLook));
        }
    }
}

template <int R, int D, bool PC, int NJ>
hipError_t launch_sd(const PlainArgs& A, hipStream_t st)
{
    const size_t shmem = single_dd_lds(A.N, D);
    const void* fn = reinterpret_cast<const void*>(&k_plain_single_dd<R, D, PC, NJ>);
    hipError_t e = allow_lds(fn, shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_plain_single_dd<R, D, PC, NJ>), dim3(1), dim3(kSdThreads), shmem, st, A);
    return hipGetLastError();
}

template <int R, int D, bool PC>
hipError_t launch_dd_t(const PlainArgs& A, bool single, hipStream_t st)
{
    if (single) {
        constexpr int MAXNJ = single_dd_max_nj(D, PC ? D : 1);
        const int64_t nj = (A.N + kSdWork - 1) / kSdWork;
        if constexpr (MAXNJ >= 2) {
            if (nj <= 2) return launch_sd<R, D, PC, 2>(A, st);
        }
        if constexpr (MAXNJ >= 4) {
            if (nj <= 4) return launch_sd<R, D, PC, 4>(A, st);
        }
        if constexpr (MAXNJ >= 8) {
            if (nj <= 8) return launch_sd<R, D, PC, 8>(A, st);
        }
        return hipErrorInvalidValue;
    }
    const size_t shmem = ((size_t)A.nloc * kCdCh * D + cd_extra_pairs(D, PC ? D : 1)) * 2 * sizeof(double);
    const void* fn = !PC && A.nloc <= 4 ? reinterpret_cast<const void*>(&k_plain_dd<R, D, false, 4>)
                                        : reinterpret_cast<const void*>(&k_plain_dd<R, D, PC, 0>);
    hipError_t e = allow_lds(fn, shmem);
    if (e != hipSuccess) return e;
    PlainArgs a = A;
    void* args[] = {&a};
    return hipLaunchCooperativeKernel(fn, dim3(A.G), dim3(kCdThreads), args, (unsigned)shmem, st);
}

}  // namespace

bool plain_dd_single_fits(int64_t N, int d, int tables)
{
    const int64_t nj = (N + kSdWork - 1) / kSdWork;
    int bucket = 0;
    for (int c : {2, 4, 8})
        if (c <= single_dd_max_nj(d, tables)) bucket = c;
    return nj <= bucket && single_dd_lds(N, d) <= kSdLds;
}

int plain_dd_max_local_chunks(int d)
{
    // the largest weight-table count a system of d components can have
    return (int)((kCdLds - cd_extra_pairs(d, d) * 2 * sizeof(double)) / ((size_t)kCdCh * d * 2 * sizeof(double)));
}

int plain_dd_part_doubles(int G) { return kCdSlots * G * kCdPartStride; }

hipError_t launch_weights_dd(double alpha, int64_t n, double* gam, double* b, double* a, double* c,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_gammas_dd, dim3(1), dim3(64), 0, st, alpha, gam);
    if (n <= 0) return hipGetLastError();
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_weights_dd, dim3((unsigned)blocks), dim3(256), 0, st, alpha, n, gam, b, a, c);
    return hipGetLastError();
}

hipError_t launch_plain_dd(const PlainArgs& A, bool single, int kind, hipStream_t st)
{
    switch (kind) {
    case ABM_RHS_LINEAR: return launch_dd_t<ABM_RHS_LINEAR, 1, false>(A, single, st);
    case ABM_RHS_DUFFING: return launch_dd_t<ABM_RHS_DUFFING, 2, false>(A, single, st);
    case ABM_RHS_LORENZ: return launch_dd_t<ABM_RHS_LORENZ, 3, false>(A, single, st);
    case ABM_RHS_POLY: return launch_dd_t<ABM_RHS_POLY, 1, false>(A, single, st);
    case ABM_RHS_LCR: return launch_dd_t<ABM_RHS_LCR, 2, false>(A, single, st);
    case ABM_RHS_DIAG: return launch_dd_t<ABM_RHS_DIAG, 2, false>(A, single, st);
    case kRhsCount + ABM_RHS_DUFFING: return launch_dd_t<ABM_RHS_DUFFING, 2, true>(A, single, st);
    case kRhsCount + ABM_RHS_LORENZ: return launch_dd_t<ABM_RHS_LORENZ, 3, true>(A, single, st);
    case kRhsCount + ABM_RHS_LCR: return launch_dd_t<ABM_RHS_LCR, 2, true>(A, single, st);
    case kRhsCount + ABM_RHS_DIAG: return launch_dd_t<ABM_RHS_DIAG, 2, true>(A, single, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace abm
