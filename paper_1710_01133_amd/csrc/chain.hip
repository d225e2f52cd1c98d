// K3: near band and predictor/corrector chain of the blocked method.
//
// One wavefront advances one trajectory through block m (rows r = 0..L-1,
// step s = mL + r + 1, n = s - 1).  The far-field product of block m covers
// the history k = 1..(m-1)L, so it can run while block m-1 is still being
// stepped; everything newer is handled here.  Lane l owns the rows
// r of block m and of block m+1 and keeps, per row and component,
//   accP = sum_k b_{n-k} f_k   (predictor history sum of eq. abm)
//   accC = c_n f_0 + sum_{k>=1} a_{n-k} f_k   (corrector history sum)
// Block m's sums start as the far-field partials (added in order) plus the
// k = 0 terms plus what block m-1 scattered into them (history
// (m-1)L+1 .. mL); block m+1's sums start at zero.  Each new f_s is scattered
// into every later row of block m (weight index r' - r - 1) and into every row
// of block m+1 (weight index L + r'' - r - 1), so when row r comes up its sums
// are complete and are broadcast from the owning lane with readlane.  The
// update
//   yP = x0 + h^a accP,  y = x0 + h^a (accC + f(t_s, yP) / Gamma(a+2))
// is computed identically by every lane; the lane owning row r keeps f_s and
// y_s, and the wave writes them (and the reduced copies of f for the far
// field) 64 rows at a time, so no memory operation sits on the sequential
// path.  At the end of the block the next block's sums go to global memory.
#include "abm_dev.h"
#include "abm_kernels.h"

namespace abm {

namespace {

// Per-wave view of one chain work item.
struct ChainArgs {
    gptr<const double> b[4];   // component i's tables (component 0's unless per-component)
    gptr<const double> a[4];
    gptr<const double> c[4];
    gptr<const double> gam[4];
    double alpha[4];
    gptr<double> F;
    gptr<float> F32;
    gptr<uint16_t> Fhi;
    gptr<uint16_t> Fmid;
    gptr<uint16_t> Flo;
    gptr<float> Fsc;       // non-null: fp16 split (Fhi, Fmid) with per-32-row scales
    gptr<int8_t> Fq[3];    // non-null: int8 limbs of the history, one scale per block
    gptr<double> Fqs;
    int64_t ldF;
    int64_t rows;
    bool narrow;           // F32 time-major [k][ldF] instead of column-blocked
    gptr<const double> part;
    int64_t ldP;
    int64_t mL;
    int32_t nchunks;
    gptr<double> accn;     // this member's carried sums [2][d][L]
};

template <int L>
__device__ __forceinline__ void chain_view(const GroupDev& G, const ChainItem& it, int D,
                                           ChainArgs& A)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        A.b[i] = as_global(G.w[i].b);
        A.a[i] = as_global(G.w[i].a);
        A.c[i] = as_global(G.w[i].c);
        A.gam[i] = as_global(G.w[i].gam);
        A.alpha[i] = G.w[i].alpha;
    }
    A.F = as_global(G.F);
    A.F32 = as_global(G.F32);
    A.Fhi = as_global(G.Fh[0]);
    A.Fmid = as_global(G.Fh[1]);
    A.Flo = as_global(G.Fh[2]);
    A.Fsc = as_global(G.Fsc);
#pragma unroll
    for (int i = 0; i < 3; ++i) A.Fq[i] = as_global(G.Fq[i]);
    A.Fqs = as_global(G.Fqs);
    A.ldF = G.ldF;
    A.rows = G.rows;
    A.narrow = G.narrow != 0;
    A.part = as_global((const double*)G.part[(it.mL / L) & 1]);
    A.ldP = it.ldP;
    A.mL = it.mL;
    A.nchunks = it.nsplit;
    A.accn = as_global(G.accn) + (size_t)it.member * 2 * D * L;
}

__device__ __forceinline__ double readlane_d(double v, int l)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// History column of component i of a trajectory.
__device__ __forceinline__ int64_t comp_col(const TrajDesc& T, int i)
{
    return (int64_t)T.col0 + (int64_t)i * T.cstride;
}

// Exponents of the fp16 split of the history: rows 32g+1 .. 32g+32 of a
// column are stored as f * 2^e with e such that the largest |f| of the 32 rows
// lies in [2^13, 2^14) (e = 0 for an all-zero group; |e| <= 100).  m: that
// largest |f|.
__device__ __forceinline__ int f16_exponent(double m)
{
    if (!(m > 0.0) || !isfinite(m)) return 0;
    int ex;
    (void)frexp(m, &ex);                       // m = f 2^ex, 0.5 <= f < 1
    int e = 14 - ex;
    return e < -100 ? -100 : (e > 100 ? 100 : e);
}

// Exponent of the int8 limbs of the history: the rows of block m of a column
// are stored as f 2^e.  The previous block's exponent (prev, from its
// recorded scale) is kept while the block's largest |f| times 2^prev lies in
// [16, 127) -- at most one bit below what a fresh scale gives, which puts that
// largest |f| in [32, 64) -- so that the far field can sum consecutive blocks
// exactly without converting in between (e = 0 for an all-zero or non-finite
// block).  A column tile's scales then change at a few percent of the block
// boundaries instead of about one in six with the band [32, 127).
__device__ __forceinline__ int q8_exponent(double m, double prev_scale)
{
    if (!(m > 0.0) || !isfinite(m)) return 0;
    if (prev_scale > 0.0) {
        int pe;
        (void)frexp(prev_scale, &pe);          // prev_scale = 2^-prev = 0.5 * 2^pe
        const double x = ldexp(m, 1 - pe);
        if (x >= 16.0 && x < 127.0) return 1 - pe;
    }
    int ex;
    (void)frexp(m, &ex);
    return 6 - ex;
}

// Row s of component i as three balanced base-256 digits of f 2^e at
// resolution 2^-16 (|f 2^e| < 127: |d0| <= 127, d1, d2 in [-128, 127]); the
// block's first row records the scale 2^-e.
template <int D>
__device__ __forceinline__ void store_history_q8(const ChainArgs& A, const TrajDesc& T, int64_t s,
                                                 int64_t block, bool first, const double* fs,
                                                 const int* q8e)
{
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const int64_t col = comp_col(T, i);
        const double x = ldexp(fs[i], q8e[i] + 16);
        int64_t I = isfinite(x) ? (int64_t)rint(x) : 0;
        const int64_t d2 = ((I + 128) & 255) - 128;
        I = (I - d2) >> 8;
        const int64_t d1 = ((I + 128) & 255) - 128;
        const int64_t d0 = (I - d1) >> 8;
        const int64_t at = q16_index(s, col, A.ldF);
        A.Fq[0][at] = (int8_t)d0;
        A.Fq[1][at] = (int8_t)d1;
        A.Fq[2][at] = (int8_t)d2;
        if (first) A.Fqs[block * A.ldF + col] = ldexp(1.0, -q8e[i]);
    }
}

template <int D>
__device__ __forceinline__ void store_history(const ChainArgs& A, const TrajDesc& T, int64_t s,
                                              const double* fs, const int* f16e)
{
    const int64_t row = s * A.ldF;
#pragma unroll
    for (int i = 0; i < D; ++i) A.F[row + comp_col(T, i)] = fs[i];
    if (A.F32) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int64_t at = A.narrow ? row + comp_col(T, i) : colblocked_index(s, comp_col(T, i), A.rows);
            A.F32[at] = (float)fs[i];
        }
    }
    if (A.Fhi && s >= 1) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int64_t at = kblocked_index(s, comp_col(T, i), A.ldF);
            if (A.Fsc) {
                // fp16 split of the scaled value: hi = fp16(x), lo = fp16(x - hi)
                const float x = (float)ldexp(fs[i], f16e[i]);
                const _Float16 hi = (_Float16)x;
                const _Float16 lo = (_Float16)(x - (float)hi);
                A.Fhi[at] = __builtin_bit_cast(uint16_t, hi);
                A.Fmid[at] = __builtin_bit_cast(uint16_t, lo);
                if (((s - 1) & 31) == 0)          // the group's first row records its scale
                    A.Fsc[((s - 1) >> 5) * A.ldF + comp_col(T, i)] = ldexpf(1.0f, -f16e[i]);
            } else {
                uint16_t t[3];
                bf16_split3(fs[i], t);
                A.Fhi[at] = t[0];
                A.Fmid[at] = t[1];
                if (A.Flo) A.Flo[at] = t[2];
            }
        }
    }
}

template <int D>
__device__ __forceinline__ void store_output(const TrajDesc& T, int64_t s, const double* y)
{
    int64_t w = -1;
    if (T.out_stride == 0) {
        if (s == T.N) w = 0;
    } else if (s % T.out_stride == 0) {
        w = s / T.out_stride;
    } else if (s == T.N) {
        w = s / T.out_stride + 1;
    }
    if (w >= 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) as_global(T.y_out)[w * D + i] = y[i];
    }
}

// W waves per workgroup: chains are latency-bound and register-heavy, so they
// are packed two waves per SIMD on as few CUs as possible, which leaves whole
// CUs to the far-field kernel running beside them.
// The block of one chain item, run by one wave (smw: that wave's 4L doubles
// of LDS per weight table in use).  PC: the components have orders of their
// own, each with its weight table, weight rings and scalar factors;
// otherwise all components share component 0's.
template <int R, int D, int L, bool PC>
__device__ __forceinline__ void chain_block(const GroupDev& G, const ChainItem& it, double* smw,
                                            int lane, uint32_t* status)
{
    constexpr int Q = L / 64;
    constexpr int NW = PC ? D : 1;            // weight tables in use
    ChainArgs A;
    chain_view<L>(G, it, D, A);
    const TrajDesc T = G.traj[it.member];
    // weight windows: table w's b[0..2L) at smw + 4Lw, a[0..2L) after it
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        double* swb = smw + (size_t)w * 4 * L;
        double* swa = swb + 2 * L;
        for (int x = lane; x < 2 * L; x += 64) {
            swb[x] = A.b[w][x];
            swa[x] = A.a[w][x];
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    const int64_t mL = A.mL;
    if (mL >= T.N) return;
    const int rows = (int)((T.N - mL) < L ? (T.N - mL) : L);
    // int8 limbs: the previous block's history scales (read now, used at the end)
    double q8prev[D];
#pragma unroll
    for (int i = 0; i < D; ++i)
        q8prev[i] = (A.Fq[0] && mL >= L) ? A.Fqs[(mL / L - 1) * A.ldF + comp_col(T, i)] : 0.0;
    const bool more = T.N > mL + L;           // a next block follows

    double x0[D], x1[D], F0[D], p[8];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        x0[i] = T.x0[i];
        x1[i] = T.x1[i];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) p[i] = T.p[i];
    const double h = T.h;
    const int deriv = G.deriv;                // components whose start term is x0 + t x1
    double ha[NW], g2inv[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        ha[w] = pow(h, A.alpha[w]);
        g2inv[w] = 1.0 / A.gam[w][1];
    }
#pragma unroll
    for (int i = 0; i < D; ++i) F0[i] = A.F[comp_col(T, i)];

    const int r0 = Q * lane;                  // first row of this lane
    // carried sums of block m (written by the previous block's chain)
    const gptr<double> accn = A.accn;
    double accP[Q][D], accC[Q][D], nxtP[Q][D], nxtC[Q][D];
    const size_t sstride = (size_t)A.ldP * (2 * L);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        // Partial slices added in slice order.  A lane's Q rows are adjacent
        // in a slice (Q even: 16-byte aligned pairs), so a slice is Q/2 pair
        // loads for the predictor rows and Q/2 for the corrector rows, four
        // slices in flight at a time.
        double sp[Q], sc[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) sp[q] = sc[q] = 0.0;
        const gptr<const double> pc0 = A.part + (size_t)comp_col(T, i) * (2 * L) + r0;
        auto load_rows = [&](size_t off, double* v) {
            if constexpr (Q % 2 == 0) {
                typedef double d2 __attribute__((ext_vector_type(2)));
                const gptr<const d2> src = (gptr<const d2>)(pc0 + off);
#pragma unroll
                for (int q = 0; q < Q / 2; ++q) {
                    const d2 x = src[q];
                    v[2 * q] = x[0];
                    v[2 * q + 1] = x[1];
                }
            } else {
#pragma unroll
                for (int q = 0; q < Q; ++q) v[q] = pc0[off + q];
            }
        };
        int ch = 0;
        for (; ch + 4 <= A.nchunks; ch += 4) {
            double vp[4][Q], vc[4][Q];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                load_rows((ch + u) * sstride, vp[u]);
                load_rows((ch + u) * sstride + L, vc[u]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    sp[q] += vp[u][q];
                    sc[q] += vc[u][q];
                }
        }
        for (; ch < A.nchunks; ++ch) {
            double vp[Q], vc[Q];
            load_rows(ch * sstride, vp);
            load_rows(ch * sstride + L, vc);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                sp[q] += vp[q];
                sc[q] += vc[q];
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = r0 + q;
            const int64_t n = mL + r;
            sp[q] += A.b[PC ? i : 0][n] * F0[i];
            sc[q] += A.c[PC ? i : 0][n] * F0[i];
            if (mL > 0) {
                sp[q] += accn[i * L + r];
                sc[q] += accn[(D + i) * L + r];
            }
            accP[q][i] = sp[q];
            accC[q][i] = sc[q];
            nxtP[q][i] = 0.0;
            nxtC[q][i] = 0.0;
        }
    }

    // forcing terms of this lane's rows, evaluated off the sequential chain
    double frc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) frc[q] = forcing<R>(p, (double)(mL + r0 + q + 1) * h);

    // weight rings (one set per table): at step r slot (x mod Q) holds w[x]
    // for x = r0-r-1 .. r0-r-2+Q (block m rows, zero for x < 0) and w[L + x]
    // (block m+1 rows)
    double rbc[NW][Q], rac[NW][Q], rbn[NW][Q], ran[NW][Q];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const double* swb = smw + (size_t)w * 4 * L;
        const double* swa = swb + 2 * L;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int x = r0 - 1 + i;
            const int sl = (x % Q + Q) % Q;
            rbc[w][sl] = x < 0 ? 0.0 : swb[x < 0 ? 0 : x];
            rac[w][sl] = x < 0 ? 0.0 : swa[x < 0 ? 0 : x];
            rbn[w][sl] = swb[L + x];
            ran[w][sl] = swa[L + x];
        }
    }

    double myF[Q][D], myY[Q][D];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < D; ++i) myF[q][i] = myY[q][i] = 0.0;

    for (int rb = 0; rb < rows; rb += Q) {
#pragma unroll
        for (int jq = 0; jq < Q; ++jq) {
            const int r = rb + jq;             // r mod Q == jq
            if (r < rows) {
                const int owner = r / Q;
                // the weights entering the rings after this step: x = r0 - r - 2
                const int xn = r0 - r - 2;
                double nbc[NW], nac[NW], nbn[NW], nan_[NW];
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    const double* swb = smw + (size_t)w * 4 * L;
                    const double* swa = swb + 2 * L;
                    nbc[w] = xn < 0 ? 0.0 : swb[xn < 0 ? 0 : xn];
                    nac[w] = xn < 0 ? 0.0 : swa[xn < 0 ? 0 : xn];
                    nbn[w] = swb[L + xn];
                    nan_[w] = swa[L + xn];
                }
                const int64_t s = mL + r + 1;
                // start term of eq. abm: x0, plus t_s x1 for orders above 1
                double base[D];
#pragma unroll
                for (int i = 0; i < D; ++i) base[i] = x0[i];
                if (deriv) {
                    const double ts = (double)s * h;
#pragma unroll
                    for (int i = 0; i < D; ++i)
                        if ((deriv >> i) & 1) base[i] = x0[i] + ts * x1[i];
                }
                double P[D], C[D], yP[D], fP[D], y[D], fs[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    P[i] = readlane_d(accP[jq][i], owner);
                    C[i] = readlane_d(accC[jq][i], owner);
                }
                const double force = readlane_d(frc[jq], owner);
#pragma unroll
                for (int i = 0; i < D; ++i) yP[i] = base[i] + ha[PC ? i : 0] * P[i];
                rhs_eval_forced<R, D>(p, yP, force, fP);
#pragma unroll
                for (int i = 0; i < D; ++i)
                    y[i] = base[i] + ha[PC ? i : 0] * (C[i] + fP[i] * g2inv[PC ? i : 0]);
                rhs_eval_forced<R, D>(p, y, force, fs);
                const bool mine = lane == owner;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    myF[jq][i] = mine ? fs[i] : myF[jq][i];
                    myY[jq][i] = mine ? y[i] : myY[jq][i];
                }
                // scatter f_s: row r0+q gets w[r0+q-r-1] (block m) and w[L+r0+q-r-1]
                // (block m+1); that weight sits in slot (q - jq - 1) mod Q
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int sl = ((q - jq - 1) % Q + Q) % Q;
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        const int w = PC ? i : 0;
                        accP[q][i] = fma(rbc[w][sl], fs[i], accP[q][i]);
                        accC[q][i] = fma(rac[w][sl], fs[i], accC[q][i]);
                        nxtP[q][i] = fma(rbn[w][sl], fs[i], nxtP[q][i]);
                        nxtC[q][i] = fma(ran[w][sl], fs[i], nxtC[q][i]);
                    }
                }
                // slide the rings: x = r0 - r - 2 replaces x = r0 - r - 2 + Q
                const int sn = ((-jq - 2) % Q + Q) % Q;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    rbc[w][sn] = nbc[w];
                    rac[w][sn] = nac[w];
                    rbn[w][sn] = nbn[w];
                    ran[w][sn] = nan_[w];
                }
            }
        }
    }

    // fp16 split: the scale of each 32-row group (32/Q consecutive lanes)
    int f16e[D];
#pragma unroll
    for (int i = 0; i < D; ++i) f16e[i] = 0;
    if (A.Fsc) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double m = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (r0 + q < rows) m = fmax(m, fabs(myF[q][i]));
#pragma unroll
            for (int x = 1; x < 32 / Q; x <<= 1) m = fmax(m, __shfl_xor(m, x, kWave));
            f16e[i] = f16_exponent(m);
        }
    }
    // int8 limbs: one scale per block and column (the whole wave's rows)
    int q8e[D];
#pragma unroll
    for (int i = 0; i < D; ++i) q8e[i] = 0;
    if (A.Fq[0]) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double m = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (r0 + q < rows) m = fmax(m, fabs(myF[q][i]));
#pragma unroll
            for (int x = 1; x < kWave; x <<= 1) m = fmax(m, __shfl_xor(m, x, kWave));
            q8e[i] = q8_exponent(m, q8prev[i]);
        }
    }
    // history rows, reduced copies and output states of this lane's rows
    bool bad = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int r = r0 + q;
        if (r < rows) {
            const int64_t s = mL + r + 1;
            store_history<D>(A, T, s, myF[q], f16e);
            if (A.Fq[0]) store_history_q8<D>(A, T, s, mL / L, r == 0, myF[q], q8e);
            store_output<D>(T, s, myY[q]);
#pragma unroll
            for (int i = 0; i < D; ++i) bad |= !isfinite(myY[q][i]);
        }
    }
    if (more) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int r = r0 + q;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                accn[i * L + r] = nxtP[q][i];
                accn[(D + i) * L + r] = nxtC[q][i];
            }
        }
    }
    if (bad) raise_status(G.status ? G.status : status, kStatusNonFinite);
}

template <int R, int D, int L, int W, bool PC>
__global__ __launch_bounds__(64 * W) void k_chain(const GroupDev* __restrict__ groups,
                                               const ChainItem* __restrict__ items, int nitems,
                                               uint32_t* status)
{
    extern __shared__ double smc[];           // per wave and table: b[0..2L), a[0..2L)
    constexpr int NW = PC ? D : 1;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int j = blockIdx.x * W + wid;
    if (j >= nitems) return;                  // whole wave: no barrier below
    const ChainItem it = items[j];
    chain_block<R, D, L, PC>(groups[it.group], it, smc + (size_t)wid * NW * 4 * L, lane, status);
}

// Items of several kinds in one launch (each wave switches on its item's):
// chains of different systems then run side by side in one kernel.  Each
// wave owns wave_lds doubles of LDS (4L per weight table of the largest kind
// in the launch).  NW3: the three-table kind (per-component Lorenz) is
// compiled in; at L = 512 it would make every kind's kernel spill, so it has
// an instantiation of its own there.
template <int L, int W, bool NW3>
__global__ __launch_bounds__(64 * W) void k_chain_mixed(const GroupDev* __restrict__ groups,
                                                     const ChainItem* __restrict__ items,
                                                     int nitems, int wave_lds, uint32_t* status)
{
    extern __shared__ double smc[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int j = blockIdx.x * W + wid;
    if (j >= nitems) return;
    const ChainItem it = items[j];
    const GroupDev& G = groups[it.group];
    double* smw = smc + (size_t)wid * wave_lds;
    constexpr int P = kRhsCount;
    switch (it.kind) {
    case ABM_RHS_LINEAR: chain_block<ABM_RHS_LINEAR, 1, L, false>(G, it, smw, lane, status); break;
    case ABM_RHS_DUFFING: chain_block<ABM_RHS_DUFFING, 2, L, false>(G, it, smw, lane, status); break;
    case ABM_RHS_LORENZ: chain_block<ABM_RHS_LORENZ, 3, L, false>(G, it, smw, lane, status); break;
    case ABM_RHS_POLY: chain_block<ABM_RHS_POLY, 1, L, false>(G, it, smw, lane, status); break;
    case ABM_RHS_LCR: chain_block<ABM_RHS_LCR, 2, L, false>(G, it, smw, lane, status); break;
    case ABM_RHS_DIAG: chain_block<ABM_RHS_DIAG, 2, L, false>(G, it, smw, lane, status); break;
    case P + ABM_RHS_DUFFING: chain_block<ABM_RHS_DUFFING, 2, L, true>(G, it, smw, lane, status); break;
    case P + ABM_RHS_LORENZ:
        if constexpr (NW3) chain_block<ABM_RHS_LORENZ, 3, L, true>(G, it, smw, lane, status);
        break;
    case P + ABM_RHS_LCR: chain_block<ABM_RHS_LCR, 2, L, true>(G, it, smw, lane, status); break;
    case P + ABM_RHS_DIAG: chain_block<ABM_RHS_DIAG, 2, L, true>(G, it, smw, lane, status); break;
    default: break;   // validated on the host
    }
}

template <int L, int W, bool NW3>
hipError_t launch_mixed_l(const GroupDev* groups, const ChainItem* items, int n, int nw,
                          uint32_t* status, hipStream_t st)
{
    if (nw > (NW3 ? 3 : 2)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + W - 1) / W));
    const int wave_lds = nw * 4 * L;
    const size_t shmem = (size_t)W * wave_lds * sizeof(double);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_chain_mixed<L, W, NW3>), shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_chain_mixed<L, W, NW3>), grid, dim3(64 * W), shmem, st, groups, items, n,
                       wave_lds, status);
    return hipGetLastError();
}

constexpr int kFewChains = 32;            // chain items of a launch
constexpr size_t kOwnCuLds = 150000;      // bytes: no far-field workgroup fits beside

template <int R, int D, int L, int W, bool PC>
hipError_t launch_rdl(const GroupDev* groups, const ChainItem* items, int n, uint32_t* status,
                      hipStream_t st)
{
    const dim3 grid((unsigned)((n + W - 1) / W));
    // A tick with few chains is bound by them: each chain workgroup then
    // asks for (nearly) the CU's whole LDS, so that no far-field workgroup
    // shares its CU (a far-field wave beside a chain wave slowed one long
    // trajectory's chain from 24 to ~110 µs per block).
    const size_t need = (size_t)W * (PC ? D : 1) * 4 * L * sizeof(double);
    const size_t shmem = n <= kFewChains && need < kOwnCuLds ? kOwnCuLds : need;
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_chain<R, D, L, W, PC>), shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_chain<R, D, L, W, PC>), grid, dim3(64 * W), shmem, st, groups, items, n,
                       status);
    return hipGetLastError();
}

// Waves per workgroup: packed, two per SIMD where the registers allow it
// (the chains then occupy few CUs and leave the rest to the far field), or
// spread, one per SIMD over more CUs (faster chains while the far field
// beside them is small); the weight windows of all waves fit the CU's LDS.
template <int R, int D, bool PC>
hipError_t launch_rd(const GroupDev* groups, const ChainItem* items, int n, int L, bool spread,
                     uint32_t* status, hipStream_t st)
{
    constexpr bool big = D > 2 || PC;   // more than half a SIMD's registers at L = 256
    switch (L) {
    case 64:
        return spread ? launch_rdl<R, D, 64, 4, PC>(groups, items, n, status, st)
                      : launch_rdl<R, D, 64, 8, PC>(groups, items, n, status, st);
    case 128:
        return spread ? launch_rdl<R, D, 128, 4, PC>(groups, items, n, status, st)
                      : launch_rdl<R, D, 128, 8, PC>(groups, items, n, status, st);
    case 256:
        if constexpr (big) return launch_rdl<R, D, 256, 4, PC>(groups, items, n, status, st);
        else
            return spread ? launch_rdl<R, D, 256, 4, PC>(groups, items, n, status, st)
                          : launch_rdl<R, D, 256, 8, PC>(groups, items, n, status, st);
    case 512: return launch_rdl<R, D, 512, (PC && D > 2 ? 2 : 4), PC>(groups, items, n, status, st);
    default: return hipErrorInvalidValue;
    }
}

template <int R, int D>
__global__ void k_chain_init(const GroupDev* groups, const ChainItem* items, int n)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const ChainItem it = items[j];
    const GroupDev& G = groups[it.group];
    ChainArgs A;
    chain_view<64>(G, it, D, A);
    const TrajDesc T = G.traj[it.member];
    double x0[D], f0[D], p[8];
#pragma unroll
    for (int i = 0; i < D; ++i) x0[i] = T.x0[i];
#pragma unroll
    for (int i = 0; i < 8; ++i) p[i] = T.p[i];
    rhs_eval<R, D>(p, 0.0, x0, f0);
    const int none[D] = {};
    store_history<D>(A, T, 0, f0, none);
    if (T.out_stride > 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) as_global(T.y_out)[i] = x0[i];
    }
}

template <int R, int D>
hipError_t launch_init_rd(const GroupDev* groups, const ChainItem* items, int n, hipStream_t st)
{
    hipLaunchKernelGGL((k_chain_init<R, D>), dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st,
                       groups, items, n);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_chain_mixed(const GroupDev* groups, const ChainItem* items, int n, int L,
                              int nw, uint32_t* status, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (nw < 1 || nw > 3) return hipErrorInvalidValue;
    // register demand is the largest system's (three components); the LDS
    // of nw weight tables per wave must fit the CU
    switch (L) {
    case 64: return launch_mixed_l<64, 8, true>(groups, items, n, nw, status, st);
    case 128: return launch_mixed_l<128, 8, true>(groups, items, n, nw, status, st);
    case 256: return launch_mixed_l<256, 4, true>(groups, items, n, nw, status, st);
    case 512:
        return nw <= 2 ? launch_mixed_l<512, 4, false>(groups, items, n, nw, status, st)
                       : launch_mixed_l<512, 2, true>(groups, items, n, nw, status, st);
    default: return hipErrorInvalidValue;
    }
}

int chain_tables(int kind)
{
    if (kind < kRhsCount) return 1;
    return kind - kRhsCount == ABM_RHS_LORENZ ? 3 : 2;
}

hipError_t launch_chain(const GroupDev* groups, const ChainItem* items, int n, int kind, int L,
                        bool spread, uint32_t* status, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    constexpr int P = kRhsCount;
    switch (kind) {
    case ABM_RHS_LINEAR: return launch_rd<ABM_RHS_LINEAR, 1, false>(groups, items, n, L, spread, status, st);
    case ABM_RHS_DUFFING: return launch_rd<ABM_RHS_DUFFING, 2, false>(groups, items, n, L, spread, status, st);
    case ABM_RHS_LORENZ: return launch_rd<ABM_RHS_LORENZ, 3, false>(groups, items, n, L, spread, status, st);
    case ABM_RHS_POLY: return launch_rd<ABM_RHS_POLY, 1, false>(groups, items, n, L, spread, status, st);
    case ABM_RHS_LCR: return launch_rd<ABM_RHS_LCR, 2, false>(groups, items, n, L, spread, status, st);
    case ABM_RHS_DIAG: return launch_rd<ABM_RHS_DIAG, 2, false>(groups, items, n, L, spread, status, st);
    case P + ABM_RHS_DUFFING: return launch_rd<ABM_RHS_DUFFING, 2, true>(groups, items, n, L, spread, status, st);
    case P + ABM_RHS_LORENZ: return launch_rd<ABM_RHS_LORENZ, 3, true>(groups, items, n, L, spread, status, st);
    case P + ABM_RHS_LCR: return launch_rd<ABM_RHS_LCR, 2, true>(groups, items, n, L, spread, status, st);
    case P + ABM_RHS_DIAG: return launch_rd<ABM_RHS_DIAG, 2, true>(groups, items, n, L, spread, status, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_chain_init(const GroupDev* groups, const ChainItem* items, int n, int rhs,
                             hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    switch (rhs) {
    case ABM_RHS_LINEAR: return launch_init_rd<ABM_RHS_LINEAR, 1>(groups, items, n, st);
    case ABM_RHS_DUFFING: return launch_init_rd<ABM_RHS_DUFFING, 2>(groups, items, n, st);
    case ABM_RHS_LORENZ: return launch_init_rd<ABM_RHS_LORENZ, 3>(groups, items, n, st);
    case ABM_RHS_POLY: return launch_init_rd<ABM_RHS_POLY, 1>(groups, items, n, st);
    case ABM_RHS_LCR: return launch_init_rd<ABM_RHS_LCR, 2>(groups, items, n, st);
    case ABM_RHS_DIAG: return launch_init_rd<ABM_RHS_DIAG, 2>(groups, items, n, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace abm
