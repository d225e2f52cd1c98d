// K1: one trajectory by the plain per-step method.
//
// Mapping of the paper's parallel scheme (Algorithm 1, with the node-level
// reduction of Algorithm 2) onto one GPU:
//   * a "process" is a workgroup; there are G of them, all co-resident
//     (cooperative launch), each owning a fixed slice of the history;
//   * the slice is block-cyclic: chunk c = indices [256c, 256c+256) belongs to
//     workgroup c mod G, one index per thread, kept in LDS, so every workgroup
//     holds an equal share of the history at every step (the paper's static
//     contiguous slices would leave most of them idle early in the run);
//   * per step every workgroup sums b_{n-k} f_k and a_{n-k} f_k over its
//     indices (thread -> wavefront butterfly -> LDS), publishes the 2d partial
//     sums and raises its step flag (the all-reduce of Algorithm 1);
//   * every workgroup waits for all G flags, adds the G partials in a fixed
//     order and takes the predictor/corrector update itself, bit-identically
//     (every process computes the update, as in Algorithm 1); the owner of
//     index s keeps f_s in its LDS slice.
// Partial slots are double-buffered by step parity: a workgroup can only
// overwrite slot s+2 after every workgroup has published s+1, which each does
// after reading slot s.
#include "abm_dev.h"
#include "abm_kernels.h"

namespace abm {

namespace {

constexpr int kCh = 256;          // history indices per chunk (= threads per workgroup)
constexpr int kPartStride = 8;    // doubles per partial slot (2d <= 6 used)
constexpr size_t kPlainLds = 160 * 1024 - 256;   // LDS of one gfx950 CU, less the static flag

// PC: the components have orders of their own (a weight table each);
// otherwise every component uses component 0's table.
template <int R, int D, bool PC>
__global__ __launch_bounds__(256) void k_plain(PlainArgs A)
{
    extern __shared__ double sm[];
    double* Fl = sm;                                   // [nloc][256][D] history slice
    double* red = sm + (size_t)A.nloc * kCh * D;       // [4][2D] per-wave partials
    __shared__ int s_abort;
    constexpr int NW = PC ? D : 1;                     // weight tables in use

    const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int G = A.G;
    const int64_t N = A.N;
    double ha[D], g2[D];
    bool deriv[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const int w = PC ? i : 0;
        ha[i] = pow(A.h, A.alpha[w]);
        g2[i] = A.gam[w][1];
        deriv[i] = A.alpha[w] > 1.0;
    }

    double x0[D], x1[D], F0[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        x0[i] = A.x0[i];
        x1[i] = A.x1[i];
    }
    rhs_eval<R, D>(A.p, 0.0, x0, F0);

    if (t == 0) s_abort = 0;
    if (g == 0 && t == 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) Fl[i] = F0[i];     // f_0: chunk 0, local chunk 0, thread 0
        if (A.out_stride > 0) {
#pragma unroll
            for (int i = 0; i < D; ++i) A.y_out[i] = x0[i];
        }
    }
    __syncthreads();

    for (int64_t s = 1; s <= N; ++s) {
        const int64_t n = s - 1;
        double P[D], C[D];
#pragma unroll
        for (int i = 0; i < D; ++i) P[i] = C[i] = 0.0;
        for (int lc = 0; lc < A.nloc; ++lc) {
            const int64_t k = (int64_t)(g + lc * G) * kCh + t;
            if (k > n) break;               // later local chunks lie further out
            double wb[NW], wa[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                wb[w] = A.b[w][n - k];
                wa[w] = (k >= 1) ? A.a[w][n - k] : 0.0;   // k = 0 enters through c_n
            }
            const double* f = Fl + ((size_t)lc * kCh + t) * D;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                P[i] = fma(wb[PC ? i : 0], f[i], P[i]);
                C[i] = fma(wa[PC ? i : 0], f[i], C[i]);
            }
        }
        // workgroup partial: wavefront butterfly, then the 4 waves in order
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double ps = wave_sum(P[i]);
            const double cs = wave_sum(C[i]);
            if (lane == 0) {
                red[wid * 2 * D + i] = ps;
                red[wid * 2 * D + D + i] = cs;
            }
        }
        __syncthreads();
        double* slot_base = A.part + (size_t)(s & 1) * G * kPartStride;
        if (t == 0) {
            double* slot = slot_base + (size_t)g * kPartStride;
#pragma unroll
            for (int j = 0; j < 2 * D; ++j)
                slot[j] = ((red[j] + red[2 * D + j]) + red[4 * D + j]) + red[6 * D + j];
            st_release(&A.flags[g], (uint32_t)s);
        }
        // wait until every workgroup has published step s
        if (t < G) {
            uint32_t spins = 0;
            while (ld_relaxed(&A.flags[t]) < (uint32_t)s) {
                if (++spins > A.spin_limit) {
                    raise_status(A.status, kStatusTimeout);
                    s_abort = 1;
                    break;
                }
                spin_pause();
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (s_abort) return;

        if (wid == 0) {
            double tot[2 * D];
#pragma unroll
            for (int j = 0; j < 2 * D; ++j) {
                double acc = 0.0;
                for (int q = lane; q < G; q += kWave) acc += slot_base[(size_t)q * kPartStride + j];
                tot[j] = wave_sum(acc);
            }
            // predictor / corrector (eq. abm and the corrector after it),
            // from the start term x0 (+ t x1 for orders above 1)
            const double td = (double)s * A.h;
            double base[D], cn[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                base[i] = deriv[i] ? x0[i] + td * x1[i] : x0[i];
                cn[i] = A.c[PC ? i : 0][n];
            }
            double yP[D], fP[D], y[D], fs[D];
#pragma unroll
            for (int i = 0; i < D; ++i) yP[i] = base[i] + ha[i] * tot[i];
            rhs_eval<R, D>(A.p, td, yP, fP);
#pragma unroll
            for (int i = 0; i < D; ++i)
                y[i] = base[i] + ha[i] * ((tot[D + i] + cn[i] * F0[i]) + fP[i] / g2[i]);
            rhs_eval<R, D>(A.p, td, y, fs);
            if (lane == 0) {
                if (s < N) {
                    const int64_t cs = s / kCh;
                    if ((int)(cs % G) == g) {
                        double* dst = Fl + ((size_t)(cs / G) * kCh + (s % kCh)) * D;
#pragma unroll
                        for (int i = 0; i < D; ++i) dst[i] = fs[i];
                    }
                }
                if (g == 0) {
                    bool bad = false;
#pragma unroll
                    for (int i = 0; i < D; ++i) bad |= !isfinite(y[i]);
                    if (bad) raise_status(A.status, kStatusNonFinite);
                    int64_t w = -1;
                    if (A.out_stride == 0) {
                        if (s == N) w = 0;
                    } else if (s % A.out_stride == 0) {
                        w = s / A.out_stride;
                    } else if (s == N) {
                        w = s / A.out_stride + 1;
                    }
                    if (w >= 0) {
#pragma unroll
                        for (int i = 0; i < D; ++i) A.y_out[w * D + i] = y[i];
                    }
                }
            }
        }
        __syncthreads();
    }
}

template <int R, int D, bool PC>
hipError_t launch_plain_t(const PlainArgs& A, hipStream_t st)
{
    const size_t shmem = ((size_t)A.nloc * kCh * D + 4 * 2 * D) * sizeof(double);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_plain<R, D, PC>), shmem);
    if (e != hipSuccess) return e;
    PlainArgs a = A;
    void* args[] = {&a};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_plain<R, D, PC>), dim3(A.G),
                                      dim3(kCh), args, (unsigned)shmem, st);
}

}  // namespace

int plain_max_local_chunks(int d)
{
    // the CU's whole LDS (one workgroup per CU): history slice + wave partials
    return (int)((kPlainLds - 4 * 2 * d * sizeof(double)) / ((size_t)kCh * d * sizeof(double)));
}

int plain_chunk() { return kCh; }

int plain_part_doubles(int G) { return 2 * G * kPartStride; }

hipError_t launch_plain(const PlainArgs& A, int kind, hipStream_t st)
{
    switch (kind) {
    case ABM_RHS_LINEAR: return launch_plain_t<ABM_RHS_LINEAR, 1, false>(A, st);
    case ABM_RHS_DUFFING: return launch_plain_t<ABM_RHS_DUFFING, 2, false>(A, st);
    case ABM_RHS_LORENZ: return launch_plain_t<ABM_RHS_LORENZ, 3, false>(A, st);
    case ABM_RHS_POLY: return launch_plain_t<ABM_RHS_POLY, 1, false>(A, st);
    case ABM_RHS_LCR: return launch_plain_t<ABM_RHS_LCR, 2, false>(A, st);
    case ABM_RHS_DIAG: return launch_plain_t<ABM_RHS_DIAG, 2, false>(A, st);
    case kRhsCount + ABM_RHS_DUFFING: return launch_plain_t<ABM_RHS_DUFFING, 2, true>(A, st);
    case kRhsCount + ABM_RHS_LORENZ: return launch_plain_t<ABM_RHS_LORENZ, 3, true>(A, st);
    case kRhsCount + ABM_RHS_LCR: return launch_plain_t<ABM_RHS_LCR, 2, true>(A, st);
    case kRhsCount + ABM_RHS_DIAG: return launch_plain_t<ABM_RHS_DIAG, 2, true>(A, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace abm
