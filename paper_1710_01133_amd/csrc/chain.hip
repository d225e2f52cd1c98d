// K3: near band and predictor/corrector chain of the blocked method.
//
// One wavefront advances one trajectory through block m (rows r = 0..L-1,
// step s = mL + r + 1, n = s - 1).  Lane l owns the rows r = l + 64q and keeps
// two running sums per row and component:
//   accP[r] = sum_{k<=n} b_{n-k} f_k   (predictor history sum of eq. abm)
//   accC[r] = c_n f_0 + sum_{1<=k<=n} a_{n-k} f_k   (corrector history sum)
// They start as the far-field sums (chunks added in order) plus the k = 0
// terms; each new f_s is then scattered into every later row of the block
// (weight index n' - s = r' - r - 1), so when row r comes up its sums are
// complete and are broadcast from the owning lane with readlane.  The update
//   yP = x0 + h^a accP,  y = x0 + h^a (accC + f(t_s, yP) / Gamma(a+2))
// is computed identically by every lane; lane 0 stores f_s (and its reduced
// copies for the far field) and the output states.
#include "abm_dev.h"
#include "abm_kernels.h"

namespace abm {

namespace {

__device__ __forceinline__ double readlane_d(double v, int l)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// bf16 of a float, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t bf16_rn(float x)
{
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f(uint16_t h)
{
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}

template <int D>
__device__ __forceinline__ void store_history(const ChainArgs& A, const TrajDesc& T, int64_t s,
                                              const double* fs)
{
    const int64_t row = s * A.ldF + T.col0;
#pragma unroll
    for (int i = 0; i < D; ++i) A.F[row + i] = fs[i];
    if (A.F32) {
#pragma unroll
        for (int i = 0; i < D; ++i) A.F32[row + i] = (float)fs[i];
    }
    if (A.Fhi) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const float x = (float)fs[i];
            const uint16_t hi = bf16_rn(x);
            const float r1 = x - bf16_f(hi);
            const uint16_t mid = bf16_rn(r1);
            A.Fhi[row + i] = hi;
            A.Fmid[row + i] = mid;
            if (A.Flo) A.Flo[row + i] = bf16_rn(r1 - bf16_f(mid));
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
        for (int i = 0; i < D; ++i) T.y_out[w * D + i] = y[i];
    }
}

template <int R, int D, int L>
__global__ __launch_bounds__(256) void k_chain(ChainArgs A)
{
    constexpr int Q = L / 64;
    __shared__ double swb[L], swa[L];
    for (int x = threadIdx.x; x < L; x += 256) {
        swb[x] = A.b[x];
        swa[x] = A.a[x];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int j = blockIdx.x * 4 + wid;
    if (j >= A.ntraj) return;
    const TrajDesc T = A.traj[j];
    const int64_t mL = A.mL;
    if (mL >= T.N) return;
    const int rows = (int)((T.N - mL) < L ? (T.N - mL) : L);

    double x0[D], F0[D], p[8];
#pragma unroll
    for (int i = 0; i < D; ++i) x0[i] = T.x0[i];
#pragma unroll
    for (int i = 0; i < 8; ++i) p[i] = T.p[i];
    const double h = T.h;
    const double ha = pow(h, A.alpha);
    const double g2 = A.gam[1];
#pragma unroll
    for (int i = 0; i < D; ++i) F0[i] = A.F[T.col0 + i];

    double accP[Q][D], accC[Q][D];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int r = lane + 64 * q;
        const int64_t n = mL + r;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double sp = 0.0, sc = 0.0;
            for (int ch = 0; ch < A.nchunks; ++ch) {
                const double* pc = A.part + ((size_t)ch * A.ldP + T.col0 + i) * (2 * L);
                sp += pc[r];
                sc += pc[L + r];
            }
            accP[q][i] = sp + A.b[n] * F0[i];
            accC[q][i] = sc + A.c[n] * F0[i];
        }
    }

    bool bad = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        for (int rr = 0; rr < 64; ++rr) {
            const int r = 64 * q + rr;
            if (r >= rows) break;
            const int64_t s = mL + r + 1;
            const double td = (double)s * h;
            double P[D], C[D], yP[D], fP[D], y[D], fs[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                P[i] = readlane_d(accP[q][i], rr);
                C[i] = readlane_d(accC[q][i], rr);
            }
#pragma unroll
            for (int i = 0; i < D; ++i) yP[i] = x0[i] + ha * P[i];
            rhs_eval<R, D>(p, td, yP, fP);
#pragma unroll
            for (int i = 0; i < D; ++i) y[i] = x0[i] + ha * (C[i] + fP[i] / g2);
            rhs_eval<R, D>(p, td, y, fs);
            if (lane == 0) {
                store_history<D>(A, T, s, fs);
                store_output<D>(T, s, y);
#pragma unroll
                for (int i = 0; i < D; ++i) bad |= !isfinite(y[i]);
            }
            // scatter f_s into the later rows of the block
#pragma unroll
            for (int q2 = 0; q2 < Q; ++q2) {
                const int widx = lane + 64 * q2 - r - 1;
                if (widx >= 0) {
                    const double wbv = swb[widx], wav = swa[widx];
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        accP[q2][i] = fma(wbv, fs[i], accP[q2][i]);
                        accC[q2][i] = fma(wav, fs[i], accC[q2][i]);
                    }
                }
            }
        }
    }
    if (bad) raise_status(A.status, kStatusNonFinite);
}

template <int R, int D>
hipError_t launch_rd(const ChainArgs& A, int L, hipStream_t st)
{
    const dim3 grid((unsigned)((A.ntraj + 3) / 4));
    switch (L) {
    case 64: hipLaunchKernelGGL((k_chain<R, D, 64>), grid, dim3(256), 0, st, A); break;
    case 128: hipLaunchKernelGGL((k_chain<R, D, 128>), grid, dim3(256), 0, st, A); break;
    case 256: hipLaunchKernelGGL((k_chain<R, D, 256>), grid, dim3(256), 0, st, A); break;
    case 512: hipLaunchKernelGGL((k_chain<R, D, 512>), grid, dim3(256), 0, st, A); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Solve start: f_0 = f(0, x0) into history row 0 (and reduced copies), y_0 = x0.
template <int R, int D>
__global__ void k_chain_init(ChainArgs A)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= A.ntraj) return;
    const TrajDesc T = A.traj[j];
    double x0[D], f0[D], p[8];
#pragma unroll
    for (int i = 0; i < D; ++i) x0[i] = T.x0[i];
#pragma unroll
    for (int i = 0; i < 8; ++i) p[i] = T.p[i];
    rhs_eval<R, D>(p, 0.0, x0, f0);
    store_history<D>(A, T, 0, f0);
    if (T.out_stride > 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) T.y_out[i] = x0[i];
    }
}

template <int R, int D>
hipError_t launch_init_rd(const ChainArgs& A, hipStream_t st)
{
    hipLaunchKernelGGL((k_chain_init<R, D>), dim3((unsigned)((A.ntraj + 63) / 64)), dim3(64), 0, st,
                       A);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_chain(const ChainArgs& A, int rhs, int L, hipStream_t st)
{
    if (A.ntraj <= 0) return hipSuccess;
    switch (rhs) {
    case ABM_RHS_LINEAR: return launch_rd<ABM_RHS_LINEAR, 1>(A, L, st);
    case ABM_RHS_DUFFING: return launch_rd<ABM_RHS_DUFFING, 2>(A, L, st);
    case ABM_RHS_LORENZ: return launch_rd<ABM_RHS_LORENZ, 3>(A, L, st);
    case ABM_RHS_POLY: return launch_rd<ABM_RHS_POLY, 1>(A, L, st);
    case ABM_RHS_LCR: return launch_rd<ABM_RHS_LCR, 2>(A, L, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_chain_init(const ChainArgs& A, int rhs, hipStream_t st)
{
    if (A.ntraj <= 0) return hipSuccess;
    switch (rhs) {
    case ABM_RHS_LINEAR: return launch_init_rd<ABM_RHS_LINEAR, 1>(A, st);
    case ABM_RHS_DUFFING: return launch_init_rd<ABM_RHS_DUFFING, 2>(A, st);
    case ABM_RHS_LORENZ: return launch_init_rd<ABM_RHS_LORENZ, 3>(A, st);
    case ABM_RHS_POLY: return launch_init_rd<ABM_RHS_POLY, 1>(A, st);
    case ABM_RHS_LCR: return launch_init_rd<ABM_RHS_LCR, 2>(A, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace abm
