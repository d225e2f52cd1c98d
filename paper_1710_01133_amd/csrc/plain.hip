// K1: one trajectory by the plain per-step method.
//
// Mapping of the paper's parallel scheme (Algorithm 1, with the node-level
// reduction of Algorithm 2) onto one GPU:
//   * a "process" is a workgroup; there are G of them, all co-resident
//     (cooperative launch), each owning a fixed slice of the history;
//   * the slice is block-cyclic: chunk c = indices [256c, 256c+256) belongs to
//     workgroup c mod G, one index per thread of its four work waves, kept in
//     LDS, so every workgroup holds an equal share of the history at every
//     step (the paper's static contiguous slices would leave most of them
//     idle early in the run);
//   * the all-reduce of Algorithm 1 is pipelined by kLook = 4 steps: during
//     step s every work thread sums b_{s+3-k} f_k and a_{s+3-k} f_k over its
//     indices k <= s-1 -- step s+4's sums without their four newest terms,
//     which need nothing that steps s .. s+3 compute; the weights were loaded
//     into registers during the previous step (they depend only on s - k), so
//     no global load waits on a step's dependent path;
//   * a fifth wave takes the predictor/corrector update itself,
//     bit-identically in every workgroup (every process computes the update,
//     as in Algorithm 1): at step s it adds the G partials of step s in a
//     fixed order, and the four newest terms b_3 f_{s-4} + .. + b_0 f_{s-1}
//     (a_j likewise) from the rows it keeps; the owner of index s keeps f_s
//     in its LDS slice;
//   * no global round trip sits on a step's path: during step s that wave
//     checks the G flags of step s+1 (loaded during step s-1; a flag reaches
//     m after its workgroup's step m-4), then issues the loads of step s+1's
//     partials, summed at step s+1, and the loads of step s+2's flags;
//   * one barrier per step; after it work wave 0 reduces the work waves'
//     partials (DPP row operations, then LDS), publishes the workgroup's 2d
//     sums of step s+4 and raises its flag to s+4;
//   * with G = 1 there is nothing to publish: the fifth wave reads the work
//     waves' partials of step s from LDS, written during step s-4.
// Partial slots (in LDS and in global memory) are kept by step mod kSlots = 8:
// a workgroup writes step m's slot after its step m-4, having seen at that
// step every flag reach m-3, i.e. every workgroup past step m-7; the readers
// of the slot's previous step, m-8, loaded it during their step m-9.
#include "abm_dev.h"
#include "abm_kernels.h"

namespace abm {

namespace {

constexpr int kCh = 256;                  // history indices per chunk (= work threads per workgroup)
constexpr int kWorkWaves = kCh / kWave;
constexpr int kThreads = kCh + kWave;     // + the wave that synchronises and updates
constexpr int kPartStride = 8;            // doubles per partial slot (2d <= 6 used)
constexpr int kLook = 4;                  // steps between a slice sum and its use
constexpr int kSlots = 8;                 // partial slots, by step mod kSlots
constexpr int kMaxGLanes = 4;             // workgroups per lane of the fifth wave (G <= 256)
constexpr size_t kPlainLds = 160 * 1024 - 256;   // LDS of one gfx950 CU, less the static flag
constexpr int kMaxPrefetch = 16;          // register-prefetched (local chunk, weight table) pairs

// v moved across lanes by one DPP control (rows outside ROWS read 0).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// lane l's value (l the same in every lane)
__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the 64 lanes of a full wave by DPP row operations in a fixed order
// (pairs, quads, half rows, rows, then the two row broadcasts that carry the
// row sums into the last row); every lane gets lane 63's total.
__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp_f64<0xB1, 0xF>(v);     // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E, 0xF>(v);     // quad_perm [2,3,0,1]
    v += dpp_f64<0x141, 0xF>(v);    // row_half_mirror
    v += dpp_f64<0x140, 0xF>(v);    // row_mirror
    v += dpp_f64<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
    return readlane_f64(v, 63);
}

// The forcing depends on t only: the updating wave evaluates it for 64 steps
// at a time, step s0 + l in lane l (s0 = 1, 65, 129, ..), and a step reads
// its lane's value (the same expression as one evaluation per step).
template <int R>
struct ForceBlock {
    double v = 0.0;
    // call with every lane of the wave at each step s = 1, 2, ..
    __device__ __forceinline__ double step(const double* __restrict__ p, double h, int64_t s, int lane)
    {
        if constexpr (R == ABM_RHS_DUFFING || R == ABM_RHS_LCR) {
            const int j = (int)((s - 1) & 63);
            if (j == 0) v = forcing<R>(p, (double)(s + lane) * h);
            return readlane_f64(v, j);
        } else {
            return forcing<R>(p, (double)s * h);
        }
    }
};

// PC: the components have orders of their own (a weight table each);
// otherwise every component uses component 0's table.  NL > 0: at most NL
// local chunks, their weights prefetched into registers; NL = 0: any number,
// weights loaded in the step (long histories).
template <int R, int D, bool PC, int NL>
__global__ __launch_bounds__(kThreads) void k_plain(PlainArgs A)
{
    extern __shared__ double sm[];
    double* Fl = sm;                                   // [nloc][256][D] history slice
    double* red = sm + (size_t)A.nloc * kCh * D;       // [kSlots][4][2D] work-wave partials by step mod kSlots
    __shared__ int s_abort;
    constexpr int NW = PC ? D : 1;                     // weight tables in use
    constexpr int NLR = NL > 0 ? NL : 1;

    const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const bool sync_wave = wid == kWorkWaves;
    const int G = A.G, nloc = A.nloc;
    const int64_t N = A.N;
    gptr<const double> bw[NW], aw[NW], cw[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        bw[w] = as_global(A.b[w]);
        aw[w] = as_global(A.a[w]);
        cw[w] = as_global(A.c[w]);
    }
    double ha[D], g2[D], x0[D], x1[D], F0[D];
    bool deriv[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const int w = PC ? i : 0;
        ha[i] = pow(A.h, A.alpha[w]);
        g2[i] = A.gam[w][1];
        deriv[i] = A.alpha[w] > 1.0;
        x0[i] = A.x0[i];
        x1[i] = A.x1[i];
    }
    rhs_eval<R, D>(A.p, 0.0, x0, F0);

    if (t == 0) s_abort = 0;
    if (sync_wave && lane == 0 && g == 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) Fl[i] = F0[i];     // f_0: chunk 0, local chunk 0, thread 0
        if (A.out_stride > 0) {
#pragma unroll
            for (int i = 0; i < D; ++i) A.y_out[i] = x0[i];
        }
    }

    // Step s's history sums in two parts (Algorithm 1's all-reduce pipelined
    // by kLook steps): the slice sums over every index but the kLook newest
    // (k <= s-5) are computed during step s-4 and published right after it;
    // the kLook newest terms, b_3 f_{s-4} + .. + b_0 f_{s-1} (a_j likewise),
    // are added by the synchronising wave, which holds f_{s-4} .. f_{s-1} from
    // its own (redundant) updates.
    // Weights b_{m-k}, a_{m-k} of this thread's indices k for the slice sums
    // of step m+1 (index clamped at 0 where k > m: those are not used).
    double wb[NLR][NW], wa[NLR][NW];
    auto fetch = [&](int64_t m) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const int64_t k = (int64_t)(g + l * G) * kCh + t;
            const int64_t idx = m - k < 0 ? 0 : m - k;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                wb[l][w] = bw[w][idx];
                wa[l][w] = aw[w][idx];
            }
        }
    };
    // synchronising wave: c_n of the coming step, b_0 .. b_3, a_0 .. a_3, the
    // kLook newest history rows (Fm[j] = f_{s-1-j}), and per lane the loaded
    // partials (pl, of step s+1) and flags (fl, of step s+2) of workgroups
    // lane, lane + 64, ..
    double cn[NW], bn[kLook][NW], an[kLook][NW];
    double Fm[kLook][D];
    double pl[kMaxGLanes][2 * D];
    uint32_t fl[kMaxGLanes];
    ForceBlock<R> fb{};
    if (!sync_wave) {
        if constexpr (NL > 0) fetch(kLook);
    } else {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            cn[w] = cw[w][0];
#pragma unroll
            for (int j = 0; j < kLook; ++j) {
                bn[j][w] = bw[w][j];
                an[j][w] = aw[w][j];
            }
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            Fm[0][i] = F0[i];
#pragma unroll
            for (int j = 1; j < kLook; ++j) Fm[j][i] = 0.0;
        }
#pragma unroll
        for (int r = 0; r < kMaxGLanes; ++r) {
            fl[r] = 0u;
#pragma unroll
            for (int j = 0; j < 2 * D; ++j) pl[r][j] = 0.0;
        }
        // flags of step kLook + 1, checked at step kLook
        if (G > 1 && kLook + 1 <= N) {
#pragma unroll
            for (int r = 0; r < kMaxGLanes; ++r)
                if (lane + kWave * r < G) fl[r] = ld_relaxed(&A.flags[lane + kWave * r]);
        }
    }
    __syncthreads();

    for (int64_t s = 1; s <= N; ++s) {
        const int64_t n = s - 1;
        // work-wave partials of step m in LDS slot m mod kSlots: written
        // during step m-kLook, read during step m (a single workgroup) or
        // published right after step m-kLook (several)
        if (sync_wave) {
            const double force = fb.step(A.p, A.h, s, lane);   // the forcing at t_s
            double tot[2 * D];
            bool ok = true;
            if (s <= kLook) {
#pragma unroll
                for (int j = 0; j < 2 * D; ++j) tot[j] = 0.0;   // no history before f_{s-kLook}
            } else if (G == 1) {
                const double* rr = red + (size_t)(s % kSlots) * kWorkWaves * 2 * D;
#pragma unroll
                for (int j = 0; j < 2 * D; ++j)
                    tot[j] = ((rr[j] + rr[2 * D + j]) + rr[4 * D + j]) + rr[6 * D + j];
            } else {
                // step s's partials, loaded during step s-1, in a fixed order
#pragma unroll
                for (int j = 0; j < 2 * D; ++j) {
                    double acc = 0.0;
#pragma unroll
                    for (int r = 0; r < kMaxGLanes; ++r)
                        if (lane + kWave * r < G) acc += pl[r][j];
                    tot[j] = wave_sum_dpp(acc);
                }
            }
            if (G > 1 && s + 1 > kLook && s + 1 <= N) {
                // every workgroup has published step s+1 (after its step
                // s+1-kLook): checked on the flags loaded during step s-1
                const uint32_t m1 = (uint32_t)(s + 1) + A.wait_bias;
#pragma unroll
                for (int r = 0; r < kMaxGLanes; ++r) {
                    const int q = lane + kWave * r;
                    if (q < G) {
                        uint32_t spins = 0;
                        while (fl[r] < m1) {
                            if (++spins > A.spin_limit) {
                                ok = false;
                                break;
                            }
                            spin_pause();
                            fl[r] = ld_relaxed(&A.flags[q]);
                        }
                    }
                }
                // the partials of step s+1 (summed at step s+1), loaded with
                // device-coherent loads issued after every flag load has
                // returned s+1: each writer's release made its partials
                // visible before its flag, so no acquire fence (which would
                // invalidate this XCD's L2 every step) is needed
                if (ok) {
                    const double* slot_base = A.part + (size_t)((s + 1) % kSlots) * G * kPartStride;
#pragma unroll
                    for (int r = 0; r < kMaxGLanes; ++r) {
                        const int q = lane + kWave * r;
                        if (q < G) {
#pragma unroll
                            for (int j = 0; j < 2 * D; ++j) pl[r][j] = ld_relaxed(&slot_base[(size_t)q * kPartStride + j]);
                        }
                    }
                }
                // the flags of step s+2, checked at step s+1
                if (s + 2 <= N) {
#pragma unroll
                    for (int r = 0; r < kMaxGLanes; ++r)
                        if (lane + kWave * r < G) fl[r] = ld_relaxed(&A.flags[lane + kWave * r]);
                }
            }
            if (!ok) {
                raise_status(A.status, kStatusTimeout);
                s_abort = 1;
                // the run is incomplete: its final state reads NaN
                if (g == 0 && lane == 0) {
                    const int64_t last = A.out_stride == 0
                                             ? 0
                                             : N / A.out_stride + (N % A.out_stride ? 1 : 0);
#pragma unroll
                    for (int i = 0; i < D; ++i) A.y_out[last * D + i] = __builtin_nan("");
                }
            } else {
                // the kLook newest terms, oldest first: k = n-j with weights
                // b_j (k >= 0) and a_j (k >= 1); the k = 0 corrector term is
                // c_n f_0
#pragma unroll
                for (int j = kLook - 1; j >= 0; --j) {
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        const int w = PC ? i : 0;
                        if (n >= j) tot[i] = fma(bn[j][w], Fm[j][i], tot[i]);
                        if (n >= j + 1) tot[D + i] = fma(an[j][w], Fm[j][i], tot[D + i]);
                    }
                }
                // predictor / corrector (eq. abm and the corrector after it),
                // from the start term x0 (+ t x1 for orders above 1)
                const double td = (double)s * A.h;
                double base[D];
#pragma unroll
                for (int i = 0; i < D; ++i) base[i] = deriv[i] ? x0[i] + td * x1[i] : x0[i];
                double yP[D], fP[D], y[D], fs[D];
#pragma unroll
                for (int i = 0; i < D; ++i) yP[i] = base[i] + ha[i] * tot[i];
                rhs_eval_forced<R, D>(A.p, yP, force, fP);
#pragma unroll
                for (int i = 0; i < D; ++i)
                    y[i] = base[i] + ha[i] * ((tot[D + i] + cn[PC ? i : 0] * F0[i]) + fP[i] / g2[i]);
                rhs_eval_forced<R, D>(A.p, y, force, fs);
#pragma unroll
                for (int i = 0; i < D; ++i) {
#pragma unroll
                    for (int j = kLook - 1; j >= 1; --j) Fm[j][i] = Fm[j - 1][i];
                    Fm[0][i] = fs[i];
                }
                if (s < N) {
#pragma unroll
                    for (int w = 0; w < NW; ++w) cn[w] = cw[w][s];   // c_n of the next step
                }
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
        } else if (s + kLook <= N) {
            // slice sums of step s+4 over this thread's indices k <= s-1:
            // b_{s+3-k} f_k and, for k >= 1, a_{s+3-k} f_k
            double* rw = red + (size_t)((s + kLook) % kSlots) * kWorkWaves * 2 * D;
            double P[D], C[D];
#pragma unroll
            for (int i = 0; i < D; ++i) P[i] = C[i] = 0.0;
            if constexpr (NL > 0) {
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    const int64_t k = (int64_t)(g + l * G) * kCh + t;
                    if (l < nloc && k <= n) {
                        const double* f = Fl + ((size_t)l * kCh + t) * D;
#pragma unroll
                        for (int i = 0; i < D; ++i) {
                            const double fa = k >= 1 ? f[i] : 0.0;   // k = 0 enters through c_n
                            P[i] = fma(wb[l][PC ? i : 0], f[i], P[i]);
                            C[i] = fma(wa[l][PC ? i : 0], fa, C[i]);
                        }
                    }
                }
                fetch(s + kLook);      // in flight while the step is synchronised
            } else {
                for (int l = 0; l < nloc; ++l) {
                    const int64_t k = (int64_t)(g + l * G) * kCh + t;
                    if (k > n) break;               // later local chunks lie further out
                    const double* f = Fl + ((size_t)l * kCh + t) * D;
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        const int w = PC ? i : 0;
                        P[i] = fma(bw[w][s + kLook - 1 - k], f[i], P[i]);
                        C[i] = fma((k >= 1) ? aw[w][s + kLook - 1 - k] : 0.0, f[i], C[i]);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const double ps = wave_sum_dpp(P[i]);
                const double cs = wave_sum_dpp(C[i]);
                if (lane == 0) {
                    rw[wid * 2 * D + i] = ps;
                    rw[wid * 2 * D + D + i] = cs;
                }
            }
        }
        // f_s is stored and step s+4's work-wave partials are in LDS
        __syncthreads();
        if (s_abort) return;
        // work wave 0 publishes the workgroup's slice sums of step s+4 and
        // raises its flag to s+4 (slots by step mod kSlots)
        if (G > 1 && t == 0 && s + kLook <= N) {
            const double* rw = red + (size_t)((s + kLook) % kSlots) * kWorkWaves * 2 * D;
            double* slot = A.part + ((size_t)((s + kLook) % kSlots) * G + g) * kPartStride;
#pragma unroll
            for (int j = 0; j < 2 * D; ++j)
                slot[j] = ((rw[j] + rw[2 * D + j]) + rw[4 * D + j]) + rw[6 * D + j];
            st_release(&A.flags[g], (uint32_t)(s + kLook));
        }
    }
}

template <int R, int D, bool PC, int NL>
hipError_t launch_plain_nl(const PlainArgs& A, hipStream_t st)
{
    const size_t shmem = ((size_t)A.nloc * kCh * D + kSlots * kWorkWaves * 2 * D) * sizeof(double);
    const void* fn = reinterpret_cast<const void*>(&k_plain<R, D, PC, NL>);
    hipError_t e = allow_lds(fn, shmem);
    if (e != hipSuccess) return e;
    PlainArgs a = A;
    void* args[] = {&a};
    return hipLaunchCooperativeKernel(fn, dim3(A.G), dim3(kThreads), args, (unsigned)shmem, st);
}

// Smallest register-prefetch size that holds the workgroup's local chunks.
template <int R, int D, bool PC>
hipError_t launch_plain_t(const PlainArgs& A, hipStream_t st)
{
    constexpr int NW = PC ? D : 1;
    const int nl = A.nloc * NW <= kMaxPrefetch ? A.nloc : 0;
    if (nl == 0) return launch_plain_nl<R, D, PC, 0>(A, st);
    if (nl <= 1) return launch_plain_nl<R, D, PC, 1>(A, st);
    if (nl <= 2) return launch_plain_nl<R, D, PC, 2>(A, st);
    if constexpr (kMaxPrefetch / NW >= 4) {
        if (nl <= 4) return launch_plain_nl<R, D, PC, 4>(A, st);
    }
    if constexpr (kMaxPrefetch / NW >= 8) {
        if (nl <= 8) return launch_plain_nl<R, D, PC, 8>(A, st);
    }
    if constexpr (kMaxPrefetch / NW >= 16) {
        if (nl <= 16) return launch_plain_nl<R, D, PC, 16>(A, st);
    }
    return launch_plain_nl<R, D, PC, 0>(A, st);
}

// ---------------------------------------------------------------------------
// One workgroup, no grid synchronisation, for histories that fit one CU's LDS.
// Weights stationary: work thread u of the NTH/64 - 1 work waves holds b_j,
// a_j for j = u + (NTH - 64) q (q < NJ) in registers for the whole run and
// reads f_{n-j} from the history in LDS (the same sums as Algorithm 1, split
// over threads by weight index instead of history index).  Wave 0 only
// updates: it adds the j = 0 terms, b_0 f_n and a_0 f_n, itself, with the f_n
// it has just computed, so the work waves can sum step s+1's terms j >= 1
// (f_{s-1} and older) while wave 0 updates step s; one barrier per step.
// Scalar systems run 1024 threads (128 registers per lane); larger systems
// 512, whose update needs more registers.
constexpr size_t kSingleLds = 160 * 1024;
constexpr int single_threads(int d, bool pc) { return (d == 1 && !pc) ? 1024 : 512; }
// most weights per thread (over all tables) that stay in registers
constexpr int single_max_nj(int d, bool pc) { return (d == 1 && !pc) ? 10 : 16; }

template <int R, int D, bool PC, int NJ>
__global__ __launch_bounds__(single_threads(D, PC)) void k_plain_single(PlainArgs A)
{
    constexpr int kSingleWork = single_threads(D, PC) - kWave;   // work threads
    constexpr int kSingleWaves = kSingleWork / kWave;
    extern __shared__ double sm[];
    double* Fl = sm;                                   // [N][D] f_0 .. f_{N-1}
    double* red = sm + (size_t)A.N * D;                // [2][work waves][2D] by step parity
    constexpr int NW = PC ? D : 1;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int64_t N = A.N;

    double wb[NJ][NW], wa[NJ][NW];                     // work waves: weights j = u + 960 q
    double ha[D], g2[D], x0[D], x1[D], F0[D], Fn[D], cn[NW], b0[NW], a0[NW];
    ForceBlock<R> fb{};
    bool deriv[D];
    if (wid == 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int w = PC ? i : 0;
            ha[i] = pow(A.h, A.alpha[w]);
            g2[i] = A.gam[w][1];
            deriv[i] = A.alpha[w] > 1.0;
            x0[i] = A.x0[i];
            x1[i] = A.x1[i];
        }
        rhs_eval<R, D>(A.p, 0.0, x0, F0);
#pragma unroll
        for (int i = 0; i < D; ++i) Fn[i] = F0[i];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            cn[w] = A.c[w][0];
            b0[w] = A.b[w][0];
            a0[w] = A.a[w][0];
        }
        if (lane == 0) {
#pragma unroll
            for (int i = 0; i < D; ++i) Fl[i] = F0[i];
            if (A.out_stride > 0) {
#pragma unroll
                for (int i = 0; i < D; ++i) A.y_out[i] = x0[i];
            }
        }
    } else {
        const int u = t - kWave;
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
            const int j = u + kSingleWork * q;        // N <= 2^30: 32-bit indices
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                wb[q][w] = j < N ? A.b[w][j] : 0.0;
                wa[q][w] = j < N ? A.a[w][j] : 0.0;
            }
        }
    }
    __syncthreads();

    for (int64_t s = 1; s <= N; ++s) {
        const int64_t n = s - 1;
        double* rp = red + (size_t)(s & 1) * kSingleWaves * 2 * D;
        if (wid != 0) {
            const int u = t - kWave, nn = (int)n;
            double P[D], C[D];
#pragma unroll
            for (int i = 0; i < D; ++i) P[i] = C[i] = 0.0;
#pragma unroll
            for (int q = 0; q < NJ; ++q) {
                const int j = u + kSingleWork * q;
                if (j >= 1 && j <= nn) {
                    const double* f = Fl + (nn - j) * D;
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        const double fc = j <= nn - 1 ? f[i] : 0.0;   // k = n - j >= 1
                        P[i] = fma(wb[q][PC ? i : 0], f[i], P[i]);
                        C[i] = fma(wa[q][PC ? i : 0], fc, C[i]);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const double ps = wave_sum_dpp(P[i]);
                const double cs = wave_sum_dpp(C[i]);
                if (lane == 0) {
                    rp[(wid - 1) * 2 * D + i] = ps;
                    rp[(wid - 1) * 2 * D + D + i] = cs;
                }
            }
        }
        __syncthreads();                           // step s's partials are in LDS
        if (wid == 0) {
            double tot[2 * D];
#pragma unroll
            for (int j = 0; j < 2 * D; ++j) {
                double acc = rp[j];
#pragma unroll
                for (int w = 1; w < kSingleWaves; ++w) acc += rp[w * 2 * D + j];
                tot[j] = acc;
            }
            // the j = 0 terms: b_0 f_n, and a_0 f_n when k = n >= 1
#pragma unroll
            for (int i = 0; i < D; ++i) {
                tot[i] = fma(b0[PC ? i : 0], Fn[i], tot[i]);
                if (n >= 1) tot[D + i] = fma(a0[PC ? i : 0], Fn[i], tot[D + i]);
            }
            const double td = (double)s * A.h;
            double base[D];
#pragma unroll
            for (int i = 0; i < D; ++i) base[i] = deriv[i] ? x0[i] + td * x1[i] : x0[i];
            double yP[D], fP[D], y[D], fs[D];
#pragma unroll
            for (int i = 0; i < D; ++i) yP[i] = base[i] + ha[i] * tot[i];
            const double force = fb.step(A.p, A.h, s, lane);
            rhs_eval_forced<R, D>(A.p, yP, force, fP);
#pragma unroll
            for (int i = 0; i < D; ++i)
                y[i] = base[i] + ha[i] * ((tot[D + i] + cn[PC ? i : 0] * F0[i]) + fP[i] / g2[i]);
            rhs_eval_forced<R, D>(A.p, y, force, fs);
            if (s < N) {
#pragma unroll
                for (int w = 0; w < NW; ++w) cn[w] = A.c[w][s];   // c_n of the next step
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
        // no second barrier: the work waves' next partials read f_{s-1} and
        // older (stored before this step's barrier) and the other half of red
    }
}

size_t single_lds(int64_t N, int d, bool pc)
{
    return ((size_t)N * d + 2 * (single_threads(d, pc) / kWave - 1) * 2 * d) * sizeof(double);
}

template <int R, int D, bool PC, int NJ>
hipError_t launch_single_nj(const PlainArgs& A, hipStream_t st)
{
    const size_t shmem = single_lds(A.N, D, PC);
    const void* fn = reinterpret_cast<const void*>(&k_plain_single<R, D, PC, NJ>);
    hipError_t e = allow_lds(fn, shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_plain_single<R, D, PC, NJ>), dim3(1), dim3(single_threads(D, PC)), shmem,
                       st, A);
    return hipGetLastError();
}

template <int R, int D, bool PC>
hipError_t launch_single_t(const PlainArgs& A, hipStream_t st)
{
    constexpr int NW = PC ? D : 1;
    constexpr int kSingleWork = single_threads(D, PC) - kWave;
    const int64_t nj = (A.N + kSingleWork - 1) / kSingleWork;
    if (nj <= 1) return launch_single_nj<R, D, PC, 1>(A, st);
    if (nj <= 2) return launch_single_nj<R, D, PC, 2>(A, st);
    if (nj <= 4) return launch_single_nj<R, D, PC, 4>(A, st);
    constexpr int MAXNJ = single_max_nj(D, PC);
    if constexpr (8 * NW <= MAXNJ) {
        if (nj <= 8) return launch_single_nj<R, D, PC, 8>(A, st);
    }
    if constexpr (10 * NW <= MAXNJ && MAXNJ < 12) {
        if (nj <= 10) return launch_single_nj<R, D, PC, 10>(A, st);
    }
    if constexpr (12 * NW <= MAXNJ) {
        if (nj <= 12) return launch_single_nj<R, D, PC, 12>(A, st);
    }
    if constexpr (16 * NW <= MAXNJ) {
        if (nj <= 16) return launch_single_nj<R, D, PC, 16>(A, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int plain_max_local_chunks(int d)
{
    // the CU's whole LDS (one workgroup per CU): history slice + wave partials
    return (int)((kPlainLds - kSlots * kWorkWaves * 2 * d * sizeof(double)) / ((size_t)kCh * d * sizeof(double)));
}

int plain_chunk() { return kCh; }

int plain_prefetch_chunks(int tables) { return kMaxPrefetch / tables; }

int plain_part_doubles(int G) { return kSlots * G * kPartStride; }

bool plain_single_fits(int64_t N, int d, int tables)
{
    const bool pc = tables > 1;
    const int64_t nj = (N + single_threads(d, pc) - kWave - 1) / (single_threads(d, pc) - kWave);
    int njmax = 0;
    for (int c : {1, 2, 4, 8, 10, 12, 16})
        if (c * tables <= single_max_nj(d, pc) && (c != 10 || single_max_nj(d, pc) < 12)) njmax = c;
    return nj <= njmax && single_lds(N, d, pc) <= kSingleLds;
}

hipError_t launch_plain_single(const PlainArgs& A, int kind, hipStream_t st)
{
    switch (kind) {
    case ABM_RHS_LINEAR: return launch_single_t<ABM_RHS_LINEAR, 1, false>(A, st);
    case ABM_RHS_DUFFING: return launch_single_t<ABM_RHS_DUFFING, 2, false>(A, st);
    case ABM_RHS_LORENZ: return launch_single_t<ABM_RHS_LORENZ, 3, false>(A, st);
    case ABM_RHS_POLY: return launch_single_t<ABM_RHS_POLY, 1, false>(A, st);
    case ABM_RHS_LCR: return launch_single_t<ABM_RHS_LCR, 2, false>(A, st);
    case ABM_RHS_DIAG: return launch_single_t<ABM_RHS_DIAG, 2, false>(A, st);
    case kRhsCount + ABM_RHS_DUFFING: return launch_single_t<ABM_RHS_DUFFING, 2, true>(A, st);
    case kRhsCount + ABM_RHS_LORENZ: return launch_single_t<ABM_RHS_LORENZ, 3, true>(A, st);
    case kRhsCount + ABM_RHS_LCR: return launch_single_t<ABM_RHS_LCR, 2, true>(A, st);
    case kRhsCount + ABM_RHS_DIAG: return launch_single_t<ABM_RHS_DIAG, 2, true>(A, st);
    default: return hipErrorInvalidValue;
    }
}

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
