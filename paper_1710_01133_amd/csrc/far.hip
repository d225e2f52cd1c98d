// K2: far-field history products of the blocked method.
//
// Block m holds the steps s = mL+1 .. mL+L (rows r = 0..L-1, n = mL + r).
// History older than the block's near band, k = 1..K (K = kfar), is complete
// when the block starts, so both history sums of every row of the block are
// one matrix product with a Toeplitz weight matrix:
//   FF[r]     = sum_{k=1..K} b_{mL+r-k} F_k          (predictor rows,  eq. abm)
//   FF[L + r] = sum_{k=1..K} a_{mL+r-k} F_k          (corrector rows)
// with F_k the time-major history row (all columns = trajectory components).
// The k = 0 terms (b_n f_0, c_n f_0) and the near band are added by the chain
// kernel.
//
// Tiling: one workgroup computes all 2L rows for 16*NT columns over a fixed
// range of history chunks [k_lo, k_hi) (chunk boundaries and their grouping
// depend only on m, never on which trajectories are batched, so every
// column's arithmetic is the same alone or in a batch).  Each of the 4 waves owns L/2 rows (MT = L/32 tiles
// of 16 rows); every 16x16 output tile is a chain of matrix-core products
// over 4-row slices of the history.  The Toeplitz operand is never formed:
// lane (i, kk) of a fragment reads the weight at index mL + r - k from an LDS
// copy of the chunk's weight window.  The partial result of each workgroup
// goes to FFpart[split][col][2L]; the chain kernel adds the splits in order.
#include "far_common.h"

namespace abm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kKS = 16;   // history rows per LDS stage

template <int MT, int NT>
__global__ __launch_bounds__(256) void k_far_f64(const GroupDev* groups, const FarItem* items,
                                                 int kchunk)
{
    constexpr int L = 32 * MT;       // block length
    constexpr int TN = 16 * NT;      // columns per workgroup
    FarArgs A;
    if (!far_view(groups, items, kchunk, L, A)) return;
    extern __shared__ double sm[];
    const int win = L + A.kchunk;    // weight window length (padded)
    double* wb = sm;                 // b window
    double* wa = sm + win;           // a window
    double* Ft = sm + 2 * win;       // [2][kKS][TN] history stages

    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int col0 = blockIdx.x * TN;
    const int64_t mL = A.mL;
    // rows of this wave: waves 0,1 predictor rows, waves 2,3 corrector rows
    const bool corr = wid >= 2;
    const int rbase = (wid & 1) * (L / 2);
    const double* wwin = corr ? wa : wb;
    const int li = lane & 15, lk = lane >> 4;

    d4 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    // stage loader: kKS x TN doubles, coalesced along columns
    constexpr int kStageElems = kKS * TN;
    constexpr int kPerThread = (kStageElems + 255) / 256;
    const gptr<const double> Fg = A.F;
    const int64_t ldF = A.ldF;
    double pre[kPerThread];
    auto load_stage = [&](int64_t k0) {
#pragma unroll
        for (int e = 0; e < kPerThread; ++e) {
            const int idx = t + e * 256;
            if (idx < kStageElems) {
                const int rr = idx / TN, cc = idx % TN;
                pre[e] = Fg[(k0 + rr) * ldF + col0 + cc];
            }
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int e = 0; e < kPerThread; ++e) {
            const int idx = t + e * 256;
            if (idx < kStageElems) Ft[buf * kStageElems + idx] = pre[e];
        }
    };

    // this workgroup's fixed range of history chunks, summed in order
    const int c_begin = blockIdx.y * A.chunks_per_split;
    int c_end = c_begin + A.chunks_per_split;
    if (c_end > A.nchunks) c_end = A.nchunks;
    for (int chunk = c_begin; chunk < c_end; ++chunk) {
        const int64_t k_lo = 1 + (int64_t)chunk * A.kchunk;
        int64_t k_hi = k_lo + A.kchunk;
        if (k_hi > A.kfar + 1) k_hi = A.kfar + 1;
        const int nk = (int)(k_hi - k_lo);                    // multiple of kKS
        const int64_t jb = mL - k_hi + 1;                     // lowest weight index used (>= 0)
        const int wlen = L + nk - 1;
        __syncthreads();   // previous chunk's readers are done with the LDS
        // weight window: the loads of a batch are all issued before its stores
        for (int x0 = t; x0 < wlen; x0 += 256 * 4) {
            double vb[4], va[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int x = x0 + 256 * u;
                vb[u] = x < wlen ? A.b[jb + x] : 0.0;
                va[u] = x < wlen ? A.a[jb + x] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int x = x0 + 256 * u;
                if (x < wlen) {
                    wb[x] = vb[u];
                    wa[x] = va[u];
                }
            }
        }
        load_stage(k_lo);
        store_stage(0);
        __syncthreads();
        const int nstages = nk / kKS;
        for (int st = 0; st < nstages; ++st) {
            const int buf = st & 1;
            if (st + 1 < nstages) load_stage(k_lo + (int64_t)(st + 1) * kKS);
            const double* Fs = Ft + buf * kStageElems;
#pragma unroll
            for (int kq = 0; kq < kKS / 4; ++kq) {
                // history index of this lane's fragment column
                const int64_t k = k_lo + (int64_t)st * kKS + kq * 4 + lk;
                double bf[NT];
#pragma unroll
                for (int j = 0; j < NT; ++j) bf[j] = Fs[(kq * 4 + lk) * TN + j * 16 + li];
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    const int r = rbase + i * 16 + li;
                    const double af = wwin[(int)(mL + r - k - jb)];
#pragma unroll
                    for (int j = 0; j < NT; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf[j], acc[i][j], 0, 0, 0);
                }
            }
            if (st + 1 < nstages) store_stage(buf ^ 1);
            __syncthreads();
        }
    }

    // FFpart[split][col][2L].  The double 16x16x4 product returns row
    // lk + 4v of column li of the tile in register v of lane (li, lk).
    const gptr<double> out = A.part + (size_t)blockIdx.y * A.ldP * (2 * L);
    const int prow = (corr ? L : 0) + rbase;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int col = col0 + j * 16 + li;
            const gptr<double> o = out + (size_t)col * (2 * L) + prow + i * 16 + lk;
#pragma unroll
            for (int v = 0; v < 4; ++v) o[4 * v] = acc[i][j][v];
        }
}

template <int MT, int NT>
hipError_t launch_t(const GroupDev* groups, const FarItem* items, int n, int max_coltiles,
                    int max_nsplit, int kchunk, hipStream_t st)
{
    constexpr int L = 32 * MT, TN = 16 * NT;
    (void)TN;
    const size_t shmem = (2 * (size_t)(L + kchunk) + 2 * kKS * TN) * sizeof(double);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_far_f64<MT, NT>), shmem);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)max_coltiles, (unsigned)max_nsplit, (unsigned)n);
    hipLaunchKernelGGL((k_far_f64<MT, NT>), grid, dim3(256), shmem, st, groups, items, kchunk);
    return hipGetLastError();
}

}  // namespace

int far_tile_cols(int L, int prec)
{
    if (prec == ABM_FAR_I8) return far_i8_tile_cols();
    if (prec != ABM_FAR_FP64) return 16;
    switch (L) {
    case 64: return 128;
    case 128: return 64;
    case 256: return 32;
    case 512: return 16;
    default: return 0;
    }
}

int far_stage_rows() { return kKS; }

size_t far_lds_bytes(int L, int kchunk, int prec)
{
    if (prec == ABM_FAR_I8) return far_i8_lds_bytes(L, kchunk);
    if (prec != ABM_FAR_FP64) return far_lp_lds_bytes(L, kchunk, prec);
    return (2 * (size_t)(L + kchunk) + 2 * kKS * far_tile_cols(L, prec)) * sizeof(double);
}

hipError_t allow_lds(const void* fn, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

int far_split_plan(int64_t kfar, int kchunk, int max_split, int* nchunks, int* chunks_per_split)
{
    if (kfar < 1) {
        *nchunks = 0;
        *chunks_per_split = 0;
        return 0;
    }
    const int nc = (int)((kfar + kchunk - 1) / kchunk);
    const int ns0 = nc < max_split ? nc : max_split;
    const int cps = (nc + ns0 - 1) / ns0;
    *nchunks = nc;
    *chunks_per_split = cps;
    return (nc + cps - 1) / cps;
}

int far_split_bound(int64_t kfar_max, int kchunk, int max_split)
{
    // the slice count of far_split_plan is not monotone in kfar (e.g. 8
    // chunks give 8 slices, 10 chunks give 5), so bound it over all blocks
    if (kfar_max < 1) return 0;
    const int64_t nc = (kfar_max + kchunk - 1) / kchunk;
    return (int)(nc < max_split ? nc : max_split);
}

hipError_t launch_far(const GroupDev* groups, const FarItem* items, int n, int max_coltiles,
                      int max_nsplit, int kchunk, int L, int cls, hipStream_t st)
{
    if (n < 1 || max_coltiles < 1 || max_nsplit < 1) return hipSuccess;
    if (cls == far_class(ABM_FAR_FP64, true) || cls == far_class(ABM_FAR_FP32, true))
        return launch_far_hankel(groups, items, n, max_coltiles, max_nsplit, L,
                                 cls == far_class(ABM_FAR_FP64, true) ? ABM_FAR_FP64 : ABM_FAR_FP32, st);
    if (cls == ABM_FAR_I8) return launch_far_i8(groups, items, n, max_coltiles, max_nsplit, kchunk, L, st);
    if (cls != ABM_FAR_FP64)
        return launch_far_lp(groups, items, n, max_coltiles, max_nsplit, kchunk, L, cls, st);
    switch (L) {
    case 64: return launch_t<2, 8>(groups, items, n, max_coltiles, max_nsplit, kchunk, st);
    case 128: return launch_t<4, 4>(groups, items, n, max_coltiles, max_nsplit, kchunk, st);
    case 256: return launch_t<8, 2>(groups, items, n, max_coltiles, max_nsplit, kchunk, st);
    case 512: return launch_t<16, 1>(groups, items, n, max_coltiles, max_nsplit, kchunk, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace abm
