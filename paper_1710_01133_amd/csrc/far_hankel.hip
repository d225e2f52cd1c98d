// K2 for narrow groups: a few history columns (typically one trajectory with
// its own alpha), where the column tiles of the Toeplitz kernels would be
// mostly padding.  The far-field sums of block m (Section 2, eq. abm,
//   FF[r] = sum_{k=1..K} w_{mL+r-k} F_k,  r = 0..L-1,  K = (m-1)L)
// are rewritten as a blocked convolution.  With r = 16 rho + i and
// k = 16 kappa + j + 1 (i, j < 16) the weight index is
//   mL - 1 + 16 (rho - kappa) + i - j,
// so for each shift delta = rho - kappa
//   FF[16 rho + i] += sum_j H_delta[i][j] G[j][rho - delta],
//   H_delta[i][j] = w_{mL - 1 + 16 delta + i - j}   (a 16x16 Toeplitz tile),
//   G[j][kappa]   = F_{16 kappa + j + 1}, zero outside 1 <= k <= K.
// One matrix-core product per delta then has M = 16 (i), K = 16 (j) and
// N = the L/16 row blocks rho of every column, so the N dimension is full
// whatever the number of columns.  delta runs over 1 - K/16 .. L/16 - 1,
// i.e. K + L - 16 history rows of work: the extra L - 16 rows of zeros are
// the price of the reshaping (small once K >> L).
//
// A workgroup of 4 waves stages a chunk of 64 shifts (the weights it needs
// and the 16 (64 + L/16 - 1) history rows they touch, zero-masked) in LDS;
// the waves take every 4th shift and reduce their sums through LDS at the
// end, in a fixed order, into one partial slice per workgroup.  Float
// products are added into double sums after every shift (16 history rows),
// as in the float Toeplitz kernel.  Operand layout of the 16x16x4 products:
// lane (li = lane%16, g = lane/16) supplies A row li, column 4s+g, and B
// row 4s+g, column li at K-step s.
#include <type_traits>

#include "far_common.h"

namespace abm {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kDch = 64;          // shifts per chunk (1024 history rows)
constexpr int64_t kMinChunks = 8; // least chunks per split slice
constexpr int kHWaves = 4;
constexpr int kRedSlots = 4;      // tiles reduced per round
constexpr int kHMaxTiles = 4;     // product tiles per item (16 columns of row blocks each)

// LDS row index with one pad word per 16 rows (B reads of 16 row blocks
// would otherwise hit the same banks)
__device__ __forceinline__ int pad16(int x) { return x + (x >> 4); }

template <int L>
constexpr int hist_stride() { return 17 * (kDch + L / 16 - 1); }

constexpr int kWlen = 16 * kDch + 16;

template <typename T>
__device__ __forceinline__ const T* hk_weights(const CompWeights& W, bool corr);
template <>
__device__ __forceinline__ const float* hk_weights<float>(const CompWeights& W, bool corr)
{
    return corr ? W.a32 : W.b32;
}
template <>
__device__ __forceinline__ const double* hk_weights<double>(const CompWeights& W, bool corr)
{
    return corr ? W.a : W.b;
}
template <typename T>
__device__ __forceinline__ const T* hk_history(const GroupDev& G);
template <>
__device__ __forceinline__ const float* hk_history<float>(const GroupDev& G) { return G.F32; }
template <>
__device__ __forceinline__ const double* hk_history<double>(const GroupDev& G) { return G.F; }

__device__ __forceinline__ f4 hk_mfma(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4 hk_mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Result row of register v in lane group g: float 16x16x4 gives row 4g + v,
// double 16x16x4 gives row g + 4v.
template <typename T>
__device__ __forceinline__ int hk_row(int g, int v)
{
    return sizeof(T) == 4 ? 4 * g + v : g + 4 * v;
}

// The whole item for exactly NT product tiles (NT is uniform per item, so
// the kernel selects the body once instead of guarding every product).
template <typename T, int L, int NT>
__device__ __forceinline__ void hankel_body(const GroupDev& G, const FarItem& it,
                                            unsigned char* hk_smem)
{
    constexpr int TMAX = NT;
    constexpr int R = L / 16;                 // 16-row blocks of the output
    constexpr int HST = hist_stride<L>();
    constexpr bool kFloat = sizeof(T) == 4;
    typedef typename std::conditional<kFloat, f4, d4>::type acc_t;

    const int ncols = it.ncols;
    // floor(e / ncols) = (e * inv_cols) >> 20 for every staged e (e < 2^17,
    // ncols <= 8; checked exhaustively)
    const unsigned inv_cols = (1u << 20) / (unsigned)ncols + 1u;
    const int64_t K = it.kfar, mL = it.mL;
    const int64_t dmin = 1 - K / 16;
    const int64_t ndelta = K / 16 + R - 1;
    // the item's columns start at coff (time-major history: a plain shift)
    const gptr<const T> wbg = as_global(hk_weights<T>(G.w[it.comp], false));
    const gptr<const T> wag = as_global(hk_weights<T>(G.w[it.comp], true));
    const gptr<const T> hist = as_global(hk_history<T>(G)) + it.coff;
    const int64_t ldF = G.ldF;

    T* sw = reinterpret_cast<T*>(hk_smem);    // [2][kWlen] predictor, corrector weights
    T* sh = sw + 2 * kWlen;                   // [ncols][HST] history

    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int li = lane & 15, g = lane >> 4;

    // B column of this lane in every tile: (history column, row block rho).
    // A column beyond the item's columns only feeds its own, discarded,
    // output column, so its lanes read column 0 instead of branching.
    int bbase[TMAX];
#pragma unroll
    for (int tau = 0; tau < TMAX; ++tau) {
        const int idx = tau * 16 + li;
        const int c = idx / R < ncols ? idx / R : 0;
        bbase[tau] = c * HST + 17 * (idx % R) + g;
    }
    // A operand: row li, column 4s + g of the tile of shift dd sits at
    // 16 dd + 15 + li - 4s - g = abase + 16 dd + 4 (3 - s)
    const int abase = 3 + li - g;

    acc_t accP[TMAX], accC[TMAX];
    d4 sumP[TMAX], sumC[TMAX];
#pragma unroll
    for (int tau = 0; tau < TMAX; ++tau) {
        accP[tau] = acc_t{0, 0, 0, 0};
        accC[tau] = acc_t{0, 0, 0, 0};
        sumP[tau] = d4{0.0, 0.0, 0.0, 0.0};
        sumC[tau] = d4{0.0, 0.0, 0.0, 0.0};
    }

    const int c_begin = blockIdx.y * it.chunks_per_split;
    int c_end = c_begin + it.chunks_per_split;
    if (c_end > it.nchunks) c_end = it.nchunks;
    for (int chunk = c_begin; chunk < c_end; ++chunk) {
        const int64_t i0 = (int64_t)chunk * kDch;
        const int nd = (int)((ndelta - i0) < kDch ? (ndelta - i0) : kDch);
        const int64_t d0 = dmin + i0, d1 = d0 + nd;
        __syncthreads();   // the previous chunk's readers are done with the LDS
        // Staging: every load of a batch is issued before its first LDS store
        // (a load-then-store loop waits on each load in turn, which made the
        // staging, not the products, the cost of a chunk).
        // weights w_{mL - 16 + 16 d0 + x}, x < 16 nd + 15
        const int64_t wlo = mL - 16 + 16 * d0;
        const int nW = 16 * nd + 15;
        {
            constexpr int kWPer = (kWlen + 255) / 256;
            T vb[kWPer], va[kWPer];
#pragma unroll
            for (int u = 0; u < kWPer; ++u) {
                const int x = t + 256 * u;
                vb[u] = x < nW ? wbg[wlo + x] : T(0);
                va[u] = x < nW ? wag[wlo + x] : T(0);
            }
#pragma unroll
            for (int u = 0; u < kWPer; ++u) {
                const int x = t + 256 * u;
                if (x < nW) {
                    sw[x] = vb[u];
                    sw[kWlen + x] = va[u];
                }
            }
        }
        // history rows klo .. klo + nH - 1, zero outside 1..K; element e is row
        // e / ncols (by a reciprocal exact for these sizes), column e % ncols
        const int64_t klo = 17 - 16 * d1;
        const int nH = 16 * (nd + R - 1);
        const int nE = nH * ncols;
        constexpr int kBatch = 8;
        for (int e0 = t; e0 < nE; e0 += 256 * kBatch) {
            T v[kBatch];
            int at[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int e = e0 + 256 * u;
                const int x = (int)(((unsigned)e * inv_cols) >> 20);
                const int c = e - x * ncols;
                const int64_t k = klo + x;
                at[u] = e < nE ? c * HST + pad16(x) : -1;
                v[u] = (e < nE && k >= 1 && k <= K) ? hist[k * ldF + c] : T(0);
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u)
                if (at[u] >= 0) sh[at[u]] = v[u];
        }
        __syncthreads();
        for (int dd = wid; dd < nd; dd += kHWaves) {
            // shift delta = d0 + dd: B row 16 (rho + nd - 1 - dd) + 4s + g of the staged rows
            const T* pa = sw + abase + 16 * dd;
            const T* pb = sh + 17 * (nd - 1 - dd);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const T aP = pa[4 * (3 - s)];
                const T aC = pa[kWlen + 4 * (3 - s)];
#pragma unroll
                for (int tau = 0; tau < TMAX; ++tau) {
                    const T bv = pb[bbase[tau] + 4 * s];
                    accP[tau] = hk_mfma(aP, bv, accP[tau]);
                    accC[tau] = hk_mfma(aC, bv, accC[tau]);
                }
            }
            if constexpr (kFloat) {
#pragma unroll
                for (int tau = 0; tau < TMAX; ++tau) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        sumP[tau][v] += (double)accP[tau][v];
                        sumC[tau][v] += (double)accC[tau][v];
                    }
                    accP[tau] = acc_t{0, 0, 0, 0};
                    accC[tau] = acc_t{0, 0, 0, 0};
                }
            }
        }
    }
    if constexpr (!kFloat) {
#pragma unroll
        for (int tau = 0; tau < TMAX; ++tau) {
            sumP[tau] = accP[tau];
            sumC[tau] = accC[tau];
        }
    }

    // reduce the four waves' sums (wave order 0..3) and store: tile q is the
    // predictor tile q (q < TMAX) or the corrector tile q - TMAX
    double* red = reinterpret_cast<double*>(hk_smem);   // [kRedSlots][kHWaves][64][4]
    const gptr<double> out = as_global(G.part[(mL / L) & 1]) +
                             ((size_t)it.coff + (size_t)blockIdx.y * it.ldP) * (2 * L);
#pragma unroll
    for (int q0 = 0; q0 < 2 * TMAX; q0 += kRedSlots) {
        __syncthreads();   // LDS free (staging or the previous round)
#pragma unroll
        for (int u = 0; u < kRedSlots; ++u) {
            const int q = q0 + u;
            const int tau = q < TMAX ? q : q - TMAX;
            if (q < 2 * TMAX) {
                const d4 v = q < TMAX ? sumP[tau] : sumC[tau];
                double* dst = red + ((size_t)(u * kHWaves + wid) * 64 + lane) * 4;
#pragma unroll
                for (int x = 0; x < 4; ++x) dst[x] = v[x];
            }
        }
        __syncthreads();
        const int q = q0 + wid;            // wave wid finishes slot wid
        const int tau = q < TMAX ? q : q - TMAX;
        if (q < 2 * TMAX) {
            double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int w = 0; w < kHWaves; ++w) {
                const double* src = red + ((size_t)(wid * kHWaves + w) * 64 + lane) * 4;
#pragma unroll
                for (int x = 0; x < 4; ++x) s[x] += src[x];
            }
            const int idx = tau * 16 + li;
            const int c = idx / R, rho = idx % R;
            if (c < ncols) {
                const gptr<double> o = out + (size_t)c * (2 * L) + (q < TMAX ? 0 : L) + 16 * rho;
#pragma unroll
                for (int v = 0; v < 4; ++v) o[hk_row<T>(g, v)] = s[v];
            }
        }
    }
}

template <typename T, int L>
__global__ __launch_bounds__(256, 2) void k_far_hankel(const GroupDev* __restrict__ groups,
                                                     const FarItem* __restrict__ items)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char hk_smem[];
    const FarItem it = items[blockIdx.z];
    if ((int)blockIdx.y >= it.nsplit) return;
    const GroupDev& G = groups[it.group];
    switch (it.ncoltiles) {
    case 1: hankel_body<T, L, 1>(G, it, hk_smem); break;
    case 2: hankel_body<T, L, 2>(G, it, hk_smem); break;
    case 3: hankel_body<T, L, 3>(G, it, hk_smem); break;
    case 4: hankel_body<T, L, 4>(G, it, hk_smem); break;
    default: break;   // the host never plans more than kHMaxTiles tiles
    }
}

template <typename T, int L>
hipError_t launch_hk(const GroupDev* groups, const FarItem* items, int n, int max_tiles,
                     int max_nsplit, hipStream_t st)
{
    const size_t shmem = hankel_lds_bytes(L, max_tiles, sizeof(T) == 4 ? ABM_FAR_FP32 : ABM_FAR_FP64);
    const dim3 grid(1u, (unsigned)max_nsplit, (unsigned)n);
    hipError_t e;
    if ((e = allow_lds(reinterpret_cast<const void*>(&k_far_hankel<T, L>), shmem)) != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_far_hankel<T, L>), grid, dim3(256), shmem, st, groups, items);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_hk_l(const GroupDev* groups, const FarItem* items, int n, int max_tiles,
                       int max_nsplit, int L, hipStream_t st)
{
    switch (L) {
    case 64: return launch_hk<T, 64>(groups, items, n, max_tiles, max_nsplit, st);
    case 128: return launch_hk<T, 128>(groups, items, n, max_tiles, max_nsplit, st);
    case 256: return launch_hk<T, 256>(groups, items, n, max_tiles, max_nsplit, st);
    case 512: return launch_hk<T, 512>(groups, items, n, max_tiles, max_nsplit, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int hankel_tiles(int64_t cols, int L)
{
    const int64_t R = L / 16;
    return (int)((cols * R + 15) / 16);
}

bool hankel_fits(int prec, int64_t cols, int L)
{
    if (prec != ABM_FAR_FP64 && prec != ABM_FAR_FP32) return false;
    return cols >= 1 && cols <= kHankelMaxCols && hankel_tiles(cols, L) <= kHMaxTiles;
}

int hankel_chunk_rows() { return 16 * kDch; }

int hankel_split_plan(int64_t kfar, int L, int max_split, int* nchunks, int* chunks_per_split)
{
    if (kfar < 1) {
        *nchunks = 0;
        *chunks_per_split = 0;
        return 0;
    }
    // shifts 1 - K/16 .. L/16 - 1 in chunks of kDch.  A slice takes at least
    // kMinChunks chunks: every slice is one more partial row the chain sums
    // before its block, and a narrow group's far field (a few tiles wide) is
    // short beside its chain anyway, so fewer, longer slices pay while the
    // history is short (one 10^6-step trajectory: 0.59 -> 0.47 s; 3·10^6 steps:
    // 2.24 -> 2.04 s, measured against 1, 4 and 16 chunks per slice).
    const int64_t rows = kfar + L - 16, chunk = 16 * kDch;
    const int64_t want = ((rows + chunk - 1) / chunk + kMinChunks - 1) / kMinChunks;
    const int cap = (int)(want < max_split ? want : max_split);
    return far_split_plan(rows, (int)chunk, cap, nchunks, chunks_per_split);
}

int hankel_split_bound(int64_t kfar_max, int L, int max_split)
{
    if (kfar_max < 1) return 0;
    // hankel_split_plan gives at most min(ceil(chunks / kMinChunks), max_split)
    // slices, and its chunk count only grows with kfar
    const int64_t nc = (kfar_max + L - 16 + 16 * kDch - 1) / (16 * kDch);
    const int64_t want = (nc + kMinChunks - 1) / kMinChunks;
    return (int)(want < max_split ? want : max_split);
}

size_t hankel_lds_bytes(int L, int max_tiles, int prec)
{
    const size_t es = prec == ABM_FAR_FP32 ? sizeof(float) : sizeof(double);
    const int R = L / 16;
    int64_t ncols = (int64_t)16 * max_tiles / R;          // columns that fit max_tiles tiles
    if (ncols > kHankelMaxCols) ncols = kHankelMaxCols;
    if (ncols < 1) ncols = 1;
    const size_t stage = (2 * (size_t)kWlen + (size_t)ncols * 17 * (kDch + R - 1)) * es;
    const size_t red = (size_t)kRedSlots * kHWaves * 64 * 4 * sizeof(double);
    return stage > red ? stage : red;
}

// The partial slices of a narrow far item summed into its first slice, in
// slice order (the order in which the chain would add them).  One thread per
// (column, row) of the item; the chain of the block then reads one slice.
// Many threads share the loads that one chain wave would otherwise make one
// lane at a time.
namespace {

__global__ __launch_bounds__(256) void k_far_reduce(const GroupDev* groups, const FarItem* items,
                                                    int L)
{
    const FarItem it = items[blockIdx.y];
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;   // col * 2L + row
    if (it.nsplit < 2 || e >= (int64_t)it.ncols * 2 * L) return;
    const GroupDev& G = groups[it.group];
    const gptr<double> base = as_global(G.part[(it.mL / L) & 1]) + (int64_t)it.coff * (2 * L) + e;
    const size_t ss = (size_t)it.ldP * (2 * L);
    double acc = base[0];
    int sl = 1;
    for (; sl + 8 <= it.nsplit; sl += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = base[(size_t)(sl + u) * ss];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; sl < it.nsplit; ++sl) acc += base[(size_t)sl * ss];
    base[0] = acc;
}

}  // namespace

hipError_t launch_far_reduce(const GroupDev* groups, const FarItem* items, int n, int max_cols,
                             int L, hipStream_t st)
{
    if (n < 1 || max_cols < 1) return hipSuccess;
    const int64_t elems = (int64_t)max_cols * 2 * L;
    hipLaunchKernelGGL(k_far_reduce, dim3((unsigned)((elems + 255) / 256), (unsigned)n), dim3(256), 0, st,
                       groups, items, L);
    return hipGetLastError();
}

hipError_t launch_far_hankel(const GroupDev* groups, const FarItem* items, int n, int max_tiles,
                             int max_nsplit, int L, int prec, hipStream_t st)
{
    if (n < 1 || max_tiles < 1 || max_nsplit < 1) return hipSuccess;
    if (max_tiles > kHMaxTiles) return hipErrorInvalidValue;
    if (prec == ABM_FAR_FP32) return launch_hk_l<float>(groups, items, n, max_tiles, max_nsplit, L, st);
    if (prec == ABM_FAR_FP64) return launch_hk_l<double>(groups, items, n, max_tiles, max_nsplit, L, st);
    return hipErrorInvalidValue;
}

}  // namespace abm
