// K2 with integer limbs: the far-field products of the blocked method on the
// int8 matrix cores, summed exactly.  The sums are those of far.hip:
//   FF[r]     = sum_{k=1..K} b_{mL+r-k} F_k,   FF[L + r] = sum_{k=1..K} a_{mL+r-k} F_k.
//
// Operands as integers.  A weight window (the weights one chunk of history
// rows meets, per table b or a) is scaled by 2^ew so that its largest |w|
// lies in [32, 64) and rounded to a multiple of 2^-24: four balanced base-256
// digits d0 + d1 2^-8 + d2 2^-16 + d3 2^-24 with |d0| <= 64 and d1..d3 in
// [-128, 127] (30 bits).  The history is scaled per block of L rows and
// column and cut into three digits e0 + e1 2^-8 + e2 2^-16 at resolution
// 2^-16 with |e0| <= 127 (written by the chain, chain.hip, which keeps a
// column's scale from one block to the next while the block's largest |f|
// stays within [16, 127) of it).  A
// product w F is then
//   2^-(ew+ef) sum_{i,j} d_i e_j 2^-8(i+j),
// and the nine digit products with i + j <= 3 are kept (the dropped ones
// weigh at most 2^-32 of the leading one).  Digit products of one level
// l = i + j go to one int32 accumulator: integer sums are exact and their
// order is immaterial, so the rows of one weight window and one history
// scale are summed with no rounding at all (a level sum grows by at most
// 3 * 2^14 per row, and a chunk is at most 4608 rows, far below 2^31).  When
// a column's history scale changes, and at the end of each chunk, the four
// levels are combined in double (exactly: every partial is a multiple of
// 2^-24 below 2^27) and added, scaled, into the double accumulator.  Weights
// need more digits than the history: a rounding error of a weight repeats in
// every step that uses it, while the history's errors do not line up, so 30
// bits of weights and 21-22 of history keep the whole sweep near 8e-8 where
// 22 bits of weights alone give about 1e-6.
//
// Tiling: v_mfma_i32_32x32x32_i8, row tiles of 32 rows and 32 columns,
// K-steps of 32 history rows.  Lane (li = lane%32, g = lane/32) supplies row
// li, history rows 16g..16g+15 of the A fragment (16 bytes) and column li, the
// same rows of the B fragment; result row 8(v/4) + 4g + v%4, column li sits in
// register v.  The Toeplitz A fragment of row tile t at K-step q starts at
// byte L-1-rbase-li+16g + 32(q - t) of the reversed weight window, so
// fragment(t, q) = fragment(t+1, q+1): one new fragment per limb and step.
// The fragments of step q + 1 (four weight limbs, three history limbs) are
// read from the LDS while step q's 18 products run, one read issued after
// each of the first eleven products.  The window is held in four copies
// shifted by 0..3 bytes; each lane reads the copy that makes its fragments
// dword-aligned, and the copies lie 8 dwords apart modulo the 32 LDS banks so
// that the lanes reading one dword offset in the four copies hit different
// banks.  Each wave holds 2 row tiles (64 rows x 32 columns), a workgroup 4
// waves (256 rows: the predictor or the corrector rows of a block at L = 256,
// both at L = 128).  Registers hold the exact level sums and two steps of
// fragments (256 per lane); the double sums between flushes live in a
// per-wave LDS region.  A workgroup's ~125 KB of LDS leaves room for one
// chain workgroup (32 KB) beside it on a CU.
#include "far_common.h"

namespace abm {

namespace {

typedef int i4 __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

constexpr int kWLimbs = 4, kFLimbs = 3, kCopies = 4;
constexpr int kCopyPad = 32;                // bytes between window copies (bank offset)

// Exponent e such that m 2^e lies in [32, 64) (0 for m = 0 or not finite).
__device__ __forceinline__ int i8_exponent(double m)
{
    if (!(m > 0.0) || !isfinite(m)) return 0;
    int ex;
    (void)frexp(m, &ex);                                   // m = f 2^ex, 0.5 <= f < 1
    return 6 - ex;
}

// Balanced base-256 digits of w 2^e (|w 2^e| < 64) at resolution 2^-24.
__device__ __forceinline__ void weight_digits(double w, int e, int (&d)[kWLimbs])
{
    int64_t I = (int64_t)rint(ldexp(w, e + 24));
#pragma unroll
    for (int i = kWLimbs - 1; i >= 1; --i) {
        const int64_t r = ((I + 128) & 255) - 128;
        d[i] = (int)r;
        I = (I - r) >> 8;
    }
    d[0] = (int)I;
}

// History stages: kStageBufs buffers of 128 rows x 32 columns x 3 limbs,
// copied global -> LDS by DMA (q32_dma_stage) kStageBufs - 1 stages ahead.
#ifndef I8_NBUF
#define I8_NBUF 2
#endif
constexpr int kStageBufs = I8_NBUF;
constexpr int kQ32Stage = 128;                               // history rows per LDS stage
constexpr int kQ32StageU4 = 3 * (kQ32Stage / 16) * 32;       // 16-byte units per stage
constexpr int kDmaPerStage = kQ32StageU4 / 256;              // copies per thread and stage (256 threads)

template <int NTH>
__device__ __forceinline__ void q32_dma_stage(gptr<const int8_t> q0, gptr<const int8_t> q1,
                                              gptr<const int8_t> q2, int64_t ldF, int col0,
                                              int64_t blk0, int t, u4* dst)
{
    constexpr int TN = 32, kLimbU4 = (kQ32Stage / 16) * TN;
    static_assert(kQ32StageU4 % 64 == 0 && NTH % 64 == 0, "a wave copies whole 1 KiB runs");
    const int lane = t & 63;
#pragma unroll
    for (int e = 0; e < (kQ32StageU4 + NTH - 1) / NTH; ++e) {
        const int u = t + e * NTH;
        if (u - lane < kQ32StageU4) {
            const int tt = u / kLimbU4, rem = u % kLimbU4;
            const int b = rem / TN, c = rem % TN;
            const gptr<const int8_t> src =
                (tt == 0 ? q0 : (tt == 1 ? q1 : q2)) + ((blk0 + b) * ldF + col0 + c) * 16;
            __builtin_amdgcn_global_load_lds((const ABM_GLOBAL void*)src,
                                             (__attribute__((address_space(3))) void*)(dst + (u - lane)),
                                             16, 0, 0);
        }
    }
}

typedef int i16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ i16v mfma_i8_32(i4 a, i4 b, i16v c)
{
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

template <int L>
__global__ __launch_bounds__(256, 2) void k_far_i8_32(const GroupDev* groups, const FarItem* items,
                                                      int kchunk, int cpad)
{
    constexpr int MT = 2, TN = 32, NTH = 256, ROWS = 256;   // rows per workgroup
    constexpr int KW = 2 * L / ROWS;            // workgroups per column tile
    constexpr int NK = ROWS / L > 1 ? ROWS / L : 1;          // row kinds per workgroup
    constexpr int QS = kQ32Stage / 32;          // K-steps per stage
    constexpr int GSTEPS = L / 32;              // K-steps per history block
    static_assert(kQ32StageU4 == kDmaPerStage * NTH, "each thread issues kDmaPerStage copies per stage");
    // blockIdx.x = sub * (column tiles of the grid) + tile: the predictor and
    // corrector workgroups of one column tile are a multiple of 8 apart in
    // dispatch order (the grid's tile count is a multiple of 8), so they land
    // on the same XCD and the second reads the tile's history from that L2
    const int ntg = (int)gridDim.x / KW;
    const int sub = KW > 1 ? (int)blockIdx.x / ntg : 0;
    const int tile = KW > 1 ? (int)blockIdx.x % ntg : (int)blockIdx.x;
    FarArgs A;
    if (!far_view_at(groups, items, blockIdx.z, tile, blockIdx.y, kchunk, L, A)) return;
    extern __shared__ __attribute__((aligned(16))) int8_t smq[];
    const int win = L + A.kchunk + cpad;
    int8_t* wq = smq;                           // [kind of the workgroup][limb][copy][win]
    u4* Bst = reinterpret_cast<u4*>(smq + NK * kWLimbs * kCopies * win);   // [kStageBufs][kQ32StageU4]

    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int col0 = tile * TN;
    const int rowbase = sub * ROWS + wid * 64;  // first of this wave's 64 rows in 0..2L
    const int kind = rowbase / L;               // 0: predictor (b), 1: corrector (a)
    const int wk = NK > 1 ? kind : 0;           // the kind's window in this workgroup
    const int rbase = rowbase % L;
    const int li = lane & 31, g = lane >> 5;
    const int abase = L - 1 - rbase - li + 16 * g;  // fragment v starts at abase + 32 v
    const int par = abase & 3;
    const int8_t* wl = wq + (wk * kWLimbs * kCopies + par) * win + (abase - par);
    auto afrag = [&](int l, int v) -> i4 {
        const uint32_t* q = reinterpret_cast<const uint32_t*>(wl + l * kCopies * win + 32 * v);
        u4 x;
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = q[k];
        return __builtin_bit_cast(i4, x);
    };

    const gptr<const int8_t> q0 = A.Fq[0], q1 = A.Fq[1], q2 = A.Fq[2];
    // the workgroup's kinds: kind0 .. kind0 + NK - 1
    const int kind0 = (sub * ROWS) / L;
    // FFpart[split][col][2L]: row 8(v/4) + 4g + v%4 of column li of tile i in
    // register v.
    const gptr<double> out = A.part + (size_t)blockIdx.y * A.ldP * (2 * L) + (size_t)(col0 + li) * (2 * L) +
                             rowbase + 4 * g;
    // The double sums of this wave's 64 x 32 outputs between flushes (a
    // history scale change or a chunk's end): values v, v + 1 of tile i of
    // lane `lane` at accs[(8 i + v/2) * 64 + lane], one LDS region per wave
    // (registers hold the exact level sums and the fragments of two K-steps).
    // The split's last flush writes FFpart instead.
    double2* accs = reinterpret_cast<double2*>(smq + NK * kWLimbs * kCopies * win + kStageBufs * kQ32StageU4 * 16) +
                    wid * (MT * 8 * 64);
    bool first = true;
    auto bfrag = [&](const u4* Bs, int qq, int j) -> i4 {
        return __builtin_bit_cast(i4, Bs[(j * (kQ32Stage / 16) + 2 * qq + g) * TN + li]);
    };

    const int c_begin = blockIdx.y * A.chunks_per_split;
    int c_end = c_begin + A.chunks_per_split;
    if (c_end > A.nchunks) c_end = A.nchunks;
    for (int chunk = c_begin; chunk < c_end; ++chunk) {
        const ChunkBounds cb = chunk_bounds(A, L, chunk);
        const int64_t kb16 = (cb.k_lo - 1) >> 4;
        const int nstages = cb.nk / kQ32Stage;
        __syncthreads();   // previous chunk's readers are done with the LDS
        int ew[2];
        ew[0] = i8_exponent(fmax(fabs(A.b[cb.jb]), fabs(A.b[cb.jb + cb.wlen - 1])));
        ew[1] = i8_exponent(fmax(fabs(A.a[cb.jb]), fabs(A.a[cb.jb + cb.wlen - 1])));
        const double wscale = ldexp(1.0, -ew[kind]);
        constexpr int WB = 12;   // all of a thread's weights of a 2304-wide window in one batch of loads
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const gptr<const double> w = (kind0 + k) == 0 ? A.b : A.a;
            const int e = ew[kind0 + k];
            int8_t* wk0 = wq + k * kWLimbs * kCopies * win;
            for (int x0 = t; x0 < cb.wlen; x0 += WB * NTH) {
                double vv[WB];
#pragma unroll
                for (int u = 0; u < WB; ++u) {
                    const int x = x0 + u * NTH;
                    vv[u] = w[cb.jb + cb.wlen - 1 - (x < cb.wlen ? x : 0)];
                }
#pragma unroll
                for (int u = 0; u < WB; ++u) {
                    const int x = x0 + u * NTH;
                    if (x >= cb.wlen) break;
                    int d[kWLimbs];
                    weight_digits(vv[u], e, d);
#pragma unroll
                    for (int p = 0; p < kCopies; ++p)
                        if (x >= p) {
#pragma unroll
                            for (int l = 0; l < kWLimbs; ++l) wk0[(l * kCopies + p) * win + x - p] = (int8_t)d[l];
                        }
                }
            }
        }
        for (int s0 = 0; s0 < kStageBufs - 1 && s0 < nstages; ++s0)
            q32_dma_stage<NTH>(q0, q1, q2, A.ldF, col0, kb16 + (int64_t)s0 * (kQ32Stage / 16), t,
                               Bst + s0 * kQ32StageU4);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        // Fragments of K-step q: aC[l] = window fragment v = q (row tile 0),
        // aP[l] = v = q - 1 (row tile 1), bC[j] the history's; those of step
        // q + 1 are read from the LDS while step q's products run.
        i4 aP[kWLimbs], aC[kWLimbs], bC[kFLimbs];
#pragma unroll
        for (int l = 0; l < kWLimbs; ++l) {
            aC[l] = afrag(l, 0);
            aP[l] = afrag(l, -1);
        }
#pragma unroll
        for (int j = 0; j < kFLimbs; ++j) bC[j] = bfrag(Bst, 0, j);
        const int64_t b0 = (cb.k_lo - 1) / L;
        double fsc = A.Fqs[b0 * A.ldF + col0 + li];
        double fsc_nx = cb.nk > L ? A.Fqs[(b0 + 1) * A.ldF + col0 + li] : 0.0;
        // [level][tile]: exact sums, flushed by the chunk's end
        i16v acc[4][MT];
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int l = 0; l < 4; ++l) acc[l][i] = i16v{};
        const int nsteps = cb.nk / 32;
        for (int st = 0; st < nstages; ++st) {
            const u4* Bs = Bst + (st % kStageBufs) * kQ32StageU4;
            const u4* Bnext = Bst + ((st + 1) % kStageBufs) * kQ32StageU4;
            // the copy of stage st + kStageBufs - 1 runs under the K-steps of
            // the stages before it (its buffer was last read before the
            // previous stage's closing barrier)
            const int sa = st + kStageBufs - 1;
            if (sa < nstages)
                q32_dma_stage<NTH>(q0, q1, q2, A.ldF, col0, kb16 + (int64_t)sa * (kQ32Stage / 16), t,
                                   Bst + (sa % kStageBufs) * kQ32StageU4);
#pragma unroll
            for (int qq = 0; qq < QS; ++qq) {
                const int q = st * QS + qq;
                const bool more = qq + 1 < QS || st + 1 < nstages;   // step q + 1 exists
                i4 aN[kWLimbs], bN[kFLimbs];
#pragma unroll
                for (int l = 0; l < kWLimbs; ++l) aN[l] = more ? afrag(l, q + 1) : aC[l];
                if (qq + 1 < QS) {
#pragma unroll
                    for (int j = 0; j < kFLimbs; ++j) bN[j] = bfrag(Bs, qq + 1, j);
                }
                // digit products (i, j), i + j <= 3, into level i + j, ordered so
                // that products of one level are at least two apart:
                // (0,0) (0,1) (0,2) (1,2) (1,0) (1,1) (2,1) (2,0) (3,0)
                constexpr int pw[9] = {0, 0, 0, 1, 1, 1, 2, 2, 3};
                constexpr int ph[9] = {0, 1, 2, 2, 0, 1, 1, 0, 0};
#pragma unroll
                for (int pp = 0; pp < 9; ++pp)
#pragma unroll
                    for (int tm = 0; tm < MT; ++tm) {
                        const int lv = pw[pp] + ph[pp];
                        const i4 a = tm == 0 ? aC[pw[pp]] : aP[pw[pp]];
                        acc[lv][tm] = mfma_i8_32(a, bC[ph[pp]], acc[lv][tm]);
                    }
                if (qq + 1 == QS) {
                    if (more) {
                        // the next stage's copy is in (later stages' copies,
                        // issued after it, may still run): its first fragments
                        if (kStageBufs > 2 && st + kStageBufs - 1 < nstages)
                            asm volatile("s_waitcnt vmcnt(%0)" ::"n"((kStageBufs - 2) * kDmaPerStage) : "memory");
                        else
                            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                        __syncthreads();
#pragma unroll
                        for (int j = 0; j < kFLimbs; ++j) bN[j] = bfrag(Bnext, 0, j);
                    } else {
#pragma unroll
                        for (int j = 0; j < kFLimbs; ++j) bN[j] = bC[j];
                    }
                }
                if ((q + 1) % GSTEPS == 0) {
                    const bool last = !more;
                    const double fnx = last ? 0.0 : fsc_nx;
                    if (last || __any(fnx != fsc)) {
                        const double sc = wscale * fsc;
                        const bool to_out = last && chunk + 1 == c_end;
#pragma unroll
                        for (int tm = 0; tm < MT; ++tm) {
                            double2 prev[8];
#pragma unroll
                            for (int vp = 0; vp < 8; ++vp)
                                prev[vp] = first ? double2{0.0, 0.0} : accs[(tm * 8 + vp) * 64 + lane];
#pragma unroll
                            for (int vp = 0; vp < 8; ++vp) {
                                double r[2];
#pragma unroll
                                for (int h = 0; h < 2; ++h) {
                                    const int v = 2 * vp + h;
                                    double T = fma((double)acc[1][tm][v], 0x1p-8, (double)acc[0][tm][v]);
                                    T = fma((double)acc[2][tm][v], 0x1p-16, T);
                                    T = fma((double)acc[3][tm][v], 0x1p-24, T);
                                    r[h] = fma(T, sc, h ? prev[vp].y : prev[vp].x);
                                }
                                if (to_out) {
                                    const gptr<double> o = out + tm * 32 + 8 * (vp / 2) + 2 * (vp % 2);
                                    o[0] = r[0];
                                    o[1] = r[1];
                                } else {
                                    accs[(tm * 8 + vp) * 64 + lane] = double2{r[0], r[1]};
                                }
                            }
#pragma unroll
                            for (int l = 0; l < 4; ++l) acc[l][tm] = i16v{};
                        }
                        first = false;
                    }
                    if (!last) {
                        fsc = fnx;
                        const int64_t nb = b0 + (q + 1) / GSTEPS + 1;
                        if ((q + 1) / GSTEPS + 1 < nsteps / GSTEPS) fsc_nx = A.Fqs[nb * A.ldF + col0 + li];
                    }
                }
#pragma unroll
                for (int l = 0; l < kWLimbs; ++l) {
                    aP[l] = aC[l];
                    aC[l] = aN[l];
                }
#pragma unroll
                for (int j = 0; j < kFLimbs; ++j) bC[j] = bN[j];
                // step q + 1's reads spread over the first products of step q
#pragma unroll
                for (int k = 0; k < 11; ++k) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one product
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
                }
                __builtin_amdgcn_sched_group_barrier(0x008, 7, 0);
                // keep the scheduler from pulling step q + 1's products up to
                // the reads that feed them
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    if (first) {   // no history rows in this split
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int v = 0; v < 16; ++v) out[i * 32 + 8 * (v / 4) + (v % 4)] = 0.0;
    }
}

template <int L>
hipError_t launch_i8_32_t(const GroupDev* groups, const FarItem* items, int n, int max_coltiles,
                          int max_nsplit, int kchunk, hipStream_t st)
{
    const size_t shmem = far_i8_lds_bytes(L, kchunk);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_far_i8_32<L>), shmem);
    if (e != hipSuccess) return e;
    constexpr int KW = 2 * L / 256;
    const int ntg = (max_coltiles + 7) / 8 * 8;     // tile count of the grid: a multiple of 8
    hipLaunchKernelGGL((k_far_i8_32<L>), dim3((unsigned)(ntg * KW), (unsigned)max_nsplit, (unsigned)n),
                       dim3(256), shmem, st, groups, items, kchunk, kCopyPad);
    return hipGetLastError();
}

}  // namespace

int far_i8_tile_cols() { return 32; }

size_t far_i8_lds_bytes(int L, int kchunk)
{
    const int nk = L >= 256 ? 1 : 2;           // weight windows per workgroup
    constexpr size_t kAccBytes = 4 * 64 * 2 * 16 * sizeof(double);   // 4 waves x 64 lanes x 2 tiles x 16
    return (size_t)nk * kWLimbs * kCopies * (L + kchunk + kCopyPad) + (size_t)kStageBufs * kQ32StageU4 * 16 +
           kAccBytes;
}

hipError_t launch_far_i8(const GroupDev* groups, const FarItem* items, int n, int max_coltiles,
                         int max_nsplit, int kchunk, int L, hipStream_t st)
{
    switch (L) {
    case 128: return launch_i8_32_t<128>(groups, items, n, max_coltiles, max_nsplit, kchunk, st);
    case 256: return launch_i8_32_t<256>(groups, items, n, max_coltiles, max_nsplit, kchunk, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace abm
