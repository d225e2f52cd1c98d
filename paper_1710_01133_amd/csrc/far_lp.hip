// K2 in reduced precision: the far-field products of the blocked method with
// the weights and the history rounded once to float, or split into bf16
// terms, on the matrix cores.  The sums are the same as in far.hip:
//   FF[r]     = sum_{k=1..K} b_{mL+r-k} F_k,   FF[L + r] = sum_{k=1..K} a_{mL+r-k} F_k.
// Accumulation is float only inside short runs of history rows (one 32-row
// bf16 product step, or 16 rows of float products): their results are then
// added into double accumulators, so float rounding is never applied to a
// sum that has grown over many rows.  A workgroup walks a fixed range of
// history chunks, carrying the double sums, and writes one partial per
// column; the chain adds the partials of the block in double.
//
// bf16 split: x ~ x0 + x1 (+ x2) with x0 = bf16(x), x1 = bf16(x - x0), ...
// (the float value of x is carried exactly by three terms).  Products kept:
//   bf16x3: w0 F0 + w0 F1 + w1 F0
//   bf16x6: the above + w1 F1 + w0 F2 + w2 F0
// so the dropped products are below 2^-16 (x3) and 2^-24 (x6) of w F.
//
// Tiling: a workgroup computes all 2L rows of the block for 16 columns.  In
// float, 8 waves: waves 0-3 hold L/4 predictor rows each, waves 4-7 the
// corrector rows.  In bf16, each wave holds 8 row tiles (128 rows) when
// L <= 256, so a workgroup is 2L/128 waves, one per SIMD with the whole
// register file: the history fragment of a product step is then read from
// LDS once per 8 tiles instead of once per 4, which halves the LDS traffic
// that otherwise limits these products (L = 512 keeps 4 tiles per wave).
// Reduced precision needs L >= 128.
//
// Operand layout of the bf16 16x16x32 product: lane (li = lane%16, g = lane/16)
// supplies row li, history rows 8g..8g+7 of the A fragment and column li,
// the same history rows of the B fragment; the result row 4g + v, column li
// sits in register v.  The Toeplitz A fragment of M-tile t at K-step q starts
// at LDS offset  L-1-rbase-li + 8g + 32q - 16t  of the reversed weight window,
// so fragment(t, q) = fragment(t+2, q+1): a ring of MT fragments per split
// term is kept in registers and only two new ones are read per K-step (the
// 2-byte-aligned 16-byte LDS reads are single ds_read_b128 on gfx950).
#include "far_common.h"

namespace abm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

template <int MT, int NT>
__device__ __forceinline__ void flush_acc(f4 (&acc)[MT][NT], d4 (&acc64)[MT][NT])
{
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[i][j][v] += (double)acc[i][j][v];
            acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
}

// Result of the workgroup: FFpart[split][col][2L]; float/bf16 products return
// row 4g + v of column li of a tile in register v of lane (li, g).
template <int MT, int NT>
__device__ __forceinline__ void store_part(const FarArgs& A, const d4 (&acc64)[MT][NT], int col0,
                                           int prow, int li, int g, int L)
{
    const gptr<double> out = A.part + (size_t)blockIdx.y * A.ldP * (2 * L);
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const gptr<double> o = out + (size_t)(col0 + j * 16 + li) * (2 * L) + prow + i * 16 + 4 * g;
#pragma unroll
            for (int v = 0; v < 4; ++v) o[v] = acc64[i][j][v];
        }
}

// ------------------------------------------------------------------ float
// 8 waves: waves 0-3 own predictor rows, 4-7 corrector rows, L/4 rows each.
template <int MT>
__global__ __launch_bounds__(512, 1) void k_far_f32(const GroupDev* groups, const FarItem* items,
                                                    int kchunk)
{
    constexpr int L = 64 * MT, TN = 16;
    FarArgs A;
    if (!far_view(groups, items, kchunk, L, A)) return;
    constexpr int KS = 32;                      // history rows per LDS stage
    constexpr int kFlushSteps = 4;              // 16 history rows per float run
    extern __shared__ float smf[];
    const int win = L + A.kchunk;
    float* wb = smf;
    float* wa = smf + win;
    float* Ft = smf + 2 * win;                  // [2][KS][TN]

    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int col0 = blockIdx.x * TN;
    const int64_t mL = A.mL;
    const bool corr = wid >= 4;
    const int rbase = (wid & 3) * (L / 4);
    const float* wwin = corr ? wa : wb;
    const int li = lane & 15, lk = lane >> 4;

    f4 acc[MT][1];
    d4 acc64[MT][1];
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        acc[i][0] = f4{0.f, 0.f, 0.f, 0.f};
        acc64[i][0] = d4{0.0, 0.0, 0.0, 0.0};
    }

    constexpr int kStageElems = KS * TN;        // 512: one element per thread
    float pre = 0.f;
    // column-blocked float history: this workgroup's 16 columns are contiguous
    const gptr<const float> Fblk = A.F32 + (int64_t)(col0 >> 4) * A.rows * 16;
    auto load_stage = [&](int64_t k0) { pre = Fblk[k0 * 16 + t]; };
    auto store_stage = [&](int buf) { Ft[buf * kStageElems + t] = pre; };

    const int c_begin = blockIdx.y * A.chunks_per_split;
    int c_end = c_begin + A.chunks_per_split;
    if (c_end > A.nchunks) c_end = A.nchunks;
    for (int chunk = c_begin; chunk < c_end; ++chunk) {
        const ChunkBounds cb = chunk_bounds(A, L, chunk);
        __syncthreads();   // previous chunk's readers are done with the LDS
        // weight window: the loads of a batch are all issued before its stores
        for (int x0 = t; x0 < cb.wlen; x0 += 512 * 4) {
            float vb[4], va[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int x = x0 + 512 * u;
                vb[u] = x < cb.wlen ? A.b32[cb.jb + x] : 0.f;
                va[u] = x < cb.wlen ? A.a32[cb.jb + x] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int x = x0 + 512 * u;
                if (x < cb.wlen) {
                    wb[x] = vb[u];
                    wa[x] = va[u];
                }
            }
        }
        load_stage(cb.k_lo);
        store_stage(0);
        __syncthreads();
        const int nstages = cb.nk / KS;
        for (int st = 0; st < nstages; ++st) {
            const int buf = st & 1;
            if (st + 1 < nstages) load_stage(cb.k_lo + (int64_t)(st + 1) * KS);
            const float* Fs = Ft + buf * kStageElems;
#pragma unroll
            for (int kq = 0; kq < KS / 4; ++kq) {
                const int64_t k = cb.k_lo + (int64_t)st * KS + kq * 4 + lk;
                const float bf = Fs[(kq * 4 + lk) * TN + li];
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    const int r = rbase + i * 16 + li;
                    const float af = wwin[(int)(mL + r - k - cb.jb)];
                    acc[i][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bf, acc[i][0], 0, 0, 0);
                }
                if ((kq + 1) % kFlushSteps == 0) flush_acc<MT, 1>(acc, acc64);
            }
            if (st + 1 < nstages) store_stage(buf ^ 1);
            __syncthreads();
        }
    }
    store_part<MT, 1>(A, acc64, col0, (corr ? L : 0) + rbase, li, lk, L);
}

// ------------------------------------------------------------------ bf16 split
// History stages of the bf16 kernels: two buffers of 128 rows x 16 columns x
// up to 3 split terms.  A stage is copied from global memory straight into
// LDS (no registers in between, which keeps the kernel within its register
// budget).  The copy of stage st+1 is issued in the last product step of
// stage st, after that step's LDS reads: the compiler makes every later LDS
// read wait for the copy, and the next such read comes after the stage
// barrier anyway, so the copy runs under the last step's products.
constexpr int kBfStageRows = 128;
constexpr int kBfStageU4 = 3 * (kBfStageRows / 8) * 16;   // 16-byte units per stage

// Copy of one history stage (8-row blocks blk0 .. blk0 + NB8 - 1 of 16
// columns from col0, TERMS split terms) into LDS at dst.  Unit
// u = tt * NB8 * 16 + 16 b + c holds the 8 rows of block b, column c, term
// tt; thread t copies units t, t + NTH, ...  A wave's 64 units are
// consecutive, so each lane's 16 bytes land at (the wave's first unit +
// lane), which is where the copy puts them.  Arguments by value: the term's
// pointer is then a select among values (a select among addresses of the
// caller's variables would move them to scratch memory).
template <int TERMS, int NB8, int NTH>
__device__ __forceinline__ void bf_dma_stage(gptr<const uint16_t> fh0, gptr<const uint16_t> fh1,
                                             gptr<const uint16_t> fh2, int64_t ldF, int col0,
                                             int64_t blk0, int t, u4* dst)
{
    constexpr int TN = 16, kTermU4 = NB8 * TN, kStageU4 = TERMS * kTermU4;
    static_assert(kTermU4 % 64 == 0 && NTH % 64 == 0, "a wave copies whole 1 KiB runs");
    const int lane = t & 63;
#pragma unroll
    for (int e = 0; e < (kStageU4 + NTH - 1) / NTH; ++e) {
        const int u = t + e * NTH;
        if (u - lane < kStageU4) {          // whole waves only
            const int tt = u / kTermU4, rem = u % kTermU4;
            const int b = rem / TN, c = rem % TN;
            const gptr<const uint16_t> src =
                (tt == 0 ? fh0 : (tt == 1 ? fh1 : fh2)) + ((blk0 + b) * ldF + col0 + c) * 8;
            __builtin_amdgcn_global_load_lds((const ABM_GLOBAL void*)src,
                                             (__attribute__((address_space(3))) void*)(dst + (u - lane)),
                                             16, 0, 0);
        }
    }
}

// Wait for this wave's stage copies (vmcnt) after the products that produce
// acc64: one element of every tile is an input of the wait.
template <int MT>
__device__ __forceinline__ void stage_wait(d4 (&acc64)[MT][1])
{
    static_assert(MT == 4 || MT == 8, "tiles per wave");
    if constexpr (MT == 4) {
        asm volatile("s_waitcnt vmcnt(0)" ::"v"(acc64[0][0][0]), "v"(acc64[1][0][0]),
                     "v"(acc64[2][0][0]), "v"(acc64[3][0][0])
                     : "memory");
    } else {
        asm volatile("s_waitcnt vmcnt(0)" ::"v"(acc64[0][0][0]), "v"(acc64[1][0][0]),
                     "v"(acc64[2][0][0]), "v"(acc64[3][0][0]), "v"(acc64[4][0][0]),
                     "v"(acc64[5][0][0]), "v"(acc64[6][0][0]), "v"(acc64[7][0][0])
                     : "memory");
    }
}

// Copy of the fp16 split's scales of one stage (groups g0 .. g0+3 of 16
// columns from col0) into LDS at dst, as [group][16] floats: lane l of the
// first wave copies 4 columns of group l/4.
__device__ __forceinline__ void f16_dma_scales(gptr<const float> fsc, int64_t ldF, int col0,
                                               int64_t g0, int t, float* dst)
{
    if (t < 16) {
        const gptr<const float> src = fsc + (g0 + (t >> 2)) * ldF + col0 + 4 * (t & 3);
        __builtin_amdgcn_global_load_lds((const ABM_GLOBAL void*)src,
                                         (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    }
}

template <bool F16> struct SplitType;
template <> struct SplitType<false> {
    typedef bf8 frag;
    static __device__ __forceinline__ f4 mfma(frag a, frag b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct SplitType<true> {
    typedef h8 frag;
    static __device__ __forceinline__ f4 mfma(frag a, frag b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// Power-of-two exponent e such that the largest |w| of a weight window lies
// in [2^13, 2^14) after scaling by 2^e; the weights are monotone in their
// index for every order, so the largest sits at one end of the window.
__device__ __forceinline__ int f16_window_exponent(float w_first, float w_last)
{
    const float m = fmaxf(fabsf(w_first), fabsf(w_last));
    if (!(m > 0.f) || !isfinite(m)) return 0;
    int ex;
    (void)frexpf(m, &ex);
    const int e = 14 - ex;
    return e < -100 ? -100 : (e > 100 ? 100 : e);
}

// MT row tiles per wave, WPR waves per row kind (predictor, corrector); with
// 4 waves two workgroups share a CU, so each SIMD runs two waves.  F16: the
// operands are a two-term fp16 split of values scaled by powers of two (the
// history per 32-row group and column, the weights per window), undone when
// each step's float sums are added into the double accumulators; otherwise a
// bf16 split with TERMS terms.
template <int MT, int TERMS, int WPR, bool F16>
__global__ __launch_bounds__(128 * WPR, WPR == 2 ? 2 : 1) void k_far_split(const GroupDev* groups,
                                                            const FarItem* items, int kchunk)
{
    typedef typename SplitType<F16>::frag frag;
    static_assert(!F16 || TERMS == 2, "the fp16 split has two terms");
    constexpr int L = 16 * MT * WPR, TN = 16;
    constexpr int NTH = 128 * WPR;              // threads
    FarArgs A;
    if (!far_view(groups, items, kchunk, L, A)) return;
    constexpr int QS = 4;                       // K-steps (32 rows) per stage
    constexpr int KS = 32 * QS;                 // history rows per stage
    constexpr int NB8 = KS / 8;                 // 8-row blocks per stage
    constexpr int kStageU4 = TERMS * NB8 * TN;  // 16-byte units per stage
    static_assert(KS == kBfStageRows && kStageU4 <= kBfStageU4, "stage buffers");
    static_assert((2 * QS) % MT == 0, "ring slots must repeat within a stage");
    extern __shared__ __attribute__((aligned(16))) uint16_t smh[];
    // Reversed weight windows, two copies each: copy 1 is copy 0 shifted by
    // one element.  A fragment starts at an element offset whose parity is
    // fixed per lane; read from the copy where that offset is even, every
    // 16-byte fragment read is 4-byte aligned (2-byte aligned reads stall
    // the LDS pipeline).
    const int win = L + A.kchunk;               // multiple of 8
    uint16_t* wrb = smh;                        // [TERMS][2][win] reversed b windows
    uint16_t* wra = smh + 2 * TERMS * win;      // [TERMS][2][win] reversed a windows
    u4* Bst = reinterpret_cast<u4*>(smh + 4 * TERMS * win);   // [2][TERMS][NB8][TN]
    float* Ssc = reinterpret_cast<float*>(Bst + 2 * kStageU4); // fp16: [2][QS][TN] scales

    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int col0 = blockIdx.x * TN;
    const bool corr = wid >= WPR;
    const int rbase = (wid % WPR) * (L / WPR);
    const uint16_t* wr = corr ? wra : wrb;
    const int li = lane & 15, g = lane >> 4;
    const int abase = L - 1 - rbase - li + 8 * g;   // fragment v starts at abase + 16 v
    const int par = abase & 1;                       // copy read by this lane
    const uint16_t* wrl = wr + par * win + (abase - par);

    f4 acc[MT][1];
    d4 acc64[MT][1];
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        acc[i][0] = f4{0.f, 0.f, 0.f, 0.f};
        acc64[i][0] = d4{0.0, 0.0, 0.0, 0.0};
    }

    const gptr<const uint16_t> fh0 = A.Fh[0], fh1 = A.Fh[1], fh2 = A.Fh[TERMS - 1];
    // a fragment as dword reads (dword-aligned through the copy choice): one
    // 16-byte read at a dword, not 16-byte, boundary would take the LDS's
    // unaligned path
    const uint32_t* wrd = reinterpret_cast<const uint32_t*>(wrl);
    auto afrag = [&](int tt, int v) -> frag {
        const uint32_t* q = wrd + tt * win + 8 * v;
        u4 x;
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = q[k];
        return __builtin_bit_cast(frag, x);
    };
    const gptr<const float> fsc_g = A.Fsc;
    double unscale_w = 1.0;                     // fp16: 2^-e of this wave's weight window

    const int c_begin = blockIdx.y * A.chunks_per_split;
    int c_end = c_begin + A.chunks_per_split;
    if (c_end > A.nchunks) c_end = A.nchunks;
    for (int chunk = c_begin; chunk < c_end; ++chunk) {
        const ChunkBounds cb = chunk_bounds(A, L, chunk);
        const int64_t kb8 = (cb.k_lo - 1) >> 3;
        __syncthreads();   // previous chunk's readers are done with the LDS
        // reversed windows: copy 0 holds w[jb + wlen - 1 - x], copy 1
        // w[jb + wlen - 2 - x] (jb >= L, so the index stays >= 0)
        if constexpr (F16) {
            // split terms of the scaled float weights, made here
            const int eb = f16_window_exponent(A.b32[cb.jb], A.b32[cb.jb + cb.wlen - 1]);
            const int ea = f16_window_exponent(A.a32[cb.jb], A.a32[cb.jb + cb.wlen - 1]);
            const float sb = ldexpf(1.f, eb), sa = ldexpf(1.f, ea);
            unscale_w = ldexp(1.0, corr ? -ea : -eb);
            auto put = [&](uint16_t* w, int copy, int x, float v) {
                const _Float16 hi = (_Float16)v;
                const _Float16 lo = (_Float16)(v - (float)hi);
                w[copy * win + x] = __builtin_bit_cast(uint16_t, hi);
                w[(2 + copy) * win + x] = __builtin_bit_cast(uint16_t, lo);
            };
            for (int x = t; x < cb.wlen; x += NTH) {
                const int64_t j = cb.jb + cb.wlen - 1 - x;
                put(wrb, 0, x, A.b32[j] * sb);
                put(wrb, 1, x, A.b32[j - 1] * sb);
                put(wra, 0, x, A.a32[j] * sa);
                put(wra, 1, x, A.a32[j - 1] * sa);
            }
        } else {
            for (int x = t; x < cb.wlen; x += NTH) {
                const int64_t j = cb.jb + cb.wlen - 1 - x;
#pragma unroll
                for (int tt = 0; tt < TERMS; ++tt) {
                    wrb[2 * tt * win + x] = A.bh[tt][j];
                    wrb[(2 * tt + 1) * win + x] = A.bh[tt][j - 1];
                    wra[2 * tt * win + x] = A.ah[tt][j];
                    wra[(2 * tt + 1) * win + x] = A.ah[tt][j - 1];
                }
            }
        }
        bf_dma_stage<TERMS, NB8, NTH>(fh0, fh1, fh2, A.ldF, col0, kb8, t, Bst);
        if constexpr (F16) f16_dma_scales(fsc_g, A.ldF, col0, kb8 >> 2, t, Ssc);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's copies are in LDS
        __syncthreads();                                      // and every other wave's
        // ring[tt][slot]: fragment v lives in slot v mod MT; start with v = -(MT-1) .. 0
        frag ring[TERMS][MT];
#pragma unroll
        for (int tt = 0; tt < TERMS; ++tt)
#pragma unroll
            for (int tm = 0; tm < MT; ++tm) ring[tt][(MT - tm) % MT] = afrag(tt, -tm);

        const int nstages = cb.nk / KS;
        for (int st = 0; st < nstages; ++st) {
            const int buf = st & 1;
            const u4* Bs = Bst + buf * kStageU4;
#pragma unroll
            for (int qq = 0; qq < QS; ++qq) {
                const int q = st * QS + qq;
                if (qq > 0 || st > 0) {
                    // fragments v = 2q-1 and 2q replace v = 2q-1-MT and 2q-MT
#pragma unroll
                    for (int tt = 0; tt < TERMS; ++tt) {
                        ring[tt][(2 * qq - 1 + 2 * QS) % MT] = afrag(tt, 2 * q - 1);
                        ring[tt][(2 * qq) % MT] = afrag(tt, 2 * q);
                    }
                }
                frag bfr[TERMS];
#pragma unroll
                for (int tt = 0; tt < TERMS; ++tt)
                    bfr[tt] = __builtin_bit_cast(frag, Bs[(tt * NB8 + 4 * qq + g) * TN + li]);
                // fp16: undoes the scaling of this step's rows of column li
                double unscale = 1.0;
                if constexpr (F16) unscale = (double)Ssc[(buf * QS + qq) * TN + li] * unscale_w;
                // the stage's last LDS reads are issued: copy the next stage
                // into the other buffer (read by nobody since the last barrier)
                if (qq == QS - 1 && st + 1 < nstages) {
                    bf_dma_stage<TERMS, NB8, NTH>(fh0, fh1, fh2, A.ldF, col0, kb8 + (int64_t)(st + 1) * NB8,
                                                  t, Bst + (buf ^ 1) * kStageU4);
                    if constexpr (F16)
                        f16_dma_scales(fsc_g, A.ldF, col0, (kb8 >> 2) + (int64_t)(st + 1) * QS, t,
                                       Ssc + (buf ^ 1) * QS * TN);
                }
                // Ordering fence (no instruction): this step's products take their
                // history operands only after the previous step's double flush, so a
                // single set of float accumulators is live.  Left alone, the compiler
                // keeps every step's accumulators of a stage and flushes them
                // together, which needs a second register set and halves occupancy.
#pragma unroll
                for (int i = 0; i < MT; ++i)
#pragma unroll
                    for (int tt = 0; tt < TERMS; ++tt)
                        asm volatile("" : "+v"(bfr[tt]) : "v"(acc64[i][0][0]), "v"(acc64[i][0][1]),
                                     "v"(acc64[i][0][2]), "v"(acc64[i][0][3]));
                // small products first, the leading w0 F0 last
                constexpr int NP = (TERMS == 2) ? 3 : 6;
                constexpr int pa[6] = {2, 0, 1, 1, 0, 0};
                constexpr int pb[6] = {0, 2, 1, 0, 1, 0};
                constexpr int p0 = (TERMS == 2) ? 3 : 0;
#pragma unroll
                for (int pp = p0; pp < p0 + NP; ++pp) {
#pragma unroll
                    for (int tm = 0; tm < MT; ++tm) {
                        const frag af = ring[pa[pp]][(2 * qq - tm + 2 * QS * MT) % MT];
                        acc[tm][0] = SplitType<F16>::mfma(af, bfr[pb[pp]], acc[tm][0]);
                    }
                }
                if constexpr (F16) {
#pragma unroll
                    for (int i = 0; i < MT; ++i) {
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            acc64[i][0][v] = fma((double)acc[i][0][v], unscale, acc64[i][0][v]);
                        acc[i][0] = f4{0.f, 0.f, 0.f, 0.f};
                    }
                } else {
                    flush_acc<MT, 1>(acc, acc64);   // one 32-row step per float run
                }
            }
            // the next stage is in LDS; the wait takes every tile's sum as an
            // operand so that the last step's products are issued before it
            // (they would otherwise be scheduled after the barrier, leaving the
            // copy nothing to overlap)
            stage_wait<MT>(acc64);
            __syncthreads();
        }
    }
    store_part<MT, 1>(A, acc64, col0, (corr ? L : 0) + rbase, li, g, L);
}

struct LpLaunch {
    const GroupDev* groups;
    const FarItem* items;
    int n, max_coltiles, max_nsplit, kchunk;
};

template <int MT>
hipError_t launch_f32_t(const LpLaunch& P, hipStream_t st)
{
    constexpr int L = 64 * MT;
    const size_t shmem = far_lp_lds_bytes(L, P.kchunk, ABM_FAR_FP32);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_far_f32<MT>), shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_far_f32<MT>), dim3((unsigned)P.max_coltiles, (unsigned)P.max_nsplit, (unsigned)P.n),
                       dim3(512), shmem, st, P.groups, P.items, P.kchunk);
    return hipGetLastError();
}

// Row tiles per wave: 8 where one wave per SIMD can hold them (L <= 256:
// the history fragment is then read once per 8 tiles), else L/64.
template <int L, int TERMS, bool F16>
hipError_t launch_split_t(const LpLaunch& P, hipStream_t st)
{
    constexpr int MT = L <= 256 ? (L / 32 < 8 ? L / 32 : 8) : L / 64;
    constexpr int WPR = L / (16 * MT);
    const size_t shmem = far_lp_lds_bytes(
        L, P.kchunk, F16 ? ABM_FAR_FP16X3 : (TERMS == 2 ? ABM_FAR_BF16X3 : ABM_FAR_BF16X6));
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_far_split<MT, TERMS, WPR, F16>), shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_far_split<MT, TERMS, WPR, F16>),
                       dim3((unsigned)P.max_coltiles, (unsigned)P.max_nsplit, (unsigned)P.n),
                       dim3(128 * WPR), shmem, st, P.groups, P.items, P.kchunk);
    return hipGetLastError();
}

}  // namespace

size_t far_lp_lds_bytes(int L, int kchunk, int prec)
{
    const int TN = 16;
    if (prec == ABM_FAR_FP32) return (2 * (size_t)(L + kchunk) + 2 * 32 * TN) * sizeof(float);
    const int terms = prec == ABM_FAR_BF16X6 ? 3 : 2;
    // reversed weight windows (two copies) + two history stages of 128 rows
    // (+ their scales for the fp16 split)
    return 4 * (size_t)terms * (L + kchunk) * 2 + 2 * (size_t)terms * (kBfStageRows / 8) * TN * 16 +
           (prec == ABM_FAR_FP16X3 ? 2 * (kBfStageRows / 32) * TN * sizeof(float) : 0);
}

hipError_t launch_far_lp(const GroupDev* groups, const FarItem* items, int n, int max_coltiles,
                         int max_nsplit, int kchunk, int L, int prec, hipStream_t st)
{
    const LpLaunch A{groups, items, n, max_coltiles, max_nsplit, kchunk};
    if (prec == ABM_FAR_FP32) {
        switch (L) {
        case 128: return launch_f32_t<2>(A, st);
        case 256: return launch_f32_t<4>(A, st);
        case 512: return launch_f32_t<8>(A, st);
        default: return hipErrorInvalidValue;
        }
    }
    if (prec == ABM_FAR_BF16X3) {
        switch (L) {
        case 128: return launch_split_t<128, 2, false>(A, st);
        case 256: return launch_split_t<256, 2, false>(A, st);
        case 512: return launch_split_t<512, 2, false>(A, st);
        default: return hipErrorInvalidValue;
        }
    }
    if (prec == ABM_FAR_FP16X3) {
        switch (L) {
        case 128: return launch_split_t<128, 2, true>(A, st);
        case 256: return launch_split_t<256, 2, true>(A, st);
        case 512: return launch_split_t<512, 2, true>(A, st);
        default: return hipErrorInvalidValue;
        }
    }
    if (prec == ABM_FAR_BF16X6) {
        switch (L) {
        case 128: return launch_split_t<128, 3, false>(A, st);
        case 256: return launch_split_t<256, 3, false>(A, st);
        case 512: return launch_split_t<512, 3, false>(A, st);
        default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace abm
