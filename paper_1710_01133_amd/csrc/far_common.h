// Per-workgroup view of one far-field work item (shared by the far kernels).
#pragma once
#include "abm_dev.h"
#include "abm_kernels.h"

namespace abm {

struct FarArgs {
    gptr<const double> b;
    gptr<const double> a;
    gptr<const float> b32;
    gptr<const float> a32;
    gptr<const uint16_t> bh[3];
    gptr<const uint16_t> ah[3];
    gptr<const double> F;
    gptr<const float> F32;
    gptr<const uint16_t> Fh[3];
    gptr<const float> Fsc;     // fp16 split: per-32-row scales of the history
    int64_t ldF;
    int64_t rows;
    int64_t mL;
    int64_t kfar;
    int32_t kchunk;
    int32_t nchunks;
    int32_t chunks_per_split;
    gptr<const int8_t> Fq[3];  // int8 limbs of the history (q16_index layout)
    gptr<const double> Fqs;    // int8 limbs: per-block scales of the history
    gptr<double> part;
    int64_t ldP;
};

// History rows k_lo .. k_hi-1 of one chunk of a far item and the window of
// weight indices jb .. jb+wlen-1 its products read (block rows r = 0..L-1).
struct ChunkBounds {
    int64_t k_lo, k_hi, jb;
    int nk, wlen;
};

__device__ __forceinline__ ChunkBounds chunk_bounds(const FarArgs& A, int L, int chunk)
{
    ChunkBounds c;
    c.k_lo = 1 + (int64_t)chunk * A.kchunk;
    c.k_hi = c.k_lo + A.kchunk;
    if (c.k_hi > A.kfar + 1) c.k_hi = A.kfar + 1;
    c.nk = (int)(c.k_hi - c.k_lo);
    c.jb = A.mL - c.k_hi + 1;
    c.wlen = L + c.nk - 1;
    return c;
}

// Fills A for work item `item`; false when column tile `tile` or history split
// `split` lies beyond the item's (the launch grid covers the largest item).
__device__ __forceinline__ bool far_view_at(const GroupDev* __restrict__ groups,
                                            const FarItem* __restrict__ items, int item, int tile,
                                            int split, int kchunk, int L, FarArgs& A)
{
    const FarItem it = items[item];
    if (tile >= it.ncoltiles || split >= it.nsplit) return false;
    const GroupDev& G = groups[it.group];
    const CompWeights& W = G.w[it.comp];
    A.b = as_global(W.b);
    A.a = as_global(W.a);
    A.b32 = as_global(W.b32);
    A.a32 = as_global(W.a32);
    // the item's columns start at coff (a multiple of 16): every layout of
    // the history and of the partial slices is shifted by whole columns or
    // whole 16-column blocks
    const int64_t coff = it.coff;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        A.bh[i] = as_global(W.bh[i]);
        A.ah[i] = as_global(W.ah[i]);
        A.Fh[i] = G.Fh[i] ? as_global((const uint16_t*)G.Fh[i]) + coff * 8 : nullptr;
    }
    A.Fsc = G.Fsc ? as_global((const float*)G.Fsc) + coff : nullptr;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        A.Fq[i] = G.Fq[i] ? as_global((const int8_t*)G.Fq[i]) + coff * 16 : nullptr;
    A.Fqs = G.Fqs ? as_global((const double*)G.Fqs) + coff : nullptr;
    A.F = as_global((const double*)G.F) + coff;
    A.F32 = G.F32 ? as_global((const float*)G.F32) + (coff >> 4) * G.rows * 16 : nullptr;
    A.ldF = G.ldF;
    A.rows = G.rows;
    A.mL = it.mL;
    A.kfar = it.kfar;
    A.kchunk = kchunk;
    A.nchunks = it.nchunks;
    A.chunks_per_split = it.chunks_per_split;
    A.part = as_global(G.part[(it.mL / L) & 1]) + coff * (2 * L);
    A.ldP = it.ldP;
    return true;
}

// The view of workgroup (blockIdx.x = column tile, blockIdx.y = split,
// blockIdx.z = item).
__device__ __forceinline__ bool far_view(const GroupDev* __restrict__ groups,
                                         const FarItem* __restrict__ items, int kchunk, int L,
                                         FarArgs& A)
{
    return far_view_at(groups, items, blockIdx.z, blockIdx.x, blockIdx.y, kchunk, L, A);
}

}  // namespace abm
