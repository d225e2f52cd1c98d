// Host-side launch interface of the libabm kernels (internal to libabm).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "abm.h"

namespace abm {

// ---- K0: weight tables ---------------------------------------------------
// Writes gam[0] = Gamma(alpha+1), gam[1] = Gamma(alpha+2), then b, a, c for
// k = 0..n-1 (each array n doubles, device memory).
hipError_t launch_weights(double alpha, int64_t n, double* gam, double* b, double* a, double* c,
                          hipStream_t st);

// Reduced copies of b, a (float and bf16 split terms) for k = 0..n-1;
// any destination may be null (bh/ah arrays of 3 pointers).
hipError_t launch_weights_lowp(int64_t n, const double* b, const double* a, float* b32, float* a32,
                               uint16_t* const* bh, uint16_t* const* ah, hipStream_t st);

// Number of right-hand sides (enum abm_rhs) and the chain kernels' kinds:
// a right-hand side, plus kRhsCount when the group's components have orders
// of their own (a weight table per component).
constexpr int kRhsCount = 6;
constexpr int kChainKinds = 2 * kRhsCount;
inline int chain_kind(int rhs, bool per_comp) { return rhs + (per_comp ? kRhsCount : 0); }

// ---- K1: plain per-step persistent kernel --------------------------------
struct PlainArgs {
    const double* b[4];  // weights b_k, k < N, of each component's order
    const double* a[4];  // weights a_k
    const double* c[4];  // weights c_k
    const double* gam[4];  // Gamma(alpha+1), Gamma(alpha+2)
    double alpha[4];
    double h;
    double x0[4];
    double x1[4];        // y'(0), used by components of order above 1
    double p[8];
    int64_t N;
    int32_t G;           // workgroups (all co-resident)
    int32_t nloc;        // history chunks held in LDS per workgroup
    double* part;        // plain_part_doubles(G) doubles
    uint32_t* flags;     // G step flags, zero at launch
    double* y_out;
    int64_t out_stride;
    uint32_t* status;    // device status word (kStatus* bits)
    uint32_t spin_limit; // bound on each device-side wait
    uint32_t wait_bias;  // added to every awaited step number: 0 (a test hook
                         // sets it so that no wait can be met)
};
int plain_max_local_chunks(int d);
int plain_chunk();
// Local chunks per workgroup whose weights the kernel prefetches into
// registers (tables: weight tables in use, 1 or d); beyond it, in-step loads.
int plain_prefetch_chunks(int tables);
int plain_part_doubles(int G);
// kind: chain_kind(rhs, components have their own orders)
hipError_t launch_plain(const PlainArgs& A, int kind, hipStream_t st);
// The one-workgroup form (no grid synchronisation, weights held in registers)
// for histories that fit one CU's LDS: whether N steps of d components with
// the given number of weight tables fit it, and its launch (G, nloc, part and
// flags of A are not used).
bool plain_single_fits(int64_t N, int d, int tables);
hipError_t launch_plain_single(const PlainArgs& A, int kind, hipStream_t st);

// ---- K0 / K1 in double-double (ABM_FAR_DD) -----------------------------------
// Tables of (hi, lo) pairs: gam holds Gamma(alpha+1), Gamma(alpha+2) (4 doubles),
// b, a, c 2n doubles each; PlainArgs pointers refer to such pairs and y_out
// receives 2d doubles per state.
hipError_t launch_weights_dd(double alpha, int64_t n, double* gam, double* b, double* a, double* c,
                             hipStream_t st);
bool plain_dd_single_fits(int64_t N, int d, int tables);
int plain_dd_max_local_chunks(int d);
int plain_dd_part_doubles(int G);
// single: the one-workgroup form; otherwise A.G cooperative workgroups (flags zero)
hipError_t launch_plain_dd(const PlainArgs& A, bool single, int kind, hipStream_t st);

// ---- blocked method: groups and work items --------------------------------
// A group is a set of trajectories sharing their orders (one weight table, or
// one per component), one right-hand side and one far-field precision; their
// components are the columns of one time-major history.  Launches take lists
// of work items that point at group descriptors in device memory, so one
// launch can advance groups that are at different blocks (differing N,
// alpha, start time).
struct TrajDesc {
    double x0[4];
    double x1[4];          // y'(0), used by components of order above 1
    double p[8];
    double h;
    int64_t N;
    int64_t out_stride;
    double* y_out;
    int32_t col0;          // column of component 0 of this trajectory in its group's history
    int32_t cstride;       // column distance between its components (1, or the
                           // component block width when columns are component-major)
};

// The weight tables of one order (padded past N by at least 2L).
struct CompWeights {
    const double* b;
    const double* a;
    const double* c;
    const double* gam;     // Gamma(alpha+1), Gamma(alpha+2)
    const float* b32;      // float copies (far_prec fp32)
    const float* a32;
    const uint16_t* bh[3]; // bf16 split terms (far_prec bf16x3 / bf16x6)
    const uint16_t* ah[3];
    double alpha;
};

struct GroupDev {
    CompWeights w[4];      // component i's tables (all equal unless per_comp)
    double* F;             // time-major double history [k][ldF]
    float* F32;            // float copy: column-blocked (colblocked_index), or
                           // time-major [k][ldF] in a narrow group

    uint16_t* Fh[3];       // bf16 (or fp16) split terms of the history, k-blocked (kblocked_index)
    float* Fsc;            // fp16 split: 2^-e of the scaling of rows 32g+1 .. 32g+32 of
                           // column c at [g * ldF + c] (null otherwise)
    int8_t* Fq[3];         // int8 limbs of the history (far_prec i8): digit i of row k,
                           // column c at q16_index(k, c, ldF)
    double* Fqs;           // int8 limbs: 2^-e of the scaling of block g (rows gL+1 ..
                           // gL+L) of column c at [g * ldF + c]
    int64_t ldF;           // padded columns
    int64_t rows;          // history rows allocated
    double* accn;          // [member][2][d][L] sums carried into the next block
    double* part[2];       // far partials [split][col][2L], by block parity
    const TrajDesc* traj;  // members
    int32_t d;
    int32_t narrow;        // 1: few columns, far field by the blocked convolution,
                           // ldF = real columns and F32 time-major
    int32_t per_comp;      // 1: components have orders of their own; columns are
                           // component-major (component i of member j at i*cstride + j)
    int32_t deriv;         // bit i: component i has order above 1 (start term x0 + t x1)
    uint32_t* status;      // status word of this group's own (kStatus* bits), or null: the
                           // chain then raises the launch's word
};

// Far field of one group (or of one component of a group whose components
// have their own orders) for block m: history k = 1..kfar, kfar = (m-1)L.
struct FarItem {
    int32_t group;
    int32_t ncoltiles;     // active columns / tile width (narrow: product tiles)
    int32_t nchunks;       // ceil(kfar / kchunk) (narrow: chunks of shifts)
    int32_t chunks_per_split;
    int32_t nsplit;        // partial slices written
    int32_t comp;          // weight tables used: the group's w[comp]
    int32_t coff;          // first history column of the item (a multiple of 16
                           // unless the group is narrow)
    int32_t ncols;         // columns of the item (narrow groups)
    int64_t mL;
    int64_t kfar;
    int64_t ldP;           // column stride of the partial slices (active columns,
                           // padded to the tile width except in narrow groups;
                           // all columns of a per-component group)
};

// Chain of one trajectory (group member) through block m.
struct ChainItem {
    int32_t group;
    int32_t member;
    int32_t nsplit;        // far partial slices of this block (0 when m < 2)
    int32_t kind;          // chain_kind of the group
    int64_t mL;
    int64_t ldP;
};

// ---- K2: far-field products ------------------------------------------------
int far_tile_cols(int L, int prec);
size_t far_lds_bytes(int L, int kchunk, int prec);
// Chunks of the far range 1..kfar and their grouping into at most max_split
// workgroup ranges; returns the number of partial slices.
int far_split_plan(int64_t kfar, int kchunk, int max_split, int* nchunks, int* chunks_per_split);
// Upper bound of far_split_plan's slice count over every kfar <= kfar_max.
int far_split_bound(int64_t kfar_max, int kchunk, int max_split);
// One launch over n items, all of launch class cls (far_class below);
// grid (max_coltiles, max_nsplit, n) for the Toeplitz kernels, (1,
// max_nsplit, n) for the blocked convolution; workgroups beyond an item's
// own tiles/splits exit.
hipError_t launch_far(const GroupDev* groups, const FarItem* items, int n, int max_coltiles,
                      int max_nsplit, int kchunk, int L, int cls, hipStream_t st);
size_t far_lp_lds_bytes(int L, int kchunk, int prec);
// Integer-limb far field (far_prec i8): LDS bytes, launch (L = 128 or 256).
size_t far_i8_lds_bytes(int L, int kchunk);
int far_i8_tile_cols();
hipError_t launch_far_i8(const GroupDev* groups, const FarItem* items, int n, int max_coltiles,
                         int max_nsplit, int kchunk, int L, hipStream_t st);
hipError_t launch_far_lp(const GroupDev* groups, const FarItem* items, int n, int max_coltiles,
                         int max_nsplit, int kchunk, int L, int prec, hipStream_t st);
hipError_t allow_lds(const void* fn, size_t bytes);   // dynamic LDS above 64 KiB

// Far-field launch classes: 0..6 the Toeplitz kernels by precision (abm_prec;
// 5, double-double, never reaches the blocked path), 7 and 8 the blocked
// convolution of narrow groups in double and float.
constexpr int kFarClasses = 9;
inline int far_class(int prec, bool narrow)
{
    return narrow ? (prec == 0 ? 7 : 8) : prec;
}
inline bool is_narrow_class(int cls) { return cls >= 7; }
// Precisions of the blocked path (abm_prec values a batch may use).
constexpr int kBlockedPrecs[6] = {ABM_FAR_FP64, ABM_FAR_FP32, ABM_FAR_BF16X3, ABM_FAR_BF16X6,
                                  ABM_FAR_FP16X3, ABM_FAR_I8};
// Blocked convolution (narrow groups, fp64 / fp32 far field): product tiles
// of a block for cols columns, whether a group qualifies, its split plan over
// the K + L - 16 rows of shifts and the bound of that plan's slice count.
constexpr int kHankelMaxCols = 8;
int hankel_tiles(int64_t cols, int L);
bool hankel_fits(int prec, int64_t cols, int L);
int hankel_chunk_rows();
int hankel_split_plan(int64_t kfar, int L, int max_split, int* nchunks, int* chunks_per_split);
int hankel_split_bound(int64_t kfar_max, int L, int max_split);
size_t hankel_lds_bytes(int L, int max_tiles, int prec);
// Sums the partial slices of each narrow far item into its first slice (in
// slice order); the chain items of those blocks then read one slice.
hipError_t launch_far_reduce(const GroupDev* groups, const FarItem* items, int n, int max_cols,
                             int L, hipStream_t st);
hipError_t launch_far_hankel(const GroupDev* groups, const FarItem* items, int n, int max_tiles,
                             int max_nsplit, int L, int prec, hipStream_t st);

// ---- K3: near band + predictor/corrector chain -----------------------------
// One wave per item; all items of a launch share the chain kind.  spread:
// one wave per SIMD instead of two (more CUs, faster chains, less room for
// a far-field launch running beside them).
hipError_t launch_chain(const GroupDev* groups, const ChainItem* items, int n, int kind, int L,
                        bool spread, uint32_t* status, hipStream_t st);
// Items of any kinds in one launch (one kernel for all systems); nw is the
// largest chain_tables over the kinds of the items.
hipError_t launch_chain_mixed(const GroupDev* groups, const ChainItem* items, int n, int L,
                              int nw, uint32_t* status, hipStream_t st);
// Weight tables a chain of this kind keeps in LDS (1, or d when per-component).
int chain_tables(int kind);
// f_0 into history row 0 and y_0 = x0 for every member of the listed groups
// (all of right-hand side rhs).
hipError_t launch_chain_init(const GroupDev* groups, const ChainItem* items, int n, int rhs,
                             hipStream_t st);

// ---- utilities -----------------------------------------------------------
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);

}  // namespace abm
